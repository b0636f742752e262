"""The served-request admission (csrc/admission.h: the arena allocator and
the first-come-first-served rule of adi_server), built with g++ and driven
on the host by a simulated executor (tests/admission_check.cpp): requests
are admitted in submission order, never beyond max_active or the budget,
without overlapping memory, as soon as the oldest one fits; the arena
coalesces back to one block."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2006_07583_amd", "csrc")


def test_admission_against_simulated_executor():
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "admission_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I", CSRC, os.path.join(HERE, "admission_check.cpp"),
                    "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
