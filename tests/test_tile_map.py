"""The LDS tile map of the wave-per-line line pass, checked on the host
(tests/tile_map_check.cpp compiled with g++ against the kernel's own header)."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2006_07583_amd", "csrc")


def test_tile_map_permutation_and_banks():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "tile_map_check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "tile_map_check.cpp"),
                        "-o", exe], check=True)
        res = subprocess.run([exe], capture_output=True, text=True)
        assert res.returncode == 0, res.stdout + res.stderr
