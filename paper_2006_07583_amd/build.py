"""Compile the HIP library ``libadi.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libadi.so")
SOURCES = ["line_pass.hip", "line_pass2.hip", "line_pass3.hip", "line_direct.hip", "adi.hip", "batch.hip",
           "serve.hip", "stream.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel) and link libadi.so; always
    recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="adi_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            cmd.remove("-shared")
            return obj, subprocess.run(cmd, capture_output=True, text=True)
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for obj, res in results:
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed compiling {os.path.basename(obj)}")
            if verbose:
                sys.stderr.write(res.stderr)
        tmp = LIB + ".tmp"
        res = subprocess.run([hipcc, *FLAGS, *[o for o, _ in results], "-o", tmp], capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libadi.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
