"""Compile tests/c_abi/plain_method.c (a C program using only the C ABI) into
tests/c_abi/_build/plain_method, linked against the in-tree library and the
HIP runtime, with $ORIGIN-relative run paths."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "_build")
EXE = os.path.join(OUT, "plain_method")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           os.path.join(HERE, "plain_method.c"), "-o", EXE + ".tmp",
           f"-L{os.path.join(ROOT, 'paper_1310_8232_amd')}", "-lpaper_1310_8232_amd",
           f"-L{ROCM}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../../paper_1310_8232_amd", f"-Wl,-rpath,{ROCM}/lib"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
