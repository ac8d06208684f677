"""Build the C oracle into oracle/libstencil_oracle.so with gcc.

Test infrastructure only: the oracle is the checker the GPU path is compared
against; building it is not using it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stencil_oracle.c")
LIB = os.path.join(HERE, "libstencil_oracle.so")


def build(verbose: bool = False) -> str:
    # Generic x86-64 code: the library is built here and loaded on other hosts.
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
