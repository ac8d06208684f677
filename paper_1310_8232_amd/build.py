"""Compile the gfx950 library libpaper_1310_8232_amd.so in-tree with hipcc.

Objects go to paper_1310_8232_amd/_build/; the shared library is written next
to this file, where the binding loads it. Compiles every time it is called.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpaper_1310_8232_amd.so")
RADII = (3, 4, 5)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _jobs():
    objs = []
    for r in RADII:
        objs.append((os.path.join(OUT, f"kernels_r{r}.o"),
                     [HIPCC, *COMMON, f"-DRADIUS={r}", "-c", os.path.join(CSRC, "kernels_radius.hip")]))
    objs.append((os.path.join(OUT, "kernels_common.o"),
                 [HIPCC, *COMMON, "-c", os.path.join(CSRC, "kernels_common.hip")]))
    objs.append((os.path.join(OUT, "api.o"),
                 [HIPCC, *COMMON, "-x", "hip", "-c", os.path.join(CSRC, "api.cpp")]))
    return objs


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    procs = []
    for obj, cmd in _jobs():
        full = cmd + ["-o", obj]
        if verbose:
            print(" ".join(full), file=sys.stderr)
        procs.append((obj, full, subprocess.Popen(full, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for obj, full, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append((obj, text))
        elif verbose and text.strip():
            print(text, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(f"{o}:\n{t}" for o, t in failed))
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for o, _ in _jobs()]
    if verbose:
        print(" ".join(link), file=sys.stderr)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
