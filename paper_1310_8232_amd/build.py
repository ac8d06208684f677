"""Compile the gfx950 library libpaper_1310_8232_amd.so in-tree with hipcc.

Objects go to paper_1310_8232_amd/_build/; the shared library is written next
to this file, where the binding loads it. Compiles every time it is called.

Every device compile asks hipcc for its per-kernel resource remarks
(-Rpass-analysis=kernel-resource-usage). The build fails when any kernel
spills SGPRs or VGPRs or uses per-lane scratch: spilled registers change a
kernel's schedule and memory traffic in ways the tests do not see, so the
product carries none. The per-kernel table is written to
_build/resource_usage.txt.

The build also disassembles the gfx950 code objects it produced and fails
when a vector-memory store of more than 8 bytes is directly followed by a
VALU instruction that writes one of the store's data registers: the store
reads its data after it issues, so without one instruction in between the
new value can be stored instead of the old one (a wait state the compiler
is meant to insert). Findings go to _build/store_hazards.txt.
"""
from __future__ import annotations

import os
import re
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
          "-Wno-unused-command-line-argument", "-Rpass-analysis=kernel-resource-usage"]
USAGE = os.path.join(OUT, "resource_usage.txt")
HAZARDS = os.path.join(OUT, "store_hazards.txt")
LLVM_BIN = os.environ.get("ROCM_LLVM_BIN", "/opt/rocm/llvm/bin")

_REMARK = re.compile(r"remark:\s+(Function Name|TotalSGPRs|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Occupancy \[waves/SIMD\]|SGPRs Spill|VGPRs Spill|LDS Size \[bytes/block\]):\s*(\S+)")


def parse_resource_usage(text: str) -> list:
    """Per-kernel records from hipcc's kernel-resource-usage remarks, in the
    order printed: dicts with the kernel's (mangled) name and its counts."""
    out, cur = [], None
    for line in text.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = {"name": val}
            out.append(cur)
        elif cur is not None:
            k = key.split(" [")[0].replace(" ", "_").lower()
            cur[k] = int(val) if val.lstrip("-").isdigit() else val
    return out


def spill_offenders(records: list) -> list:
    """Kernels that spill registers or use scratch memory."""
    return [r for r in records
            if r.get("sgprs_spill", 0) or r.get("vgprs_spill", 0) or r.get("scratchsize", 0)]


# The data operand: first for buffer stores (vdata, vaddr, ...), second for
# global / flat / scratch stores (vaddr, vdata, ...).
_STORE = re.compile(r"^\s*(?:buffer_store_(?:dwordx[34]|b96|b128)\s+(v\d+|v\[\d+:\d+\])"
                    r"|(?:global|flat|scratch)_store_(?:dwordx[34]|b96|b128)\s+\S+,\s*(v\d+|v\[\d+:\d+\]))")
_VALU_DST = re.compile(r"^\s*v_\w+\s+(v\d+|v\[\d+:\d+\])")
_FUNC = re.compile(r"^[0-9a-f]+ <([^>]+)>:")


def _vgprs(tok: str) -> set:
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    return {int(tok[1:])}


def store_data_hazards(disasm: str) -> list:
    """(kernel, store, next instruction) for every store of more than 8 bytes
    whose next instruction in address order is a VALU write of one of the
    store's data VGPRs (llvm-objdump text of a gfx950 code object)."""
    out, func, pending = [], None, None
    for line in disasm.splitlines():
        m = _FUNC.match(line)
        if m:
            func, pending = m.group(1), None
            continue
        text = line.split("//")[0].split(";")[0].strip()
        if not text or text.endswith(":"):
            continue
        if pending is not None:
            v = _VALU_DST.match(text)
            if v and _vgprs(v.group(1)) & pending[1]:
                out.append((func, pending[0], text))
            pending = None
        st = _STORE.match(text)
        if st:
            pending = (text, _vgprs(st.group(1) or st.group(2)))
    return out


def disassemble(obj: str) -> str:
    """llvm-objdump text of the gfx950 code object embedded in one of this
    build's object files (its .hip_fatbin bundle)."""
    fat, co = obj + ".fatbin", obj + ".co"
    heads = subprocess.run([os.path.join(LLVM_BIN, "llvm-objdump"), "-h", obj], check=True, capture_output=True,
                           text=True).stdout
    if ".hip_fatbin" not in heads:
        return ""  # no device code in this object
    subprocess.run([os.path.join(LLVM_BIN, "llvm-objcopy"), "--dump-section", f".hip_fatbin={fat}", obj,
                    obj + ".strip"], check=True, capture_output=True)
    os.remove(obj + ".strip")
    subprocess.run([os.path.join(LLVM_BIN, "clang-offload-bundler"), "--unbundle", "--type=o", f"--input={fat}",
                    f"--targets=hipv4-amdgcn-amd-amdhsa--{ARCH}", f"--output={co}"], check=True, capture_output=True)
    r = subprocess.run([os.path.join(LLVM_BIN, "llvm-objdump"), "-d", f"--mcpu={ARCH}", co], check=True,
                       capture_output=True, text=True)
    os.remove(fat)
    os.remove(co)
    return r.stdout


ARCH = "gfx950"


def source_hash() -> str:
    """Hash of every source compiled into the library and of its public
    header: the code identity that tune cache entries carry."""
    import hashlib
    h = hashlib.sha256()
    names = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".h", ".cpp")))
    for n in names:
        h.update(n.encode() + b"\0")
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    with open(os.path.join(HERE, "..", "include", "stencil.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def _jobs():
    objs = []
    for r in RADII:
        objs.append((os.path.join(OUT, f"kernels_r{r}.o"),
                     [HIPCC, *COMMON, f"-DRADIUS={r}", "-c", os.path.join(CSRC, "kernels_radius.hip")]))
    objs.append((os.path.join(OUT, "kernels_common.o"),
                 [HIPCC, *COMMON, "-c", os.path.join(CSRC, "kernels_common.hip")]))
    objs.append((os.path.join(OUT, "api.o"),
                 [HIPCC, *COMMON, f'-DP1310_SOURCE_HASH="{source_hash()}"', f'-DP1310_ARCH="{ARCH}"',
                  "-x", "hip", "-c", os.path.join(CSRC, "api.cpp")]))
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
    records = []
    for obj, full, p in procs:
        out, _ = p.communicate()
        raw = out.decode(errors="replace")
        records += parse_resource_usage(raw)
        # Everything but the resource remarks (and their source excerpts) and
        # the host pass's note about the packed-FP32 feature.
        text = "\n".join(l for l in raw.splitlines()
                         if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l
                         and not re.match(r"^\s*(\d+ \||\|)", l))
        if p.returncode != 0:
            failed.append((obj, text))
        elif verbose and text.strip():
            print(text, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed:\n" + "\n\n".join(f"{o}:\n{t}" for o, t in failed))
    with open(USAGE, "w") as f:
        for r in records:
            f.write(" ".join(f"{k}={v}" for k, v in r.items()) + "\n")
    if not records:
        raise RuntimeError("hipcc printed no kernel resource remarks; the spill check cannot run")
    bad = spill_offenders(records)
    if bad:
        raise RuntimeError("kernels spill registers or use scratch (see " + USAGE + "):\n" +
                           "\n".join(f"  {r['name']}: SGPR spill {r.get('sgprs_spill')}, "
                                      f"VGPR spill {r.get('vgprs_spill')}, scratch {r.get('scratchsize')} B/lane"
                                      for r in bad))
    hazards = []
    for obj, _ in _jobs():
        hazards += store_data_hazards(disassemble(obj))
    with open(HAZARDS, "w") as f:
        f.write(f"stores of more than 8 bytes directly followed by a VALU write of their data: {len(hazards)}\n")
        for k, st, nx in hazards:
            f.write(f"{k}\n    {st}\n    {nx}\n")
    if hazards:
        raise RuntimeError("store data overwritten by the next instruction (see " + HAZARDS + "):\n" +
                           "\n".join(f"  {k}: {st} / {nx}" for k, st, nx in hazards[:10]))
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + [o for o, _ in _jobs()]
    if verbose:
        print(" ".join(link), file=sys.stderr)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
