"""The library build's register-spill check: hipcc's per-kernel resource
remarks are parsed, every compiled kernel is listed, and a kernel that spills
SGPRs or VGPRs or uses scratch fails the build."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build_module():
    spec = importlib.util.spec_from_file_location("_p1310_build_check",
                                                  os.path.join(ROOT, "paper_1310_8232_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


SAMPLE = """\
x.hip:10:1: remark: Function Name: _Z3fooPf [-Rpass-analysis=kernel-resource-usage]
   10 | {
      | ^
x.hip:10:1: remark:     TotalSGPRs: 24 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     VGPRs: 16 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark: Function Name: _Z3barPf [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     VGPRs: 168 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     SGPRs Spill: 85 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:30:1: remark: Function Name: _Z3bazPf [-Rpass-analysis=kernel-resource-usage]
x.hip:30:1: remark:     ScratchSize [bytes/lane]: 156 [-Rpass-analysis=kernel-resource-usage]
x.hip:30:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:30:1: remark:     VGPRs Spill: 139 [-Rpass-analysis=kernel-resource-usage]
"""


def test_remarks_are_parsed_and_spills_flagged():
    b = _build_module()
    recs = b.parse_resource_usage(SAMPLE)
    assert [r["name"] for r in recs] == ["_Z3fooPf", "_Z3barPf", "_Z3bazPf"]
    assert recs[0]["vgprs"] == 16 and recs[0]["totalsgprs"] == 24
    assert recs[1]["sgprs_spill"] == 85 and recs[2]["vgprs_spill"] == 139 and recs[2]["scratchsize"] == 156
    # SGPR spills (into VGPR lanes), VGPR spills and scratch each fail the check.
    assert [r["name"] for r in b.spill_offenders(recs)] == ["_Z3barPf", "_Z3bazPf"]


def test_build_flags_ask_for_the_remarks():
    b = _build_module()
    assert "-Rpass-analysis=kernel-resource-usage" in b.COMMON
    for _, cmd in b._jobs():
        assert "-Rpass-analysis=kernel-resource-usage" in cmd


def test_built_library_passed_the_check():
    # The table the last build wrote lists every sweep family and no spills.
    b = _build_module()
    if not os.path.exists(b.USAGE):
        pytest.skip("library not built in this tree")
    recs = []
    with open(b.USAGE) as f:
        for line in f:
            rec = dict(kv.split("=", 1) for kv in line.split())
            recs.append(rec)
    names = " ".join(r["name"] for r in recs)
    for fam in ("zmarch_kernel", "zmarch2_kernel", "zmarch_batch_kernel", "plain_kernel", "inject_kernel",
                "gradn_kernel"):
        assert fam in names, fam
    for r in recs:
        assert int(r.get("sgprs_spill", 0)) == 0 and int(r.get("vgprs_spill", 0)) == 0, r["name"]
        assert int(r.get("scratchsize", 0)) == 0, r["name"]
