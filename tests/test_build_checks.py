"""The library build's checks: hipcc's per-kernel resource remarks are
parsed, every compiled kernel is listed, and a kernel that spills SGPRs or
VGPRs or uses scratch fails the build; the disassembled code objects are
scanned for a store whose data registers the next instruction overwrites."""
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


DISASM = """\
0000000000001000 <_Z3fooPf>:
	buffer_store_dwordx4 v[68:71], v100, s[36:39], s10 offen nt // 000000001000: E07E1000 0A094464
	v_cndmask_b32_e64 v68, 0, 1, s[42:43]                      // 000000001008: D1000044 00A90280
	buffer_store_dwordx4 v[20:23], v1, s[36:39], s10 offen nt  // 000000001010: E07E1000 0A091401
	s_nop 0                                                    // 000000001018: BF800000
	v_mov_b32_e32 v21, 0                                       // 00000000101C: 7E2A0280
	buffer_store_dwordx2 v[30:31], v1, s[36:39], 0 offen       // 000000001020: E0741000 80091E01
	v_mov_b32_e32 v30, 0                                       // 000000001028: 7E3C0280
0000000000002000 <_Z3barPf>:
	global_store_dwordx4 v[0:1], v[8:11], off                  // 000000002000: DC7C0000 007D0800
	v_lshl_add_u64 v[0:1], v[0:1], 0, s[6:7]                   // 000000002008: D2080000 00190100
	global_store_dwordx4 v[0:1], v[8:11], off                  // 000000002010: DC7C0000 007D0800
	v_add_f32_e32 v9, v2, v3                                   // 000000002018: 02120702
	buffer_store_dwordx4 v[40:43], v1, s[36:39], 0 offen       // 000000002020: E07C1000 80092801
	v_add_f32_e32 v44, v2, v3                                  // 000000002028: 02580702
"""


def test_store_data_hazards_are_found():
    # A store of more than 8 bytes whose next instruction is a VALU write of
    # one of its data registers; not after a wait state, not for an 8-byte
    # store, not for a write of a global store's address or of another
    # register.
    b = _build_module()
    got = b.store_data_hazards(DISASM)
    assert [(k, st.split()[0], nx.split()[0]) for k, st, nx in got] == [
        ("_Z3fooPf", "buffer_store_dwordx4", "v_cndmask_b32_e64"),
        ("_Z3barPf", "global_store_dwordx4", "v_add_f32_e32"),
    ]


def test_built_library_has_no_store_data_hazard():
    b = _build_module()
    if not os.path.exists(b.HAZARDS):
        pytest.skip("library not built in this tree")
    with open(b.HAZARDS) as f:
        first = f.readline()
    assert first.strip().endswith(": 0"), first
