"""CPU tests of the C-ABI library: it loads, exports every declared entry
point, and its host-only logic (argument validation, the blocksize-selection
rule, the P-part grid, weights, stability limit) agrees with the oracle. No
call here launches a kernel."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

import oracle
import paper_1310_8232_amd as p

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil.h")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z_0-9]+)\s*\(", text)))


def test_header_and_library_agree():
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(p._lib, n), f"library does not export {n}"
    assert set(names) == set(p.EXPORTED)


def test_strerror_covers_codes():
    for code in (p.OK, p.EINVAL, p.EUNSTABLE, p.ENOMEM, p.EDEVICE, p.EUNSUPPORTED, p.EALIAS):
        assert p.stencil_strerror(code) not in ("", "unknown status")


@pytest.mark.parametrize("R", [3, 4, 5])
def test_weights_match_oracle(R):
    c = oracle.fd_coefficients(R)
    got = p.stencil_coefficients(R)
    assert len(got) == R + 1
    assert got[0] == np.float32(3.0 * c[0])
    for m in range(1, R + 1):
        assert got[m] == np.float32(c[m])


@pytest.mark.parametrize("R", [3, 4, 5])
def test_cfl_limit_matches_oracle(R):
    assert abs(p.stencil_cfl_limit(R) - oracle.cfl_limit(R)) < 1e-12


def test_pgrid_matches_paper_and_oracle():
    g = json.load(open(os.path.join(GOLDEN, "pgrid_paper_example.json")))
    for S, expect in zip(g["S"], g["lists"]):
        assert p.stencil_pgrid(S, g["P"]) == expect
    rng = np.random.default_rng(1)
    for _ in range(300):
        S = int(rng.integers(1, 3000))
        P = int(rng.integers(2, 25))
        assert p.stencil_pgrid(S, P) == oracle.pgrid(S, P)


@pytest.mark.parametrize("policy", ["worst", "min", "avg", "ob"])
def test_select_matches_oracle(policy):
    rng = np.random.default_rng(9)
    for _ in range(300):
        nn, nk, nc = (int(rng.integers(1, 4)), int(rng.integers(1, 6)), int(rng.integers(1, 7)))
        t = rng.integers(1, 7, size=(nn, nk, nc)).astype(float)
        if rng.random() < 0.5:
            t = t + rng.random(size=t.shape)
        ids = [list(range(i * nc, (i + 1) * nc)) for i in range(nn)]
        assert p.stencil_select(t.tolist(), policy) == oracle.select_block(t.tolist(), ids, policy)


def _init(**kw):
    args = dict(nx=32, ny=32, nz=32, h=10.0, dt=0.002, vmax=2000.0)
    args.update(kw)
    return p.stencil_init(**args)


def test_init_validation():
    ctx = _init()
    p.stencil_destroy(ctx)
    for bad in (dict(nx=0), dict(ny=-1), dict(h=0.0), dict(dt=-1.0), dict(vmax=float("nan")), dict(radius=2),
                dict(radius=6), dict(device=-1)):
        with pytest.raises(p.StencilError) as e:
            _init(**bad)
        assert e.value.status == p.EINVAL, bad
    lim = p.stencil_cfl_limit(4)
    ctx = _init(dt=0.999 * lim * 10.0 / 2000.0)
    p.stencil_destroy(ctx)
    with pytest.raises(p.StencilError) as e:
        _init(dt=1.001 * lim * 10.0 / 2000.0)
    assert e.value.status == p.EUNSTABLE


def test_storage_validation():
    d = p.StencilDesc(16, 16, 16, 4, 7, 10.0, 0.001, 2000.0, 0, p.StencilTile(), 1.0)
    out = ctypes.c_void_p()
    assert p._lib.stencil_init(ctypes.byref(d), ctypes.byref(out)) == p.EUNSUPPORTED
    for st in ("f16", "bf16"):
        ctx = _init(storage=st, storage_scale=1024.0)
        assert p.stencil_get_tile(ctx).vw == 4
        p.stencil_destroy(ctx)
        with pytest.raises(p.StencilError) as e:
            _init(storage=st, radius=3)  # 16-bit kernels exist for R = 4, 5
        assert e.value.status == p.EUNSUPPORTED
        with pytest.raises(p.StencilError) as e:
            _init(storage=st, storage_scale=3.0)  # not a power of two
        assert e.value.status == p.EINVAL
        assert len(p.stencil_list_tiles(4, True, st)) >= 5
        assert len(p.stencil_list_tiles(5, False, st)) >= 1
    assert len(p.stencil_list_tiles(3, True, "f16")) == 0


def test_tiles_default_set_and_reject():
    ctx = _init(nx=64, ny=48, nz=40)
    t = p.stencil_get_tile(ctx)
    assert t.kind == p.TILE_ZMARCH and t.vw == 4 and t.dz >= 1
    tiles = p.stencil_list_tiles(4, True)
    assert len(tiles) >= 10
    for tt in tiles:
        tt.dz = 16
        p.stencil_set_tile(ctx, tt)
        got = p.stencil_get_tile(ctx)
        assert (got.bx, got.by, got.ry, got.vw, got.pf, got.dz) == (tt.bx, tt.by, tt.ry, tt.vw, tt.pf, 16)
    before = p.stencil_get_tile(ctx)
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, p.make_tile(bx=7, by=3, ry=1, dz=8, vw=4))
    assert e.value.status == p.EUNSUPPORTED
    assert p.stencil_get_tile(ctx).as_dict() == before.as_dict()
    with pytest.raises(p.StencilError):
        p.stencil_set_tile(ctx, p.make_tile(p.TILE_PLAIN, bx=64, by=32, dz=1))  # 2048 threads
    p.stencil_set_tile(ctx, p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=2))
    p.stencil_destroy(ctx)
    # nx % 4 != 0: vector tiles are refused, the default falls back to vw = 1.
    ctx = _init(nx=61, ny=45, nz=37)
    assert p.stencil_get_tile(ctx).vw == 1
    with pytest.raises(p.StencilError):
        p.stencil_set_tile(ctx, p.make_tile(bx=16, by=8, ry=2, dz=16, vw=4))
    p.stencil_destroy(ctx)


def test_step_argument_errors_before_launch():
    # Validation runs before any HIP call, so fake pointers exercise it on the CPU.
    ctx = _init(nx=16, ny=16, nz=16)
    n = 16 ** 3 * 4
    base = 1 << 40
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base, base + 2 * n, base + 2 * n + 64, 0, None, 0)
    assert e.value.status == p.EALIAS
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base + 2 * n, base, base + n // 2, 0, None, 0)
    assert e.value.status == p.EALIAS
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base, base + 4 * n + 4, base + 8 * n, 0, None, 0)
    assert e.value.status == p.EINVAL  # misaligned for vw = 4
    src = p.StencilSrc(1, base + 64 * n, base + 65 * n, 5)
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base, base + 2 * n, base + 4 * n, 5, src, 0)
    assert e.value.status == p.EINVAL  # it >= nt
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, 0, base + 2 * n, base + 4 * n, 0, None, 0)
    assert e.value.status == p.EINVAL
    assert "null" in p.stencil_last_error(ctx)
    with pytest.raises(p.StencilError) as e:
        p.stencil_tune(ctx, base, base, base + 4 * n, stream=0)
    assert e.value.status == p.EALIAS
    p.stencil_destroy(ctx)


def test_stream_probe_validation():
    with pytest.raises(p.StencilError):
        p.stencil_stream_probe(1 << 40, None, None, (1 << 40) + 4096, 102, stream=0)
    with pytest.raises(p.StencilError):
        p.stencil_stream_probe(1 << 40, None, (1 << 40) + 8192, (1 << 40) + 4096, 4096, stream=0)


def test_two_step_tile_and_validation():
    ctx = _init(nx=64, ny=48, nz=40)
    t2 = p.stencil_get_tile2(ctx)
    assert t2.kind == p.TILE_ZMARCH2 and t2.vw == 4 and t2.ry == 1
    tiles = p.stencil_list_tiles2(4, True)
    assert len(tiles) >= 3
    for tt in tiles:
        tt.dz = 8
        p.stencil_set_tile(ctx, tt)
        g = p.stencil_get_tile2(ctx)
        assert (g.bx, g.by, g.dz) == (tt.bx, tt.by, 8)
    assert p.stencil_get_tile(ctx).kind == p.TILE_ZMARCH  # the one-step tile is unchanged
    # pf bits 1-3: edge pacing codes 0..7 on any compiled two-step shape;
    # larger values are refused.
    tt = tiles[0]
    for pf in (tt.pf | (5 << 1), tt.pf | (7 << 1)):
        tt.pf = pf
        p.stencil_set_tile(ctx, tt)
        assert p.stencil_get_tile2(ctx).pf == pf
    tt.pf = 16
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, tt)
    assert e.value.status == p.EUNSUPPORTED
    n = 64 * 48 * 40 * 4
    base = 1 << 40
    k, a, b, c, d = (base + i * 2 * n for i in range(5))
    with pytest.raises(p.StencilError) as e:
        p.stencil_step2(ctx, k, a, b, a + 64, d, 0, None, 0)  # output overlaps an input
    assert e.value.status == p.EALIAS
    with pytest.raises(p.StencilError) as e:
        p.stencil_step2(ctx, k, a, b, c, c, 0, None, 0)       # both outputs the same buffer
    assert e.value.status == p.EALIAS
    src3 = p.StencilSrc(3, base + 64 * n, base + 65 * n, 10)
    with pytest.raises(p.StencilError) as e:
        p.stencil_step2(ctx, k, a, b, c, d, 0, src3, 0)
    assert e.value.status == p.EUNSUPPORTED
    src1 = p.StencilSrc(1, base + 64 * n, base + 65 * n, 10)
    with pytest.raises(p.StencilError) as e:
        p.stencil_step2(ctx, k, a, b, c, d, 9, src1, 0)        # step it+1 = 10 has no sample
    assert e.value.status == p.EINVAL
    p.stencil_destroy(ctx)
    # No two-step kernels for 16-bit storage: the context reports it.
    ctx = _init(storage="f16")
    with pytest.raises(p.StencilError) as e:
        p.stencil_get_tile2(ctx)
    assert e.value.status == p.EUNSUPPORTED
    p.stencil_destroy(ctx)


def test_vector_width_follows_nx():
    # nx % 4 == 2: two-point tiles by default, four-point tiles rejected;
    # odd nx: one-point tiles only. Alignment is checked per vector width.
    ctx = _init(nx=70, ny=20, nz=12)
    assert p.stencil_get_tile(ctx).vw == 2
    two = p.stencil_list_tiles(4, 2)
    assert len(two) >= 5 and all(t.vw == 2 for t in two)
    for t in two:
        t.dz = 8
        p.stencil_set_tile(ctx, t)
        assert p.stencil_get_tile(ctx).vw == 2
    four = p.stencil_list_tiles(4, True)[0]
    four.dz = 8
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, four)
    assert e.value.status == p.EUNSUPPORTED and "divide" in p.stencil_last_error(ctx)
    n = 70 * 20 * 12 * 4
    base = 1 << 40
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base, base + 2 * n + 4, base + 4 * n, 0, None, 0)
    assert e.value.status == p.EINVAL  # one value off for vw = 2
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base + 4, base + 2 * n, base + 4 * n, 0, None, 0)
    assert e.value.status == p.EINVAL  # kappa not 8-byte aligned
    p.stencil_destroy(ctx)
    ctx = _init(nx=71, ny=20, nz=12)
    assert p.stencil_get_tile(ctx).vw == 1
    two[0].dz = 8
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, two[0])
    assert e.value.status == p.EUNSUPPORTED
    p.stencil_destroy(ctx)
    # 16-bit storage has no two-point kernels: nx % 4 == 2 falls back to one.
    ctx = _init(nx=70, ny=20, nz=12, storage="f16", storage_scale=1024.0)
    assert p.stencil_get_tile(ctx).vw == 1
    p.stencil_destroy(ctx)


def test_pitch_validation_and_vector_width():
    # pitch >= nx; vector tiles need vw to divide nx and the pitch; sizes
    # checked against the padded rows; 0 means nx.
    with pytest.raises(p.StencilError) as e:
        _init(nx=64, pitch=63)
    assert e.value.status == p.EINVAL
    with pytest.raises(p.StencilError) as e:
        _init(nx=4096, ny=8192, nz=4, pitch=65536 + 4096)  # a plane of pitch * ny values over 2^29
    assert e.value.status == p.EINVAL
    for nx, pitch, vw in ((250, 256, 2), (200, 224, 4), (200, 226, 2), (61, 64, 1), (64, 0, 4)):
        ctx = _init(nx=nx, ny=20, nz=12, pitch=pitch)
        assert p.stencil_get_tile(ctx).vw == vw, (nx, pitch)
        if vw < 4:
            four = p.stencil_list_tiles(4, True)[0]
            four.dz = 8
            with pytest.raises(p.StencilError) as e:
                p.stencil_set_tile(ctx, four)
            assert e.value.status == p.EUNSUPPORTED
        p.stencil_destroy(ctx)
    # Field sizes follow the pitch: u_cur overlapping the padded u_prev is an alias.
    ctx = _init(nx=250, ny=20, nz=12, pitch=256)
    n = 256 * 20 * 12 * 4
    base = 1 << 40
    with pytest.raises(p.StencilError) as e:
        p.stencil_step(ctx, base, base + 2 * n, base + 2 * n + 250 * 20 * 12 * 4, 0, None, 0)
    assert e.value.status == p.EALIAS
    p.stencil_destroy(ctx)


def test_eight_point_tiles_for_16bit_storage():
    # 16-bit storage has eight-point tiles (one 16-byte access per lane) for
    # nx % 8 == 0; FP32 storage has none.
    assert p.stencil_list_tiles(4, 8, "f32") == []
    for st in ("f16", "bf16"):
        eight = p.stencil_list_tiles(4, 8, st)
        assert len(eight) >= 4 and all(t.vw == 8 for t in eight)
        ctx = _init(nx=64, ny=20, nz=12, storage=st, storage_scale=1024.0)
        for t in eight:
            t.dz = 8
            p.stencil_set_tile(ctx, t)
            assert p.stencil_get_tile(ctx).vw == 8
        p.stencil_destroy(ctx)
        ctx = _init(nx=68, ny=20, nz=12, storage=st, storage_scale=1024.0)
        eight[0].dz = 8
        with pytest.raises(p.StencilError) as e:
            p.stencil_set_tile(ctx, eight[0])
        assert e.value.status == p.EUNSUPPORTED
        p.stencil_destroy(ctx)


def test_gradient2_validation():
    ctx = _init(nx=16, ny=16, nz=16)
    n = 16 ** 3 * 4
    base = 1 << 40
    f = [base + i * 2 * n for i in range(6)]
    g = base + 20 * n
    with pytest.raises(p.StencilError) as e:
        p.stencil_gradient2(ctx, *f, f[3] + 8, stream=0)  # grad overlaps u^{k-1}
    assert e.value.status == p.EALIAS
    with pytest.raises(p.StencilError) as e:
        p.stencil_gradient2(ctx, f[0], 0, *f[2:], g, stream=0)
    assert e.value.status == p.EINVAL
    p.stencil_destroy(ctx)
    ctx = _init(nx=16, ny=16, nz=16, storage="f16", storage_scale=1024.0)
    with pytest.raises(p.StencilError) as e:
        p.stencil_gradient2(ctx, *f, g, stream=0)
    assert e.value.status == p.EUNSUPPORTED
    p.stencil_destroy(ctx)


def test_c_program_links_and_checks_arguments():
    # The C program that uses the ABI without Python: built by build(); with
    # wrong arguments it exits with status 2 before touching the GPU.
    import subprocess
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "_build", "plain_method")
    if not os.path.exists(exe):
        pytest.skip("C program not built")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=30)
    assert r.returncode == 2 and "usage" in r.stderr


def test_stream_probe_march_validation():
    base = 1 << 40
    n = 8 * 8 * 8 * 4
    for args in ((base, base + n, base + 2 * n, base + 3 * n, 6, 8, 8),   # nx % 4
                 (base, base + n, base + 2 * n, base + 3 * n + 4, 8, 8, 8),  # alignment
                 (base, 0, base + 2 * n, base + 3 * n, 8, 8, 8)):  # null input
        assert p._lib.stencil_stream_probe_march(*args, None) == p.EINVAL
    assert p._lib.stencil_stream_probe_march(base, base + n, base + 2 * n, base + n + 16, 8, 8, 8, None) == p.EALIAS


def test_large_planes_fall_back_to_plain_tiling():
    # A z-march window of dz + 2R planes must stay below 2 GiB: with
    # 16384 x 16384 planes (1 GiB each) no z-march tile fits, the default is
    # plain tiling, and z-march tiles are rejected with a clear message.
    ctx = _init(nx=16384, ny=16384, nz=4)
    t = p.stencil_get_tile(ctx)
    assert t.kind == p.TILE_PLAIN
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, p.make_tile(p.TILE_ZMARCH, bx=64, by=4, ry=1, dz=1, vw=4))
    assert e.value.status == p.EUNSUPPORTED and "2 GiB" in p.stencil_last_error(ctx)
    p.stencil_destroy(ctx)
    # 4096 x 4096 planes (64 MiB): dz + 8 planes fit up to dz = 23; the
    # default tile takes that depth and deeper tiles are rejected.
    ctx = _init(nx=4096, ny=4096, nz=64)
    t = p.stencil_get_tile(ctx)
    assert t.kind == p.TILE_ZMARCH and t.dz == 23
    p.stencil_set_tile(ctx, p.make_tile(p.TILE_ZMARCH, bx=64, by=4, ry=1, dz=23, vw=4))
    with pytest.raises(p.StencilError):
        p.stencil_set_tile(ctx, p.make_tile(p.TILE_ZMARCH, bx=64, by=4, ry=1, dz=24, vw=4))
    p.stencil_destroy(ctx)


def test_make_src_validates_and_keeps_its_tensors():
    import torch
    with pytest.raises(ValueError):
        p.make_src(torch.zeros(1, dtype=torch.int64), torch.zeros(4, 1))  # CPU tensors
    # The source object keeps the tensors alive (the C struct holds raw
    # device pointers); checked here on the reference it stores.
    src = p.StencilSrc(0, None, None, 0)
    src._keep = ("idx", "amp")
    assert src._keep == ("idx", "amp")


def test_launch_size_limits():
    # 4096 x 4096 x 300 (5e9 points): a one-point-per-thread tile marching one
    # plane per workgroup would need over 2^32 work-items, which one dispatch
    # cannot hold; two rows per thread (or a deeper march) fits.
    ctx = _init(nx=4096, ny=4096, nz=300)
    one_row = [t for t in p.stencil_list_tiles(4, False) if t.ry == 1]
    two_rows = [t for t in p.stencil_list_tiles(4, False) if t.ry == 2]
    assert one_row and two_rows
    t = one_row[0]
    t.dz = 1
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, t)
    assert e.value.status == p.EUNSUPPORTED and "work-items" in p.stencil_last_error(ctx)
    t.dz = 2
    p.stencil_set_tile(ctx, t)
    t = two_rows[0]
    t.dz = 1
    p.stencil_set_tile(ctx, t)
    # The two-step kernel with one point per thread: 24 x 8 own points per
    # 512-thread workgroup.
    t2 = [t for t in p.stencil_list_tiles2(4, False)][0]
    t2.dz = 1
    with pytest.raises(p.StencilError) as e:
        p.stencil_set_tile(ctx, t2)
    assert e.value.status == p.EUNSUPPORTED
    t2.dz = 8
    p.stencil_set_tile(ctx, t2)
    p.stencil_destroy(ctx)


def test_step2_rejects_negative_source_count():
    ctx = _init(nx=64, ny=48, nz=40)
    n = 64 * 48 * 40 * 4
    base = 1 << 40
    k, a, b, c, d = (base + i * 2 * n for i in range(5))
    with pytest.raises(p.StencilError) as e:
        p.stencil_step2(ctx, k, a, b, c, d, 0, p.StencilSrc(-1, base + 64 * n, base + 65 * n, 10), 0)
    assert e.value.status == p.EINVAL
    p.stencil_destroy(ctx)


def test_batch_rejects_buffers_shared_between_shots():
    # Fake device pointers: validation happens before any HIP call, and with
    # plain tiles a batch holds no device table, so even a valid batch is
    # created and destroyed on the CPU.
    ctxs = [_init(nx=32, ny=32, nz=32) for _ in range(2)]
    for c in ctxs:
        p.stencil_set_tile(c, p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1))
    n = 32 ** 3 * 4
    base = 1 << 40
    f = [base + i * 2 * n for i in range(8)]
    ok = [(ctxs[0], f[0], f[1], f[2], None), (ctxs[1], f[0], f[3], f[4], None)]  # one kappa for both
    p.stencil_batch_destroy(p.stencil_batch_create(ok))
    bad = [
        [(ctxs[0], f[0], f[1], f[2], None), (ctxs[1], f[5], f[2], f[4], None)],           # same u buffer
        [(ctxs[0], f[0], f[1], f[2], None), (ctxs[1], f[5], f[3], f[1] + 64, None)],      # partial overlap
        [(ctxs[0], f[0], f[1], f[2], None), (ctxs[1], f[1], f[3], f[4], None)],           # kappa is another's u
        [(ctxs[0], f[5], f[1], f[2], None), (ctxs[1], f[0], f[5] + 256, f[4], None)],     # u is another's kappa
    ]
    for shots in bad:
        with pytest.raises(p.StencilError) as e:
            p.stencil_batch_create(shots)
        assert e.value.status == p.EALIAS
        with pytest.raises(p.StencilError) as e:
            p.stencil_batch_tune(shots, stream=0)
        assert e.value.status == p.EALIAS
    for c in ctxs:
        p.stencil_destroy(c)


def test_static_batch_table_limit():
    # The static-table batch refuses a descriptor table larger than its
    # 64 KiB array before any device call (fake pointers); a batch of plain
    # tiles needs no table and is created on the CPU.
    n_shots = 300
    ctxs = [_init(nx=8, ny=8, nz=8) for _ in range(n_shots)]
    assert p.stencil_get_tile(ctxs[0]).kind == p.TILE_ZMARCH
    fb = 8 ** 3 * 4
    base = 1 << 40
    shots = [(c, base + 3 * i * fb, base + (3 * i + 1) * fb, base + (3 * i + 2) * fb, None)
             for i, c in enumerate(ctxs)]
    with pytest.raises(p.StencilError) as e:
        p.stencil_batch_create_static(shots)
    assert e.value.status == p.EINVAL and "static table holds 65536" in str(e.value)
    for c in ctxs[:2]:
        p.stencil_set_tile(c, p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1))
    p.stencil_batch_destroy(p.stencil_batch_create_static(shots[:2]))
    for c in ctxs:
        p.stencil_destroy(c)


def test_static_batch_table_boundary():
    # 224 z-march shots of one tile shape fill the 64 KiB table exactly
    # (two parity tables of 224 x 144 B and 224 first-workgroup ints, each
    # rounded up to 256 B); 225 are refused before any device call. Without
    # a GPU the 224-shot batch passes the size check and then fails at the
    # table's device address instead.
    ctxs = [_init(nx=8, ny=8, nz=8) for _ in range(225)]
    fb = 8 ** 3 * 4
    base = 1 << 40
    shots = [(c, base + 3 * i * fb, base + (3 * i + 1) * fb, base + (3 * i + 2) * fb, None)
             for i, c in enumerate(ctxs)]
    with pytest.raises(p.StencilError) as e:
        p.stencil_batch_create_static(shots)
    assert e.value.status == p.EINVAL and "needs 66048 bytes" in str(e.value)
    try:
        p.stencil_batch_destroy(p.stencil_batch_create_static(shots[:224]))
    except p.StencilError as err:
        assert "static table holds" not in str(err), str(err)
    for c in ctxs:
        p.stencil_destroy(c)


@pytest.mark.parametrize("policy", ["worst", "min", "avg", "ob"])
def test_select_skips_failed_candidates(policy):
    # A candidate whose launch failed is timed as +inf. As long as every
    # replicate has one finite entry, no rule picks a failed candidate, and the
    # library agrees with the oracle's rule.
    rng = np.random.default_rng(19)
    for _ in range(200):
        nn, nk, nc = (int(rng.integers(1, 3)), int(rng.integers(1, 5)), int(rng.integers(2, 7)))
        t = rng.random(size=(nn, nk, nc)) + 1.0
        t[rng.random(size=t.shape) < 0.4] = np.inf
        for i in range(nn):
            for k in range(nk):
                if not np.isfinite(t[i, k]).any():
                    t[i, k, int(rng.integers(0, nc))] = 1.5
        ids = [list(range(i * nc, (i + 1) * nc)) for i in range(nn)]
        got = p.stencil_select(t.tolist(), policy)
        assert got == oracle.select_block(t.tolist(), ids, policy)
        assert np.isfinite(got[1])


def _entry(rest, bid=None):
    return f"v2 {bid or p.stencil_build_id()} {rest}\n"


def test_tune_cache_entries_at_init(tmp_path, monkeypatch):
    # stencil_init takes the last matching line of STENCIL_TUNE_CACHE; lines
    # that do not parse, belong to another grid, radius or storage, or name a
    # tile no compiled kernel runs are ignored or fall back to the default.
    cache = tmp_path / "cache.txt"
    monkeypatch.setenv("STENCIL_TUNE_CACHE", str(cache))
    ctx = _init(nx=64, ny=48, nz=40)
    default = p.stencil_get_tile(ctx).as_dict()
    p.stencil_destroy(ctx)
    cache.write_text("garbage line\n" +
                     _entry("R4 f32 64 48 41 64 2 32 8 1 16 4 1 0 1.0 1.0") +    # another grid
                     _entry("R4 f32 64 48 40 128 2 32 8 1 16 4 1 0 1.0 1.0") +   # another row pitch
                     _entry("R5 f32 64 48 40 64 2 32 8 1 16 4 1 0 1.0 1.0") +    # another radius
                     _entry("R4 f16 64 48 40 64 2 32 8 1 16 4 1 0 1.0 1.0") +    # another storage
                     _entry("R4 f32 64 48 40 64 3 18 40 1 16 4 1 0 1.0 1.0"))    # a two-step entry
    ctx = _init(nx=64, ny=48, nz=40)
    assert p.stencil_get_tile(ctx).as_dict() == default
    p.stencil_destroy(ctx)
    with open(cache, "a") as f:
        f.write(_entry("R4 f32 64 48 40 64 2 32 8 1 16 4 1 0 1.0 1.0"))
    ctx = _init(nx=64, ny=48, nz=40)
    t = p.stencil_get_tile(ctx)
    assert (t.kind, t.bx, t.by, t.ry, t.dz, t.vw, t.pf) == (p.TILE_ZMARCH, 32, 8, 1, 16, 4, 0)
    p.stencil_destroy(ctx)
    with open(cache, "a") as f:
        f.write(_entry("R4 f32 64 48 40 64 2 7 3 1 16 4 1 0 1.0 1.0"))  # no such kernel: default
    ctx = _init(nx=64, ny=48, nz=40)
    assert p.stencil_get_tile(ctx).as_dict() == default
    p.stencil_destroy(ctx)


def test_build_id_names_arch_versions_and_source_hash():
    bid = p.stencil_build_id()
    arch, hip, rt, src = bid.split("/")
    assert arch == "gfx950" and hip.startswith("hip") and rt.startswith("rt")
    import importlib.util
    spec = importlib.util.spec_from_file_location("_p1310_build", os.path.join(ROOT, "paper_1310_8232_amd", "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    # The library was built from the sources in the tree.
    assert src == "src" + b.source_hash()


def _tune_from_cache_only(ctx, cache):
    # Fake, non-overlapping, aligned field addresses: the call either returns
    # a cache entry (no device work) or goes on to the device, which the
    # context's device number 1000 does not name (EDEVICE before any launch).
    n = 64 * 48 * 40 * 4
    base = 1 << 40
    rep = p.StencilTuneReport()
    opts = p.StencilTuneOpts()
    opts.cache_path = str(cache).encode()
    st = p._lib.stencil_tune(ctx, base, base + n, base + 2 * n, ctypes.byref(opts), ctypes.byref(rep), None)
    return st, rep


def test_tune_cache_ignores_entries_of_other_builds(tmp_path, monkeypatch):
    # An entry measured with other code (another source hash, compiler or
    # runtime version, or the unversioned format) is stale: neither init nor
    # stencil_tune takes it.
    cache = tmp_path / "cache.txt"
    bid = p.stencil_build_id()
    arch, hip, rt, src = bid.split("/")
    stale = [f"{arch}/{hip}/{rt}/src0123456789abcdef", f"{arch}/hip1/{rt}/{src}", f"{arch}/{hip}/rt1/{src}",
             f"gfx942/{hip}/{rt}/{src}"]
    good = "R4 f32 64 48 40 64 2 32 8 1 16 4 1 0 1.0 1.0"
    cache.write_text("".join(_entry(good, b) for b in stale) + "gfx950 " + good + "\n")
    monkeypatch.setenv("STENCIL_TUNE_CACHE", str(cache))
    monkeypatch.delenv("STENCIL_LOG", raising=False)
    ctx = _init(nx=64, ny=48, nz=40, device=1000)
    t = p.stencil_get_tile(ctx)
    assert (t.bx, t.by, t.dz) != (32, 8, 16)  # the built-in default, not the stale tile
    st, rep = _tune_from_cache_only(ctx, cache)
    assert st == p.EDEVICE and rep.from_cache == 0
    p.stencil_destroy(ctx)
    # The same entry under this build's id is taken by both.
    with open(cache, "a") as f:
        f.write(_entry(good))
    ctx = _init(nx=64, ny=48, nz=40, device=1000)
    t = p.stencil_get_tile(ctx)
    assert (t.bx, t.by, t.dz) == (32, 8, 16)
    st, rep = _tune_from_cache_only(ctx, cache)
    assert st == p.OK and rep.from_cache == 1 and (rep.tile.bx, rep.tile.by, rep.tile.dz) == (32, 8, 16)
    p.stencil_destroy(ctx)


def test_log_lines_on_request(monkeypatch, capfd):
    monkeypatch.delenv("STENCIL_LOG", raising=False)
    p.stencil_destroy(_init(nx=64, ny=48, nz=40))
    assert "stencil:" not in capfd.readouterr().err
    monkeypatch.setenv("STENCIL_LOG", "1")
    ctx = _init(nx=64, ny=48, nz=40, tile=p.make_tile(bx=32, by=8, ry=1, dz=16))
    err = capfd.readouterr().err
    assert "stencil: init 64x48x40 R4 f32" in err and "zmarch 32x8 ry1 dz16 vw4" in err and "(given)" in err
    p.stencil_destroy(ctx)
    monkeypatch.setenv("STENCIL_LOG", "0")
    p.stencil_destroy(_init(nx=64, ny=48, nz=40))
    assert "stencil:" not in capfd.readouterr().err


def test_max_abs_validation():
    ctx = _init(nx=16, ny=16, nz=16)
    base = 1 << 40
    n = 16 ** 3 * 4
    with pytest.raises(p.StencilError) as e:
        p._check(p._lib.stencil_max_abs(ctx, None, base, 0), ctx)
    assert e.value.status == p.EINVAL
    with pytest.raises(p.StencilError) as e:
        p._check(p._lib.stencil_max_abs(ctx, base, base + n // 2, 0), ctx)
    assert e.value.status == p.EALIAS
    assert "diverged" in p.stencil_strerror(p.EDIVERGED)
    p.stencil_destroy(ctx)


def test_gradient_terms_validation():
    ctx = _init(nx=16, ny=16, nz=16)
    base = 1 << 40
    n = 16 ** 3 * 4
    f = [base + i * 2 * n for i in range(10)]
    g = base + 64 * n
    for m in (0, 5):
        mu = (p._vp * max(m, 1))(*f[:max(m, 1)])
        u = (p._vp * (m + 2))(*f[4:4 + m + 2])
        with pytest.raises(p.StencilError) as e:
            p._check(p._lib.stencil_gradient_terms(ctx, m, mu, u, g, 0), ctx)
        assert e.value.status == p.EINVAL
    with pytest.raises(p.StencilError) as e:
        p.stencil_gradient_terms(ctx, f[:2], f[4:8], f[5] + 8, stream=0)  # grad inside a field
    assert e.value.status == p.EALIAS
    with pytest.raises(ValueError):
        p.stencil_gradient_terms(ctx, f[:2], f[4:7], g, stream=0)
    p.stencil_destroy(ctx)
