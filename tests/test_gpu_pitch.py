"""Padded rows (stencil_desc.pitch): every field stored as [nz, ny, pitch]
with the grid in the first nx values of each row. The grid points must get
the bits of the unpadded run on every tile (so the oracle comparison of the
unpadded run carries over), and the padding must never be read as a grid
point nor written: it is filled with NaN here and must stay NaN while no NaN
reaches a grid point."""
import sys

import numpy as np
import pytest
import torch

import oracle
from compare import check_close
import paper_1310_8232_amd as p
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def _padded(a, pitch, fill=np.nan):
    nz, ny, nx = a.shape
    out = np.full((nz, ny, pitch), fill, dtype=np.float32)
    out[..., :nx] = a
    return out


def _case(nx, ny, nz, seed):
    v = workloads.layered_model(nx, ny, nz, seed=seed)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    return v, dt, vmax, workloads.random_field(nx, ny, nz, seed + 1), workloads.random_field(nx, ny, nz, seed + 2)


def _run(v, dt, vmax, R, nt, u0, um1, tile=None, pitch=None, src=None):
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax, tile=tile, pitch=pitch)
    if prop.pitch != v.shape[2]:
        a, b = cuda(_padded(u0, prop.pitch)), cuda(_padded(um1, prop.pitch))
    else:
        a, b = cuda(u0), cuda(um1)
    a, b = prop.run(a, b, nt, src)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), prop


def _tiles(R, vw_ok):
    out = []
    for w in (4, 2, 1):
        if not vw_ok(w):
            continue
        for t in p.stencil_list_tiles(R, {4: 1, 2: 2, 1: 0}[w]):
            for dz in (7, 64):
                out.append(p.make_tile(p.TILE_ZMARCH, t.bx, t.by, t.ry, dz, t.vw, 1, t.pf))
    out.append(p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1))
    return out


@pytest.mark.parametrize("R,shape,pitch", [(4, (250, 29, 23), 256), (5, (200, 45, 37), 224),
                                           (3, (61, 29, 23), 64), (4, (70, 20, 12), 96),
                                           (5, (300, 17, 40), "align")])
def test_padded_rows_give_the_unpadded_bits(R, shape, pitch):
    nx, ny, nz = shape
    v, dt, vmax, u0, um1 = _case(nx, ny, nz, seed=500 + R)
    nt = 6
    ref_n, ref_nm1, _ = _run(v, dt, vmax, R, nt, u0, um1)
    kap = oracle.kappa(v, dt, 10.0)
    o_n, o_nm1 = oracle.leapfrog(kap, u0, um1, R, nt)
    check_close(ref_n, o_n, 1e-5, "unpadded u^n")
    check_close(ref_nm1, o_nm1, 1e-5, "unpadded u^n-1")
    prop0 = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax, pitch=pitch)
    P = prop0.pitch
    log(f"case: {nx}x{ny}x{nz} R={R} pitch {P}, {nt} steps, every tile")
    tiles = [None] + _tiles(R, lambda w: nx % w == 0 and P % w == 0)
    for t in tiles:
        un, unm1, prop = _run(v, dt, vmax, R, nt, u0, um1, tile=t, pitch=P)
        assert un.shape == (nz, ny, P)
        assert np.array_equal(un[..., :nx], ref_n) and np.array_equal(unm1[..., :nx], ref_nm1), f"tile {prop.tile}"
        assert np.all(np.isnan(un[..., nx:])) and np.all(np.isnan(unm1[..., nx:])), f"padding written, {prop.tile}"
    log(f"  {len(tiles)} tiles: grid bits equal the unpadded run, padding untouched")


def test_padded_sources_receivers_two_step_and_search():
    nx, ny, nz, P = 250, 40, 36, 256
    v, dt, vmax, _, _ = _case(nx, ny, nz, seed=610)
    nt = 20
    pts = [(18, 20, 125), (5, 3, 249), (30, 39, 0)]
    amp = np.stack([workloads.ricker(nt, dt, 20.0 + 5 * j) for j in range(4)], 1)
    log("case: padded 250x40x36 (pitch 256): sources, receivers, two-step launches, search")
    z = np.zeros((nz, ny, nx), np.float32)

    def src_for(prop, idx):
        keep = (cuda(np.array(idx, np.int64), torch.int64), cuda(amp[:, : len(idx)]))
        return p.make_src(*keep), keep

    # Unpadded reference with three sources.
    prop_u = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    s_u, keep_u = src_for(prop_u, [prop_u.index(*q) for q in pts])
    ref = prop_u.run(prop_u.zeros(), prop_u.zeros(), nt, s_u)
    # Padded: the same points by their padded index, plus one index in a
    # row's padding, which is skipped.
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, pitch=P)
    pad_idx = prop.index(10, 10, 0) - 3  # x = 253 of row (10, 9)
    s_p, keep_p = src_for(prop, [prop.index(*q) for q in pts] + [pad_idx])
    got = prop.run(prop.zeros(), prop.zeros(), nt, s_p)
    torch.cuda.synchronize()
    for r, g in zip(ref, got):
        assert torch.equal(prop.grid(g), r)
        assert torch.count_nonzero(g[..., nx:]) == 0
    # Receivers: padded indices sample the same values; one in padding gives 0.
    rec_u = cuda(np.array([prop_u.index(*q) for q in pts], np.int64), torch.int64)
    rec_p = cuda(np.array([prop.index(*q) for q in pts] + [pad_idx], np.int64), torch.int64)
    out_u = torch.empty(3, device="cuda:0")
    out_p = torch.full((4,), 7.0, device="cuda:0")
    p.stencil_sample(prop_u.ctx, ref[0], rec_u, out_u)
    p.stencil_sample(prop.ctx, got[0], rec_p, out_p)
    torch.cuda.synchronize()
    assert torch.equal(out_p[:3], out_u) and float(out_p[3]) == 0.0
    # Two steps per launch on padded rows (they take one source, fused): the
    # bits of one-step launches.
    s_1, keep_1 = src_for(prop, [prop.index(*pts[0])])
    one = prop.run(prop.zeros(), prop.zeros(), nt, s_1)
    two = prop.run(prop.zeros(), prop.zeros(), nt, s_1, temporal=2)
    torch.cuda.synchronize()
    for o, t in zip(one, two):
        assert torch.equal(o, t)
    # The search runs on padded rows; its tile gives the same bits.
    rep, _, _ = prop.tune(n_iter=2, n_rep=1)
    again = prop.run(prop.zeros(), prop.zeros(), nt, s_p)
    torch.cuda.synchronize()
    log(f"  searched tile {rep['tile']}")
    for g, a in zip(got, again):
        assert torch.equal(g, a)
    del keep_u, keep_p, keep_1, z


def test_padded_shot_in_a_batch():
    nt = 12
    shots = []
    for i, (shape, pitch) in enumerate((((250, 30, 20), 256), ((64, 32, 24), None), ((200, 24, 16), 224))):
        nx, ny, nz = shape
        v = workloads.layered_model(nx, ny, nz, seed=700 + i)
        dt, vmax = workloads.dt_for_courant(v, 10.0)
        prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, pitch=pitch)
        keep = (cuda(np.array([prop.index(nz // 2, ny // 2, nx // 2)], np.int64), torch.int64),
                cuda(workloads.ricker(nt, dt).reshape(-1, 1)))
        shots.append((prop, p.make_src(*keep), keep))
    log("case: batch with padded and unpadded shots")
    batch = p.Batch([(pr, s) for pr, s, _ in shots])
    batch.run(nt)
    torch.cuda.synchronize()
    for (pr, s, _), (bn, bnm1) in zip(shots, batch.current(nt)):
        a, b = pr.run(pr.zeros(), pr.zeros(), nt, s)
        torch.cuda.synchronize()
        assert torch.equal(a, bn) and torch.equal(b, bnm1)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_padded_rows_16bit_storage(storage):
    # 16-bit wavefields with rows padded to 128 bytes (64 values): grid bits
    # equal the unpadded run's for the default tile and every 16-bit tile.
    nx, ny, nz = 200, 30, 26
    v, dt, vmax, u0, um1 = _case(nx, ny, nz, seed=800)
    nt = 5
    log(f"case: {storage} storage, {nx}x{ny}x{nz}, rows padded to 128 bytes")

    def run(pitch, tile):
        prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, storage=storage, storage_scale=256.0, pitch=pitch,
                            tile=tile)
        P = prop.pitch
        a = prop.to_storage(cuda(_padded(u0, P, 0.0) if P != nx else u0))
        b = prop.to_storage(cuda(_padded(um1, P, 0.0) if P != nx else um1))
        a, b = prop.run(a, b, nt)
        torch.cuda.synchronize()
        return prop.grid(a).cpu(), prop.grid(b).cpu(), P

    ref = run(None, None)
    assert run("align", None)[2] == 256
    tiles = [None] + [p.make_tile(p.TILE_ZMARCH, t.bx, t.by, t.ry, 8, t.vw, 1, t.pf)
                      for w in (1, 8) for t in p.stencil_list_tiles(4, w, storage)]
    for t in tiles:
        got = run("align", t)
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), f"tile {t}"


def test_padded_rows_one_point_two_step_and_gradient():
    # nx = 61 with rows of 64: one-point vectors; the one-point two-step tile
    # gives the one-step bits; the misfit gradient on padded fields equals the
    # unpadded gradient at every grid point (padding stays 0).
    from paper_1310_8232_amd import adjoint
    nx, ny, nz, nt = 61, 29, 23, 30
    c = workloads.config_gradient(nx, ny, nz, nt=nt)
    log("case: 61x29x23 rows of 64: one-point two-step tile, misfit gradient")
    out = {}
    for pitch in (None, 64):
        prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True, pitch=pitch)
        src_idx = [prop.index(*np.unravel_index(int(s), (nz, ny, nx))) for s in c["src_idx"]]
        rec_idx = [prop.index(*np.unravel_index(int(r), (nz, ny, nx))) for r in c["rec_idx"]]
        survey = adjoint.Survey(cuda(np.array(src_idx, np.int64), torch.int64), cuda(c["amp"].reshape(-1, 1)),
                                cuda(np.array(rec_idx, np.int64), torch.int64))
        s = survey.src()
        one = prop.run(prop.zeros(), prop.zeros(), nt, s)
        prop.tile = p.make_tile(p.TILE_ZMARCH2, 32, 16, 1, 8, 1, 1, 0)
        two = prop.run(prop.zeros(), prop.zeros(), nt, s, temporal=2)
        torch.cuda.synchronize()
        for o, t in zip(one, two):
            assert torch.equal(o, t), f"pitch {pitch}"
        obs = torch.zeros((nt, len(rec_idx)), device="cuda:0")
        J, g, tr = adjoint.misfit_gradient(prop, survey, obs, checkpoint_every=7)
        torch.cuda.synchronize()
        out[pitch] = (J.item(), prop.grid(g).cpu(), tr.cpu(), g.cpu())
    assert out[None][0] == out[64][0]
    assert torch.equal(out[None][1], out[64][1]) and torch.equal(out[None][2], out[64][2])
    assert torch.count_nonzero(out[64][3][..., nx:]) == 0
