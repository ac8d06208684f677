"""Two leapfrog steps per launch (blocking in time) against one-step
launches: every two-step tile must give the bits of the one-step path (which
the parity tests tie to the FP64 oracle), and the 512^3 run is also checked
against the oracle directly."""
import sys
import time

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


def _case(shape, seed, R, nt):
    nx, ny, nz = shape
    v = workloads.layered_model(nx, ny, nz, seed=seed)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    u0 = workloads.random_field(nx, ny, nz, seed + 1)
    um1 = workloads.random_field(nx, ny, nz, seed + 2)
    idx = np.array([workloads.centre_index(nx, ny, nz)], np.int64)
    amp = workloads.ricker(nt, dt, 25.0).reshape(-1, 1)
    return v, dt, vmax, u0, um1, idx, amp


def _run(v, dt, vmax, R, u0, um1, idx, amp, nt, temporal, tile2=None):
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax)
    if tile2 is not None:
        prop.tile = tile2
    keep = (cuda(idx, torch.int64), cuda(amp))
    src = p.make_src(*keep)
    a, b = prop.run(cuda(u0), cuda(um1), nt, src, temporal=temporal)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


@pytest.mark.parametrize("R,shape", [(4, (72, 45, 37)), (3, (72, 45, 37)), (5, (72, 45, 37)), (4, (61, 29, 23)),
                                     (4, (260, 67, 19)), (3, (260, 67, 19)), (5, (200, 45, 21)), (5, (61, 29, 23)),
                                     (4, (12, 10, 6)), (4, (1, 1, 1)), (4, (8, 40, 3))])
def test_two_step_bits_equal_one_step(R, shape):
    nt = 7  # three two-step launches and one closing one-step launch
    v, dt, vmax, u0, um1, idx, amp = _case(shape, 50 + R, R, nt)
    log(f"case: two-step vs one-step, R={R} {shape}, {nt} steps")
    ref = _run(v, dt, vmax, R, u0, um1, idx, amp, nt, temporal=1)
    nz = shape[2]
    tiles = []
    for t in p.stencil_list_tiles2(R, shape[0] % 4 == 0):
        for dz in (1, 7, 16, nz):
            for xcd in (1, 0):
                tiles.append(p.make_tile(p.TILE_ZMARCH2, t.bx, t.by, t.ry, dz, t.vw, xcd, t.pf))
            # Edge pacing (pf bits 1-3; active with three or more tile
            # columns, e.g. 260 points wide): timing only, the same bits.
            tiles.append(p.make_tile(p.TILE_ZMARCH2, t.bx, t.by, t.ry, dz, t.vw, 1, t.pf | (5 << 1)))
    assert tiles
    for t in tiles:
        got = _run(v, dt, vmax, R, u0, um1, idx, amp, nt, temporal=2, tile2=t)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), f"tile {t}"
    log(f"  {len(tiles)} two-step tiles bit-identical to one-step")


def test_two_step_search_and_512_against_oracle():
    nx = ny = nz = 512
    log("case: 512^3 layered kappa, random fields, source, 4 steps: searched two-step tile vs oracle and one-step")
    t0 = time.time()
    v, dt, vmax, u0, um1, idx, amp = _case((nx, ny, nz), workloads.SEED, 4, 4)
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    rep, _, _ = prop.tune(temporal=2, n_iter=4, n_rep=2)
    log(f"  searched {rep['n_candidates']} two-step tiles -> {rep['tile']} gap {rep['gap']:+.4f} ({rep['seconds']:.1f}s)")
    assert rep["tile"]["kind"] == p.TILE_ZMARCH2 and prop.tile2.as_dict() == rep["tile"]
    tile2 = prop.tile2
    del prop
    torch.cuda.empty_cache()
    two = _run(v, dt, vmax, 4, u0, um1, idx, amp, 4, temporal=2, tile2=tile2)
    one = _run(v, dt, vmax, 4, u0, um1, idx, amp, 4, temporal=1)
    assert np.array_equal(two[0], one[0]) and np.array_equal(two[1], one[1])
    kap = oracle.kappa(v, dt, 10.0)
    ref_n, ref_nm1 = oracle.leapfrog(kap, u0, um1, 4, 4, src_idx=idx, amp=amp)
    log(f"  ({time.time() - t0:.1f}s)")
    check_close(two[0], ref_n, 1e-5, "u^4")
    check_close(two[1], ref_nm1, 1e-5, "u^3")


def test_run_in_segments_with_spare_list():
    # Two-step runs resumed segment after segment with the spare buffers
    # handed back in place: odd and even segment lengths, a graph-free loop
    # like the bench's timed segments. Equal to one-step launches bit for bit.
    shape, R = (72, 45, 37), 4
    v, dt, vmax, u0, um1, idx, amp = _case(shape, 91, R, 40)
    log(f"case: two-step runs in segments 6, 5, 10, 1, 8 with a spare list, {shape}")
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax)
    src = p.make_src(cuda(idx, torch.int64), cuda(amp))
    a, b = cuda(u0), cuda(um1)
    spare = [prop.zeros(), prop.zeros()]
    it = 0
    for n in (6, 5, 10, 1, 8):
        a, b = prop.run(a, b, n, src, it0=it, temporal=2, spare=spare)
        it += n
        ptrs = {t.data_ptr() for t in (a, b, *spare)}
        assert len(ptrs) == 4  # the pair and the spares never alias
    ra, rb = prop.run(cuda(u0), cuda(um1), it, src, temporal=1)
    torch.cuda.synchronize()
    assert torch.equal(a, ra) and torch.equal(b, rb)


def test_two_step_graph_capture_replays_match_eager():
    # Three two-step launches and a closing one-step launch (7 steps)
    # captured in one HIP graph on a side stream; each replay, with eager
    # work in between, gives the bits of the eager run.
    shape, R, nt = (64, 48, 40), 4, 7
    v, dt, vmax, u0, um1, idx, amp = _case(shape, 77, R, nt)
    log(f"case: two-step graph capture, {shape}, {nt} steps, 3 replays")
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax)
    src = p.make_src(cuda(idx, torch.int64), cuda(amp))
    a0, b0 = cuda(u0), cuda(um1)
    c, d = prop.zeros(), prop.zeros()
    ea, eb = prop.run(a0.clone(), b0.clone(), nt, src, temporal=2, spare=(c, d))
    torch.cuda.synchronize()
    eager = (ea.clone(), eb.clone())
    ga, gb, gc, gd = a0.clone(), b0.clone(), prop.zeros(), prop.zeros()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            ra, rb = prop.run(ga, gb, nt, src, temporal=2, spare=(gc, gd))
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        ga.copy_(a0)
        gb.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ra, eager[0]) and torch.equal(rb, eager[1]), f"replay {rep}"
        _ = (ga * 2).sum().item()  # eager work between replays
