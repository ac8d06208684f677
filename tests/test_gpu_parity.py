"""GPU parity: the gfx950 path (through the C ABI) against the FP64 oracle.

Bars: relative L2 <= 1e-5 per output against the FP64 oracle (FP32 storage and
arithmetic), and the largest single-point deviation <= 1e-4 of the field's
peak; bit-identical outputs across every tile shape, march depth, XCD
order and the plain-tiling kernel (all use one canonical FP32 operation
order); kappa bit-identical to the FP64 formula rounded once.
"""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_1310_8232_amd as p
from compare import check_close

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def gpu_run(v, h, dt, vmax, R, nt, u0=None, um1=None, src_idx=None, amp=None, tile=None, it0=0):
    prop = p.Propagator(cuda(v), h, dt, R, vmax=vmax, tile=tile)
    shape = v.shape
    a = cuda(u0) if u0 is not None else torch.zeros(shape, device="cuda:0")
    b = cuda(um1) if um1 is not None else torch.zeros(shape, device="cuda:0")
    src = None
    keep = None
    if src_idx is not None:
        idx_t = cuda(np.asarray(src_idx, np.int64), torch.int64)
        amp_t = cuda(np.asarray(amp, np.float32).reshape(len(amp), -1))
        keep = (idx_t, amp_t)
        src = p.make_src(idx_t, amp_t)
    a, b = prop.run(a, b, nt, src, it0=it0)
    torch.cuda.synchronize()
    del keep
    return a.cpu().numpy(), b.cpu().numpy(), prop


def oracle_run(v, h, dt, R, nt, u0=None, um1=None, src_idx=None, amp=None, it0=0):
    kap = oracle.kappa(v, dt, h)
    z = np.zeros(v.shape)
    return oracle.leapfrog(kap, z if u0 is None else u0, z if um1 is None else um1, R, nt, it0=it0,
                           src_idx=src_idx, amp=None if amp is None else np.asarray(amp, np.float64))


def assert_close(got, ref, tol=TOL, what=""):
    # rel-L2 over the field and the largest single-point deviation (bound:
    # ten times the rel-L2 bar; see tests/compare.py).
    check_close(got, ref, tol, what)


def test_kappa_bit_exact():
    v = workloads.layered_model(33, 20, 17, seed=5)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    got = prop.kappa.cpu().numpy()
    ref = oracle.kappa(v, dt, 10.0).astype(np.float32)
    assert np.array_equal(got, ref)


def test_plain_method_64cube_100_steps():
    c = workloads.config_plain()
    log(f"case: {c['name']} R=4 100 steps, default tile")
    ref_n, ref_nm1 = oracle_run(c["v"], c["h"], c["dt"], 4, 100, src_idx=c["src_idx"], amp=c["amp"])
    un, unm1, prop = gpu_run(c["v"], c["h"], c["dt"], c["vmax"], 4, 100, src_idx=c["src_idx"], amp=c["amp"])
    log(f"  tile {prop.tile}")
    assert_close(un, ref_n, what="u^100")
    assert_close(unm1, ref_nm1, what="u^99")
    # The plain-tiling kernel gives the same bits.
    pn, pnm1, _ = gpu_run(c["v"], c["h"], c["dt"], c["vmax"], 4, 100, src_idx=c["src_idx"], amp=c["amp"],
                          tile=p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1))
    assert np.array_equal(pn, un) and np.array_equal(pnm1, unm1)


@pytest.mark.parametrize("R", [3, 4, 5])
def test_layered_128cube_100_steps(R):
    c = workloads.config_layered(128, 128, 128, nt=100, radius=R)
    log(f"case: {c['name']} R={R} 100 steps")
    ref_n, ref_nm1 = oracle_run(c["v"], c["h"], c["dt"], R, 100, src_idx=c["src_idx"], amp=c["amp"])
    un, unm1, _ = gpu_run(c["v"], c["h"], c["dt"], c["vmax"], R, 100, src_idx=c["src_idx"], amp=c["amp"])
    assert_close(un, ref_n, what="u^100")
    assert_close(unm1, ref_nm1, what="u^99")


def _random_case(nx, ny, nz, seed, R=4):
    v = workloads.layered_model(nx, ny, nz, seed=seed)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    u0 = workloads.random_field(nx, ny, nz, seed + 1)
    um1 = workloads.random_field(nx, ny, nz, seed + 2)
    return v, dt, vmax, u0, um1


def _tiles(R, nx, dzs):
    # Every compiled vector width that divides nx (4, 2, 1 points per thread).
    out = []
    ts = [t for w in (4, 2, 1) if nx % w == 0 for t in p.stencil_list_tiles(R, {4: 1, 2: 2, 1: 0}[w])]
    for t in ts:
        for dz in dzs:
            for xcd in (1, 0):
                out.append(p.make_tile(p.TILE_ZMARCH, t.bx, t.by, t.ry, dz, t.vw, xcd, t.pf))
    for sh in ((64, 4, 1), (32, 8, 2), (8, 8, 8), (128, 1, 1)):
        out.append(p.make_tile(p.TILE_PLAIN, bx=sh[0], by=sh[1], dz=sh[2]))
    return out


@pytest.mark.parametrize("R,shape", [(4, (72, 45, 37)), (3, (72, 45, 37)), (5, (72, 45, 37)),
                                     (4, (61, 45, 37)), (5, (61, 29, 23)), (4, (260, 67, 19)),
                                     (4, (70, 45, 37)), (5, (250, 29, 23)), (3, (66, 20, 12))])
def test_tile_invariance_and_oracle(R, shape):
    nx, ny, nz = shape
    v, dt, vmax, u0, um1 = _random_case(nx, ny, nz, seed=100 + R, R=R)
    nsteps = 6
    log(f"case: random fields {nx}x{ny}x{nz} R={R}, {nsteps} steps, every tile")
    ref_n, ref_nm1 = oracle_run(v, 10.0, dt, R, nsteps, u0, um1)
    base = None
    tiles = _tiles(R, nx, (1, 7, 16, nz))
    for t in tiles:
        un, unm1, _ = gpu_run(v, 10.0, dt, vmax, R, nsteps, u0, um1, tile=t)
        if base is None:
            base = (un, unm1, t)
            assert_close(un, ref_n, what=f"u^n {t}")
            assert_close(unm1, ref_nm1, what=f"u^n-1 {t}")
        else:
            assert np.array_equal(un, base[0]), f"tile {t} differs from {base[2]}"
            assert np.array_equal(unm1, base[1]), f"tile {t} differs from {base[2]}"
    log(f"  {len(tiles)} tiles bit-identical")


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 7), (4, 1, 9), (9, 1, 1), (8, 8, 1), (1, 17, 3),
                                   (5, 4, 2), (12, 2, 30)])
def test_degenerate_grids(shape):
    nx, ny, nz = shape
    v, dt, vmax, u0, um1 = _random_case(nx, ny, nz, seed=7)
    log(f"case: degenerate grid {shape}")
    ref_n, ref_nm1 = oracle_run(v, 10.0, dt, 4, 4, u0, um1)
    for t in (None, p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1)):
        un, unm1, _ = gpu_run(v, 10.0, dt, vmax, 4, 4, u0, um1, tile=t)
        assert_close(un, ref_n, what=f"u^n {shape}")
        assert_close(unm1, ref_nm1, what=f"u^n-1 {shape}")


def test_several_sources_and_out_of_range_index():
    nx, ny, nz = 40, 36, 30
    v, dt, vmax, _, _ = _random_case(nx, ny, nz, seed=21)
    n = nx * ny * nz
    a_idx, b_idx = (10 * ny + 12) * nx + 7, (25 * ny + 3) * nx + 39
    nt = 20
    amp3 = np.stack([workloads.ricker(nt, dt, 25.0), -workloads.ricker(nt, dt, 20.0),
                     0.5 * workloads.ricker(nt, dt, 30.0)], axis=1)
    log("case: three sources (one repeated) plus one index outside the grid")
    ref_n, ref_nm1 = oracle_run(v, 10.0, dt, 4, nt, src_idx=[a_idx, b_idx, a_idx], amp=amp3)
    amp4 = np.concatenate([amp3, np.ones((nt, 1), np.float32)], axis=1)
    un, unm1, _ = gpu_run(v, 10.0, dt, vmax, 4, nt, src_idx=[a_idx, b_idx, a_idx, n + 5], amp=amp4)
    assert_close(un, ref_n, what="u^n")
    assert_close(unm1, ref_nm1, what="u^n-1")


def test_many_sources_with_repeats_across_blocks_and_chunks():
    # 2600 sources: the injection kernel runs 11 workgroups of 256 threads and
    # scans the index list in three LDS chunks of 1024. Repeats sit inside a
    # workgroup, across workgroups, across a chunk boundary and at the two ends
    # of the list; two indices are outside the grid. From rest the sweep gives
    # exactly 0, and with kappa = 1/16 (v dt / h = 1/4) and amplitudes in
    # multiples of 1/8 every sum is exact, so the field must equal the plain
    # sum of kappa * amp per point bit for bit.
    nx, ny, nz = 64, 48, 40
    n = nx * ny * nz
    v = np.full((nz, ny, nx), 2048.0, np.float32)
    h, dt = 8.0, 1.0 / 1024.0
    rng = np.random.default_rng(workloads.SEED + 61)
    nsrc, nt, it = 2600, 5, 3
    idx = rng.integers(0, n, nsrc).astype(np.int64)
    for a, b in ((3, 17), (5, 700), (1023, 1024), (40, 2047), (0, nsrc - 1), (2048, 2599), (100, 1500)):
        idx[b] = idx[a]
    idx[9], idx[1030] = n + 3, -1
    amp = (rng.integers(-64, 65, (nt, nsrc)) / 8.0).astype(np.float32)
    log(f"case: {nsrc} sources with repeats, step it={it} from rest, exact arithmetic")
    prop = p.Propagator(cuda(v), h, dt, 4, vmax=2048.0)
    src = p.make_src(cuda(idx, torch.int64), cuda(amp))
    a, b = prop.zeros(), prop.zeros()
    prop.step(a, b, it, src)
    torch.cuda.synchronize()
    ref = np.zeros(n, np.float64)
    for k in range(nsrc):
        if 0 <= idx[k] < n:
            ref[idx[k]] += 0.0625 * float(amp[it, k])
    got = b.cpu().numpy().reshape(-1).astype(np.float64)
    assert np.array_equal(got, ref)
    assert a.abs().max().item() == 0.0


def test_tune_selection_follows_rule_and_cache(tmp_path):
    nx, ny, nz = 96, 64, 48
    v, dt, vmax, _, _ = _random_case(nx, ny, nz, seed=31)
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    log("case: tune 96x64x48, full candidate list, 3 replicates")
    rep, table, cands = prop.tune(n_iter=4, n_rep=3, table_cap=1024, include_plain=True)
    log(f"  nC={rep['n_candidates']} chosen={rep['tile']} min={rep['min_time_ms']:.4f} "
        f"actual={rep['actual_time_ms']:.4f} gap={rep['gap']:+.3f} s={rep['seconds']:.2f}")
    assert rep["n_candidates"] == len(cands) > 10
    ids = [list(range(len(cands)))]
    best, t = oracle.select_block([table], ids, "worst")
    assert cands[best] == rep["tile"]
    assert t == rep["min_time_ms"]
    assert abs(rep["gap"] - oracle.gap(rep["min_time_ms"], rep["actual_time_ms"])) < 1e-12
    assert prop.tile.as_dict() == rep["tile"]
    # Cache round trip.
    cache = str(tmp_path / "tune.txt")
    rep1, _, _ = prop.tune(n_iter=2, n_rep=1, parts=3, cache_path=cache)
    rep2, _, _ = prop.tune(n_iter=2, n_rep=1, parts=3, cache_path=cache)
    assert not rep1["from_cache"] and rep2["from_cache"]
    assert rep2["tile"] == rep1["tile"]
    assert 0 < rep1["n_candidates"] <= 27 * 8


def test_graph_capture_replays_match_eager():
    nx, ny, nz = 64, 48, 40
    v, dt, vmax, u0, um1 = _random_case(nx, ny, nz, seed=41)
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    amp = cuda(workloads.ricker(8, dt, 25.0).reshape(8, 1))
    idx = cuda(np.array([workloads.centre_index(nx, ny, nz)], np.int64), torch.int64)
    src = p.make_src(idx, amp)
    a0, b0 = cuda(u0), cuda(um1)
    a, b = a0.clone(), b0.clone()
    torch.cuda.synchronize()
    prop.run(a, b, 4, src)
    torch.cuda.synchronize()
    eager_a, eager_b = a.clone(), b.clone()

    ga, gb = a0.clone(), b0.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            prop.run(ga, gb, 4, src)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        ga.copy_(a0)
        gb.copy_(b0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ga, eager_a) and torch.equal(gb, eager_b), f"replay {rep}"
        _ = (ga * 2).sum().item()  # eager work between replays


def test_stream_probe():
    x, y, z = (torch.randn(1 << 20, device="cuda:0") for _ in range(3))
    out = torch.empty_like(x)
    p.stencil_stream_probe(x, None, None, out, x.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(out, x)
    p.stencil_stream_probe(x, y, z, out, x.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(out, (x + y) + z)
    # Odd size and 4-byte offsets take the scalar path.
    out.zero_()
    p.stencil_stream_probe(x[1:], None, None, out[1:], (x.numel() - 3) * 4)
    torch.cuda.synchronize()
    assert torch.equal(out[1:-2], x[1:-2]) and out[0] == 0 and out[-2:].eq(0).all()


@pytest.mark.slow
def test_full_size_512_tuned_default_plain():
    nx = ny = nz = 512
    log("case: 512^3 layered kappa, random fields, 3 steps: searched one- and two-step tiles, default and plain "
        "tiles vs oracle")
    t0 = time.time()
    v, dt, vmax, u0, um1 = _random_case(nx, ny, nz, seed=workloads.SEED)
    log(f"  inputs {time.time() - t0:.1f}s")
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    _bench_mode(prop)  # the bench's searches: every compiled one- and two-step tile
    tuned, tuned2 = prop.tile, prop.tile2
    log(f"  searched {tuned.as_dict()} and {tuned2.as_dict()}")
    del prop
    torch.cuda.empty_cache()
    t0 = time.time()
    ref_n, ref_nm1 = oracle_run(v, 10.0, dt, 4, 3, u0, um1)
    log(f"  oracle {time.time() - t0:.1f}s")
    base = None
    for t in (tuned, None, p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1)):
        un, unm1, _ = gpu_run(v, 10.0, dt, vmax, 4, 3, u0, um1, tile=t)
        torch.cuda.empty_cache()
        if base is None:
            base = (un, unm1)
            assert_close(un, ref_n, what="u^3")
            assert_close(unm1, ref_nm1, what="u^2")
        else:
            assert np.array_equal(un, base[0]) and np.array_equal(unm1, base[1])
    # The searched two-step tile: one two-step launch and a closing one-step
    # launch give the same bits.
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    prop.tile = tuned2
    a, b = prop.run(cuda(u0), cuda(um1), 3, None, temporal=2)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), base[0]) and np.array_equal(b.cpu().numpy(), base[1])


def _bench_mode(prop):
    # The bench's launch configuration: both searches (one-step tiles, then
    # two-step tiles, n_iter 10, 3 replicates); the mode with the smaller
    # verified time per step runs. Returns temporal (1 or 2); the context
    # keeps both chosen tiles.
    r1, _, _ = prop.tune(n_iter=10, n_rep=3)
    r2, _, _ = prop.tune(n_iter=10, n_rep=3, temporal=2)
    return 2 if r2["actual_time_ms"] < r1["actual_time_ms"] else 1


def _throughput_workload_vs_oracle(nt, n=512):
    # The throughput workload exactly as the bench runs it (n^3 layered
    # model, source at the centre, from rest), in the bench's launch
    # configuration (searched mode and tile), against the FP64 oracle after
    # nt steps.
    c = workloads.config_layered(n, n, n, nt=nt)
    log(f"case: {n}^3 throughput workload from rest, the bench's searched mode and tile, {nt} steps vs oracle")
    prop = p.Propagator(cuda(c["v"]), c["h"], c["dt"], 4, vmax=c["vmax"])
    temporal = _bench_mode(prop)
    log(f"  mode {temporal}-step, tile {(prop.tile2 if temporal == 2 else prop.tile).as_dict()}")
    idx = cuda(c["src_idx"], torch.int64)
    amp_t = cuda(c["amp"].reshape(-1, 1))
    a, b = prop.run(prop.zeros(), prop.zeros(), nt, p.make_src(idx, amp_t), temporal=temporal)
    torch.cuda.synchronize()
    un, unm1 = a.cpu().numpy(), b.cpu().numpy()
    del prop, a, b
    torch.cuda.empty_cache()
    t0 = time.time()
    kap = oracle.kappa(c["v"], c["dt"], c["h"])
    amp = c["amp"].reshape(-1, 1).astype(np.float64)
    ref_n = np.zeros(kap.shape)
    ref_nm1 = np.zeros(kap.shape)
    for it in range(0, nt, 50):  # in chunks, with a progress line per chunk
        k = min(50, nt - it)
        ref_n, ref_nm1 = oracle.leapfrog(kap, ref_n, ref_nm1, 4, k, it0=it, src_idx=c["src_idx"], amp=amp)
        log(f"  oracle {it + k}/{nt} steps, {time.time() - t0:.0f}s")
    return (oracle.rel_l2(un, ref_n), oracle.rel_l2(unm1, ref_nm1)), (un, unm1, ref_n, ref_nm1)


@pytest.mark.slow
def test_throughput_workload_512_100_steps():
    _, (un, unm1, ref_n, ref_nm1) = _throughput_workload_vs_oracle(100)
    assert_close(un, ref_n, what="u^100")
    assert_close(unm1, ref_nm1, what="u^99")


@pytest.mark.slow
def test_throughput_workload_256_1000_steps():
    # The throughput recipe for 1000 steps on a grid the FP64 oracle finishes
    # in about a minute. FP32 rounding grows about linearly with the step
    # count (rel-L2 <= 1e-5 holds at 100 steps), so 2e-4 bounds 1000 steps
    # with a factor-of-two margin; the per-point bound is ten times that.
    _, (un, unm1, ref_n, ref_nm1) = _throughput_workload_vs_oracle(1000, n=256)
    assert_close(un, ref_n, tol=2e-4, what="u^1000")
    assert_close(unm1, ref_nm1, tol=2e-4, what="u^999")


def _energy(u_next, u_cur, kap):
    # Discrete energy of the source-free leapfrog scheme between levels n and
    # n+1: sum (u^{n+1} - u^n)^2 / kappa - <u^{n+1}, L u^n>, in FP64; with L
    # symmetric it is the same at every n.
    u1 = u_next.astype(np.float64)
    u0 = u_cur.astype(np.float64)
    d = u1 - u0
    return float(np.sum(d * d / kap)) - float(np.sum(u1 * oracle.laplacian(u0, 4)))


@pytest.mark.slow
def test_throughput_workload_512_1000_steps_energy():
    # The bench's workload for 1000 steps on the searched tile, checked by a
    # property that holds at any size: once the Ricker wavelet has died out
    # (it is below 1e-17 of its peak after 3 t0 = 200 ms, step 228), the
    # discrete energy stays constant. FP32 rounding perturbs it by about
    # eps/(omega dt) = 6e-8/0.083 = 7e-7 relative per step with random sign,
    # sqrt(700) * 7e-7 = 1.9e-5 over the 700 steps checked; the bound is
    # 2e-5 (a wrong tap or tile seam breaks the symmetry of the operator and
    # with it the conservation by orders of magnitude more).
    c = workloads.config_layered(512, 512, 512, nt=1000)
    log("case: 512^3 throughput workload, 1000 steps in the bench's mode and tile, energy after the source")
    prop = p.Propagator(cuda(c["v"]), c["h"], c["dt"], 4, vmax=c["vmax"])
    temporal = _bench_mode(prop)
    log(f"  mode {temporal}-step, tile {(prop.tile2 if temporal == 2 else prop.tile).as_dict()}")
    idx = cuda(c["src_idx"], torch.int64)
    amp = cuda(c["amp"].reshape(-1, 1))
    src = p.make_src(idx, amp)
    a, b = torch.zeros_like(prop.kappa), torch.zeros_like(prop.kappa)
    spare = [prop.zeros(), prop.zeros()] if temporal == 2 else None
    a, b = prop.run(a, b, 300, src, temporal=temporal, spare=spare)
    torch.cuda.synchronize()
    u300, u299 = a.cpu().numpy(), b.cpu().numpy()
    a, b = prop.run(a, b, 700, src, it0=300, temporal=temporal, spare=spare)
    torch.cuda.synchronize()
    u1000, u999 = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(np.isfinite(u1000)) and np.all(np.isfinite(u999))
    # The GPU's kappa: the FP64 formula rounded once to FP32 (bit-exact, tested).
    kap = oracle.kappa(c["v"], c["dt"], c["h"]).astype(np.float32).astype(np.float64)
    e300 = _energy(u300, u299, kap)
    e1000 = _energy(u1000, u999, kap)
    drift = abs(e1000 - e300) / abs(e300)
    log(f"  energy at 299.5: {e300:.9e}, at 999.5: {e1000:.9e}, relative drift {drift:.3e}")
    assert e300 > 0 and drift <= 2e-5


@pytest.mark.slow
@pytest.mark.skipif(not os.environ.get("P1310_LONG"),
                    reason="the 1000-step FP64 oracle run at 512^3 takes several minutes of host time; "
                           "set P1310_LONG=1 to run it")
def test_throughput_workload_512_1000_steps():
    # FP32 rounding grows about linearly with the step count (1e-5 holds at
    # 100 steps); 2e-4 is the sanity bound at 1000.
    (e1, e2), _ = _throughput_workload_vs_oracle(1000)
    log(f"  u^1000 rel_l2 {e1:.3e}   u^999 rel_l2 {e2:.3e}")
    assert e1 <= 2e-4 and e2 <= 2e-4


def test_stream_probe_sweep_order():
    # The streaming reference in the sweep's access order covers every point
    # once (ragged x and y tiles, two z chunks): out == (a + b) + c exactly.
    shape = (300, 45, 72)  # nz, ny, nx
    g = torch.Generator(device="cpu").manual_seed(5)
    a, b, c = (torch.rand(shape, generator=g).to("cuda:0") for _ in range(3))
    out = torch.full(shape, -1.0, device="cuda:0")
    p.stencil_stream_probe_march(a, b, c, out, shape)
    torch.cuda.synchronize()
    assert torch.equal(out, (a + b) + c)


@pytest.mark.slow
@pytest.mark.parametrize("shape,kind", [((4096, 4096, 40), "zmarch"), ((16384, 16384, 2), "plain")])
def test_largest_planes(shape, kind):
    # Planes at the size limits: 4096^2 (64 MiB) takes the deepest z-march
    # window below 2 GiB (dz + 2R = 31 planes); 16384^2 (1 GiB) fits no
    # z-march window and runs plain tiling. Random fields, 3 steps, all
    # points against the oracle.
    nx, ny, nz = shape
    log(f"case: largest planes {shape} ({kind}), 3 steps")
    t0 = time.time()
    v, dt, vmax, u0, um1 = _random_case(nx, ny, nz, seed=17)
    un, unm1, prop = gpu_run(v, 10.0, dt, vmax, 4, 3, u0, um1)
    t = prop.tile.as_dict()
    del prop
    torch.cuda.empty_cache()
    log(f"  tile {t} ({time.time() - t0:.0f}s)")
    assert t["kind"] == (p.TILE_ZMARCH if kind == "zmarch" else p.TILE_PLAIN)
    if kind == "zmarch":
        assert t["dz"] == 23
    ref_n, ref_nm1 = oracle_run(v, 10.0, dt, 4, 3, u0, um1)
    log(f"  oracle ({time.time() - t0:.0f}s)")
    assert_close(un, ref_n, what="u^3")
    assert_close(unm1, ref_nm1, what="u^2")


def test_two_streams_concurrently():
    # Two grids advanced at the same time on two streams (the stream argument
    # of every call is honoured; contexts share no device state): each equals
    # its run on the default stream bit for bit.
    cases = []
    for seed, shape in ((61, (72, 45, 37)), (62, (64, 40, 48))):
        v, dt, vmax, u0, um1 = _random_case(*shape, seed=seed)
        prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
        ref = prop.run(cuda(u0), cuda(um1), 9)
        cases.append((prop, u0, um1, ref))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = []
    for (prop, u0, um1, _), s in zip(cases, streams):
        a, b = cuda(u0), cuda(um1)
        torch.cuda.synchronize()
        outs.append(prop.run(a, b, 9, stream=s))
    torch.cuda.synchronize()
    for (_, _, _, ref), got in zip(cases, outs):
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])


def test_empty_inputs():
    # Zero steps leave the fields as they are (one- and two-step loops); a
    # source list of n = 0, zero receivers, an empty misfit (J = 0) and the
    # gradient terms over no steps are no-ops, not errors.
    nx, ny, nz = 40, 24, 16
    v, dt, vmax, u0, um1 = _random_case(nx, ny, nz, seed=31)
    prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax)
    a, b = cuda(u0), cuda(um1)
    for temporal in (1, 2):
        x, y = prop.run(a, b, 0, None, temporal=temporal)
        torch.cuda.synchronize()
        assert x is a and y is b and np.array_equal(a.cpu().numpy(), u0) and np.array_equal(b.cpu().numpy(), um1)
    empty_src = p.make_src(torch.zeros(0, dtype=torch.int64, device="cuda:0"),
                           torch.zeros((5, 0), dtype=torch.float32, device="cuda:0"))
    ref = gpu_run(v, 10.0, dt, vmax, 4, 3, u0, um1)[:2]
    x, y = prop.run(cuda(u0), cuda(um1), 3, empty_src)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), ref[0]) and np.array_equal(y.cpu().numpy(), ref[1])
    out = torch.full((1,), 5.0, device="cuda:0")
    p.stencil_sample(prop.ctx, x, torch.zeros(0, dtype=torch.int64, device="cuda:0"), out)
    J = torch.full((), 7.0, dtype=torch.float64, device="cuda:0")
    e = torch.zeros(0, device="cuda:0")
    p.stencil_misfit(e, e, None, J)
    torch.cuda.synchronize()
    assert float(out[0]) == 5.0 and float(J) == 0.0
