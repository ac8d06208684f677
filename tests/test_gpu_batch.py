"""Batched uneven shots: one launch per tile-shape group per step must give,
for every shot, the same bits as running that shot alone (which the parity
tests tie to the FP64 oracle), and a batch shot is also checked against the
oracle directly. Graph replay of batch steps matches eager."""
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


SHAPES = [(72, 45, 37), (64, 32, 40), (61, 29, 23), (33, 20, 17), (96, 40, 24), (40, 36, 30)]
TILES = [p.make_tile(bx=64, by=4, ry=1, dz=16), p.make_tile(bx=64, by=4, ry=1, dz=7),  # one group, two dz
         None,                                                                          # vw = 1 default
         p.make_tile(p.TILE_PLAIN, bx=32, by=4, dz=2),                                  # plain, solo
         p.make_tile(bx=16, by=8, ry=2, dz=64, xcd=0),
         p.make_tile(bx=64, by=4, ry=1, dz=16)]                                         # joins group 1


def _shots(nt):
    out = []
    for i, (shape, tile) in enumerate(zip(SHAPES, TILES)):
        nx, ny, nz = shape
        v = workloads.layered_model(nx, ny, nz, seed=200 + i)
        dt, vmax = workloads.dt_for_courant(v, 10.0)
        if i == 4:  # three sources, one repeated
            idx = np.array([workloads.centre_index(nx, ny, nz), 7, 7], np.int64)
        elif i == 5:  # no source
            idx = None
        else:
            idx = np.array([workloads.centre_index(nx, ny, nz)], np.int64)
        amp = None if idx is None else np.stack([workloads.ricker(nt, dt, 20.0 + 5 * j) for j in range(len(idx))], 1)
        out.append(dict(v=v, dt=dt, vmax=vmax, idx=idx, amp=amp, tile=tile))
    return out


def _make(sh):
    prop = p.Propagator(cuda(sh["v"]), 10.0, sh["dt"], 4, vmax=sh["vmax"], tile=sh["tile"])
    keep = None
    src = None
    if sh["idx"] is not None:
        keep = (cuda(sh["idx"], torch.int64), cuda(sh["amp"]))
        src = p.make_src(*keep)
    return prop, src, keep


def test_batch_matches_single_shots_and_oracle():
    nt = 23
    shots = _shots(nt)
    made = [_make(sh) for sh in shots]
    batch = p.Batch([(pr, src) for pr, src, _ in made])
    log(f"case: batch of {len(shots)} uneven shots, {batch.launches_per_step} launches per step, {nt} steps")
    # groups: {0, 1, 5} (64x4x1, vw 4, XCD order), {2} (vw 1), {4} (16x8x2, linear order);
    # shot 3 plain on its own; shot 4's three sources need an injection launch.
    assert batch.launches_per_step == 5
    batch.run(nt)
    torch.cuda.synchronize()
    final = batch.current(nt)
    for i, ((pr, src, _), sh) in enumerate(zip(made, shots)):
        a = torch.zeros(pr.shape, device="cuda:0")
        b = torch.zeros(pr.shape, device="cuda:0")
        a, b = pr.run(a, b, nt, src)
        torch.cuda.synchronize()
        assert torch.equal(final[i][0], a) and torch.equal(final[i][1], b), f"shot {i} {SHAPES[i]}"
    # Shot 4 (three sources, ragged) against the oracle.
    sh = shots[4]
    kap = oracle.kappa(sh["v"], sh["dt"], 10.0)
    z = np.zeros(kap.shape)
    ref_n, ref_nm1 = oracle.leapfrog(kap, z, z, 4, nt, src_idx=sh["idx"], amp=sh["amp"])
    check_close(final[4][0].cpu().numpy(), ref_n, 1e-5, "shot 4 u^n")
    check_close(final[4][1].cpu().numpy(), ref_nm1, 1e-5, "shot 4 u^n-1")


def test_batch_graph_replay():
    nt = 12
    shots = _shots(nt)
    made = [_make(sh) for sh in shots]
    batch = p.Batch([(pr, src) for pr, src, _ in made])
    batch.run(nt)
    torch.cuda.synchronize()
    eager = [(x.clone(), y.clone()) for x, y in batch.current(nt)]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            batch.run(nt)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for x, y in zip(batch.u_a, batch.u_b):
            x.zero_()
            y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, (x, y) in enumerate(batch.current(nt)):
            assert torch.equal(x, eager[i][0]) and torch.equal(y, eager[i][1]), (rep, i)


def test_batch_rejects_bad_step():
    shots = _shots(5)
    made = [_make(sh) for sh in shots[:2]]
    batch = p.Batch([(pr, src) for pr, src, _ in made], it0=0)
    with pytest.raises(p.StencilError):
        batch.step(5)  # beyond the sources' samples
    with pytest.raises(p.StencilError):
        batch.step(-1)


@pytest.mark.slow
def test_batch_16_shots_bits_and_oracle():
    # The 16-shot workload, per-shape tuned tiles, 8 steps: every shot equals
    # its single-shot run bit for bit; the 96^3 shot is checked against the
    # oracle at 100 steps.
    cfgs = workloads.config_batch(nt=100)
    props = []
    for c in cfgs:
        pr = p.Propagator(cuda(c["v"]), c["h"], c["dt"], 4, vmax=c["vmax"])
        pr.tune(parts=3, n_iter=3, n_rep=2)
        idx, amp = cuda(c["src_idx"], torch.int64), cuda(c["amp"].reshape(-1, 1))
        props.append((pr, p.make_src(idx, amp), (idx, amp)))
    batch = p.Batch([(pr, src) for pr, src, _ in props])
    log(f"case: 16-shot batch, {batch.launches_per_step} launches per step")
    batch.run(8)
    torch.cuda.synchronize()
    for i, ((pr, src, _), (x, y)) in enumerate(zip(props, batch.current(8))):
        a = torch.zeros(pr.shape, device="cuda:0")
        b = torch.zeros(pr.shape, device="cuda:0")
        a, b = pr.run(a, b, 8, src)
        assert torch.equal(x, a) and torch.equal(y, b), f"shot {i}"
    batch.run(92, it0=8)
    torch.cuda.synchronize()
    x, y = batch.current(100)[1]
    c = cfgs[1]
    kap = oracle.kappa(c["v"], c["dt"], c["h"])
    z = np.zeros(kap.shape)
    ref_n, ref_nm1 = oracle.leapfrog(kap, z, z, 4, 100, src_idx=c["src_idx"], amp=c["amp"])
    log("  96^3 shot after 100 batch steps:")
    check_close(x.cpu().numpy(), ref_n, 1e-5, "u^100")
    check_close(y.cpu().numpy(), ref_nm1, 1e-5, "u^99")


def test_batch_tune_sets_one_tile_and_keeps_bits():
    nt = 10
    shots = [s for s in _shots(nt) if s["v"].shape[2] % 4 == 0]  # vector tiles for every shot
    made = [_make(sh) for sh in shots]
    batch = p.Batch([(pr, src) for pr, src, _ in made], tune=dict(n_iter=2, n_rep=2, parts=3))
    rep = batch.tune_report
    log(f"case: batch search over {rep['n_candidates']} candidates -> {rep['tile']} gap {rep['gap']:+.3f}")
    assert rep["n_candidates"] > 0 and np.isfinite(rep["actual_time_ms"])
    key = {k: rep["tile"][k] for k in ("kind", "bx", "by", "ry", "vw", "xcd", "pf")}
    for pr, _, _ in made:
        t = pr.tile.as_dict()
        assert {k: t[k] for k in key} == key
        assert t["dz"] == min(rep["tile"]["dz"], pr.shape[0])
    assert batch.launches_per_step == 1 + sum(1 for s in shots if s["idx"] is not None and len(s["idx"]) > 1)
    batch.run(nt)
    torch.cuda.synchronize()
    for i, ((pr, src, _), (x, y)) in enumerate(zip(made, batch.current(nt))):
        a = torch.zeros(pr.shape, device="cuda:0")
        b = torch.zeros(pr.shape, device="cuda:0")
        a, b = pr.run(a, b, nt, src)
        assert torch.equal(x, a) and torch.equal(y, b), f"shot {i}"
