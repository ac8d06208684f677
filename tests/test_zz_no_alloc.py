"""stencil_batch_create_static (the batch whose descriptor table sits in the
library's static per-GPU array, no device allocation) against
stencil_batch_create on the same shots: every shot's wavefields must be the
same bits after the same steps. Two static batches in a row, the second
smaller; the first is refused once the second has replaced the table."""
import sys

import numpy as np
import pytest
import torch

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


def _shots(shapes, tiles, nt, seed):
    out = []
    for i, ((nx, ny, nz), tile) in enumerate(zip(shapes, tiles)):
        v = workloads.layered_model(nx, ny, nz, seed=seed + i)
        dt, vmax = workloads.dt_for_courant(v, 10.0)
        prop = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, tile=tile)
        if i % 3 == 2:  # two sources, one repeated index
            idx = np.array([workloads.centre_index(nx, ny, nz), 5, 5], np.int64)
        else:
            idx = np.array([workloads.centre_index(nx, ny, nz)], np.int64)
        amp = np.stack([workloads.ricker(nt, dt, 20.0 + 3 * j) for j in range(len(idx))], 1)
        keep = (cuda(idx, torch.int64), cuda(amp))
        out.append((prop, p.make_src(*keep), keep))
    return out


def _run(shots, nt, create):
    bufs = [(pr.zeros(), pr.zeros()) for pr, _, _ in shots]
    spec = [(pr.ctx, pr.kappa, a, b, src) for (pr, src, _), (a, b) in zip(shots, bufs)]
    h = create(spec, 0)
    for it in range(nt):
        p.stencil_batch_step(h, it)
    torch.cuda.synchronize()
    # After nt steps from 0: u_a holds the newest level when nt is even.
    out = [(a.cpu().numpy(), b.cpu().numpy()) for a, b in bufs]
    return h, out


def _same(x, y, what):
    for i, ((a0, b0), (a1, b1)) in enumerate(zip(x, y)):
        assert np.array_equal(a0, a1) and np.array_equal(b0, b1), f"{what}: shot {i} differs"


def test_static_batch_matches_allocating_batch_twice():
    nt = 21
    shapes = [(72, 45, 37), (64, 32, 40), (61, 29, 23), (96, 40, 24), (40, 36, 30)]
    tiles = [p.make_tile(bx=64, by=4, ry=1, dz=16), p.make_tile(bx=64, by=4, ry=1, dz=7), None,
             p.make_tile(bx=16, by=8, ry=2, dz=64, xcd=0), p.make_tile(p.TILE_PLAIN, bx=32, by=4, dz=2)]
    shots = _shots(shapes, tiles, nt, seed=300)
    log(f"case: static-table batch vs allocating batch, {len(shots)} shots, {nt} steps")
    h_ref, ref = _run(shots, nt, p.stencil_batch_create)
    h_s1, got = _run(shots, nt, p.stencil_batch_create_static)
    _same(ref, got, "first static batch")
    assert p.stencil_batch_launches(h_s1) == p.stencil_batch_launches(h_ref)
    p.stencil_batch_destroy(h_ref)

    # Second call, smaller input: two shots on smaller grids. It replaces the
    # table, so the first static batch is refused from now on.
    nt2 = 8
    small = _shots([(32, 20, 17), (41, 24, 12)], [p.make_tile(bx=16, by=8, ry=1, dz=4), None], nt2, seed=400)
    log(f"case: second static batch, {len(small)} smaller shots, {nt2} steps")
    h_ref2, ref2 = _run(small, nt2, p.stencil_batch_create)
    h_s2, got2 = _run(small, nt2, p.stencil_batch_create_static)
    _same(ref2, got2, "second static batch")
    with pytest.raises(p.StencilError) as e:
        p.stencil_batch_step(h_s1, 0)
    assert e.value.status == p.EINVAL and "replaced" in str(e.value)
    for h in (h_ref2, h_s2, h_s1):
        p.stencil_batch_destroy(h)
