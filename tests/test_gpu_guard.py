"""Guard regions around every field. Each field is a view into a larger
allocation whose elements before and after it hold NaN (at least two planes'
worth on each side). No kernel may store outside its fields (the guards stay
NaN) and no load outside a field may reach the arithmetic (a NaN would spread
into the results): every result is finite and equals the same computation on
unguarded buffers bit for bit. Covers every one-step tile of every vector
width and both XCD orders, plain tiling, the fused and the several-source
injection, two-step launches, 16-bit storage, batches, the adjoint step with
its gradient terms, receiver samples, kappa and the storage conversions."""
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


def guard_len(shape):
    """NaN elements on each side: two planes, at least 4096, a multiple of 64
    (so a field keeps the 256-byte alignment of its allocation)."""
    plane = shape[-2] * shape[-1] if len(shape) >= 2 else 0
    return max(4096, (2 * plane + 63) // 64 * 64)


class Guarded:
    """A field of `shape` and `dtype` inside NaN guards."""

    def __init__(self, shape, dtype=torch.float32, init=None):
        self.n = int(np.prod(shape))
        self.g = guard_len(shape)
        self.buf = torch.full((self.g + self.n + self.g,), float("nan"), dtype=dtype, device="cuda:0")
        self.t = self.buf[self.g:self.g + self.n].view(shape)
        if init is not None:
            self.t.copy_(init)

    def intact(self):
        return bool(torch.isnan(self.buf[:self.g]).all()) and bool(torch.isnan(self.buf[self.g + self.n:]).all())


def _case(shape, seed):
    nx, ny, nz = shape
    v = workloads.layered_model(nx, ny, nz, seed=seed)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    u0 = workloads.random_field(nx, ny, nz, seed + 1)
    um1 = workloads.random_field(nx, ny, nz, seed + 2)
    return v, dt, vmax, u0, um1


def _sources(shape, dt, nt):
    """A single centred source (fused into the sweep) and four sources that
    hit the first and last points of the grid and repeat one index (the
    injection kernel)."""
    nx, ny, nz = shape
    n = nx * ny * nz
    c = workloads.centre_index(nx, ny, nz)
    idx1 = cuda(np.array([c], np.int64), torch.int64)
    amp1 = cuda(workloads.ricker(nt, dt, 25.0).reshape(-1, 1))
    idx4 = cuda(np.array([c, 0, n - 1, c], np.int64), torch.int64)
    amp4 = cuda(np.stack([workloads.ricker(nt, dt, 20.0 + 5 * j) for j in range(4)], 1))
    return [p.make_src(idx1, amp1), p.make_src(idx4, amp4)]


def _one_step_tiles(R, nx, nz):
    widths = [w for w, ok in ((4, nx % 4 == 0), (2, nx % 2 == 0), (1, True)) if ok]
    out = []
    for w in widths:
        for t in p.stencil_list_tiles(R, {4: True, 2: 2, 1: False}[w]):
            for dz in (7, nz):
                for xcd in (1, 0):
                    out.append(p.make_tile(p.TILE_ZMARCH, t.bx, t.by, t.ry, dz, t.vw, xcd, t.pf))
    out.append(p.make_tile(p.TILE_PLAIN, 32, 4, 1, 2))
    out.append(p.make_tile(p.TILE_PLAIN, 64, 2, 1, 1))
    return out


@pytest.mark.parametrize("R,shape", [(4, (72, 45, 37)), (5, (61, 29, 23)), (3, (66, 20, 12))])
def test_one_step_tiles_keep_guards(R, shape):
    nx, ny, nz = shape
    nt = 3
    v, dt, vmax, u0, um1 = _case(shape, 300 + R)
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax)
    grid = (nz, ny, nx)
    kg = Guarded(grid, init=prop.kappa)
    srcs = _sources(shape, dt, nt)
    refs = []
    for src in srcs:  # unguarded reference with the context's default tile
        a, b = prop.run(cuda(u0), cuda(um1), nt, src)
        torch.cuda.synchronize()
        refs.append((a.clone(), b.clone()))
    tiles = _one_step_tiles(R, nx, nz)
    log(f"case: guards, one step, R={R} {shape}, {len(tiles)} tiles x 2 source sets x {nt} steps")
    for t in tiles:
        prop.tile = t
        for src, (ra, rb) in zip(srcs, refs):
            a, b = Guarded(grid, init=cuda(u0)), Guarded(grid, init=cuda(um1))
            for it in range(nt):
                p.stencil_step(prop.ctx, kg.t, a.t, b.t, it, src)
                a, b = b, a
            torch.cuda.synchronize()
            assert a.intact() and b.intact() and kg.intact(), f"guard written, tile {t}"
            assert torch.equal(a.t, ra) and torch.equal(b.t, rb), f"tile {t}"
            assert bool(torch.isfinite(a.t).all()), f"tile {t}"


def test_two_step_keeps_guards():
    shape, R, nt = (72, 45, 37), 4, 6
    nx, ny, nz = shape
    grid = (nz, ny, nx)
    v, dt, vmax, u0, um1 = _case(shape, 310)
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax)
    kg = Guarded(grid, init=prop.kappa)
    src = _sources(shape, dt, nt)[0]
    ra, rb = prop.run(cuda(u0), cuda(um1), nt, src)
    torch.cuda.synchronize()
    ra, rb = ra.clone(), rb.clone()
    tiles = [p.make_tile(p.TILE_ZMARCH2, t.bx, t.by, 1, dz, t.vw, xcd, t.pf)
             for t in p.stencil_list_tiles2(R, True) for dz in (7, nz) for xcd in (1, 0)]
    log(f"case: guards, two-step launches, {shape}, {len(tiles)} tiles x {nt // 2} launches")
    for t in tiles:
        prop.tile = t
        f = [Guarded(grid, init=cuda(u0)), Guarded(grid, init=cuda(um1)), Guarded(grid), Guarded(grid)]
        for it in range(0, nt, 2):
            p.stencil_step2(prop.ctx, kg.t, f[0].t, f[1].t, f[2].t, f[3].t, it, src)
            f = [f[3], f[2], f[1], f[0]]
        torch.cuda.synchronize()
        assert all(g.intact() for g in f) and kg.intact(), f"guard written, tile {t}"
        assert torch.equal(f[0].t, ra) and torch.equal(f[1].t, rb), f"tile {t}"


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_16bit_storage_keeps_guards(storage):
    shape, R, nt = (72, 45, 37), 4, 3
    nx, ny, nz = shape
    grid = (nz, ny, nx)
    v, dt, vmax, u0, um1 = _case(shape, 320)
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax, storage=storage, storage_scale=256.0)
    dtype = prop.dtype
    kg = Guarded(grid, init=prop.kappa)
    srcs = _sources(shape, dt, nt)
    s0, s1 = prop.to_storage(cuda(u0)), prop.to_storage(cuda(um1))
    # The conversions themselves, into and out of guarded buffers.
    cg = Guarded(grid, dtype)
    p.stencil_convert(prop.ctx, cuda(u0), cg.t, True)
    bg = Guarded(grid)
    p.stencil_convert(prop.ctx, cg.t, bg.t, False)
    torch.cuda.synchronize()
    assert cg.intact() and bg.intact() and torch.equal(cg.t, s0) and torch.equal(bg.t, prop.to_f32(s0))
    refs = []
    for src in srcs:
        a, b = prop.run(s0.clone(), s1.clone(), nt, src)
        torch.cuda.synchronize()
        refs.append((a.clone(), b.clone()))
    tiles = []
    for w in (8, 4, 1):
        for t in p.stencil_list_tiles(R, {8: 8, 4: True, 1: False}[w], storage):
            for dz in (7, nz):
                tiles.append(p.make_tile(p.TILE_ZMARCH, t.bx, t.by, t.ry, dz, t.vw, 1, t.pf))
    tiles.append(p.make_tile(p.TILE_PLAIN, 32, 4, 1, 2))
    log(f"case: guards, {storage} storage, {shape}, {len(tiles)} tiles x 2 source sets")
    for t in tiles:
        prop.tile = t
        for src, (ra, rb) in zip(srcs, refs):
            a, b = Guarded(grid, dtype, s0), Guarded(grid, dtype, s1)
            for it in range(nt):
                p.stencil_step(prop.ctx, kg.t, a.t, b.t, it, src)
                a, b = b, a
            torch.cuda.synchronize()
            assert a.intact() and b.intact() and kg.intact(), f"guard written, tile {t}"
            assert torch.equal(a.t, ra) and torch.equal(b.t, rb), f"tile {t}"


def test_batch_keeps_guards():
    shapes = [(72, 45, 37), (40, 36, 30), (61, 29, 23)]
    tiles = [p.make_tile(bx=64, by=8, ry=2, dz=16), p.make_tile(bx=64, by=8, ry=2, dz=7), None]
    nt = 4
    props, srcs, inits, spec, guards, refs = [], [], [], [], [], []
    for i, (shape, tile) in enumerate(zip(shapes, tiles)):
        nx, ny, nz = shape
        grid = (nz, ny, nx)
        v, dt, vmax, u0, um1 = _case(shape, 330 + i)
        pr = p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, tile=tile)
        src = _sources(shape, dt, nt)[i % 2]
        a, b = pr.run(cuda(u0), cuda(um1), nt, src)
        torch.cuda.synchronize()
        refs.append((a.clone(), b.clone()))
        kg, ua, ub = Guarded(grid, init=pr.kappa), Guarded(grid, init=cuda(u0)), Guarded(grid, init=cuda(um1))
        props.append(pr)
        srcs.append(src)
        guards.append((kg, ua, ub))
        spec.append((pr.ctx, kg.t, ua.t, ub.t, src))
    log(f"case: guards, batch of {len(shapes)} shots, {nt} steps")
    h = p.stencil_batch_create(spec, 0)
    try:
        for it in range(nt):
            p.stencil_batch_step(h, it)
        torch.cuda.synchronize()
    finally:
        p.stencil_batch_destroy(h)
    for (kg, ua, ub), (ra, rb) in zip(guards, refs):
        assert kg.intact() and ua.intact() and ub.intact()
        # After an even number of steps u_a holds u^n and u_b u^{n-1}.
        assert torch.equal(ua.t, ra) and torch.equal(ub.t, rb)


def test_adjoint_gradient_samples_and_kappa_keep_guards():
    shape, R = (40, 36, 30), 4
    nx, ny, nz = shape
    grid = (nz, ny, nx)
    n = nx * ny * nz
    v, dt, vmax, u0, um1 = _case(shape, 340)
    prop = p.Propagator(cuda(v), 10.0, dt, R, vmax=vmax)
    log(f"case: guards, kappa, samples, adjoint steps and gradient terms, {shape}")
    # kappa from a guarded model into a guarded output.
    vg, kg = Guarded(grid, init=cuda(v)), Guarded(grid)
    p.stencil_kappa(prop.ctx, vg.t, kg.t)
    torch.cuda.synchronize()
    assert vg.intact() and kg.intact() and torch.equal(kg.t, prop.kappa)
    # Receiver samples into a guarded trace row (indices include ones outside the grid).
    rec = cuda(np.array([0, n - 1, workloads.centre_index(nx, ny, nz), n + 5, -3], np.int64), torch.int64)
    ug = Guarded(grid, init=cuda(u0))
    og = Guarded((rec.numel(),))
    p.stencil_sample(prop.ctx, ug.t, rec, og.t)
    ref_s = torch.zeros(rec.numel(), device="cuda:0")
    p.stencil_sample(prop.ctx, cuda(u0), rec, ref_s)
    torch.cuda.synchronize()
    assert ug.intact() and og.intact() and torch.equal(og.t, ref_s)
    # Adjoint steps with the gradient accumulated, single and paired.
    nt = 4
    resid = cuda(np.stack([workloads.ricker(nt, dt, 20.0 + 3 * j) for j in range(rec.numel())], 1))
    rs = p.make_src(rec, resid)
    fields = [workloads.random_field(nx, ny, nz, 350 + j) for j in range(6)]

    def run(make, make64):
        lam_c, lam_p = make(fields[0]), make(fields[1])
        u3, u2, u1, u0_ = make(fields[2]), make(fields[3]), make(fields[4]), make(fields[5])
        grad = make64()
        p.stencil_adjoint_step(prop.ctx, kg.t, lam_c, lam_p, 2, rs, u3, u2, u1, grad)
        p.stencil_adjoint_step(prop.ctx, kg.t, lam_p, lam_c, 1, rs)
        p.stencil_gradient2(prop.ctx, lam_p, lam_c, u3, u2, u1, u0_, grad)
        torch.cuda.synchronize()
        return lam_c, lam_p, grad

    ref = run(lambda f: cuda(f), lambda: torch.zeros(grid, dtype=torch.float64, device="cuda:0"))
    keep = []

    def make_g(f):
        g = Guarded(grid, init=cuda(f))
        keep.append(g)
        return g.t

    def make_g64():
        g = Guarded(grid, torch.float64)
        g.t.zero_()
        keep.append(g)
        return g.t

    got = run(make_g, make_g64)
    assert all(g.intact() for g in keep) and kg.intact()
    for x, y in zip(got, ref):
        assert torch.equal(x, y)
    assert bool(torch.isfinite(got[2]).all())
