"""Divergence watchdog: stencil_max_abs against torch on the same field (FP32
through both the vector and the scalar path, 16-bit storage with its scale),
NaN above +inf above every finite value, the Propagator's check_every loop
(same bits as an unchecked run, EDIVERGED once a NaN or a limit is hit), and
replays of a captured graph that contains the reduction."""
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


def _prop(shape, storage="f32", scale=1.0, seed=400):
    nx, ny, nz = shape
    v = workloads.layered_model(nx, ny, nz, seed=seed)
    dt, vmax = workloads.dt_for_courant(v, 10.0)
    return p.Propagator(cuda(v), 10.0, dt, 4, vmax=vmax, storage=storage, storage_scale=scale), dt


@pytest.mark.parametrize("shape", [(72, 45, 37), (61, 29, 23), (1, 1, 1)])
def test_max_abs_matches_torch_fp32(shape):
    nx, ny, nz = shape
    prop, _ = _prop(shape)
    u = cuda(workloads.random_field(nx, ny, nz, 401, scale=3.0))
    log(f"case: max_abs FP32 {shape}")
    got = prop.max_abs(u)
    assert float(got.item()) == float(u.abs().max().item())
    # A field starting 4 bytes into its allocation takes the scalar path.
    buf = torch.zeros(u.numel() + 1, device="cuda:0")
    w = buf[1:].view(u.shape)
    w.copy_(u)
    w.view(-1)[-1] = -1000.5
    assert float(prop.max_abs(w).item()) == 1000.5


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_max_abs_16bit_storage(storage):
    shape = (72, 45, 37)
    nx, ny, nz = shape
    prop, _ = _prop(shape, storage, 256.0)
    u32 = cuda(workloads.random_field(nx, ny, nz, 402, scale=2.0))
    s = prop.to_storage(u32)
    log(f"case: max_abs {storage}, scale 256")
    assert float(prop.max_abs(s).item()) == float(prop.to_f32(s).abs().max().item())


def test_nan_above_inf_above_finite():
    shape = (40, 36, 30)
    nx, ny, nz = shape
    prop, _ = _prop(shape)
    u = cuda(workloads.random_field(nx, ny, nz, 403))
    u.view(-1)[123] = float("-inf")
    assert float(prop.max_abs(u).item()) == float("inf")
    u.view(-1)[4567] = float("nan")
    assert np.isnan(float(prop.max_abs(u).item()))
    with pytest.raises(p.StencilError) as e:
        prop.check_finite(u)
    assert e.value.status == p.EDIVERGED


def test_watchdog_run_same_bits_and_stops_on_divergence():
    shape, nt = (64, 48, 40), 12
    nx, ny, nz = shape
    prop, dt = _prop(shape, seed=404)
    idx = cuda(np.array([workloads.centre_index(nx, ny, nz)], np.int64), torch.int64)
    amp = cuda(workloads.ricker(nt, dt, 25.0).reshape(-1, 1))
    src = p.make_src(idx, amp)
    u0 = cuda(workloads.random_field(nx, ny, nz, 405))
    um1 = cuda(workloads.random_field(nx, ny, nz, 406))
    log("case: watchdog every 5 steps, one- and two-step loops")
    ra, rb = prop.run(u0.clone(), um1.clone(), nt, src)
    for temporal in (1, 2):
        a, b = prop.run(u0.clone(), um1.clone(), nt, src, temporal=temporal, check_every=5)
        torch.cuda.synchronize()
        assert torch.equal(a, ra) and torch.equal(b, rb)
    # Two-step segments with the spares given as a tuple and as a list: the
    # segments hand the free pair on, and a list comes back holding it.
    for kind in (tuple, list):
        spare = kind([prop.zeros(), prop.zeros()])
        a, b = prop.run(u0.clone(), um1.clone(), nt, src, temporal=2, check_every=3, spare=spare)
        torch.cuda.synchronize()
        assert torch.equal(a, ra) and torch.equal(b, rb)
        if kind is list:
            assert len({t.data_ptr() for t in (a, b, *spare)}) == 4
    bad = u0.clone()
    bad.view(-1)[workloads.centre_index(nx, ny, nz)] = float("nan")
    with pytest.raises(p.StencilError) as e:
        prop.run(bad, um1.clone(), nt, src, check_every=5)
    assert e.value.status == p.EDIVERGED
    m = prop.check_finite(ra)
    with pytest.raises(p.StencilError) as e:
        prop.run(u0.clone(), um1.clone(), nt, src, check_every=4, limit=0.1 * m)
    assert e.value.status == p.EDIVERGED


def test_max_abs_in_a_captured_graph():
    shape = (64, 48, 40)
    nx, ny, nz = shape
    prop, _ = _prop(shape, seed=407)
    u = cuda(workloads.random_field(nx, ny, nz, 408))
    out = torch.zeros((), device="cuda:0")
    log("case: max_abs captured in a HIP graph, 3 replays with new data")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            p.stencil_max_abs(prop.ctx, u, out, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        u.mul_(0.5 if rep % 2 else 3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert float(out.item()) == float(u.abs().max().item()), f"replay {rep}"
        _ = (u * 2).sum().item()
