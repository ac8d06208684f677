"""GPU misfit gradient (adjoint steps + checkpointed forward) against the
FP64 oracle's gradient, plus properties that hold at any size.

Bars: gradient rel-L2 <= 1e-4 against the oracle's (and its largest
single-point deviation <= 1e-3 of its peak); misfit within 1e-4 relative;
the adjoint dot-product identity to FP32 accuracy at 256^3."""
import sys

import numpy as np
import pytest
import torch

import oracle
from compare import check_close
from oracle import adjoint as oadj
import paper_1310_8232_amd as p
from paper_1310_8232_amd import adjoint
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


def _problem(nx, ny, nz, nt, seed, radius=4, f0=25.0, blob=-0.15, width=None):
    # A strong, wide blob so that the residual is a sizeable fraction of the
    # traces (15-25%): the FP32 traces' own error then stays far below the
    # residual and the gradient comparison measures the adjoint, not FP32
    # cancellation in a tiny residual.
    c = workloads.config_gradient(nx, ny, nz, nt=nt, seed=seed, radius=radius, f0=f0, blob=blob,
                                  blob_width=width if width is not None else min(nx, ny, nz) / 4.0)
    kap_true = oadj.kappa_from_slowness2(c["m_true"], c["dt"], c["h"])
    obs = oadj.traces(oadj.forward_all(kap_true, radius, nt, c["src_idx"], c["amp"]), c["rec_idx"])
    return c, obs.astype(np.float32)


def _survey(c):
    return adjoint.Survey(cuda(c["src_idx"], torch.int64), cuda(c["amp"].reshape(-1, 1)),
                          cuda(c["rec_idx"], torch.int64))


@pytest.mark.parametrize("shape,nt,radius,every", [((32, 32, 32), 150, 4, 7), ((48, 40, 36), 200, 5, 16),
                                                   ((61, 29, 23), 120, 4, 120), ((40, 34, 30), 90, 4, 0)])
def test_gradient_vs_oracle(shape, nt, radius, every):
    c, obs = _problem(*shape, nt, seed=77, radius=radius)
    log(f"case: gradient {shape} nt={nt} R={radius} checkpoint every {every}")
    J_ref, g_ref = oadj.misfit_and_gradient(c["m_cur"].astype(np.float64), c["dt"], c["h"], radius, nt,
                                            c["src_idx"], c["amp"], c["rec_idx"], obs)
    prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], radius, slowness2=True)
    J, g, _ = adjoint.misfit_gradient(prop, _survey(c), cuda(obs), checkpoint_every=every)
    torch.cuda.synchronize()
    J = float(J.item())
    log(f"  J gpu {J:.8e} oracle {J_ref:.8e}")
    check_close(g.cpu().numpy(), g_ref, 1e-4, "gradient")
    assert abs(J - J_ref) <= 1e-4 * J_ref


@pytest.mark.parametrize("n", [64, 128])
def test_gradient_config4_inputs(n):
    # The gradient workload's own inputs: layered true model, current model
    # with a -5% Gaussian blob (width n/8), 15 Hz Ricker, source and receiver
    # line at z = 2R, 500 steps, checkpoints every 50. The observed data are
    # each side's forward modelling of the true model (FP32 on the GPU, FP64
    # in the oracle), as in a synthetic inversion. The residual is only 2-5%
    # of the traces, but the rounding the GPU's two forward runs share (all
    # of it until the wave meets the blob) cancels in it. Bar: rel-L2 <= 1e-4
    # (per point: 1e-3 of the gradient's peak); misfit within 1e-4.
    nt = 500
    c = workloads.config_gradient(n, n, n, nt=nt)
    log(f"case: gradient, config-4 inputs at {n}^3, {nt} steps, checkpoints every 50")
    kap_true = oadj.kappa_from_slowness2(c["m_true"], c["dt"], c["h"])
    obs_ref = oadj.traces(oadj.forward_all(kap_true, 4, nt, c["src_idx"], c["amp"]), c["rec_idx"])
    J_ref, g_ref = oadj.misfit_and_gradient(c["m_cur"].astype(np.float64), c["dt"], c["h"], 4, nt,
                                            c["src_idx"], c["amp"], c["rec_idx"], obs_ref)
    survey = _survey(c)
    prop_true = p.Propagator(cuda(c["m_true"]), c["h"], c["dt"], 4, slowness2=True)
    obs, _, _ = adjoint.forward(prop_true, survey)
    del prop_true
    prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
    J, g, tr = adjoint.misfit_gradient(prop, survey, obs, checkpoint_every=50)
    torch.cuda.synchronize()
    J = float(J.item())
    tr_ref_norm = float(np.linalg.norm(obs_ref)) or 1.0
    log(f"  residual / traces {np.sqrt(2.0 * J_ref) / tr_ref_norm:.3e}; J gpu {J:.8e} oracle {J_ref:.8e}")
    check_close(g.cpu().numpy(), g_ref, 1e-4, "gradient")
    assert abs(J - J_ref) <= 1e-4 * J_ref


def test_checkpoint_interval_does_not_change_bits():
    c, obs = _problem(40, 36, 30, 45, seed=3)
    prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
    out = []
    for every in (1, 7, 45, 100, 0):  # 0: every level kept, no recompute
        J, g, tr = adjoint.misfit_gradient(prop, _survey(c), cuda(obs), checkpoint_every=every)
        out.append((J.item(), g.cpu().numpy(), tr.cpu().numpy()))
    for J, g, tr in out[1:]:
        assert J == out[0][0] and np.array_equal(g, out[0][1]) and np.array_equal(tr, out[0][2])


def test_gradient_terms_are_the_bits_of_single_terms():
    # m terms in one pass (m = 1..4, also the scalar path on a grid whose point
    # count is not a multiple of 4) equal m single-term passes; the one-term
    # pass equals the accumulation inside stencil_adjoint_step.
    for shape in ((40, 34, 30), (61, 29, 23)):
        nx, ny, nz = shape
        c, _ = _problem(nx, ny, nz, 8, seed=5)
        prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
        f = [cuda(workloads.random_field(nx, ny, nz, 90 + j)) for j in range(10)]
        g0 = torch.from_numpy(np.random.default_rng(7).standard_normal((nz, ny, nx))).to("cuda:0")
        log(f"case: gradient terms m = 1..4 against single terms, {shape}")
        for m in (1, 2, 3, 4):
            mu, u = f[:m], f[4:4 + m + 2]
            ga, gb = g0.clone(), g0.clone()
            p.stencil_gradient_terms(prop.ctx, mu, u, ga)
            for j in range(m):
                p.stencil_gradient_terms(prop.ctx, [mu[j]], u[j:j + 3], gb)
            torch.cuda.synchronize()
            assert torch.equal(ga, gb), f"m={m}"
        lam_c, lam_p = f[0].clone(), f[1].clone()
        ga, gb = g0.clone(), g0.clone()
        p.stencil_adjoint_step(prop.ctx, prop.kappa, lam_c, lam_p, 3, None, f[4], f[5], f[6], ga)
        p.stencil_gradient_terms(prop.ctx, [lam_p], [f[4], f[5], f[6]], gb)
        torch.cuda.synchronize()
        assert torch.equal(ga, gb)


def test_autograd_function():
    c, obs = _problem(32, 28, 24, 40, seed=12)
    m = cuda(c["m_cur"]).requires_grad_(True)
    J = adjoint.SlownessMisfit.apply(m, _survey(c), cuda(obs), c["h"], c["dt"], 4, 10)
    J.backward()
    prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
    J2, g2, _ = adjoint.misfit_gradient(prop, _survey(c), cuda(obs), checkpoint_every=10)
    assert float(J.item()) == float(J2.item())
    assert torch.equal(m.grad, g2.to(torch.float32))


def test_kappa_from_slowness2_bit_exact():
    c, _ = _problem(20, 18, 16, 5, seed=1)
    prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
    ref = oadj.kappa_from_slowness2(c["m_cur"], c["dt"], c["h"]).astype(np.float32)
    assert np.array_equal(prop.kappa.cpu().numpy(), ref)


def test_misfit_kernel_fp64_reduction():
    rng = np.random.default_rng(8)
    tr = rng.standard_normal((300, 77)).astype(np.float32)
    ob = rng.standard_normal((300, 77)).astype(np.float32)
    J, resid = adjoint.misfit(cuda(tr), cuda(ob))
    r = tr - ob
    assert np.array_equal(resid.cpu().numpy(), r)
    ref = 0.5 * np.sum(r.astype(np.float64) ** 2)
    assert abs(float(J.item()) - ref) <= 1e-13 * ref


@pytest.mark.slow
def test_adjoint_dot_product_256():
    # F: source samples -> receiver traces at fixed kappa; its adjoint is the
    # adjoint step driven by receiver data: <F a, b> = sum_n a_n mu^{n+1}(s).
    # With b = F a (the traces themselves) both sides equal ||F a||^2, a sum
    # of positive terms, so FP32 rounding is not amplified by cancellation
    # (random a and b would cancel ~sqrt(#samples)-fold).
    c = workloads.config_gradient(256, 256, 256, nt=500)
    log("case: adjoint dot-product identity, 256^3, 500 steps")
    nt = c["nt"]
    prop = p.Propagator(cuda(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
    a = c["amp"].astype(np.float32)
    survey = adjoint.Survey(cuda(c["src_idx"], torch.int64), cuda(a.reshape(-1, 1)), cuda(c["rec_idx"], torch.int64))
    tr, _, _ = adjoint.forward(prop, survey)
    b = tr.clone()
    lhs = float(np.sum(tr.cpu().numpy().astype(np.float64) * b.cpu().numpy().astype(np.float64)))
    rs = p.make_src(survey.rec_idx, b)
    mu_cur = torch.zeros(prop.shape, device="cuda:0")
    mu_prev = torch.zeros(prop.shape, device="cuda:0")
    at_s = torch.empty(nt, device="cuda:0")
    for k in range(nt, 0, -1):
        p.stencil_adjoint_step(prop.ctx, prop.kappa, mu_cur, mu_prev, k - 1, rs)
        mu_cur, mu_prev = mu_prev, mu_cur
        p.stencil_sample(prop.ctx, mu_cur, survey.src_idx, at_s[k - 1:k])
    rhs = float(np.dot(a.astype(np.float64), at_s.cpu().numpy().astype(np.float64)))
    log(f"  <F a, F a> = {lhs:.9e}   <a, F^T F a> = {rhs:.9e}   rel diff {abs(lhs - rhs) / lhs:.2e}")
    assert lhs > 0
    assert abs(lhs - rhs) <= 1e-4 * lhs
