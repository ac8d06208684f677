"""Pins of the oracle's misfit gradient (FP64): central finite differences of
the misfit along seeded directions, and the adjoint dot-product identity."""
import numpy as np
import pytest

import oracle
from oracle import adjoint
import workloads


def _case(nx, ny, nz, nt, seed):
    c = workloads.config_gradient(nx, ny, nz, nt=nt, seed=seed)
    # Observed data: the true model's traces (oracle, FP64), stored as FP32
    # as the GPU path receives them.
    kap_true = adjoint.kappa_from_slowness2(c["m_true"], c["dt"], c["h"])
    obs = adjoint.traces(adjoint.forward_all(kap_true, 4, nt, c["src_idx"], c["amp"]), c["rec_idx"])
    return c, obs.astype(np.float32)


@pytest.mark.parametrize("shape,nt", [((14, 13, 12), 25), ((32, 32, 32), 50)])
def test_gradient_matches_central_differences(shape, nt):
    c, obs = _case(*shape, nt, seed=77)
    m = c["m_cur"].astype(np.float64)
    J, g = adjoint.misfit_and_gradient(m, c["dt"], c["h"], 4, nt, c["src_idx"], c["amp"], c["rec_idx"], obs)
    assert J > 0
    rng = np.random.default_rng(5)
    for trial in range(2):
        dm = rng.standard_normal(m.shape) * m * 1e-2
        eps = 1e-4
        jp = adjoint.misfit_of_model(m + eps * dm, c["dt"], c["h"], 4, nt, c["src_idx"], c["amp"], c["rec_idx"], obs)
        jm = adjoint.misfit_of_model(m - eps * dm, c["dt"], c["h"], 4, nt, c["src_idx"], c["amp"], c["rec_idx"], obs)
        fd = (jp - jm) / (2 * eps)
        an = float(np.sum(g * dm))
        assert abs(fd - an) <= 1e-6 * abs(an), (trial, fd, an)


def test_adjoint_dot_product():
    # F: source samples a -> traces (fixed kappa); F^T b = kappa(s) lambda^{n+1}(s).
    c, _ = _case(18, 16, 15, 30, seed=9)
    kap = adjoint.kappa_from_slowness2(c["m_cur"], c["dt"], c["h"])
    rng = np.random.default_rng(3)
    a = rng.standard_normal(30)
    b = rng.standard_normal((30, len(c["rec_idx"])))
    Fa = adjoint.traces(adjoint.forward_all(kap, 4, 30, c["src_idx"], a), c["rec_idx"])
    lams = adjoint.adjoint_traces(kap, 4, b, c["rec_idx"])
    s = int(c["src_idx"][0])
    FTb = np.array([kap.ravel()[s] * lams[n].ravel()[s] for n in range(30)])
    lhs, rhs = float(np.sum(Fa * b)), float(np.dot(a, FTb))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300)


def test_misfit_zero_at_true_model_and_gradient_zero():
    c, obs = _case(12, 12, 12, 20, seed=4)
    kap_true = adjoint.kappa_from_slowness2(c["m_true"], c["dt"], c["h"])
    tr = adjoint.traces(adjoint.forward_all(kap_true, 4, 20, c["src_idx"], c["amp"]), c["rec_idx"])
    J, g = adjoint.misfit_and_gradient(c["m_true"].astype(np.float64), c["dt"], c["h"], 4, 20, c["src_idx"],
                                       c["amp"], c["rec_idx"], tr)
    assert J == 0.0 and np.all(g == 0.0)
