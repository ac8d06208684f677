"""FP64 reference for receiver traces, the L2 misfit and its gradient with
respect to squared slowness.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward model is the leapfrog scheme of the "3D model" step (Section 2,
time loop of Algorithm 1): u^{n+1} = 2u^n - u^{n-1} + K L u^n + f^n with
K = diag(kappa), f^n = kappa(s) w_n at the source, u^0 = u^{-1} = 0, for
n = 0..N-1. Traces are u^k at the receivers for k = 1..N. The paper does not
define an imaging condition; the misfit taken here is
    J = 1/2 sum_{k=1..N} sum_r (u^k(r) - d^k(r))^2
and kappa = dt^2 / (h^2 m) with m = 1/v^2.

Gradient, written out from the Lagrangian of the recurrence (plain
definition, no reformulation):
    lambda^k = 2 lambda^{k+1} - lambda^{k+2} + L (K lambda^{k+1}) + r^k,   k = N..1,
    lambda^{N+1} = lambda^{N+2} = 0,   r^k = S^T (S u^k - d^k),
    dJ/dkappa(p) = sum_{n=0..N-1} lambda^{n+1}(p) [ (L u^n)(p) + [p = s] w_n ],
    dJ/dm(p) = dJ/dkappa(p) * dkappa/dm(p),   dkappa/dm = -dt^2 / (h^2 m^2).
L is the oracle's Laplacian (symmetric, so L^T = L).
"""
from __future__ import annotations

import numpy as np

from . import laplacian, leapfrog


def kappa_from_slowness2(m: np.ndarray, dt: float, h: float) -> np.ndarray:
    """kappa = dt^2 / (h^2 m) in FP64."""
    return dt * dt / (h * h * np.asarray(m, dtype=np.float64))


def forward_all(kap: np.ndarray, R: int, nt: int, src_idx, amp):
    """All time levels u^{-1}, u^0, ..., u^{nt} (FP64) from rest."""
    z = np.zeros(kap.shape)
    us = [z.copy(), z.copy()]  # u^{-1}, u^0
    uc, up = z, z
    for n in range(nt):
        uc, up = leapfrog(kap, uc, up, R, 1, it0=n, src_idx=src_idx, amp=amp)
        us.append(uc.copy())
    return us  # us[n + 1] = u^n


def traces(us, rec_idx) -> np.ndarray:
    """[nt, nrec] samples u^k(r), k = 1..nt."""
    rec = np.asarray(rec_idx, dtype=np.int64)
    return np.stack([u.ravel()[rec] for u in us[2:]])


def misfit(tr: np.ndarray, observed: np.ndarray) -> float:
    d = np.asarray(tr, np.float64) - np.asarray(observed, np.float64)
    return 0.5 * float(np.sum(d * d))


def misfit_of_model(m, dt, h, R, nt, src_idx, amp, rec_idx, observed) -> float:
    kap = kappa_from_slowness2(m, dt, h)
    return misfit(traces(forward_all(kap, R, nt, src_idx, amp), rec_idx), observed)


def adjoint_traces(kap: np.ndarray, R: int, resid: np.ndarray, rec_idx):
    """The adjoint recurrence driven by receiver residuals resid [nt, nrec];
    returns lambda^1..lambda^{nt} as a list (index k-1)."""
    nt = resid.shape[0]
    rec = np.asarray(rec_idx, dtype=np.int64)
    shape = kap.shape
    lam_next = np.zeros(shape)   # lambda^{k+1}
    lam_next2 = np.zeros(shape)  # lambda^{k+2}
    out = [None] * nt
    for k in range(nt, 0, -1):
        r = np.zeros(kap.size)
        np.add.at(r, rec, resid[k - 1])
        lam = 2.0 * lam_next - lam_next2 + laplacian(kap * lam_next, R) + r.reshape(shape)
        out[k - 1] = lam
        lam_next2, lam_next = lam_next, lam
    return out


def misfit_and_gradient(m, dt, h, R, nt, src_idx, amp, rec_idx, observed):
    """(J, dJ/dm) in FP64. amp: [nt, nsrc] (or [nt]) source samples."""
    m = np.asarray(m, dtype=np.float64)
    kap = kappa_from_slowness2(m, dt, h)
    us = forward_all(kap, R, nt, src_idx, amp)
    tr = traces(us, rec_idx)
    resid = tr - np.asarray(observed, np.float64)
    J = 0.5 * float(np.sum(resid * resid))
    lams = adjoint_traces(kap, R, resid, rec_idx)
    src = np.asarray(src_idx, dtype=np.int64).ravel()
    a = np.asarray(amp, dtype=np.float64).reshape(nt, -1)
    g_kappa = np.zeros(m.shape)
    for n in range(nt):
        term = laplacian(us[n + 1], R)  # L u^n
        flat = term.ravel()
        for j, s in enumerate(src):
            flat[s] += a[n, j]
        g_kappa += lams[n] * term  # lams[n] = lambda^{n+1}
    dkdm = -dt * dt / (h * h * m * m)
    return J, g_kappa * dkdm
