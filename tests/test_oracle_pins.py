"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against mathematics or printed values that fix
the result independently: textbook central-difference weights, polynomial
exactness, the closed-form leading truncation error, a dense Kronecker-sum
operator on a small non-cubic grid, the plane-wave symbol, the discrete
energy of leapfrog, exact discrete dispersion, reciprocity, and the leapfrog
stability limit from brute-force eigenvalues.
"""
from fractions import Fraction
import math

import numpy as np
import pytest

import oracle
import workloads

# Textbook order-2R central second-difference weights (Fornberg's tables).
EXACT = {
    1: [Fraction(-2), Fraction(1)],
    2: [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)],
    3: [Fraction(-49, 18), Fraction(3, 2), Fraction(-3, 20), Fraction(1, 90)],
    4: [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)],
    5: [Fraction(-5269, 1800), Fraction(5, 3), Fraction(-5, 21), Fraction(5, 126),
        Fraction(-5, 1008), Fraction(1, 3150)],
}


@pytest.mark.parametrize("R", [1, 2, 3, 4, 5])
def test_coefficients_match_textbook(R):
    c = oracle.fd_coefficients(R)
    ref = np.array([float(f) for f in EXACT[R]])
    np.testing.assert_allclose(c, ref, rtol=2e-15, atol=0)


@pytest.mark.parametrize("R", range(1, 9))
def test_coefficient_moment_conditions(R):
    # sum_m 2 c_m m^{2j} = 2 delta_{j1}, j = 1..R; c_0 = -2 sum c_m.
    c = oracle.fd_coefficients(R)
    for j in range(1, R + 1):
        mom = sum(2.0 * c[m] * m ** (2 * j) for m in range(1, R + 1))
        scale = sum(abs(2.0 * c[m]) * m ** (2 * j) for m in range(1, R + 1))
        assert abs(mom - (2.0 if j == 1 else 0.0)) <= 1e-13 * scale
    assert abs(c[0] + 2.0 * c[1:].sum()) <= 1e-14 * abs(c[0])


def _grid(n, h):
    # Coordinates symmetric about 0: x_i = (i - (n-1)/2) h.
    return (np.arange(n) - (n - 1) / 2.0) * h


def _poly_field(a, b, cc, shape, h):
    nz, ny, nx = shape
    z = _grid(nz, h)[:, None, None]
    y = _grid(ny, h)[None, :, None]
    x = _grid(nx, h)[None, None, :]
    u = (x ** a) * (y ** b) * (z ** cc)
    d2 = lambda t, p: p * (p - 1) * t ** (p - 2) if p >= 2 else 0.0 * t
    lap = d2(x, a) * y ** b * z ** cc + x ** a * d2(y, b) * z ** cc + x ** a * y ** b * d2(z, cc)
    return np.ascontiguousarray(np.broadcast_to(u, shape)), np.broadcast_to(lap, shape)


@pytest.mark.parametrize("R", [4, 5])
@pytest.mark.parametrize("abc", [(0, 0, 0), (1, 1, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2),
                                 (9, 0, 0), (0, 9, 0), (0, 0, 9), (2, 3, 4), (5, 2, 2), (8, 1, 0)])
def test_polynomials_are_exact(R, abc):
    a, b, cc = abc
    if max(abc) > 2 * R + 1:
        pytest.skip("degree above 2R+1")
    shape, h = (22, 23, 24), 1.0 / 12.0
    u, lap = _poly_field(a, b, cc, shape, h)
    got = oracle.laplacian(u, R) / h ** 2
    sl = (slice(R, -R),) * 3
    np.testing.assert_allclose(got[sl], lap[sl], rtol=0, atol=1e-8 * max(1.0, np.abs(lap[sl]).max()))


@pytest.mark.parametrize("R,const", [(4, -1152.0), (5, 28800.0)])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_leading_truncation_error(R, const, axis):
    # For u = t^{2R+2} along one axis, Lu/h^2 - u'' = h^{2R} sum_m 2 c_m m^{2R+2},
    # a constant; the sum is -1152 for R=4 and 28800 for R=5.
    p = 2 * R + 2
    exps = [0, 0, 0]
    exps[2 - axis] = p  # (a, b, c) are the x, y, z exponents; axis 0 = z
    shape, h = (26, 27, 28), 1.0 / 8.0
    u, lap = _poly_field(exps[0], exps[1], exps[2], shape, h)
    got = oracle.laplacian(u, R) / h ** 2 - lap
    sl = (slice(R, -R),) * 3
    np.testing.assert_allclose(got[sl], const * h ** (2 * R), rtol=2e-5)


def test_constant_field_interior_zero():
    u = np.full((20, 21, 22), 3.25)
    got = oracle.laplacian(u, 4)
    assert np.abs(got[4:-4, 4:-4, 4:-4]).max() <= 1e-13


@pytest.mark.parametrize("R", [4, 5])
def test_plane_wave_symbol(R):
    shape, h = (24, 25, 26), 1.0
    k = np.array([0.7, -1.3, 2.1])  # (kz, ky, kx)
    phi = 0.3
    zz, yy, xx = np.meshgrid(*(np.arange(n, dtype=np.float64) for n in shape), indexing="ij")
    u = np.cos(k[0] * zz + k[1] * yy + k[2] * xx + phi)
    c = [float(f) for f in EXACT[R]]
    sigma = sum(c[0] + 2 * sum(c[m] * math.cos(m * kd * h) for m in range(1, R + 1)) for kd in k)
    got = oracle.laplacian(u, R)
    sl = (slice(R, -R),) * 3
    np.testing.assert_allclose(got[sl], sigma * u[sl], rtol=0, atol=1e-12)


def _toeplitz(n, R):
    c = [float(f) for f in EXACT[R]]
    T = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if abs(i - j) <= R:
                T[i, j] = c[abs(i - j)]
    return T


@pytest.mark.parametrize("R", [4, 5])
def test_dense_operator_brute_force(R):
    # A = Tz (x) Iy (x) Ix + Iz (x) Ty (x) Ix + Iz (x) Iy (x) Tx on a non-cubic
    # grid, with the truncated Toeplitz T (zero outside = zero Dirichlet).
    nz, ny, nx = 7, 8, 9
    A = (np.kron(np.kron(_toeplitz(nz, R), np.eye(ny)), np.eye(nx))
         + np.kron(np.kron(np.eye(nz), _toeplitz(ny, R)), np.eye(nx))
         + np.kron(np.kron(np.eye(nz), np.eye(ny)), _toeplitz(nx, R)))
    rng = np.random.default_rng(5)
    for _ in range(3):
        u = rng.standard_normal((nz, ny, nx))
        got = oracle.laplacian(u, R).ravel()
        np.testing.assert_allclose(got, A @ u.ravel(), rtol=0, atol=1e-12)
    # Symmetric, negative definite, spectrum inside (0, 3|chat(pi)|).
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(-A)
    chat_pi = abs(sum(2 * float(EXACT[R][m]) * (-1) ** m for m in range(1, R + 1)) + float(EXACT[R][0]))
    assert ev.min() > 0 and ev.max() < 3 * chat_pi


@pytest.mark.parametrize("R,limit", [(4, 0.452856), (5, 0.441942)])
def test_cfl_limit_from_eigenvalues(R, limit):
    # The 1D operator's largest |eigenvalue| tends to |chat(pi)| as n grows;
    # leapfrog is stable while kappa * 3 * that value <= 4.
    lam = np.linalg.eigvalsh(-_toeplitz(600, R)).max()
    brute = 2.0 / math.sqrt(3.0 * lam)
    assert abs(oracle.cfl_limit(R) - brute) < 1e-5
    assert abs(oracle.cfl_limit(R) - limit) < 1e-6


def test_cfl_limit_separates_stable_from_unstable():
    R, shape = 4, (16, 17, 18)
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(shape)
    lim = oracle.cfl_limit(R)
    norms = {}
    for f in (0.98, 1.08):
        kap = np.full(shape, (f * lim) ** 2)
        uc, _ = oracle.leapfrog(kap, u0, u0, R, 300)
        norms[f] = np.abs(uc).max()
    assert norms[0.98] < 50.0
    assert norms[1.08] > 1e6


def test_kappa_definition():
    v = np.array([2000.0, 1500.0, 4500.0], np.float32).reshape(1, 1, 3)
    got = oracle.kappa(v, 0.002, 10.0)
    np.testing.assert_allclose(got.ravel(), [0.16, 0.09, 0.81], rtol=1e-15)


def test_leapfrog_energy_is_conserved():
    # E^{n+1/2} = sum (u^{n+1}-u^n)^2 / kappa - <u^{n+1}, L u^n> is exactly
    # conserved by source-free leapfrog when L is symmetric; variable kappa.
    R, shape = 4, (18, 19, 20)
    rng = np.random.default_rng(11)
    kap = rng.uniform(0.02, 0.18, size=shape)
    up = rng.standard_normal(shape)
    uc = up + 0.05 * rng.standard_normal(shape)

    def energy(a, b):  # a = u^{n+1}, b = u^n
        return float(np.sum((a - b) ** 2 / kap) - np.sum(a * oracle.laplacian(b, R)))

    e0 = energy(uc, up)
    for _ in range(4):
        uc, up = oracle.leapfrog(kap, uc, up, R, 50)
        assert abs(energy(uc, up) - e0) <= 1e-11 * abs(e0)


def test_leapfrog_discrete_dispersion():
    # With constant kappa, u^n = cos(k.x - w n dt), cos(w dt) = 1 + kappa sigma(k)/2,
    # solves the recurrence exactly away from the faces (influence R per step).
    R, n, nsteps = 4, 44, 5
    k = np.array([0.9, 0.4, -1.7])
    kap = 0.1
    c = [float(f) for f in EXACT[R]]
    sigma = sum(c[0] + 2 * sum(c[m] * math.cos(m * kd) for m in range(1, R + 1)) for kd in k)
    wdt = math.acos(1.0 + kap * sigma / 2.0)
    zz, yy, xx = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    phase = k[0] * zz + k[1] * yy + k[2] * xx
    uc, up = oracle.leapfrog(np.full((n, n, n), kap), np.cos(phase), np.cos(phase + wdt), R, nsteps)
    lo, hi = R * nsteps, n - R * nsteps
    sl = (slice(lo, hi),) * 3
    np.testing.assert_allclose(uc[sl], np.cos(phase - nsteps * wdt)[sl], rtol=0, atol=1e-12)
    np.testing.assert_allclose(up[sl], np.cos(phase - (nsteps - 1) * wdt)[sl], rtol=0, atol=1e-12)


def test_source_first_two_steps_exact():
    # From zero fields: u^1 = kappa_s w_0 at s only; u^2 = 2u^1 + kappa L u^1 + kappa_s w_1 d_s.
    R, (nz, ny, nx) = 4, (9, 11, 13)
    rng = np.random.default_rng(2)
    kap = rng.uniform(0.05, 0.15, size=(nz, ny, nx))
    s = workloads.centre_index(nx, ny, nz)
    sz, sy, sx = nz // 2, ny // 2, nx // 2
    assert s == (sz * ny + sy) * nx + sx
    amp = np.array([0.7, -0.4], np.float64)
    z0 = np.zeros((nz, ny, nx))
    u1, u0 = oracle.leapfrog(kap, z0, z0, R, 1, src_idx=[s], amp=amp)
    expect1 = np.zeros((nz, ny, nx))
    expect1[sz, sy, sx] = kap[sz, sy, sx] * 0.7
    np.testing.assert_array_equal(u1, expect1)
    np.testing.assert_array_equal(u0, z0)
    u2, _ = oracle.leapfrog(kap, u1, u0, R, 1, it0=1, src_idx=[s], amp=amp)
    a = expect1[sz, sy, sx]
    c = [float(f) for f in EXACT[R]]
    assert abs(u2[sz, sy, sx] - (2 * a + kap[sz, sy, sx] * 3 * c[0] * a + kap[sz, sy, sx] * -0.4)) < 1e-15
    for m in range(1, R + 1):
        for dz, dy, dx in ((m, 0, 0), (-m, 0, 0), (0, m, 0), (0, -m, 0), (0, 0, m), (0, 0, -m)):
            p = (sz + dz, sy + dy, sx + dx)
            assert abs(u2[p] - kap[p] * c[m] * a) < 1e-16
    mask = np.zeros_like(u2, dtype=bool)
    mask[sz, sy, sx] = True
    for m in range(1, R + 1):
        mask[sz - m: sz + m + 1, sy, sx] = True
        mask[sz, sy - m: sy + m + 1, sx] = True
        mask[sz, sy, sx - m: sx + m + 1] = True
    assert np.all(u2[~mask] == 0.0)


def test_reciprocity_constant_kappa():
    R, shape = 4, (14, 15, 17)
    kap = np.full(shape, 0.12)
    nsteps = 30
    amp = workloads.ricker(nsteps, 0.004, f0=25.0).astype(np.float64)
    a = (3 * shape[1] + 5) * shape[2] + 4
    b = (10 * shape[1] + 9) * shape[2] + 12
    z = np.zeros(shape)
    ua, _ = oracle.leapfrog(kap, z, z, R, nsteps, src_idx=[a], amp=amp)
    ub, _ = oracle.leapfrog(kap, z, z, R, nsteps, src_idx=[b], amp=amp)
    assert abs(ua.ravel()[b]) > 1e-8
    assert abs(ua.ravel()[b] - ub.ravel()[a]) <= 1e-12 * abs(ua.ravel()[b])


def test_linear_in_sources():
    R, shape = 4, (12, 13, 14)
    rng = np.random.default_rng(4)
    kap = rng.uniform(0.05, 0.15, size=shape)
    idx = [100, 1000]
    amp = rng.standard_normal((6, 2))
    z = np.zeros(shape)
    both, _ = oracle.leapfrog(kap, z, z, R, 6, src_idx=idx, amp=amp)
    one, _ = oracle.leapfrog(kap, z, z, R, 6, src_idx=[idx[0]], amp=amp[:, 0].copy())
    two, _ = oracle.leapfrog(kap, z, z, R, 6, src_idx=[idx[1]], amp=amp[:, 1].copy())
    np.testing.assert_allclose(both, one + two, rtol=0, atol=1e-14)
