"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds only input recipes (velocity models, the source wavelet,
random fields, the source position and the time step chosen from a Courant
number); none of the method's arithmetic (coefficients, kappa, the stencil,
the time step update) lives here. Both the FP64 oracle and the GPU path take
these arrays as inputs.

The paper (RTM on field data from deep-water surveys) uses no public dataset;
these synthetic models stand in for its velocity models.
"""
from __future__ import annotations

import math

import numpy as np

SEED = 13108232


def ricker(nt: int, dt: float, f0: float = 15.0, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(t_n), t_n = n dt: (1 - 2a) exp(-a), a = (pi f0 (t - t0))^2.

    Sampled in FP64, returned as FP32 (the GPU path's input type)."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f0 * (t - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def constant_model(nx: int, ny: int, nz: int, v: float = 2000.0) -> np.ndarray:
    """Homogeneous velocity model [nz, ny, nx], FP32."""
    return np.full((nz, ny, nx), v, dtype=np.float32)


def layered_model(nx: int, ny: int, nz: int, seed: int = SEED, nlayers: int = 20,
                  vlo: float = 1500.0, vhi: float = 4500.0, noise: float = 0.02) -> np.ndarray:
    """Layered model [nz, ny, nx], FP32.

    Draw order from ``numpy.random.default_rng(seed)``: (1) nlayers-1 distinct
    interface depths from 1..nz-1, sorted; (2) nlayers layer velocities
    U[vlo, vhi]; (3) per-point factors 1 + U[-noise, noise] in C order
    (z, then y, then x), drawn plane by plane. Layers are capped at nz.
    """
    rng = np.random.default_rng(seed)
    nl = max(1, min(nlayers, nz))
    depths = np.sort(rng.choice(np.arange(1, nz), size=nl - 1, replace=False)) if nl > 1 else np.zeros(0, np.int64)
    vel = rng.uniform(vlo, vhi, size=nl)
    layer_of_z = np.searchsorted(depths, np.arange(nz), side="right")
    out = np.empty((nz, ny, nx), dtype=np.float32)
    for z in range(nz):
        f = 1.0 + rng.uniform(-noise, noise, size=(ny, nx))
        out[z] = (vel[layer_of_z[z]] * f).astype(np.float32)
    return out


def random_field(nx: int, ny: int, nz: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded U[-scale, scale] field [nz, ny, nx], FP32 (drawn in FP64)."""
    rng = np.random.default_rng(seed)
    out = np.empty((nz, ny, nx), dtype=np.float32)
    for z in range(nz):
        out[z] = (rng.uniform(-scale, scale, size=(ny, nx))).astype(np.float32)
    return out


def centre_index(nx: int, ny: int, nz: int) -> int:
    """Linear index (z*ny + y)*nx + x of (nz//2, ny//2, nx//2)."""
    return ((nz // 2) * ny + ny // 2) * nx + nx // 2


def dt_for_courant(v: np.ndarray, h: float, courant: float = 0.4) -> tuple[float, float]:
    """(dt, vmax) with vmax the largest value of the FP32 model and
    dt = courant * h / vmax."""
    vmax = float(np.max(v))
    return courant * h / vmax, vmax


def config_plain(nx: int = 64, ny: int = 64, nz: int = 64, nt: int = 100):
    """Plain-method workload: constant 2000 m/s, h = 10 m, Courant 0.4 (dt = 2 ms),
    15 Hz Ricker at the grid centre, 8th order, ``nt`` steps."""
    h = 10.0
    v = constant_model(nx, ny, nz, 2000.0)
    dt, vmax = dt_for_courant(v, h)
    return dict(name=f"constant {nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, dt=dt, vmax=vmax,
                v=v, radius=4, nt=nt, src_idx=np.array([centre_index(nx, ny, nz)], np.int64),
                amp=ricker(nt, dt))


def config_layered(nx: int = 512, ny: int = 512, nz: int = 512, nt: int = 1000, seed: int = SEED,
                   radius: int = 4):
    """Throughput workload: layered model (20 layers, 1500-4500 m/s, 2% noise),
    h = 10 m, Courant 0.4 on the model's max velocity, centred 15 Hz Ricker."""
    h = 10.0
    v = layered_model(nx, ny, nz, seed)
    dt, vmax = dt_for_courant(v, h)
    return dict(name=f"layered {nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, dt=dt, vmax=vmax,
                v=v, radius=radius, nt=nt, src_idx=np.array([centre_index(nx, ny, nz)], np.int64),
                amp=ricker(nt, dt))


def blob_factor(nx: int, ny: int, nz: int, seed: int, amplitude: float = -0.05, width: float | None = None):
    """1 + amplitude * exp(-r^2 / (2 w^2)) around a seeded centre in the middle
    half of each axis (w = min(n)/8 by default), FP64 [nz, ny, nx]."""
    rng = np.random.default_rng(seed)
    cz, cy, cx = (rng.uniform(0.25, 0.75) * (n - 1) for n in (nz, ny, nx))
    w = width if width is not None else min(nx, ny, nz) / 8.0
    z = np.arange(nz)[:, None, None] - cz
    y = np.arange(ny)[None, :, None] - cy
    x = np.arange(nx)[None, None, :] - cx
    return 1.0 + amplitude * np.exp(-(x * x + y * y + z * z) / (2.0 * w * w))


def receiver_line(nx: int, ny: int, nz: int, radius: int = 4) -> np.ndarray:
    """Linear indices of every x in [R, nx-R) at y = ny//2, z = min(2R, nz-1)."""
    z = min(2 * radius, nz - 1)
    xs = np.arange(radius, max(nx - radius, radius + 1))
    xs = xs[xs < nx]
    return ((z * ny + ny // 2) * nx + xs).astype(np.int64)


def config_gradient(nx: int = 256, ny: int = 256, nz: int = 256, nt: int = 500, seed: int = SEED + 2,
                    radius: int = 4, courant: float = 0.4, f0: float = 15.0, blob: float = -0.05,
                    blob_width: float | None = None):
    """Gradient workload: true layered model (seed), current model with a
    seeded Gaussian blob of `blob` relative velocity (-5%), source
    (z = 2R, ny//2, nx//2), Ricker of peak frequency f0, receiver line at
    z = 2R; squared slowness m = 1/v^2 (FP32)."""
    h = 10.0
    v_true = layered_model(nx, ny, nz, seed)
    v_cur = (v_true.astype(np.float64) * blob_factor(nx, ny, nz, seed + 1, blob, blob_width)).astype(np.float32)
    dt, vmax = dt_for_courant(v_true, h, courant)
    zs = min(2 * radius, nz - 1)
    src = np.array([(zs * ny + ny // 2) * nx + nx // 2], np.int64)
    m_true = (1.0 / (v_true.astype(np.float64) ** 2)).astype(np.float32)
    m_cur = (1.0 / (v_cur.astype(np.float64) ** 2)).astype(np.float32)
    return dict(name=f"gradient {nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, h=h, dt=dt, vmax=vmax, radius=radius,
                nt=nt, v_true=v_true, v_cur=v_cur, m_true=m_true, m_cur=m_cur, src_idx=src,
                amp=ricker(nt, dt, f0), rec_idx=receiver_line(nx, ny, nz, radius))


def batch_shapes(seed: int = SEED + 1, n: int = 16):
    """Shot grid sizes (nx, ny, nz): 384x192x128, 96^3, 256^3, then dims drawn
    from multiples of 32 in [96, 384], redrawn until the volume lies in
    [96^3, 256^3]."""
    rng = np.random.default_rng(seed)
    out = [(384, 192, 128), (96, 96, 96), (256, 256, 256)]
    choices = np.arange(96, 385, 32)
    while len(out) < n:
        d = tuple(int(x) for x in rng.choice(choices, size=3))
        if 96 ** 3 <= d[0] * d[1] * d[2] <= 256 ** 3:
            out.append(d)
    return out[:n]


def config_batch(n: int = 16, nt: int = 500, seed: int = SEED + 1, shapes=None):
    """Uneven shots: each with its own layered model (seed SEED + 100 + i),
    h = 10 m, Courant 0.4 on its own max velocity, centred 15 Hz Ricker."""
    shapes = shapes or batch_shapes(seed, n)
    shots = []
    for i, (nx, ny, nz) in enumerate(shapes):
        c = config_layered(nx, ny, nz, nt=nt, seed=SEED + 100 + i)
        shots.append(c)
    return shots
