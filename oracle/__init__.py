"""FP64 CPU oracle for the leapfrog star-stencil step and the blocksize search.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU path (``paper_1310_8232_amd``) and imports nothing from it.

Contents
--------
* ``fd_coefficients``, ``cfl_limit``, ``kappa``, ``laplacian``, ``leapfrog``:
  thin ctypes wrappers over ``stencil_oracle.c`` (plain FP64 loops), following
  the paper's Section 2 (the "3D model" finite-difference step of Algorithm 1,
  star stencil of Fig. 1(a)).
* ``select_block``: the three-stage blocksize selection of Section 3.3
  (Eqs. 1-3 and the stage-3 rule), as a pure function of a timing table.
* ``pgrid``: the per-dimension candidate lists of Section 3.7.
* ``rel_l2``, ``max_rel``: the comparison measures used against the GPU path
  (a global one and a per-element one).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .tuner import POLICIES, gap, pgrid, pgrid_candidates, select_block  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libstencil_oracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_lp = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_fd_coefficients.argtypes = [ctypes.c_int, _dp]
    lib.oracle_fd_coefficients.restype = ctypes.c_int
    lib.oracle_cfl_limit.argtypes = [ctypes.c_int]
    lib.oracle_cfl_limit.restype = ctypes.c_double
    lib.oracle_kappa.argtypes = [_i64, _fp, ctypes.c_double, ctypes.c_double, _dp]
    lib.oracle_kappa.restype = None
    lib.oracle_laplacian.argtypes = [ctypes.c_int, _i64, _i64, _i64, _dp, _dp]
    lib.oracle_laplacian.restype = ctypes.c_int
    lib.oracle_leapfrog.argtypes = [ctypes.c_int, _i64, _i64, _i64, _dp, _dp, _dp,
                                    _i64, _i64, _i32, _lp, _dp]
    lib.oracle_leapfrog.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def fd_coefficients(R: int) -> np.ndarray:
    """c_0..c_R of the order-2R central second difference (Section 2 states
    order 10 in space; the weights themselves are not printed)."""
    c = np.zeros(9, dtype=np.float64)
    if _load().oracle_fd_coefficients(R, _ptr(c, _dp)) != 0:
        raise ValueError(f"radius {R} outside 1..8")
    return c[: R + 1].copy()


def cfl_limit(R: int) -> float:
    """Largest stable v*dt/h of the 3D leapfrog scheme with radius R."""
    r = _load().oracle_cfl_limit(R)
    if r < 0:
        raise ValueError(f"radius {R} outside 1..8")
    return r


def kappa(v: np.ndarray, dt: float, h: float) -> np.ndarray:
    """(v dt / h)^2 in FP64 from an FP32 velocity model."""
    v = np.ascontiguousarray(v, dtype=np.float32)
    out = np.empty(v.shape, dtype=np.float64)
    _load().oracle_kappa(v.size, _ptr(v, _fp), float(dt), float(h), _ptr(out, _dp))
    return out


def laplacian(u: np.ndarray, R: int) -> np.ndarray:
    """Dimensionless star Laplacian L u of a [nz, ny, nx] field, zero outside."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    if _load().oracle_laplacian(R, nx, ny, nz, _ptr(u, _dp), _ptr(out, _dp)) != 0:
        raise ValueError(f"radius {R} outside 1..8")
    return out


def leapfrog(kap: np.ndarray, u_cur: np.ndarray, u_prev: np.ndarray, R: int,
             nsteps: int, it0: int = 0, src_idx=None, amp=None):
    """Advance (u^{it0}, u^{it0-1}) by ``nsteps`` leapfrog steps in FP64.

    ``src_idx``: linear source indices (int64, [nsrc]); ``amp``: wavelet
    samples [nt, nsrc] (or [nt] for one source), row n injected at step n.
    Returns (u^{it0+nsteps}, u^{it0+nsteps-1}) as new float64 arrays.
    """
    kap = np.ascontiguousarray(kap, dtype=np.float64)
    uc = np.array(u_cur, dtype=np.float64, order="C", copy=True)
    up = np.array(u_prev, dtype=np.float64, order="C", copy=True)
    if kap.shape != uc.shape or up.shape != uc.shape or uc.ndim != 3:
        raise ValueError("kappa, u_cur and u_prev must share one [nz, ny, nx] shape")
    nz, ny, nx = uc.shape
    if src_idx is None or len(np.atleast_1d(src_idx)) == 0:
        idx = np.zeros(1, dtype=np.int64)
        a = np.zeros(1, dtype=np.float64)
        nsrc = 0
    else:
        idx = np.ascontiguousarray(np.atleast_1d(src_idx), dtype=np.int64)
        nsrc = idx.size
        a = np.ascontiguousarray(amp, dtype=np.float64).reshape(-1, nsrc)
        if a.shape[0] < it0 + nsteps:
            raise ValueError("amp holds fewer rows than it0 + nsteps")
    rc = _load().oracle_leapfrog(R, nx, ny, nz, _ptr(kap, _dp), _ptr(uc, _dp), _ptr(up, _dp),
                                 int(it0), int(nsteps), int(nsrc), _ptr(idx, _lp), _ptr(a, _dp))
    if rc == -1:
        raise ValueError(f"radius {R} outside 1..8")
    if rc == -2:
        raise ValueError("source index outside the grid")
    if rc != 0:
        raise MemoryError("oracle work buffer")
    return uc, up


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's later loops (for timing on one core)."""
    _load().oracle_set_num_threads(int(n))


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2, accumulated in FP64."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if a.size != ref.size:
        raise ValueError("a and ref must hold the same number of values")
    den = float(np.sqrt(np.dot(ref, ref)))
    num = float(np.sqrt(np.dot(a - ref, a - ref)))
    return num / den if den > 0 else num


def max_rel(a: np.ndarray, ref: np.ndarray) -> float:
    """max_i |a_i - ref_i| / max_i |ref_i| in FP64: the largest single-point
    deviation, on the scale of the reference's largest value (a zero
    reference gives the largest absolute deviation). A defect confined to a
    few points, which a global norm over a large grid can hide, shows here."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if a.size != ref.size:
        raise ValueError("a and ref must hold the same number of values")
    if a.size == 0:
        return 0.0
    den = float(np.max(np.abs(ref)))
    num = float(np.max(np.abs(a - ref)))
    return num / den if den > 0 else num

