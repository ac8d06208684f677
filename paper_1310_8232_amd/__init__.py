"""Python binding of libpaper_1310_8232_amd.so (C ABI in include/stencil.h).

Argument marshalling only: every step of the computation runs in the gfx950
kernels of the library. PyTorch provides device memory and streams. Importing
this module fails loudly if the compiled library is missing; there is no CPU
fallback.

Functions carry the C names (``stencil_init``, ``stencil_step``, ...); they
accept torch tensors or raw integer device pointers and raise
``StencilError`` on a non-zero status. ``Propagator`` wraps a context for a
leapfrog time loop.
"""
from __future__ import annotations

import ctypes
import os

# torch ships its own HIP runtime (libamdhip64.so.7). Loading it before the
# library makes the library's libamdhip64.so.7 dependency resolve to that same
# runtime, so the process holds one HIP runtime and torch tensors, streams and
# the library's kernels share one device context.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaper_1310_8232_amd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_1310_8232_amd/build.py` (hipcc, gfx950). There is no CPU fallback.")

_lib = ctypes.CDLL(LIB_PATH)

# ---- status codes and enums (include/stencil.h) ----------------------------
OK, EINVAL, EUNSTABLE, ENOMEM, EDEVICE, EUNSUPPORTED, EALIAS, EDIVERGED = 0, -1, -2, -3, -4, -5, -6, -7
F32, F16, BF16 = 0, 1, 2
STORAGES = {"f32": F32, "f16": F16, "bf16": BF16}
TILE_AUTO, TILE_PLAIN, TILE_ZMARCH, TILE_ZMARCH2 = 0, 1, 2, 3
POLICY_WORST, POLICY_MIN, POLICY_AVG, POLICY_OB = 0, 1, 2, 3
POLICIES = {"worst": POLICY_WORST, "mwmb": POLICY_WORST, "min": POLICY_MIN, "mmmb": POLICY_MIN,
            "avg": POLICY_AVG, "mamb": POLICY_AVG, "ob": POLICY_OB}


class StencilTile(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("bx", ctypes.c_int32), ("by", ctypes.c_int32),
                ("ry", ctypes.c_int32), ("dz", ctypes.c_int32), ("vw", ctypes.c_int32),
                ("xcd", ctypes.c_int32), ("pf", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

    def __repr__(self):
        return "StencilTile(" + ", ".join(f"{k}={v}" for k, v in self.as_dict().items()) + ")"


class StencilDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("radius", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("h", ctypes.c_double), ("dt", ctypes.c_double), ("vmax", ctypes.c_double),
                ("device", ctypes.c_int32), ("tile", StencilTile), ("storage_scale", ctypes.c_double),
                ("pitch", ctypes.c_int64)]


class StencilSrc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("idx", ctypes.c_void_p), ("amp", ctypes.c_void_p),
                ("nt", ctypes.c_int64)]


class StencilShot(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("kappa", ctypes.c_void_p), ("u_a", ctypes.c_void_p),
                ("u_b", ctypes.c_void_p), ("src", StencilSrc)]


class StencilTuneOpts(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("n_iter", ctypes.c_int32), ("n_rep", ctypes.c_int32),
                ("warmup", ctypes.c_int32), ("parts", ctypes.c_int32), ("include_plain", ctypes.c_int32),
                ("cache_path", ctypes.c_char_p), ("table", ctypes.POINTER(ctypes.c_double)),
                ("candidates", ctypes.POINTER(StencilTile)), ("table_cap", ctypes.c_int32),
                ("temporal", ctypes.c_int32), ("scratch_c", ctypes.c_void_p), ("scratch_d", ctypes.c_void_p)]


class StencilTuneReport(ctypes.Structure):
    _fields_ = [("tile", StencilTile), ("min_time_ms", ctypes.c_double), ("actual_time_ms", ctypes.c_double),
                ("gap", ctypes.c_double), ("default_time_ms", ctypes.c_double), ("seconds", ctypes.c_double),
                ("n_candidates", ctypes.c_int32), ("from_cache", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sig = {
    "stencil_init": (_i32, [ctypes.POINTER(StencilDesc), ctypes.POINTER(_vp)]),
    "stencil_destroy": (None, [_vp]),
    "stencil_kappa": (_i32, [_vp, _vp, _vp, _vp]),
    "stencil_step": (_i32, [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(StencilSrc), _vp]),
    "stencil_step_to": (_i32, [_vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(StencilSrc), _vp]),
    "stencil_step2": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(StencilSrc), _vp]),
    "stencil_get_tile2": (_i32, [_vp, ctypes.POINTER(StencilTile)]),
    "stencil_list_tiles2": (_i32, [_i32, _i32, ctypes.POINTER(StencilTile), _i32]),
    "stencil_kappa_slowness2": (_i32, [_vp, _vp, _vp, _vp]),
    "stencil_sample": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "stencil_adjoint_step": (_i32, [_vp, _vp, _vp, _vp, _i64, ctypes.POINTER(StencilSrc), _vp, _vp, _vp, _vp,
                                    _vp]),
    "stencil_gradient2": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "stencil_gradient_terms": (_i32, [_vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp]),
    "stencil_misfit": (_i32, [_vp, _vp, _i64, _vp, _vp, _vp]),
    "stencil_batch_create": (_i32, [ctypes.POINTER(StencilShot), _i32, _i64, ctypes.POINTER(_vp)]),
    "stencil_batch_create_static": (_i32, [ctypes.POINTER(StencilShot), _i32, _i64, ctypes.POINTER(_vp)]),
    "stencil_batch_step": (_i32, [_vp, _i64, _vp]),
    "stencil_batch_tune": (_i32, [ctypes.POINTER(StencilShot), _i32, ctypes.POINTER(StencilTuneOpts),
                                  ctypes.POINTER(StencilTuneReport), _vp]),
    "stencil_batch_launches": (_i32, [_vp]),
    "stencil_batch_destroy": (None, [_vp]),
    "stencil_tune": (_i32, [_vp, _vp, _vp, _vp, ctypes.POINTER(StencilTuneOpts),
                            ctypes.POINTER(StencilTuneReport), _vp]),
    "stencil_get_tile": (_i32, [_vp, ctypes.POINTER(StencilTile)]),
    "stencil_set_tile": (_i32, [_vp, ctypes.POINTER(StencilTile)]),
    "stencil_list_tiles": (_i32, [_i32, _i32, _i32, ctypes.POINTER(StencilTile), _i32]),
    "stencil_convert": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "stencil_coefficients": (_i32, [_i32, ctypes.POINTER(ctypes.c_float)]),
    "stencil_cfl_limit": (ctypes.c_double, [_i32]),
    "stencil_select": (_i32, [ctypes.POINTER(ctypes.c_double), _i32, _i32, _i32, _i32,
                              ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_double)]),
    "stencil_pgrid": (_i32, [_i64, _i32, ctypes.POINTER(_i64), _i32]),
    "stencil_stream_probe": (_i32, [_vp, _vp, _vp, _vp, _i64, _vp]),
    "stencil_stream_probe_march": (_i32, [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp]),
    "stencil_max_abs": (_i32, [_vp, _vp, _vp, _vp]),
    "stencil_strerror": (ctypes.c_char_p, [_i32]),
    "stencil_build_id": (ctypes.c_char_p, []),
    "stencil_last_error": (ctypes.c_char_p, [_vp]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class StencilError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{message} (status {status})")
        self.status = status


def _check(status: int, ctx=None):
    if status != OK:
        msg = stencil_strerror(status)
        extra = _lib.stencil_last_error(ctx)
        if extra:
            msg = f"{msg}: {extra.decode()}"
        raise StencilError(status, msg)


def _ptr(x) -> int:
    """Device pointer of a tensor (or an int passed through)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def stencil_strerror(status: int) -> str:
    return _lib.stencil_strerror(status).decode()


def stencil_last_error(ctx) -> str:
    return _lib.stencil_last_error(ctx).decode()


def make_tile(kind=TILE_ZMARCH, bx=0, by=0, ry=1, dz=0, vw=0, xcd=1, pf=0, pace=0) -> StencilTile:
    """A tile (stencil_tile). pf bit 0: prefetch; for two-step tiles, pace 0..7
    is the edge pacing code (stored in pf bits 1-3)."""
    if not 0 <= pace <= 7:
        raise ValueError("pace must be in 0..7")
    return StencilTile(kind, bx, by, ry, dz, vw, xcd, pf | (pace << 1))


def stencil_init(nx, ny, nz, h, dt, vmax, radius=4, device=0, tile: StencilTile | None = None, storage=F32,
                 storage_scale: float = 1.0, pitch: int = 0):
    """Create a context; returns an opaque handle (int). pitch = 0: rows of nx
    values; else the row stride of every field (>= nx)."""
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    d = StencilDesc(nx, ny, nz, radius, st, h, dt, vmax, device, tile if tile is not None else StencilTile(),
                    storage_scale, int(pitch))
    out = _vp()
    _check(_lib.stencil_init(ctypes.byref(d), ctypes.byref(out)))
    return out.value


def stencil_build_id() -> str:
    """The code identity that tune cache entries carry."""
    return _lib.stencil_build_id().decode()


def stencil_destroy(ctx):
    _lib.stencil_destroy(ctx)


def stencil_kappa(ctx, v, kappa, stream=None):
    _check(_lib.stencil_kappa(ctx, _ptr(v), _ptr(kappa), _stream(stream)), ctx)


def make_src(idx, amp) -> StencilSrc:
    """Source description from device tensors idx [n] (int64) and amp [nt, n]
    (float32; [nt] when n = 1). The returned object holds references to both
    tensors, so their memory stays valid as long as it is in use."""
    import torch
    if idx.dtype != torch.int64 or amp.dtype != torch.float32 or not idx.is_cuda or not amp.is_cuda:
        raise ValueError("source idx must be an int64 and amp a float32 CUDA tensor")
    if not idx.is_contiguous() or not amp.is_contiguous():
        raise ValueError("source tensors must be contiguous")
    n = int(idx.numel())
    nt = int(amp.shape[0])
    if amp.numel() != nt * n:
        raise ValueError(f"amp must hold [nt, n] = [{nt}, {n}] samples")
    src = StencilSrc(n, _ptr(idx), _ptr(amp), nt)
    src._keep = (idx, amp)
    return src


def stencil_step(ctx, kappa, u_cur, u_prev_next, it=0, src: StencilSrc | None = None, stream=None):
    _check(_lib.stencil_step(ctx, _ptr(kappa), _ptr(u_cur), _ptr(u_prev_next), int(it),
                             ctypes.byref(src) if src is not None else None, _stream(stream)), ctx)


def stencil_step_to(ctx, kappa, u_cur, u_prev, u_next, it=0, src: StencilSrc | None = None, stream=None):
    _check(_lib.stencil_step_to(ctx, _ptr(kappa), _ptr(u_cur), _ptr(u_prev), _ptr(u_next), int(it),
                                ctypes.byref(src) if src is not None else None, _stream(stream)), ctx)


def stencil_step2(ctx, kappa, u_cur, u_prev, u_next, u_next2, it=0, src: StencilSrc | None = None, stream=None):
    _check(_lib.stencil_step2(ctx, _ptr(kappa), _ptr(u_cur), _ptr(u_prev), _ptr(u_next), _ptr(u_next2), int(it),
                              ctypes.byref(src) if src is not None else None, _stream(stream)), ctx)


def stencil_get_tile2(ctx) -> StencilTile:
    t = StencilTile()
    _check(_lib.stencil_get_tile2(ctx, ctypes.byref(t)), ctx)
    return t


def stencil_list_tiles2(radius: int, vec4: bool = True):
    n = _lib.stencil_list_tiles2(radius, int(vec4), None, 0)
    _check(min(n, 0))
    arr = (StencilTile * max(n, 1))()
    _lib.stencil_list_tiles2(radius, int(vec4), arr, n)
    return [arr[i] for i in range(n)]


def stencil_kappa_slowness2(ctx, m, kappa, stream=None):
    _check(_lib.stencil_kappa_slowness2(ctx, _ptr(m), _ptr(kappa), _stream(stream)), ctx)


def stencil_sample(ctx, u, idx, out, stream=None):
    """out[j] = u[idx[j]]; idx int64 and out float32 device tensors of one length."""
    if out.numel() < idx.numel():
        raise ValueError("out holds fewer entries than idx")
    _check(_lib.stencil_sample(ctx, _ptr(u), _ptr(idx), int(idx.numel()), _ptr(out), _stream(stream)), ctx)


def stencil_adjoint_step(ctx, kappa, lam_cur, lam_prev_next, it, resid: StencilSrc | None, u_next=None, u_cur=None,
                         u_prev=None, grad=None, stream=None):
    _check(_lib.stencil_adjoint_step(ctx, _ptr(kappa), _ptr(lam_cur), _ptr(lam_prev_next), int(it),
                                     ctypes.byref(resid) if resid is not None else None, _ptr(u_next), _ptr(u_cur),
                                     _ptr(u_prev), _ptr(grad), _stream(stream)), ctx)


def stencil_gradient2(ctx, mu_k, mu_km1, u_k, u_km1, u_km2, u_km3, grad, stream=None):
    """The gradient terms of adjoint steps k and k-1 in one pass (see the header)."""
    _check(_lib.stencil_gradient2(ctx, _ptr(mu_k), _ptr(mu_km1), _ptr(u_k), _ptr(u_km1), _ptr(u_km2), _ptr(u_km3),
                                  _ptr(grad), _stream(stream)), ctx)


def stencil_gradient_terms(ctx, mu, u, grad, stream=None):
    """m = len(mu) (1..4) consecutive gradient terms in one pass; u holds
    m + 2 levels (u^k, u^{k-1}, ...). See the header."""
    m = len(mu)
    if len(u) != m + 2:
        raise ValueError("u must hold len(mu) + 2 fields")
    mus = (_vp * max(m, 1))(*[_ptr(x) for x in mu])
    us = (_vp * (m + 2))(*[_ptr(x) for x in u])
    _check(_lib.stencil_gradient_terms(ctx, int(m), mus, us, _ptr(grad), _stream(stream)), ctx)


def stencil_misfit(traces, observed, resid, misfit, stream=None):
    """resid = traces - observed; misfit (float64 device scalar) = 1/2 sum resid^2."""
    if observed.numel() != traces.numel() or (resid is not None and resid.numel() != traces.numel()):
        raise ValueError("traces, observed and resid must hold the same number of samples")
    _check(_lib.stencil_misfit(_ptr(traces), _ptr(observed), int(traces.numel()), _ptr(resid), _ptr(misfit),
                               _stream(stream)))


def stencil_batch_create(shots, it0: int = 0):
    """shots: list of (ctx, kappa, u_a, u_b, StencilSrc or None). Returns a handle."""
    out = _vp()
    _check(_lib.stencil_batch_create(_shot_array(shots), len(shots), int(it0), ctypes.byref(out)))
    return out.value


def stencil_batch_create_static(shots, it0: int = 0):
    """As stencil_batch_create, with the descriptor table in the library's
    static per-GPU table (no device allocation). Returns a handle."""
    out = _vp()
    _check(_lib.stencil_batch_create_static(_shot_array(shots), len(shots), int(it0), ctypes.byref(out)))
    return out.value


def _shot_array(shots):
    arr = (StencilShot * len(shots))()
    for i, (ctx, kap, ua, ub, src) in enumerate(shots):
        arr[i] = StencilShot(ctx, _ptr(kap), _ptr(ua), _ptr(ub), src if src is not None else StencilSrc())
    return arr


def stencil_batch_tune(shots, policy="worst", n_iter=0, n_rep=0, warmup=0, parts=0, include_plain=False,
                       stream=None):
    """Search one tile for a whole batch; shots as for stencil_batch_create.
    Returns the report dict; every shot's context tile is set to the winner."""
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    opts = StencilTuneOpts(pol, n_iter, n_rep, warmup, parts, int(bool(include_plain)), None, None, None, 0, 1,
                           None, None)
    rep = StencilTuneReport()
    _check(_lib.stencil_batch_tune(_shot_array(shots), len(shots), ctypes.byref(opts), ctypes.byref(rep),
                                   _stream(stream)))
    return {"tile": rep.tile.as_dict(), "min_time_ms": rep.min_time_ms, "actual_time_ms": rep.actual_time_ms,
            "gap": rep.gap, "default_time_ms": rep.default_time_ms, "seconds": rep.seconds,
            "n_candidates": rep.n_candidates}


def stencil_batch_step(batch, it: int, stream=None):
    _check(_lib.stencil_batch_step(batch, int(it), _stream(stream)))


def stencil_batch_launches(batch) -> int:
    n = _lib.stencil_batch_launches(batch)
    _check(min(n, 0))
    return n


def stencil_batch_destroy(batch):
    _lib.stencil_batch_destroy(batch)


def stencil_tune(ctx, kappa, scratch_a, scratch_b, policy="worst", n_iter=0, n_rep=0, warmup=0, parts=0,
                 include_plain=False, cache_path=None, table_cap=0, stream=None, temporal=1, scratch_c=None,
                 scratch_d=None):
    """Run the blocksize search. Returns (report dict, table [n_rep][nC] or None,
    candidates list or None)."""
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    table = (ctypes.c_double * (max(n_rep or 3, 1) * table_cap))() if table_cap else None
    cands = (StencilTile * table_cap)() if table_cap else None
    opts = StencilTuneOpts(pol, n_iter, n_rep, warmup, parts, int(bool(include_plain)),
                           cache_path.encode() if cache_path else None,
                           ctypes.cast(table, ctypes.POINTER(ctypes.c_double)) if table else None,
                           ctypes.cast(cands, ctypes.POINTER(StencilTile)) if cands else None, table_cap,
                           int(temporal), _ptr(scratch_c), _ptr(scratch_d))
    rep = StencilTuneReport()
    _check(_lib.stencil_tune(ctx, _ptr(kappa), _ptr(scratch_a), _ptr(scratch_b), ctypes.byref(opts),
                             ctypes.byref(rep), _stream(stream)), ctx)
    report = {"tile": rep.tile.as_dict(), "min_time_ms": rep.min_time_ms, "actual_time_ms": rep.actual_time_ms,
              "gap": rep.gap, "default_time_ms": rep.default_time_ms, "seconds": rep.seconds,
              "n_candidates": rep.n_candidates, "from_cache": bool(rep.from_cache)}
    tab = None
    cl = None
    if table_cap and not rep.from_cache:
        nrep = n_rep or 3
        nc = min(rep.n_candidates, table_cap)
        tab = [[table[r * table_cap + c] for c in range(nc)] for r in range(nrep)]
        cl = [cands[c].as_dict() for c in range(nc)]
    return report, tab, cl


def stencil_get_tile(ctx) -> StencilTile:
    t = StencilTile()
    _check(_lib.stencil_get_tile(ctx, ctypes.byref(t)), ctx)
    return t


def stencil_set_tile(ctx, tile: StencilTile):
    _check(_lib.stencil_set_tile(ctx, ctypes.byref(tile)), ctx)


def stencil_list_tiles(radius: int, vec4: bool = True, storage=F32):
    """Compiled one-step tiles; vec4: True/1 = four x points per thread,
    8 = eight (16-bit storage), 2 = two, False/0 = one."""
    st = STORAGES[storage] if isinstance(storage, str) else int(storage)
    n = _lib.stencil_list_tiles(radius, int(vec4), st, None, 0)
    _check(min(n, 0))
    arr = (StencilTile * max(n, 1))()
    _lib.stencil_list_tiles(radius, int(vec4), st, arr, n)
    return [arr[i] for i in range(n)]


def stencil_convert(ctx, src, dst, to_storage: bool, stream=None):
    _check(_lib.stencil_convert(ctx, _ptr(src), _ptr(dst), int(bool(to_storage)), _stream(stream)), ctx)


def stencil_coefficients(radius: int):
    out = (ctypes.c_float * 8)()
    n = _lib.stencil_coefficients(radius, out)
    _check(min(n, 0))
    return [out[i] for i in range(n)]


def stencil_cfl_limit(radius: int) -> float:
    r = _lib.stencil_cfl_limit(radius)
    if r < 0:
        raise StencilError(EINVAL, "unsupported radius")
    return r


def stencil_select(table, policy="worst"):
    """table: nested [nodes][cores][candidates] times. Returns (global id, time)."""
    nn = len(table)
    nk = len(table[0])
    nc = len(table[0][0])
    flat = (ctypes.c_double * (nn * nk * nc))(*[v for node in table for row in node for v in row])
    best = _i32()
    t = ctypes.c_double()
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    _check(_lib.stencil_select(flat, nn, nk, nc, pol, ctypes.byref(best), ctypes.byref(t)))
    return best.value, t.value


def stencil_pgrid(S: int, P: int):
    n = _lib.stencil_pgrid(S, P, None, 0)
    _check(min(n, 0))
    out = (_i64 * max(n, 1))()
    _lib.stencil_pgrid(S, P, out, n)
    return [out[i] for i in range(n)]


def stencil_stream_probe(a, b, c, out, nbytes: int, stream=None):
    """out = a (+ b) (+ c) over nbytes; b and c may be None."""
    _check(_lib.stencil_stream_probe(_ptr(a), _ptr(b), _ptr(c), _ptr(out), int(nbytes), _stream(stream)))


def stencil_max_abs(ctx, u, out, stream=None):
    """out (a float32 device tensor of at least one element) <- max |u| in
    storage units: NaN if any value is NaN, +inf if any is infinite."""
    if out.dtype.itemsize != 4 or out.numel() < 1:
        raise ValueError("out must hold at least one 4-byte value")
    _check(_lib.stencil_max_abs(ctx, _ptr(u), _ptr(out), _stream(stream)), ctx)


def stencil_stream_probe_march(a, b, c, out, shape, stream=None):
    """out = (a + b) + c over [nz, ny, nx] FP32 fields in the sweep's access order."""
    nz, ny, nx = shape
    _check(_lib.stencil_stream_probe_march(_ptr(a), _ptr(b), _ptr(c), _ptr(out), int(nx), int(ny), int(nz),
                                           _stream(stream)))


class Propagator:
    """A context bound to one grid and velocity model on one device.

    ``v`` is a float32 CUDA tensor [nz, ny, nx]; kappa = (v dt / h)^2 is formed
    on the device by the library. The time loop alternates the two wavefield
    buffers: step n reads (u^n, u^{n-1}) and overwrites the u^{n-1} buffer
    with u^{n+1}.

    ``pitch``: None for rows of nx values; an integer >= nx, or "align" (nx
    rounded up to 128 bytes), stores every field as [nz, ny, pitch] with zero
    padding at the end of each row. Fields passed in and returned then have
    that shape (``store_shape``); ``grid(u)`` is the [nz, ny, nx] view of the
    grid points and ``index(z, y, x)`` the linear index of a point."""

    def __init__(self, v, h: float, dt: float, radius: int = 4, vmax: float | None = None,
                 tile: StencilTile | None = None, slowness2: bool = False, storage="f32",
                 storage_scale: float = 1.0, pitch=None):
        import torch
        if v.dtype != torch.float32 or not v.is_cuda or v.dim() != 3 or not v.is_contiguous():
            raise ValueError("the model must be a contiguous float32 CUDA tensor [nz, ny, nx]")
        self.shape = tuple(v.shape)
        nz, ny, nx = self.shape
        if vmax is None:
            vmax = float(v.max().item()) if not slowness2 else float(v.min().item()) ** -0.5
        self.h, self.dt, self.radius = float(h), float(dt), int(radius)
        self.device = v.device
        self.storage = STORAGES[storage] if isinstance(storage, str) else int(storage)
        self.storage_scale = float(storage_scale)
        self.dtype = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}[self.storage]
        if pitch == "align":
            per_line = 128 // (4 if self.storage == F32 else 2)
            pitch = -(-nx // per_line) * per_line
        self.pitch = int(pitch) if pitch else nx
        self.store_shape = (nz, ny, self.pitch)
        self.ctx = stencil_init(nx, ny, nz, h, dt, vmax, radius, v.device.index or 0, tile, self.storage,
                                storage_scale, self.pitch if self.pitch != nx else 0)
        if self.pitch != nx:
            vp = torch.zeros(self.store_shape, dtype=torch.float32, device=self.device)
            vp[..., :nx] = v
            if slowness2:
                vp[..., nx:] = 1.0  # any finite positive value; padding is never a grid point
            v = vp
        self.kappa = torch.empty_like(v)
        if slowness2:
            stencil_kappa_slowness2(self.ctx, v, self.kappa)
        else:
            stencil_kappa(self.ctx, v, self.kappa)

    def __del__(self, _destroy=_lib.stencil_destroy):
        ctx = getattr(self, "ctx", None)
        if ctx:
            _destroy(ctx)
            self.ctx = None

    def _check_field(self, t):
        if t.dtype != self.dtype or not t.is_cuda or tuple(t.shape) != self.store_shape or not t.is_contiguous():
            raise ValueError(f"fields must be contiguous {self.dtype} CUDA tensors of shape {self.store_shape}")

    def zeros(self):
        """A zero wavefield in the storage type (padding included)."""
        import torch
        return torch.zeros(self.store_shape, dtype=self.dtype, device=self.device)

    def grid(self, u):
        """The [nz, ny, nx] view of a field's grid points (no copy)."""
        return u[..., : self.shape[2]]

    def index(self, z: int, y: int, x: int) -> int:
        """Linear index of grid point (z, y, x) in the stored layout."""
        return (z * self.shape[1] + y) * self.pitch + x

    def to_storage(self, u32):
        """storage_scale * u rounded to the storage type (device kernel)."""
        import torch
        out = torch.empty(self.store_shape, dtype=self.dtype, device=self.device)
        stencil_convert(self.ctx, u32.contiguous(), out, True)
        return out

    def to_f32(self, u):
        """FP32 u from a stored wavefield (device kernel)."""
        import torch
        out = torch.empty(self.store_shape, dtype=torch.float32, device=self.device)
        stencil_convert(self.ctx, u, out, False)
        return out

    @property
    def tile(self) -> StencilTile:
        return stencil_get_tile(self.ctx)

    @property
    def tile2(self) -> StencilTile:
        return stencil_get_tile2(self.ctx)

    @tile.setter
    def tile(self, t: StencilTile):
        stencil_set_tile(self.ctx, t)

    def max_abs(self, u, out=None, stream=None):
        """max |u| as a float32 device scalar (NaN if any value is NaN, +inf if
        any is infinite), in the wavefield's own units; asynchronous."""
        import torch
        self._check_field(u)
        if out is None:
            out = torch.empty((), dtype=torch.float32, device=self.device)
        stencil_max_abs(self.ctx, u, out, stream)
        if self.storage_scale != 1.0:
            out.div_(self.storage_scale)  # a power of two: exact
        return out

    def check_finite(self, u, limit: float = 0.0, stream=None) -> float:
        """Waits for the stream and raises StencilError(EDIVERGED) when u holds
        a NaN or an infinity, or (limit > 0) a magnitude above limit;
        returns max |u|."""
        import torch
        m = float(self.max_abs(u, stream=stream).item())
        if not (m == m) or m == float("inf") or (limit > 0 and m > limit):
            raise StencilError(EDIVERGED, f"{stencil_strerror(EDIVERGED)}: max |u| = {m}")
        return m

    def step(self, u_cur, u_prev_next, it: int = 0, src: StencilSrc | None = None, stream=None):
        self._check_field(u_cur)
        self._check_field(u_prev_next)
        stencil_step(self.ctx, self.kappa, u_cur, u_prev_next, it, src, stream)

    def run(self, u_cur, u_prev, nt: int, src: StencilSrc | None = None, it0: int = 0, stream=None,
            temporal: int = 1, spare=None, check_every: int = 0, limit: float = 0.0):
        """Advance nt steps from (u^{it0}, u^{it0-1}); returns the tensors now
        holding (u^{it0+nt}, u^{it0+nt-1}).

        check_every = k > 0 is a divergence watchdog: after every k steps (and
        at the end) the newest wavefield's max |u| is read back, and a NaN, an
        infinity or (limit > 0) a value above limit raises
        StencilError(EDIVERGED). Each check waits for the stream, so leave it
        0 inside graph capture.

        temporal=2 uses two-step launches (bit-identical results), which need
        two more wavefield buffers: ``spare`` = (c, d), allocated if None; an
        odd nt ends with one one-step launch. The four buffers rotate, so the
        returned pair may be two of the spares; pass ``spare`` as a list to
        get back, in place, the two buffers that are free afterwards."""
        self._check_field(u_cur)
        self._check_field(u_prev)
        if check_every < 0:
            raise ValueError("check_every must be >= 0")
        if check_every:
            # The watchdog runs the loop in segments of check_every steps; one
            # spare list carries the two free buffers from segment to segment.
            sp = list(spare) if spare is not None else None
            if temporal == 2 and nt >= 2 and sp is None:
                sp = [self.zeros(), self.zeros()]
            done = 0
            a, b = u_cur, u_prev
            while done < nt:
                k = min(check_every, nt - done)
                a, b = self.run(a, b, k, src, it0 + done, stream, temporal, sp)
                self.check_finite(a, limit, stream)
                done += k
            if isinstance(spare, list) and sp is not None:
                spare[:] = sp
            return a, b
        a, b = u_cur, u_prev
        it = it0
        if temporal == 2 and nt >= 2:
            c, d = spare if spare is not None else (self.zeros(), self.zeros())
            self._check_field(c)
            self._check_field(d)
            while it + 2 <= it0 + nt:
                stencil_step2(self.ctx, self.kappa, a, b, c, d, it, src, stream)
                a, b, c, d = d, c, b, a
                it += 2
            if isinstance(spare, list):
                spare[:] = [c, d]
        while it < it0 + nt:
            stencil_step(self.ctx, self.kappa, a, b, it, src, stream)
            a, b = b, a
            it += 1
        return a, b

    def tune(self, scratch_a=None, scratch_b=None, **opts):
        if scratch_a is None:
            scratch_a = self.zeros()
        if scratch_b is None:
            scratch_b = self.zeros()
        if opts.get("temporal", 1) == 2:
            opts.setdefault("scratch_c", self.zeros())
            opts.setdefault("scratch_d", self.zeros())
        return stencil_tune(self.ctx, self.kappa, scratch_a, scratch_b, **opts)


class Batch:
    """Several Propagators (shots) stepped together by stencil_batch_step.

    ``shots``: list of (Propagator, StencilSrc or None). Each shot gets two
    zeroed wavefield buffers; after an even number of steps from it0 buffer
    ``u_a`` holds the newest wavefield, after an odd number ``u_b``."""

    def __init__(self, shots, it0: int = 0, tune: dict | None = None):
        import torch
        self.props = [pr for pr, _ in shots]
        self.srcs = [src for _, src in shots]
        self.u_a = [pr.zeros() for pr in self.props]
        self.u_b = [pr.zeros() for pr in self.props]
        self.it0 = int(it0)
        spec = [(pr.ctx, pr.kappa, a, b, src) for pr, a, b, src in zip(self.props, self.u_a, self.u_b, self.srcs)]
        self.tune_report = None
        if tune is not None:
            # One tile for the whole batch, searched under batch contention;
            # the buffers were scratch during the search and are cleared.
            self.tune_report = stencil_batch_tune(spec, **tune)
            for x, y in zip(self.u_a, self.u_b):
                x.zero_()
                y.zero_()
        self.handle = stencil_batch_create(spec, it0)

    def __del__(self, _destroy=_lib.stencil_batch_destroy):
        h = getattr(self, "handle", None)
        if h:
            _destroy(h)
            self.handle = None

    @property
    def launches_per_step(self) -> int:
        return stencil_batch_launches(self.handle)

    def step(self, it: int, stream=None):
        stencil_batch_step(self.handle, it, stream)

    def run(self, nt: int, it0: int | None = None, stream=None):
        start = self.it0 if it0 is None else it0
        for it in range(start, start + nt):
            stencil_batch_step(self.handle, it, stream)

    def current(self, steps_done: int):
        """(u^n, u^{n-1}) tensors of every shot after `steps_done` steps from it0."""
        if steps_done % 2 == 0:
            return list(zip(self.u_a, self.u_b))
        return list(zip(self.u_b, self.u_a))
