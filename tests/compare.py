"""Comparison of a GPU output with the FP64 oracle's, per output, by two
measures: the relative L2 norm of the difference over the whole field, and
the largest single-point deviation on the scale of the reference's largest
value (oracle.rel_l2, oracle.max_rel).

Bound on the per-point measure. The FP32 error at a point is the rounding
its own history accumulated, which scales with the local wave amplitude, so
the error field is distributed like the wavefield and
    max|e| / max|ref| = rel_l2 * (max|e| / rms e) / (max|ref| / rms ref)
stays within a small factor of rel_l2. The bound is MAX_FACTOR times the
rel-L2 bound: at the FP32 bar of 1e-5 a single point wrong by 1e-4 of the
field's peak fails, which no global norm over 10^8 points would show.
"""
import sys

import numpy as np

import oracle

MAX_FACTOR = 10.0


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def measures(got, ref):
    return oracle.rel_l2(got, ref), oracle.max_rel(got, ref)


def check_close(got, ref, tol, what="", max_tol=None):
    """Assert rel_l2 <= tol and max_rel <= max_tol (MAX_FACTOR * tol by
    default); logs both; returns them."""
    got = np.asarray(got)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    e, m = measures(got, ref)
    mt = MAX_FACTOR * tol if max_tol is None else max_tol
    log(f"  {what} rel_l2 = {e:.3e}  max_rel = {m:.3e}")
    assert e <= tol, f"{what}: rel_l2 {e:.3e} > {tol:.1e}"
    assert m <= mt, f"{what}: max_rel {m:.3e} > {mt:.1e}"
    return e, m
