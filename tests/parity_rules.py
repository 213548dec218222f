"""Comparison rules shared by the GPU parity tests (no oracle arithmetic)."""
import numpy as np


def rel(a, ref):
    """Normwise relative difference ||a - ref|| / ||ref|| (absolute when ref = 0)."""
    a = np.asarray(a)
    ref = np.asarray(ref)
    d = np.linalg.norm(ref)
    return np.linalg.norm(a - ref) / (d if d > 0 else 1.0)


def near_tie(lam_tau, rel_gap=1e-4, same=1e-9):
    """True when the two largest DISTINCT selection values of a component
    differ by less than `rel_gap` relative: FP32 and FP64 runs may then select
    different fixed points, and the end-to-end FP32 comparison of that
    component (and of every later one, which follow a different deflation)
    is reported rather than failed.  Restarts that reach the same fixed point
    agree to `same` relative and count as one value."""
    v = np.asarray(lam_tau, dtype=np.float64)
    v = np.sort(v[np.isfinite(v)])[::-1]
    if v.size < 2:
        return False
    top = v[0]
    distinct = v[(top - v) > same * abs(top)]
    return bool(distinct.size > 0 and (top - distinct[0]) < rel_gap * abs(top))
