"""Comparison metrics for field results -- TEST INFRASTRUCTURE.

Per-component relative L2 error: rel_c = ||x_c - y_c||_2 / ||y_c||_2 over
all observation points.  A component whose reference norm is below 1e-6 of
the whole field's norm (E or B as a vector field) is normalised by the
field norm instead and flagged, since its own norm is round-off (for
example B_z of a source whose J is parallel to z).

Per-point bound beside it: pt_c = max_i |x_ci - y_ci| / max_i |y_ci|, with
the same fallback to the whole field's largest value.  An L2 norm over n
points dilutes a few wrong points by about sqrt(n) (one edge tile, one
padded wavefront); the per-point bound does not.
"""
from __future__ import annotations

import numpy as np


def rel_l2(x: np.ndarray, y: np.ndarray):
    """x, y: [3][n].  Returns (list of 3 errors, list of 3 'field-normalised' flags)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    field = float(np.sqrt((y * y).sum()))
    errs, flags = [], []
    for c in range(3):
        nc = float(np.linalg.norm(y[c]))
        diff = float(np.linalg.norm(x[c] - y[c]))
        if nc < 1e-6 * field or nc == 0.0:
            errs.append(diff / field if field > 0 else diff)
            flags.append(True)
        else:
            errs.append(diff / nc)
            flags.append(False)
    return errs, flags


def max_rel_l2(xE, xB, yE, yB) -> float:
    e, _ = rel_l2(xE, yE)
    b, _ = rel_l2(xB, yB)
    return max(e + b)


def point_rel(x: np.ndarray, y: np.ndarray):
    """x, y: [3][n].  Per component max_i |x_ci - y_ci| / max_i |y_ci|."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if y.size == 0:
        return [0.0, 0.0, 0.0]
    field = float(np.abs(y).max())
    out = []
    for c in range(3):
        mc = float(np.abs(y[c]).max())
        diff = float(np.abs(x[c] - y[c]).max())
        norm = field if (mc < 1e-6 * field or mc == 0.0) else mc
        out.append(diff / norm if norm > 0 else diff)
    return out


def check_fields(xE, xB, yE, yB, tol: float, label: str = "", point_tol: float | None = None):
    """Asserts finite results, per-component relative L2 <= tol and the
    per-point bound <= point_tol (default 10 * tol).  Returns the largest
    (relative L2, per-point) errors."""
    xE = np.asarray(xE, dtype=np.float64)
    xB = np.asarray(xB, dtype=np.float64)
    if point_tol is None:
        point_tol = 10.0 * tol
    e, _ = rel_l2(xE, yE)
    b, _ = rel_l2(xB, yB)
    pe = point_rel(xE, yE)
    pb = point_rel(xB, yB)
    l2, pt = max(e + b), max(pe + pb)
    if label:
        print(f"{label} rel L2 E={['%.2e' % v for v in e]} B={['%.2e' % v for v in b]} "
              f"point {pt:.2e}", flush=True)
    assert np.all(np.isfinite(xE)) and np.all(np.isfinite(xB)), label
    assert l2 <= tol, (label, "rel L2", e, b)
    assert pt <= point_tol, (label, "per point", pe, pb)
    return l2, pt
