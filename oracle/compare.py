"""Comparison metrics for field results -- TEST INFRASTRUCTURE.

Per-component relative L2 error: rel_c = ||x_c - y_c||_2 / ||y_c||_2 over
all observation points.  A component whose reference norm is below 1e-6 of
the whole field's norm (E or B as a vector field) is normalised by the
field norm instead and flagged, since its own norm is round-off (for
example B_z of a source whose J is parallel to z).
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
