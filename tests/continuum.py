"""Closed-form continuum fields for the accuracy tests (test infrastructure).

The field of a uniformly charged cuboid: (1/4pi) times the integral of
(r - r')/|r - r'|^3 over the box, per unit density, in the units of the
paper's Jefimenko equations (section "Jefimenko's equations": prefactor
1/4pi).  Per axis the integral is a signed sum over the 8 corners of the
antiderivative  v ln(w + R) + w ln(v + R) - u atan(v w / (u R))  with
(u, v, w) the offsets from the corner along (that axis, the next two) --
the standard result for the field of a rectangular prism.  Stationary
uniform currents J give B = J x (that field): the static limits the paper's
constant sources saturate to (section "Constant sources").
"""
import math

import numpy as np


def _antiderivative(u, v, w):
    R = math.sqrt(u * u + v * v + w * w)
    t = v * math.log(w + R) + w * math.log(v + R)
    if u != 0.0:
        t -= u * math.atan(v * w / (u * R))
    return t


def box_field(p, lo, hi):
    """E at point p (not on a face plane of the box) of unit charge density
    filling [lo, hi]: a length-3 array."""
    E = np.zeros(3)
    for a in range(3):
        ax = (a, (a + 1) % 3, (a + 2) % 3)
        tot = 0.0
        for i, xs in enumerate((lo[ax[0]], hi[ax[0]])):
            for j, ys in enumerate((lo[ax[1]], hi[ax[1]])):
                for k, zs in enumerate((lo[ax[2]], hi[ax[2]])):
                    tot += (-1) ** (i + j + k) * _antiderivative(p[ax[0]] - xs, p[ax[1]] - ys, p[ax[2]] - zs)
        E[a] = -tot / (4.0 * math.pi)
    return E


def box_fields(points, lo, hi):
    """[3][n] fields at the points ([n][3])."""
    return np.stack([box_field(tuple(float(c) for c in q), lo, hi) for q in points], axis=1)
