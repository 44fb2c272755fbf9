"""Pins of the closed-form cuboid field used as the continuum reference of
the accuracy tests: Gauss-Legendre quadrature outside the box, the far
field of a point charge, Gauss's law (div E = density inside, 0 outside)
and the box's point symmetry."""
import math

import numpy as np

from tests.continuum import box_field

LO, HI = (-3.0, -2.0, -1.5), (3.0, 2.5, 1.0)


def _gauss_box(p, n=48):
    x, w = np.polynomial.legendre.leggauss(n)
    axes = [0.5 * (HI[a] - LO[a]) * x + 0.5 * (HI[a] + LO[a]) for a in range(3)]
    wts = [0.5 * (HI[a] - LO[a]) * w for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    W = wts[0][:, None, None] * wts[1][None, :, None] * wts[2][None, None, :]
    d = np.stack([p[0] - X, p[1] - Y, p[2] - Z])
    R3 = (d * d).sum(0) ** 1.5
    return (d / R3 * W).reshape(3, -1).sum(1) / (4 * math.pi)


def test_matches_quadrature_outside():
    for p in [(9.0, 2.0, -1.0), (4.5, 0.5, 0.3), (-5.0, 7.0, 3.0), (0.2, -0.1, 6.0)]:
        assert np.allclose(box_field(p, LO, HI), _gauss_box(p), rtol=1e-9, atol=1e-12), p


def test_far_field_is_a_point_charge():
    vol = np.prod([HI[a] - LO[a] for a in range(3)])
    c = np.array([(HI[a] + LO[a]) / 2 for a in range(3)])
    p = c + np.array([300.0, -170.0, 220.0])
    d = p - c
    ref = vol * d / (4 * math.pi * np.linalg.norm(d) ** 3)
    assert np.allclose(box_field(tuple(p), LO, HI), ref, rtol=1e-4)


def test_gauss_law():
    h = 1e-4
    for p, rho in [((0.31, -0.7, 0.2), 1.0), ((2.9, 2.4, -1.4), 1.0), ((4.0, 0.3, 0.1), 0.0),
                   ((0.0, 3.1, 0.0), 0.0)]:
        div = 0.0
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            div += (box_field(tuple(np.add(p, e)), LO, HI)[a] - box_field(tuple(np.subtract(p, e)), LO, HI)[a]) / (2 * h)
        assert abs(div - rho) < 1e-6, (p, div)


def test_point_symmetry():
    lo, hi = (-3.0, -3.0, -3.0), (3.0, 3.0, 3.0)
    for p in [(0.13, 0.27, -0.41), (2.6, -1.3, 0.7), (-4.0, 1.0, 5.0)]:
        assert np.allclose(box_field(p, lo, hi), -box_field(tuple(-np.array(p)), lo, hi), atol=1e-14)
    assert np.allclose(box_field((1e-9, 2e-9, -1e-9), lo, hi), 0.0, atol=1e-8)
