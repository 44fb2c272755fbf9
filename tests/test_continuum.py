"""Pins of the continuum references of the accuracy tests.

The closed-form cuboid field: Gauss-Legendre quadrature outside the box,
the far field of a point charge, Gauss's law (div E = density inside, 0
outside) and the box's point symmetry.

The switched-on box (constant sources from t = 0, with and without the
switch-on shell): a ball wholly inside the box (no net Coulomb field, the
shell gives E = -J t), a ball cut by one face (closed forms of the cap), the
saturated limit (the closed-form cuboid field), cuts through edges and
corners against an independent equal-area direction sum, convergence in the
number of nodes, and the shell-less reading against the discretised
Coulomb sum over the ball, refined."""
import math

import numpy as np

from tests.continuum import (_sphere_integrals, ball_sum_plane, box_field, switched_on_box_fields,
                             switched_on_box_plane)

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


CUBE = ((-3.0, -3.0, -3.0), (3.0, 3.0, 3.0))


def test_switched_on_ball_inside_the_box():
    # the ball R < t lies inside the box: the Coulomb parts cancel, the shell
    # int n dOmega = 0, and the current shell gives E = -J (1/4pi) t 4pi
    J = np.array([1.0, -0.5, 2.0])
    for p, t in [((0.3, -0.2, 0.1), 2.5), ((1.0, 1.5, -0.4), 1.4)]:
        E, B = switched_on_box_fields(p, t, *CUBE, J=J)
        assert np.allclose(E, -J * t, atol=1e-12) and np.allclose(B, 0.0, atol=1e-12), (p, t, E, B)
        E0, B0 = switched_on_box_fields(p, t, *CUBE, J=J, shell=False)
        assert np.allclose(E0, 0.0, atol=1e-12) and np.allclose(B0, 0.0, atol=1e-12)


def test_switched_on_one_face_cut():
    # the ball crosses the face x = 3 only (h = distance to it): the missing
    # cap, seen from the centre, gives A_x = (t - h)^2 / (4 t); the shell
    # misses a cap of solid angle 2 pi (1 - h/t): S0 = (t + h) / 2 and
    # S1_x = (t^2 - h^2) / (4 t)
    for p, t in [((2.0, 0.1, -0.2), 1.5), ((1.2, -0.3, 0.5), 2.4)]:
        h = 3.0 - p[0]
        A, S1, S0 = _sphere_integrals(p, t, *CUBE, 24)
        assert np.allclose(A, [(t - h) ** 2 / (4 * t), 0, 0], atol=1e-12), (p, A)
        assert np.allclose(S1, [(t * t - h * h) / (4 * t), 0, 0], atol=1e-12), (p, S1)
        assert abs(S0 - (t + h) / 2) < 1e-12, (p, S0)
        J = np.array([1.0, 1.0, 1.0])
        E, B = switched_on_box_fields(p, t, *CUBE, J=J)
        assert np.allclose(E, A + S1 - J * S0, atol=1e-14) and np.allclose(B, np.cross(J, A + S1), atol=1e-14)


def test_switched_on_saturates_to_the_box_field():
    lo, hi = (-3.0, -2.0, -1.5), (3.0, 2.5, 1.0)
    for p in [(2.6, -1.3, 0.7), (-2.9, 2.4, -1.4), (0.1, 0.2, 0.3)]:
        # (-2.9, 2.4, -1.4) lies 0.1 from a corner: the hardest case for the nodes
        E, B = switched_on_box_fields(p, 9.0, lo, hi, J=(0.5, -1.0, 2.0))
        ref = box_field(p, lo, hi)
        assert np.allclose(E, ref, rtol=0, atol=2e-8), (p, E, ref)
        assert np.allclose(B, np.cross([0.5, -1.0, 2.0], ref), rtol=0, atol=5e-8)
        E0, _ = switched_on_box_fields(p, 9.0, lo, hi, shell=False)
        assert np.allclose(E0, ref, rtol=0, atol=2e-8)


def _direction_sum(p, t, lo, hi, N=1_000_000):
    """(A, S1, S0) by an equal-area (Fibonacci) sum over N directions d from
    p: R_box(d) straight from the ray-box exit, no faces, no polar maps."""
    p, lo, hi = (np.asarray(v, dtype=np.float64) for v in (p, lo, hi))
    i = np.arange(N) + 0.5
    z = 1.0 - 2.0 * i / N
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(1.0 - z * z)
    d = np.stack([s * np.cos(phi), s * np.sin(phi), z], 1)
    with np.errstate(divide="ignore"):
        exit_t = np.where(d > 0, (hi - p) / d, np.where(d < 0, (lo - p) / d, np.inf))
    rb = exit_t.min(1)
    w = 1.0 / N                                   # (4 pi / N) / (4 pi)
    inside = rb >= t
    A = -(d * np.minimum(t, rb)[:, None]).sum(0) * w
    S1 = -t * (d * inside[:, None]).sum(0) * w
    return A, S1, t * inside.sum() * w


def test_switched_on_edges_and_corners_against_direction_sum():
    lo, hi = (-3.0, -2.0, -1.5), (3.0, 2.5, 1.0)
    for p, t in [((2.6, -1.6, 0.4), 3.3), ((-2.8, 2.2, 0.8), 5.5), ((0.2, 0.3, -0.1), 2.9)]:
        A, S1, S0 = _sphere_integrals(p, t, lo, hi, 24)
        A2, S12, S02 = _direction_sum(p, t, lo, hi)
        # A's integrand is continuous (error ~1e-8); the shell's jumps at R_box = t (~1e-5)
        assert np.allclose(A, A2, atol=1e-6), (p, t, A, A2)
        assert np.allclose(S1, S12, atol=2e-4 * t) and abs(S0 - S02) < 2e-4 * t, (p, t, S1, S12, S0, S02)


def test_switched_on_converges_in_nodes():
    for p, t in [((2.8, 2.4, 0.0), 5.0), ((-2.8, -2.8, 0.0), 2.5), ((2.8, 0.0, 0.0), 7.5)]:
        a = np.concatenate([np.ravel(v) for v in _sphere_integrals(p, t, *CUBE, 16)])
        b = np.concatenate([np.ravel(v) for v in _sphere_integrals(p, t, *CUBE, 32)])
        assert np.allclose(a, b, atol=1e-7), (p, t, np.abs(a - b).max())


def test_switched_on_without_shell_is_the_limit_of_the_ball_sum():
    """Without the shell the field at (r, t) is the Coulomb field of the part
    of the box within distance t.  Its midpoint sum over cells of side 0.4/r
    (the observation cell screened) approaches the quadrature as r grows."""
    pts = [(2.8, 2.4, 0.0), (-1.2, 2.8, 0.0), (2.8, -2.8, 0.0)]
    t = 2.5
    ref = switched_on_box_plane(pts, t, *CUBE)["no_shell"]
    devs = []
    for r in (1, 2, 4):
        E, B = ball_sum_plane(pts, t, *CUBE, 0.4 / r, 0.2)
        devs.append(max(float(np.abs(E - ref[0]).max() / np.abs(ref[0]).max()),
                        float(np.abs(B - ref[1]).max() / np.abs(ref[1]).max())))
    assert devs[2] < devs[0] and devs[2] < 0.01, devs
