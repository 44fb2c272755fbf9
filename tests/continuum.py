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


# Constant sources switched on at t = 0 (section "Constant sources": rho = 1,
# J = const for t >= 0, zero before) have the retarded values rho(t - R) =
# theta(t - R).  Put into Jefimenko's equations (section "Jefimenko's
# equations"), with r' = r - R n, n the unit vector from r' to r:
#   value terms      -> the Coulomb and Biot-Savart fields of the part of the
#                       box inside the ball R < t:
#                       A = (1/4pi) int n min(t, R_box(n)) dOmega,
#                       E += A, B += J x A;
#   derivative terms -> d/dt theta(t - R) = delta(t - R), a shell on the
#                       sphere R = t inside the box:
#                       S1 = (t/4pi) int_{R_box(n) >= t} n dOmega,
#                       S0 = (t/4pi) int_{R_box(n) >= t} dOmega,
#                       E += S1 - J S0, B += J x S1.
# R_box(n) is the distance from r to the box boundary along -n.  The
# screening cube (all |x_i - x_i'| <= delta) around a point inside the box
# removes nothing from A (the cube is centred on r, its contribution
# int n R_cube(n) dOmega vanishes by symmetry) nor from the shell once t is
# beyond the cube's corners.  The sphere integrals are taken face by face:
# the directions that leave the box through one face are that face seen from
# r, with dOmega = h / rho^3 du dv (h the distance to the face plane, rho
# the distance to the face point), in polar coordinates (varrho, phi) about
# the foot of the perpendicular; Gauss-Legendre in both, with breakpoints at
# the face corners, at the circle rho = t and geometrically near the foot.

def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w   # nodes and weights on [0, 1]


def _sphere_integrals(p, t, lo, hi, n):
    """(A, S1, S0) for the point p strictly inside [lo, hi] at time t > 0."""
    xg, wg = _gl(n)
    A = np.zeros(3)
    S1 = np.zeros(3)
    S0 = 0.0
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s, plane in ((1.0, hi[a]), (-1.0, lo[a])):
            h = s * (plane - p[a])
            if not h > 0.0:
                raise ValueError("the point must lie strictly inside the box")
            rc = math.sqrt(max(t * t - h * h, 0.0))   # radius of the circle rho = t on the face
            for su, U in ((1.0, hi[b] - p[b]), (-1.0, p[b] - lo[b])):
                for sv, V in ((1.0, hi[c] - p[c]), (-1.0, p[c] - lo[c])):
                    if U <= 0.0 or V <= 0.0:
                        continue
                    pc = math.atan2(V, U)
                    # triangle 1: phi in [0, pc], edge |u| = U; triangle 2: [pc, pi/2], edge |v| = V
                    for f0, f1, D, edge_u in ((0.0, pc, U, True), (pc, 0.5 * math.pi, V, False)):
                        cuts = [f0, f1]
                        if D < rc:   # where the circle meets the edge
                            fs = math.acos(D / rc) if edge_u else math.asin(D / rc)
                            if f0 < fs < f1:
                                cuts.insert(1, fs)
                        for g0, g1 in zip(cuts[:-1], cuts[1:]):
                            phi = g0 + (g1 - g0) * xg
                            wphi = (g1 - g0) * wg
                            rmax = D / np.cos(phi) if edge_u else D / np.sin(phi)
                            brk = np.stack([np.zeros_like(phi)] + [np.full_like(phi, h * 3.0 ** j) for j in range(4)]
                                           + [np.full_like(phi, rc), rmax], axis=1)
                            brk = np.sort(np.minimum(brk, rmax[:, None]), axis=1)
                            r0, r1 = brk[:, :-1], brk[:, 1:]          # pieces [nphi][6]
                            vr = r0[..., None] + (r1 - r0)[..., None] * xg        # [nphi][6][n]
                            wr = (r1 - r0)[..., None] * wg
                            beyond = (0.5 * (r0 + r1) >= rc)[..., None]           # piece lies at rho >= t
                            rho = np.sqrt(h * h + vr * vr)
                            cphi, sphi = np.cos(phi)[:, None, None], np.sin(phi)[:, None, None]
                            # w = r' - r on the face; d = w / rho points from r to r', n = -d
                            wv = [None, None, None]
                            wv[a] = np.full_like(vr, s * h)
                            wv[b] = su * vr * cphi
                            wv[c] = sv * vr * sphi
                            jac = (wphi[:, None, None] * wr) * h / rho ** 3 * vr   # dOmega
                            m = np.minimum(t, rho)
                            for k in range(3):
                                dk = wv[k] / rho
                                A[k] -= (dk * m * jac).sum()
                                S1[k] -= t * (dk * jac * beyond).sum()
                            S0 += t * (jac * beyond).sum()
    k4 = 1.0 / (4.0 * math.pi)
    return A * k4, S1 * k4, S0 * k4


def switched_on_box_fields(p, t, lo, hi, J=(1.0, 1.0, 1.0), shell=True, n=32):
    """E and B (length-3 arrays) at p inside [lo, hi] at time t > 0 of the
    sources rho = 1, J constant on the box, switched on at t = 0, from the
    continuous Jefimenko integrals.  shell=True keeps the delta-function
    shell of the switch-on (the time derivatives at t - R = 0); shell=False
    leaves it out: the Coulomb and Biot-Savart fields of box n {R < t}.
    With n = 32 nodes per piece the error is below 1e-8 even 0.1 from a
    corner of the box."""
    A, S1, S0 = _sphere_integrals(tuple(float(v) for v in p), float(t), lo, hi, n)
    Jv = np.asarray(J, dtype=np.float64)
    if shell:
        return A + S1 - Jv * S0, np.cross(Jv, A + S1)
    return A, np.cross(Jv, A)


def switched_on_box_plane(points, t, lo, hi, J=(1.0, 1.0, 1.0), n=32):
    """Both readings at the points ([n_points][3]) from one set of sphere
    integrals: {"shell": (E, B), "no_shell": (E, B)}, each [3][n_points]."""
    Jv = np.asarray(J, dtype=np.float64)
    out = {"shell": ([], []), "no_shell": ([], [])}
    for q in points:
        A, S1, S0 = _sphere_integrals(tuple(float(v) for v in q), float(t), lo, hi, n)
        out["shell"][0].append(A + S1 - Jv * S0)
        out["shell"][1].append(np.cross(Jv, A + S1))
        out["no_shell"][0].append(A)
        out["no_shell"][1].append(np.cross(Jv, A))
    return {k: (np.stack(e, axis=1), np.stack(b, axis=1)) for k, (e, b) in out.items()}


def ball_sum_plane(points, t, lo, hi, cell, screen, J=(1.0, 1.0, 1.0)):
    """The discretised sum that leaves out the switch-on derivative: for the
    constant sources it is the static (Coulomb, Biot-Savart) midpoint sum
    over the cells of side `cell` tiling [lo, hi] whose centres lie within
    distance t of the point (retarded time >= 0), the cells inside the
    screening cube (all |x_i - x_i'| <= screen) left out.  [3][n] E and B."""
    axes = [lo[a] + cell * (np.arange(int(round((hi[a] - lo[a]) / cell))) + 0.5) for a in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    cells = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    Jv = np.asarray(J, dtype=np.float64)
    E = np.zeros((3, len(points)))
    for i, q in enumerate(points):
        w = np.asarray(q, dtype=np.float64)[None, :] - cells
        R = np.sqrt((w * w).sum(1))
        keep = (R <= t) & ~np.all(np.abs(w) <= screen, axis=1)
        E[:, i] = (w[keep] / R[keep, None] ** 3).sum(0) * cell ** 3 / (4.0 * math.pi)
    return E, np.cross(Jv[None, :], E.T).T
