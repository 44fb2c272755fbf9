"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a textbook
closed form (Coulomb, Biot-Savart, a current ring), an integral law (Gauss),
an exact property of the interpolation readings (linear and quadratic
histories, the switch-on at the oldest slice) or the paper's saturation
statement for constant sources (section "Constant sources").  A plausible
mistake in the oracle (a dropped term, a flipped sign, a wrong slice index,
a transposed cross product, a missing volume factor) fails at least one.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import tiny
from workloads import Grid, centred_grid

FOUR_PI = 4.0 * math.pi


def _single_cell(r=(0.0, 0.0, 0.0), h=(0.1, 0.2, 0.15)):
    return Grid((1, 1, 1), tuple(r), tuple(h))


def _hist_from(fn, nt, s_old, dt, t0=0.0, n_src=1):
    """h[j][ch][s] = fn(time)[ch] for logical slice j (absolute step s_old+j)."""
    out = np.zeros((nt, 4, n_src))
    for j in range(nt):
        out[j, :, :] = np.asarray(fn(t0 + (s_old + j) * dt), dtype=np.float64)[:, None]
    return out


def _obs_points(n=(5, 4, 3), origin=(0.7, -0.45, 0.33), sp=(0.21, 0.17, 0.19)):
    return Grid(n, origin, sp)


def _centres(g):
    from workloads import cell_centres
    return cell_centres(g)


def test_static_cell_is_coulomb_and_biot_savart():
    """Static single cell: E = q dOmega d/(4 pi R^3), B = dOmega J x d/(4 pi R^3)."""
    src = _single_cell()
    obs = _obs_points()
    q, J = 0.8, np.array([0.3, -1.1, 0.6])
    dt = 0.05
    nt = 120  # every pair's stencil sits well inside the stored history
    hist = _hist_from(lambda t: [q, *J], nt, 0, dt)
    E, B = oracle.eval_fields(src, obs, hist, dt, t=(nt - 1) * dt, screen=(0, 0, 0))
    dom = 0.1 * 0.2 * 0.15
    d = _centres(obs)  # source sits at the origin
    R = np.linalg.norm(d, axis=1)
    E_ref = (q * dom / FOUR_PI) * d.T / R ** 3
    B_ref = (dom / FOUR_PI) * np.cross(J[None, :], d).T / R ** 3
    assert np.allclose(E, E_ref, rtol=1e-14, atol=0)
    assert np.allclose(B, B_ref, rtol=1e-14, atol=1e-18)


def test_self_cell_is_screened_and_R0_excluded():
    """Fields in a cell come only from other cells: a coincident grid sees
    nothing from the cell it sits in, even with zero screening width."""
    g = centred_grid((1, 1, 1), 0.1)
    hist = np.ones((4, 4, 1))
    for screen in [(0.05, 0.05, 0.05), (0.0, 0.0, 0.0)]:
        E, B = oracle.eval_fields(g, g, hist, 0.05, t=0.15, screen=screen)
        assert np.all(E == 0.0) and np.all(B == 0.0)


def test_screening_cube_excludes_exactly_the_neighbourhood():
    """With half-width = one spacing, the 27-cell neighbourhood is excluded
    and the next shell is not (per-axis test |d_a| <= delta_a)."""
    src = centred_grid((5, 5, 5), 0.1)
    obs = Grid((1, 1, 1), (0.0, 0.0, 0.0), (0.1, 0.1, 0.1))
    dump = oracle.slice_index_dump(src, obs, nt=80, dt=0.05, t=79 * 0.05, screen=(0.1 + 1e-12,) * 3)
    c = _centres(src)
    inside = np.all(np.abs(c) <= 0.1 + 1e-9, axis=1)
    assert np.all(dump[0, inside] == oracle.SCREENED)
    assert np.all(dump[0, ~inside] != oracle.SCREENED)
    assert inside.sum() == 27


def test_linear_history_is_reproduced_exactly():
    """rho, J linear in t: the interpolant and the backward difference are
    exact, so E = dOmega/(4 pi) [d (a + b t_r)/R^3 + d b/R^2 - J1/R] and
    B = dOmega/(4 pi) [(J0 + J1 t_r) x d/R^3 + J1 x d/R^2], t_r = t - R/c."""
    src = _single_cell(r=(0.05, -0.02, 0.01))
    obs = _obs_points()
    a, b = 0.7, -1.3
    J0, J1 = np.array([0.2, 0.5, -0.4]), np.array([-0.9, 0.3, 0.8])
    dt, c = 0.04, 0.9
    nt, s_old, t0 = 150, 37, -0.6

    def fn(t):
        return [a + b * t, *(J0 + J1 * t)]

    hist = _hist_from(fn, nt, s_old, dt, t0)
    newest = s_old + nt - 1
    t = t0 + newest * dt - 0.013  # between slices
    E, B = oracle.eval_fields(src, obs, hist, dt, t=t, t0=t0, newest=newest, c=c, screen=(0, 0, 0))
    d = _centres(obs) - np.array(src.origin)[None, :]
    R = np.linalg.norm(d, axis=1)
    tr = t - R / c
    dom = 0.1 * 0.2 * 0.15
    rho = a + b * tr
    E_ref = (dom / FOUR_PI) * (d.T * rho / R ** 3 + d.T * b / R ** 2 - J1[:, None] / R)
    Jr = J0[None, :] + J1[None, :] * tr[:, None]
    B_ref = (dom / FOUR_PI) * (np.cross(Jr, d).T / R ** 3 + np.cross(J1[None, :], d).T / R ** 2)
    assert np.allclose(E, E_ref, rtol=1e-11, atol=1e-14)
    assert np.allclose(B, B_ref, rtol=1e-11, atol=1e-14)


def test_quadratic_history_pins_the_derivative_reading():
    """rho = beta t^2: the value read is beta (t_r^2 + f (1-f) dt^2) and the
    derivative is beta (2 t_r - dt) (the backward difference taken on the
    linear interpolant).  The derivative of the interpolant would instead
    give beta (2 t_r + (1 - 2f) dt); the test tells the two apart."""
    src = _single_cell()
    obs = _obs_points(n=(4, 3, 3), origin=(0.55, 0.1, -0.2), sp=(0.13, 0.11, 0.07))
    beta, dt = 0.6, 0.05
    nt = 100
    hist = _hist_from(lambda t: [beta * t * t, 0.0, 0.0, 0.0], nt, 0, dt)
    t = (nt - 1) * dt
    E, _ = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0))
    d = _centres(obs)
    R = np.linalg.norm(d, axis=1)
    tr = t - R
    pos = tr / dt
    f = pos - np.floor(pos)
    val = beta * (tr ** 2 + f * (1 - f) * dt ** 2)
    der = beta * (2 * tr - dt)
    dom = 0.1 * 0.2 * 0.15
    E_ref = (dom / FOUR_PI) * (d.T * val / R ** 3 + d.T * der / R ** 2)
    assert np.allclose(E, E_ref, rtol=1e-10, atol=1e-15)
    der_alt = beta * (2 * tr + (1 - 2 * f) * dt)
    E_alt = (dom / FOUR_PI) * (d.T * val / R ** 3 + d.T * der_alt / R ** 2)
    assert not np.allclose(E, E_alt, rtol=1e-6, atol=0)


@pytest.mark.parametrize("where", ["k=-1", "k=0", "dead"])
def test_switch_on_at_the_oldest_slice(where):
    """Constant rho = h from the oldest slice on, zero before it:
    k = -1 -> value f h, derivative f h/dt; k = 0 -> value h, derivative
    (1-f) h/dt; a stencil wholly before the oldest slice -> exactly 0."""
    h, dt = 2.5, 0.1
    nt = 6
    src = _single_cell(h=(0.1, 0.1, 0.1))
    # choose R so that t_r falls where wanted: t = newest time = 0.5 (s_old = 0)
    t = (nt - 1) * dt
    target = {"k=-1": -0.037, "k=0": 0.063, "dead": -0.13}[where]
    R = t - target
    obs = Grid((1, 1, 1), (R * 0.6, R * 0.8, 0.0), (0.1, 0.1, 0.1))
    hist = _hist_from(lambda tt: [h, 0.0, 0.0, 0.0], nt, 0, dt)
    E, B = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0))
    d = _centres(obs)[0]
    Rr = float(np.linalg.norm(d))
    pos = (t - Rr) / dt
    f = pos - math.floor(pos)
    dom = 1e-3
    if where == "dead":
        assert np.all(E == 0.0) and np.all(B == 0.0)
        return
    if where == "k=-1":
        val, der = f * h, f * h / dt
    else:
        val, der = h, (1 - f) * h / dt
    E_ref = (dom / FOUR_PI) * (d * val / Rr ** 3 + d * der / Rr ** 2)
    assert np.allclose(E[:, 0], E_ref, rtol=1e-12, atol=0)
    assert np.all(B == 0.0)


def test_quadratic_history_slope_reading():
    """The slope reading (stencil bit 0) on rho = beta t^2: the value is the
    same interpolant, the derivative is the slope of the interpolant on the
    interval holding t_r, beta (t_(k+1)^2 - t_k^2)/dt = beta (2 t_r + (1 - 2f) dt)."""
    src = _single_cell()
    obs = _obs_points(n=(4, 3, 3), origin=(0.55, 0.1, -0.2), sp=(0.13, 0.11, 0.07))
    beta, dt = 0.6, 0.05
    nt = 100
    hist = _hist_from(lambda t: [beta * t * t, 0.0, 0.0, 0.0], nt, 0, dt)
    t = (nt - 1) * dt
    E, _ = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0), stencil=oracle.STENCIL_SLOPE)
    d = _centres(obs)
    R = np.linalg.norm(d, axis=1)
    tr = t - R
    pos = tr / dt
    f = pos - np.floor(pos)
    val = beta * (tr ** 2 + f * (1 - f) * dt ** 2)
    der = beta * (2 * tr + (1 - 2 * f) * dt)
    dom = 0.1 * 0.2 * 0.15
    E_ref = (dom / FOUR_PI) * (d.T * val / R ** 3 + d.T * der / R ** 2)
    assert np.allclose(E, E_ref, rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("where", ["k=-1", "k=0", "dead"])
def test_switch_on_slope_reading(where):
    """Constant rho = h from the oldest slice on, zero before it, slope
    reading: k = -1 -> value f h, derivative h/dt (the whole jump over one
    interval); k = 0 -> value h, derivative 0; wholly before -> 0."""
    h, dt = 2.5, 0.1
    nt = 6
    src = _single_cell(h=(0.1, 0.1, 0.1))
    t = (nt - 1) * dt
    target = {"k=-1": -0.037, "k=0": 0.063, "dead": -0.13}[where]
    R = t - target
    obs = Grid((1, 1, 1), (R * 0.6, R * 0.8, 0.0), (0.1, 0.1, 0.1))
    hist = _hist_from(lambda tt: [h, 0.0, 0.0, 0.0], nt, 0, dt)
    E, B = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0), stencil=oracle.STENCIL_SLOPE)
    d = _centres(obs)[0]
    Rr = float(np.linalg.norm(d))
    pos = (t - Rr) / dt
    f = pos - math.floor(pos)
    if where == "dead":
        assert np.all(E == 0.0) and np.all(B == 0.0)
        return
    val, der = (f * h, h / dt) if where == "k=-1" else (h, 0.0)
    E_ref = (1e-3 / FOUR_PI) * (d * val / Rr ** 3 + d * der / Rr ** 2)
    assert np.allclose(E[:, 0], E_ref, rtol=1e-12, atol=0)


def _poly_fields(coef_rho, coef_J, stencil, nt=120, dt=0.05):
    """Oracle E and a closed form for sources polynomial in time (rho and
    every J component), every stencil inside the stored window; the closed
    form takes value and derivative of the same polynomial at t_r."""
    src = _single_cell()
    obs = _obs_points(n=(4, 3, 3), origin=(0.55, 0.1, -0.2), sp=(0.13, 0.11, 0.07))
    pr = np.polynomial.Polynomial(coef_rho)
    pj = [np.polynomial.Polynomial(c) for c in coef_J]
    hist = _hist_from(lambda t: [pr(t), pj[0](t), pj[1](t), pj[2](t)], nt, 0, dt)
    t = (nt - 1) * dt - 0.013
    E, B = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0), stencil=stencil)
    d = _centres(obs)
    R = np.linalg.norm(d, axis=1)
    tr = t - R
    return E, B, d, R, tr, pr, pj, dt


def test_cubic_history_is_reproduced_exactly():
    """Cubic time interpolation (stencil bit 2) is exact for sources cubic
    in time: value and time derivative at t_r are those of the polynomial,
    so E and B equal the retarded closed forms."""
    E, B, d, R, tr, pr, pj, _ = _poly_fields([0.3, -0.7, 0.4, 0.25],
                                             [[0.1, 0.2, -0.3, 0.05], [-0.2, 0.0, 0.1, -0.15],
                                              [0.4, -0.1, 0.0, 0.2]], oracle.STENCIL_CUBIC)
    dom = 0.1 * 0.2 * 0.15
    Jr = np.stack([p(tr) for p in pj], axis=1)
    Jd = np.stack([p.deriv()(tr) for p in pj], axis=1)
    E_ref = (dom / FOUR_PI) * (d.T * pr(tr) / R ** 3 + d.T * pr.deriv()(tr) / R ** 2 - Jd.T / R)
    B_ref = (dom / FOUR_PI) * (np.cross(Jr, d).T / R ** 3 + np.cross(Jd, d).T / R ** 2)
    assert np.allclose(E, E_ref, rtol=1e-9, atol=1e-13)
    assert np.allclose(B, B_ref, rtol=1e-9, atol=1e-13)
    # the linear default is not exact for these sources
    E_lin, _, _, _, _, _, _, _ = _poly_fields([0.3, -0.7, 0.4, 0.25], [[0.0]] * 3, 0)
    assert not np.allclose(E_lin, E, rtol=1e-6, atol=0)


def test_quartic_history_pins_the_cubic_nodes():
    """rho = t^4: the cubic through slices k-2 .. k+1 misses it by
    dt^4 g(f), g(f) = (f+2)(f+1)f(f-1) (the interpolation error of t^4 is
    exact: its fourth derivative is 24 = 4!), and its derivative by
    dt^3 g'(f).  Nodes k-1 .. k+2 would give (f+1)f(f-1)(f-2) instead."""
    E, _, d, R, tr, _, _, dt = _poly_fields([0.0, 0.0, 0.0, 0.0, 1.0], [[0.0]] * 3, oracle.STENCIL_CUBIC)
    pos = tr / dt
    f = pos - np.floor(pos)
    g = (f + 2) * (f + 1) * f * (f - 1)
    gp = 4 * f ** 3 + 6 * f ** 2 - 2 * f - 2
    val = tr ** 4 - dt ** 4 * g
    der = 4 * tr ** 3 - dt ** 3 * gp
    dom = 0.1 * 0.2 * 0.15
    E_ref = (dom / FOUR_PI) * (d.T * val / R ** 3 + d.T * der / R ** 2)
    assert np.allclose(E, E_ref, rtol=1e-10, atol=1e-15)
    g_alt = (f + 1) * f * (f - 1) * (f - 2)
    E_alt = (dom / FOUR_PI) * (d.T * (tr ** 4 - dt ** 4 * g_alt) / R ** 3 + d.T * der / R ** 2)
    assert not np.allclose(E, E_alt, rtol=1e-9, atol=0)


@pytest.mark.parametrize("where", ["k=-1", "k=-2"])
def test_switch_on_cubic_reading(where):
    """Constant rho = h from the oldest slice on, zero before it, cubic
    reading: at k = -1 the nodes -3 .. 0 carry 0, 0, 0, h, so the value is
    h (f+2)(f+1)f/6 and the derivative h (3f^2 + 6f + 2)/(6 dt); at k = -2
    every node lies before the oldest slice and the pair gives exactly 0."""
    h, dt = 2.5, 0.1
    nt = 6
    src = _single_cell(h=(0.1, 0.1, 0.1))
    t = (nt - 1) * dt
    target = {"k=-1": -0.037, "k=-2": -0.13}[where]
    R = t - target
    obs = Grid((1, 1, 1), (R * 0.6, R * 0.8, 0.0), (0.1, 0.1, 0.1))
    hist = _hist_from(lambda tt: [h, 0.0, 0.0, 0.0], nt, 0, dt)
    E, B = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0), stencil=oracle.STENCIL_CUBIC)
    if where == "k=-2":
        assert np.all(E == 0.0) and np.all(B == 0.0)
        return
    d = _centres(obs)[0]
    Rr = float(np.linalg.norm(d))
    pos = (t - Rr) / dt
    f = pos - math.floor(pos)
    val = h * (f + 2) * (f + 1) * f / 6
    der = h * (3 * f * f + 6 * f + 2) / (6 * dt)
    E_ref = (1e-3 / FOUR_PI) * (d * val / Rr ** 3 + d * der / Rr ** 2)
    assert np.allclose(E[:, 0], E_ref, rtol=1e-12, atol=0)


def test_slope_and_cubic_readings_exclude_each_other():
    src = _single_cell()
    obs = _obs_points()
    hist = np.zeros((4, 4, 1))
    for st in (oracle.STENCIL_SLOPE | oracle.STENCIL_CUBIC, 7):
        with pytest.raises(Exception):
            oracle.eval_fields(src, obs, hist, 0.05, t=0.15, screen=(0, 0, 0), stencil=st)


@pytest.mark.parametrize("stencil", [2, 3, 6])
def test_held_past_constant_history_is_static_at_any_time(stencil):
    """History held at the oldest slice (stencil bit 1) and constant sources:
    the retarded sources are the constant ones at every t_r, so E and B are
    the static Coulomb and Biot-Savart fields at every evaluation time,
    including times long before the oldest slice, where the zero past gives
    exactly nothing."""
    src = _single_cell()
    obs = _obs_points()
    q, J = 0.8, np.array([0.3, -1.1, 0.6])
    dt, nt = 0.05, 4
    hist = _hist_from(lambda t: [q, *J], nt, 0, dt)
    d = _centres(obs)
    R = np.linalg.norm(d, axis=1)
    dom = 0.1 * 0.2 * 0.15
    E_ref = (q * dom / FOUR_PI) * d.T / R ** 3
    B_ref = (dom / FOUR_PI) * np.cross(J[None, :], d).T / R ** 3
    # the cubic's weights and their derivatives sum to 1 and 0 only up to rounding
    rtol = 1e-12 if stencil & oracle.STENCIL_CUBIC else 1e-14
    for t in [(nt - 1) * dt, 0.0, -0.4, -7.0]:
        E, B = oracle.eval_fields(src, obs, hist, dt, t=t, screen=(0, 0, 0), stencil=stencil)
        assert np.allclose(E, E_ref, rtol=rtol, atol=0), t
        assert np.allclose(B, B_ref, rtol=rtol, atol=1e-18), t
    E0, B0 = oracle.eval_fields(src, obs, hist, dt, t=-7.0, screen=(0, 0, 0))
    assert np.all(E0 == 0.0) and np.all(B0 == 0.0)


@pytest.mark.parametrize("stencil", [2, 3])
def test_held_past_linear_history(stencil):
    """rho = a + b t from the oldest slice t_old on, held at a + b t_old
    before it.  Value: a + b max(t_r, t_old) (the interpolant between two
    held slices is flat).  Derivative: 0 while t_r < t_old; on the first
    interval [t_old, t_old + dt) the interpolated backward difference gives
    f b (D_0 = 0 since h_(-1) = h_0) and the slope reading gives b; b later."""
    a, b = 0.7, -1.3
    dt, nt, s_old = 0.05, 8, 3
    t_old = s_old * dt
    newest = s_old + nt - 1
    t = newest * dt
    hist = _hist_from(lambda tt: [a + b * tt, 0.0, 0.0, 0.0], nt, s_old, dt)
    src = _single_cell(h=(0.1, 0.1, 0.1))
    # retarded times spread over the held past, the first interval and later
    Rs = t - (t_old + np.array([-0.31, -0.12, -0.037, 0.011, 0.029, 0.047, 0.09, 0.2]))
    E = np.zeros((3, len(Rs)))
    for i, R in enumerate(Rs):
        g = Grid((1, 1, 1), (R * 0.36, R * 0.48, R * 0.8), (0.1, 0.1, 0.1))
        e, _ = oracle.eval_fields(src, g, hist, dt, t=t, newest=newest, screen=(0, 0, 0), stencil=stencil)
        E[:, i] = e[:, 0]
    d = np.stack([Rs * 0.36, Rs * 0.48, Rs * 0.8])
    Rr = np.linalg.norm(d, axis=0)
    tr = t - Rr
    pos = (tr - t_old) / dt
    f = pos - np.floor(pos)
    val = a + b * np.maximum(tr, t_old)
    first = (tr >= t_old) & (tr < t_old + dt)
    if stencil & 1:
        der = np.where(tr >= t_old, b, 0.0)
    else:
        der = np.where(tr >= t_old + dt, b, np.where(first, f * b, 0.0))
    assert first.sum() == 3 and (tr < t_old).sum() == 3
    E_ref = (1e-3 / FOUR_PI) * (d * val / Rr ** 3 + d * der / Rr ** 2)
    assert np.allclose(E, E_ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("stencil", [8, 9])
def test_history_start_linear_history(stencil):
    """The history starts at the oldest slice (stencil bit 3): rho = a + b t
    from t_old on.  A pair whose retarded time precedes t_old contributes
    exactly nothing.  After it: value a + b t_r; derivative f b on the
    first interval (D_0 = 0: no difference is taken across the start) and
    b later; the slope reading (bit 0) gives b from t_old on."""
    a, b = 0.7, -1.3
    dt, nt, s_old = 0.05, 8, 3
    t_old = s_old * dt
    newest = s_old + nt - 1
    t = newest * dt
    hist = _hist_from(lambda tt: [a + b * tt, 0.0, 0.0, 0.0], nt, s_old, dt)
    src = _single_cell(h=(0.1, 0.1, 0.1))
    Rs = t - (t_old + np.array([-0.31, -0.12, -0.037, -0.004, 0.011, 0.029, 0.047, 0.09, 0.2]))
    E = np.zeros((3, len(Rs)))
    for i, R in enumerate(Rs):
        g = Grid((1, 1, 1), (R * 0.36, R * 0.48, R * 0.8), (0.1, 0.1, 0.1))
        e, bb = oracle.eval_fields(src, g, hist, dt, t=t, newest=newest, screen=(0, 0, 0), stencil=stencil)
        E[:, i] = e[:, 0]
        assert np.all(bb == 0.0)
    d = np.stack([Rs * 0.36, Rs * 0.48, Rs * 0.8])
    Rr = np.linalg.norm(d, axis=0)
    tr = t - Rr
    pos = (tr - t_old) / dt
    f = pos - np.floor(pos)
    live = tr >= t_old
    first = live & (tr < t_old + dt)
    val = np.where(live, a + b * tr, 0.0)
    if stencil & 1:
        der = np.where(live, b, 0.0)
    else:
        der = np.where(tr >= t_old + dt, b, np.where(first, f * b, 0.0))
    assert first.sum() == 3 and (~live).sum() == 4
    E_ref = (1e-3 / FOUR_PI) * (d * val / Rr ** 3 + d * der / Rr ** 2)
    assert np.allclose(E, E_ref, rtol=1e-11, atol=0)
    assert np.all(E[:, ~live] == 0.0)


@pytest.mark.parametrize("stencil", [8, 9, 12])
def test_history_start_constant_sources_are_the_static_ball_sum(stencil):
    """Constant rho and J from the oldest slice on, history starting there:
    every pair whose source lies within c (t - t_old) of the observation
    point carries the static Coulomb / Biot-Savart term, every other pair
    nothing (no switch-on shell).  Against that sum written out directly."""
    from tests.continuum import ball_sum_plane
    lo, hi = (-0.6, -0.6, -0.6), (0.6, 0.6, 0.6)
    cell = 0.2
    src = Grid((6, 6, 6), (-0.5, -0.5, -0.5), (cell,) * 3)
    obs = Grid((3, 3, 1), (-0.37, -0.21, 0.13), (0.41, 0.29, 0.2))  # clear of ties with cell edges
    dt, nt = 0.05, 40
    hist = _hist_from(lambda tt: [1.0, 1.0, 1.0, 1.0], nt, 0, dt, n_src=src.size)
    pts = _centres(obs)
    for t in (0.27, 0.61, 1.13):
        E, B = oracle.eval_fields(src, obs, hist, dt, t=t, newest=nt - 1, screen=(0.1, 0.1, 0.1), stencil=stencil)
        E_ref, B_ref = ball_sum_plane(pts, t, lo, hi, cell, 0.1)
        # the ball sum's B is J x E_coulomb; the Jefimenko B is -(1/4pi) sum d x J / R^3, the same
        assert np.allclose(E, E_ref, rtol=1e-12, atol=1e-15), t
        assert np.allclose(B, B_ref, rtol=1e-12, atol=1e-15), t
        # the zero past adds the switch-on shell
        E0, _ = oracle.eval_fields(src, obs, hist, dt, t=t, newest=nt - 1, screen=(0.1, 0.1, 0.1))
        assert np.abs(E0 - E_ref).max() > 1e-3 * np.abs(E_ref).max(), t


def test_history_start_and_held_past_exclude_each_other():
    src = _single_cell()
    obs = _obs_points()
    hist = np.zeros((4, 4, 1))
    for st in (oracle.STENCIL_HOLD | oracle.STENCIL_CUT, 16):
        with pytest.raises(Exception):
            oracle.eval_fields(src, obs, hist, 0.05, t=0.15, screen=(0, 0, 0), stencil=st)


def _sphere_quadrature(n_theta=24, n_phi=48):
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * (2 * math.pi / n_phi)
    pts, wts = [], []
    for ct, wt in zip(x, w):
        st = math.sqrt(1 - ct * ct)
        for p in phi:
            pts.append((st * math.cos(p), st * math.sin(p), ct))
            wts.append(wt * (2 * math.pi / n_phi))
    return np.array(pts), np.array(wts)


def _fields_at_points(src, hist, dt, t, pts):
    E = np.zeros((3, len(pts)))
    B = np.zeros((3, len(pts)))
    for i, p in enumerate(pts):
        g = Grid((1, 1, 1), tuple(map(float, p)), (1.0, 1.0, 1.0))
        e, b = oracle.eval_fields(src, g, hist, dt, t=t, screen=(0, 0, 0))
        E[:, i] = e[:, 0]
        B[:, i] = b[:, 0]
    return E, B


def test_gauss_flux_equals_enclosed_charge_and_B_flux_vanishes():
    """Static charges and currents: the flux of E through a sphere enclosing
    them equals the enclosed charge sum(rho dOmega) (rationalised units), and
    the flux of B through any closed surface is zero."""
    rng = np.random.default_rng(11)
    src = centred_grid((3, 3, 2), 0.1)
    nt, dt = 80, 0.05
    rho = rng.uniform(-1, 1, src.size)
    J = rng.uniform(-1, 1, (3, src.size))
    hist = np.zeros((nt, 4, src.size))
    hist[:, 0, :] = rho
    hist[:, 1:, :] = J
    pts, wts = _sphere_quadrature()
    radius = 1.1
    E, B = _fields_at_points(src, hist, dt, (nt - 1) * dt, pts * radius)
    flux_E = float(np.sum(wts * (E * pts.T).sum(axis=0))) * radius ** 2
    flux_B = float(np.sum(wts * (B * pts.T).sum(axis=0))) * radius ** 2
    Q = float(rho.sum()) * 0.1 ** 3
    assert abs(flux_E - Q) <= 1e-9 * max(1e-3, abs(Q)) + 1e-12
    Bscale = float(np.abs(J).sum()) * 0.1 ** 3 / (4 * math.pi * radius ** 2) * 4 * math.pi * radius ** 2
    assert abs(flux_B) <= 1e-9 * Bscale


def test_current_ring_on_axis():
    """Four cells carrying a counter-clockwise tangential current I around the
    z axis at radius a: on the axis B_z = 4 dOmega I a / (4 pi (a^2 + z^2)^(3/2))
    (right-hand rule, positive), B_x = B_y = 0, and E = 0 without charge."""
    a, I = 0.2, 1.7
    src = Grid((3, 3, 1), (-a, -a, 0.0), (a, a, 0.1))
    nt, dt = 60, 0.05
    hist = np.zeros((nt, 4, src.size))
    # cells (i, j): (2,1) at (+a, 0), (1,2) at (0, +a), (0,1) at (-a, 0), (1,0) at (0, -a)
    def lin(i, j):
        return i + 3 * j
    hist[:, 2, lin(2, 1)] = I     # +y current at +x
    hist[:, 1, lin(1, 2)] = -I    # -x current at +y
    hist[:, 2, lin(0, 1)] = -I    # -y current at -x
    hist[:, 1, lin(1, 0)] = I     # +x current at -y
    obs = Grid((1, 1, 7), (0.0, 0.0, -0.3), (1.0, 1.0, 0.1))
    E, B = oracle.eval_fields(src, obs, hist, dt, t=(nt - 1) * dt, screen=(0, 0, 0))
    z = -0.3 + 0.1 * np.arange(7)
    dom = a * a * 0.1
    Bz = 4 * dom * I * a / (FOUR_PI * (a * a + z * z) ** 1.5)
    assert np.allclose(B[2], Bz, rtol=1e-13, atol=0)
    assert np.all(np.abs(B[:2]) <= 1e-15 * np.abs(Bz).max())
    assert np.all(E == 0.0)


def test_saturation_for_constant_sources():
    """Constant sources switched on long enough ago (t - t_oldest >= d_m/c +
    2 dt) give fields that no longer change from one step to the next, equal
    to the static Coulomb/Biot-Savart superposition (the paper's saturation
    argument for constant sources)."""
    src = centred_grid((4, 3, 3), 0.1)
    obs = Grid((3, 3, 2), (0.25, -0.1, 0.07), (0.11, 0.1, 0.09))
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 1.0, src.size)
    J = rng.uniform(-1, 1, (3, src.size))
    dt = 0.05
    nt = 40
    hist = np.zeros((nt + 1, 4, src.size))
    hist[:, 0] = rho
    hist[:, 1:] = J
    E1, B1 = oracle.eval_fields(src, obs, hist[:nt], dt, t=(nt - 1) * dt, newest=nt - 1)
    E2, B2 = oracle.eval_fields(src, obs, hist[1:], dt, t=nt * dt, newest=nt)
    assert np.allclose(E1, E2, rtol=1e-14, atol=0) and np.allclose(B1, B2, rtol=1e-14, atol=0)
    rs = _centres(src)
    ro = _centres(obs)
    dom = 0.1 ** 3
    E_ref = np.zeros((3, obs.size))
    B_ref = np.zeros((3, obs.size))
    for s in range(src.size):
        d = ro - rs[s][None, :]
        R = np.linalg.norm(d, axis=1)
        E_ref += rho[s] * d.T / R ** 3
        B_ref += np.cross(J[:, s][None, :], d).T / R ** 3
    assert np.allclose(E1, E_ref * dom / FOUR_PI, rtol=1e-12)
    assert np.allclose(B1, B_ref * dom / FOUR_PI, rtol=1e-12)


def _static_fields(src, rho, J, pts, dt=0.5):
    """Oracle fields of time-independent sources (every stencil inside the
    stored history, so all backward differences vanish) at the points."""
    R = max(np.linalg.norm(np.asarray(p) - np.asarray(c)) for p in pts for c in _centres(src)[[0, -1]])
    nt = int(math.ceil((R + 2.0) / dt)) + 3
    hist = np.zeros((nt, 4, src.size))
    hist[:, 0, :] = rho
    hist[:, 1:4, :] = np.asarray(J, dtype=np.float64).reshape(3, -1) if np.ndim(J) > 1 else \
        np.asarray(J, dtype=np.float64)[:, None] * np.ones(src.size)[None, :]
    Es, Bs = [], []
    for p in pts:
        g = Grid((1, 1, 1), tuple(float(v) for v in p), (1.0, 1.0, 1.0))
        E, B = oracle.eval_fields(src, g, hist, dt, t=(nt - 1) * dt, screen=(0, 0, 0))
        Es.append(E[:, 0])
        Bs.append(B[:, 0])
    return np.array(Es).T, np.array(Bs).T


def test_voxelised_uniform_sphere_is_coulomb_outside():
    """Cells of a cubic grid whose centres lie within radius 0.5 carry unit
    charge density.  Outside, the field is that of the point charge
    Q = (cells) * h^3: the voxel set has cubic symmetry, so its dipole and
    quadrupole moments vanish and the relative deviation falls off like
    (a/r)^4 (the l = 4 moment)."""
    h, a = 0.1, 0.5
    src = centred_grid((11, 11, 11), h)
    c = _centres(src)
    rho = (np.linalg.norm(c, axis=1) <= a + 1e-12).astype(np.float64)
    Q = rho.sum() * h ** 3
    u = np.array([0.48, -0.36, 0.8])
    u /= np.linalg.norm(u)
    dists = [1.5, 3.0, 6.0]
    E, _ = _static_fields(src, rho, (0.0, 0.0, 0.0), [d * u for d in dists])
    devs = []
    for i, d in enumerate(dists):
        ref = Q / (FOUR_PI * d * d) * u
        devs.append(np.linalg.norm(E[:, i] - ref) / np.linalg.norm(ref))
    assert devs[0] < 0.02 and devs[2] < 1e-4, devs
    for k in (1, 2):
        assert 1 / 32 < devs[k] / devs[k - 1] < 1 / 8, devs   # ~ (1/2)^4


def test_uniform_charge_and_current_box_match_the_continuum():
    """A box of uniform charge density 1 and uniform current J: outside it,
    E is the closed-form field of a uniformly charged box and B = J x E (the
    static limits: Coulomb and Biot-Savart).  The cell sums are midpoint
    rules whose h^2 term is proportional to the Laplacian of the kernel,
    zero outside the sources (harmonic), so the error falls like h^4."""
    from tests.continuum import box_fields
    J = np.array([0.3, -0.7, 0.4])
    pts = [np.array([1.3, 0.2, -0.4]), np.array([-0.9, 1.1, 0.7]), np.array([0.1, -0.2, 1.6])]
    E_ex = box_fields(np.array(pts), (-0.5,) * 3, (0.5,) * 3)
    B_ex = np.cross(J[None, :], E_ex.T).T
    errs = []
    for n in (4, 8, 16):
        src = centred_grid((n, n, n), 1.0 / n)
        E, B = _static_fields(src, 1.0, J, pts)
        errs.append(max(np.abs(E - E_ex).max() / np.abs(E_ex).max(), np.abs(B - B_ex).max() / np.abs(B_ex).max()))
    assert errs[0] < 1e-4 and errs[2] < 1e-6, errs
    for k in (1, 2):
        assert 1 / 32 < errs[k] / errs[k - 1] < 1 / 8, errs   # ~ (1/2)^4


def _random_problem(rng, n_src=(3, 2, 3), n_obs=(2, 3, 2)):
    sp = tuple(rng.uniform(0.05, 0.15, 3))
    src = Grid(n_src, tuple(rng.uniform(-0.2, 0.0, 3)), sp)
    obs = Grid(n_obs, tuple(rng.uniform(-0.2, 0.3, 3)), tuple(rng.uniform(0.05, 0.15, 3)))
    nt = int(rng.integers(2, 12))
    dt = float(rng.uniform(0.02, 0.08))
    c = float(rng.uniform(0.7, 1.3))
    hist = rng.normal(size=(nt, 4, src.size))
    s_old = int(rng.integers(-5, 10))
    newest = s_old + nt - 1
    t0 = float(rng.uniform(-0.3, 0.3))
    t = t0 + newest * dt - float(rng.uniform(0, 2 * dt))
    if t < t0 + s_old * dt - 3 * dt:
        t = t0 + newest * dt
    screen = tuple(rng.uniform(0.0, 0.06, 3))
    return src, obs, hist, dt, t, t0, newest, c, screen


def test_c_oracle_matches_pure_python_on_the_tiny_workload():
    import workloads
    p = workloads.config_tiny()
    sel = list(range(0, p.obs.size, 7))
    E, B = oracle.eval_problem(p, sel=sel)
    E2, B2 = tiny.eval_fields(p.src, p.obs, p.hist, p.dt, p.t, p.t0, p.newest, p.c, p.screen, sel=sel)
    from oracle.compare import max_rel_l2
    assert max_rel_l2(E, B, np.array(E2), np.array(B2)) <= 1e-13
    dump = oracle.slice_index_dump(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    dump2 = np.array(tiny.slice_index_dump(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen))
    assert np.array_equal(dump, dump2)


@pytest.mark.parametrize("seed", range(12))
def test_c_oracle_matches_pure_python_on_random_tiny_problems(seed):
    rng = np.random.default_rng(100 + seed)
    src, obs, hist, dt, t, t0, newest, c, screen = _random_problem(rng)
    E, B = oracle.eval_fields(src, obs, hist, dt, t, t0, newest, c, screen)
    E2, B2 = tiny.eval_fields(src, obs, hist, dt, t, t0, newest, c, screen)
    E2, B2 = np.array(E2), np.array(B2)
    scale = max(np.abs(E2).max(), np.abs(B2).max(), 1e-300)
    assert np.abs(E - E2).max() <= 1e-13 * scale
    assert np.abs(B - B2).max() <= 1e-13 * scale
    nt = hist.shape[0]
    d1 = oracle.slice_index_dump(src, obs, nt, dt, t, t0, newest, c, screen)
    d2 = np.array(tiny.slice_index_dump(src, obs, nt, dt, t, t0, newest, c, screen))
    assert np.array_equal(d1, d2)


@pytest.mark.parametrize("seed,stencil", [(s, st) for s in range(4) for st in (1, 2, 3, 4, 6, 8, 9, 12)])
def test_c_oracle_matches_pure_python_stencil_readings(seed, stencil):
    rng = np.random.default_rng(300 + seed)
    src, obs, hist, dt, t, t0, newest, c, screen = _random_problem(rng)
    if seed % 2:
        t -= 0.5  # many stencils in the past
    E, B = oracle.eval_fields(src, obs, hist, dt, t, t0, newest, c, screen, stencil=stencil)
    E2, B2 = tiny.eval_fields(src, obs, hist, dt, t, t0, newest, c, screen, stencil=stencil)
    E2, B2 = np.array(E2), np.array(B2)
    scale = max(np.abs(E2).max(), np.abs(B2).max(), 1e-300)
    assert np.abs(E - E2).max() <= 1e-13 * scale
    assert np.abs(B - B2).max() <= 1e-13 * scale


def test_exact_integer_retarded_positions():
    """Pairs whose R/(c dt) is an exact integer (d = 0.5, dt = 0.25): the
    canonical FP64 sequence lands exactly on the slice boundary, f = 0 and
    slice k+1 is not needed."""
    src = Grid((1, 1, 1), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5))
    obs = Grid((4, 1, 1), (0.5, 0.0, 0.0), (0.5, 0.5, 0.5))
    nt, dt = 9, 0.25
    hist = np.zeros((nt, 4, 1))
    hist[:, 0, 0] = np.arange(nt) + 1.0
    t = (nt - 1) * dt
    dump = oracle.slice_index_dump(src, obs, nt, dt, t, screen=(0, 0, 0))
    # R = 0.5, 1.0, 1.5, 2.0 -> R/(c dt) = 2, 4, 6, 8 slices back
    assert dump[:, 0].tolist() == [6, 4, 2, 0]
    E, _ = oracle.eval_fields(src, obs, hist, dt, t, screen=(0, 0, 0))
    R = 0.5 * (np.arange(4) + 1)
    k = np.array([6, 4, 2, 0])
    val = k + 1.0
    der = np.where(k >= 1, 1.0 / dt, (k + 1.0) / dt)
    dom = 0.125
    E_ref = dom / FOUR_PI * (R * val / R ** 3 + R * der / R ** 2)
    assert np.allclose(E[0], E_ref, rtol=1e-14)


def test_time_after_newest_slice_is_rejected():
    src = centred_grid((2, 2, 2), 0.1)
    hist = np.ones((5, 4, src.size))
    with pytest.raises(ValueError):
        oracle.eval_fields(src, src, hist, 0.05, t=4 * 0.05 + 0.01)
    # exactly the newest time (up to rounding of t) is accepted
    oracle.eval_fields(src, src, hist, 0.05, t=4 * 0.05)
