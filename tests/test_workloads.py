"""The seeded input generators: the paper's sinusoidal sources and the
moving Gaussian blobs conserve charge (discrete continuity to second order
in the spacing and the time step), blob currents are charge density times
velocity, a blob moves rigidly, and draws are reproducible."""
import math

import numpy as np

import workloads
from workloads import Blob, Grid, blob_history, centred_grid, sinusoidal_history


def _continuity_residual(g, hist3, dt):
    """Max over interior cells of |d rho/dt + div J| from central differences:
    hist3 holds the slices at t - dt, t, t + dt; the spacing is uniform."""
    n = g.n[::-1]  # arrays are [z][y][x]
    rho_m = hist3[0, 0].reshape(n)
    rho_p = hist3[2, 0].reshape(n)
    jx, jy, jz = (hist3[1, c].reshape(n) for c in (1, 2, 3))
    h = g.spacing[0]
    drho = (rho_p - rho_m) / (2.0 * dt)
    div = ((jx[1:-1, 1:-1, 2:] - jx[1:-1, 1:-1, :-2]) + (jy[1:-1, 2:, 1:-1] - jy[1:-1, :-2, 1:-1])
           + (jz[2:, 1:-1, 1:-1] - jz[:-2, 1:-1, 1:-1])) / (2.0 * h)
    res = drho[1:-1, 1:-1, 1:-1] + div
    return float(np.max(np.abs(res))), float(np.max(np.abs(drho)))


def test_sinusoidal_sources_conserve_charge():
    """rho = 3 (cos t - 1) cos(x+y+z), J = sin(x+y+z) sin t (1,1,1): the
    discrete continuity residual falls about 4x when spacing and step halve
    (the paper states the continuity of this source family)."""
    res = []
    for n, h in ((12, 0.2), (24, 0.1)):
        g = centred_grid((n, n, n), h)
        dt = h / 2
        hist = sinusoidal_history(g, [19, 20, 21], dt)
        r, scale = _continuity_residual(g, hist, dt)
        res.append(r / scale)
    assert res[1] < 0.02
    assert 3.2 < res[0] / res[1] < 4.8, res


def test_blob_sources_conserve_charge():
    blobs = [Blob(0.8, 0.15, (0.05, -0.1, 0.0), (0.5, -0.3, 0.2)),
             Blob(-0.5, 0.2, (-0.2, 0.1, 0.1), (-0.2, 0.4, -0.1))]
    res = []
    for n, h in ((24, 0.05), (48, 0.025)):
        g = centred_grid((n, n, n), h)
        dt = h / 2
        hist = blob_history(g, blobs, [3, 4, 5], dt)
        r, scale = _continuity_residual(g, hist, dt)
        res.append(r / scale)
    assert res[1] < 0.05
    assert 3.0 < res[0] / res[1] < 5.0, res


def test_blob_current_is_density_times_velocity():
    v = (0.3, -0.6, 0.1)
    g = centred_grid((10, 9, 8), 0.07)
    h = blob_history(g, [Blob(1.3, 0.12, (0.02, 0.0, -0.05), v)], 4, 0.02)
    for a in range(3):
        assert np.allclose(h[:, 1 + a], h[:, 0] * v[a], rtol=1e-13, atol=0.0)


def test_blob_moves_rigidly():
    """Advancing time by s steps equals shifting the grid by -v*s*dt."""
    v = (0.4, 0.0, -0.2)
    dt, s = 0.025, 6
    g = Grid((8, 8, 8), (-0.3, -0.2, -0.25), (0.05, 0.05, 0.05))
    b = Blob(0.9, 0.1, (0.0, 0.05, 0.0), v)
    later = blob_history(g, [b], [s], dt)[0, 0]
    g2 = Grid(g.n, tuple(g.origin[a] - v[a] * s * dt for a in range(3)), g.spacing)
    now = blob_history(g2, [b], [0], dt)[0, 0]
    assert np.allclose(later, now, rtol=1e-12, atol=1e-300)


def test_total_charge_of_a_resolved_blob():
    """The sampled density integrates to q (the Gaussian is normalised)."""
    g = centred_grid((40, 40, 40), 0.04)
    q = -0.7
    h = blob_history(g, [Blob(q, 0.15, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))], 1, 0.01)
    total = h[0, 0].sum() * 0.04 ** 3
    assert math.isclose(total, q, rel_tol=1e-6)


def test_draws_are_reproducible_and_in_range():
    a = workloads.draw_blobs(np.random.default_rng(12), 30, (-0.8, 0.8))
    b = workloads.draw_blobs(np.random.default_rng(12), 30, (-0.8, 0.8))
    assert a == b
    for bl in a:
        assert all(-0.8 <= c <= 0.8 for c in bl.centre)
        assert 0.05 <= bl.sigma <= 0.2 and -1.0 <= bl.q <= 1.0
        assert math.sqrt(sum(x * x for x in bl.velocity)) <= 0.8 + 1e-12


def test_paper_source_factors_compose_the_paper_histories():
    """Time factor x spatial pattern (the form the accuracy study builds on
    the device) gives exactly the paper's constant and sinusoidal histories."""
    import workloads as W
    g = W.centred_grid((5, 4, 3), 0.4)
    ph = W.cell_centres(g).sum(1)
    steps = [-2, 0, 3, 7]
    for kind, fn, pr, pj in [("constant", W.constant_step_history, np.ones_like(ph), np.ones_like(ph)),
                             ("sinusoidal", W.sinusoidal_history, np.cos(ph), np.sin(ph))]:
        h = fn(g, steps, 0.3)
        for si, s in enumerate(steps):
            a, b = W.paper_source_factors(kind, s * 0.3)
            assert np.array_equal(h[si], np.stack([a * pr, b * pj, b * pj, b * pj])), (kind, s)
