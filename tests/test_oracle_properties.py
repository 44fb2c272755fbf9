"""Structural properties of the discretised sums, checked on the oracle:
linearity in the sources, superposition over disjoint cell subsets, the
mirror parities (E polar, B axial), invariance under translating both grids
by whole cells and under shifting the time origin."""
import numpy as np
import pytest

import oracle
from workloads import Grid, centred_grid, blob_history, Blob


def _setup(seed=0):
    rng = np.random.default_rng(seed)
    src = centred_grid((5, 4, 4), 0.1)
    obs = Grid((4, 3, 3), (0.31, -0.17, 0.05), (0.1, 0.1, 0.1))
    nt = 24
    h1 = rng.normal(size=(nt, 4, src.size))
    h2 = rng.normal(size=(nt, 4, src.size))
    return src, obs, h1, h2, 0.05, (nt - 1) * 0.05 - 0.013


def _close(a, b, tol):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() <= tol * scale


def test_linearity():
    src, obs, h1, h2, dt, t = _setup(1)
    E1, B1 = oracle.eval_fields(src, obs, h1, dt, t)
    E2, B2 = oracle.eval_fields(src, obs, h2, dt, t)
    E3, B3 = oracle.eval_fields(src, obs, 2.5 * h1 - 0.75 * h2, dt, t)
    assert _close(E3, 2.5 * E1 - 0.75 * E2, 1e-13)
    assert _close(B3, 2.5 * B1 - 0.75 * B2, 1e-13)


def test_superposition_over_disjoint_cells():
    src, obs, h1, _, dt, t = _setup(2)
    rng = np.random.default_rng(9)
    part = rng.integers(0, 3, src.size)
    E, B = oracle.eval_fields(src, obs, h1, dt, t)
    Es, Bs = np.zeros_like(E), np.zeros_like(B)
    for p in range(3):
        hp = h1 * (part == p)[None, None, :]
        e, b = oracle.eval_fields(src, obs, hp, dt, t)
        Es += e
        Bs += b
    assert _close(Es, E, 1e-13) and _close(Bs, B, 1e-13)


def test_mirror_x_parities():
    """Reflect sources through x = 0 (rho, Jy, Jz even, Jx odd): E_x flips,
    E_y, E_z keep; B (axial) keeps B_x and flips B_y, B_z."""
    src = centred_grid((6, 3, 4), 0.1)
    obs = centred_grid((4, 3, 2), 0.13)
    rng = np.random.default_rng(4)
    nt = 30
    h = rng.normal(size=(nt, 4, src.size)).reshape(nt, 4, 4, 3, 6)
    hm = h[..., ::-1].copy()
    hm[:, 1] *= -1.0
    h = h.reshape(nt, 4, -1)
    hm = hm.reshape(nt, 4, -1)
    dt, t = 0.05, (nt - 1) * 0.05
    E, B = oracle.eval_fields(src, obs, h, dt, t)
    Em, Bm = oracle.eval_fields(src, obs, hm, dt, t)
    n = obs.n
    def mirror(F):
        return F.reshape(3, n[2], n[1], n[0])[..., ::-1].reshape(3, -1)
    sE = np.array([-1, 1, 1])[:, None]
    sB = np.array([1, -1, -1])[:, None]
    assert _close(Em, sE * mirror(E), 1e-12)
    assert _close(Bm, sB * mirror(B), 1e-12)


def test_translation_by_whole_cells():
    src, obs, h1, _, dt, t = _setup(5)
    E, B = oracle.eval_fields(src, obs, h1, dt, t)
    Et, Bt = oracle.eval_fields(src.shifted_cells(3, -2, 5), obs.shifted_cells(3, -2, 5), h1, dt, t)
    assert _close(Et, E, 1e-12) and _close(Bt, B, 1e-12)


def test_time_origin_shift():
    """Moving the time origin and the step numbering together changes nothing."""
    src, obs, h1, _, dt, t = _setup(6)
    E, B = oracle.eval_fields(src, obs, h1, dt, t, t0=0.0, newest=h1.shape[0] - 1)
    m = 1000
    Es, Bs = oracle.eval_fields(src, obs, h1, dt, t, t0=-m * dt, newest=h1.shape[0] - 1 + m)
    assert _close(Es, E, 1e-10) and _close(Bs, B, 1e-10)


def test_uniformly_moving_blob_fields_are_finite_and_thread_independent():
    src = centred_grid((6, 6, 6), 0.1)
    obs = src.shifted_cells(2, 1, 0)
    h = blob_history(src, [Blob(1.0, 0.2, (0, 0, 0), (0, 0, 0.5))], 12, 0.05)
    E1, B1 = oracle.eval_fields(src, obs, h, 0.05, 11 * 0.05, threads=1)
    E4, B4 = oracle.eval_fields(src, obs, h, 0.05, 11 * 0.05, threads=4)
    assert np.all(np.isfinite(E1)) and np.array_equal(E1, E4) and np.array_equal(B1, B4)
