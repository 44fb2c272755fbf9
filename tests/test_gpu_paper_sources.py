"""The paper's own analytic workloads on the GPU (section on comparisons):
15^3 source and observation grids over [-3, 3]^3 (cell 0.4, screening
half-width 0.2), constant sources observed at t = 2.5, 5 and 7.5, and the
sinusoidal sources observed on [-3, 3]^2 x [10, 16]; both precisions
against the oracle.  With constant sources the fields stop changing once
every retarded time lies after the switch-on (the paper's saturation): the
device results at t and t + dt are then identical."""
import numpy as np
import pytest

import oracle
from oracle.compare import check_fields
from workloads import Grid, Problem, constant_step_history, sinusoidal_history

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
DX, N, DT = 0.4, 15, 0.1
SCREEN = (0.2, 0.2, 0.2)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import _gpu as G
    return G


def _box(z0=-3.0):
    """15 cells of 0.4 spanning [lo, lo + 6]: centres lo + 0.2 + 0.4 i."""
    return Grid((N, N, N), (-3.0 + 0.5 * DX, -3.0 + 0.5 * DX, z0 + 0.5 * DX), (DX, DX, DX))


def _check(G, p, label):
    Er, Br = oracle.eval_problem(p)
    for prec in ("f64", "f32"):
        Eg, Bg = G.gpu_eval(p, prec)
        check_fields(Eg, Bg, Er, Br, TOL[prec], f"{label} {prec}")


@pytest.mark.parametrize("t", [2.5, 5.0, 7.5])
def test_constant_sources(t):
    G = _gpu()
    src = _box()
    newest = int(round(t / DT))
    hist = constant_step_history(src, newest + 1, DT)
    p = Problem(f"const-{t}", src, src, hist, DT, newest * DT, 0.0, newest, 1.0, SCREEN)
    _check(G, p, f"constant t={t}")


@pytest.mark.parametrize("t", [5.0, 9.0, 12.0])
def test_sinusoidal_sources(t):
    """At t = 5 no retarded time from the source box (at least 7.4 away)
    has reached the observation box yet: exact zeros.  Later the front
    sweeps through it (t = 9) and covers it (t = 12)."""
    G = _gpu()
    src = _box()
    obs = _box(z0=10.0)
    newest = int(round(t / DT))
    hist = sinusoidal_history(src, newest + 1, DT)
    p = Problem(f"sin-{t}", src, obs, hist, DT, newest * DT, 0.0, newest, 1.0, SCREEN)
    if t < 7.0:
        for prec in ("f64", "f32"):
            Eg, Bg = G.gpu_eval(p, prec)
            assert np.all(Eg == 0.0) and np.all(Bg == 0.0)
        return
    _check(G, p, f"sinusoidal t={t}")


def test_constant_sources_saturate():
    """Longest separation 5.6 * sqrt(3) < 9.8: from t = 10 on (all retarded
    times after the switch-on plus one step) the fields are identical."""
    G = _gpu()
    src = _box()
    outs = {}
    for newest in (110, 111):
        hist = constant_step_history(src, newest + 1, DT)
        p = Problem(f"sat-{newest}", src, src, hist, DT, newest * DT, 0.0, newest, 1.0, SCREEN)
        for prec in ("f64", "f32"):
            outs[(newest, prec)] = G.gpu_eval(p, prec)
    for prec in ("f64", "f32"):
        a, b = outs[(110, prec)], outs[(111, prec)]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), prec
