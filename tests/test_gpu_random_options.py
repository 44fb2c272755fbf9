"""Randomised parity sweep over option combinations: ragged random problems
(partial tiles and bricks, unequal spacings, c != 1, screening widths from
0 to a few cells, windows not starting at step 0), each evaluated with a
random index mode, time-stencil reading and launch shape in both
precisions, at a time inside the window or before it; fields against the
oracle with the same reading, fingerprints against the oracle's."""
import numpy as np
import pytest

import oracle
from oracle.compare import check_fields
from tests.test_gpu_parity import _ragged_problem
from workloads import Problem

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


# oracle stencil bits: 1 slope, 2 hold, 4 cubic, 8 history start (slope and cubic,
# hold and history start exclude each other)
READINGS = (0, 1, 2, 3, 4, 6, 8, 9, 12)


@pytest.mark.parametrize("seed", range(6 * len(READINGS)))
def test_random_option_combinations(seed):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import _gpu as G
    rng = np.random.default_rng(1000 + seed)
    p = _ragged_problem(200 + seed, smooth=bool(seed % 3))
    if seed % 4 == 3:  # evaluation time before the window's oldest slice
        t_old = p.t0 + (p.newest - p.nt + 1) * p.dt
        p = Problem(p.name + "-early", p.src, p.obs, p.hist, p.dt, t_old - float(rng.uniform(0.2, 4.0)) * p.dt,
                    p.t0, p.newest, p.c, p.screen)
    idx = seed % 3                               # auto, guard, table
    stencil = READINGS[(seed // 3) % len(READINGS)]  # each (index mode, reading) pair twice
    flags = idx | (stencil << 2)  # JEFI_FLAG_DERIV_SLOPE = 4, _PAST_HOLD = 8, _TIME_CUBIC = 16, _PAST_CUT = 32
    tile = int(rng.integers(0, 3))
    Er, Br = oracle.eval_problem(p, stencil=stencil)
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    for prec in ("f64", "f32"):
        Eg, Bg = G.gpu_eval(p, prec, tile=tile, flags=flags)
        check_fields(Eg, Bg, Er, Br, TOL[prec], f"{p.name} {prec} flags {flags} tile {tile}")
        assert np.array_equal(G.gpu_fingerprint(p, prec, tile=tile, flags=flags), fp_ref), (p.name, prec, flags)


@pytest.mark.parametrize("seed", [74, 243])
def test_fields_made_by_the_switch_on_front(seed):
    """Two draws of the same generator whose fields come from the switch-on
    front alone (a 5-slice window read from its start; an evaluation just
    before the window's oldest slice), so that the terms cancel to a few
    percent: the FP64 path stays within its bar, and the FP32 path's slice
    indices stay exact (its fields carry its per-term error times that
    cancellation, about 2e-5, and are not held to the FP32 bar here)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import _gpu as G
    rng = np.random.default_rng(1000 + seed)
    p = _ragged_problem(200 + seed, smooth=bool(seed % 3))
    if seed % 4 == 3:
        t_old = p.t0 + (p.newest - p.nt + 1) * p.dt
        p = Problem(p.name + "-early", p.src, p.obs, p.hist, p.dt, t_old - float(rng.uniform(0.2, 4.0)) * p.dt,
                    p.t0, p.newest, p.c, p.screen)
    stencil = READINGS[(seed // 3) % len(READINGS)]
    flags = (seed % 3) | (stencil << 2)
    tile = int(rng.integers(0, 3))
    Er, Br = oracle.eval_problem(p, stencil=stencil)
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    Eg, Bg = G.gpu_eval(p, "f64", tile=tile, flags=flags)
    check_fields(Eg, Bg, Er, Br, TOL["f64"], f"{p.name} f64 flags {flags} tile {tile}")
    for prec in ("f64", "f32"):
        assert np.array_equal(G.gpu_fingerprint(p, prec, tile=tile, flags=flags), fp_ref), (p.name, prec, flags)
