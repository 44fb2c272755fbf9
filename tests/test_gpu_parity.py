"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: the slice index is bit-exact (per-pair dumps on small problems,
per-point fingerprints taken by the field kernel itself on larger ones);
E and B agree per component in relative L2 within 1e-12 (FP64 path) and
1e-5 (FP32 compensated path), and at every point within ten times that of
the component's largest value."""
import math

import numpy as np
import pytest

import oracle
import workloads
from oracle.compare import check_fields, rel_l2
from workloads import Grid, Problem, blob_history, centred_grid, Blob

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}

_ORACLE_CACHE = {}


def _oracle(p, sel=None, kind="fields"):
    """Oracle results cached per problem within the test session."""
    key = (p.name, kind, None if sel is None else tuple(int(v) for v in sel))
    if key not in _ORACLE_CACHE:
        if kind == "fields":
            _ORACLE_CACHE[key] = oracle.eval_problem(p, sel=sel)
        else:
            _ORACLE_CACHE[key] = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest,
                                                          p.c, p.screen, sel=sel)
    return _ORACLE_CACHE[key]


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import _gpu as G
    return G


_PROBLEMS = {}


def _medium():
    if "medium" not in _PROBLEMS:
        _PROBLEMS["medium"] = workloads.config_medium()
    return _PROBLEMS["medium"]


def _large():
    if "large" not in _PROBLEMS:
        _PROBLEMS["large"] = workloads.config_large()
    return _PROBLEMS["large"]


def _assert_fields(Eg, Bg, Er, Br, tol, label=""):
    """Relative L2 per component <= tol and every point within 10 tol of
    its component's largest value."""
    check_fields(Eg, Bg, Er, Br, tol, label or "fields")


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tiny_fields(prec, tile):
    G = _gpu()
    p = workloads.config_tiny()
    Er, Br = oracle.eval_problem(p)
    Eg, Bg = G.gpu_eval(p, prec, tile=tile)
    _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"tiny {prec} tile {tile}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tiny_slice_index_bit_exact(prec):
    G = _gpu()
    p = workloads.config_tiny()
    ref = oracle.slice_index_dump(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    got = G.gpu_dump(p, prec)
    assert np.array_equal(got, ref)
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    fp = G.gpu_fingerprint(p, prec)
    assert np.array_equal(fp, fp_ref)


@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_medium_fields_and_fingerprint(prec, tile):
    G = _gpu()
    p = _medium()
    Er, Br = _oracle(p)
    Eg, Bg = G.gpu_eval(p, prec, tile=tile)
    _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"medium {prec} tile {tile}")
    fp_ref = _oracle(p, kind="fp")
    fp = G.gpu_fingerprint(p, prec, tile=tile)
    assert np.array_equal(fp, fp_ref)


def test_tile_shapes_agree():
    """The two launch shapes sum in different orders; their results agree
    far inside the tolerance (FP32 1e-6, FP64 1e-14)."""
    G = _gpu()
    p = _medium()
    for prec, tol in (("f32", 1e-6), ("f64", 1e-14)):
        E1, B1 = G.gpu_eval(p, prec, tile=1)
        E2, B2 = G.gpu_eval(p, prec, tile=2)
        _assert_fields(E1, B1, E2, B2, tol, f"tile shapes {prec}")


@pytest.mark.parametrize("flags", [1, 2])
@pytest.mark.parametrize("which", ["medium", "ragged"])
def test_index_modes(which, flags):
    """Both ways of reaching the canonical slice index in FP32 (guard band
    with FP64 re-decision; threshold table for every pair) give the oracle's
    indices bit for bit and its fields within tolerance, on an aligned grid
    (many exact-integer retarded positions) and a generic one."""
    G = _gpu()
    p = _medium() if which == "medium" else _ragged_problem(11)
    Er, Br = _oracle(p)
    Eg, Bg = G.gpu_eval(p, "f32", flags=flags)
    _assert_fields(Eg, Bg, Er, Br, TOL["f32"], f"{which} flags {flags}")
    fp = G.gpu_fingerprint(p, "f32", flags=flags)
    assert np.array_equal(fp, _oracle(p, kind="fp"))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_large_sampled(prec):
    """64^3 x 64^3, 128 slices, at full size in the launch shape the bench
    times; 192 seeded observation points checked against the oracle one by
    one, fingerprints too."""
    G = _gpu()
    p = _large()
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(p.obs.size, size=192, replace=False))
    Er, Br = _oracle(p, sel=sel)
    Eg, Bg = G.gpu_eval(p, prec)
    _assert_fields(Eg[:, sel], Bg[:, sel], Er, Br, TOL[prec], f"large {prec}")
    fp_ref = _oracle(p, sel=sel, kind="fp")
    fp = G.gpu_fingerprint(p, prec)
    assert np.array_equal(fp[sel], fp_ref)


def _ragged_problem(seed, smooth=True):
    rng = np.random.default_rng(seed)
    ns = tuple(int(v) for v in rng.integers(3, 19, 3))
    no = tuple(int(v) for v in rng.integers(1, 21, 3))
    hs = float(rng.uniform(0.04, 0.09))
    src = Grid(ns, tuple(rng.uniform(-0.5, -0.2, 3)), (hs, hs * rng.uniform(0.8, 1.2), hs))
    obs = Grid(no, tuple(rng.uniform(-0.6, 0.2, 3)), tuple(rng.uniform(0.03, 0.1, 3)))
    dt = float(rng.uniform(0.3, 0.7)) * hs
    nt = int(rng.integers(4, 40))
    s_old = int(rng.integers(0, 50))
    newest = s_old + nt - 1
    c = float(rng.uniform(0.8, 1.25))
    if smooth:
        blobs = workloads.draw_blobs(rng, 3, (-0.5, 0.3))
        hist = blob_history(src, blobs, list(range(s_old, newest + 1)), dt)
    else:
        hist = rng.normal(size=(nt, 4, src.size))
    t = newest * dt - float(rng.uniform(0, 1.5)) * dt
    screen = tuple(float(v) for v in rng.uniform(0.0, 0.06, 3))
    return Problem(f"ragged{seed}", src, obs, hist, dt, t, 0.0, newest, c, screen)


@pytest.mark.parametrize("when,ratio", [("all-past", 2), ("front", 2), ("front", 10)])
def test_fingerprint_counts_screened_pairs_in_the_past(when, ratio):
    """Every screened pair is counted, also where a brick lies wholly before
    the oldest slice: a time before the window (every brick dead) and a time
    just after its start with a screening cube of several cells, so that
    near bricks are dead too (spacing / (c dt) = 10 takes the chunked
    kernel).  Fingerprints against the oracle, both precisions and tiles."""
    G = _gpu()
    h = 0.05
    src = Grid((12, 10, 9), (-0.3, -0.2, -0.25), (h, h, h))
    obs = Grid((9, 11, 6), tuple(src.origin[a] + (3, -2, 1)[a] * h for a in range(3)), (h, h, h))
    dt, nt, s_old = h / ratio, 4 * ratio, 5
    newest = s_old + nt - 1
    hist = blob_history(src, [Blob(1.0, 0.1, (0.0, 0.0, 0.0), (0.2, 0.0, 0.1))], list(range(s_old, newest + 1)), dt)
    # evaluation time in steps after the oldest slice: before it, or where only
    # pairs closer than about 3 spacings are live (inside the screening cube's reach)
    x = -3.2 if when == "all-past" else 3.0 * ratio - 0.9
    p = Problem(f"screened-{when}-{ratio}", src, obs, hist, dt, (s_old + x) * dt, 0.0, newest, 1.0,
                (2.5 * h, 2.5 * h, 2.5 * h))
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    assert fp_ref[:, 3].sum() > 0
    assert (fp_ref[:, 0].sum() > 0) == (when == "front")
    for prec in ["f64", "f32"]:
        for tile in [1, 2]:
            fp = G.gpu_fingerprint(p, prec, tile=tile)
            assert np.array_equal(fp, fp_ref), (p.name, prec, tile, fp.sum(axis=0), fp_ref.sum(axis=0))


@pytest.mark.parametrize("seed", range(8))
def test_ragged_random_problems(seed):
    """Ragged grid sizes (partial tiles and bricks), unequal spacings, c != 1,
    t between slices, a window not starting at step 0, arbitrary screening."""
    G = _gpu()
    p = _ragged_problem(seed)
    Er, Br = oracle.eval_problem(p)
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    for prec in ["f64", "f32"]:
        for tile in [1, 2]:
            Eg, Bg = G.gpu_eval(p, prec, tile=tile)
            _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"{p.name} {prec} tile {tile}")
            assert np.array_equal(G.gpu_fingerprint(p, prec, tile=tile), fp_ref)


@pytest.mark.parametrize("seed", [3, 5])
def test_large_step_numbers(seed):
    """The window starts at step ~3e7 (t/dt ~ 3e7, far beyond FP32's integer
    range; the time origin keeps the blobs in view): the FP64 split of the
    evaluation time keeps both paths exact."""
    G = _gpu()
    base = _ragged_problem(seed)
    rng = np.random.default_rng(seed)
    s_old = int(rng.integers(2 * 10 ** 7, 4 * 10 ** 7))
    newest = s_old + base.nt - 1
    t0 = -s_old * base.dt
    blobs = workloads.draw_blobs(rng, 3, (-0.5, 0.3))
    hist = blob_history(base.src, blobs, list(range(s_old, newest + 1)), base.dt, t0)
    t = t0 + newest * base.dt - 0.37 * base.dt
    p = Problem(f"bigstep{seed}", base.src, base.obs, hist, base.dt, t, t0, newest, base.c, base.screen)
    Er, Br = oracle.eval_problem(p)
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    for prec in ["f64", "f32"]:
        Eg, Bg = G.gpu_eval(p, prec)
        _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"{p.name} {prec}")
        assert np.array_equal(G.gpu_fingerprint(p, prec), fp_ref)


@pytest.mark.parametrize("seed", range(4))
def test_rough_histories_fp64(seed):
    """White-noise histories (no smoothness to hide interpolation mistakes)."""
    G = _gpu()
    p = _ragged_problem(100 + seed, smooth=False)
    Er, Br = oracle.eval_problem(p)
    Eg, Bg = G.gpu_eval(p, "f64")
    _assert_fields(Eg, Bg, Er, Br, TOL["f64"], f"{p.name} rough")


def test_long_windows_take_the_chunked_path():
    """dt much smaller than the spacing: slice windows longer than one LDS
    staging chunk."""
    G = _gpu()
    src = centred_grid((6, 5, 7), 0.1)
    obs = src.shifted_cells(3, 1, -2)
    dt = 0.01
    nt = 120
    blobs = [Blob(1.0, 0.15, (0.0, 0.05, 0.0), (0.3, 0.0, 0.2)), Blob(-0.5, 0.1, (0.1, 0, 0), (0, 0.4, 0))]
    hist = blob_history(src, blobs, nt, dt)
    p = Problem("chunked", src, obs, hist, dt, (nt - 1) * dt, 0.0, nt - 1, 1.0, workloads.default_screen(src))
    Er, Br = oracle.eval_problem(p)
    for prec in ["f64", "f32"]:
        Eg, Bg = G.gpu_eval(p, prec)
        _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"chunked {prec}")
        fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
        assert np.array_equal(G.gpu_fingerprint(p, prec), fp_ref)


@pytest.mark.parametrize("ratio", [4, 8, 10])
def test_staging_window_sizes(ratio):
    """Spacing / (c dt) = 4, 8, 10 with 8x8x8 tiles: slice windows of about
    58, 114 and 142 slots, i.e. the 64- and 128-slot staging shapes and the
    chunked kernel (FP64 stages at most 64 slots); fields and fingerprints
    against the oracle, including points near the switch-on front."""
    G = _gpu()
    h = 0.1
    src = centred_grid((10, 9, 11), h)
    obs = Grid((9, 10, 8), tuple(src.origin[a] + (3, -2, 4)[a] * h for a in range(3)), (h, h, h))
    dt = h / ratio
    nt = 9 * ratio  # shorter than the longest separation: some pairs lie before the oldest slice
    blobs = [Blob(1.0, 0.15, (0.0, 0.05, 0.0), (0.3, 0.0, 0.2)), Blob(-0.5, 0.1, (0.1, 0, 0), (0, 0.4, 0))]
    hist = blob_history(src, blobs, nt, dt)
    p = Problem(f"window{ratio}", src, obs, hist, dt, (nt - 1) * dt - 0.3 * dt, 0.0, nt - 1, 1.0,
                workloads.default_screen(src))
    Er, Br = oracle.eval_problem(p)
    fp_ref = oracle.slice_fingerprint(p.src, p.obs, p.nt, p.dt, p.t, p.t0, p.newest, p.c, p.screen)
    for prec in ["f64", "f32"]:
        Eg, Bg = G.gpu_eval(p, prec)
        _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"window ratio {ratio} {prec}")
        assert np.array_equal(G.gpu_fingerprint(p, prec), fp_ref)


def test_exact_integer_boundaries_dump():
    """R/(c dt) exactly integral (d = 0.5, dt = 0.25): both device index
    paths return the canonical k, including on the slice boundary."""
    G = _gpu()
    src = Grid((3, 3, 3), (0.0, 0.0, 0.0), (0.5, 0.5, 0.5))
    obs = Grid((5, 4, 3), (0.5, 0.0, 0.0), (0.5, 0.5, 0.5))
    nt, dt = 12, 0.25
    p = Problem("int", src, obs, np.zeros((nt, 4, src.size)), dt, (nt - 1) * dt, 0.0, nt - 1, 1.0,
                (0.0, 0.0, 0.0))
    ref = oracle.slice_index_dump(src, obs, nt, dt, p.t, 0.0, nt - 1, 1.0, (0.0, 0.0, 0.0))
    for prec in ["f64", "f32"]:
        assert np.array_equal(G.gpu_dump(p, prec), ref)


def test_random_pairs_dump_bit_exact():
    """Many random pairs with large R/(c dt): the FP32 guard band holds."""
    G = _gpu()
    rng = np.random.default_rng(5)
    for trial in range(4):
        src = Grid((17, 13, 11), tuple(rng.uniform(-1, 0, 3)), tuple(rng.uniform(0.01, 0.05, 3)))
        obs = Grid((19, 7, 9), tuple(rng.uniform(0, 2, 3)), tuple(rng.uniform(0.01, 0.1, 3)))
        dt = float(rng.uniform(0.002, 0.02))
        nt = 1000
        newest = nt - 1 + int(rng.integers(0, 10 ** 6))
        t = newest * dt - float(rng.uniform(0, 3)) * dt
        p = Problem("rp", src, obs, np.zeros((nt, 4, 0)), dt, t, 0.0, newest, 1.0, (0.0, 0.0, 0.0))
        ref = oracle.slice_index_dump(src, obs, nt, dt, t, 0.0, newest, 1.0, (0.0, 0.0, 0.0))
        for prec in ["f64", "f32"]:
            assert np.array_equal(G.gpu_dump(p, prec), ref)


@pytest.mark.parametrize("kind", ["random", "aligned"])
def test_index_function_on_1e7_pairs(kind):
    """About 10^7 pairs, per-pair slice indices from the dump kernel and
    per-point fingerprints from the field kernel in both FP32 index modes,
    all equal to the oracle's canonical FP64 decisions.  'aligned' puts a
    few percent of the pairs at exact integer retarded positions."""
    G = _gpu()
    rng = np.random.default_rng(99 if kind == "random" else 98)
    if kind == "random":
        src = Grid((31, 29, 23), tuple(rng.uniform(-1, 0, 3)), tuple(rng.uniform(0.01, 0.04, 3)))
        obs = Grid((10, 10, 5), tuple(rng.uniform(-0.5, 1.5, 3)), tuple(rng.uniform(0.01, 0.08, 3)))
        dt = float(rng.uniform(0.002, 0.01))
    else:
        h = 0.02
        src = centred_grid((31, 29, 23), h)
        obs = src.shifted_cells(9, -4, 3)
        obs = Grid((10, 10, 5), obs.origin, obs.spacing)
        dt = h / 2.0  # c*dt divides the spacing
    nt = 400
    newest = nt - 1 + int(rng.integers(0, 10 ** 5))
    t = newest * dt
    screen = (0.0, 0.0, 0.0)
    p = Problem(kind, src, obs, np.zeros((nt, 4, src.size)), dt, t, 0.0, newest, 1.0, screen)
    assert src.size * obs.size > 10 ** 7
    ref = oracle.slice_index_dump(src, obs, nt, dt, t, 0.0, newest, 1.0, screen)
    for prec in ["f64", "f32"]:
        assert np.array_equal(G.gpu_dump(p, prec), ref), prec
    fp_ref = _oracle(p, kind="fp")
    assert np.array_equal(G.gpu_fingerprint(p, "f64"), fp_ref)
    for flags in (1, 2):
        assert np.array_equal(G.gpu_fingerprint(p, "f32", flags=flags), fp_ref), flags


def test_edge_cases():
    import torch
    import paper_2104_05426_amd as J
    G = _gpu()
    base = workloads.config_tiny()
    # empty observation grid: no-op
    empty = Grid((0, 0, 0), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    E, B = G.gpu_eval(base, "f32", obs=empty)
    assert E.shape == (3, 0)
    # a single source cell, nt = 1 (the only slice, zero before it)
    src1 = Grid((1, 1, 1), (0.0, 0.0, 0.0), (0.1, 0.1, 0.1))
    obs1 = Grid((3, 2, 2), (0.03, 0.02, 0.01), (0.05, 0.05, 0.05))
    h = np.zeros((1, 4, 1))
    h[0, :, 0] = [1.0, 0.5, -0.25, 2.0]
    p1 = Problem("one", src1, obs1, h, 0.1, 0.0, 0.0, 0, 1.0, (0.0, 0.0, 0.0))
    Er, Br = oracle.eval_problem(p1)
    for prec in ["f64", "f32"]:
        Eg, Bg = G.gpu_eval(p1, prec)
        _assert_fields(Eg, Bg, Er, Br, TOL[prec], f"one-cell {prec}")
    # evaluation time long before the window: every stencil is in the past -> zeros
    pe = Problem("past", base.src, base.obs, base.hist, base.dt, -5.0, 0.0, base.newest, 1.0, base.screen)
    Eg, Bg = G.gpu_eval(pe, "f32")
    assert np.all(Eg == 0.0) and np.all(Bg == 0.0)
    # FP64 output dtype from the FP32 path, and FP32 output from the FP64 path
    Er, Br = oracle.eval_problem(base)
    Eg, Bg = G.gpu_eval(base, "f32", out_dtype="f64")
    _assert_fields(Eg, Bg, Er, Br, TOL["f32"], "f32->f64 out")
    Eg, Bg = G.gpu_eval(base, "f64", out_dtype="f32")
    _assert_fields(Eg, Bg, Er, Br, 1e-6, "f64->f32 out")


def test_invalid_arguments_leave_outputs_untouched():
    import torch
    import paper_2104_05426_amd as J
    _gpu()
    p = workloads.config_tiny()
    store, h = J.upload_history(p.src, p.hist, J.JEFI_F32, newest=p.newest)
    E = torch.full((3, p.obs.size), 7.0, device="cuda")
    B = torch.full((3, p.obs.size), 7.0, device="cuda")
    with pytest.raises(J.JefiError):
        J.jefi_eval_fields(p.src, h, p.dt, p.nt, p.obs, p.t + 1.0, E, B)
    with pytest.raises(J.JefiError):
        J.jefi_eval_fields(p.src, h, p.dt, p.nt, p.obs, p.t, E, B,
                           J.jefi_options_default(precision=J.JEFI_PREC_F64))
    torch.cuda.synchronize()
    assert bool((E == 7.0).all()) and bool((B == 7.0).all())


def test_ring_wraparound_matches_fresh_upload():
    """Pushing past the capacity overwrites the oldest slots; evaluating the
    last nt steps of a wrapped ring equals a ring holding just those steps."""
    import torch
    import paper_2104_05426_amd as J
    G = _gpu()
    src = centred_grid((9, 7, 6), 0.05)
    obs = src.shifted_cells(4, -2, 1)
    dt = 0.025
    total, cap, nt = 75, 32, 30
    blobs = [Blob(0.7, 0.08, (0.02, 0.0, -0.03), (0.4, 0.2, 0.0))]
    hall = blob_history(src, blobs, total, dt)
    store, h = J.upload_history(src, hall, J.JEFI_F32, capacity=cap)
    assert h.newest == total - 1
    E = torch.empty((3, obs.size), device="cuda")
    B = torch.empty((3, obs.size), device="cuda")
    t = (total - 1) * dt
    J.jefi_eval_fields(src, h, dt, nt, obs, t, E, B)
    torch.cuda.synchronize()
    p = Problem("wrap", src, obs, hall[total - nt:], dt, t, 0.0, total - 1, 1.0, workloads.default_screen(src))
    Er, Br = oracle.eval_problem(p)
    _assert_fields(E.double().cpu().numpy(), B.double().cpu().numpy(), Er, Br, TOL["f32"], "wrap")
    Eg2, Bg2 = G.gpu_eval(p, "f32")
    assert np.array_equal(Eg2, E.double().cpu().numpy()) and np.array_equal(Bg2, B.double().cpu().numpy())


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_wrapped_rings_give_identical_fields(prec):
    """A wavefront stages its raw slices through one scalar offset when they
    lie in 0..nt-1 in consecutive ring slots, and slot by slot with the wrap
    otherwise. Rings whose oldest used slice sits at many different slots
    (capacity nt and nt + 7) give, bit for bit, the fields of a ring that
    holds just the used slices from slot 0, at the newest time, inside the
    window and before its start."""
    import torch
    import paper_2104_05426_amd as J
    _gpu()
    src = centred_grid((10, 8, 6), 0.05)
    obs = src.shifted_cells(6, -1, 2)  # near and far bricks
    dt, nt = 0.025, 40
    blobs = [Blob(0.7, 0.08, (0.02, 0.0, -0.03), (0.4, 0.2, 0.0)), Blob(-0.4, 0.12, (0.1, 0.05, 0.0), (0.0, -0.3, 0.2))]
    hall = blob_history(src, blobs, nt + 2 * (nt + 7), dt)
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)

    def fields(h, t):
        E = torch.empty((3, obs.size), dtype=tdt, device="cuda")
        B = torch.empty((3, obs.size), dtype=tdt, device="cuda")
        J.jefi_eval_fields(src, h, dt, nt, obs, t, E, B, opt)
        torch.cuda.synchronize()
        return E.cpu().numpy(), B.cpu().numpy()

    checked = 0
    for cap in (nt, nt + 7):
        for extra in (0, 1, 5, 13, cap - 1, cap + 3, 2 * cap - 2):
            total = nt + extra
            ring_store, ring = J.upload_history(src, hall[:total], hdt, capacity=cap)
            ref_store, ref = J.upload_history(src, hall[total - nt:total], hdt, newest=total - 1, capacity=nt)
            for back in (0.0, 7.3, nt - 0.5, nt + 2.0):
                t = (total - 1 - back) * dt
                Ew, Bw = fields(ring, t)
                Er, Br = fields(ref, t)
                assert np.array_equal(Ew, Er) and np.array_equal(Bw, Br), (prec, cap, extra, back)
                checked += 1
            del ring_store, ref_store
    assert checked == 2 * 7 * 4


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_ring_above_2gib_matches_small_ring(prec):
    """A ring of more than 2 GiB (64-bit staging addresses) gives exactly
    the fields of a ring holding only the used steps (32-bit buffer
    addressing), and the oracle's on sampled points."""
    import torch
    import paper_2104_05426_amd as J
    G = _gpu()
    src = centred_grid((64, 64, 64), 0.025)
    obs = Grid((8, 8, 8), tuple(src.origin[a] + (28 + (8 if a == 0 else 0)) * 0.025 for a in range(3)),
               (0.025, 0.025, 0.025))
    dt, total, nt = 0.0125, 14, 12
    blobs = workloads.draw_blobs(np.random.default_rng(21), 6, (-0.8, 0.8))
    hall = blob_history(src, blobs, total, dt)
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    cap = 600 if prec == "f32" else 300
    assert J.jefi_history_bytes(src, cap, hdt) > (1 << 31)
    t = (total - 1) * dt
    outs = []
    for capacity in (cap, nt):
        store, h = J.upload_history(src, hall[total - nt:], hdt, newest=total - 1, capacity=capacity)
        tdt = torch.float64 if prec == "f64" else torch.float32
        E = torch.empty((3, obs.size), dtype=tdt, device="cuda")
        B = torch.empty((3, obs.size), dtype=tdt, device="cuda")
        opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
        J.jefi_eval_fields(src, h, dt, nt, obs, t, E, B, opt)
        torch.cuda.synchronize()
        outs.append((E.double().cpu().numpy(), B.double().cpu().numpy()))
        del store
        torch.cuda.empty_cache()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(obs.size, size=24, replace=False))
    p = Problem("big-ring", src, obs, hall[total - nt:], dt, t, 0.0, total - 1, 1.0, workloads.default_screen(src))
    Er, Br = oracle.eval_problem(p, sel=sel)
    _assert_fields(outs[0][0][:, sel], outs[0][1][:, sel], Er, Br, TOL[prec], f"ring > 2 GiB {prec}")


def test_history_below_fp32_range():
    """Sources of order 1e-60 (a blob far outside a small box): the FP64
    path matches the oracle; the FP32 path receives an all-zero history
    after rounding and returns exactly the fields of those inputs, zero."""
    G = _gpu()
    p0 = workloads.config_tiny()
    hist = 1e-60 * np.random.default_rng(4).normal(size=p0.hist.shape)
    p = Problem("tiny-1e-60", p0.src, p0.obs, hist, p0.dt, p0.t, p0.t0, p0.newest, p0.c, p0.screen)
    Er, Br = oracle.eval_problem(p)
    assert 0.0 < np.abs(Er).max() < 1e-50
    Eg, Bg = G.gpu_eval(p, "f64")
    _assert_fields(Eg, Bg, Er, Br, TOL["f64"], "1e-60 sources f64")
    assert not np.any(hist.astype(np.float32))
    Eg, Bg = G.gpu_eval(p, "f32")
    assert np.all(Eg == 0.0) and np.all(Bg == 0.0)


def test_deterministic_repeat():
    G = _gpu()
    p = _medium()
    for prec in ["f64", "f32"]:
        a = G.gpu_eval(p, prec)
        b = G.gpu_eval(p, prec)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
