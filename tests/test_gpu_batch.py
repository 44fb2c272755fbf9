"""Batched persistent evaluation: every problem of an uneven batch gives
the same fields as its own single launch (and as the oracle on sampled
points), for both launch shapes and both precisions; graph replays agree;
instances the persistent kernel leaves out (empty, wholly-past, long
windows) still come out right; a batch split into two launch groups (one
per tile shape) and the autotuner's choices give the same fields."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.compare import check_fields
from workloads import Blob, Grid, Problem, blob_history, centred_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
SOLO = {"f64": 1e-13, "f32": 2e-6}


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import _gpu as G
    return G


def _small_batch(count=12, seed=31):
    """Uneven instances drawn like the batch workload, at sizes the oracle
    samples quickly: source edge 4..24, observation edge 3..28."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        es = int(rng.integers(4, 25))
        eo = int(rng.integers(3, 29))
        dx = 1.6 / es
        dt = dx / 2.0
        nt = 2 * es + 8
        src = centred_grid((es, es, es), dx)
        m = (es - eo) // 2
        obs = Grid((eo, eo, eo), tuple(src.origin[a] + m * dx for a in range(3)), (dx, dx, dx))
        blobs = workloads.draw_blobs(rng, int(rng.integers(1, 8)), (-0.8, 0.8))
        hist = blob_history(src, blobs, nt, dt)
        out.append(Problem(f"b{i}", src, obs, hist, dt, (nt - 1) * dt, 0.0, nt - 1, 1.0,
                           workloads.default_screen(src)))
    return out


def _check_against(results, refs, tol, label):
    for k, ((Eg, Bg), (Er, Br)) in enumerate(zip(results, refs)):
        check_fields(Eg, Bg, Er, Br, tol, f"{label} #{k}" if k < 4 else "")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("tile", [1, 2])
def test_batch_equals_solo_and_oracle(prec, tile):
    G = _gpu()
    probs = _small_batch()
    run = G.BatchRun(probs, prec)
    solo = run.run_solo(tile)
    batch = run.run_batch(tile)
    _check_against(batch, solo, SOLO[prec], f"batch vs solo {prec} tile {tile}")
    rng = np.random.default_rng(9)
    for k, p in enumerate(probs):
        sel = np.sort(rng.choice(p.obs.size, size=min(24, p.obs.size), replace=False))
        Er, Br = oracle.eval_problem(p, sel=sel)
        _check_against([(batch[k][0][:, sel], batch[k][1][:, sel])], [(Er, Br)], TOL[prec],
                       f"batch vs oracle {prec} tile {tile} #{k}")
    print(f"batch of {len(probs)} ({prec}, tile {tile}) matches solo and oracle", flush=True)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_with_wrapped_rings(prec):
    """The persistent kernel stages through the same wavefront-uniform ring
    offsets as a single launch: instances whose rings have wrapped at
    different slots give, bit for bit, the batch results of rings holding
    just their used slices."""
    import torch
    import paper_2104_05426_amd as J
    _gpu()
    rng = np.random.default_rng(57)
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
    keep, specs = [], []
    for k in range(8):
        es = int(rng.integers(6, 17))
        eo = int(rng.integers(5, 21))
        dx = 1.6 / es
        dt = dx / 2.0
        nt = 2 * es + 8
        extra = int(rng.integers(0, 3 * nt))
        cap = nt + 5 * (k % 3)
        src = centred_grid((es, es, es), dx)
        m = (es - eo) // 2
        obs = Grid((eo, eo, eo), tuple(src.origin[a] + m * dx for a in range(3)), (dx, dx, dx))
        blobs = workloads.draw_blobs(rng, int(rng.integers(1, 6)), (-0.8, 0.8))
        hall = blob_history(src, blobs, nt + extra, dt)
        specs.append((src, obs, dt, nt, extra, cap, hall))
    outs = []
    for wrapped in (True, False):
        probs = []
        res = []
        for src, obs, dt, nt, extra, cap, hall in specs:
            newest = nt + extra - 1
            if wrapped:
                st, h = J.upload_history(src, hall, hdt, capacity=cap)
            else:
                st, h = J.upload_history(src, hall[extra:], hdt, newest=newest, capacity=nt)
            assert h.newest == newest
            E = torch.empty((3, obs.size), dtype=tdt, device="cuda")
            B = torch.empty((3, obs.size), dtype=tdt, device="cuda")
            keep.append(st)
            res.append((E, B))
            probs.append(J.make_problem(src, h, dt, nt, obs, (newest - 0.35) * dt, E, B))
        J.jefi_eval_batch(probs, opt)
        torch.cuda.synchronize()
        outs.append([(E.cpu().numpy(), B.cpu().numpy()) for E, B in res])
    for k, ((Ew, Bw), (Ef, Bf)) in enumerate(zip(*outs)):
        assert np.array_equal(Ew, Ef) and np.array_equal(Bw, Bf), (prec, k)
    assert any(s[4] >= s[5] for s in specs)  # some rings did wrap


@pytest.mark.parametrize("flags", [1, 2])
def test_batch_index_modes(flags):
    """The persistent kernel in both FP32 index modes (guard band; threshold
    table for every pair) matches the single launches in the same mode."""
    G = _gpu()
    probs = _small_batch(10, seed=17)
    run = G.BatchRun(probs, "f32")
    solo = run.run_solo(1, flags)
    batch = run.run_batch(1, flags)
    _check_against(batch, solo, SOLO["f32"], f"batch vs solo flags {flags}")


def test_graph_replays_agree():
    """Several replays of the captured launch sequence, with eager work and
    synchronisations in between, each equal to the first."""
    import torch
    G = _gpu()
    probs = _small_batch(8, seed=4)
    run = G.BatchRun(probs, "f32")
    first = run.run_batch()
    for r in range(4):
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        again = run.run_batch()
        for (a, b), (c, d) in zip(first, again):
            assert np.array_equal(a, c) and np.array_equal(b, d), r
        del junk


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_cu_reserve_leaves_results_unchanged(prec):
    """A persistent launch that leaves compute units free (reserve_cus) takes
    the same items and reduces them in the same order: bitwise the same
    results as the full launch, also for a reserve beyond half the device."""
    G = _gpu()
    probs = _small_batch(10, seed=8)
    run = G.BatchRun(probs, prec)
    full = run.run_batch()
    for reserve in (32, 1024):
        part = run.run_batch(reserve_cus=reserve)
        for k, ((a, b), (c, d)) in enumerate(zip(full, part)):
            assert np.array_equal(a, c) and np.array_equal(b, d), (prec, reserve, k)


def test_batch_with_fallback_instances():
    """An empty observation grid, an evaluation time before every stencil
    and a long-window instance (dt << spacing) inside one batch."""
    G = _gpu()
    probs = _small_batch(4, seed=8)
    base = probs[0]
    probs.append(Problem("empty-obs", base.src, Grid((0, 0, 0), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)),
                         base.hist, base.dt, base.t, 0.0, base.newest, 1.0, base.screen))
    probs.append(Problem("past", base.src, base.obs, base.hist, base.dt, -5.0, 0.0, base.newest, 1.0,
                         base.screen))
    src = centred_grid((6, 5, 7), 0.1)
    dt = 0.01
    nt = 100
    hist = blob_history(src, [Blob(1.0, 0.15, (0.0, 0.05, 0.0), (0.3, 0.0, 0.2))], nt, dt)
    probs.append(Problem("long-window", src, src.shifted_cells(3, 1, -2), hist, dt, (nt - 1) * dt, 0.0,
                         nt - 1, 1.0, workloads.default_screen(src)))
    run = G.BatchRun(probs, "f32")
    batch = run.run_batch()
    for k, p in enumerate(probs):
        if p.obs.size == 0:
            continue
        Er, Br = oracle.eval_problem(p)
        if p.name == "past":
            assert np.all(batch[k][0] == 0.0) and np.all(batch[k][1] == 0.0)
            continue
        _check_against([batch[k]], [(Er, Br)], TOL["f32"], p.name)


def _mixed_batch(seed=41):
    """Small instances and two with at least 32768 observation points (a
    32^3 grid of the source spacing around an 8^3 or 12^3 source), so that
    the per-problem size rule puts them in different launch groups."""
    probs = _small_batch(6, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for i, es in enumerate((8, 12)):
        dx = 1.6 / es
        dt = dx / 2.0
        nt = 2 * es + 8
        src = centred_grid((es, es, es), dx)
        obs = Grid((32, 32, 32), tuple(src.origin[a] - 12 * dx for a in range(3)), (dx, dx, dx))
        blobs = workloads.draw_blobs(rng, 4, (-0.8, 0.8))
        probs.append(Problem(f"big{i}", src, obs, blob_history(src, blobs, nt, dt), dt, (nt - 1) * dt, 0.0,
                             nt - 1, 1.0, workloads.default_screen(src)))
    return probs


def _against_oracle(batch, probs, prec, label, seed=9):
    rng = np.random.default_rng(seed)
    for k, p in enumerate(probs):
        sel = np.sort(rng.choice(p.obs.size, size=min(24, p.obs.size), replace=False))
        Er, Br = oracle.eval_problem(p, sel=sel)
        _check_against([(batch[k][0][:, sel], batch[k][1][:, sel])], [(Er, Br)], TOL[prec], f"{label} #{k}")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_mixed_tile_groups(prec):
    """tile_config 3 (size rule per problem): the large instances run with
    8x8x8 tiles and the small ones with 8x8x4, as two persistent launches of
    one batch; every instance matches its own single launch and the oracle."""
    G = _gpu()
    probs = _mixed_batch()
    run = G.BatchRun(probs, prec)
    batch = run.run_batch(3)
    solo = run.run_solo(3)
    _check_against(batch, solo, SOLO[prec], f"mixed groups vs solo {prec}")
    _against_oracle(batch, probs, prec, f"mixed groups vs oracle {prec}")
    # and the same problems with one tile for all give the same fields
    one = run.run_batch(1)
    _check_against(batch, one, SOLO[prec], f"mixed groups vs one group {prec}")


def test_autotune_single_problem():
    """One problem: every configuration it admits is timed; the packed
    result is a valid configuration, and tile_config = 0 then evaluates
    with it and matches the oracle."""
    G = _gpu()
    probs = _mixed_batch(seed=5)[-1:]
    run = G.BatchRun(probs, "f32")
    best, ms = run.J.jefi_autotune(run.problem_structs(), run.options(0), reps=1)
    tile, idx, gran = best & 3, (best >> 2) & 3, (best >> 4) & 3
    assert tile in (1, 2) and idx in (1, 2) and gran in (0, 1, 2) and ms > 0.0, best
    tuned = run.run_solo(0)
    _against_oracle(tuned, probs, "f32", "tuned single")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_autotune_batch_equals_solo_and_oracle(prec):
    """A batch: the tuner's greedy search (tile per size class, index mode,
    granularity) leaves a table under which the batch (tile_config = 0)
    equals each problem's single launch and the oracle."""
    G = _gpu()
    probs = _mixed_batch(seed=13)
    run = G.BatchRun(probs, prec)
    best, ms = run.J.jefi_autotune(run.problem_structs(), run.options(0), reps=1)
    assert best & 3 == 0 and ((best >> 2) & 3) in (0, 1, 2) and ((best >> 4) & 3) in (0, 1, 2), best
    assert ms > 0.0
    batch = run.run_batch(0)
    solo = run.run_solo(0)
    _check_against(batch, solo, SOLO[prec], f"tuned batch vs solo {prec}")
    _against_oracle(batch, probs, prec, f"tuned batch vs oracle {prec}")


def test_full_size_batch_of_the_benchmark():
    """The 64-instance batch at the benchmark's own sizes (source edges
    8..40, observation edges 8..48, histories 2 e_s + 8; 4.4e10 pairs): the
    batched FP32 and FP64 results against the per-instance FP64 path on every
    point, and against the oracle on sampled points of every instance."""
    _gpu()
    import torch
    import paper_2104_05426_amd as J
    probs = workloads.batch_instances(64, seed=3)
    outs = {}
    for prec, batched in (("f64", False), ("f64", True), ("f32", True)):
        hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
        tdt = torch.float64 if prec == "f64" else torch.float32
        opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
        rings = [J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest, capacity=p.nt) for p in probs]
        res = [(torch.empty((3, p.obs.size), dtype=tdt, device="cuda"),
                torch.empty((3, p.obs.size), dtype=tdt, device="cuda")) for p in probs]
        if batched:
            J.jefi_eval_batch([J.make_problem(p.src, h, p.dt, p.nt, p.obs, p.t, E, B)
                               for (st, h), p, (E, B) in zip(rings, probs, res)], opt)
        else:
            for (st, h), p, (E, B) in zip(rings, probs, res):
                J.jefi_eval_fields(p.src, h, p.dt, p.nt, p.obs, p.t, E, B, opt)
        torch.cuda.synchronize()
        outs[prec, batched] = [(E.double().cpu().numpy(), B.double().cpu().numpy()) for E, B in res]
        del rings, res
        torch.cuda.empty_cache()
    ref = outs["f64", False]
    for key, tol in ((("f64", True), 1e-12), (("f32", True), 1e-5)):
        for i, ((E, B), (Er, Br)) in enumerate(zip(outs[key], ref)):
            check_fields(E, B, Er, Br, tol, "" if i else f"full batch {key[0]} vs FP64 path")
    rng = np.random.default_rng(17)
    for i, p in enumerate(probs):
        sel = np.sort(rng.choice(p.obs.size, size=min(4, p.obs.size), replace=False))
        Er, Br = oracle.eval_problem(p, sel=sel)
        check_fields(ref[i][0][:, sel], ref[i][1][:, sel], Er, Br, 1e-12, "" if i else "FP64 path vs oracle")
