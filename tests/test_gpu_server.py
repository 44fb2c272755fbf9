"""Serving loop on the GPU: every request's result equals the same
evaluation run alone (a fresh ring holding that session's window, one
jefi_eval_fields launch), also when the arena is too small for all sessions
and sessions are evicted and brought back; bad requests fail cleanly."""
import math
import time

import numpy as np
import pytest

import oracle
import workloads
from oracle.compare import check_fields
from workloads import Grid, Problem, blob_history, centred_grid

pytestmark = pytest.mark.gpu

SOLO_TOL = {"f32": 2e-6, "f64": 1e-13}    # batched vs alone (different split sums)
ORACLE_TOL = {"f32": 1e-5, "f64": 1e-12}


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_05426_amd as J
    return J


def _sessions(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        es = int(rng.integers(5, 17))
        dx = 1.6 / es
        cap = 2 * es + 8
        window = cap
        blobs = workloads.draw_blobs(rng, int(rng.integers(1, 6)), (-0.8, 0.8))
        src = centred_grid((es, es, es), dx)
        out.append(dict(id=100 + s, src=src, dx=dx, dt=dx / 2, cap=cap, window=window, blobs=blobs))
    return out


def _obs_for(sess, rng):
    eo = int(rng.integers(3, 19))
    dx = sess["dx"]
    m = (sess["src"].n[0] - eo) // 2
    return Grid((eo, eo, eo), tuple(sess["src"].origin[a] + m * dx for a in range(3)), (dx, dx, dx))


def _solo(J, src, hist_window, dt, newest, obs, t, prec="f32", flags=0):
    """One evaluation alone: a ring holding exactly the window."""
    import torch
    f64 = prec == "f64"
    store, h = J.upload_history(src, hist_window, J.JEFI_F64 if f64 else J.JEFI_F32, t0=0.0, newest=newest)
    E = torch.empty((3, max(obs.size, 1)), dtype=torch.float64 if f64 else torch.float32, device="cuda")
    B = torch.empty_like(E)
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if f64 else J.JEFI_PREC_F32_COMP)
    opt.flags = flags
    J.jefi_eval_fields(src, h, dt, hist_window.shape[0], obs, t, E[:, :obs.size], B[:, :obs.size], opt)
    torch.cuda.synchronize()
    return E[:, :obs.size].double().cpu().numpy(), B[:, :obs.size].double().cpu().numpy()


def _run_stream(J, arena_bytes, n_sessions, n_req, seed, init_steps=6, prec="f32", max_inflight=2,
                blocker=False, flags=0, reserve_cus=0, express_pairs=0):
    """n_req requests over n_sessions sessions, submitted back to back.
    blocker: first submit one large request of an extra session, so that
    (with max_inflight = 1) the others queue up behind it and are batched."""
    import torch
    rng = np.random.default_rng(seed)
    sess = _sessions(n_sessions, seed)
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")
    f64 = prec == "f64"
    ndt = np.float64 if f64 else np.float32
    sv = J.Server(arena, precision=J.JEFI_PREC_F64 if f64 else J.JEFI_PREC_F32_COMP, max_inflight=max_inflight,
                  max_batch=64, flags=flags, reserve_cus=reserve_cus, express_pairs=express_pairs)
    if blocker:
        bsrc = centred_grid((48, 48, 48), 1.6 / 48)
        bh = blob_history(bsrc, workloads.draw_blobs(np.random.default_rng(1), 3, (-0.8, 0.8)), 8, 0.8 / 48)
        sv.open_session(1, bsrc, 8, 8, 0.0, 0.8 / 48, bh.astype(ndt))
        bobs = centred_grid((64, 64, 64), 1.6 / 48)
        bE = np.empty((3, bobs.size), ndt)
        bB = np.empty((3, bobs.size), ndt)
        st, btk = sv.submit(1, bobs, bE, bB)
        assert st == J.JEFI_OK
    full = {}
    for s in sess:
        steps = init_steps + n_req  # enough slices for every push
        full[s["id"]] = blob_history(s["src"], s["blobs"], steps, s["dt"])
        sv.open_session(s["id"], s["src"], s["cap"], s["window"], 0.0, s["dt"],
                        full[s["id"]][:init_steps].astype(ndt))
    newest = {s["id"]: init_steps - 1 for s in sess}
    reqs = []
    for q in range(n_req):
        s = sess[int(rng.integers(0, n_sessions))]
        sid = s["id"]
        newest[sid] += 1
        obs = _obs_for(s, rng)
        E = np.full((3, obs.size), np.nan, dtype=ndt)
        B = np.full((3, obs.size), np.nan, dtype=ndt)
        st, tk = sv.submit(sid, obs, E, B, new_slice=full[sid][newest[sid]].astype(ndt))
        assert st == J.JEFI_OK, J.jefi_last_error()
        reqs.append(dict(ticket=tk, sid=sid, newest=newest[sid], obs=obs, E=E, B=B, s=s))
    results = []
    if blocker:
        st, res = sv.wait(btk)
        assert st == J.JEFI_OK and res.status == J.JEFI_OK
    for r in reqs:
        st, res = sv.wait(r["ticket"])
        assert st == J.JEFI_OK and res.status == J.JEFI_OK, (st, res.status)
        results.append(res)
    stats = sv.stats()
    assert sv.destroy() == J.JEFI_OK
    return reqs, results, stats, full


def _check_solo(J, reqs, full, n_oracle=4, prec="f32", flags=0):
    rng = np.random.default_rng(1)
    for i, r in enumerate(reqs):
        s = r["s"]
        nt = min(s["window"], r["newest"] + 1)
        window = full[r["sid"]][r["newest"] - nt + 1:r["newest"] + 1]
        if prec == "f32":
            window = window.astype(np.float32).astype(np.float64)
        t = r["newest"] * s["dt"]
        Es, Bs = _solo(J, s["src"], window, s["dt"], r["newest"], r["obs"], t, prec, flags)
        check_fields(r["E"], r["B"], Es, Bs, SOLO_TOL[prec], f"served #{i} vs solo" if i < 4 else "")
        if i < n_oracle:
            p = Problem("srv", s["src"], r["obs"], window, s["dt"], t, 0.0, r["newest"], 1.0,
                        workloads.default_screen(s["src"]))
            # library stencil flags 4, 8, 16, 32 -> oracle stencil bits 1, 2, 4, 8
            Er, Br = oracle.eval_problem(p, stencil=(flags >> 2) & 15)
            check_fields(r["E"], r["B"], Er, Br, ORACLE_TOL[prec], f"served #{i} vs oracle")


def test_server_results_equal_solo_in_the_mix():
    """Requests queued behind a large one are batched together (one stream
    slot), and each result equals the same evaluation alone."""
    J = _gpu()
    reqs, results, stats, full = _run_stream(J, 1 << 30, n_sessions=6, n_req=60, seed=3, max_inflight=1,
                                             blocker=True)
    assert stats["completed"] == 61 and stats["failed"] == 0
    print(f"server: {stats['batches']} batches, largest {stats['max_batch']}", flush=True)
    assert max(r.batch_size for r in results) > 1
    for r in results:
        assert r.t_submit_ns <= r.t_admit_ns <= r.t_start_ns <= r.t_done_ns
    _check_solo(J, reqs, full)


def test_server_overlapping_batches_keep_session_order():
    """Several batches in flight on different streams, with later requests of
    a session admitted while its earlier ones still run (stream-ordered by
    events): every result equals the same evaluation alone."""
    J = _gpu()
    reqs, results, stats, full = _run_stream(J, 1 << 30, n_sessions=3, n_req=45, seed=13, max_inflight=4)
    assert stats["completed"] == 45 and stats["failed"] == 0
    _check_solo(J, reqs, full, n_oracle=2)


def test_server_fp64_results_equal_solo():
    """The server in FP64: FP64 rings, FP64 outputs, each result equal to
    the same FP64 evaluation alone and to the oracle."""
    J = _gpu()
    reqs, results, stats, full = _run_stream(J, 1 << 30, n_sessions=4, n_req=24, seed=8, prec="f64")
    assert stats["completed"] == 24 and stats["failed"] == 0
    _check_solo(J, reqs, full, n_oracle=3, prec="f64")


def test_server_with_cu_reserve():
    """Three batches in flight whose launches leave 32 compute units free:
    every result equals the same evaluation alone."""
    J = _gpu()
    reqs, results, stats, full = _run_stream(J, 1 << 30, n_sessions=5, n_req=24, seed=17, max_inflight=3,
                                             reserve_cus=32)
    assert stats["completed"] == 24 and stats["failed"] == 0
    _check_solo(J, reqs, full, n_oracle=2)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_server_express_lane(prec):
    """Small requests in an express lane (a stream on a few reserved compute
    units), large ones behind a blocker in the regular lane, sessions mixing
    both: every result equals the same evaluation alone and the oracle."""
    J = _gpu()
    reqs, results, stats, full = _run_stream(J, 1 << 30, n_sessions=5, n_req=40, seed=21, prec=prec,
                                             max_inflight=1, blocker=True, express_pairs=200000)
    assert stats["completed"] == 41 and stats["failed"] == 0
    assert 1 <= stats["express_batches"] < stats["batches"], stats
    assert stats["express_cus"] == 16
    small = sum(1 for r in results if r.pairs <= 200000)
    print(f"express lane ({prec}): {small} small of {len(results)} requests, {stats['express_batches']} of "
          f"{stats['batches']} batches, CU-masked streams: {stats['cu_masked']}", flush=True)
    _check_solo(J, reqs, full, n_oracle=3, prec=prec)


@pytest.mark.parametrize("prec,reading", [("f32", "slope"), ("f64", "slope"), ("f32", "cubic"), ("f64", "cubic"),
                                          ("f32", "cut"), ("f64", "cut")])
def test_server_with_stencil_flags(prec, reading):
    """A server whose evaluations use alternative stencil readings (slope
    derivative or cubic interpolation, with the held past; or the history
    starting at the oldest slice) and the table index mode: every result
    equals the same evaluation alone with those flags, and the oracle with
    those readings."""
    J = _gpu()
    if reading == "cut":
        flags = J.JEFI_FLAG_PAST_CUT
    else:
        flags = (J.JEFI_FLAG_DERIV_SLOPE if reading == "slope" else J.JEFI_FLAG_TIME_CUBIC) | J.JEFI_FLAG_PAST_HOLD
    flags |= J.JEFI_FLAG_INDEX_TABLE if prec == "f32" else 0
    reqs, results, stats, full = _run_stream(J, 1 << 30, n_sessions=4, n_req=20, seed=12, prec=prec, flags=flags)
    assert stats["completed"] == 20 and stats["failed"] == 0
    _check_solo(J, reqs, full, n_oracle=3, prec=prec, flags=flags)


def test_server_evicts_and_rematerialises():
    """An arena that holds only a few session rings at once."""
    J = _gpu()
    sess = _sessions(6, 5)
    rings = [J.jefi_history_bytes(s["src"], s["cap"], J.JEFI_F32) for s in sess]
    shadows = [s["cap"] * 16 * s["src"].size for s in sess]  # FP32 host copies of the rings
    # room for the largest request on its own (ring, staged shadow, slice,
    # outputs), but not for every ring at once
    arena = max(rings) + max(shadows) + (512 << 10)
    assert sum(rings) > arena
    reqs, results, stats, full = _run_stream(J, arena, n_sessions=6, n_req=40, seed=5)
    print(f"evictions {stats['evictions']} rematerialisations {stats['rematerialisations']}", flush=True)
    assert stats["evictions"] > 0 and stats["rematerialisations"] > 0
    assert stats["arena_high_water"] <= arena
    _check_solo(J, reqs, full, n_oracle=2)


def test_server_rejections():
    import torch
    J = _gpu()
    arena = torch.empty(8 << 20, dtype=torch.uint8, device="cuda")
    sv = J.Server(arena)
    src = centred_grid((6, 6, 6), 0.1)
    h0 = blob_history(src, workloads.draw_blobs(np.random.default_rng(0), 2, (-0.3, 0.3)), 4, 0.05)
    sv.open_session(7, src, 12, 12, 0.0, 0.05, h0.astype(np.float32))
    obs = centred_grid((4, 4, 4), 0.1)
    E = np.zeros((3, obs.size), np.float32)
    B = np.zeros((3, obs.size), np.float32)
    st, _ = sv.submit(99, obs, E, B)
    assert st == J.JEFI_ENOENT
    big = centred_grid((200, 200, 200), 0.01)
    Eb = np.zeros((3, 1), np.float32)
    st, _ = sv.submit(7, big, Eb, Eb)
    assert st == J.JEFI_ETOOLARGE
    # a time after the newest step fails at admission
    st, tk = sv.submit(7, obs, E, B, t=10.0)
    assert st == J.JEFI_OK
    st, res = sv.wait(tk)
    assert res.status == J.JEFI_EINVAL
    # a valid request still runs afterwards
    st, tk = sv.submit(7, obs, E, B)
    st, res = sv.wait(tk)
    assert res.status == J.JEFI_OK and np.all(np.isfinite(E))
    assert sv.close_session(7) == J.JEFI_OK
    st, _ = sv.submit(7, obs, E, B)
    assert st == J.JEFI_ENOENT
    with pytest.raises(J.JefiError):
        sv.open_session(8, centred_grid((300, 300, 300), 0.01), 64, 64, 0.0, 0.005)
    assert sv.destroy() == J.JEFI_OK
