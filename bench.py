"""Benchmark of the Jefimenko field evaluation on one MI355X.

A step is one pass of the hot path over one time step of a time-stepping
source: push the newest rho/J slice into the resident ring (device to
device) and evaluate E and B on the observation grid at that newest time
(FP64 time prelude, tile/brick pair kernel with LDS-staged slice windows,
FP64 epilogue).  Inputs are resident in HBM before the timed region.

Workload (default): 64^3 source cells x 64^3 observation points, 128-slice
history of 100 seeded Gaussian blobs, observation grid displaced by half a
box in x.  Prints one JSON line (rank 0).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_LIVE_PAIR = 68          # algorithmic FP32 flops per live pair (FMA = 2)
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X: 256 CU x 2.4 GHz x 256 flop/clk
METRIC = "G source-obs pairs/s (FP32-comp vs FP64, same GPU) at 1e-5 rel L2; p99 latency"


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ["jefi_kernels.hip", "jefi_internal.h", "jefi_api.cpp"]:
        with open(os.path.join(ROOT, "paper_2104_05426_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload):
    """HBM bytes per FP32 launch from the committed rocprofv3 counters, or
    None when the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", f"pair_kernel_fast_f32_{workload}-64x64x64.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "`", "#")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    try:
        return int(vals["traffic_bytes_per_launch_f32"])
    except (KeyError, ValueError):
        return None


FP32_RANGE_FLOOR = 1e-30  # fields smaller than this come from FP32 inputs near or below underflow


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    import workloads
    if name == "large":
        return workloads.config_large()
    if name == "medium":
        return workloads.config_medium()
    if name == "tiny":
        return workloads.config_tiny()
    raise SystemExit(f"unknown workload {name}")


def run_path(p, extra, prec, steps, warmup, flags=0):
    """Time `steps` steps (push + eval) after `warmup`; returns a dict."""
    import torch
    import paper_2104_05426_amd as J
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP,
                                 c=p.c, screen=p.screen)
    opt.flags = flags
    store, h = J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest, capacity=p.nt)
    slices = [torch.as_tensor(extra[i], dtype=tdt).cuda().contiguous() for i in range(extra.shape[0])]
    n_obs = p.obs.size
    E = torch.empty((3, n_obs), dtype=tdt, device="cuda")  # FP64 path: FP64 outputs
    B = torch.empty((3, n_obs), dtype=tdt, device="cuda")

    def step(i, evs=None):
        if evs:
            evs[0].record()
        J.jefi_history_push(h, p.src, slices[i])
        if evs:
            evs[1].record()
        t = p.t0 + h.newest * p.dt
        J.jefi_eval_fields(p.src, h, p.dt, p.nt, p.obs, t, E, B, opt)
        if evs:
            evs[2].record()

    assert warmup + steps <= len(slices)
    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        step(warmup + i, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    eval_ms = np.array([evs[i][1].elapsed_time(evs[i][2]) for i in range(steps)])
    step_ms = np.array([evs[i][0].elapsed_time(evs[i][2]) for i in range(steps)])
    # live pairs of the final state (slice decisions taken by the kernel path)
    fp = torch.zeros((n_obs, 4), dtype=torch.int64, device="cuda")
    J.jefi_slice_fingerprint(p.src, h, p.dt, p.nt, p.obs, p.t0 + h.newest * p.dt, fp, opt)
    torch.cuda.synchronize()
    live = int(fp[:, 0].sum().item())
    out = dict(wall_s=t1 - t0, eval_ms=eval_ms, step_ms=step_ms, live=live, newest=int(h.newest),
               E=E.double().cpu().numpy(), B=B.double().cpu().numpy())
    del store, slices
    return out


def run_companion(args):
    """The 32^3 x 32^3 single instance (64 slices, 20 blobs, coincident
    grids), FP32-comp against FP64 on the same GPU, reported beside the 64^3
    headline, with its parity against the oracle on sampled points."""
    import workloads
    import oracle
    from oracle.compare import max_rel_l2
    p = workloads.config_medium()
    K, W = 20, 3
    extra = workloads.blob_history(p.src, p.blobs, list(range(p.newest + 1, p.newest + 1 + W + K)), p.dt, p.t0)
    r32 = run_path(p, extra, "f32", K, W)
    r64 = run_path(p, extra, "f64", K, W)
    pairs = p.src.size * p.obs.size
    full = np.concatenate([p.hist, extra], axis=0)
    last = r32["newest"]
    win = full[last - p.nt + 1:last + 1]
    sel = np.sort(np.random.default_rng(12).choice(p.obs.size, size=32, replace=False))
    Er, Br = oracle.eval_fields(p.src, p.obs, win, p.dt, p.t0 + last * p.dt, p.t0, last, p.c, p.screen, sel=sel)
    e32 = max_rel_l2(r32["E"][:, sel], r32["B"][:, sel], Er, Br)
    e64 = max_rel_l2(r64["E"][:, sel], r64["B"][:, sel], Er, Br)
    v32 = pairs * K / r32["wall_s"] / 1e9
    v64 = pairs * K / r64["wall_s"] / 1e9
    log(f"32^3 companion: f32 {v32:.1f} G pairs/s, f64 {v64:.1f} G pairs/s, parity {e32:.2e} / {e64:.2e}")
    return {"workload": p.name, "value": round(v32, 3), "unit": "G pairs/s", "steps": K,
            "ms_per_step": round(r32["wall_s"] * 1e3 / K, 4),
            "eval_ms_p50": round(float(np.percentile(r32["eval_ms"], 50)), 4),
            "eval_ms_p99": round(float(np.percentile(r32["eval_ms"], 99)), 4),
            "fp64_path": round(v64, 3), "fp32_over_fp64": round(v32 / v64, 3),
            "parity": {"max_rel_l2_f32": float(f"{e32:.3e}"), "max_rel_l2_f64": float(f"{e64:.3e}"),
                       "ok": bool(e32 <= 1e-5 and e64 <= 1e-12)}}


def batch_measure(K, W, tune=True):
    """64 uneven instances: one push per instance and one batched persistent
    evaluation per step, against one launch per instance, in FP32 and FP64;
    with the size heuristic's launch shapes and, after one jefi_autotune
    call on the batch, with the tuned ones."""
    import torch
    import workloads
    import oracle
    import paper_2104_05426_amd as J
    from oracle.compare import max_rel_l2
    probs = workloads.batch_instances(64, seed=3)
    pairs = sum(p.pairs for p in probs)
    log(f"batch: {len(probs)} instances, {pairs:.3e} pairs per evaluation")
    extras = [workloads.blob_history(p.src, p.blobs, list(range(p.newest + 1, p.newest + 1 + W + K)), p.dt)
              for p in probs]

    def setup(prec):
        hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
        tdt = torch.float64 if prec == "f64" else torch.float32
        rings = [J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest, capacity=p.nt) for p in probs]
        sl = [[torch.as_tensor(x[i], dtype=tdt).cuda() for i in range(x.shape[0])] for x in extras]
        # outputs in the path's own precision (FP64 results are not rounded to FP32)
        outs = [(torch.empty((3, p.obs.size), dtype=tdt, device="cuda"),
                 torch.empty((3, p.obs.size), dtype=tdt, device="cuda")) for p in probs]
        opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
        return rings, sl, outs, opt

    def problems(rings, outs):
        return [J.make_problem(p.src, h, p.dt, p.nt, p.obs, p.t0 + h.newest * p.dt, E, B)
                for (st, h), p, (E, B) in zip(rings, probs, outs)]

    def timed(prec, batched, steps, do_tune=False):
        rings, sl, outs, opt = setup(prec)
        if do_tune:
            # the tuner times candidate shapes on the batch as it stands (its
            # runs leave the rings unchanged), then the same steps as the others
            best = J.jefi_autotune(problems(rings, outs), opt, reps=3)
            log(f"autotune {prec}: {best}")

        def step(i):
            for (st, h), p, x in zip(rings, probs, sl):
                J.jefi_history_push(h, p.src, x[i])
            if batched:
                J.jefi_eval_batch(problems(rings, outs), opt)
            else:
                for (st, h), p, (E, B) in zip(rings, probs, outs):
                    J.jefi_eval_fields(p.src, h, p.dt, p.nt, p.obs, p.t0 + h.newest * p.dt, E, B, opt)
        for i in range(W):
            step(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(W + i)
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t0
        res = [(E.double().cpu().numpy(), B.double().cpu().numpy()) for E, B in outs]
        newest = [h.newest for st, h in rings]
        del rings, sl, outs
        return dt_ / steps, res, newest

    tb, res_b, newest = timed("f32", True, K)
    log(f"batched f32: {tb*1e3:.2f} ms/step")
    ts, res_s, _ = timed("f32", False, K)
    log(f"per-instance f32: {ts*1e3:.2f} ms/step")
    t64, res_64, _ = timed("f64", False, K)  # same steps: same newest slice as the FP32 runs
    log(f"per-instance f64: {t64*1e3:.2f} ms/step")
    t64b, res_64b, _ = timed("f64", True, K)
    log(f"batched f64: {t64b*1e3:.2f} ms/step")
    out = {}
    if tune:
        tt, res_t, _ = timed("f32", True, K, do_tune=True)
        log(f"batched f32 (tuned shapes): {tt*1e3:.2f} ms/step")
        worst_t = max(max_rel_l2(Et, Bt, E6, B6) for (Et, Bt), (E6, B6) in zip(res_t, res_64))
        out["batched_f32_tuned"] = {"value": round(pairs / tt / 1e9, 3), "ms_per_step": round(tt * 1e3, 3),
                                    "max_rel_l2_vs_fp64_path": float(f"{worst_t:.3e}")}
        out["tuned_over_default"] = round(tb / tt, 3)
    # parity: batched FP32 against the per-instance FP64 results, batched
    # FP64 against per-instance FP64, and sampled oracle points
    worst_vs64 = max(max_rel_l2(Eb, Bb, E6, B6) for (Eb, Bb), (E6, B6) in zip(res_b, res_64))
    worst_64b = max(max_rel_l2(Eb, Bb, E6, B6) for (Eb, Bb), (E6, B6) in zip(res_64b, res_64))
    rng = np.random.default_rng(4)
    worst_or = 0.0
    for k in rng.choice(len(probs), size=6, replace=False):
        p = probs[k]
        full = np.concatenate([p.hist, extras[k]], axis=0)
        last = newest[k]
        win = full[last - p.nt + 1:last + 1]
        sel = np.sort(rng.choice(p.obs.size, size=min(16, p.obs.size), replace=False))
        Er, Br = oracle.eval_fields(p.src, p.obs, win, p.dt, p.t0 + last * p.dt, p.t0, last, p.c, p.screen, sel=sel)
        worst_or = max(worst_or, max_rel_l2(res_b[k][0][:, sel], res_b[k][1][:, sel], Er, Br))
    ok = worst_vs64 <= 1e-5 and worst_or <= 1e-5 and worst_64b <= 1e-12
    if tune:
        ok = ok and out["batched_f32_tuned"]["max_rel_l2_vs_fp64_path"] <= 1e-5
    out.update({
        "workload": "batch: 64 independent problems, source edge {8..40}, observation edge {8..48}, "
                    "history 2 e_s + 8, 1-30 Gaussian blobs each; one slice pushed per instance and one "
                    "persistent batched launch per step",
        "pairs_per_step": pairs, "steps": K, "warmup": W,
        "batched_f32": {"value": round(pairs / tb / 1e9, 3), "ms_per_step": round(tb * 1e3, 3)},
        "per_instance_f32": {"value": round(pairs / ts / 1e9, 3), "ms_per_step": round(ts * 1e3, 3)},
        "batched_f64": {"value": round(pairs / t64b / 1e9, 3), "ms_per_step": round(t64b * 1e3, 3)},
        "per_instance_f64": {"value": round(pairs / t64 / 1e9, 3), "ms_per_step": round(t64 * 1e3, 3)},
        "batched_over_per_instance_f32": round(ts / tb, 3),
        "batched_over_per_instance_f64": round(t64 / t64b, 3),
        "parity": {"max_rel_l2_batched_f32_vs_fp64_path": float(f"{worst_vs64:.3e}"),
                   "max_rel_l2_batched_f64_vs_fp64_path": float(f"{worst_64b:.3e}"),
                   "max_rel_l2_vs_oracle_sampled": float(f"{worst_or:.3e}"), "tol": 1e-5, "tol_f64": 1e-12,
                   "ok": bool(ok)},
    })
    return out


def run_batch_workload(args):
    b = batch_measure(args.steps, args.warmup, tune=not args.no_tune)
    return {
        "metric": METRIC, "value": b["batched_f32"]["value"], "unit": "G pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["batched_f32"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": b["workload"], "pairs_per_step": b["pairs_per_step"]},
        **{k: v for k, v in b.items() if k not in ("workload", "pairs_per_step", "steps", "warmup")},
    }


def serve_measure(seconds, inflight, reserve_cus, small_arena_bytes=1 << 30, express_pairs=0, express_cus=16):
    """Poisson request stream over 128 sessions through the serving loop:
    real-time replay for latency, back to back for throughput, back to back
    again in a small arena that cannot hold every session (admission by
    budget, eviction and re-materialisation); and the same requests as one
    launch per request, FP64 and FP32."""
    import threading
    import torch
    import workloads
    import oracle
    import paper_2104_05426_amd as J
    from oracle.compare import max_rel_l2
    specs, reqs = workloads.serving_trace(rate=200.0, duration=seconds, sessions=128, seed=5)
    log(f"serve: {len(reqs)} requests over {seconds:.0f} s, {len(specs)} sessions")
    grids, hist0, slices, obs_of = {}, {}, [], []
    next_step = {}
    for sp in specs:
        es, dx = sp["edge"], sp["dx"]
        grids[sp["session"]] = workloads.centred_grid((es, es, es), dx)
        hist0[sp["session"]] = workloads.blob_history(grids[sp["session"]], sp["blobs"], sp["capacity"], sp["dt"])
        next_step[sp["session"]] = sp["capacity"]
    steps_of = []
    for r in reqs:
        sp = specs[r["session"]]
        g = grids[r["session"]]
        st = next_step[r["session"]]
        next_step[r["session"]] += 1
        steps_of.append(st)
        slices.append(workloads.blob_history(g, sp["blobs"], [st], sp["dt"])[0])
        eo = r["obs_edge"]
        m = (sp["edge"] - eo) // 2
        obs_of.append(workloads.Grid((eo, eo, eo), tuple(g.origin[a] + m * sp["dx"] for a in range(3)),
                                     (sp["dx"],) * 3))
    pairs = np.array([grids[r["session"]].size * obs_of[i].size for i, r in enumerate(reqs)], dtype=np.float64)
    total_pairs = float(pairs.sum())
    ring_bytes = sum(J.jefi_history_bytes(grids[sp["session"]], sp["capacity"], J.JEFI_F32) for sp in specs)
    log(f"serve: inputs ready, {total_pairs:.3e} pairs in total, rings {ring_bytes/1e9:.2f} GB (FP32)")
    rng_s = np.random.default_rng(6)
    keep_fp64 = set(range(0, len(reqs), max(1, len(reqs) // 200)))
    keep_oracle = set(int(v) for v in rng_s.choice(len(reqs), size=4, replace=False))
    keep = keep_fp64 | keep_oracle
    free = torch.cuda.mem_get_info()[0]
    arena_bytes = int(min(200e9, 0.6 * free))

    def serve(paced, arena_size, express=True):
        arena = torch.empty(arena_size, dtype=torch.uint8, device="cuda")
        sv = J.Server(arena, precision=J.JEFI_PREC_F32_COMP, max_inflight=inflight, max_batch=256,
                      reserve_cus=reserve_cus, express_pairs=int(express_pairs) if express else 0,
                      express_cus=express_cus)
        for sp in specs:
            sv.open_session(sp["session"], grids[sp["session"]], sp["capacity"], sp["capacity"], 0.0, sp["dt"],
                            hist0[sp["session"]].astype(np.float32))
        outs = [None] * len(reqs)
        tickets = [None] * len(reqs)
        lat = np.zeros(len(reqs))
        bsz = np.zeros(len(reqs))
        done_evt = threading.Event()

        def waiter():
            for i in range(len(reqs)):
                while tickets[i] is None:
                    time.sleep(0.0002)
                st, res = sv.wait(tickets[i])
                assert res.status == J.JEFI_OK, (i, res.status)
                lat[i] = (res.t_done_ns - res.t_submit_ns) / 1e6
                bsz[i] = res.batch_size
                if i not in keep:
                    outs[i] = None
            done_evt.set()

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            if paced:
                delay = r["arrival"] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            E = np.empty((3, obs_of[i].size), np.float32)
            B = np.empty((3, obs_of[i].size), np.float32)
            outs[i] = (E, B)
            while True:
                st, tk = sv.submit(r["session"], obs_of[i], E, B, new_slice=slices[i].astype(np.float32))
                if st != J.JEFI_EBUSY:
                    break
                time.sleep(0.0005)
            assert st == J.JEFI_OK, (i, st, J.jefi_last_error())
            tickets[i] = tk
            if i % 2000 == 0:
                log(f"  submitted {i}")
        done_evt.wait()
        wall = time.perf_counter() - t0
        th.join()
        stats = sv.stats()
        sv.destroy()
        del arena
        return wall, lat, bsz, outs, stats

    def lat_summary(lat):
        return {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                "max": round(float(lat.max()), 3)}

    wall_p, lat_p, bsz_p, outs_p, stats_p = serve(True, arena_bytes)
    log(f"paced: {len(reqs)/wall_p:.1f} req/s, p50 {np.percentile(lat_p, 50):.2f} ms p99 {np.percentile(lat_p, 99):.2f} ms")
    # paced latency by request size (source cells x observation points, quartiles)
    cls = np.digitize(pairs, np.quantile(pairs, [0.25, 0.5, 0.75]))
    by_size = []
    for q in range(4):
        m = cls == q
        if m.any():
            by_size.append({"pairs_median": float(f"{np.median(pairs[m]):.3e}"), "requests": int(m.sum()),
                            "p50": round(float(np.percentile(lat_p[m], 50)), 3),
                            "p99": round(float(np.percentile(lat_p[m], 99)), 3)})
    log("paced latency by size quartile: " + ", ".join(f"{d['pairs_median']:.1e} pairs p50 {d['p50']} p99 {d['p99']} ms"
                                                      for d in by_size))
    wall_o, lat_o, bsz_o, outs_o, stats_o = serve(False, arena_bytes)
    log(f"back-to-back: {len(reqs)/wall_o:.1f} req/s")
    if express_pairs > 0:
        # the same stream without the express lane: what the lane costs in throughput
        wall_n, lat_n, bsz_n, outs_n, stats_n = serve(False, arena_bytes, express=False)
        log(f"back-to-back without the express lane: {len(reqs)/wall_n:.1f} req/s")
    wall_s, lat_s, bsz_s, outs_s, stats_s = serve(False, small_arena_bytes)
    log(f"back-to-back, {small_arena_bytes/2**30:.1f} GiB arena: {len(reqs)/wall_s:.1f} req/s, "
        f"{stats_s['evictions']} evictions, {stats_s['rematerialisations']} re-materialisations")

    def one_launch_per_request(prec):
        hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
        tdt = torch.float64 if prec == "f64" else torch.float32
        rings = {}
        for sp in specs:
            rings[sp["session"]] = J.upload_history(grids[sp["session"]], hist0[sp["session"]], hdt,
                                                    capacity=sp["capacity"])
        opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            sp = specs[r["session"]]
            store, h = rings[r["session"]]
            g = grids[r["session"]]
            J.jefi_history_push(h, g, torch.as_tensor(slices[i], dtype=tdt).cuda())
            E = torch.empty((3, obs_of[i].size), dtype=tdt, device="cuda")
            B = torch.empty_like(E)
            J.jefi_eval_fields(g, h, sp["dt"], sp["capacity"], obs_of[i], h.newest * sp["dt"], E, B, opt)
            out = (E.cpu().numpy(), B.cpu().numpy())  # copy back + sync, as a client would
            res.append(out if i in keep else None)
            if i % 4000 == 0:
                log(f"  {prec} one launch per request: {i}")
        wall = time.perf_counter() - t0
        del rings
        return wall, res

    wall64, res64 = one_launch_per_request("f64")
    log(f"fp64 one-launch-per-request: {len(reqs)/wall64:.1f} req/s")
    wall32, res32 = one_launch_per_request("f32")
    log(f"fp32 one-launch-per-request: {len(reqs)/wall32:.1f} req/s")
    # Sessions whose blobs have drifted far from their box have fields below
    # FP32 range (their FP32 history rounds to zero): relative errors there
    # say nothing about arithmetic, so they are counted and left out.
    below = sum(1 for i in keep_fp64 if max(np.abs(res64[i][0]).max(initial=0.0),
                                             np.abs(res64[i][1]).max(initial=0.0)) < FP32_RANGE_FLOOR)

    def worst_vs64(outs):
        w = 0.0
        for i in sorted(keep_fp64):
            if max(np.abs(res64[i][0]).max(initial=0.0), np.abs(res64[i][1]).max(initial=0.0)) < FP32_RANGE_FLOOR:
                continue
            w = max(w, max_rel_l2(np.asarray(outs[i][0], np.float64), np.asarray(outs[i][1], np.float64),
                                  res64[i][0], res64[i][1]))
        return w
    worst_p, worst_s, worst_32 = worst_vs64(outs_p), worst_vs64(outs_s), worst_vs64(res32)
    # a few requests against the oracle
    worst_or = 0.0
    rng = np.random.default_rng(7)
    for i in sorted(keep_oracle):
        r = reqs[i]
        sp = specs[r["session"]]
        g = grids[r["session"]]
        cap = sp["capacity"]
        st = steps_of[i]
        win = workloads.blob_history(g, sp["blobs"], list(range(st - cap + 1, st + 1)), sp["dt"])
        sel = np.sort(rng.choice(obs_of[i].size, size=min(16, obs_of[i].size), replace=False))
        Er, Br = oracle.eval_fields(g, obs_of[i], win, sp["dt"], st * sp["dt"], 0.0, st, 1.0, None, sel=sel)
        if max(np.abs(Er).max(initial=0.0), np.abs(Br).max(initial=0.0)) < FP32_RANGE_FLOOR:
            below += 1
            continue
        worst_or = max(worst_or, max_rel_l2(outs_p[i][0][:, sel].astype(np.float64),
                                            outs_p[i][1][:, sel].astype(np.float64), Er, Br))
    return {
        "workload": f"serve: Poisson 200 req/s for {seconds:.0f} s over 128 sessions (source edge log-U[8,48], "
                    "observation edge log-U[8,64], ring 2 e_s + 8, one new slice per request), "
                    "FP32-compensated, HBM arena budget "
                    f"{arena_bytes/1e9:.0f} GB (a second back-to-back run in {small_arena_bytes/2**30:.0f} GiB)",
        "requests": len(reqs), "pairs": total_pairs, "session_rings_gb": round(ring_bytes / 1e9, 3),
        "batches_in_flight": inflight, "reserve_cus": reserve_cus,
        "express_lane": ({"max_pairs": express_pairs, "cus": stats_p["express_cus"],
                          "cu_masked_streams": bool(stats_p["cu_masked"]),
                          "paced_express_batches": stats_p["express_batches"],
                          "back_to_back_without_it": {"req_per_s": round(len(reqs) / wall_n, 2),
                                                      "value": round(total_pairs / wall_n / 1e9, 3)},
                          "back_to_back_with_over_without": round(wall_n / wall_o, 3)}
                         if express_pairs > 0 else None),
        "paced": {"req_per_s": round(len(reqs) / wall_p, 2), "latency_ms": lat_summary(lat_p),
                  "mean_batch": round(float(bsz_p.mean()), 2), "batches": stats_p["batches"],
                  "latency_ms_by_size_quartile": by_size},
        "back_to_back": {"req_per_s": round(len(reqs) / wall_o, 2), "value": round(total_pairs / wall_o / 1e9, 3),
                         "unit": "G pairs/s", "latency_ms": lat_summary(lat_o),
                         "mean_batch": round(float(bsz_o.mean()), 2)},
        "small_arena": {"arena_gb": round(small_arena_bytes / 1e9, 3), "req_per_s": round(len(reqs) / wall_s, 2),
                        "value": round(total_pairs / wall_s / 1e9, 3), "latency_ms": lat_summary(lat_s),
                        "evictions": stats_s["evictions"], "rematerialisations": stats_s["rematerialisations"],
                        "max_rel_l2_vs_fp64_sampled": float(f"{worst_s:.3e}")},
        "fp64_one_launch_per_request": {"req_per_s": round(len(reqs) / wall64, 2),
                                        "value": round(total_pairs / wall64 / 1e9, 3)},
        "fp32_one_launch_per_request": {"req_per_s": round(len(reqs) / wall32, 2),
                                        "value": round(total_pairs / wall32 / 1e9, 3),
                                        "max_rel_l2_vs_fp64_sampled": float(f"{worst_32:.3e}")},
        "server_over_fp64_one_launch_per_request": round(wall64 / wall_o, 3),
        "server_over_fp32_one_launch_per_request": round(wall32 / wall_o, 3),
        "parity": {"max_rel_l2_vs_fp64_sampled": float(f"{worst_p:.3e}"), "sampled": len(keep),
                   "sampled_below_fp32_range": below,
                   "max_rel_l2_vs_oracle_sampled": float(f"{worst_or:.3e}"), "tol": 1e-5,
                   "ok": bool(max(worst_p, worst_s, worst_32, worst_or) <= 1e-5)},
    }


def run_serve_workload(args):
    sv = serve_measure(args.serve_seconds, args.serve_inflight, args.serve_reserve_cus,
                       int(args.serve_small_arena_gib * 2**30), args.serve_express_pairs, args.serve_express_cus)
    b2b = sv["back_to_back"]
    return {
        "metric": METRIC, "value": b2b["value"], "unit": "G pairs/s", "n_gpus": 1,
        "steps": sv["requests"], "warmup": 0, "ms_per_step": round(1e3 / b2b["req_per_s"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": sv["workload"], "requests": sv["requests"],
                   "batches_in_flight": sv["batches_in_flight"], "reserve_cus": sv["reserve_cus"]},
        "p99_latency_ms": sv["paced"]["latency_ms"]["p99"],
        **{k: v for k, v in sv.items() if k not in ("workload", "requests", "batches_in_flight", "reserve_cus")},
    }


def run_stencil_variants(args, p, extra):
    """The same workload under the alternative time-stencil readings (FP32
    path): derivative as the slope of the interpolant, history before the
    oldest slice held at its values (no pair culled as past), both, and
    cubic time interpolation; rate and parity against the oracle with the
    same reading on sampled points."""
    import oracle
    import paper_2104_05426_amd as J
    from oracle.compare import max_rel_l2
    K, W = 5, 2
    pairs = p.src.size * p.obs.size
    full = np.concatenate([p.hist, extra], axis=0)
    sel = np.sort(np.random.default_rng(13).choice(p.obs.size, size=8, replace=False))
    out = {}
    for name, flag, st in [("slope", J.JEFI_FLAG_DERIV_SLOPE, oracle.STENCIL_SLOPE),
                           ("hold", J.JEFI_FLAG_PAST_HOLD, oracle.STENCIL_HOLD),
                           ("slope+hold", J.JEFI_FLAG_DERIV_SLOPE | J.JEFI_FLAG_PAST_HOLD,
                            oracle.STENCIL_SLOPE | oracle.STENCIL_HOLD),
                           ("cubic", J.JEFI_FLAG_TIME_CUBIC, oracle.STENCIL_CUBIC)]:
        r = run_path(p, extra, "f32", K, W, flags=flag)
        last = r["newest"]
        win = full[last - p.nt + 1:last + 1]
        Er, Br = oracle.eval_fields(p.src, p.obs, win, p.dt, p.t0 + last * p.dt, p.t0, last, p.c, p.screen,
                                    sel=sel, stencil=st)
        err = max_rel_l2(r["E"][:, sel], r["B"][:, sel], Er, Br)
        v = pairs * K / r["wall_s"] / 1e9
        log(f"stencil {name}: {v:.1f} G pairs/s, eval {np.mean(r['eval_ms']):.2f} ms, parity {err:.2e}")
        out[name] = {"value": round(v, 3), "unit": "G pairs/s", "steps": K,
                     "eval_ms_mean": round(float(np.mean(r["eval_ms"])), 3),
                     "parity": {"sampled_points": int(len(sel)), "max_rel_l2_f32": float(f"{err:.3e}"),
                                "ok": bool(err <= 1e-5)}}
    return out


# The paper's accuracy experiments (section "Comparisons with the
# theoretical results"): 15^3 source grids of cell 0.4 over [-3, 3]^3,
# screening half-width 0.2, time step 0.05 (410 snapshots over 0 .. 20.5),
# fields compared in the XOY plane by max |(dEx, dEy)| / max |(Ex, Ey)|.
# The reference is the same discretisation refined r times in space and
# time with the screening cube held at 0.2: it converges to the continuous
# integrals with that cube left out.
ACC_CASES = {
    "constant": {"obs_z": 0.0, "times": (2.5, 5.0, 7.5)},
    "sinusoidal": {"obs_z": 13.0, "times": (14.0, 17.0, 20.0)},
}


def accuracy_fields(kind, r, times, obs_z, prec="f64", flags=0):
    """E, B [3][225] on the XOY plane at each time, from the paper's source
    on a (15 r)^3 grid with time step 0.05 / r; returns {t: (E, B)}.
    ``flags``: time-stencil reading (JEFI_FLAG_*), default the zero past."""
    import torch
    import workloads
    import paper_2104_05426_amd as J
    n, dx, dt = 15 * r, 0.4 / r, 0.05 / r
    src = workloads.Grid((n, n, n), (-3.0 + 0.5 * dx,) * 3, (dx,) * 3)
    obs = workloads.Grid((15, 15, 1), (-2.8, -2.8, obs_z), (0.4, 0.4, 0.4))
    newest = int(round(max(times) / dt))
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    tdt = torch.float64 if prec == "f64" else torch.float32
    store = torch.empty(J.jefi_history_bytes(src, newest + 1, hdt), dtype=torch.uint8, device="cuda")
    h = J.jefi_history_init(store, src, newest + 1, hdt)
    ax = [torch.arange(n, dtype=torch.float64, device="cuda") * dx + (-3.0 + 0.5 * dx)]
    zz, yy, xx = torch.meshgrid(ax[0], ax[0], ax[0], indexing="ij")
    phase = (xx + yy + zz).reshape(-1)
    if kind == "constant":
        p_rho = torch.ones_like(phase)
        p_j = torch.ones_like(phase)
    else:
        p_rho, p_j = torch.cos(phase), torch.sin(phase)
    slice_ = torch.empty((4, src.size), dtype=tdt, device="cuda")
    for k in range(newest + 1):
        a, b = workloads.paper_source_factors(kind, k * dt)
        slice_[0] = (a * p_rho).to(tdt)
        slice_[1:4] = (b * p_j).to(tdt)[None, :]
        J.jefi_history_push(h, src, slice_)
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP,
                                 screen=(0.2, 0.2, 0.2))
    opt.flags = flags
    out = {}
    for t in times:
        E = torch.empty((3, obs.size), dtype=torch.float64, device="cuda")
        B = torch.empty_like(E)
        J.jefi_eval_fields(src, h, dt, newest + 1, obs, t, E, B, opt)
        torch.cuda.synchronize()
        out[t] = (E.cpu().numpy(), B.cpu().numpy())
    del store, slice_, phase, p_rho, p_j, xx, yy, zz
    torch.cuda.empty_cache()
    return out


def xoy_deviation(x, ref):
    """max |(dx, dy)| over the plane / max |(ref_x, ref_y)| (z components
    left out, as in the paper's norms)."""
    d = np.sqrt((x[0] - ref[0]) ** 2 + (x[1] - ref[1]) ** 2).max()
    m = np.sqrt(ref[0] ** 2 + ref[1] ** 2).max()
    return float(d / m) if m > 0 else float(d)


def accuracy_study(levels=(1, 2, 4, 8), cases=ACC_CASES, ref_prec_bytes=40e9):
    """Deviations of each refinement level from the finest, per case and
    time, for E and B; the finest level runs in FP32-comp when its FP64 ring
    would exceed ref_prec_bytes."""
    import paper_2104_05426_amd as J
    import workloads
    res = {}
    for kind, cfg in cases.items():
        fields = {}
        for r in levels:
            n = 15 * r
            slots = int(round(max(cfg["times"]) / (0.05 / r))) + 1
            nbytes = J.jefi_history_bytes(workloads.Grid((n, n, n), (0.0,) * 3, (1.0,) * 3), slots, J.JEFI_F64)
            prec = "f64" if nbytes <= ref_prec_bytes else "f32"
            t0 = time.perf_counter()
            fields[r] = accuracy_fields(kind, r, cfg["times"], cfg["obs_z"], prec)
            log(f"accuracy {kind} r={r} ({n}^3, {slots} slices, {prec}): {time.perf_counter() - t0:.1f} s")
        fields["1-f32"] = accuracy_fields(kind, 1, cfg["times"], cfg["obs_z"], "f32")
        if kind == "constant":
            # the reading that leaves the switch-on shell out (history starting at t = 0)
            for r in [v for v in levels if v <= 4]:
                fields[f"cut{r}"] = accuracy_fields(kind, r, cfg["times"], cfg["obs_z"], "f64", J.JEFI_FLAG_PAST_CUT)
        top = max(levels)
        res[kind] = {}
        for t in cfg["times"]:
            ref_E, ref_B = fields[top][t]
            row = {"max_E_xy": float(np.sqrt(ref_E[0] ** 2 + ref_E[1] ** 2).max()),
                   "max_B_xy": float(np.sqrt(ref_B[0] ** 2 + ref_B[1] ** 2).max())}
            for key in [r for r in levels if r != top] + ["1-f32"]:
                E, B = fields[key][t]
                row[f"r{key}"] = {"E": round(xoy_deviation(E, ref_E), 5), "B": round(xoy_deviation(B, ref_B), 5)}
            if kind == "constant":
                row["continuum"] = continuum_deviations(fields, levels, t)
            res[kind][str(t)] = row
    return res


def continuum_deviations(fields, levels, t):
    """The constant-source sums against the continuous equations (FP64
    quadrature) in two readings: with the switch-on shell, and without it
    (the Coulomb and Biot-Savart fields of the box within distance t).  Also
    the discretised sum that leaves the switch-on derivative out (the static
    sum over the cells within distance t) against the second reading."""
    import workloads
    from tests.continuum import ball_sum_plane, switched_on_box_plane
    obs = workloads.Grid((15, 15, 1), (-2.8, -2.8, 0.0), (0.4, 0.4, 0.4))
    pts = workloads.cell_centres(obs)
    box = ((-3.0,) * 3, (3.0,) * 3)
    refs = switched_on_box_plane(pts, t, *box)
    out = {}
    for reading, (rE, rB) in refs.items():
        row = {"max_E_xy": round(float(np.sqrt(rE[0] ** 2 + rE[1] ** 2).max()), 5),
               "max_B_xy": round(float(np.sqrt(rB[0] ** 2 + rB[1] ** 2).max()), 5)}
        for r in levels:
            E, B = fields[r][t]
            row[f"r{r}"] = {"E": round(xoy_deviation(E, rE), 5), "B": round(xoy_deviation(B, rB), 5)}
        out[reading] = row
    E, B = ball_sum_plane(pts, t, *box, 0.4, 0.2)
    rE, rB = refs["no_shell"]
    out["no_shell"]["r1_without_switch_on_derivative"] = {"E": round(xoy_deviation(E, rE), 5),
                                                          "B": round(xoy_deviation(B, rB), 5)}
    # the library's history-start reading (JEFI_FLAG_PAST_CUT) against the same
    for key in sorted(k for k in fields if str(k).startswith("cut")):
        E, B = fields[key][t]
        out["no_shell"][f"{key}_history_start"] = {"E": round(xoy_deviation(E, rE), 5),
                                                   "B": round(xoy_deviation(B, rB), 5)}
    return out


def run_accuracy_workload(args):
    t0 = time.perf_counter()
    res = accuracy_study()
    wall = time.perf_counter() - t0
    worst = max(max(v["r1"]["E"], v["r1"]["B"]) for c in res.values() for v in c.values())
    log(json.dumps(res, indent=1))
    return {"metric": "max XOY-plane field deviation of the 15^3 paper configuration from a refined reference "
                      "(paper: 3 % constant, 11.2 % / 14.3 % sinusoidal)",
            "value": round(worst, 5), "unit": "fraction of max field", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": round(wall * 1e3, 1), "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic (the paper's analytic sources)",
            "config": {"workload": "accuracy: the paper's constant and sinusoidal sources on 15^3 grids over "
                                   "[-3,3]^3, screening 0.2, dt 0.05, against refinements r = 2, 4, 8 "
                                   "(cell 0.4/r, dt 0.05/r)"},
            "cases": res}


# The paper's per-step timing table (section "Parameter dependence",
# Table 4): coincident n^3 source and observation grids ("ntg" [n^3, n^3])
# with a history of lts + 1 slices; per step, one new slice goes host to
# device, the fields are evaluated, E and B come back to the host.  The
# paper's V100 figures (exec, [DToH, HToD] in s at lts 500) for context.
PAPER_TABLE4 = {20: (1.001, 0.0004, 0.002), 60: (2.720, 0.002, 0.004), 70: (4.858, 0.009, 0.005),
                100: (32.565, 0.027, 0.009), 160: (521.970, 0.060, 0.042)}


def run_paper_steps(args):
    """Per-step time at the paper's grid sizes in three couplings:
    serial (copy in, push, evaluate, copy out, as the paper times it);
    overlapped (the library's coupler: step s's E/B copy out and slice
    s+1's copy in run on copy streams while step s+1 evaluates); device
    producer (the slice is made on the device and handed to the coupler
    from there, E/B copy out overlapped)."""
    import torch
    import workloads
    import paper_2104_05426_amd as J
    lts, dt = 500, 0.05
    sizes = [20, 60, 70, 100, 160] if not args.paper_sizes else [int(v) for v in args.paper_sizes.split(",")]
    out = {}
    for n in sizes:
        dx = 6.0 / n
        g = workloads.Grid((n, n, n), (-3.0 + 0.5 * dx,) * 3, (dx,) * 3)
        ns = g.size
        ax = torch.arange(n, dtype=torch.float64, device="cuda") * dx + (-3.0 + 0.5 * dx)
        zz, yy, xx = torch.meshgrid(ax, ax, ax, indexing="ij")
        phase = (xx + yy + zz).reshape(-1)
        p_rho, p_j = torch.cos(phase).float(), torch.sin(phase).float()
        del zz, yy, xx, phase

        def make_slice(k, dst):
            a, b = workloads.paper_source_factors("sinusoidal", k * dt)
            torch.mul(p_rho, a, out=dst[0])
            torch.mul(p_j, b, out=dst[1])
            dst[2].copy_(dst[1])
            dst[3].copy_(dst[1])

        store = torch.empty(J.jefi_history_bytes(g, lts + 1, J.JEFI_F32), dtype=torch.uint8, device="cuda")
        h = J.jefi_history_init(store, g, lts + 1, J.JEFI_F32)
        dev_slice = [torch.empty((4, ns), dtype=torch.float32, device="cuda") for _ in range(2)]
        for k in range(lts + 1):
            make_slice(k, dev_slice[0])
            J.jefi_history_push(h, g, dev_slice[0])
        host_slice = [torch.empty((4, ns), dtype=torch.float32, pin_memory=True) for _ in range(2)]
        E = [torch.empty((3, ns), dtype=torch.float32, device="cuda") for _ in range(2)]
        B = [torch.empty((3, ns), dtype=torch.float32, device="cuda") for _ in range(2)]
        hE = [torch.empty((3, ns), dtype=torch.float32, pin_memory=True) for _ in range(2)]
        hB = [torch.empty((3, ns), dtype=torch.float32, pin_memory=True) for _ in range(2)]
        opt = J.jefi_options_default(precision=J.JEFI_PREC_F32_COMP)
        steps = {20: 40, 60: 8, 70: 6}.get(n, 2 if n >= 160 else 3)  # about a second or more per mode
        warm = 0 if n >= 160 else 1
        k_next = [lts + 1]

        def host_make(i):
            make_slice(k_next[0] + i, dev_slice[1])
            host_slice[i % 2].copy_(dev_slice[1])
        # serial: copy in, push, evaluate, copy out, each timed
        parts = []
        for i in range(warm + steps):
            host_make(0)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            ev[0].record()
            dev_slice[0].copy_(host_slice[0], non_blocking=True)
            ev[1].record()
            J.jefi_history_push(h, g, dev_slice[0])
            J.jefi_eval_fields(g, h, dt, lts + 1, g, h.newest * dt, E[0], B[0], opt)
            ev[2].record()
            hE[0].copy_(E[0], non_blocking=True)
            hB[0].copy_(B[0], non_blocking=True)
            ev[3].record()
            torch.cuda.synchronize()
            k_next[0] += 1
            if i >= warm:
                parts.append([ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])])
        parts = np.array(parts) / 1e3
        serial = float(parts.sum(axis=1).mean())

        def pipelined(device_producer):
            # the library's coupler: slice copy-in, push + evaluation and
            # E/B copy-out on three streams, one step in flight behind the newest
            cp = J.Coupler(g, h, dt, lts + 1, g, opt, J.JEFI_F32)
            hs = [host_slice[0].numpy(), host_slice[1].numpy()]
            oE, oB = hE[0].numpy(), hB[0].numpy()
            host_make(0)
            host_make(1)
            # untimed steps: the coupler's streams get their workspaces, both
            # staging slots their first copies
            cwarm = 1 if n >= 160 else 4
            for i in range(cwarm):
                cp.collect(cp.step(hs[i % 2]), oE, oB)
            k_next[0] += cwarm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prev = None
            for i in range(steps):
                if device_producer:
                    make_slice(k_next[0] + i, dev_slice[i % 2])   # on torch's stream
                    s = cp.step(dev_slice[i % 2], torch.cuda.current_stream())
                else:
                    s = cp.step(hs[i % 2])
                if prev is not None:
                    cp.collect(prev, oE, oB)
                prev = s
            cp.collect(prev, oE, oB)
            dt_step = (time.perf_counter() - t0) / steps
            cp.destroy()
            k_next[0] += steps
            return dt_step

        log(f"paper-steps n={n}: serial {serial:.4f} s/step")
        over = pipelined(False)
        log(f"paper-steps n={n}: overlapped {over:.4f} s/step")
        dev = pipelined(True)
        pairs = float(ns) * ns
        ref = PAPER_TABLE4.get(n)
        row = {"pairs": pairs, "exec_s": round(float(parts[:, 1].mean()), 5),
               "dtoh_s": round(float(parts[:, 2].mean()), 5), "htod_s": round(float(parts[:, 0].mean()), 5),
               "serial_step_s": round(serial, 5), "overlapped_step_s": round(over, 5),
               "device_producer_step_s": round(dev, 5),
               "exec_G_pairs_per_s": round(pairs / float(parts[:, 1].mean()) / 1e9, 2)}
        if ref:
            row["paper_v100_lts500"] = {"exec_s": ref[0], "dtoh_s": ref[1], "htod_s": ref[2]}
            row["exec_speedup_vs_paper"] = round(ref[0] / float(parts[:, 1].mean()), 1)
        log(f"paper-steps n={n}: {json.dumps(row)}")
        out[f"{n}^3"] = row
        del store, dev_slice, host_slice, E, B, hE, hB, p_rho, p_j
        torch.cuda.empty_cache()
    big = out[f"{sizes[-1]}^3"]
    return {"metric": "G source-obs pairs/s per evaluation at the paper's per-step configurations "
                      "(ntg [n^3, n^3], lts 500)", "value": big["exec_G_pairs_per_s"], "unit": "G pairs/s",
            "n_gpus": 1, "steps": 2, "warmup": 0, "ms_per_step": round(big["serial_step_s"] * 1e3, 2),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (the paper's sinusoidal source)",
            "config": {"workload": f"paper-steps: coincident n^3 grids over [-3,3]^3, n = {sizes}, lts 500, "
                                   "dt 0.05, FP32-compensated; serial / overlapped / device-producer steps"},
            "sizes": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-companion", action="store_true",
                    help="skip the 32^3 single-instance line reported beside the 64^3 headline")
    ap.add_argument("--paper-sizes", default="",
                    help="comma-separated grid edges for --workload paper-steps (default 20,60,70,100,160)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the time-stencil variants of the headline workload")
    ap.add_argument("--serve-inflight", type=int, default=2,
                    help="serve workload: batches in flight at once (server streams)")
    ap.add_argument("--serve-reserve-cus", type=int, default=0,
                    help="serve workload: compute units each batch launch leaves free for the others")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson request stream (serving block and --workload serve)")
    ap.add_argument("--serve-express-pairs", type=float, default=5e7,
                    help="serving: requests of at most this many pairs take the express lane (0 = none)")
    ap.add_argument("--serve-express-cus", type=int, default=16,
                    help="serving: compute units of the express lane")
    ap.add_argument("--serve-small-arena-gib", type=float, default=1.0,
                    help="arena of the serving run whose budget binds (sessions are evicted)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-instance batch block of the default run")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving block of the default run")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch: skip the autotuned launch shapes")
    ap.add_argument("--batch-steps", type=int, default=5,
                    help="timed steps of each batch variant in the default run")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (a known-size "
                         "reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2104_05426_amd as J  # fails loudly when libjefi.so is not built
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 4} bytes read and written")
        del a, b

    if args.workload == "batch":
        print(json.dumps(run_batch_workload(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve_workload(args)), flush=True)
        return
    if args.workload == "paper-steps":
        print(json.dumps(run_paper_steps(args)), flush=True)
        return
    if args.workload == "accuracy":
        print(json.dumps(run_accuracy_workload(args)), flush=True)
        return

    p = make_workload(args.workload)
    K, W = args.steps, args.warmup
    K64 = args.fp64_steps if args.fp64_steps is not None else max(2, K // 2)
    n_extra = max(W + max(K, K64), 7)  # the stencil variants run 2 + 5 steps
    log(f"workload {p.name}: {p.src.size} src x {p.obs.size} obs, nt {p.nt}; {n_extra} extra slices")
    extra = workloads.blob_history(p.src, p.blobs, list(range(p.newest + 1, p.newest + 1 + n_extra)), p.dt,
                                   p.t0)
    pairs = p.src.size * p.obs.size

    r32 = run_path(p, extra, "f32", K, W)
    log(f"f32: {r32['wall_s']*1e3/K:.2f} ms/step, eval {np.mean(r32['eval_ms']):.2f} ms")
    r64 = run_path(p, extra, "f64", K64, W)
    log(f"f64: {r64['wall_s']*1e3/K64:.2f} ms/step, eval {np.mean(r64['eval_ms']):.2f} ms")

    value = pairs * K / r32["wall_s"] / 1e9
    value64 = pairs * K64 / r64["wall_s"] / 1e9
    eval_s = float(np.mean(r32["eval_ms"])) / 1e3
    achieved = FLOPS_PER_LIVE_PAIR * r32["live"] / eval_s / 1e12
    res = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(r32["wall_s"] * 1e3 / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{p.name}: {p.src.n[0]}x{p.src.n[1]}x{p.src.n[2]} source cells x "
                               f"{p.obs.n[0]}x{p.obs.n[1]}x{p.obs.n[2]} observation points, {p.nt}-slice "
                               f"ring of Gaussian-blob rho/J, one slice pushed per step",
                   "n_src": p.src.size, "n_obs": p.obs.size, "nt": p.nt,
                   "precision": "FP32 pair arithmetic, compensated accumulation, canonical FP64 slice "
                                "index (threshold table or guard band), FP64 epilogue"},
        "fp64_path": {"value": round(value64, 3), "unit": "G pairs/s", "steps": K64,
                      "ms_per_step": round(r64["wall_s"] * 1e3 / K64, 3)},
        "fp32_over_fp64": round(value / value64, 3),
        "live_pairs_per_eval": r32["live"],
        "live_fraction": round(r32["live"] / pairs, 4),
        "eval_ms": {"mean": round(float(np.mean(r32["eval_ms"])), 3),
                    "p50": round(float(np.percentile(r32["eval_ms"], 50)), 3),
                    "p99": round(float(np.percentile(r32["eval_ms"], 99)), 3)},
        "step_latency_ms": {"p50": round(float(np.percentile(r32["step_ms"], 50)), 3),
                            "p99": round(float(np.percentile(r32["step_ms"], 99)), 3)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                     "traffic": profiled_traffic(args.workload),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "kernel": "pair_kernel_fast<float> (+ epilogue) per jefi_eval_fields, HIP events on its stream",
                     "flops_per_live_pair": FLOPS_PER_LIVE_PAIR},
    }

    if args.workload == "large" and not args.no_companion:
        res["single_instance_32^3"] = run_companion(args)
    if args.workload == "large" and not args.no_variants:
        res["stencil_variants"] = run_stencil_variants(args, p, extra)
    if args.workload == "large" and not args.no_batch:
        res["batch"] = batch_measure(args.batch_steps, 2, tune=not args.no_tune)
    if args.workload == "large" and not args.no_serve:
        res["serve"] = serve_measure(args.serve_seconds, args.serve_inflight, args.serve_reserve_cus,
                                     int(args.serve_small_arena_gib * 2**30), args.serve_express_pairs,
                                     args.serve_express_cus)
        res["p99_latency_ms"] = res["serve"]["paced"]["latency_ms"]["p99"]

    if not args.no_parity or not args.no_cpu_baseline:
        import oracle
        # history window of the final state: the last nt steps
        full = np.concatenate([p.hist, extra], axis=0)
        last = r32["newest"]
        first = last - p.nt + 1          # absolute step of the window's oldest slice
        win = full[first:last + 1]
        t_last = p.t0 + last * p.dt

    if not args.no_parity:
        from oracle.compare import max_rel_l2
        rng = np.random.default_rng(11)
        sel = np.sort(rng.choice(p.obs.size, size=min(32, p.obs.size), replace=False))
        Er, Br = oracle.eval_fields(p.src, p.obs, win, p.dt, t_last, p.t0, last, p.c, p.screen, sel=sel)
        err32 = max_rel_l2(r32["E"][:, sel], r32["B"][:, sel], Er, Br)
        # the same against the oracle on the FP32-rounded history: arithmetic error alone
        win32 = win.astype(np.float32).astype(np.float64)
        Er32, Br32 = oracle.eval_fields(p.src, p.obs, win32, p.dt, t_last, p.t0, last, p.c, p.screen, sel=sel)
        err32_arith = max_rel_l2(r32["E"][:, sel], r32["B"][:, sel], Er32, Br32)
        # the FP64 path at its own final step
        last64 = r64["newest"]
        win64 = full[last64 - p.nt + 1:last64 + 1]
        Er64, Br64 = oracle.eval_fields(p.src, p.obs, win64, p.dt, p.t0 + last64 * p.dt, p.t0, last64, p.c,
                                        p.screen, sel=sel)
        err64 = max_rel_l2(r64["E"][:, sel], r64["B"][:, sel], Er64, Br64)
        from oracle.compare import rel_l2

        def per_component(Eg, Bg, Er_, Br_):
            e, _ = rel_l2(Eg, Er_)
            b, _ = rel_l2(Bg, Br_)
            return {k: float(f"{v:.3e}") for k, v in zip(("Ex", "Ey", "Ez", "Bx", "By", "Bz"), e + b)}
        res["parity"] = {"sampled_points": int(len(sel)), "max_rel_l2_f32": float(f"{err32:.3e}"),
                         "rel_l2_f32_per_component": per_component(r32["E"][:, sel], r32["B"][:, sel], Er, Br),
                         "rel_l2_f64_per_component": per_component(r64["E"][:, sel], r64["B"][:, sel], Er64, Br64),
                         "max_rel_l2_f32_vs_fp32_inputs": float(f"{err32_arith:.3e}"),
                         "max_rel_l2_f64": float(f"{err64:.3e}"), "tol": 1e-5, "tol_f64": 1e-12,
                         "ok": bool(err32 <= 1e-5 and err64 <= 1e-12)}
        log(f"parity on {len(sel)} sampled points: f32 {err32:.3e} (arithmetic {err32_arith:.3e}), "
            f"f64 {err64:.3e}")

    if not args.no_cpu_baseline:
        threads = oracle.max_threads()
        # enough probe points to occupy every thread, so the rate is the parallel one
        n_probe = min(p.obs.size, 4 * threads)
        probe = np.linspace(0, p.obs.size - 1, n_probe).astype(np.int64)
        t0 = time.perf_counter()
        oracle.eval_fields(p.src, p.obs, win, p.dt, t_last, p.t0, last, p.c, p.screen, sel=probe)
        rate = len(probe) * p.src.size / max(time.perf_counter() - t0, 1e-6)
        n_pts = int(min(p.obs.size, max(8, args.cpu_seconds * rate / p.src.size)))
        sel = np.linspace(0, p.obs.size - 1, n_pts).astype(np.int64)
        t0 = time.perf_counter()
        oracle.eval_fields(p.src, p.obs, win, p.dt, t_last, p.t0, last, p.c, p.screen, sel=sel)
        dt_cpu = time.perf_counter() - t0
        cpu_val = n_pts * p.src.size / dt_cpu / 1e9
        # single-thread rates on the two small configurations: the tiny one
        # whole, the 32^3 one on evenly spaced observation points (~3 s)
        single = {}
        for name, q in (("tiny-8^3x8^3-nt16", workloads.config_tiny()),
                        ("medium-32^3x32^3-nt64", workloads.config_medium())):
            n_q = q.obs.size if q.obs.size <= 512 else 256
            sel_q = np.linspace(0, q.obs.size - 1, n_q).astype(np.int64)
            t0 = time.perf_counter()
            oracle.eval_problem(q, sel=sel_q, threads=1)
            dtq = time.perf_counter() - t0
            single[name] = {"value": round(n_q * q.src.size / dtq / 1e9, 6), "unit": "G pairs/s",
                            "sample": f"{n_q} of {q.obs.size} observation points x {q.src.size} source cells",
                            "seconds": round(dtq, 3)}
        res["cpu_baseline"] = {"value": round(cpu_val, 5), "unit": "G pairs/s", "cores": threads,
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"{n_pts} evenly spaced observation points x all {p.src.size} "
                                         f"source cells of the final step ({dt_cpu:.1f} s, FP64, "
                                         f"OpenMP over points)",
                               "single_thread": single}
        log(f"cpu oracle: {cpu_val:.4f} G pairs/s on {threads} threads ({cpu_model()}); single thread "
            + ", ".join(f"{k} {v['value']:.5f}" for k, v in single.items()))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
