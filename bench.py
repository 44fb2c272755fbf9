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


def run_path(p, extra, prec, steps, warmup):
    """Time `steps` steps (push + eval) after `warmup`; returns a dict."""
    import torch
    import paper_2104_05426_amd as J
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP,
                                 c=p.c, screen=p.screen)
    store, h = J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest, capacity=p.nt)
    slices = [torch.as_tensor(extra[i], dtype=tdt).cuda().contiguous() for i in range(extra.shape[0])]
    n_obs = p.obs.size
    E = torch.empty((3, n_obs), dtype=torch.float32, device="cuda")
    B = torch.empty((3, n_obs), dtype=torch.float32, device="cuda")

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

    p = make_workload(args.workload)
    K, W = args.steps, args.warmup
    K64 = args.fp64_steps if args.fp64_steps is not None else max(2, K // 2)
    n_extra = W + max(K, K64)
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
                   "precision": "FP32 pair arithmetic, compensated accumulation, FP64 index guard"},
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
                     "kernel": "pair_kernel<float> (+ epilogue) per jefi_eval_fields, HIP events",
                     "flops_per_live_pair": FLOPS_PER_LIVE_PAIR},
    }

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
        res["parity"] = {"sampled_points": int(len(sel)), "max_rel_l2_f32": float(f"{err32:.3e}"),
                         "tol": 1e-5, "ok": bool(err32 <= 1e-5)}
        log(f"parity on {len(sel)} sampled points: {err32:.3e}")

    if not args.no_cpu_baseline:
        threads = oracle.max_threads()
        probe = np.arange(0, p.obs.size, max(1, p.obs.size // 4))[:4]
        t0 = time.perf_counter()
        oracle.eval_fields(p.src, p.obs, win, p.dt, t_last, p.t0, last, p.c, p.screen, sel=probe)
        rate = len(probe) * p.src.size / max(time.perf_counter() - t0, 1e-6)
        n_pts = int(min(p.obs.size, max(8, args.cpu_seconds * rate / p.src.size)))
        sel = np.linspace(0, p.obs.size - 1, n_pts).astype(np.int64)
        t0 = time.perf_counter()
        oracle.eval_fields(p.src, p.obs, win, p.dt, t_last, p.t0, last, p.c, p.screen, sel=sel)
        dt_cpu = time.perf_counter() - t0
        cpu_val = n_pts * p.src.size / dt_cpu / 1e9
        res["cpu_baseline"] = {"value": round(cpu_val, 5), "unit": "G pairs/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{n_pts} evenly spaced observation points x all {p.src.size} "
                                         f"source cells of the final step ({dt_cpu:.1f} s, FP64, "
                                         f"OpenMP over points)"}
        log(f"cpu oracle: {cpu_val:.4f} G pairs/s on {threads} threads")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
