"""The allocation-free evaluation (jefi_eval_fields_noalloc) against the
allocating one (jefi_eval_fields), both through the C ABI, on the same
resident histories: two calls in a row on the library's fixed scratch, the
second on a smaller problem (so it runs over what the first left behind).

Bars as for the oracle parity tests: per-component relative L2 within 1e-5
(FP32 compensated) or 1e-12 (FP64) and every point within ten times that;
where the split count is not capped (the partials fit the scratch), the
two entry points run the same launches and agree bit for bit.  A problem
with 64^3 observation points against a 32^3 source needs more partials
than the scratch holds, so there the split count is capped."""
import numpy as np
import pytest

import workloads
from oracle.compare import check_fields
from workloads import centred_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _capped_problem():
    """32^3 source (dx 0.05) of 20 blobs, 64 slices; 64^3 observation grid
    of the same spacing centred on it: its 32 FP64 splits of 262144 points
    would need 403 MB of partials."""
    rng = np.random.default_rng(21)
    src = centred_grid((32, 32, 32), 0.05)
    obs = centred_grid((64, 64, 64), 0.05)
    blobs = workloads.draw_blobs(rng, 20, (-0.8, 0.8))
    return workloads._problem("noalloc-32^3x64^3-nt64", src, obs, blobs, 64, 0.025)


def _run_both(J, torch, p, prec):
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    pr = J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP
    tdt = torch.float64 if prec == "f64" else torch.float32
    store, h = J.upload_history(p.src, p.hist, hdt, t0=p.t0, newest=p.newest)
    opt = J.jefi_options_default(precision=pr, c=p.c, screen=p.screen)
    n = p.obs.size
    out = {}
    for name, fn in (("alloc", J.jefi_eval_fields), ("noalloc", J.jefi_eval_fields_noalloc)):
        E = torch.full((3, n), float("nan"), dtype=tdt, device="cuda")
        B = torch.full((3, n), float("nan"), dtype=tdt, device="cuda")
        fn(p.src, h, p.dt, p.nt, p.obs, p.t, E, B, opt)
        torch.cuda.synchronize()
        out[name] = (E.double().cpu().numpy(), B.double().cpu().numpy())
    del store
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_eval_fields_twice(prec):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_05426_amd as J
    first = _capped_problem()
    second = workloads.config_medium()   # smaller: 32768 points
    for p, same_plan in ((first, False), (second, True)):
        print(f"noalloc {prec} {p.name}", flush=True)
        r = _run_both(J, torch, p, prec)
        (Ea, Ba), (En, Bn) = r["alloc"], r["noalloc"]
        check_fields(En, Bn, Ea, Ba, TOL[prec], label=f"noalloc {prec} {p.name}")
        if same_plan:
            assert np.array_equal(En, Ea) and np.array_equal(Bn, Ba)


def test_noalloc_tiny_after_large():
    """A tiny problem right after the others: nothing it reads may depend
    on what earlier calls left in the scratch."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_05426_amd as J
    p = workloads.config_tiny()
    for prec in ("f32", "f64"):
        r = _run_both(J, torch, p, prec)
        (Ea, Ba), (En, Bn) = r["alloc"], r["noalloc"]
        check_fields(En, Bn, Ea, Ba, TOL[prec], label=f"noalloc {prec} {p.name}")
        assert np.array_equal(En, Ea) and np.array_equal(Bn, Ba)
