"""Per-step coupling with a producer (jefi_coupler_*, through the C ABI): a
time-stepping loop hands one slice per step and takes E and B back, with
the copies of one step overlapping the neighbouring evaluations.  At every
step the coupled fields equal, bit for bit, those of the plain serial loop
(push, evaluate, synchronise, copy) on the same slices, for host and device
slices and both precisions; one step is checked against the oracle; a slot
still holding an uncollected step refuses the next step."""
import numpy as np
import pytest

import oracle
import workloads
from oracle.compare import check_fields
from workloads import Blob, blob_history, centred_grid

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
N_INIT, N_STEPS, CAP = 10, 8, 24


def _setup():
    src = centred_grid((16, 16, 16), 0.1)
    obs = src.shifted_cells(4, -2, 3)
    dt = 0.05
    blobs = [Blob(1.0, 0.25, (0.1, -0.2, 0.0), (0.3, 0.1, -0.2)), Blob(-0.6, 0.2, (-0.3, 0.2, 0.1), (0.0, 0.4, 0.2))]
    hist = blob_history(src, blobs, N_INIT + N_STEPS, dt)
    return src, obs, dt, hist


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_05426_amd as J
    return J, torch


def _serial(J, torch, src, obs, dt, hist, prec):
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
    store, h = J.upload_history(src, hist[:N_INIT], hdt, capacity=CAP)
    out = []
    for k in range(N_STEPS):
        J.jefi_history_push(h, src, torch.as_tensor(hist[N_INIT + k], dtype=tdt).cuda())
        E = torch.empty((3, obs.size), dtype=tdt, device="cuda")
        B = torch.empty_like(E)
        J.jefi_eval_fields(src, h, dt, min(CAP, h.newest + 1), obs, h.newest * dt, E, B, opt)
        torch.cuda.synchronize()
        out.append((E.cpu().numpy(), B.cpu().numpy()))
    del store
    return out


def _coupled(J, torch, src, obs, dt, hist, prec, on_host):
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    ndt = np.float64 if prec == "f64" else np.float32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
    store, h = J.upload_history(src, hist[:N_INIT], hdt, capacity=CAP)
    cp = J.Coupler(src, h, dt, CAP, obs, opt, out_dtype=hdt)
    # device slices stay alive until their step is collected
    dev = [torch.as_tensor(hist[N_INIT + k], dtype=tdt).cuda() for k in range(N_STEPS)]
    out, steps = [], []
    for k in range(N_STEPS):
        sl = np.ascontiguousarray(hist[N_INIT + k], dtype=ndt) if on_host else dev[k]
        steps.append(cp.step(sl))
        if k >= 1:  # one step in flight behind the newest
            E = np.empty((3, obs.size), ndt)
            B = np.empty((3, obs.size), ndt)
            cp.collect(steps[k - 1], E, B)
            out.append((E, B))
    E = np.empty((3, obs.size), ndt)
    B = np.empty((3, obs.size), ndt)
    cp.collect(steps[-1], E, B)
    out.append((E, B))
    assert steps == list(range(N_INIT, N_INIT + N_STEPS))
    assert cp.destroy() == J.JEFI_OK
    del store, dev
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("on_host", [True, False])
def test_coupled_steps_equal_serial_loop(prec, on_host):
    J, torch = _gpu()
    src, obs, dt, hist = _setup()
    serial = _serial(J, torch, src, obs, dt, hist, prec)
    coupled = _coupled(J, torch, src, obs, dt, hist, prec, on_host)
    for k, ((Es, Bs), (Ec, Bc)) in enumerate(zip(serial, coupled)):
        assert np.array_equal(Es, Ec) and np.array_equal(Bs, Bc), (prec, on_host, k)
    # the last coupled step against the oracle
    last = N_INIT + N_STEPS - 1
    nt = min(CAP, last + 1)
    p = workloads.Problem("coupled", src, obs, hist[last - nt + 1:last + 1], dt, last * dt, 0.0, last, 1.0,
                          workloads.default_screen(src))
    if prec == "f32":
        p.hist = p.hist.astype(np.float32).astype(np.float64)
    Er, Br = oracle.eval_problem(p)
    check_fields(coupled[-1][0], coupled[-1][1], Er, Br, TOL[prec], f"coupled last step {prec}")


def test_coupler_slot_rules():
    """A third step while the first is uncollected is refused (EBUSY), and
    collecting a step twice or one never enqueued is ENOENT."""
    J, torch = _gpu()
    src, obs, dt, hist = _setup()
    store, h = J.upload_history(src, hist[:N_INIT], J.JEFI_F32, capacity=CAP)
    cp = J.Coupler(src, h, dt, CAP, obs, J.jefi_options_default(precision=J.JEFI_PREC_F32_COMP))
    s0 = cp.step(np.ascontiguousarray(hist[N_INIT], dtype=np.float32))
    s1 = cp.step(np.ascontiguousarray(hist[N_INIT + 1], dtype=np.float32))
    with pytest.raises(J.JefiError) as ei:
        cp.step(np.ascontiguousarray(hist[N_INIT + 2], dtype=np.float32))
    assert ei.value.status == J.JEFI_EBUSY
    E = np.empty((3, obs.size), np.float32)
    B = np.empty((3, obs.size), np.float32)
    cp.collect(s0, E, B)
    with pytest.raises(J.JefiError) as ei:
        cp.collect(s0, E, B)
    assert ei.value.status == J.JEFI_ENOENT
    with pytest.raises(J.JefiError) as ei:
        cp.collect(s1 + 5, E, B)
    assert ei.value.status == J.JEFI_ENOENT
    cp.collect(s1, E, B)
    assert np.all(np.isfinite(E)) and np.all(np.isfinite(B))
    assert cp.destroy() == J.JEFI_OK
    del store


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_device_producer_on_its_own_stream(prec):
    """A producer that writes each slice on a stream of its own, after a
    delay, into one of two reused buffers: the coupler's push waits for that
    stream, so the coupled steps still equal the serial loop bit for bit."""
    J, torch = _gpu()
    src, obs, dt, hist = _setup()
    serial = _serial(J, torch, src, obs, dt, hist, prec)
    hdt = J.JEFI_F64 if prec == "f64" else J.JEFI_F32
    ndt = np.float64 if prec == "f64" else np.float32
    tdt = torch.float64 if prec == "f64" else torch.float32
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64 if prec == "f64" else J.JEFI_PREC_F32_COMP)
    store, h = J.upload_history(src, hist[:N_INIT], hdt, capacity=CAP)
    cp = J.Coupler(src, h, dt, CAP, obs, opt, out_dtype=hdt)
    staged = [torch.as_tensor(hist[N_INIT + k], dtype=tdt).cuda() for k in range(N_STEPS)]
    buf = [torch.zeros_like(staged[0]) for _ in range(2)]
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    out, steps = [], []
    for k in range(N_STEPS):
        with torch.cuda.stream(side):
            torch.cuda._sleep(2_000_000)   # the producer is still busy when the step is enqueued
            buf[k % 2].copy_(staged[k])
        steps.append(cp.step(buf[k % 2], side))
        if k >= 1:
            E = np.empty((3, obs.size), ndt)
            B = np.empty((3, obs.size), ndt)
            cp.collect(steps[k - 1], E, B)   # also frees buf[(k - 1) % 2] for step k + 1
            out.append((E, B))
    E = np.empty((3, obs.size), ndt)
    B = np.empty((3, obs.size), ndt)
    cp.collect(steps[-1], E, B)
    out.append((E, B))
    assert cp.destroy() == J.JEFI_OK
    for k, ((Es, Bs), (Ec, Bc)) in enumerate(zip(serial, out)):
        assert np.array_equal(Es, Ec) and np.array_equal(Bs, Bc), (prec, k)
    del store, staged, buf
