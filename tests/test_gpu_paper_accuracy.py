"""The paper's accuracy experiments (section "Comparisons with the
theoretical results") on the GPU path: 15^3 source grids of cell 0.4 over
[-3, 3]^3, screening half-width 0.2, deviations in the XOY plane measured
as max |(dEx, dEy)| / max |(Ex, Ey)| (the paper's norms).

- Saturated constant sources against the exact continuum: once every
  retarded time is past the switch-on, constant rho = 1, J = (1, 1, 1) give
  the static field of a uniformly charged box (closed form, B = J x E; the
  screening cube around an interior point adds nothing by symmetry).  The
  discrete sum is taken with the held-past stencil on a two-slice ring, and
  is checked to equal the zero-past sum at a saturated time on a full ring.
  Refining the grid 1, 2, 4, 8, 16 times converges to the closed form.
- The paper's snapshots t = 2.5, 5, 7.5 (time step 0.05): the deviation
  from the same discretisation refined 4 times shrinks as the grid is
  refined.
- The same snapshots against the continuous equations, computed by FP64
  quadrature (tests/continuum.py): the discretised sums converge to the
  reading that keeps the switch-on shell; the reading without it (the
  Coulomb and Biot-Savart fields of the box within distance t) has the
  paper's field scale (peak 0.529 at t = 2.5) and is far from the sums.
- The library's history-start reading (JEFI_FLAG_PAST_CUT: the sources
  begin at the oldest slice, no derivative across the start) converges to
  the shell-less continuum, within 1 % at 15^3 like the paper's figure."""
import numpy as np
import pytest

import workloads
from tests.continuum import box_fields, switched_on_box_plane

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2104_05426_amd as J
    return torch, J


def _xoy_dev(x, ref):
    d = np.sqrt((x[0] - ref[0]) ** 2 + (x[1] - ref[1]) ** 2).max()
    return float(d / np.sqrt(ref[0] ** 2 + ref[1] ** 2).max())


def _plane(z=0.0):
    return workloads.Grid((15, 15, 1), (-2.8, -2.8, z), (0.4, 0.4, 0.4))


def _static_fields(torch, J, r, zero_past_slices=0):
    """Constant sources on the (15 r)^3 grid: held past on 2 slices, or the
    zero past on a ring of `zero_past_slices` ones evaluated at its newest step."""
    n, dx = 15 * r, 0.4 / r
    src = workloads.Grid((n, n, n), (-3.0 + 0.5 * dx,) * 3, (dx,) * 3)
    dt = 0.05 / r
    nt = zero_past_slices or 2
    store = torch.empty(J.jefi_history_bytes(src, nt, J.JEFI_F64), dtype=torch.uint8, device="cuda")
    h = J.jefi_history_init(store, src, nt, J.JEFI_F64)
    ones = torch.ones((4, src.size), dtype=torch.float64, device="cuda")
    for _ in range(nt):
        J.jefi_history_push(h, src, ones)
    obs = _plane()
    E = torch.empty((3, obs.size), dtype=torch.float64, device="cuda")
    B = torch.empty_like(E)
    opt = J.jefi_options_default(precision=J.JEFI_PREC_F64, screen=(0.2, 0.2, 0.2))
    if not zero_past_slices:
        opt.flags = J.JEFI_FLAG_PAST_HOLD
    J.jefi_eval_fields(src, h, dt, nt, obs, (nt - 1) * dt, E, B, opt)
    torch.cuda.synchronize()
    out = E.cpu().numpy(), B.cpu().numpy()
    del store, ones
    torch.cuda.empty_cache()
    return out


def test_saturated_constant_sources_converge_to_the_box_field():
    torch, J = _gpu()
    pts = workloads.cell_centres(_plane())
    E_ex = box_fields(pts, (-3.0,) * 3, (3.0,) * 3)
    B_ex = np.cross(np.ones(3)[None, :], E_ex.T).T
    devs = {}
    for r in (1, 2, 4, 8, 16):
        E, B = _static_fields(torch, J, r)
        devs[r] = (_xoy_dev(E, E_ex), _xoy_dev(B, B_ex))
        print(f"saturated constant sources, {15 * r}^3: deviation E {devs[r][0]:.4%}, B {devs[r][1]:.4%}",
              flush=True)
    # the held-past two-slice ring equals the saturated zero-past sum (t = 11 > box diagonal 10.4)
    E1, B1 = _static_fields(torch, J, 1)
    E2, B2 = _static_fields(torch, J, 1, zero_past_slices=221)
    assert np.allclose(E1, E2, rtol=1e-12, atol=1e-14) and np.allclose(B1, B2, rtol=1e-12, atol=1e-14)
    for r0, r1 in [(1, 2), (2, 4), (4, 8), (8, 16)]:
        assert devs[r1][0] < devs[r0][0] and devs[r1][1] < devs[r0][1], (r0, r1, devs)
    assert devs[16][0] < 0.01 and devs[16][1] < 0.01, devs


def test_paper_snapshots_converge():
    _gpu()
    import bench
    times = (2.5, 5.0, 7.5)
    f = {r: bench.accuracy_fields("constant", r, times, 0.0) for r in (1, 2, 4)}
    for t in times:
        d1 = [bench.xoy_deviation(f[1][t][i], f[4][t][i]) for i in (0, 1)]
        d2 = [bench.xoy_deviation(f[2][t][i], f[4][t][i]) for i in (0, 1)]
        print(f"constant sources t = {t}: 15^3 deviates {d1[0]:.3%} (E) {d1[1]:.3%} (B), "
              f"30^3 {d2[0]:.3%} {d2[1]:.3%} from 60^3", flush=True)
        assert d2[0] < d1[0] and d2[1] < d1[1], (t, d1, d2)


def test_paper_snapshots_against_the_continuum():
    _gpu()
    import bench
    times = (2.5, 5.0, 7.5)
    pts = workloads.cell_centres(_plane())
    f = {r: bench.accuracy_fields("constant", r, times, 0.0) for r in (1, 2, 4)}
    for t in times:
        ref = switched_on_box_plane(pts, t, (-3.0,) * 3, (3.0,) * 3)
        dev = {k: {r: [_xoy_dev(f[r][t][i], ref[k][i]) for i in (0, 1)] for r in f} for k in ref}
        print(f"constant sources t = {t}: with the shell " +
              ", ".join(f"{15 * r}^3 {d[0]:.3%} (E) {d[1]:.3%} (B)" for r, d in dev["shell"].items()) +
              "; without it " + ", ".join(f"{15 * r}^3 {d[0]:.1%} {d[1]:.1%}" for r, d in dev["no_shell"].items()),
              flush=True)
        # the sums converge to the reading with the shell ...
        assert dev["shell"][4][0] < dev["shell"][1][0] and dev["shell"][4][1] < dev["shell"][1][1], (t, dev)
        # ... and stay far from the one without it
        assert min(dev["no_shell"][r][0] for r in f) > 0.2, (t, dev)
    # the reading without the shell has the paper's scale: the one-face cap
    # field (t - h)^2 / (4 t) at h = 0.2 from a face
    E0 = switched_on_box_plane(pts, 2.5, (-3.0,) * 3, (3.0,) * 3)["no_shell"][0]
    assert abs(np.sqrt(E0[0] ** 2 + E0[1] ** 2).max() - 2.3 ** 2 / 10.0) < 1e-9


def test_history_start_reading_matches_the_shell_less_continuum():
    torch, J = _gpu()
    import bench
    times = (2.5, 5.0, 7.5)
    pts = workloads.cell_centres(_plane())
    f = {r: bench.accuracy_fields("constant", r, times, 0.0, "f64", J.JEFI_FLAG_PAST_CUT) for r in (1, 2, 4)}
    f32 = bench.accuracy_fields("constant", 1, times, 0.0, "f32", J.JEFI_FLAG_PAST_CUT)
    for t in times:
        ref = switched_on_box_plane(pts, t, (-3.0,) * 3, (3.0,) * 3)["no_shell"]
        dev = {r: [_xoy_dev(f[r][t][i], ref[i]) for i in (0, 1)] for r in f}
        print(f"constant sources t = {t}, history start: " +
              ", ".join(f"{15 * r}^3 {d[0]:.3%} (E) {d[1]:.3%} (B)" for r, d in dev.items()), flush=True)
        assert max(dev[1]) < 0.01, (t, dev)
        assert dev[4][0] < dev[1][0] and dev[4][1] < dev[1][1], (t, dev)
        d32 = [_xoy_dev(f32[t][i], ref[i]) for i in (0, 1)]
        assert abs(d32[0] - dev[1][0]) < 1e-4 and abs(d32[1] - dev[1][1]) < 1e-4, (t, d32, dev[1])
