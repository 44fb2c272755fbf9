"""The pins catch plausible mistakes: each test here compiles a copy of the
oracle with one planted error (on the CPU) and checks that at least one pin
of ``test_oracle_pins`` fails against it."""
import os

import pytest

import oracle
from tests import test_oracle_fingerprint as fpins
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "jefi_oracle.c")

MUTATIONS = {
    "E: sign of the -Jdot/R term": ("- Jd[a] * iR)", "+ Jd[a] * iR)"),
    "B: overall sign": ("orc_nadd(&acc[3 + a], -(cJ[a] * iR3 + cD[a] * iR2))",
                        "orc_nadd(&acc[3 + a], (cJ[a] * iR3 + cD[a] * iR2))"),
    "cross product transposed": ("double cJ[3] = {d[1] * J[2] - d[2] * J[1], d[2] * J[0] - d[0] * J[2], d[0] * J[1] - d[1] * J[0]};",
                                 "double cJ[3] = {d[2] * J[1] - d[1] * J[2], d[0] * J[2] - d[2] * J[0], d[1] * J[0] - d[0] * J[1]};"),
    "volume element dropped": ("const double pref = (src->spacing[0] * src->spacing[1] * src->spacing[2]) / (4.0 * M_PI);",
                               "const double pref = 1.0 / (4.0 * M_PI);"),
    "prefactor 1/(2 pi)": ("/ (4.0 * M_PI);", "/ (2.0 * M_PI);"),
    "rho_dot weighted by 1/R^3": ("d[a] * rhod * iR2", "d[a] * rhod * iR3"),
    "derivative of the interpolant": ("double d0 = (h0 - hm) * inv_dt;",
                                      "double d0 = (orc_h(hist, ns, k + 1, ch, s, hold) - h0) * inv_dt;"),
    "slice index one late": ("*k = tm->a_i + (int64_t)m;", "*k = tm->a_i + (int64_t)m + 1;"),
    "weight f complemented": ("*f = u - m;", "*f = 1.0 - (u - m);"),
    "past held at the oldest slice": ("if (!hold) return 0.0;", "if (0) return 0.0;"),
    "retarded time uses R*c*dt": ("out->inv_cdt = 1.0 / (c * dt);", "out->inv_cdt = c / dt;"),
    "Jdot missing from B": ("-(cJ[a] * iR3 + cD[a] * iR2)", "-(cJ[a] * iR3)"),
    "slope reading uses the backward difference": ("if (slope) w = (orc_h(hist, ns, k + 1, ch, s, hold) - h0) * inv_dt;",
                                                   "if (slope) w = (h0 - hm) * inv_dt;"),
    "held past still culls old stencils": ("if (k < -1 && !hold) continue;", "if (k < -1) continue;"),
    "cubic on nodes k-1 .. k+2": ("static const double x[4] = {-2.0, -1.0, 0.0, 1.0};\n",
                                  "static const double x[4] = {-1.0, 0.0, 1.0, 2.0};\n"),
    "cubic derivative not divided by dt": ("der[ch] = d * inv_dt;", "der[ch] = d;"),
    "cubic derivative weights unscaled": ("double q = 1.0 / (x[i] - x[m]);", "double q = 1.0;"),
    "cubic read one slice early": ("double h = orc_h(hist, ns, k - 2 + i, ch, s, hold);",
                                   "double h = orc_h(hist, ns, k - 3 + i, ch, s, hold);"),
    "held past keeps h(-1) = 0 in D_0": ("double hm = orc_h(hist, ns, k - 1, ch, s, hold);",
                                         "double hm = k - 1 < 0 ? 0.0 : orc_h(hist, ns, k - 1, ch, s, hold);"),
    "history start keeps pairs at k = -1": ("if (cut && k < 0) continue;", "if (cut && k < -1) continue;"),
    "history start reads a zero past": ("const int hold = (stencil & 2) != 0 || cut;",
                                        "const int hold = (stencil & 2) != 0;"),
}

PIN_CALLS = [
    pins.test_static_cell_is_coulomb_and_biot_savart,
    pins.test_linear_history_is_reproduced_exactly,
    pins.test_quadratic_history_pins_the_derivative_reading,
    lambda: pins.test_switch_on_at_the_oldest_slice("k=-1"),
    lambda: pins.test_switch_on_at_the_oldest_slice("k=0"),
    pins.test_gauss_flux_equals_enclosed_charge_and_B_flux_vanishes,
    pins.test_current_ring_on_axis,
    pins.test_exact_integer_retarded_positions,
    pins.test_saturation_for_constant_sources,
    pins.test_quadratic_history_slope_reading,
    lambda: pins.test_switch_on_slope_reading("k=-1"),
    lambda: pins.test_held_past_constant_history_is_static_at_any_time(2),
    lambda: pins.test_held_past_linear_history(2),
    lambda: pins.test_held_past_linear_history(3),
    lambda: pins.test_history_start_linear_history(8),
    lambda: pins.test_history_start_constant_sources_are_the_static_ball_sum(8),
    pins.test_voxelised_uniform_sphere_is_coulomb_outside,
    pins.test_uniform_charge_and_current_box_match_the_continuum,
    pins.test_cubic_history_is_reproduced_exactly,
    pins.test_quartic_history_pins_the_cubic_nodes,
    lambda: pins.test_switch_on_cubic_reading("k=-1"),
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation anchor not found: {old}"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(text.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    oracle.build(source=str(mutated), target=lib)
    failures = 0
    oracle._use_library(lib)
    try:
        for call in PIN_CALLS:
            try:
                call()
            except (AssertionError, ValueError):
                failures += 1
    finally:
        oracle._use_library(None)
    assert failures >= 1, f"no pin caught: {name}"


# Mistakes in the per-point fingerprint of the slice decisions; caught by the
# fingerprint pins (hand-computed rows, rows rebuilt from the pure-Python
# per-pair decisions).
FP_MUTATIONS = {
    "fingerprint drops pairs at k = -1": ("if (k < -1) continue;\n      ++nlive;",
                                          "if (k <= -1) continue;\n      ++nlive;"),
    "fingerprint counts pairs at k = -2": ("if (k < -1) continue;\n      ++nlive;",
                                           "if (k < -2) continue;\n      ++nlive;"),
    "fingerprint weights by s instead of s+1": ("skw += (uint64_t)k * (uint64_t)(s + 1);",
                                                "skw += (uint64_t)k * (uint64_t)s;"),
    "fingerprint does not count screened pairs": ("{ ++nscr; continue; }", "{ continue; }"),
    "fingerprint ignores the point selection": (
        "int64_t o = sel ? sel[q] : q;\n    if (o < 0 || o >= no) { bad = 1; continue; }\n    double ro[3];\n"
        "    orc_centre(obs, o, ro);\n    int64_t nlive",
        "int64_t o = q;\n    if (o < 0 || o >= no) { bad = 1; continue; }\n    double ro[3];\n"
        "    orc_centre(obs, o, ro);\n    int64_t nlive"),
}

FP_PIN_CALLS = [
    fpins.test_hand_computed_fingerprints,
    fpins.test_hand_computed_fingerprint_off_slice_and_screening_cube,
    lambda: fpins.test_fingerprint_equals_the_pure_python_pair_decisions(0),
    lambda: fpins.test_fingerprint_equals_the_pure_python_pair_decisions(1),
    fpins.test_negative_indices_wrap_the_weighted_sum,
]


@pytest.mark.parametrize("name", sorted(FP_MUTATIONS))
def test_planted_fingerprint_mistake_is_caught(name, tmp_path):
    old, new = FP_MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not found once: {old}"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(text.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    oracle.build(source=str(mutated), target=lib)
    failures = 0
    oracle._use_library(lib)
    try:
        for call in FP_PIN_CALLS:
            try:
                call()
            except (AssertionError, ValueError):
                failures += 1
    finally:
        oracle._use_library(None)
    assert failures >= 1, f"no fingerprint pin caught: {name}"
