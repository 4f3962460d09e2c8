"""The pins must catch plausible mistakes: each mutant below is a copy of the
oracle source with one planted error (a swapped interpolation weight, a lost
1/R, a flipped sign, an off-by-half pixel position, a wrong CG coefficient...),
compiled on the CPU.  At least one pin has to fail for every mutant."""
import ctypes
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins
from golden_cases import load_point_sources

SRC = os.path.join(os.path.dirname(oracle.__file__), "pa_oracle.c")

MUTANTS = {
    "swap_interp_weights_forward": ("row[(int64_t)k0d] += w * (1.0 - f) * x[p];",
                                    "row[(int64_t)k0d] += w * f * x[p];"),
    "drop_inverse_distance": ("double w = 1.0 / R;", "double w = 1.0 / (R * 0 + 1.0);"),
    "t0_sign": ("return (R / g->c - g->t0) / g->dt;", "return (R / g->c + g->t0) / g->dt;"),
    "pixel_offset_half": ("r[0] = g->center[0] + ((double)ix - 0.5 * (g->nx - 1)) * g->h;",
                          "r[0] = g->center[0] + ((double)ix - 0.5 * g->nx) * g->h;"),
    "adjoint_late_tap_index": ("acc += w * f * row[(int64_t)k0d + 1];", "acc += w * f * row[(int64_t)k0d];"),
    "cgls_beta_inverted": ("double beta = gamma1 / gamma;", "double beta = gamma / gamma1;"),
    "cgls_lambda_sign": ("for (int64_t i = 0; i < P; ++i) s[i] -= lambda * x[i];\n    double gamma1",
                         "for (int64_t i = 0; i < P; ++i) s[i] += lambda * x[i];\n    double gamma1"),
    "clamp_full_pitch": ("return g->r_min > 0 ? g->r_min : 0.5 * g->h;", "return g->r_min > 0 ? g->r_min : g->h;"),
    "landweber_step_sign": ("x[i] += omega * (s[i] - lambda * x[i]);", "x[i] += omega * (s[i] + lambda * x[i]);"),
    "tv_gradient_lost_term": ("          grad[p] -= dy / m;\n", ""),
    "tv_vertical_difference": ("const double dy = iy + 1 < ny ? x[p + nx] - x[p] : 0.0;",
                               "const double dy = iy + 1 < ny ? x[p + 1] - x[p] : 0.0;"),
    "fista_no_momentum": ("const double mu = (t - 1.0) / t1;", "const double mu = 0.0 * (t - 1.0) / t1;"),
    "fista_momentum_reversed": ("z[i] = xn[i] + mu * (xn[i] - x[i]);", "z[i] = xn[i] + mu * (x[i] - xn[i]);"),
    "fista_full_threshold": ("const double tau = omega * alpha / 2.0;", "const double tau = omega * alpha;"),
    "fista_full_tv_weight": ("grad[i] += 0.5 * beta * tvg[i];", "grad[i] += beta * tvg[i];"),
    "fista_lambda_dropped": ("grad[i] += lambda * z[i];", "grad[i] += 0.0 * z[i];"),
    "freq_sin_cos_swapped": ("re += x[p] * OR_TWO_PI * fn * sin(kn * R) / R;",
                             "re += x[p] * OR_TWO_PI * fn * cos(kn * R) / R;"),
    "freq_phase_sign": ("re += x[p] * OR_TWO_PI * fn * sin(kn * R) / R;",
                        "re -= x[p] * OR_TWO_PI * fn * sin(kn * R) / R;"),
    "freq_adjoint_imag_sign": ("+ kim * Y[((int64_t)s * nf + n) * 2 + 1];", "- kim * Y[((int64_t)s * nf + n) * 2 + 1];"),
    "freq_frequency_index": ("const double fn = f0 + n * df;", "const double fn = f0 + (n + 1) * df;"),
    "fista_nonneg_ignores_threshold": ("if (nonneg) return v > tau ? v - tau : 0.0;",
                                       "if (nonneg) return v > 0.0 ? v : 0.0;"),
}

PINS = [
    lambda: [pins.test_point_source_golden(c) for c in load_point_sources()],
    lambda: pins.test_zeroth_and_first_moment(2),
    lambda: pins.test_zeroth_and_first_moment(3),
    pins.test_adjoint_of_unit_trace_is_inverse_distance,
    lambda: pins.test_adjoint_identity(2, 3.7e-7),
    pins.test_rotation_by_quarter_turn_shifts_sensors,
    pins.test_time_origin_shift,
    lambda: pins.test_cgls_reaches_regularised_normal_equations(1e-2),
    pins.test_cgls_iterates_minimise_over_krylov_spaces,
    pins.test_landweber_closed_form,
    pins.test_tv_closed_forms,
    pins.test_tv_gradient_matches_finite_differences_and_shift_invariance,
    lambda: pins.test_fista_without_penalties_reaches_normal_equations(False),
    lambda: pins.test_fista_l1_satisfies_kkt(True),
    pins.test_fista_tv_satisfies_kkt,
    pins.test_fista_meets_the_accelerated_rate_bound,
    pins.test_freq_point_source_quarter_cycles,
    lambda: pins.test_freq_adjoint_identity(2),
    pins.test_freq_is_the_spectrum_of_the_time_domain_derivative,
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation site not found"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    hdr_dir = os.path.dirname(SRC)
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-I", hdr_dir,
                           "-o", str(so), str(mut), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle._configure(ctypes.CDLL(str(so))))
    failed = []
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed.append(pin)
    assert failed, f"no pin caught mutant {name}"
