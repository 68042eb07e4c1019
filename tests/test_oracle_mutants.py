"""Planted mistakes in the oracle must fail at least one pin (no GPU).

Each case copies the oracle's C source, plants one plausible mistake (a dropped term,
a wrong sign, a transposed operand, a wrong index), compiles the copy and runs the pins
of test_oracle_pins.py against it.  A mutant that passes every pin would mean the pins
cannot tell that mistake from the paper's method.
"""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "npf_oracle.c")

MUTANTS = {
    "drop 1/M! (sym)": ("const npfo_c c = Tprev[r] / fact;", "const npfo_c c = Tprev[r];"),
    "drop 1/M! (full)": ("C[j * nm + t] = s / fact;", "C[j * nm + t] = s;"),
    "divisor sign": ("npfo_c d = acc - lam[j];", "npfo_c d = lam[j] - acc;"),
    "divisor drops last term": ("for (int i = 1; i < M; ++i) acc = acc + lam[s[i]];",
                                "for (int i = 1; i < M - 1; ++i) acc = acc + lam[s[i]];"),
    "P sign (sym)": ("P_rows[q * n + k] = -s;", "P_rows[q * n + k] = s;"),
    "P sign (full)": ("P[j * n + k] = -s;", "P[j * n + k] = s;"),
    "Phi transposed (sym)": ("acc[t] = acc[t] + x * Phi[a * n + t];",
                             "acc[t] = acc[t] + x * Phi[t * n + a];"),
    "Phi transposed (full)": ("s = s + T[(o * n + a) * inner + in] * Phi[a * n + tp];",
                              "s = s + T[(o * n + a) * inner + in] * Phi[tp * n + a];"),
    "Psi transposed in G": ("                s = s + Psi[j * n + k] * a;",
                            "                s = s + Psi[k * n + j] * a;"),
    "multiplicity dropped": ("s = s + multiplicity(t, M) * (h[r] * z);", "s = s + (h[r] * z);"),
    "delta dropped in zeta": ("return Z ? Z[t * n + k] : delta * Psi[t * n + k];",
                              "return Z ? Z[t * n + k] : Psi[t * n + k];"),
    "zeta index transposed": ("return Z ? Z[t * n + k] : delta * Psi[t * n + k];",
                              "return Z ? Z[t * n + k] : delta * Psi[k * n + t];"),
    "zeta* index transposed": ("return Z ? Z[t * n + k] : delta * Psi[t * n + k];",
                               "return Z ? Z[k * n + t] : delta * Psi[t * n + k];"),
    "zeta* ignored": ("return Z ? Z[t * n + k] : delta * Psi[t * n + k];",
                      "return delta * Psi[t * n + k];"),
    "assembly transposed": ("npfo_c z = delta * Psi[i * n + k];", "npfo_c z = delta * Psi[k * n + i];"),
    "assembly mode index": ("npf[k * n + i] = Phi[k * n + i] * z;", "npf[k * n + i] = Phi[i * n + k] * z;"),
    "clamp ignored": ("if (mag2 < eps * eps) d = eps;", "(void)mag2;"),
    "clamp sign": ("if (mag2 < eps * eps) d = eps;", "if (mag2 < eps * eps) d = -eps;"),
    "stage keeps unsorted tail": ("const int64_t last = (i > 1) ? p[i - 2] : 0;",
                                  "const int64_t last = 0;"),
    "full sum skips a lower index": ("for (int i = 1; i < M; ++i) z = z * zeta_at(Z, Psi, delta, n, digits[i], k);",
                                     "for (int i = 2; i < M; ++i) z = z * zeta_at(Z, Psi, delta, n, digits[i], k);"),
    "Taylor drops the binomial": ("w *= (double)npfo_binom(e[l], j[l]) * factorial(j[l]);",
                                  "w *= factorial(j[l]);"),
    "Taylor drops the factorial": ("w *= (double)npfo_binom(e[l], j[l]) * factorial(j[l]);",
                                   "w *= (double)npfo_binom(e[l], j[l]);"),
    "Taylor power of x* off by one": ("for (int r = 0; r < e[l] - j[l]; ++r) w *= xs;",
                                      "for (int r = 1; r < e[l] - j[l]; ++r) w *= xs;"),
}

PIN_CALLS = [
    lambda: pins.test_p2_linear_limit(0.3),
    lambda: pins.test_p2_order_scales_as_delta_power(3),
    lambda: pins.test_p3_conjugate_modes(3),
    lambda: pins.test_p4_eigenvector_scaling_and_mode_permutation(3),
    lambda: pins.test_p5_diagonal_closed_form(),
    lambda: pins.test_p6_damped_oscillator_closed_form("full"),
    lambda: pins.test_p6_damped_oscillator_closed_form("sym"),
    lambda: pins.test_p7_polarization_finite_differences(3, 3),
    lambda: pins.test_p8_homological_residual_order(2),
    lambda: pins.test_p10_full_equals_sym(5, 3),
    lambda: pins.test_p10_full_equals_sym(4, 4),
    lambda: pins.test_clamp_exact_resonance(),
    lambda: pins.test_p11_interaction_full_equals_sym(4, 2),
    lambda: pins.test_p12_interaction_factors_reconstruct_the_kick([2], 3),
    lambda: pins.test_p13_poly_tensor_closed_forms(),
    lambda: pins.test_p13_poly_tensor_polarization(3),
    lambda: pins.test_p13_poly_tensor_taylor_expansion_at_equilibrium(),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not unique: {old}"
    mut = tmp_path / "npf_oracle.c"
    mut.write_text(text.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC), "npf_oracle.h")
    (tmp_path / "npf_oracle.h").write_text(open(hdr).read())
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", so, str(mut), "-lm"])
    caught = []
    with oracle.use_library(so):
        for i, call in enumerate(PIN_CALLS):
            try:
                call()
            except (AssertionError, ValueError, FloatingPointError, np_errors()):
                caught.append(i)
    assert caught, f"mutant '{name}' passed every pin"


def np_errors():
    import numpy as np
    return np.linalg.LinAlgError
