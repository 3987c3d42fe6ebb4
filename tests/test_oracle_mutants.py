"""Strength of the oracle pins: plausible mistakes planted in copies of the
oracle source (CPU only) must each fail at least one pin.

Every mutant is a one-token edit of ``oracle/tmm_oracle.c`` compiled into a
temporary library; the pins of ``test_oracle_pins.py`` are then run against it.
"""
import os

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "tmm_oracle.c")

MUTANTS = {
    "r_p sign": ("r = (n2 * c1 - n1 * c2) / den;", "r = (n1 * c2 - n2 * c1) / den;"),
    "t_p numerator": ("den = n2 * c1 + n1 * c2;\n            t = 2.0 * n1 * c1 / den;",
                      "den = n2 * c1 + n1 * c2;\n            t = 2.0 * n2 * c1 / den;"),
    "r_s sign": ("r = (n1 * c1 - n2 * c2) / den;", "r = (n2 * c2 - n1 * c1) / den;"),
    "dropped 2 pi": ("delta = 2.0 * ORACLE_PI * n1 * d[j - 1] * c1 / lam;",
                     "delta = n1 * d[j - 1] * c1 / lam;"),
    "phase uses next medium": ("delta = 2.0 * ORACLE_PI * n1 * d[j - 1] * c1 / lam;",
                               "delta = 2.0 * ORACLE_PI * n2 * d[j - 1] * c2 / lam;"),
    "phase sign": ("cplx em = cexp(-I * delta), ep = cexp(I * delta);",
                   "cplx em = cexp(I * delta), ep = cexp(-I * delta);"),
    "transposed product": ("mat2_mul(Mt, Mj, Mt);", "mat2_mul(Mj, Mt, Mt);"),
    "r from wrong entry": ("cplx r = Mt[2] / Mt[0];", "cplx r = Mt[1] / Mt[0];"),
    "T without flux ratio": ("T = tt * creal(n[L + 1] * cos_buf[L + 1]) / creal(n[0] * cos_buf[0]);",
                             "T = tt;"),
    "no branch fix-up": ("if (!is_forward(n[j] * c)) c = -c;", ";"),
    "Snell without n_0": ("cplx kx = n[0] * sin_t;", "cplx kx = sin_t;"),
    "T_p flux without conj": ("T = tt * creal(n[L + 1] * conj(cos_buf[L + 1])) / creal(n[0] * conj(cos_buf[0]));",
                              "T = tt * creal(n[L + 1] * cos_buf[L + 1]) / creal(n[0] * conj(cos_buf[0]));"),
    "matrix off-diagonal": ("cplx Mj[4] = {em / t, em * r / t, ep * r / t, ep / t};",
                            "cplx Mj[4] = {em / t, ep * r / t, em * r / t, ep / t};"),
}

PIN_TESTS = [
    (pins.test_normal_incidence_single_interface_textbook, {}),
    (pins.test_brewster_angle_kills_p_reflection, {}),
    (pins.test_total_internal_reflection, {}),
    (pins.test_stokes_relations_interface_reversal, {}),
    (pins.test_single_layer_airy_sum, {"seed": 0}),
    (pins.test_quarter_wave_mirror_normal_incidence, {}),
    (pins.test_quarter_wave_stack_oblique_tilted_admittances, {}),
    (pins.test_lossless_energy_conservation, {}),
    (pins.test_passivity_lossy, {}),
    (pins.test_zero_thickness_layer_is_invisible, {}),
    (pins.test_half_wave_absentee_layer, {}),
    (pins.test_reciprocity_of_transmittance, {}),
    (pins.test_normal_incidence_polarisation_relations, {}),
    (pins.test_against_50_digit_abeles_matrices, {"seed": 0}),
    (pins.test_against_50_digit_abeles_matrices, {"seed": 4}),
    (pins.test_against_50_digit_abeles_matrices, {"seed": 8}),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not found exactly once"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(path), str(tmp_path / "libmutant.so"))
    caught = []
    with oracle.using(lib):
        for fn, kw in PIN_TESTS:
            try:
                fn(**kw)
            except (AssertionError, ValueError, FloatingPointError):
                caught.append(fn.__name__)
    assert caught, f"no pin fails for the planted mistake {name!r}"
