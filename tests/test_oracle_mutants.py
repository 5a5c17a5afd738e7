"""Planted mistakes in a COPY of the oracle must each fail a pin.

Each mutant is a plausible slip (a transposed operand, a dropped term, a wrong
sign, an inverted control test, a missing bit reversal, a dropped norm term).
It is compiled from a string-edited copy of sv_oracle.c into a temporary
library on the CPU, and the pins of test_oracle.py run against it. The real
oracle is restored afterwards. Every mutant must fail at least one pin.
"""
import os
import subprocess

import pytest

import oracle
from oracle import build_oracle
from tests import test_oracle as pins

MUTANTS = {
    "transposed_q12_q21": [("q12r = m[2], q12i = m[3]", "q12r = m[4], q12i = m[5]"),
                           ("q21r = m[4], q21i = m[5]", "q21r = m[2], q21i = m[3]")],
    "dropped_q12_term": [("double nar = (q11r * ar - q11i * ai) + (q12r * br - q12i * bi);",
                          "double nar = (q11r * ar - q11i * ai);")],
    "wrong_sign_imag": [("double nai = (q11r * ai + q11i * ar)",
                         "double nai = (q11r * ai - q11i * ar)")],
    "inverted_control": [("if (k & cbit)", "if (!(k & cbit))")],
    "conjugated_phase": [("cos(theta), sin(theta)", "cos(theta), -sin(theta)")],
    "qft_no_bit_reversal": [("<< (n - 1 - b);", "<< b;")],
    "norm_drops_imag": [("+ psi[2 * i + 1] * psi[2 * i + 1];", ";")],
    "probs_drops_imag": [("out[i] = re * re + im * im;", "out[i] = re * re;")],
    "probs_ignores_first": [("double re = psi[2 * (first + i)], im = psi[2 * (first + i) + 1];",
                             "double re = psi[2 * i], im = psi[2 * i + 1];")],
    "mcu_any_control": [("if ((k & cmask) == cmask)", "if (k & cmask)")],
    "unitary_transposed": [("double ur = U[2 * (r * D + c)], ui = U[2 * (r * D + c) + 1];",
                            "double ur = U[2 * (c * D + r)], ui = U[2 * (c * D + r) + 1];")],
    "unitary_qubits_reversed": [("off[c] |= (uint64_t)1 << q[m];",
                                 "off[c] |= (uint64_t)1 << q[k - 1 - m];")],
    "unitary_conjugated": [("im += ur * a[2 * c + 1] + ui * a[2 * c];",
                            "im += ur * a[2 * c + 1] - ui * a[2 * c];")],
}

PINS = [
    pins.test_pauli_x_and_hadamard_worked_values,
    pins.test_cnot_printed_matrix_and_truth_table,
    pins.test_two_qubit_tensor_example,
    pins.test_n3_pairing_strides_and_locality,
    pins.test_qft_two_qubit_hand_values,
    lambda: pins.test_qft_stride_tier_matches_closed_form(5),
    lambda: pins.test_stride_tier_matches_dense_tier(5),
    pins.test_layer_and_qft_circuits_match_dense_tier,
    pins.test_product_state_rule,
    pins.test_norm_and_probs_against_exact_sums,
    pins.test_probabilities_of_circuit_results_sum_to_one,
    lambda: pins.test_qft_probabilities_are_uniform(8),
    pins.test_product_state_probabilities_factorise,
    pins.test_controlled_gate_leaves_control_zero_half_untouched,
    pins.test_toffoli_truth_table,
    lambda: pins.test_mcu_stride_tier_matches_dense_tier((0, 2, 4), 5),
    pins.test_unitary_on_one_qubit_is_the_stride_update,
    pins.test_unitary_tensor_product_of_one_qubit_gates,
    pins.test_unitary_cnot_matrix_is_the_controlled_x,
    lambda: pins.test_unitary_stride_tier_matches_dense_tier((6, 2, 4, 1)),
]


def _build_mutant(tmp_path, name, edits):
    with open(build_oracle.SRC) as f:
        src = f.read()
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    c = os.path.join(tmp_path, f"{name}.c")
    so = os.path.join(tmp_path, f"{name}.so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", so, c, "-lm"], check=True)
    return so


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    so = _build_mutant(str(tmp_path), name, MUTANTS[name])
    real = oracle.lib()
    failed = []
    try:
        oracle._lib = oracle.load(so)
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                failed.append(getattr(pin, "__name__", "lambda"))
    finally:
        oracle._lib = real
    assert failed, f"mutant {name} passed every pin"


def test_real_oracle_passes_the_same_pins():
    for pin in PINS:
        pin()
