"""The pins must catch plausible mistakes in the oracle.

Each case copies oracle.c, plants one mistake (a transposed operand, a
reversed bit order, an ignored control value, a dropped conjugate, a wrong
sign, a dropped term, a wrong normalisation), builds the mutant with gcc on
the CPU, swaps it in for the real library and checks that at least one pin
test fails.  Nothing here runs on a GPU.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "transposed_matrix": ("acc += u[r * d + t]", "acc += u[t * d + r]"),
    "bit_order_reversed": ("return (int)((i >> (n - 1 - q)) & 1u);",
                           "return (int)((i >> (q)) & 1u);"),
    "control_value_ignored": ("!= (ctrl_val[a] ? 1 : 0)", "!= 1"),
    "conjugate_dropped": ("cplx term = conj(psi[i]) * coef * psi[j];",
                          "cplx term = psi[i] * coef * psi[j];"),
    "pauli_y_sign": ("(row == 0 ? -I : I)", "(row == 0 ? I : -I)"),
    "imag_part_dropped": ("csum_add(&mine[read_local(i, n, m, qubits)], a * a + b * b);",
                          "csum_add(&mine[read_local(i, n, m, qubits)], a * a);"),
    "collapse_norm": ("1.0 / sqrt(pr[b])", "1.0 / pr[b]"),
}

PIN_TESTS = [
    pins.test_paper_bell,
    pins.test_paper_teleportation,
    pins.test_paper_tomography_exact_part,
    pins.test_paper_grover,
    pins.test_paper_qec,
    lambda: pins.test_1q_every_target_vs_dense(5),
    pins.test_2q_every_ordered_pair_vs_dense,
    pins.test_controlled_all_values_vs_dense,
    pins.test_probs_sum_and_marginals_vs_reshape,
    pins.test_expect_pauli_vs_dense,
    pins.test_collapse_renormalises,
    pins.test_tfim_product_state_closed_forms,
]


def _build_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site for %s not found exactly once" % name
    path = tmp_path / ("%s.c" % name)
    path.write_text(src.replace(old, new))
    so = tmp_path / ("lib%s.so" % name)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fcx-limited-range",
                           "-fPIC", "-shared", str(path), "-o", str(so), "-lm"])
    return str(so)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    so = _build_mutant(tmp_path, name, old, new)
    real = oracle._load()
    mut = ctypes.CDLL(so)
    for fn in ("oracle_apply", "oracle_probs", "oracle_expect_pauli", "oracle_collapse",
               "oracle_threads", "oracle_set_threads"):
        f, g = getattr(real, fn), getattr(mut, fn)
        g.argtypes, g.restype = f.argtypes, f.restype
    monkeypatch.setattr(oracle, "_lib", mut)
    failures = 0
    for t in PIN_TESTS:
        try:
            t()
        except (AssertionError, ValueError):
            failures += 1
    assert failures > 0, "no pin caught the planted mistake %s" % name


# ---- mistakes in the oracle's gate library (oracle/__init__.py) -------------

def _mutated_gate_matrix(real, kind_hit, change):
    def gm(kind, angle=None):
        m = real(kind, angle)
        return change(m) if kind == kind_hit else m
    return gm


GATE_MUTANTS = {
    # RX with the sign of its off-diagonal entries flipped: exp(+i t X/2)
    "rx_offdiag_sign": ("RX", lambda m: np.array([[m[0, 0], -m[0, 1]], [-m[1, 0], m[1, 1]]])),
    # RY transposed
    "ry_transposed": ("RY", lambda m: m.T.copy()),
    # RZ conjugated
    "rz_conjugated": ("RZ", lambda m: m.conj()),
    # Y with the wrong sign
    "y_sign": ("Y", lambda m: -m),
    # S and its adjoint swapped
    "s_conjugated": ("S", lambda m: m.conj()),
    "sdg_conjugated": ("SDG", lambda m: m.conj()),
    # phase gate conjugated
    "p_conjugated": ("P", lambda m: m.conj()),
    # H with its rows swapped
    "h_rows_swapped": ("H", lambda m: m[::-1].copy()),
    # X replaced by the identity
    "x_identity": ("X", lambda m: np.eye(2, dtype=complex)),
    # Z replaced by X
    "z_as_x": ("Z", lambda m: np.array([[0, 1], [1, 0]], dtype=complex)),
}

GATE_PIN_TESTS = [
    pins.test_gate_library_vs_definitions,
    pins.test_every_gate_kind_through_run_vs_dense,
    pins.test_named_gates_vs_dense,
    pins.test_paper_tomography_exact_part,
    pins.test_paper_grover,
    pins.test_paper_qec,
    pins.test_qft_basis_state_closed_form,
]


@pytest.mark.parametrize("name", sorted(GATE_MUTANTS))
def test_pins_catch_gate_library_mistake(name, monkeypatch):
    kind, change = GATE_MUTANTS[name]
    monkeypatch.setattr(oracle, "gate_matrix", _mutated_gate_matrix(oracle.gate_matrix, kind, change))
    failures = 0
    for t in GATE_PIN_TESTS:
        try:
            t()
        except (AssertionError, ValueError):
            failures += 1
    assert failures > 0, "no pin caught the planted gate-library mistake %s" % name
