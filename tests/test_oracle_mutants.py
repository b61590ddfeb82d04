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
