"""Pins of the FP64 oracle against things other than itself.

* values the paper prints for its worked examples (tests/golden),
* brute-force dense Kronecker operators (numpy, no index arithmetic),
* the paper's own method: a sparse I_l (x) U' (x) I_r (scipy.sparse),
* closed forms (GHZ, QFT of a basis state, QFT = sqrt(N) * inverse FFT,
  TFIM energies of product states, gradients of one-qubit circuits),
* invariants (norm, U U^dagger = I, circuit then inverse, sum of p = 1).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import workloads as W
from dense_ref import (dense_gate, dense_pauli, random_state, random_unitary)

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def cplx(lst):
    return np.array([complex(a, b) for a, b in lst])


def tol(ex):
    return 0.5 * 10.0 ** (-ex["printed_digits"]) + 1e-12


# ------------------------------------------------------------- paper examples

def test_paper_bell():
    ex = GOLD["bell"]
    br = oracle.simulate(2, [W.Op("H", (0,)), W.Op("CNOT", (0, 1)), ("M", 0), ("M", 1)],
                         ex["init"])
    assert [b[0] for b in br] == ex["results"]
    np.testing.assert_allclose([b[1] for b in br], ex["probabilities"], atol=tol(ex))
    for (_, _, s), ref in zip(br, ex["states"]):
        np.testing.assert_allclose(s, cplx(ref), atol=tol(ex))


def _teleport_init():
    v = np.array([1.0, 1j]) / math.sqrt(2.0)
    bell = np.array([1.0, 0, 0, 1.0]) / math.sqrt(2.0)
    return np.kron(v, bell)


def test_paper_teleportation():
    ex = GOLD["teleportation"]
    br = oracle.simulate(3, W.teleportation(), _teleport_init())
    assert [b[0] for b in br] == ex["results"]
    np.testing.assert_allclose([b[1] for b in br], ex["probabilities"], atol=tol(ex))
    np.testing.assert_allclose(br[0][2], cplx(ex["state_00"]), atol=tol(ex))
    red = oracle.reduced_statevector(br[0][2], ex["reduced_00_known_qubits"], br[0][0])
    np.testing.assert_allclose(red, cplx(ex["reduced_00"]), atol=tol(ex))
    # every branch teleports v onto qubit 2 exactly (the corrections undo the
    # Pauli frame), which pins CNOT/CZ directions and the qubit order
    v = np.array([1.0, 1j]) / math.sqrt(2.0)
    for res, _, s in br:
        np.testing.assert_allclose(oracle.reduced_statevector(s, [0, 1], res), v, atol=1e-14)


def test_paper_tomography_exact_part():
    ex = GOLD["tomography"]
    v = np.array([1.0, 1j]) / math.sqrt(2.0)
    bx = oracle.simulate(1, [("M", 0, "x")], v)
    probs = {r: p for r, p, _ in bx}
    assert abs(probs["0"] - ex["px0"]) < 1e-14 and abs(probs["1"] - ex["px1"]) < 1e-14
    by = oracle.simulate(1, [("M", 0, "y")], v)
    assert [r for r, _, _ in by] == ["0"] and abs(by[0][1] - 1.0) < 1e-14
    # the reconstruction formula with exact coefficients gives rho_v
    sx = oracle.expect_pauli(v, "X").real
    sy = oracle.expect_pauli(v, "Y").real
    sz = oracle.expect_pauli(v, "Z").real
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1, -1])
    rho = 0.5 * (np.eye(2) + sx * X + sy * Y + sz * Z)
    ref = np.array([[complex(*e) for e in row] for row in ex["rho_v"]])
    np.testing.assert_allclose(rho, ref, atol=1e-14)
    # the same coefficients are the basis-measurement differences
    assert abs(sx - (probs["0"] - probs["1"])) < 1e-14
    assert abs(sy - 1.0) < 1e-14


def test_paper_grover():
    ex = GOLD["grover"]
    br = oracle.simulate(2, W.grover2("11"), ex["init"])
    assert [b[0] for b in br] == ex["results"]
    np.testing.assert_allclose([b[1] for b in br], ex["probabilities"], atol=1e-14)
    # one Grover iteration finds any marked state of N = 4 with certainty
    for marked in ("00", "01", "10", "11"):
        br = oracle.simulate(2, W.grover2(marked), "00")
        assert [b[0] for b in br] == [marked] and abs(br[0][1] - 1.0) < 1e-14


def test_paper_qec():
    ex = GOLD["qec"]
    v = np.array([1.0, 1j]) / math.sqrt(2.0)
    init = np.kron(v, np.eye(16)[:, 0])
    br = oracle.simulate(5, W.bitflip_code(error_qubit=0), init)
    assert [b[0] for b in br] == ex["results"]
    np.testing.assert_allclose([b[1] for b in br], ex["probabilities"], atol=1e-14)
    # closed form of this circuit: the error on q0 is undone, leaving
    # (|000> + i|111>)/sqrt2 on q0..q2 with both ancillas in |1>
    ref = np.zeros(32, dtype=complex)
    ref[0b00011] = 1 / math.sqrt(2)
    ref[0b11111] = 1j / math.sqrt(2)
    np.testing.assert_allclose(br[0][2], ref, atol=1e-14)


def test_bitflip_code_corrects_every_single_error():
    # syndrome (parity q0q1, parity q0q2) names the flipped qubit; after the
    # correction the encoded state is (|000> + i|111>)/sqrt2 whatever the error
    v = np.array([1.0, 1j]) / math.sqrt(2.0)
    init = np.kron(v, np.eye(16)[:, 0])
    syndromes = {None: "00", 0: "11", 1: "10", 2: "01"}
    for err, syn in syndromes.items():
        br = oracle.simulate(5, W.bitflip_code(error_qubit=err), init)
        assert [b[0] for b in br] == [syn] and abs(br[0][1] - 1.0) < 1e-14
        anc = int(syn, 2)
        ref = np.zeros(32, dtype=complex)
        ref[anc] = 1 / math.sqrt(2)
        ref[0b11100 | anc] = 1j / math.sqrt(2)
        np.testing.assert_allclose(br[0][2], ref, atol=1e-14)


# ------------------------------------------------ measurement bases and reset

def test_custom_basis_h_is_the_x_basis():
    # sections 2 and 3.3: a custom basis change V = H is the preconfigured
    # X-basis measurement: same outcomes, probabilities and post-states
    rng = np.random.default_rng(41)
    psi = random_state(3, rng)
    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2.0)
    for q in range(3):
        a = oracle.simulate(3, [("M", q, "x")], psi)
        b = oracle.simulate(3, [("M", q, H)], psi)
        assert [r for r, _, _ in a] == [r for r, _, _ in b]
        for (_, pa, sa), (_, pb, sb) in zip(a, b):
            assert abs(pa - pb) < 1e-15
            np.testing.assert_allclose(sa, sb, atol=1e-15)
        # X-basis probabilities are the |+>/|-> projections, from dense algebra
        plus = np.array([1, 1]) / math.sqrt(2.0)
        proj = dense_gate(3, [q], np.outer(plus, plus))
        assert abs(a[0][1] - np.vdot(psi, proj @ psi).real) < 1e-14


def test_custom_basis_hsdg_gives_tomography_s2():
    # section 5.2: v = (1, i)/sqrt2 measured in the Y basis gives 0 with
    # certainty, so S_2 = P(0) - P(1) = 1; a custom V = H S^dagger (the
    # matrix product, built here from its factors) reproduces it
    v = np.array([1.0, 1j]) / math.sqrt(2.0)
    Hm = np.array([[1, 1], [1, -1]]) / math.sqrt(2.0)
    Sdg = np.diag([1, -1j])
    br = oracle.simulate(1, [("M", 0, Hm @ Sdg)], v)
    p = {r: pr for r, pr, _ in br}
    assert abs(p.get("0", 0.0) - p.get("1", 0.0) - 1.0) < 1e-14
    # the basis change is reverted after the measurement: the branch state
    # is the Y eigenvector again
    np.testing.assert_allclose(br[0][2], v, atol=1e-15)
    # a basis V whose rows are arbitrary orthonormal vectors: P(b) = |<row_b|v>|^2
    rng = np.random.default_rng(43)
    V = random_unitary(2, rng)
    br = oracle.simulate(1, [("M", 0, V)], v)
    for r, pr, _ in br:
        assert abs(pr - abs(V[int(r)] @ v) ** 2) < 1e-14


def test_reset_bell_branches():
    # section 3.3 resets: reset q0 of (|00> + |11>)/sqrt2.  Outcome 0 (p 1/2)
    # leaves |00>; outcome 1 (p 1/2) collapses to |11> and flips q0 back: |01>
    bell = np.array([1, 0, 0, 1]) / math.sqrt(2.0)
    br = oracle.simulate(2, [("R", 0)], bell)
    assert [r for r, _, _ in br] == ["0", "1"]
    np.testing.assert_allclose([p for _, p, _ in br], [0.5, 0.5], atol=1e-15)
    np.testing.assert_allclose(br[0][2], [1, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(br[1][2], [0, 1, 0, 0], atol=1e-15)
    # a reset qubit reads 0 with certainty in every branch, for any state
    psi = random_state(4, np.random.default_rng(44))
    for q in range(4):
        for _, _, s in oracle.simulate(4, [("R", q)], psi):
            assert abs(oracle.probs(s, [q])[0] - 1.0) < 1e-14
    # reset of a qubit already in |0> is one branch with the state unchanged
    prod = np.kron([1, 0], random_state(2, np.random.default_rng(45)))
    br = oracle.simulate(3, [("R", 0)], prod)
    assert len(br) == 1 and abs(br[0][1] - 1.0) < 1e-14
    np.testing.assert_allclose(br[0][2], prod, atol=1e-15)


def test_counts_over_measured_qubits():
    # section 5.2 counts: shots recorded under the values of the listed
    # qubits; a product state |1>|+>|0> gives "10"/"11" half each on (0, 1)
    n = 3
    plus = np.array([1, 1]) / math.sqrt(2.0)
    psi = np.kron(np.kron([0, 1], plus), [1, 0]).astype(complex)
    u = (np.arange(1000) + 0.5) / 1000
    c = oracle.counts(psi, [0, 1], u)
    assert list(c) == [0, 0, 500, 500]
    # listing order sets the bit order of the outcome
    assert list(oracle.counts(psi, [1, 0], u)) == [0, 500, 0, 500]
    assert int(oracle.counts(psi, [2], u)[0]) == 1000 and n == 3


def test_open_control_only_fires_on_zero():
    # MCX with control value 0 acts exactly when that control reads 0
    for c0 in (0, 1):
        for c1 in (0, 1):
            psi = oracle.basis_state(3, f"{c0}{c1}0")
            out = oracle.run([W.Op("MCX", (0, 1, 2), ctrl_val=(0, 1))], psi)
            flip = (c0 == 0 and c1 == 1)
            assert np.argmax(np.abs(out)) == int(f"{c0}{c1}{int(flip)}", 2)


# ------------------------------------------------------- dense Kronecker pins

@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_1q_every_target_vs_dense(n):
    rng = np.random.default_rng(100 + n)
    psi = random_state(n, rng)
    for q in range(n):
        u = random_unitary(2, rng)
        np.testing.assert_allclose(oracle.apply(psi, [q], u), dense_gate(n, [q], u) @ psi,
                                   atol=1e-13)


def test_2q_every_ordered_pair_vs_dense():
    n = 5
    rng = np.random.default_rng(7)
    psi = random_state(n, rng)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            u = random_unitary(4, rng)
            np.testing.assert_allclose(oracle.apply(psi, [a, b], u),
                                       dense_gate(n, [a, b], u) @ psi, atol=1e-13)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_kq_random_qubit_lists_vs_dense(k):
    n = 7
    rng = np.random.default_rng(30 + k)
    psi = random_state(n, rng)
    for _ in range(4):
        qs = list(rng.permutation(n)[:k])
        u = random_unitary(1 << k, rng)
        np.testing.assert_allclose(oracle.apply(psi, qs, u), dense_gate(n, qs, u) @ psi,
                                   atol=1e-12)


def test_controlled_all_values_vs_dense():
    n = 5
    rng = np.random.default_rng(11)
    psi = random_state(n, rng)
    for nc in (1, 2, 3):
        for vals in range(1 << nc):
            perm = list(rng.permutation(n))
            ctrl, t = perm[:nc], perm[nc]
            cv = [(vals >> j) & 1 for j in range(nc)]
            u = random_unitary(2, rng)
            np.testing.assert_allclose(oracle.apply(psi, [t], u, ctrl, cv),
                                       dense_gate(n, [t], u, ctrl, cv) @ psi, atol=1e-13)
    # a controlled two-qubit gate
    u = random_unitary(4, rng)
    np.testing.assert_allclose(oracle.apply(psi, [4, 1], u, [2], [1]),
                               dense_gate(n, [4, 1], u, [2], [1]) @ psi, atol=1e-13)


def test_gate_library_vs_definitions():
    """Every named one-qubit matrix of the oracle's gate library against its
    definition from the Pauli matrices: R_P(t) = exp(-i t P / 2) by scipy's
    matrix exponential, H = (X + Z)/sqrt2, S = exp(i pi/4 (I - Z)),
    P(phi) = exp(i phi (I - Z)/2), SWAP = (I I + X X + Y Y + Z Z)/2."""
    from scipy.linalg import expm
    from dense_ref import PAULI
    I, X, Y, Z = (PAULI[c] for c in "IXYZ")
    for k in "IXYZ":
        np.testing.assert_allclose(oracle.gate_matrix(k), PAULI[k], atol=0)
    np.testing.assert_allclose(oracle.gate_matrix("H"), (X + Z) / math.sqrt(2.0), atol=1e-16)
    S = expm(0.25j * math.pi * (I - Z))
    np.testing.assert_allclose(oracle.gate_matrix("S"), S, atol=1e-15)
    np.testing.assert_allclose(oracle.gate_matrix("SDG"), S.conj().T, atol=1e-15)
    for t in (0.0, 0.37, -1.2, 2.9, 5.5, 2 * math.pi):
        for k, P in (("RX", X), ("RY", Y), ("RZ", Z)):
            np.testing.assert_allclose(oracle.gate_matrix(k, t), expm(-0.5j * t * P), atol=1e-15)
        np.testing.assert_allclose(oracle.gate_matrix("P", t), expm(0.5j * t * (I - Z)),
                                   atol=1e-15)
    swap = 0.5 * sum(np.kron(PAULI[c], PAULI[c]) for c in "IXYZ")
    np.testing.assert_allclose(oracle.gate_matrix("SWAP"), swap, atol=1e-16)


def test_every_gate_kind_through_run_vs_dense():
    """run() on each kind it accepts, against the dense register operator of
    the gate's definition (controls as projectors, section 3.2)."""
    from scipy.linalg import expm
    from dense_ref import PAULI
    I, X, Y, Z = (PAULI[c] for c in "IXYZ")
    n = 4
    psi = random_state(n, np.random.default_rng(6))
    u = random_unitary(4, np.random.default_rng(7))
    t = 0.83
    cases = [
        (W.Op("I", (1,)), dense_gate(n, [1], I)),
        (W.Op("X", (2,)), dense_gate(n, [2], X)),
        (W.Op("Y", (0,)), dense_gate(n, [0], Y)),
        (W.Op("Z", (3,)), dense_gate(n, [3], Z)),
        (W.Op("H", (1,)), dense_gate(n, [1], (X + Z) / math.sqrt(2.0))),
        (W.Op("S", (2,)), dense_gate(n, [2], expm(0.25j * math.pi * (I - Z)))),
        (W.Op("SDG", (0,)), dense_gate(n, [0], expm(-0.25j * math.pi * (I - Z)))),
        (W.Op("RX", (3,), angle=t), dense_gate(n, [3], expm(-0.5j * t * X))),
        (W.Op("RY", (1,), pidx=0), dense_gate(n, [1], expm(-0.5j * t * Y))),
        (W.Op("RZ", (2,), pidx=0), dense_gate(n, [2], expm(-0.5j * t * Z))),
        (W.Op("P", (0,), angle=t), dense_gate(n, [0], expm(0.5j * t * (I - Z)))),
        (W.Op("CP", (3, 0), angle=t), dense_gate(n, [0], expm(0.5j * t * (I - Z)), [3], [1])),
        (W.Op("MCX", (0, 2, 1), ctrl_val=(1, 0)), dense_gate(n, [1], X, [0, 2], [1, 0])),
        (W.Op("U", (2, 0), matrix=u), dense_gate(n, [2, 0], u)),
    ]
    for op, mat in cases:
        np.testing.assert_allclose(oracle.run([op], psi, np.array([t])), mat @ psi, atol=1e-13)


def test_named_gates_vs_dense():
    n = 4
    rng = np.random.default_rng(5)
    psi = random_state(n, rng)
    X = np.array([[0, 1], [1, 0]])
    Z = np.diag([1.0, -1.0])
    cases = [
        (W.Op("CNOT", (2, 0)), dense_gate(n, [0], X, [2], [1])),
        (W.Op("CNOT", (0, 2)), dense_gate(n, [2], X, [0], [1])),
        (W.Op("CZ", (3, 1)), dense_gate(n, [1], Z, [3], [1])),
        (W.Op("CP", (1, 3), angle=0.3), dense_gate(n, [3], np.diag([1, np.exp(0.3j)]), [1], [1])),
        (W.Op("SWAP", (0, 3)), dense_gate(n, [0, 3], np.eye(4)[[0, 2, 1, 3]])),
        (W.Op("RY", (2,), angle=0.7),
         dense_gate(n, [2], np.array([[math.cos(.35), -math.sin(.35)],
                                      [math.sin(.35), math.cos(.35)]]))),
        (W.Op("RZ", (1,), angle=0.7), dense_gate(n, [1], np.diag([np.exp(-.35j), np.exp(.35j)]))),
    ]
    for op, mat in cases:
        np.testing.assert_allclose(oracle.run([op], psi), mat @ psi, atol=1e-13)
    # CZ is symmetric in its qubits
    np.testing.assert_allclose(oracle.run([W.Op("CZ", (1, 3))], psi),
                               oracle.run([W.Op("CZ", (3, 1))], psi), atol=0)


# ------------------------------------------------- the paper's sparse method

@pytest.mark.parametrize("n,k", [(10, 1), (12, 2), (14, 3)])
def test_vs_paper_sparse_kron(n, k):
    """Section 3.2: U = I_l (x) U' (x) I_r as a sparse matrix times psi, for
    gates on contiguous qubits a..a+k-1."""
    rng = np.random.default_rng(1000 + n)
    psi = random_state(n, rng)
    for a in (0, n // 2, n - k):
        u = random_unitary(1 << k, rng)
        big = sp.kron(sp.kron(sp.identity(1 << a), sp.csr_matrix(u)),
                      sp.identity(1 << (n - a - k)), format="csr")
        np.testing.assert_allclose(oracle.apply(psi, list(range(a, a + k)), u), big @ psi,
                                   atol=1e-13)


# ------------------------------------------------------------- closed forms

def test_ghz_closed_form():
    n = 12
    out = oracle.run(W.ghz(n), oracle.basis_state(n, 0))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    np.testing.assert_allclose(out, ref, atol=1e-15)
    np.testing.assert_allclose(oracle.probs(out, [0]), [0.5, 0.5], atol=1e-15)


@pytest.mark.parametrize("n", [3, 8, 12])
def test_qft_is_scaled_inverse_fft(n):
    psi = W.random_state(n, seed=n)
    out = oracle.run(W.qft(n), psi)
    np.testing.assert_allclose(out, np.fft.ifft(psi) * math.sqrt(1 << n), atol=1e-13)
    for y in (0, 1, (1 << n) - 1, 5 % (1 << n)):
        assert abs(oracle.qft_amplitude(psi, y) - out[y]) < 1e-13


def test_qft_basis_state_closed_form():
    n = 9
    N = 1 << n
    for x in (0, 1, 77, N - 1):
        out = oracle.run(W.qft(n), oracle.basis_state(n, x))
        ref = np.exp(2j * math.pi * x * np.arange(N) / N) / math.sqrt(N)
        np.testing.assert_allclose(out, ref, atol=1e-13)


def test_brickwork_norm_and_inverse():
    n = 10
    ops = W.brickwork(n, 6, seed=3, entangler="CNOT") + W.brickwork(n, 3, seed=4, entangler="CZ")
    psi0 = oracle.basis_state(n, 0)
    psi = oracle.run(ops, psi0)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-13
    # circuit followed by its inverse (reversed order, adjoint matrices)
    for op in reversed(ops):
        if op.kind == "U":
            psi = oracle.apply(psi, op.qubits, op.matrix.conj().T)
        else:  # CNOT and CZ are their own inverses
            psi = oracle.run([op], psi)
    np.testing.assert_allclose(psi, psi0, atol=1e-12)


def test_haar_inputs_are_unitary():
    rng = np.random.default_rng(0)
    for _ in range(50):
        u = W.haar_u2(rng)
        np.testing.assert_allclose(u @ u.conj().T, np.eye(2), atol=1e-14)


# ------------------------------------------------------------ probabilities

def test_probs_sum_and_marginals_vs_reshape():
    n = 9
    rng = np.random.default_rng(9)
    psi = random_state(n, rng)
    p = oracle.probs(psi)
    assert abs(p.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(p, np.abs(psi) ** 2, atol=1e-16)
    t = (np.abs(psi) ** 2).reshape([2] * n)   # axis q is qubit q
    for qs in ([0], [8], [3, 1], [2, 7, 5], [0, 1, 2, 3, 4, 5, 6, 7]):
        other = tuple(a for a in range(n) if a not in qs)
        # first listed qubit is the most significant bit of the outcome
        ref = t.sum(axis=other)
        order = sorted(qs)
        ref = np.transpose(ref, [order.index(q) for q in qs]).reshape(-1)
        np.testing.assert_allclose(oracle.probs(psi, qs), ref, atol=1e-15)


def test_collapse_renormalises():
    n = 6
    psi = random_state(n, np.random.default_rng(2))
    p1 = oracle.probs(psi, [2])[1]
    post, pr = oracle.collapse(psi, 2, 1)
    assert abs(pr - p1) < 1e-15
    assert abs(np.vdot(post, post).real - 1.0) < 1e-14
    assert abs(oracle.probs(post, [2])[1] - 1.0) < 1e-14


# --------------------------------------------------------------- expectation

def test_expect_pauli_vs_dense():
    n = 5
    rng = np.random.default_rng(21)
    psi = random_state(n, rng)
    for _ in range(30):
        p = "".join(rng.choice(list("IXYZ"), n))
        ref = np.vdot(psi, dense_pauli(p) @ psi)
        got = oracle.expect_pauli(psi, p)
        assert abs(got - ref) < 1e-14
        assert abs(got.imag) < 1e-14   # Pauli strings are Hermitian


def test_tfim_product_state_closed_forms():
    n = 10
    terms = W.tfim_terms(n)
    zero = oracle.basis_state(n, 0)
    assert abs(oracle.energy(zero, terms) + (n - 1)) < 1e-13
    plus = np.full(1 << n, 1 / math.sqrt(1 << n), dtype=complex)
    assert abs(oracle.energy(plus, terms) + n) < 1e-12


def test_tfim_energy_above_ground_state():
    n = 10
    terms = W.tfim_terms(n)
    H = sum(c * sp.csr_matrix(dense_pauli(p)) for p, c in terms)
    e0 = spla.eigsh(H, k=1, which="SA")[0][0]
    theta = np.random.default_rng(3).uniform(0, 2 * math.pi, 2 * n * 2)
    psi = oracle.run(W.hea(n, 2), oracle.basis_state(n, 0), theta)
    e = oracle.energy(psi, terms)
    assert e >= e0 - 1e-10
    assert abs(e - np.vdot(psi, H @ psi).real) < 1e-12


# ---------------------------------------------------------------- gradients

def test_gradient_one_qubit_closed_forms():
    # RY(a) then RZ(b) on |0>, H = -X: E = -sin a cos b
    ops = [W.Op("RY", (0,), pidx=0), W.Op("RZ", (0,), pidx=1)]
    terms = [("X", -1.0)]
    for a, b in [(0.3, 0.0), (1.1, 0.4), (2.5, -1.3)]:
        th = np.array([a, b])
        e = oracle.energy(oracle.run(ops, oracle.basis_state(1, 0), th), terms)
        assert abs(e + math.sin(a) * math.cos(b)) < 1e-14
        g = oracle.param_shift_grad(ops, th, terms, oracle.basis_state(1, 0))
        np.testing.assert_allclose(g, [-math.cos(a) * math.cos(b), math.sin(a) * math.sin(b)],
                                   atol=1e-14)


def test_parameter_shift_vs_finite_differences():
    n = 4
    ops = W.hea(n, 2)
    terms = W.tfim_terms(n)
    theta = np.random.default_rng(8).uniform(0, 2 * math.pi, 2 * n * 2)
    psi0 = oracle.basis_state(n, 0)
    g_ps = oracle.param_shift_grad(ops, theta, terms, psi0)
    g_fd = oracle.fd_grad(ops, theta, terms, psi0, eps=1e-5)
    np.testing.assert_allclose(g_ps, g_fd, atol=1e-8)


def test_sampling_closed_forms():
    n = 6
    N = 1 << n
    # a basis state always yields its own index
    assert np.all(oracle.sample(oracle.basis_state(n, 37), np.linspace(0, 0.999, 50)) == 37)
    # the uniform superposition maps u in [k/N, (k+1)/N) to k
    plus = np.full(N, 1 / math.sqrt(N), dtype=complex)
    u = (np.arange(N) + 0.5) / N
    assert np.array_equal(oracle.sample(plus, u), np.arange(N))
    # empirical frequencies converge to |psi|^2 (chi-square, 63 dof)
    psi = random_state(n, np.random.default_rng(4))
    idx = oracle.sample(psi, np.random.default_rng(5).uniform(size=200000))
    counts = np.bincount(idx, minlength=N)
    exp = 200000 * np.abs(psi) ** 2
    chi2 = np.sum((counts - exp) ** 2 / exp)
    assert chi2 < 120   # p ~ 1e-5 for 63 degrees of freedom
    # zero-probability indices are never drawn
    half = np.zeros(N, dtype=complex)
    half[::2] = 1 / math.sqrt(N / 2)
    assert np.all(oracle.sample(half, np.random.default_rng(6).uniform(size=1000)) % 2 == 0)


def test_oracle_rejects_bad_arguments():
    psi = oracle.basis_state(3, 0)
    with pytest.raises(ValueError):
        oracle.apply(psi, [0, 0], np.eye(4))
    with pytest.raises(ValueError):
        oracle.apply(psi, [3], np.eye(2))
    with pytest.raises(ValueError):
        oracle.apply(psi, [1], np.eye(2), [1], [1])
