"""Measurement on the GPU (collapse, reduced state, sampling, branching
simulation) against the oracle and the values the paper prints."""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2503_03016_amd import qc as mod
    return mod


def dev(psi, dtype):
    return torch.from_numpy(np.ascontiguousarray(psi)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_collapse_vs_oracle(qc, dtype):
    n = 13
    psi0 = W.random_state(n, 31)
    for q in (0, 6, 12):
        for b in (0, 1):
            t = dev(psi0, dtype)
            held = host(t)
            p = qc.collapse(t, q, b).item()
            ref, pref = oracle.collapse(held, q, b)
            assert abs(p - pref) < 1e-13
            tol = 1e-13 if dtype == torch.complex128 else 1e-6
            assert np.max(np.abs(host(t) - ref)) < tol
    # an impossible outcome leaves the state as it is
    t = dev(oracle.basis_state(n, 0), dtype)
    assert qc.collapse(t, 3, 1).item() == 0.0
    assert np.array_equal(host(t), oracle.basis_state(n, 0))


def test_reduced_state_vs_oracle(qc):
    n = 10
    psi0 = W.random_state(n, 8)
    t = dev(psi0, torch.complex128)
    for known, vals in (([2, 7], "10"), ([0], "1"), ([9, 3, 5], "011")):
        got = host(qc.reduced_state(t, known, [int(c) for c in vals]))
        np.testing.assert_allclose(got, oracle.reduced_statevector(psi0, known, vals), atol=0)


@pytest.mark.parametrize("n", [1, 3, 7, 11, 12, 15])
def test_sampling_vs_oracle(qc, n):
    psi0 = W.random_state(n, 44)
    t = dev(psi0, torch.complex128)
    u = np.random.default_rng(n).uniform(size=20000)
    got = qc.sample(t, torch.from_numpy(u).cuda()).cpu().numpy()
    ref = oracle.sample(psi0, u)
    # both sides decide in FP64; they may differ only where u sits on a CDF
    # boundary to within rounding
    cdf = np.cumsum(np.abs(psi0) ** 2)
    x = u * cdf[-1]
    mism = np.where(got != ref)[0]
    assert len(mism) <= 2
    for k in mism:
        r = int(ref[k])
        bounds = [cdf[r]] + ([cdf[r - 1]] if r > 0 else [])
        assert min(abs(x[k] - b) for b in bounds) < 1e-12, (k, got[k], r)


def test_sampling_statistics_and_zero_probabilities(qc):
    n = 12
    N = 1 << n
    v = np.zeros(N, dtype=complex)
    v[::3] = 1.0
    v /= np.linalg.norm(v)
    t = dev(v, torch.complex64)
    u = torch.from_numpy(np.random.default_rng(1).uniform(size=300000)).cuda()
    idx = qc.sample(t, u).cpu().numpy()
    assert np.all(idx % 3 == 0)
    counts = np.bincount(idx, minlength=N)[::3]
    exp = 300000 / len(counts)
    chi2 = np.sum((counts - exp) ** 2 / exp)
    dof = len(counts) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


def test_simulate_paper_examples_on_gpu(qc):
    from paper_2503_03016_amd.simulate import simulate
    ex = GOLD["bell"]
    br = simulate(2, [W.Op("H", (0,)), W.Op("CNOT", (0, 1)), ("M", 0), ("M", 1)], "00")
    assert [b[0] for b in br] == ex["results"]
    np.testing.assert_allclose([b[1] for b in br], ex["probabilities"], atol=1e-14)
    ex = GOLD["teleportation"]
    v = np.array([1.0, 1j]) / math.sqrt(2)
    init = np.kron(v, np.array([1.0, 0, 0, 1.0]) / math.sqrt(2))
    br = simulate(3, W.teleportation(), init)
    assert [b[0] for b in br] == ex["results"]
    np.testing.assert_allclose([b[1] for b in br], ex["probabilities"], atol=1e-14)
    ref = np.array([complex(a, b) for a, b in ex["state_00"]])
    np.testing.assert_allclose(host(br[0][2]), ref, atol=0.5e-4)
    for res, _, st in br:   # every branch carries v on qubit 2
        red = host(qc.reduced_state(st, [0, 1], [int(c) for c in res]))
        np.testing.assert_allclose(red, v, atol=1e-14)
    # tomography: X basis 0.5 / 0.5, Y basis certain
    bx = simulate(1, [("M", 0, "x")], v)
    np.testing.assert_allclose([b[1] for b in bx], [0.5, 0.5], atol=1e-14)
    by = simulate(1, [("M", 0, "y")], v)
    assert [b[0] for b in by] == ["0"] and abs(by[0][1] - 1) < 1e-14
    # error correction: syndrome '11' with probability 1
    init = np.kron(v, np.eye(16)[:, 0])
    items = W.bitflip_code(error_qubit=0)
    br = simulate(5, items, init)
    assert [b[0] for b in br] == GOLD["qec"]["results"]
    assert abs(br[0][1] - 1.0) < 1e-14
    # agreement with the oracle's own branching simulation
    ob = oracle.simulate(5, items, init)
    np.testing.assert_allclose(host(br[0][2]), ob[0][2], atol=1e-14)

    # Grover: every marked state of N = 4 found with probability 1
    for marked in ("00", "01", "10", "11"):
        br = simulate(2, W.grover2(marked), "00")
        assert [b[0] for b in br] == [marked] and abs(br[0][1] - 1.0) < 1e-14


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_reset_vs_oracle(qc, dtype):
    n = 13
    psi0 = W.random_state(n, 37)
    tol = 1e-13 if dtype == torch.complex128 else 1e-6
    for q in (0, 5, 12):
        for b in (0, 1):
            t = dev(psi0, dtype)
            held = host(t)
            p = qc.reset(t, q, b).item()
            ref, pref = oracle.reset(held, q, b)
            assert abs(p - pref) < 1e-13
            assert np.max(np.abs(host(t) - ref)) < tol
            # the qubit reads 0 with certainty afterwards
            assert abs(qc.probs(t, [q])[0].item() - 1.0) < (1e-13 if tol < 1e-10 else 1e-6)
    # an impossible outcome leaves the state unchanged and reports 0
    t = dev(oracle.basis_state(n, 0), dtype)
    assert qc.reset(t, 3, 1).item() == 0.0
    assert np.array_equal(host(t), oracle.basis_state(n, 0))


def test_simulate_reset_and_custom_basis_vs_oracle(qc):
    from paper_2503_03016_amd.simulate import simulate
    # reset of a Bell pair's first qubit: |00> and |01>, half each
    bell = np.array([1, 0, 0, 1]) / math.sqrt(2.0)
    br = simulate(2, [("R", 0)], bell)
    assert [b[0] for b in br] == ["0", "1"]
    np.testing.assert_allclose([b[1] for b in br], [0.5, 0.5], atol=1e-14)
    np.testing.assert_allclose(host(br[0][2]), [1, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(host(br[1][2]), [0, 1, 0, 0], atol=1e-15)
    # custom bases: V = H is the X basis; V = H S^dagger gives S_2 = 1 (5.2)
    v = np.array([1.0, 1j]) / math.sqrt(2)
    Hm = np.array([[1, 1], [1, -1]]) / math.sqrt(2.0)
    bx = simulate(1, [("M", 0, Hm)], v)
    np.testing.assert_allclose([b[1] for b in bx], [0.5, 0.5], atol=1e-14)
    by = simulate(1, [("M", 0, Hm @ np.diag([1, -1j]))], v)
    assert [b[0] for b in by] == ["0"] and abs(by[0][1] - 1) < 1e-14
    np.testing.assert_allclose(host(by[0][2]), v, atol=1e-15)
    # a mixed program of gates, custom-basis measurements and resets on 6
    # qubits, branch by branch against the oracle
    n = 6
    rng = np.random.default_rng(61)
    V = W.haar_u2(rng)
    items = (W.brickwork(n, 2, seed=62, entangler="CNOT") + [("M", 2, V), ("R", 4)] +
             W.brickwork(n, 1, seed=63, entangler="CZ") + [("M", 0, "y"), ("R", 2), ("M", 5, "x")])
    gb = simulate(n, items, 0)
    ob = oracle.simulate(n, items, 0)
    assert [b[0] for b in gb] == [b[0] for b in ob]
    for (_, pg, sg), (_, po, so) in zip(gb, ob):
        assert abs(pg - po) < 1e-13
        np.testing.assert_allclose(host(sg), so, atol=1e-12)


@pytest.mark.parametrize("n,qubits", [(7, [0]), (12, [3, 11, 0]), (15, [14, 2, 7, 9])])
def test_counts_vs_oracle(qc, n, qubits):
    psi0 = W.random_state(n, 70 + n)
    t = dev(psi0, torch.complex128)
    u = np.random.default_rng(n).uniform(size=50000)
    got = qc.counts(t, qubits, torch.from_numpy(u).cuda()).cpu().numpy()
    ref = oracle.counts(psi0, qubits, u)
    assert got.sum() == len(u)
    # shots may differ only where u sits on a CDF boundary (see sampling)
    assert np.abs(got - ref).sum() <= 4
    # and the per-shot indices agree with qc_sample, bit for bit, otherwise
    idx = qc.sample(t, torch.from_numpy(u).cuda()).cpu().numpy()
    out = np.zeros_like(idx)
    for q in qubits:
        out = 2 * out + ((idx >> (n - 1 - q)) & 1)
    assert np.array_equal(np.bincount(out, minlength=1 << len(qubits)), got)


def test_marginal_over_24_qubits(qc):
    # 26-qubit register, marginal over 24 listed qubits (2^24 bins)
    n = 26
    t = torch.zeros(1 << n, dtype=torch.complex64, device="cuda")
    rng = np.random.default_rng(26)
    idx = rng.choice(1 << n, size=4096, replace=False)
    vals = rng.standard_normal(4096) + 1j * rng.standard_normal(4096)
    vals /= np.linalg.norm(vals)
    t[torch.from_numpy(idx).cuda()] = torch.from_numpy(vals.astype(np.complex64)).cuda()
    qubits = [int(q) for q in rng.permutation(n)[:24]]
    got = qc.probs(t, qubits).cpu().numpy()
    full = np.zeros(1 << n, dtype=np.complex128)
    full[idx] = vals.astype(np.complex64)
    ref = oracle.probs(full, qubits)
    del full
    np.testing.assert_allclose(got, ref, atol=1e-12)
    assert abs(got.sum() - 1.0) < 1e-6
