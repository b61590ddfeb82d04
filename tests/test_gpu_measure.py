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
    items = [W.Op("CNOT", (0, 1)), W.Op("H", (0,)), ("M", 0), ("M", 1), W.Op("CNOT", (1, 2)),
             W.Op("CZ", (0, 2))]
    br = simulate(3, items, init)
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
    items = [W.Op("CNOT", (0, 1)), W.Op("CNOT", (0, 2)), W.Op("X", (0,)), W.Op("CNOT", (0, 3)),
             W.Op("CNOT", (1, 3)), W.Op("CNOT", (0, 4)), W.Op("CNOT", (2, 4)), ("M", 3), ("M", 4),
             W.Op("MCX", (3, 4, 2), ctrl_val=(0, 1)), W.Op("MCX", (3, 4, 1), ctrl_val=(1, 0)),
             W.Op("MCX", (3, 4, 0), ctrl_val=(1, 1))]
    br = simulate(5, items, init)
    assert [b[0] for b in br] == GOLD["qec"]["results"]
    assert abs(br[0][1] - 1.0) < 1e-14
    # agreement with the oracle's own branching simulation
    ob = oracle.simulate(5, items, init)
    np.testing.assert_allclose(host(br[0][2]), ob[0][2], atol=1e-14)
