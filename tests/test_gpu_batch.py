"""Batched persistent launch (qc_run_batch) against the FP64 oracle.

Energies are compared with |dE| <= 2 ||H|| * state error (||H|| <= 2n - 1
for the transverse-field Ising chain); states of complex64 runs with the
relative 2-norm bound 1e-5, complex128 with max-abs 1e-12.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2503_03016_amd import qc as mod
    return mod


@pytest.fixture(scope="module")
def G():
    from paper_2503_03016_amd import gates
    return gates


def hea_circuit(G, n, theta, layers):
    ops = W.hea(n, layers)
    return ops, (n, G.gate_tuples(ops, theta), W.tfim_terms(n))


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_batch_mixed_sizes_states_and_energies(qc, G, dtype):
    rng = np.random.default_rng(7)
    sizes = [3, 5, 8, 11, 12, 13, 14, 15, 16, 9, 13, 14]
    layers = 3
    circuits, refs = [], []
    for n in sizes:
        theta = rng.uniform(0, 2 * math.pi, layers * n * 2)
        ops, c = hea_circuit(G, n, theta, layers)
        circuits.append(c)
        psi = oracle.run(ops, oracle.basis_state(n, 0), theta)
        refs.append((psi, oracle.energy(psi, c[2])))
    b = qc.Batch(circuits, dtype=dtype, keep_states=True)
    e = b.run().cpu().numpy()
    assert b.status() == 0
    for i, (n, (psi, eref)) in enumerate(zip(sizes, refs)):
        got = b.state(i).cpu().numpy().astype(np.complex128)
        if dtype == torch.complex128:
            assert np.max(np.abs(got - psi)) < 1e-12, (i, n)
            assert abs(e[i] - eref) < 1e-11 * (2 * n - 1), (i, n)
        else:
            rel = np.linalg.norm(got - psi) / np.linalg.norm(psi)
            assert rel < 1e-5, (i, n, rel)
            assert abs(e[i] - eref) < 2 * (2 * n - 1) * 1e-5, (i, n)


def test_batch_general_gates_and_terms(qc, G):
    """Dense 1q/2q gates, controls (open and closed), phases, Y terms, and
    QFT circuits (controlled-phase fans, SWAPs)."""
    rng = np.random.default_rng(3)
    from dense_ref import random_unitary
    circuits, refs = [], []
    for n in (6, 13, 15):
        ops = []
        for _ in range(40):
            q = [int(x) for x in rng.permutation(n)[:3]]
            k = rng.integers(0, 4)
            if k == 0:
                ops.append(W.Op("U", (q[0],), matrix=random_unitary(2, rng)))
            elif k == 1:
                ops.append(W.Op("U", (q[0], q[1]), matrix=random_unitary(4, rng)))
            elif k == 2:
                ops.append(W.Op("MCX", (q[0], q[1], q[2]), ctrl_val=(0, 1)))
            else:
                ops.append(W.Op("CP", (q[0], q[1]), angle=0.4))
        terms = [("".join(rng.choice(list("IXYZ"), n)), float(rng.normal())) for _ in range(9)]
        circuits.append((n, G.gate_tuples(ops), terms))
        psi = oracle.run(ops, oracle.basis_state(n, 0))
        refs.append(oracle.energy(psi, terms))
        # a QFT after a layer of random one-qubit gates: controlled-phase
        # fans and SWAPs inside the batch kernel
        rq = np.random.default_rng(30 + n)   # its own stream: the draws above stay as they were
        qops = [W.Op("U", (q,), matrix=random_unitary(2, rq)) for q in range(n)] + W.qft(n)
        circuits.append((n, G.gate_tuples(qops), W.tfim_terms(n)))
        refs.append(oracle.energy(oracle.run(qops, oracle.basis_state(n, 0)), W.tfim_terms(n)))
    b = qc.Batch(circuits, dtype=torch.complex128)
    e = b.run().cpu().numpy()
    assert b.status() == 0
    np.testing.assert_allclose(e, refs, atol=1e-11)


def test_batch512_config_sampled(qc, G):
    """512 circuits, n uniform in [10, 20], 8-layer HEA, TFIM energies, one
    persistent launch in complex64; sampled circuits (the largest included)
    against the oracle, every energy above the chain's ground energy bound
    -(2n - 1), run-to-run bitwise determinism."""
    cfg = W.batch_config()
    circuits = [(n, G.gate_tuples(W.hea(n, 8), th), W.tfim_terms(n)) for n, th in cfg]
    b = qc.Batch(circuits, dtype=torch.complex64)
    e1 = b.run().cpu().numpy()
    assert b.status() == 0
    e2 = b.run().cpu().numpy()
    assert np.array_equal(e1, e2)
    ns = np.array([n for n, _ in cfg])
    assert np.all(np.isfinite(e1)) and np.all(e1 >= -(2 * ns - 1) - 1e-6)
    rng = np.random.default_rng(1)
    largest = [int(i) for i in np.where(ns == 20)[0][:2]]
    sample = sorted(set(largest + [int(i) for i in rng.choice(len(cfg), 6, replace=False)]))
    for i in sample:
        n, th = cfg[i]
        psi = oracle.run(W.hea(n, 8), oracle.basis_state(n, 0), th)
        eref = oracle.energy(psi, W.tfim_terms(n))
        assert abs(e1[i] - eref) < 2 * (2 * n - 1) * 1e-5, (i, n, e1[i], eref)


def test_batch_graph_capture_replay(qc, G):
    rng = np.random.default_rng(11)
    circuits = []
    for n in (10, 12, 14, 16, 11):
        theta = rng.uniform(0, 2 * math.pi, 2 * n * 2)
        circuits.append(hea_circuit(G, n, theta, 2)[1])
    b = qc.Batch(circuits, dtype=torch.complex64)
    eager = b.run().clone()
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(out)       # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(out)
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        del junk
