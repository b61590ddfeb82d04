"""HIP-graph capture of gate, circuit, reduction and measurement calls.

After qc_reserve, a stream capture of qc_apply_circuit (fused and tiled),
qc_apply_1q, qc_probs and qc_expect_pauli records no allocation, memset or
host synchronisation; every replay, with unrelated eager library calls
between replays, must give the eager result bit for bit.
"""
import numpy as np
import pytest
import torch

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


@pytest.mark.parametrize("dt", [torch.complex64, torch.complex128])
def test_capture_replay_circuits_and_reductions(qc, G, dt):
    n = 16
    fused = qc.GateList(G.gate_tuples(W.brickwork(n, 6, seed=81, entangler="CZ")))
    tiled = qc.GateList(G.gate_tuples(W.qft(n)))
    u = W.haar_u2(np.random.default_rng(82))
    terms = W.tfim_terms(n)
    psi0 = torch.from_numpy(W.random_state(n, 83)).to(dt).cuda()

    def program(psi, p_out, e_out):
        qc.state_copy(psi, psi0)
        qc.apply_circuit(psi, fused, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        qc.apply_1q(psi, 3, u)
        qc.apply_circuit(psi, tiled, mode=qc.QC_EXEC_TILED)
        p_out.copy_(qc.probs(psi, [0, 5, 9]))
        e_out.copy_(qc.expect_pauli(psi, terms, per_term=True))

    eager_psi = qc.new_state(n, dt)
    eager_p = torch.empty(8, dtype=torch.float64, device="cuda")
    eager_e = torch.empty(1 + len(terms), dtype=torch.float64, device="cuda")
    program(eager_psi, eager_p, eager_e)
    torch.cuda.synchronize()

    psi = qc.new_state(n, dt)
    p_out = torch.empty_like(eager_p)
    e_out = torch.empty_like(eager_e)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        program(psi, p_out, e_out)    # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    qc.reserve()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        program(psi, p_out, e_out)
    other = qc.new_state(n, dt)
    for rep in range(3):
        psi.zero_()
        p_out.fill_(float("nan"))
        e_out.fill_(float("nan"))
        # eager library calls between replays take further ring slots
        qc.state_init(other, rep)
        qc.apply_circuit(other, fused, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        qc.apply_circuit(other, tiled, mode=qc.QC_EXEC_TILED)
        qc.probs(other, [1])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(psi, eager_psi), rep
        assert torch.equal(p_out, eager_p), rep
        assert torch.equal(e_out, eager_e), rep
    del g


def test_reserve_refused_while_capturing(qc):
    psi = qc.new_state(10, torch.complex64)
    qc.reserve()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g, stream=s):
        qc.state_init(psi, 0)
        try:
            qc.reserve()
        except qc.QcError as e:
            err = e
    assert err is not None and err.status == -4
    g.replay()
    torch.cuda.synchronize()
    assert psi[0].item() == 1
