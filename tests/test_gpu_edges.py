"""Edge cases and large sizes on the GPU: empty inputs, one-qubit
registers, controls on every other qubit, repeated qubits, and the
fused complex64 path against the unfused complex128 path near full size
(the unfused kernels themselves are oracle-checked at smaller sizes)."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from dense_ref import random_unitary

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


DT = {"c128": torch.complex128, "c64": torch.complex64}


def dev(psi, dtype):
    return torch.from_numpy(np.ascontiguousarray(psi)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_empty_gate_list_is_identity(qc, mode):
    psi0 = W.random_state(9, 1)
    t = dev(psi0, torch.complex128)
    st = qc.apply_circuit(t, qc.GateList([]), mode=mode, fuse_k=5)
    assert st["gates"] == 0 and st["launches"] == 0
    assert np.array_equal(host(t), psi0)


def test_one_qubit_register_everywhere(qc, G):
    v = np.array([0.6, 0.8j])
    u = random_unitary(2, np.random.default_rng(1))
    for dtype in (torch.complex64, torch.complex128):
        for mode in (0, 1, 2):
            t = dev(v, dtype)
            qc.apply_circuit(t, qc.GateList([((0,), (), (), u)]), mode=mode, fuse_k=5)
            np.testing.assert_allclose(host(t), u @ v, atol=1e-6)
        t = dev(v, dtype)
        np.testing.assert_allclose(qc.probs(t).cpu().numpy(), [0.36, 0.64], atol=1e-7)
        e = qc.expect_pauli(t, [("Z", 1.0), ("X", 2.0), ("Y", -1.0), ("I", 0.5)], per_term=True)
        e = e.cpu().numpy()
        ref = [oracle.expect_pauli(v, p).real for p in "ZXYI"]
        np.testing.assert_allclose(e[1:], ref, atol=1e-7)
        qc.state_init(t, 1)
        assert np.array_equal(host(t), [0, 1])


def test_controls_on_every_other_qubit(qc):
    n = 11
    psi0 = W.random_state(n, 4)
    rng = np.random.default_rng(2)
    u = random_unitary(2, rng)
    for tgt in (0, 5, 10):
        ctrl = [q for q in range(n) if q != tgt]
        cv = [int(x) for x in rng.integers(0, 2, n - 1)]
        t = dev(psi0, torch.complex128)
        qc.apply_controlled(t, ctrl, cv, tgt, u)
        np.testing.assert_allclose(host(t), oracle.apply(psi0, [tgt], u, ctrl, cv), atol=1e-12)
        # the phase-only path with every other qubit controlling
        ph = np.diag([1.0, np.exp(0.3j)])
        t = dev(psi0, torch.complex128)
        qc.apply_controlled(t, ctrl, cv, tgt, ph)
        np.testing.assert_allclose(host(t), oracle.apply(psi0, [tgt], ph, ctrl, cv), atol=1e-12)


def test_repeated_gates_on_one_qubit_fuse_to_identity(qc, G):
    """A gate followed by its inverse many times on the same qubits, in
    every mode: the result is the input state."""
    n = 13
    rng = np.random.default_rng(5)
    gts = []
    for _ in range(20):
        u = random_unitary(4, rng)
        gts += [((3, 11), (), (), u), ((3, 11), (), (), u.conj().T)]
    psi0 = W.random_state(n, 6)
    for mode in (0, 1, 2):
        t = dev(psi0, torch.complex128)
        qc.apply_circuit(t, qc.GateList(gts), mode=mode, fuse_k=5)
        np.testing.assert_allclose(host(t), psi0, atol=1e-12)


def test_fused_c64_vs_unfused_c128_at_30_qubits(qc, G):
    """30-qubit brickwork, depth 40 (1780 gates): the fused complex64 path
    against the unfused complex128 path, relative 2-norm error <= 1e-5, and
    the state norm within the FP32 bound."""
    n, ops = W.config_brickwork32(n=30, layers=40)
    gl = qc.GateList(G.gate_tuples(ops))
    ref = qc.new_state(n, torch.complex128)
    qc.state_init(ref, 0)
    qc.apply_circuit(ref, gl, mode=qc.QC_EXEC_UNFUSED)
    t = qc.new_state(n, torch.complex64)
    qc.state_init(t, 0)
    st = qc.apply_circuit(t, gl, mode=qc.QC_EXEC_FUSED, fuse_k=5)
    assert st["fused_blocks"] < len(ops) / 10
    d = qc.state_diff(t, ref).cpu().numpy()
    assert math.sqrt(d[0] / d[1]) < 1e-5
    assert abs(d[1] - 1.0) < 1e-10           # the complex128 run keeps the norm
    p = qc.probs(t, [0, 29]).cpu().numpy()
    assert abs(p.sum() - 1.0) < 1e-5
    del t, ref
    torch.cuda.empty_cache()


def test_unfused_c128_vs_oracle_at_22_qubits(qc, G):
    """The unfused complex128 kernels that anchor the chain of trust, on the
    same circuit family at 22 qubits against the oracle."""
    n, ops = W.config_brickwork32(n=22, layers=6)
    ref = oracle.run(ops, oracle.basis_state(n, 0))
    t = qc.new_state(n, torch.complex128)
    qc.state_init(t, 0)
    qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=qc.QC_EXEC_UNFUSED)
    assert np.max(np.abs(host(t) - ref)) < 1e-12


@pytest.mark.parametrize("dt,fuse_k", [("c128", 5), ("c64", 5), ("c128", 2), ("c64", 3)])
def test_fused_mode_with_diagonal_and_controlled_gates_across_blocks(qc, G, dt, fuse_k):
    """QC_EXEC_FUSED on a circuit where controls and diagonal gates reach
    outside the blocks (multiplexed blocks), open controls, a controlled
    gate with a non-diagonal target, and a 9-qubit MCX too wide for any
    block (applied on its own), against the oracle."""
    n = 14
    rng = np.random.default_rng(31 + fuse_k)
    ops = []
    for layer in range(6):
        for q in range(n):
            ops.append(W.Op("U", (q,), matrix=random_unitary(2, rng)))
        for q in range(layer % 2, n - 1, 2):
            ops.append(W.Op("CZ", (q, q + 1)))
        a, b = [int(x) for x in rng.permutation(n)[:2]]
        ops.append(W.Op("CP", (a, b), angle=float(rng.uniform(0, 2 * np.pi))))
        a, b = [int(x) for x in rng.permutation(n)[:2]]
        ops.append(W.Op("CNOT", (a, b)))
        qs = [int(x) for x in rng.permutation(n)[:3]]
        ops.append(W.Op("MCX", tuple(qs), ctrl_val=(0, 1)))
        ops.append(W.Op("RZ", (int(rng.integers(n)),), angle=float(rng.uniform(0, 6))))
    ops.append(W.Op("MCX", tuple(range(9)), ctrl_val=(1, 0, 1, 1, 0, 1, 0, 1)))
    psi0 = W.random_state(n, 77)
    ref = oracle.run(ops, psi0)
    t = dev(psi0, DT[dt])
    st = qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=qc.QC_EXEC_FUSED,
                          fuse_k=fuse_k)
    assert st["fused_blocks"] < len(ops) / 2
    got = host(t)
    if dt == "c128":
        assert np.max(np.abs(got - ref)) <= 1e-12
    else:
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


def test_fused_launches_on_two_streams(qc, G):
    """Fused matrix-core sweeps of two circuits interleaved on two streams:
    every launch takes its tiles from its own counter, so the results equal
    those of the same circuits run one after the other (bit for bit; the
    kernels are deterministic), and the first circuit also matches the
    oracle's gate-by-gate result."""
    n = 18
    ops_a = W.brickwork(n, 12, seed=71, entangler="CZ")
    ops_b = W.brickwork(n, 12, seed=72, entangler="CNOT")
    gl_a = qc.GateList(G.gate_tuples(ops_a))
    gl_b = qc.GateList(G.gate_tuples(ops_b))
    seq = []
    for gl in (gl_a, gl_b):
        t = qc.new_state(n, torch.complex64)
        qc.state_init(t, 0)
        qc.apply_circuit(t, gl, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        seq.append(host(t))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ta = qc.new_state(n, torch.complex64)
    tb = qc.new_state(n, torch.complex64)
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(sa):
            qc.state_init(ta, 0)
            qc.apply_circuit(ta, gl_a, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        with torch.cuda.stream(sb):
            qc.state_init(tb, 0)
            qc.apply_circuit(tb, gl_b, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        torch.cuda.synchronize()
        assert np.array_equal(host(ta), seq[0])
        assert np.array_equal(host(tb), seq[1])
    ref = oracle.run(ops_a, oracle.basis_state(n, 0))
    err = np.linalg.norm(seq[0] - ref) / np.linalg.norm(ref)
    assert err < 1e-5, err


def test_fused_c64_32_qubit_circuit_then_inverse(qc, G):
    """The 32-qubit, depth-40 brickwork at full size, in the launch
    configuration bench.py times (fused 5-qubit blocks, complex64, default
    knobs): after the circuit the norm is 1 within the FP32 bound, and the
    circuit followed by its inverse (reversed gates, adjoint matrices, also
    fused) returns |0...0>.  The unfused complex128 comparison at this size
    is bench.py's err_rel_vs_c128; at 30 qubits it is a test above."""
    n, ops = W.config_brickwork32()
    gts = G.gate_tuples(ops)
    inv = [(tg, cs, cv, np.conj(np.asarray(m)).T.copy()) for tg, cs, cv, m in reversed(gts)]
    t = qc.new_state(n, torch.complex64)
    qc.state_init(t, 0)
    st = qc.apply_circuit(t, qc.GateList(gts), mode=qc.QC_EXEC_FUSED, fuse_k=5)
    assert st["fused_blocks"] < 70
    p = qc.probs(t, [0]).cpu().numpy()
    assert abs(p.sum() - 1.0) < 1e-5
    qc.apply_circuit(t, qc.GateList(inv), mode=qc.QC_EXEC_FUSED, fuse_k=5)
    p0 = qc.probs(t, list(range(8))).cpu().numpy()     # outcome 0 of the first 8 qubits
    amp0 = t[0].item()
    assert abs(abs(amp0) ** 2 - 1.0) < 1e-4, amp0
    assert abs(p0[0] - 1.0) < 1e-4
    del t
    torch.cuda.empty_cache()
