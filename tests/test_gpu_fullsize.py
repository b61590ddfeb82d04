"""Parity at the sizes bench.py times, in the launch configurations it uses.

* 28-qubit QFT on the seeded Gaussian state: every execution mode
  (LDS tile runs in complex64 and complex128, fused complex64) against the
  unfused complex128 run over the whole state (qc_state_diff), and 16
  output amplitudes against the FP64 oracle's discrete Fourier sums
  (stored by tests/golden/make_golden.py, which calls only the oracle).
* 512-circuit batch: all 512 energies against the oracle's.
* 28-qubit TFIM expectation: all 55 per-term values and the energy, complex128
  and complex64, against the oracle's (tests/golden/tfim28_terms.json).
* 24-qubit adjoint gradient: every one of the 768 complex128 gradients
  against central differences (eps = 1e-4) of complex128 forward runs, the
  energy and six gradients against the oracle's energy and parameter-shift
  values; the complex64 gradient against the complex128 one.

Tolerances: complex128 states 1e-12 max-abs; complex64 states 1e-5
relative 2-norm; energies |dE| <= 2 ||H|| eps_state with ||H|| <= 2n - 1.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2503_03016_amd import qc as mod
    return mod


@pytest.fixture(scope="module")
def G():
    from paper_2503_03016_amd import gates
    return gates


def golden(name):
    return json.load(open(os.path.join(GOLDEN, name)))


def test_qft28_every_mode_full_state(qc, G):
    n, ops, psi0 = W.config_qft28()
    gl = qc.GateList(G.gate_tuples(ops))
    ref = torch.from_numpy(psi0).cuda()
    st = qc.apply_circuit(ref, gl, mode=qc.QC_EXEC_UNFUSED)
    assert st["sweeps"] == len(ops)
    gold = golden("qft28_amplitudes.json")
    idx = torch.tensor(gold["indices"], dtype=torch.int64, device="cuda")
    want = np.array([complex(a, b) for a, b in gold["amplitudes"]])
    got = ref[idx].cpu().numpy()
    assert np.max(np.abs(got - want)) < 1e-12, np.max(np.abs(got - want))
    results = {}
    for dt, mode in ((torch.complex128, qc.QC_EXEC_TILED), (torch.complex64, qc.QC_EXEC_TILED),
                     (torch.complex64, qc.QC_EXEC_FUSED), (torch.complex128, qc.QC_EXEC_FUSED)):
        t = torch.from_numpy(psi0).to(dt).cuda()
        qc.apply_circuit(t, gl, mode=mode, fuse_k=5)
        d = qc.state_diff(t, ref).cpu().numpy()
        rel, mx = math.sqrt(d[0] / d[1]), d[2]
        results[(str(dt), mode)] = (rel, mx)
        if dt == torch.complex128:
            assert mx < 1e-12, (mode, mx)
            assert np.max(np.abs(t[idx].cpu().numpy() - want)) < 1e-12
        else:
            assert rel < 1e-5, (mode, rel)
            a = t[idx].cpu().numpy().astype(np.complex128)
            assert np.max(np.abs(a - want)) < 1e-5 * np.max(np.abs(want)) * 10
        del t
        torch.cuda.empty_cache()
    print("qft28 errors vs unfused complex128:", results)
    del ref
    torch.cuda.empty_cache()


def test_batch512_every_energy_vs_oracle(qc, G):
    cfg = W.batch_config()
    ref = np.array(golden("batch512_energies.json")["energies"])
    assert len(ref) == len(cfg)
    circuits = [(n, G.gate_tuples(W.hea(n, 8), th), W.tfim_terms(n)) for n, th in cfg]
    b = qc.Batch(circuits, dtype=torch.complex64)
    e = b.run().cpu().numpy()
    assert b.status() == 0
    ns = np.array([n for n, _ in cfg])
    err = np.abs(e - ref)
    bound = 2 * (2 * ns - 1) * 1e-5
    print("batch512 max |dE| = %.3e (bound at n = 20: %.1e)" % (err.max(), bound.max()))
    assert np.all(err < bound), (int(np.argmax(err - bound)), float(err.max()))


class _Forward:
    """complex128 forward runs of the adjoint workload with one parameter
    changed: the gate list is built once and the one rotation's matrix is
    rewritten in place between runs (the GateList keeps every matrix in
    one host array)."""

    def __init__(self, qc, G, n, ops, theta, terms):
        self.qc, self.G, self.ops, self.terms = qc, G, ops, terms
        self.theta = np.array(theta, dtype=np.float64)
        gts = G.gate_tuples(ops, self.theta)
        self.gl = qc.GateList(gts)
        sizes = [np.asarray(g[3]).size for g in gts]
        self.off = np.concatenate(([0], np.cumsum(sizes)[:-1]))
        self.op_of = {op.pidx: k for k, op in enumerate(ops) if op.pidx is not None}
        self.t = qc.new_state(n, torch.complex128)

    def energy(self, p=None, value=None):
        qc = self.qc
        if p is not None:
            k = self.op_of[p]
            th = self.theta.copy()
            th[p] = value
            m = self.G.gate_tuple(self.ops[k], th)[3].reshape(-1)
            self.gl._mats[self.off[k]:self.off[k] + 4] = m
        qc.state_init(self.t, 0)
        qc.apply_circuit(self.t, self.gl, mode=qc.QC_EXEC_TILED)
        e = qc.expect_pauli(self.t, self.terms)[0].item()
        if p is not None:   # put the original matrix back
            m = self.G.gate_tuple(self.ops[k], self.theta)[3].reshape(-1)
            self.gl._mats[self.off[k]:self.off[k] + 4] = m
        return e


def test_adjoint24_every_gradient_vs_central_differences(qc, G):
    n, ops, theta, terms = W.adjoint_config()
    psi = qc.new_state(n, torch.complex128)
    lam = qc.new_state(n, torch.complex128)
    qc.state_init(psi, 0)
    e128, g128 = qc.adjoint_grad(psi, lam, ops, theta, terms)
    e128, g128 = e128.item(), g128.cpu().numpy()
    del psi, lam
    gold = golden("adjoint24.json")
    assert abs(e128 - gold["energy"]) < 1e-10 * len(terms)
    np.testing.assert_allclose(g128[gold["params"]], gold["grad"], atol=1e-9)
    f = _Forward(qc, G, n, ops, theta, terms)
    assert abs(f.energy() - gold["energy"]) < 1e-10 * len(terms)
    eps = 1e-4
    fd = np.empty(len(theta))
    for p in range(len(theta)):
        fd[p] = (f.energy(p, theta[p] + eps) - f.energy(p, theta[p] - eps)) / (2 * eps)
    err = np.abs(fd - g128)
    print("adjoint24 complex128: max |g - FD| = %.3e over %d parameters" % (err.max(), len(fd)))
    # FD truncation eps^2/6 * ||H|| ~ 8e-8, rounding ~ 1e-15 ||H|| / eps
    assert err.max() < 1e-6, (int(np.argmax(err)), float(err.max()))


def test_adjoint24_complex64_vs_complex128(qc):
    n, ops, theta, terms = W.adjoint_config()
    out = {}
    for dt in (torch.complex128, torch.complex64):
        psi = qc.new_state(n, dt)
        lam = qc.new_state(n, dt)
        qc.state_init(psi, 0)
        e, g = qc.adjoint_grad(psi, lam, ops, theta, terms)
        out[dt] = (e.item(), g.cpu().numpy())
    gold = golden("adjoint24.json")
    e64, g64 = out[torch.complex64]
    e128, g128 = out[torch.complex128]
    dg = np.max(np.abs(g64 - g128))
    print("adjoint24 complex64: |dE| vs oracle = %.3e, max |dg| vs complex128 = %.3e"
          % (abs(e64 - gold["energy"]), dg))
    bound = 2 * (2 * n - 1) * 1e-5
    assert abs(e64 - gold["energy"]) < bound
    assert dg < bound


def test_tfim28_every_term_vs_oracle(qc):
    """The 28-qubit TFIM expectation that bench.py times (energy only) and
    with per-term output, complex128 and complex64, against the oracle's
    <P_t> of all 55 terms.  Bounds: complex128 1e-12 per term (the terms
    are O(1e-4) on this state); complex64 4 * 2^-24 per term, from the
    rounding of the state to complex64 (relative 2^-24 per component, so
    |d<P>| <= 2 ||dpsi|| + ||dpsi||^2) plus the single-precision products."""
    n = 28
    terms = W.tfim_terms(n)
    gold = golden("tfim28_terms.json")
    assert gold["terms"] == [p for p, _ in terms]
    want = np.array(gold["values"])
    host = torch.from_numpy(W.random_state(n, seed=28))
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 4 * 2.0 ** -24)):
        psi = host.to(dt).cuda()
        e = qc.expect_pauli(psi, terms)[0].item()
        v = qc.expect_pauli(psi, terms, per_term=True).cpu().numpy()
        err = np.abs(v[1:] - want)
        print("tfim28 %s: |dE| = %.3e, max per-term error %.3e"
              % (dt, abs(e - gold["energy"]), err.max()))
        assert err.max() < tol, (dt, int(np.argmax(err)), float(err.max()))
        assert abs(e - gold["energy"]) < tol * sum(abs(c) for _, c in terms)
        assert abs(v[0] - e) < tol * sum(abs(c) for _, c in terms)
        del psi
        torch.cuda.empty_cache()
