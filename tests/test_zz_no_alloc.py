"""qc_probs_noalloc (the allocation-free variant of qc_probs) against
qc_probs through the C ABI: the same kernels in the same order, so the
results must agree bit for bit.  Two calls in a row, the second on a smaller
register, on the shared static scratch array; the allocation-free call comes
first so that it also runs before the library has allocated anything."""
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


CASES = [
    # (n, listed qubits): partial sums in the scratch array (several blocks
    # per bin), then a smaller register, then the straight-to-output shapes
    (22, [3, 17, 9]),
    (14, [0, 13]),
    (20, list(range(12))),       # 4096 bins: one block per bin
    (16, list(range(16))[::-1]),  # every qubit: one output per amplitude
]


@pytest.mark.parametrize("dt", [torch.complex64, torch.complex128])
def test_noalloc_probs_matches_probs(qc, dt):
    for n, qubits in CASES:
        psi = torch.from_numpy(W.random_state(n, 100 + n)).to(dt).cuda()
        out = torch.full((1 << len(qubits),), float("nan"), dtype=torch.float64, device="cuda")
        qc.probs_noalloc(psi, out, qubits)
        ref = qc.probs(psi, qubits)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (n, qubits)
        assert abs(out.sum().item() - 1.0) < (1e-12 if dt == torch.complex128 else 1e-5)


def test_noalloc_probs_rejects_bad_arguments(qc):
    psi = qc.new_state(10, torch.complex64)
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    for bad in ([0, 0], [0, 11]):
        with pytest.raises(qc.QcError) as e:
            qc.probs_noalloc(psi, out, bad)
        assert e.value.status == -2
