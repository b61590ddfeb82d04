"""Write the stored expected values that the GPU parity tests compare with.

Every value here comes from the FP64 oracle (``oracle/``) on the seeded
synthetic inputs of ``workloads``; nothing is read from the GPU library.
Run from the repository root:

    python tests/golden/make_golden.py [batch512] [adjoint24] [qft28] [tfim28]

* ``batch512_energies.json``: <H> of all 512 circuits of the batch workload
  (qubit counts uniform in [10, 20], 8-layer hardware-efficient ansatz,
  open-chain transverse-field Ising H), one oracle forward each.
* ``adjoint24.json``: the 24-qubit, 16-layer ansatz's energy and the
  parameter-shift gradient of a few parameters (first and last layer, RY
  and RZ), each from two oracle forwards.
* ``qft28_amplitudes.json``: 16 output amplitudes of the 28-qubit QFT of the
  seeded random state, each from the discrete Fourier sum.
* ``tfim28_terms.json``: <P_t> of each of the 55 Pauli terms of the 28-qubit
  open-chain transverse-field Ising H on the same seeded random state, and
  the energy sum_t c_t <P_t>.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

ADJOINT_PARAMS = [0, 1, 25, 383, 766, 767]
QFT_INDICES = [0, 1, 2, 3, 255, 4096, 65535, 1 << 20, 12345678, (1 << 27) - 1, 1 << 27,
               (1 << 27) + 1, 200000003, (1 << 28) - 3, (1 << 28) - 2, (1 << 28) - 1]


def batch512():
    cfg = W.batch_config()
    out = []
    t0 = time.time()
    for i, (n, th) in enumerate(cfg):
        psi = oracle.run(W.hea(n, 8), oracle.basis_state(n, 0), th)
        out.append(oracle.energy(psi, W.tfim_terms(n)))
        if i % 64 == 63:
            print("batch512: %d circuits, %.0f s" % (i + 1, time.time() - t0), flush=True)
    json.dump({"about": "FP64 oracle <H> of the 512-circuit batch workload (seed 512), "
                        "written by tests/golden/make_golden.py",
               "energies": out}, open(os.path.join(HERE, "batch512_energies.json"), "w"))


def adjoint24():
    n, ops, theta, terms = W.adjoint_config()
    psi0 = oracle.basis_state(n, 0)
    t0 = time.time()
    e = oracle.energy(oracle.run(ops, psi0, theta), terms)
    print("adjoint24: energy %.15f (%.0f s)" % (e, time.time() - t0), flush=True)
    g = oracle.param_shift_grad(ops, theta, terms, psi0, indices=ADJOINT_PARAMS)
    print("adjoint24: gradients done (%.0f s)" % (time.time() - t0), flush=True)
    json.dump({"about": "FP64 oracle energy and parameter-shift gradients of the 24-qubit "
                        "16-layer ansatz (seed 24), written by tests/golden/make_golden.py",
               "energy": e, "params": ADJOINT_PARAMS, "grad": [float(x) for x in g]},
              open(os.path.join(HERE, "adjoint24.json"), "w"))


def qft28():
    n, _, psi = W.config_qft28()
    t0 = time.time()
    amps = []
    for y in QFT_INDICES:
        a = oracle.qft_amplitude(psi, y)
        amps.append([a.real, a.imag])
    print("qft28: %d amplitudes (%.0f s)" % (len(amps), time.time() - t0), flush=True)
    json.dump({"about": "FP64 oracle QFT output amplitudes of the 28-qubit seeded random state "
                        "(seed 28), written by tests/golden/make_golden.py",
               "indices": QFT_INDICES, "amplitudes": amps},
              open(os.path.join(HERE, "qft28_amplitudes.json"), "w"))


def tfim28():
    n = 28
    terms = W.tfim_terms(n)
    psi = W.random_state(n, seed=28)
    t0 = time.time()
    vals = [oracle.expect_pauli(psi, p).real for p, _ in terms]
    print("tfim28: %d terms (%.0f s)" % (len(vals), time.time() - t0), flush=True)
    json.dump({"about": "FP64 oracle <P_t> of the 55 open-chain TFIM terms on the 28-qubit "
                        "seeded random state (seed 28), written by tests/golden/make_golden.py",
               "terms": [p for p, _ in terms], "values": vals,
               "energy": float(sum(c * v for (_, c), v in zip(terms, vals)))},
              open(os.path.join(HERE, "tfim28_terms.json"), "w"))


if __name__ == "__main__":
    which = sys.argv[1:] or ["batch512", "adjoint24", "qft28", "tfim28"]
    for w in which:
        globals()[w]()
