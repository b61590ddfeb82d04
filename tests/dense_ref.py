"""Brute-force dense operators built from Kronecker products (numpy only).

Used to pin the oracle: the register operator of a gate is assembled as an
explicit sum of Kronecker chains over the qubits 0..n-1 (qubit 0 leftmost,
as in the paper's kron(v, bell) inputs), with no index arithmetic at all.
"""
from functools import reduce

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
PAULI = {
    "I": I2,
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def kron_chain(factors):
    return reduce(np.kron, factors)


def unit(r, c):
    e = np.zeros((2, 2), dtype=np.complex128)
    e[r, c] = 1.0
    return e


def dense_gate(n, targets, u, ctrl=(), ctrl_val=()):
    """Register operator: sum over control-active part Pc (x) u on the
    targets plus (I - Pc) (x) I."""
    targets = list(targets)
    ctrl = list(ctrl)
    k = len(targets)
    d = 1 << k
    full = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for r in range(d):
        for c in range(d):
            if u[r, c] == 0:
                continue
            fac = []
            for q in range(n):
                if q in targets:
                    j = targets.index(q)
                    fac.append(unit((r >> (k - 1 - j)) & 1, (c >> (k - 1 - j)) & 1))
                elif q in ctrl:
                    v = ctrl_val[ctrl.index(q)]
                    fac.append(unit(v, v))
                else:
                    fac.append(I2)
            full += u[r, c] * kron_chain(fac)
    if ctrl:
        pc = kron_chain([unit(ctrl_val[ctrl.index(q)], ctrl_val[ctrl.index(q)])
                         if q in ctrl else I2 for q in range(n)])
        full += np.eye(1 << n) - pc
    return full


def dense_pauli(p):
    return kron_chain([PAULI[c] for c in p])


def random_unitary(d, rng):
    z = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def random_state(n, rng):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return v / np.linalg.norm(v)
