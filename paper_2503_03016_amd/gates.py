"""FP64 matrices of named gates and conversion of circuit descriptions
(workloads.Op) into the (targets, controls, control values, matrix) tuples
that qc_gate_t carries across the C ABI.

Matrices the paper uses (Hadamard, Pauli X/Z, CNOT, CZ, multi-controlled X
with open controls; QCLAB sections 2 and 5) and the standard ones it does
not print (Nielsen & Chuang): RX/RY/RZ(t) = exp(-i t X/Y/Z / 2),
phase P(phi) = diag(1, e^{i phi}) (controlled: CP), S = diag(1, i), SWAP.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

_R2 = math.sqrt(0.5)


def matrix(kind: str, angle: float = 0.0) -> np.ndarray:
    k = kind.upper()
    if k == "H":
        return np.array([[_R2, _R2], [_R2, -_R2]], dtype=np.complex128)
    if k == "X":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if k == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if k == "Z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if k == "S":
        return np.array([[1, 0], [0, 1j]], dtype=np.complex128)
    if k == "SDG":
        return np.array([[1, 0], [0, -1j]], dtype=np.complex128)
    if k == "I":
        return np.eye(2, dtype=np.complex128)
    half = 0.5 * angle
    c, s = math.cos(half), math.sin(half)
    if k == "RX":
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if k == "RY":
        return np.array([[c, -s], [s, c]], dtype=np.complex128)
    if k == "RZ":
        return np.array([[c - 1j * s, 0], [0, c + 1j * s]], dtype=np.complex128)
    if k == "P":
        return np.array([[1, 0], [0, complex(math.cos(angle), math.sin(angle))]],
                        dtype=np.complex128)
    if k == "SWAP":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = m[1, 2] = m[2, 1] = m[3, 3] = 1
        return m
    raise ValueError("unknown gate %r" % kind)


def gate_tuple(op, theta=None) -> Tuple[Tuple[int, ...], Tuple[int, ...], Tuple[int, ...], np.ndarray]:
    """(targets, ctrls, ctrl_vals, matrix) of one workloads.Op."""
    angle = op.angle
    if op.pidx is not None:
        angle = float(theta[op.pidx])
    k = op.kind
    if k == "U":
        return tuple(op.qubits), (), (), np.asarray(op.matrix, dtype=np.complex128)
    if k == "CNOT":
        return (op.qubits[1],), (op.qubits[0],), (1,), matrix("X")
    if k == "CZ":
        return (op.qubits[1],), (op.qubits[0],), (1,), matrix("Z")
    if k == "CP":
        return (op.qubits[1],), (op.qubits[0],), (1,), matrix("P", angle)
    if k == "MCX":
        return (op.qubits[-1],), tuple(op.qubits[:-1]), tuple(op.ctrl_val), matrix("X")
    if k == "SWAP":
        return tuple(op.qubits), (), (), matrix("SWAP")
    return tuple(op.qubits), (), (), matrix(k, angle if angle is not None else 0.0)


def gate_tuples(ops: Sequence, theta=None) -> List[tuple]:
    return [gate_tuple(op, theta) for op in ops]
