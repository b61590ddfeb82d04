"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module only draws random numbers and describes circuit *structure*
(which named gate acts on which qubits, in which order, with which angle or
parameter index).  It holds none of the simulation arithmetic: it never
builds a gate matrix for a named gate, never applies a gate and never
reduces a state.  Each side (the oracle and the GPU binding) maps gate names
to matrices with its own gate library.  The only matrices produced here are
Haar-random U(2) draws, which are random *inputs* to the method.

Qubit labels follow the paper's convention (QCLAB, section 3.1/3.2 and the
teleportation example of section 5.1): qubit 0 is the leftmost Kronecker
factor, i.e. the most significant bit of the amplitude index.

Workloads (all synthetic, seeded with numpy's PCG64 ``default_rng``):

* ``brickwork``      - layers of Haar U(2) on every qubit, then an entangler
                        (CNOT or CZ) on neighbour pairs (0,1),(2,3),... in
                        even layers and (1,2),(3,4),... in odd layers.
* ``qft``            - quantum Fourier transform gate list (H, controlled
                        phase 2*pi/2^k, final swap network).
* ``hea``            - hardware-efficient ansatz: RY and RZ on every qubit,
                        then a CZ ladder (0,1),(1,2),...,(n-2,n-1).
* ``tfim_terms``     - open-chain transverse-field Ising Hamiltonian
                        H = -sum Z_i Z_{i+1} - sum X_i as Pauli strings.
* ``random_state``   - i.i.d. complex Gaussian amplitudes, normalised.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Op", "haar_u2", "brickwork", "qft", "hea", "tfim_terms", "random_state",
    "batch_config", "adjoint_config", "config_brickwork12",
    "config_qft28", "config_brickwork32", "ghz", "teleportation", "grover2",
    "bitflip_code",
]


@dataclasses.dataclass(frozen=True)
class Op:
    """One circuit element.

    kind     : gate name ("H", "X", "Y", "Z", "S", "SDG", "RX", "RY", "RZ",
               "CP", "CZ", "CNOT", "SWAP", "MCX", "U").
    qubits   : operand qubits in the gate's own order.  CNOT/CZ/CP: (c, t).
               MCX: controls..., target (the target is last).  U: targets.
    ctrl_val : MCX control values (1 = closed control, 0 = open control).
    angle    : rotation / phase angle in radians when it is fixed.
    pidx     : index into a parameter vector when the angle is a parameter.
    matrix   : explicit unitary for kind "U" (complex128, 2^k x 2^k).
    """

    kind: str
    qubits: Tuple[int, ...]
    ctrl_val: Tuple[int, ...] = ()
    angle: Optional[float] = None
    pidx: Optional[int] = None
    matrix: Optional[np.ndarray] = dataclasses.field(default=None, compare=False)


def haar_u2(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 2x2 unitary (Mezzadri, arXiv:math-ph/0609050).

    Draw a complex Ginibre matrix Z = (A + iB)/sqrt(2), take its QR
    factorisation and rescale the columns of Q by the phases of diag(R), so
    that the distribution is exactly Haar.
    """
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    ph = d / np.abs(d)
    return (q * ph[None, :]).astype(np.complex128)


def brickwork(n: int, layers: int, seed: int, entangler: str = "CNOT") -> List[Op]:
    """Brickwork random circuit: per layer Haar U(2) on qubits 0..n-1 in
    order, then the entangler on (0,1),(2,3),... (even layer) or
    (1,2),(3,4),... (odd layer).  The lower label is the CNOT control."""
    rng = np.random.default_rng(seed)
    ops: List[Op] = []
    for layer in range(layers):
        for q in range(n):
            ops.append(Op("U", (q,), matrix=haar_u2(rng)))
        start = 0 if layer % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            ops.append(Op(entangler, (a, a + 1)))
    return ops


def qft(n: int) -> List[Op]:
    """QFT gate list (Nielsen & Chuang section 5.1): for each qubit j, H on
    j then controlled phases 2*pi/2^k from qubit j+k-1 onto j, k = 2..n-j;
    finally swap qubit j with n-1-j for j < n/2."""
    ops: List[Op] = []
    for j in range(n):
        ops.append(Op("H", (j,)))
        for k in range(2, n - j + 1):
            ops.append(Op("CP", (j + k - 1, j), angle=2.0 * math.pi / (2 ** k)))
    for j in range(n // 2):
        ops.append(Op("SWAP", (j, n - 1 - j)))
    return ops


def hea(n: int, layers: int) -> List[Op]:
    """Hardware-efficient ansatz structure.  Parameter index of the RY on
    qubit q in layer l is l*2n + 2q, of the RZ it is l*2n + 2q + 1."""
    ops: List[Op] = []
    for layer in range(layers):
        for q in range(n):
            ops.append(Op("RY", (q,), pidx=layer * 2 * n + 2 * q))
            ops.append(Op("RZ", (q,), pidx=layer * 2 * n + 2 * q + 1))
        for a in range(n - 1):
            ops.append(Op("CZ", (a, a + 1)))
    return ops


def ghz(n: int) -> List[Op]:
    """GHZ preparation: H on qubit 0, then CNOT(q, q+1) down the chain."""
    ops = [Op("H", (0,))]
    for q in range(n - 1):
        ops.append(Op("CNOT", (q, q + 1)))
    return ops


def teleportation(src: int = 0, a: int = 1, b: int = 2) -> list:
    """Quantum teleportation of the state of qubit ``src`` onto qubit ``b``
    (section 5.1): qubits a and b share a Bell pair.  Bell-basis measurement
    of (src, a) = CNOT(src, a), H(src), measure both; then the corrections
    X^m_a and Z^m_src on b, written as gates controlled by the measured
    qubits (they hold their collapsed values)."""
    return [Op("CNOT", (src, a)), Op("H", (src,)), ("M", src), ("M", a),
            Op("CNOT", (a, b)), Op("CZ", (src, b))]


def _flip_phase_of(bits: str) -> List[Op]:
    """-1 on the two-qubit basis state |bits> only: X on the qubits that read
    0 in ``bits`` turns it into |11>, CZ flips |11>, the X gates go back."""
    xs = [Op("X", (q,)) for q, c in enumerate(bits) if c == "0"]
    return xs + [Op("CZ", (0, 1))] + xs


def grover2(marked: str) -> list:
    """Grover search on two qubits for the basis state ``marked`` (section
    5.3): uniform superposition, the phase oracle of the marked state, the
    diffusion operator H^2 (2|00><00| - I) H^2 (up to a global phase:
    -1 on every basis state but |00>, i.e. Z on both qubits then CZ), and a
    measurement of both qubits.  One iteration finds the marked state with
    probability 1 for N = 4."""
    if len(marked) != 2 or any(c not in "01" for c in marked):
        raise ValueError("marked must be a two-character bitstring")
    h = [Op("H", (0,)), Op("H", (1,))]
    diffuse = h + [Op("Z", (0,)), Op("Z", (1,)), Op("CZ", (0, 1))] + h
    return h + _flip_phase_of(marked) + diffuse + [("M", 0), ("M", 1)]


def bitflip_code(error_qubit: Optional[int] = None) -> list:
    """Three-qubit bit-flip code with syndrome measurement (section 5.4):
    qubit 0 is encoded onto qubits 0..2 with two CNOTs; an X error hits
    ``error_qubit`` (none if None); ancilla 3 records the parity of qubits
    0 and 1, ancilla 4 that of qubits 0 and 2; both ancillas are measured
    and the qubit whose flip explains the syndrome is flipped back by an X
    controlled by the ancillas' values (open control = 0)."""
    items: list = [Op("CNOT", (0, 1)), Op("CNOT", (0, 2))]
    if error_qubit is not None:
        items.append(Op("X", (error_qubit,)))
    for anc, pair in ((3, (0, 1)), (4, (0, 2))):
        for q in pair:
            items.append(Op("CNOT", (q, anc)))
    items += [("M", 3), ("M", 4)]
    for q in (2, 1, 0):
        syndrome = (int(q in (0, 1)), int(q in (0, 2)))
        items.append(Op("MCX", (3, 4, q), ctrl_val=syndrome))
    return items


def tfim_terms(n: int, j: float = 1.0, h: float = 1.0) -> List[Tuple[str, float]]:
    """Open-chain TFIM H = -J sum_{i<n-1} Z_i Z_{i+1} - h sum_i X_i as a list
    of (Pauli string, coefficient).  Character q of a string acts on qubit q."""
    terms: List[Tuple[str, float]] = []
    for i in range(n - 1):
        s = ["I"] * n
        s[i] = "Z"
        s[i + 1] = "Z"
        terms.append(("".join(s), -j))
    for i in range(n):
        s = ["I"] * n
        s[i] = "X"
        terms.append(("".join(s), -h))
    return terms


def random_state(n: int, seed: int) -> np.ndarray:
    """i.i.d. complex Gaussian amplitudes (real parts drawn first, then
    imaginary parts), normalised in FP64."""
    rng = np.random.default_rng(seed)
    dim = 1 << n
    re = rng.standard_normal(dim)
    im = rng.standard_normal(dim)
    v = re + 1j * im
    v /= math.sqrt(float(np.vdot(v, v).real))
    return v


# ---- the five synthetic configurations --------------------------------------

def config_brickwork12() -> Tuple[int, List[Op]]:
    """12-qubit brickwork, 20 layers, Haar U(2) + CNOT, seed 12."""
    return 12, brickwork(12, 20, seed=12, entangler="CNOT")


def config_qft28(n: int = 28) -> Tuple[int, List[Op], np.ndarray]:
    """28-qubit QFT on a seeded random state (seed 28)."""
    return n, qft(n), random_state(n, seed=28)


def config_brickwork32(n: int = 32, layers: int = 40) -> Tuple[int, List[Op]]:
    """32-qubit brickwork, depth 40, Haar U(2) + CZ, seed 32."""
    return n, brickwork(n, layers, seed=32, entangler="CZ")


def batch_config(count: int = 512, layers: int = 8, seed: int = 512,
                 n_lo: int = 10, n_hi: int = 20):
    """Batch of circuits: qubit counts uniform in [n_lo, n_hi], angles uniform
    in [0, 2pi), shape (layers, n, 2) per circuit (RY, RZ), flattened in the
    ``hea`` parameter order.  Returns a list of (n, theta)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, count)
    out = []
    for n in ns:
        theta = rng.uniform(0.0, 2.0 * math.pi, (layers, int(n), 2)).reshape(-1)
        out.append((int(n), theta))
    return out


def adjoint_config(n: int = 24, layers: int = 16, seed: int = 24):
    """Adjoint-gradient workload: HEA with 16 layers on 24 qubits, angles
    uniform in [0, 2pi) drawn with shape (layers, n, 2), seed 24."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * math.pi, (layers, n, 2)).reshape(-1)
    return n, hea(n, layers), theta, tfim_terms(n)


def count_gates(ops: Sequence[Op]) -> int:
    return len(ops)
