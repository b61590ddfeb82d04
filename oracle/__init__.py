"""FP64 CPU oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and the
two share no code: this package has its own gate library, its own circuit
runner and its own C kernels (``oracle.c``).  The seeded input generators
in ``workloads`` (random numbers and circuit structure only) are the one
module both sides use.

What it computes, and where the paper defines it (QCLAB, Keip, Camps and
Van Beeumen, 2025):

* ``apply`` / ``run``          gate application, section 3.2: the state is
                               multiplied by I_l (x) U' (x) I_r, one output
                               amplitude at a time (see ``oracle.c``).
* ``probs``                    measurement probabilities, section 3.3.
* ``collapse`` / ``simulate``  collapse and renormalisation, section 3.3;
                               one branch per outcome with non-zero
                               probability (mid-circuit measurements,
                               section 3.3 and the examples of section 5),
                               measurements in the Z, X, Y or a custom basis
                               (basis change V before, V^dagger after,
                               sections 2 and 3.3) and qubit resets
                               (section 3.3).
* ``reset``                    one branch of a qubit reset: the outcome-b
                               collapse of section 3.3 followed, for b = 1,
                               by X on the qubit.
* ``counts``                   shot counts over the measured qubits (the
                               ``counts`` of section 5.2) from caller-given
                               uniforms.
* ``reduced_statevector``      state of the unmeasured qubits once the
                               measured ones are known (section 5.1).
* ``expect_pauli`` / ``energy``  <psi|P|psi> for Pauli strings, the quantity
                               behind the tomography coefficients of 5.2.
* ``param_shift_grad``         gradient of <H> for RX/RY/RZ parameters by the
                               parameter-shift rule (exact for exp(-i t G/2)
                               with G^2 = I).  The paper has no gradients;
                               this is the textbook rule.
* ``qft_amplitude``            one QFT output amplitude from the discrete
                               Fourier sum (Nielsen & Chuang eq. 5.1).

Gate matrices not printed in the paper follow Nielsen & Chuang, the text the
paper refers to for the basics: RX/RY/RZ(t) = exp(-i t X/Y/Z / 2),
CP(phi) = diag(1, 1, 1, e^{i phi}), S = diag(1, i).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = [
    "build", "gate_matrix", "apply", "run", "probs", "collapse", "simulate",
    "reduced_statevector", "expect_pauli", "energy", "param_shift_grad",
    "fd_grad", "qft_amplitude", "basis_state", "set_threads", "threads",
    "reset", "sample", "counts",
]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fcx-limited-range", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, ip, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_apply.argtypes = [vp, vp, i, i, ip, vp, i, ip, ip]
    lib.oracle_apply.restype = i
    lib.oracle_probs.argtypes = [vp, i, i, ip, dp]
    lib.oracle_probs.restype = i
    lib.oracle_expect_pauli.argtypes = [vp, i, ctypes.c_char_p, dp, dp]
    lib.oracle_expect_pauli.restype = i
    lib.oracle_collapse.argtypes = [vp, i, i, i, dp]
    lib.oracle_collapse.restype = i
    lib.oracle_threads.restype = i
    lib.oracle_set_threads.argtypes = [i]
    _lib = lib
    return lib


def threads() -> int:
    return _load().oracle_threads()


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def _ints(xs: Sequence[int]):
    arr = (ctypes.c_int * max(1, len(xs)))(*[int(x) for x in xs])
    return arr


def _cvec(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.complex128)


def nqubits(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.ndim != 1 or (1 << n) != psi.size:
        raise ValueError("state length must be a power of two")
    return n


# ---------------------------------------------------------------- gate library

_SQ2 = 1.0 / math.sqrt(2.0)
_FIXED: Dict[str, np.ndarray] = {
    "I": np.eye(2, dtype=np.complex128),
    "H": np.array([[_SQ2, _SQ2], [_SQ2, -_SQ2]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "S": np.array([[1, 0], [0, 1j]], dtype=np.complex128),
    "SDG": np.array([[1, 0], [0, -1j]], dtype=np.complex128),
    "SWAP": np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]],
                     dtype=np.complex128),
}


def gate_matrix(kind: str, angle: Optional[float] = None) -> np.ndarray:
    """Target-space matrix of a named gate (controls are handled separately)."""
    if kind in _FIXED:
        return _FIXED[kind].copy()
    if kind in ("RX", "RY", "RZ"):
        c, s = math.cos(angle / 2.0), math.sin(angle / 2.0)
        if kind == "RX":
            return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
        if kind == "RY":
            return np.array([[c, -s], [s, c]], dtype=np.complex128)
        return np.array([[complex(c, -s), 0], [0, complex(c, s)]], dtype=np.complex128)
    if kind == "P":
        return np.array([[1, 0], [0, np.exp(1j * angle)]], dtype=np.complex128)
    raise ValueError("unknown gate kind %r" % kind)


def _op_parts(op, theta=None):
    """(targets, matrix, controls, control values) of a workloads.Op."""
    k = op.kind
    ang = op.angle
    if op.pidx is not None:
        ang = float(theta[op.pidx])
    if k == "U":
        return tuple(op.qubits), np.asarray(op.matrix, dtype=np.complex128), (), ()
    if k == "CNOT":
        return (op.qubits[1],), gate_matrix("X"), (op.qubits[0],), (1,)
    if k == "CZ":
        return (op.qubits[1],), gate_matrix("Z"), (op.qubits[0],), (1,)
    if k == "CP":
        return (op.qubits[1],), gate_matrix("P", ang), (op.qubits[0],), (1,)
    if k == "MCX":
        return (op.qubits[-1],), gate_matrix("X"), tuple(op.qubits[:-1]), tuple(op.ctrl_val)
    if k == "SWAP":
        return tuple(op.qubits), gate_matrix("SWAP"), (), ()
    return tuple(op.qubits), gate_matrix(k, ang), (), ()


# ---------------------------------------------------------------- primitives

def apply(psi: np.ndarray, qubits: Sequence[int], u: np.ndarray,
          ctrl: Sequence[int] = (), ctrl_val: Sequence[int] = ()) -> np.ndarray:
    """Return (controlled) I_l (x) u (x) I_r applied to psi (section 3.2)."""
    lib = _load()
    psi = _cvec(psi)
    n = nqubits(psi)
    u = _cvec(np.asarray(u).reshape(-1))
    k = len(qubits)
    if u.size != (1 << k) ** 2:
        raise ValueError("matrix size does not match the qubit count")
    if len(ctrl_val) != len(ctrl):
        raise ValueError("one control value per control qubit")
    out = np.empty_like(psi)
    rc = lib.oracle_apply(psi.ctypes.data, out.ctypes.data, n, k, _ints(qubits),
                          u.ctypes.data, len(ctrl), _ints(ctrl), _ints(ctrl_val))
    if rc != 0:
        raise ValueError("oracle_apply rejected its arguments")
    return out


def basis_state(n: int, bits) -> np.ndarray:
    """|b> for a bitstring (first character = qubit 0 = most significant
    bit, section 3.1) or an integer index."""
    if isinstance(bits, str):
        if len(bits) != n or any(c not in "01" for c in bits):
            raise ValueError("bitstring must have n characters from {0,1}")
        idx = 0
        for c in bits:
            idx = 2 * idx + (1 if c == "1" else 0)
    else:
        idx = int(bits)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[idx] = 1.0
    return psi


def run(ops, psi0: np.ndarray, theta=None) -> np.ndarray:
    """Apply a list of workloads.Op gates in order (no measurements)."""
    psi = _cvec(psi0).copy()
    for op in ops:
        t, u, c, cv = _op_parts(op, theta)
        psi = apply(psi, t, u, c, cv)
    return psi


def probs(psi: np.ndarray, qubits: Optional[Sequence[int]] = None) -> np.ndarray:
    """Marginal distribution over the listed qubits (all qubits by default);
    the first listed qubit is the most significant bit of the outcome."""
    lib = _load()
    psi = _cvec(psi)
    n = nqubits(psi)
    qs = list(range(n)) if qubits is None else list(qubits)
    out = np.empty(1 << len(qs), dtype=np.float64)
    rc = lib.oracle_probs(psi.ctypes.data, n, len(qs), _ints(qs),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != 0:
        raise ValueError("oracle_probs rejected its arguments")
    return out


def collapse(psi: np.ndarray, q: int, outcome: int) -> Tuple[np.ndarray, float]:
    """Post-measurement state for outcome on qubit q and its probability."""
    lib = _load()
    out = _cvec(psi).copy()
    p = ctypes.c_double()
    rc = lib.oracle_collapse(out.ctypes.data, nqubits(out), q, outcome, ctypes.byref(p))
    if rc < 0:
        raise ValueError("oracle_collapse rejected its arguments")
    return out, p.value


def expect_pauli(psi: np.ndarray, pauli: str) -> complex:
    lib = _load()
    psi = _cvec(psi)
    n = nqubits(psi)
    if len(pauli) != n:
        raise ValueError("Pauli string must have one character per qubit")
    re, im = ctypes.c_double(), ctypes.c_double()
    rc = lib.oracle_expect_pauli(psi.ctypes.data, n, pauli.encode(), ctypes.byref(re),
                                 ctypes.byref(im))
    if rc != 0:
        raise ValueError("oracle_expect_pauli rejected its arguments")
    return complex(re.value, im.value)


def energy(psi: np.ndarray, terms) -> float:
    """sum_t c_t <psi|P_t|psi> (real part) for a list of (string, c_t)."""
    return float(sum(c * expect_pauli(psi, p).real for p, c in terms))


# ------------------------------------------------------------ measurement (3.3)

_BASIS_CHANGE = {
    # measure in basis b: apply V, measure Z, apply V^dagger.  X: V = H.
    # Y: V = H S^dagger, which maps the +1 eigenvector (1, i)/sqrt2 of Y to |0>.
    "z": None,
    "x": ("H",),
    "y": ("SDG", "H"),
}


def basis_change(basis) -> Optional[np.ndarray]:
    """The matrix V applied before a measurement in ``basis`` (None for the
    computational basis): "x", "y", or a caller-given 2 x 2 unitary (a
    custom basis, section 2).  V^dagger is applied after the measurement
    (section 3.3)."""
    if isinstance(basis, str):
        seq = _BASIS_CHANGE[basis]
        if seq is None:
            return None
        v = np.eye(2, dtype=np.complex128)
        for g in seq:          # applied in this order: V = last @ ... @ first
            v = gate_matrix(g) @ v
        return v
    v = np.asarray(basis, dtype=np.complex128)
    if v.shape != (2, 2):
        raise ValueError("a custom measurement basis is a 2 x 2 matrix")
    return v


def reset(psi: np.ndarray, q: int, outcome: int) -> Tuple[np.ndarray, float]:
    """One branch of a reset of qubit q (section 3.3): collapse onto
    ``outcome`` (renormalised), then, if the outcome is 1, flip the qubit
    back to |0> with X.  Returns the branch state and its probability."""
    post, pb = collapse(psi, q, outcome)
    if outcome == 1 and pb > 0.0:
        post = apply(post, (q,), gate_matrix("X"))
    return post, pb


def simulate(n: int, items, init) -> List[Tuple[str, float, np.ndarray]]:
    """Branching simulation as in section 3.3: ``items`` is a list of
    workloads.Op gates, ``("M", qubit[, basis])`` measurements (basis "z",
    "x", "y" or a 2 x 2 basis-change matrix V) and ``("R", qubit)`` resets.
    Returns one (outcome string, probability, final state) per branch with
    non-zero probability, outcomes ordered lexicographically, one character
    per measurement or reset in the order performed (a reset records the
    outcome of its measurement: its two branches are different states)."""
    psi0 = basis_state(n, init) if isinstance(init, (str, int)) else _cvec(init)
    branches = [("", 1.0, psi0.copy())]
    for it in items:
        if isinstance(it, tuple) and it and it[0] in ("M", "R"):
            q = it[1]
            is_reset = it[0] == "R"
            v = None if is_reset else basis_change(it[2] if len(it) > 2 else "z")
            new = []
            for res, p, psi in branches:
                if v is not None:
                    psi = apply(psi, (q,), v)
                for b in (0, 1):
                    if is_reset:
                        post, pb = reset(psi, q, b)
                    else:
                        post, pb = collapse(psi, q, b)
                    if pb > 1e-14:
                        if v is not None:
                            post = apply(post, (q,), v.conj().T)
                        new.append((res + str(b), p * pb, post))
            branches = new
        else:
            branches = [(r, p, run([it], psi)) for r, p, psi in branches]
    branches.sort(key=lambda x: x[0])
    return branches


def reduced_statevector(psi: np.ndarray, known_qubits: Sequence[int],
                        known_values: str) -> np.ndarray:
    """Amplitudes of the remaining qubits when the known qubits hold the
    given values (section 5.1).  Remaining qubits keep their relative order."""
    psi = _cvec(psi)
    n = nqubits(psi)
    rest = [q for q in range(n) if q not in known_qubits]
    out = np.zeros(1 << len(rest), dtype=np.complex128)
    for i in range(1 << n):
        bits = [(i >> (n - 1 - q)) & 1 for q in range(n)]
        if all(bits[q] == int(v) for q, v in zip(known_qubits, known_values)):
            r = 0
            for q in rest:
                r = 2 * r + bits[q]
            out[r] = psi[i]
    return out


# --------------------------------------------------------------- gradients

def param_shift_grad(ops, theta, terms, psi0, indices=None) -> np.ndarray:
    """dE/dtheta_p by the parameter-shift rule,
    g_p = [E(theta + pi/2 e_p) - E(theta - pi/2 e_p)] / 2, which is exact
    for gates exp(-i theta G/2) with G^2 = I (RX, RY, RZ).  A parameter used
    by several gates gets the sum over those gates (chain rule)."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = range(theta.size) if indices is None else indices
    g = np.zeros(len(list(idx)))
    for a, p in enumerate(idx):
        users = [j for j, op in enumerate(ops) if op.pidx == p]
        total = 0.0
        for j in users:
            vals = []
            for sgn in (+1.0, -1.0):
                shifted = list(ops)
                o = ops[j]
                shifted[j] = type(o)(o.kind, o.qubits, o.ctrl_val,
                                     float(theta[p]) + sgn * math.pi / 2.0, None, o.matrix)
                vals.append(energy(run(shifted, psi0, theta), terms))
            total += 0.5 * (vals[0] - vals[1])
        g[a] = total
    return g


def fd_grad(ops, theta, terms, psi0, indices=None, eps: float = 1e-4) -> np.ndarray:
    """Central finite differences of E(theta) with step eps."""
    theta = np.asarray(theta, dtype=np.float64)
    idx = list(range(theta.size) if indices is None else indices)
    g = np.zeros(len(idx))
    for a, p in enumerate(idx):
        tp = theta.copy()
        tm = theta.copy()
        tp[p] += eps
        tm[p] -= eps
        g[a] = (energy(run(ops, psi0, tp), terms) - energy(run(ops, psi0, tm), terms)) / (2 * eps)
    return g


# --------------------------------------------------------------- sampling

def sample(psi: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF sampling of the measurement distribution of all qubits:
    for each uniform u_k in [0, 1) the first basis index whose cumulative
    probability (index order) exceeds u_k times the total probability."""
    p = probs(psi)
    cdf = np.cumsum(p)
    x = np.asarray(u, dtype=np.float64) * cdf[-1]
    return np.searchsorted(cdf, x, side="right").astype(np.int64)


def counts(psi: np.ndarray, qubits: Sequence[int], u: np.ndarray) -> np.ndarray:
    """Shot counts over the measured qubits (``counts`` of section 5.2): each
    uniform draws one basis index with ``sample``; the shot is recorded
    under the values of the listed qubits (first listed = most significant
    bit of the outcome).  Returns 2^len(qubits) integer counts."""
    n = nqubits(_cvec(psi))
    idx = sample(psi, u)
    out = np.zeros(idx.shape, dtype=np.int64)
    for q in qubits:
        out = 2 * out + ((idx >> (n - 1 - q)) & 1)
    return np.bincount(out, minlength=1 << len(qubits)).astype(np.int64)


# ------------------------------------------------------------------- QFT

def qft_amplitude(psi: np.ndarray, y: int) -> complex:
    """Output amplitude y of the quantum Fourier transform of psi:
    (1/sqrt N) sum_x exp(2 pi i x y / N) psi_x  (Nielsen & Chuang eq. 5.1)."""
    psi = _cvec(psi)
    dim = psi.size
    x = np.arange(dim, dtype=np.float64)
    # reduce x*y modulo N exactly in integers before forming the phase
    ph = ((np.arange(dim, dtype=np.int64) * int(y)) % dim).astype(np.float64)
    del x
    return complex(np.sum(np.exp(2j * math.pi * ph / dim) * psi) / math.sqrt(dim))
