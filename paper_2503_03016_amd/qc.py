"""Thin ctypes binding of libqc.so (include/qc.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI.  Torch tensors provide device memory and the
current stream; nothing here computes on a state.  If libqc.so is missing
this module raises at import time: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqc.so")

QC_C64, QC_C128 = 1, 2
QC_EXEC_UNFUSED, QC_EXEC_FUSED, QC_EXEC_TILED = 0, 1, 2
QC_MAX_FUSED, QC_MAX_CTRLS, QC_MAX_SEL = 5, 16, 2
STATUS = {0: "QC_OK", -1: "QC_ERR_ARG", -2: "QC_ERR_QUBIT", -3: "QC_ERR_DTYPE",
          -4: "QC_ERR_UNSUPPORTED", -5: "QC_ERR_HIP", -6: "QC_ERR_NOMEM"}
OP_KIND = {"RX": 1, "RY": 2, "RZ": 3, "H": 4, "X": 5, "Y": 6, "Z": 7, "CZ": 8, "CNOT": 9}

EXPORTS = [
    "qc_status_string", "qc_last_error", "qc_version", "qc_state_init", "qc_state_copy",
    "qc_state_diff", "qc_apply_1q", "qc_apply_2q", "qc_apply_controlled", "qc_apply_fused_k",
    "qc_apply_multiplexed", "qc_permute_qubits",
    "qc_apply_circuit", "qc_fuse_plan", "qc_block_matrices", "qc_probs", "qc_expect_pauli", "qc_adjoint_grad",
    "qc_timing_enable", "qc_timing_query", "qc_batch_create", "qc_batch_info", "qc_run_batch",
    "qc_batch_state", "qc_batch_status", "qc_batch_destroy", "qc_collapse", "qc_reduced_state",
    "qc_sample", "qc_set_knob", "qc_get_knob", "qc_autotune", "qc_reset", "qc_counts",
    "qc_reserve", "qc_probs_noalloc",
]
QC_MAX_COUNT_QUBITS, QC_MAX_COUNT_SHOTS = 24, 1 << 21
(QC_KNOB_MFMA_WG_PER_CU, QC_KNOB_TILE_WG_PER_CU, QC_KNOB_FUSE_LOOKAHEAD, QC_KNOB_MFMA_TILE_BITS,
 QC_KNOB_TILE_BITS, QC_KNOB_TILE_ENGINE, QC_KNOB_WIDE_MIN_TILES) = 1, 2, 3, 4, 5, 6, 7


class QcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__("%s failed: %s (%s)" % (where, STATUS.get(status, status), detail))
        self.status = status


class QcState(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_void_p), ("n", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class QcGate(ctypes.Structure):
    _fields_ = [("n_targets", ctypes.c_int32), ("n_ctrls", ctypes.c_int32),
                ("targets", ctypes.c_int32 * QC_MAX_FUSED),
                ("ctrls", ctypes.c_int32 * QC_MAX_CTRLS),
                ("ctrl_vals", ctypes.c_int32 * QC_MAX_CTRLS),
                ("matrix", ctypes.POINTER(ctypes.c_double))]


class QcStats(ctypes.Structure):
    _fields_ = [("gates", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("sweeps", ctypes.c_int64), ("fused_blocks", ctypes.c_int64),
                ("state_bytes", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class QcCircuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.POINTER(QcGate)), ("n_terms", ctypes.c_int32),
                ("paulis", ctypes.c_char_p), ("coeff", ctypes.POINTER(ctypes.c_double))]


class QcTuneEntry(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("fuse_k", ctypes.c_int32),
                ("mfma_wg_per_cu", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("ms", ctypes.c_float), ("mfma_tile_bits", ctypes.c_int32),
                ("tile_bits", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class QcOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("param", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqc.so is not built (run __graft_entry__.build() or "
                          "python paper_2503_03016_amd/build.py); there is no fallback")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    S = QcState
    sig = {
        "qc_status_string": ([i], ctypes.c_char_p),
        "qc_last_error": ([], ctypes.c_char_p),
        "qc_version": ([], i),
        "qc_state_init": ([S, u64, vp], i),
        "qc_state_copy": ([S, S, vp], i),
        "qc_state_diff": ([S, S, vp, vp], i),
        "qc_apply_1q": ([S, i, dp, vp], i),
        "qc_apply_2q": ([S, i, i, dp, vp], i),
        "qc_apply_controlled": ([S, i, ip, ip, i, dp, vp], i),
        "qc_apply_fused_k": ([S, i, ip, dp, vp], i),
        "qc_apply_multiplexed": ([S, i, ip, i, ip, dp, vp], i),
        "qc_permute_qubits": ([S, ip, vp], i),
        "qc_apply_circuit": ([S, i, ctypes.POINTER(QcGate), i, i, ctypes.POINTER(QcStats), vp], i),
        "qc_fuse_plan": ([i, i, ctypes.POINTER(QcGate), i, ip, ip], i),
        "qc_block_matrices": ([i, ctypes.POINTER(QcGate), i, ip, i, ip, dp], i),
        "qc_probs": ([S, i, ip, vp, vp], i),
        "qc_expect_pauli": ([S, i, ctypes.c_char_p, dp, i, vp, vp], i),
        "qc_adjoint_grad": ([S, S, ctypes.POINTER(QcOp), i, dp, i, i, ctypes.c_char_p, dp, vp,
                             vp, vp], i),
        "qc_timing_enable": ([i], i),
        "qc_timing_query": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64), dp], i),
        "qc_batch_create": ([i, ctypes.POINTER(QcCircuit), i, i, ctypes.POINTER(vp)], i),
        "qc_batch_info": ([vp, ctypes.POINTER(ctypes.c_uint64), ip, ip], i),
        "qc_run_batch": ([vp, vp, vp, vp], i),
        "qc_batch_state": ([vp, vp, i, ctypes.POINTER(QcState)], i),
        "qc_batch_status": ([vp, ip], i),
        "qc_batch_destroy": ([vp], i),
        "qc_collapse": ([S, i, i, vp, vp], i),
        "qc_reduced_state": ([S, i, ip, ip, S, vp], i),
        "qc_sample": ([S, i, vp, vp, vp], i),
        "qc_reset": ([S, i, i, vp, vp], i),
        "qc_counts": ([S, i, ip, i, vp, vp, vp], i),
        "qc_reserve": ([vp], i),
        "qc_probs_noalloc": ([S, i, ip, vp, vp], i),
        "qc_set_knob": ([i, i], i),
        "qc_get_knob": ([i, ip], i),
        "qc_autotune": ([S, i, ctypes.POINTER(QcGate), i, ctypes.POINTER(QcTuneEntry), i, ip, vp],
                        i),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise QcError(rc, where, lib.qc_last_error().decode())


def _ints(xs: Sequence[int]):
    xs = [int(x) for x in xs]
    return (ctypes.c_int * max(1, len(xs)))(*xs)


def _mat(u) -> Tuple[np.ndarray, ctypes.POINTER(ctypes.c_double)]:
    a = np.ascontiguousarray(np.asarray(u, dtype=np.complex128)).view(np.float64).reshape(-1)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(t: Optional[torch.Tensor] = None):
    dev = t.device if t is not None else torch.device("cuda")
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def state_view(psi: torch.Tensor) -> QcState:
    """Describe a contiguous complex64/complex128 CUDA tensor of 2^n entries."""
    if not isinstance(psi, torch.Tensor) or psi.device.type != "cuda":
        raise TypeError("state must be a CUDA tensor")
    if psi.dim() != 1 or not psi.is_contiguous():
        raise ValueError("state must be a contiguous 1-D tensor")
    n = int(psi.numel()).bit_length() - 1
    if (1 << n) != psi.numel():
        raise ValueError("state length must be a power of two")
    if psi.dtype == torch.complex64:
        dt = QC_C64
    elif psi.dtype == torch.complex128:
        dt = QC_C128
    else:
        raise TypeError("state dtype must be complex64 or complex128")
    return QcState(psi.data_ptr(), n, dt)


def new_state(n: int, dtype=torch.complex64, device="cuda") -> torch.Tensor:
    return torch.empty(1 << n, dtype=dtype, device=device)


# ------------------------------------------------------------- entry points

def state_init(psi: torch.Tensor, basis_index: int = 0) -> torch.Tensor:
    _check(lib.qc_state_init(state_view(psi), int(basis_index), _stream(psi)), "qc_state_init")
    return psi


def state_copy(dst: torch.Tensor, src: torch.Tensor) -> torch.Tensor:
    _check(lib.qc_state_copy(state_view(dst), state_view(src), _stream(dst)), "qc_state_copy")
    return dst


def state_diff(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """[sum |a-b|^2, sum |b|^2, max |a-b|] (FP64, on the device)."""
    out = torch.empty(3, dtype=torch.float64, device=a.device)
    _check(lib.qc_state_diff(state_view(a), state_view(b), ctypes.c_void_p(out.data_ptr()),
                             _stream(a)), "qc_state_diff")
    return out


def apply_1q(psi: torch.Tensor, q: int, u) -> torch.Tensor:
    m, p = _mat(u)
    _check(lib.qc_apply_1q(state_view(psi), int(q), p, _stream(psi)), "qc_apply_1q")
    return psi


def apply_2q(psi: torch.Tensor, qa: int, qb: int, u) -> torch.Tensor:
    m, p = _mat(u)
    _check(lib.qc_apply_2q(state_view(psi), int(qa), int(qb), p, _stream(psi)), "qc_apply_2q")
    return psi


def apply_controlled(psi: torch.Tensor, ctrl: Sequence[int], ctrl_val: Sequence[int],
                     target: int, u) -> torch.Tensor:
    m, p = _mat(u)
    _check(lib.qc_apply_controlled(state_view(psi), len(ctrl), _ints(ctrl), _ints(ctrl_val),
                                   int(target), p, _stream(psi)), "qc_apply_controlled")
    return psi


def apply_fused_k(psi: torch.Tensor, qubits: Sequence[int], u) -> torch.Tensor:
    m, p = _mat(u)
    _check(lib.qc_apply_fused_k(state_view(psi), len(qubits), _ints(qubits), p, _stream(psi)),
           "qc_apply_fused_k")
    return psi


def apply_multiplexed(psi: torch.Tensor, qubits: Sequence[int], sel_qubits: Sequence[int],
                      us) -> torch.Tensor:
    """psi := sum_v P_v (x) U_v psi; `us` holds 2^len(sel_qubits) matrices
    (v = selector value, sel_qubits[0] = most significant bit)."""
    arr = np.asarray(us, dtype=np.complex128)
    m, p = _mat(arr)
    _check(lib.qc_apply_multiplexed(state_view(psi), len(qubits), _ints(qubits), len(sel_qubits),
                                    _ints(sel_qubits), p, _stream(psi)), "qc_apply_multiplexed")
    return psi


def permute_qubits(psi: torch.Tensor, perm: Sequence[int]) -> torch.Tensor:
    """Qubit q of the register becomes qubit perm[q] (in place)."""
    _check(lib.qc_permute_qubits(state_view(psi), _ints(perm), _stream(psi)), "qc_permute_qubits")
    return psi


_GATE_DTYPE = np.dtype([("n_targets", "<i4"), ("n_ctrls", "<i4"),
                        ("targets", "<i4", (QC_MAX_FUSED,)), ("ctrls", "<i4", (QC_MAX_CTRLS,)),
                        ("ctrl_vals", "<i4", (QC_MAX_CTRLS,)), ("matrix", "<u8")], align=True)


class GateList:
    """qc_gate_t array built from (targets, ctrls, ctrl_vals, matrix) tuples
    (filled in bulk through a numpy record array of the same layout); keeps
    the host matrices alive while the library reads them."""

    def __init__(self, gates: Iterable[Tuple[Sequence[int], Sequence[int], Sequence[int], np.ndarray]]):
        gates = list(gates)
        assert _GATE_DTYPE.itemsize == ctypes.sizeof(QcGate)
        count = len(gates)
        rec = np.zeros(max(1, count), dtype=_GATE_DTYPE)
        if count:
            nt = np.fromiter((len(g[0]) for g in gates), dtype=np.int32, count=count)
            nc = np.fromiter((len(g[1]) for g in gates), dtype=np.int32, count=count)
            if nt.max() > QC_MAX_FUSED or nc.max() > QC_MAX_CTRLS:
                raise ValueError("gate too wide for qc_gate_t")
            rec["n_targets"][:count] = nt
            rec["n_ctrls"][:count] = nc
            for i, (t, c, cv, _) in enumerate(gates):
                if len(t):
                    rec["targets"][i, :len(t)] = t
                if len(c):
                    rec["ctrls"][i, :len(c)] = c
                    rec["ctrl_vals"][i, :len(c)] = cv
            mats = [np.asarray(g[3], dtype=np.complex128).reshape(-1) for g in gates]
            sizes = np.fromiter((m.size for m in mats), dtype=np.int64, count=count)
            if np.any(sizes != (1 << (2 * nt.astype(np.int64)))):
                raise ValueError("matrix size does not match the target count")
            self._mats = np.ascontiguousarray(np.concatenate(mats))
            offsets = np.concatenate(([0], np.cumsum(sizes)[:-1]))
            rec["matrix"][:count] = self._mats.ctypes.data + 16 * offsets
        else:
            self._mats = np.zeros(1, dtype=np.complex128)
        self._rec = rec
        self.arr = rec.ctypes.data_as(ctypes.POINTER(QcGate))
        self.count = count


def apply_circuit(psi: torch.Tensor, gates: GateList, mode: int = QC_EXEC_UNFUSED,
                  fuse_k: int = 5) -> dict:
    st = QcStats()
    _check(lib.qc_apply_circuit(state_view(psi), gates.count, gates.arr, int(mode), int(fuse_k),
                                ctypes.byref(st), _stream(psi)), "qc_apply_circuit")
    return st.as_dict()


def fuse_plan(n: int, gates: GateList, fuse_k: int = 5) -> Tuple[List[int], int]:
    block_of = (ctypes.c_int * max(1, gates.count))()
    nb = ctypes.c_int()
    _check(lib.qc_fuse_plan(int(n), gates.count, gates.arr, int(fuse_k), block_of,
                            ctypes.byref(nb)), "qc_fuse_plan")
    return list(block_of[:gates.count]), nb.value


def block_matrices(gates: GateList, qubits: Sequence[int], sel: Sequence[int] = ()
                   ) -> np.ndarray:
    """qc_block_matrices: the fuser's FP64 block matrices of `gates` on the
    block `qubits` (qubits[0] = MSB) for every value of the selector qubits
    `sel`; shape (2^len(sel), 2^k, 2^k), complex128.  Host only."""
    k, ns = len(qubits), len(sel)
    out = np.zeros(2 * (4 ** k << ns), dtype=np.float64)
    _check(lib.qc_block_matrices(gates.count, gates.arr, k, _ints(qubits), ns,
                                 _ints(sel) if ns else None,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "qc_block_matrices")
    return out.view(np.complex128).reshape(1 << ns, 1 << k, 1 << k)


def probs(psi: torch.Tensor, qubits: Optional[Sequence[int]] = None) -> torch.Tensor:
    sv = state_view(psi)
    qs = list(range(sv.n)) if qubits is None else list(qubits)
    out = torch.empty(1 << len(qs), dtype=torch.float64, device=psi.device)
    _check(lib.qc_probs(sv, len(qs), _ints(qs), ctypes.c_void_p(out.data_ptr()), _stream(psi)),
           "qc_probs")
    return out


def probs_noalloc(psi: torch.Tensor, out: torch.Tensor,
                  qubits: Optional[Sequence[int]] = None) -> torch.Tensor:
    """qc_probs_noalloc into a caller-given FP64 device tensor `out` of
    2^len(qubits) entries (the library allocates nothing)."""
    sv = state_view(psi)
    qs = list(range(sv.n)) if qubits is None else list(qubits)
    if out.dtype != torch.float64 or out.numel() != (1 << len(qs)) or not out.is_contiguous():
        raise ValueError("out must be a contiguous FP64 tensor of 2^len(qubits) entries")
    _check(lib.qc_probs_noalloc(sv, len(qs), _ints(qs), ctypes.c_void_p(out.data_ptr()),
                                _stream(psi)), "qc_probs_noalloc")
    return out


def _terms(terms, n):
    strings = "".join(p for p, _ in terms)
    if len(strings) != n * len(terms):
        raise ValueError("every Pauli string needs n characters")
    coeff = np.ascontiguousarray([float(c) for _, c in terms], dtype=np.float64)
    return strings.encode(), coeff


def expect_pauli(psi: torch.Tensor, terms, per_term: bool = False) -> torch.Tensor:
    """terms: list of (Pauli string, coefficient).  Returns a device FP64
    tensor [sum_t c_t <P_t>, (<P_t> for each t if per_term)]."""
    sv = state_view(psi)
    s, coeff = _terms(terms, sv.n)
    out = torch.empty(1 + (len(terms) if per_term else 0), dtype=torch.float64, device=psi.device)
    _check(lib.qc_expect_pauli(sv, len(terms), s, coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               int(bool(per_term)), ctypes.c_void_p(out.data_ptr()), _stream(psi)),
           "qc_expect_pauli")
    return out


def collapse(psi: torch.Tensor, q: int, outcome: int) -> torch.Tensor:
    """Collapse onto outcome of qubit q and renormalise in place; returns
    P(outcome) as a device FP64 tensor of one element."""
    p = torch.empty(1, dtype=torch.float64, device=psi.device)
    _check(lib.qc_collapse(state_view(psi), int(q), int(outcome), ctypes.c_void_p(p.data_ptr()),
                           _stream(psi)), "qc_collapse")
    return p


def reset(psi: torch.Tensor, q: int, outcome: int) -> torch.Tensor:
    """One branch of a reset of qubit q in place (collapse onto `outcome`,
    renormalise, then X on q for outcome 1); returns P(outcome) as a device
    FP64 tensor of one element."""
    p = torch.empty(1, dtype=torch.float64, device=psi.device)
    _check(lib.qc_reset(state_view(psi), int(q), int(outcome), ctypes.c_void_p(p.data_ptr()),
                        _stream(psi)), "qc_reset")
    return p


def counts(psi: torch.Tensor, qubits: Sequence[int], u: torch.Tensor) -> torch.Tensor:
    """Shot counts over the listed qubits for the uniforms u (device FP64):
    a device int64 tensor of 2^len(qubits) counts (qubits[0] = most
    significant bit of the outcome)."""
    if u.dtype != torch.float64 or u.device != psi.device or not u.is_contiguous():
        raise TypeError("u must be a contiguous FP64 tensor on the state's device")
    out = torch.empty(1 << len(qubits), dtype=torch.int64, device=psi.device)
    _check(lib.qc_counts(state_view(psi), len(qubits), _ints(qubits), int(u.numel()),
                         ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                         _stream(psi)), "qc_counts")
    return out


def reserve(device=None) -> None:
    """qc_reserve: allocate the workspace and empty the staging ring before a
    HIP graph capture (host-synchronous)."""
    dev = torch.device("cuda") if device is None else torch.device(device)
    _check(lib.qc_reserve(ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)),
           "qc_reserve")


def reduced_state(psi: torch.Tensor, qubits: Sequence[int], values) -> torch.Tensor:
    """Amplitudes of the other qubits when `qubits` hold `values`."""
    sv = state_view(psi)
    vals = [int(v) for v in values]
    out = torch.empty(1 << (sv.n - len(qubits)), dtype=psi.dtype, device=psi.device)
    _check(lib.qc_reduced_state(sv, len(qubits), _ints(qubits), _ints(vals), state_view(out),
                                _stream(psi)), "qc_reduced_state")
    return out


def sample(psi: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Basis indices drawn by inverse CDF for the uniforms u (device FP64)."""
    if u.dtype != torch.float64 or u.device != psi.device or not u.is_contiguous():
        raise TypeError("u must be a contiguous FP64 tensor on the state's device")
    out = torch.empty(u.numel(), dtype=torch.int64, device=psi.device)
    _check(lib.qc_sample(state_view(psi), int(u.numel()), ctypes.c_void_p(u.data_ptr()),
                         ctypes.c_void_p(out.data_ptr()), _stream(psi)), "qc_sample")
    return out


def set_knob(knob: int, value: int) -> None:
    _check(lib.qc_set_knob(int(knob), int(value)), "qc_set_knob")


def get_knob(knob: int) -> int:
    v = ctypes.c_int()
    _check(lib.qc_get_knob(int(knob), ctypes.byref(v)), "qc_get_knob")
    return v.value


def autotune(scratch: torch.Tensor, gates: GateList, reps: int = 3) -> List[dict]:
    """Time every execution strategy (qc_autotune); fastest first."""
    ents = (QcTuneEntry * 32)()
    cnt = ctypes.c_int()
    _check(lib.qc_autotune(state_view(scratch), gates.count, gates.arr, int(reps), ents, 32,
                           ctypes.byref(cnt), _stream(scratch)), "qc_autotune")
    return [ents[i].as_dict() for i in range(cnt.value)]


_OPS_MEMO = {}   # the last op list marshalled: id -> (snapshot, array, count)


def make_ops(ops) -> Tuple[ctypes.Array, int]:
    """qc_op_t array from workloads.Op entries of kinds RX/RY/RZ/H/X/Y/Z/CZ/CNOT
    (filled through one int32 array of the same layout).  The array of the
    last list is kept and returned again while the list holds the same ops
    (a gradient loop passes one list with new angles)."""
    snap = tuple(ops)
    hit = _OPS_MEMO.get(id(ops))
    if hit is not None and hit[0] == snap:
        return hit[1], hit[2]
    flat = []
    put = flat.extend
    for op in snap:
        kind = OP_KIND.get(op.kind)
        if kind is None:
            raise ValueError("op kind %s is not supported by qc_adjoint_grad" % op.kind)
        q = op.qubits
        put((kind, q[0], q[1] if len(q) > 1 else 0, -1 if op.pidx is None else op.pidx))
    buf = np.fromiter(flat if flat else (0, 0, 0, 0), dtype=np.int32)
    assert 4 * 4 == ctypes.sizeof(QcOp)
    arr = (QcOp * (buf.size // 4)).from_buffer(buf)   # keeps buf alive
    _OPS_MEMO.clear()
    _OPS_MEMO[id(ops)] = (snap, arr, len(snap))
    return arr, len(snap)


def adjoint_grad(psi: torch.Tensor, lam: torch.Tensor, ops, theta, terms):
    """Returns (energy, grad) as device FP64 tensors; psi holds the input
    state on entry and (up to rounding) again on return."""
    sv, lv = state_view(psi), state_view(lam)
    arr, nops = make_ops(ops)
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    s, coeff = _terms(terms, sv.n)
    energy = torch.empty(1, dtype=torch.float64, device=psi.device)
    grad = torch.empty(th.size, dtype=torch.float64, device=psi.device)
    _check(lib.qc_adjoint_grad(sv, lv, arr, nops, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               int(th.size), len(terms), s,
                               coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.c_void_p(energy.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                               _stream(psi)), "qc_adjoint_grad")
    return energy, grad


def timing_enable(on: bool = True) -> None:
    _check(lib.qc_timing_enable(int(bool(on))), "qc_timing_enable")


def timing_query(name: str) -> Tuple[int, float]:
    cnt = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib.qc_timing_query(name.encode(), ctypes.byref(cnt), ctypes.byref(ms)),
           "qc_timing_query")
    return cnt.value, ms.value


class Batch:
    """A batch of circuits run in one persistent launch (qc_batch_* / qc_run_batch).

    circuits: list of (n, gate tuples, terms) with gate tuples as accepted by
    GateList and terms as in expect_pauli.  The arena (caller-owned device
    memory for the states of large circuits) is a torch tensor owned here."""

    def __init__(self, circuits, dtype=torch.complex64, keep_states: bool = False,
                 device="cuda"):
        self.dtype = dtype
        dt = QC_C64 if dtype == torch.complex64 else QC_C128
        arr = (QcCircuit * len(circuits))()
        self._keep = []
        for c, (n, gts, terms) in zip(arr, circuits):
            gl = GateList(gts)
            s, coeff = _terms(terms, n)
            self._keep += [gl, s, coeff]
            c.n, c.n_gates, c.gates = n, gl.count, gl.arr
            c.n_terms, c.paulis = len(terms), s
            c.coeff = coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        _check(lib.qc_batch_create(len(circuits), arr, dt, int(bool(keep_states)), ctypes.byref(h)),
               "qc_batch_create")
        self.handle = h
        self._destroy = lib.qc_batch_destroy   # usable during interpreter shutdown
        self._keep = None
        nbytes, grid, phases = ctypes.c_uint64(), ctypes.c_int(), ctypes.c_int()
        _check(lib.qc_batch_info(h, ctypes.byref(nbytes), ctypes.byref(grid), ctypes.byref(phases)),
               "qc_batch_info")
        self.arena_bytes, self.grid, self.phases = nbytes.value, grid.value, phases.value
        elem = 8 if dt == QC_C64 else 16
        self.arena = torch.empty(max(1, self.arena_bytes // elem), dtype=dtype, device=device)
        self.count = len(circuits)

    def run(self, energy: Optional[torch.Tensor] = None) -> torch.Tensor:
        if energy is None:
            energy = torch.empty(self.count, dtype=torch.float64, device=self.arena.device)
        _check(lib.qc_run_batch(self.handle, ctypes.c_void_p(self.arena.data_ptr()),
                                ctypes.c_void_p(energy.data_ptr()), _stream(self.arena)),
               "qc_run_batch")
        return energy

    def state(self, i: int) -> torch.Tensor:
        v = QcState()
        _check(lib.qc_batch_state(self.handle, ctypes.c_void_p(self.arena.data_ptr()), int(i),
                                  ctypes.byref(v)), "qc_batch_state")
        elem = 8 if self.dtype == torch.complex64 else 16
        off = (v.amp - self.arena.data_ptr()) // elem
        return self.arena[off: off + (1 << v.n)]

    def status(self) -> int:
        f = ctypes.c_int()
        _check(lib.qc_batch_status(self.handle, ctypes.byref(f)), "qc_batch_status")
        return f.value

    def __del__(self):
        h = getattr(self, "handle", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and h.value and destroy is not None:
            destroy(h)
            self.handle = None


# the C entry-point names, for callers who prefer them
qc_state_init = state_init
qc_state_copy = state_copy
qc_state_diff = state_diff
qc_apply_1q = apply_1q
qc_apply_2q = apply_2q
qc_apply_controlled = apply_controlled
qc_apply_fused_k = apply_fused_k
qc_apply_multiplexed = apply_multiplexed
qc_permute_qubits = permute_qubits
qc_apply_circuit = apply_circuit
qc_fuse_plan = fuse_plan
qc_block_matrices = block_matrices
qc_probs = probs
qc_expect_pauli = expect_pauli
qc_adjoint_grad = adjoint_grad
qc_timing_enable = timing_enable
qc_timing_query = timing_query
qc_collapse = collapse
qc_reduced_state = reduced_state
qc_sample = sample
qc_reset = reset
qc_counts = counts
qc_reserve = reserve
qc_probs_noalloc = probs_noalloc
