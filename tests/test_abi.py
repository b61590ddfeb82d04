"""C ABI checks that need no GPU: every symbol declared in include/qc.h is
exported by libqc.so, malformed arguments are rejected on the host with the
documented status before anything is enqueued, and the host-only fusion
planner (qc_fuse_plan) returns a valid dependency-respecting partition."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def qc():
    from paper_2503_03016_amd import qc as mod
    return mod


def test_package_modules_import_and_constants_match_header():
    import importlib
    for mod in ("qc", "gates", "simulate", "autograd", "autotune"):
        importlib.import_module("paper_2503_03016_amd." + mod)
    from paper_2503_03016_amd import qc as q
    text = open(HEADER).read()
    for name in ("QC_C64", "QC_C128", "QC_EXEC_UNFUSED", "QC_EXEC_FUSED", "QC_EXEC_TILED",
                 "QC_MAX_FUSED", "QC_MAX_CTRLS", "QC_MAX_SEL", "QC_KNOB_MFMA_WG_PER_CU",
                 "QC_KNOB_TILE_WG_PER_CU", "QC_KNOB_FUSE_LOOKAHEAD", "QC_KNOB_MFMA_TILE_BITS", "QC_KNOB_TILE_BITS",
                 "QC_KNOB_TILE_ENGINE", "QC_KNOB_WIDE_MIN_TILES"):
        m = re.search(r"#define\s+%s\s+(-?\d+)" % name, text)
        assert m and getattr(q, name) == int(m.group(1)), name
    for kind, code in q.OP_KIND.items():
        m = re.search(r"#define\s+QC_OP_%s\s+(\d+)" % kind, text)
        assert m and int(m.group(1)) == code, kind


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("qc_state_init", "qc_apply_1q", "qc_apply_2q", "qc_apply_controlled",
                     "qc_apply_fused_k", "qc_probs", "qc_expect_pauli", "qc_adjoint_grad"):
        assert required in names


def test_library_exports_every_declared_symbol(qc):
    lib = ctypes.CDLL(qc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(qc.EXPORTS)


FAKE = 0x10000  # never dereferenced: every call below fails validation first


def st(qc, n=4, dtype=1, amp=FAKE):
    return qc.QcState(amp, n, dtype)


def test_status_strings(qc):
    assert qc.lib.qc_status_string(0) == b"ok"
    assert qc.lib.qc_status_string(-2) == b"invalid qubit"
    assert qc.lib.qc_version() >= 10000


def test_state_validation(qc):
    lib = qc.lib
    assert lib.qc_state_init(st(qc, amp=None), 0, None) == -1
    assert lib.qc_state_init(st(qc, n=0), 0, None) == -1
    assert lib.qc_state_init(st(qc, n=37), 0, None) == -1
    assert lib.qc_state_init(st(qc, dtype=3), 0, None) == -3
    assert lib.qc_state_init(st(qc, n=4), 16, None) == -1
    assert b"basis" in lib.qc_last_error()


def test_gate_validation(qc):
    lib = qc.lib
    u, p = qc._mat(np.eye(2))
    u4, p4 = qc._mat(np.eye(4))
    assert lib.qc_apply_1q(st(qc), 4, p, None) == -2
    assert lib.qc_apply_1q(st(qc), -1, p, None) == -2
    assert lib.qc_apply_1q(st(qc), 0, None, None) == -1
    assert lib.qc_apply_2q(st(qc), 1, 1, p4, None) == -2
    assert lib.qc_apply_2q(st(qc), 0, 4, p4, None) == -2
    assert lib.qc_apply_2q(st(qc, n=1), 0, 0, p4, None) == -2
    c = qc._ints([1])
    bad = qc._ints([2])
    assert lib.qc_apply_controlled(st(qc), 1, c, bad, 0, p, None) == -1
    assert lib.qc_apply_controlled(st(qc), 1, c, qc._ints([1]), 1, p, None) == -2
    assert lib.qc_apply_controlled(st(qc), 4, qc._ints([0, 1, 2, 3]), qc._ints([1] * 4), 0, p,
                                   None) == -1
    u32, p32 = qc._mat(np.eye(32))
    assert lib.qc_apply_fused_k(st(qc), 6, qc._ints(range(6)), p32, None) == -1
    assert lib.qc_apply_fused_k(st(qc), 5, qc._ints(range(5)), p32, None) == -2
    assert lib.qc_apply_fused_k(st(qc, n=6), 2, qc._ints([3, 3]), p4, None) == -2
    mux = qc.lib.qc_apply_multiplexed
    u8, p8 = qc._mat(np.stack([np.eye(2)] * 8))
    assert mux(st(qc, n=6), 1, qc._ints([0]), 3, qc._ints([1, 2, 3]), p8, None) == -1
    assert mux(st(qc, n=6), 1, qc._ints([0]), -1, qc._ints([1]), p8, None) == -1
    assert mux(st(qc, n=6), 1, qc._ints([0]), 2, qc._ints([1, 0]), p8, None) == -2
    assert mux(st(qc, n=6), 1, qc._ints([0]), 2, qc._ints([1, 6]), p8, None) == -2
    assert mux(st(qc, n=6), 1, qc._ints([0]), 2, None, p8, None) == -1
    assert mux(st(qc, n=6), 1, qc._ints([0]), 2, qc._ints([1, 2]), None, None) == -1
    assert mux(st(qc, n=2), 1, qc._ints([0]), 2, qc._ints([1, 2]), p8, None) == -2
    assert mux(st(qc, n=6), 0, qc._ints([0]), 1, qc._ints([1]), p8, None) == -1
    perm = qc.lib.qc_permute_qubits
    assert perm(st(qc), None, None) == -1
    assert perm(st(qc), qc._ints([0, 1, 1, 3]), None) == -2
    assert perm(st(qc), qc._ints([0, 1, 2, 4]), None) == -2
    assert perm(st(qc), qc._ints([3, 2, 1, -1]), None) == -2
    assert perm(st(qc), qc._ints([0, 1, 2, 3]), None) == 0   # identity: no device work


def test_reduction_validation(qc):
    lib = qc.lib
    out = ctypes.c_void_p(FAKE)
    assert lib.qc_probs(st(qc), 0, qc._ints([0]), out, None) == -1
    assert lib.qc_probs(st(qc), 5, qc._ints(range(5)), out, None) == -1
    assert lib.qc_probs(st(qc), 2, qc._ints([1, 1]), out, None) == -2
    assert lib.qc_probs(st(qc), 1, qc._ints([0]), None, None) == -1
    assert lib.qc_probs(st(qc, n=30), 25, qc._ints(range(25)), out, None) == -4
    coeff = np.ones(1)
    cp = coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.qc_expect_pauli(st(qc), 1, b"XYZQ", cp, 0, out, None) == -1
    assert lib.qc_expect_pauli(st(qc), 0, b"", cp, 0, out, None) == -1


def test_measurement_validation(qc):
    lib = qc.lib
    out = ctypes.c_void_p(FAKE)
    for fn in (lib.qc_collapse, lib.qc_reset):
        assert fn(st(qc), 4, 0, out, None) == -2
        assert fn(st(qc), -1, 1, out, None) == -2
        assert fn(st(qc), 0, 2, out, None) == -1
        assert fn(st(qc, amp=None), 0, 0, out, None) == -1
    cnt = lib.qc_counts
    u = ctypes.c_void_p(FAKE)
    assert cnt(st(qc), 0, qc._ints([0]), 10, u, out, None) == -1
    assert cnt(st(qc), 5, qc._ints(range(5)), 10, u, out, None) == -1
    assert cnt(st(qc), 2, qc._ints([1, 1]), 10, u, out, None) == -2
    assert cnt(st(qc), 1, qc._ints([0]), -1, u, out, None) == -1
    assert cnt(st(qc), 1, qc._ints([0]), qc.QC_MAX_COUNT_SHOTS + 1, u, out, None) == -1
    assert cnt(st(qc), 1, qc._ints([0]), 10, None, out, None) == -1
    assert cnt(st(qc), 1, qc._ints([0]), 10, u, None, None) == -1
    assert cnt(st(qc, n=30), 25, qc._ints(range(25)), 10, u, out, None) == -1
    text = open(HEADER).read()
    for name in ("QC_MAX_COUNT_QUBITS", "QC_MAX_COUNT_SHOTS"):
        m = re.search(r"#define\s+%s\s+(\(?[-\d <]+\)?)" % name, text)
        assert m and eval(m.group(1)) == getattr(qc, name), name


def test_adjoint_validation(qc):
    lib = qc.lib
    ops, nops = qc.make_ops([W.Op("RY", (0,), pidx=3)])
    th = np.zeros(2)
    tp = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    coeff = np.ones(1)
    cp = coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    out = ctypes.c_void_p(FAKE)
    a, b = st(qc, amp=FAKE), st(qc, amp=FAKE * 4096)
    # parameter index 3 with only 2 parameters
    assert lib.qc_adjoint_grad(a, b, ops, nops, tp, 2, 1, b"ZIII", cp, out, out, None) == -1
    # psi and lam must not overlap
    assert lib.qc_adjoint_grad(a, a, ops, nops, tp, 4, 1, b"ZIII", cp, out, out, None) == -1
    ops2, n2 = qc.make_ops([W.Op("CZ", (1, 1))])
    assert lib.qc_adjoint_grad(a, b, ops2, n2, tp, 2, 1, b"ZIII", cp, out, out, None) == -2


def test_knobs(qc):
    old = qc.get_knob(qc.QC_KNOB_MFMA_WG_PER_CU)
    assert qc.lib.qc_set_knob(qc.QC_KNOB_MFMA_WG_PER_CU, 0) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_MFMA_WG_PER_CU, 6) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_TILE_WG_PER_CU, 17) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_FUSE_LOOKAHEAD, -1) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_FUSE_LOOKAHEAD, 257) == -1
    assert qc.get_knob(qc.QC_KNOB_FUSE_LOOKAHEAD) == 16
    assert qc.lib.qc_set_knob(qc.QC_KNOB_MFMA_TILE_BITS, 11) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_MFMA_TILE_BITS, 14) == -1
    assert qc.get_knob(qc.QC_KNOB_MFMA_TILE_BITS) == 13
    assert qc.lib.qc_set_knob(qc.QC_KNOB_TILE_BITS, 5) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_TILE_BITS, 14) == -1
    assert qc.get_knob(qc.QC_KNOB_TILE_BITS) == 13
    assert qc.lib.qc_set_knob(qc.QC_KNOB_WIDE_MIN_TILES, 7) == -1
    assert qc.lib.qc_set_knob(qc.QC_KNOB_WIDE_MIN_TILES, 31) == -1
    assert qc.get_knob(qc.QC_KNOB_WIDE_MIN_TILES) == 12
    assert qc.lib.qc_set_knob(99, 1) == -1
    qc.set_knob(qc.QC_KNOB_MFMA_WG_PER_CU, 3)
    assert qc.get_knob(qc.QC_KNOB_MFMA_WG_PER_CU) == 3
    qc.set_knob(qc.QC_KNOB_MFMA_WG_PER_CU, old)
    ents = (qc.QcTuneEntry * 4)()
    cnt = ctypes.c_int()
    gl = qc.GateList([((0,), (), (), np.eye(2))])
    assert qc.lib.qc_autotune(st(qc), 1, gl.arr, 0, ents, 4, ctypes.byref(cnt), None) == -1
    assert qc.lib.qc_autotune(st(qc), 0, gl.arr, 3, ents, 4, ctypes.byref(cnt), None) == -1


def test_batch_validation(qc):
    """qc_batch_create rejects malformed circuits while planning, before any
    device call."""
    from paper_2503_03016_amd import gates as G

    def create(n, ops, terms, dtype=1):
        gl = qc.GateList(G.gate_tuples(ops))
        s, coeff = qc._terms(terms, n)
        arr = (qc.QcCircuit * 1)()
        arr[0].n, arr[0].n_gates, arr[0].gates = n, gl.count, gl.arr
        arr[0].n_terms, arr[0].paulis = len(terms), s
        arr[0].coeff = coeff.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        h = ctypes.c_void_p()
        return qc.lib.qc_batch_create(1, arr, dtype, 0, ctypes.byref(h))

    assert create(31, [], [("Z" * 31, 1.0)]) == -1
    assert create(4, [], [("ZQZZ", 1.0)]) == -1
    assert create(4, [W.Op("CNOT", (1, 1))], [("ZZZZ", 1.0)]) == -2
    u8 = np.eye(8)
    assert create(4, [W.Op("U", (0, 1, 2), matrix=u8)], [("ZZZZ", 1.0)]) == -4
    assert create(4, [], [("ZZZZ", 1.0)], dtype=5) == -3
    h = ctypes.c_void_p()
    assert qc.lib.qc_batch_create(0, None, 1, 0, ctypes.byref(h)) == -1


def _gate_list(qc, ops):
    from paper_2503_03016_amd import gates as G
    return qc.GateList(G.gate_tuples(ops))


def _check_partition(ops, block_of, nb, k, max_sel=2):
    """A block acts non-diagonally on <= k qubits and touches <= k + max_sel
    qubits (or is a single gate); a gate placed in an earlier block than a
    gate that precedes it must commute with it: every qubit they share is a
    control or a target of a diagonal matrix for both."""
    from paper_2503_03016_amd import gates as G
    tuples = G.gate_tuples(ops)

    def diag_qubits(t):
        tg, cs, _, m = t
        m = np.asarray(m)
        is_diag = not np.any(m - np.diag(np.diag(m)))
        return set(cs) | (set(tg) if is_diag else set())

    dq = [diag_qubits(t) for t in tuples]
    allq = [set(t[0]) | set(t[1]) for t in tuples]
    members = {}
    for i, b in enumerate(block_of):
        assert 0 <= b < nb
        members.setdefault(b, []).append(i)
    assert sorted(members) == list(range(nb))
    for b, idx in members.items():
        nd = set().union(*[allq[i] - dq[i] for i in idx])
        touched = set().union(*[allq[i] for i in idx])
        assert len(idx) == 1 or (len(nd) <= k and len(touched) <= k + max_sel), (b, nd, touched)
    per_qubit = {}
    for i, qs in enumerate(allq):
        for q in qs:
            per_qubit.setdefault(q, []).append(i)
    for q, lst in per_qubit.items():
        for a in range(len(lst)):
            for c in range(a + 1, len(lst)):
                i, j = lst[a], lst[c]
                if block_of[j] < block_of[i]:
                    shared = allq[i] & allq[j]
                    assert shared <= (dq[i] & dq[j]), ("non-commuting gates swapped", i, j)


@pytest.mark.parametrize("look", [0, 16])
@pytest.mark.parametrize("n,layers,k", [(12, 20, 5), (16, 8, 4), (32, 40, 5), (10, 6, 3)])
def test_fuse_plan_is_a_valid_partition(qc, n, layers, k, look):
    old = qc.get_knob(qc.QC_KNOB_FUSE_LOOKAHEAD)
    qc.set_knob(qc.QC_KNOB_FUSE_LOOKAHEAD, look)
    try:
        ops = W.brickwork(n, layers, seed=n, entangler="CZ")
        gl = _gate_list(qc, ops)
        block_of, nb = qc.fuse_plan(n, gl, k)
    finally:
        qc.set_knob(qc.QC_KNOB_FUSE_LOOKAHEAD, old)
    _check_partition(ops, block_of, nb, k)
    assert nb < len(ops)


def test_fuse_plan_qft_and_mcx(qc):
    n = 12
    ops = W.qft(n) + [W.Op("MCX", (3, 4, 2), ctrl_val=(0, 1))]
    gl = _gate_list(qc, ops)
    block_of, nb = qc.fuse_plan(n, gl, 5)
    _check_partition(ops, block_of, nb, 5)


def test_fuse_plan_rejects_bad_gates(qc):
    gl = _gate_list(qc, [W.Op("CNOT", (0, 0))])
    with pytest.raises(qc.QcError):
        qc.fuse_plan(4, gl, 5)


def test_gate_list_marshalling_round_trip(qc):
    """GateList fills qc_gate_t records in bulk: every field and every matrix
    entry reads back through the C layout."""
    rng = np.random.default_rng(3)
    tuples = []
    for i in range(50):
        k = int(rng.integers(1, 4))
        qs = [int(x) for x in rng.permutation(10)[:k + 2]]
        nc = int(rng.integers(0, 3))
        u = rng.normal(size=(1 << k, 1 << k)) + 1j * rng.normal(size=(1 << k, 1 << k))
        tuples.append((tuple(qs[:k]), tuple(qs[k:k + nc]), tuple(int(v) for v in rng.integers(0, 2, nc)), u))
    gl = qc.GateList(tuples)
    assert gl.count == len(tuples)
    for i, (t, c, cv, u) in enumerate(tuples):
        g = gl.arr[i]
        assert g.n_targets == len(t) and g.n_ctrls == len(c)
        assert list(g.targets[:len(t)]) == list(t)
        assert list(g.ctrls[:len(c)]) == list(c)
        assert list(g.ctrl_vals[:len(c)]) == list(cv)
        d = 1 << len(t)
        got = np.ctypeslib.as_array(g.matrix, shape=(2 * d * d,)).view(np.complex128).reshape(d, d)
        assert np.array_equal(got, u)
    with pytest.raises(ValueError):
        qc.GateList([((0,), (), (), np.eye(4))])     # 4x4 matrix on one target
    empty = qc.GateList([])
    assert empty.count == 0


def _random_block_gates(rng, blk, sel, count):
    """Gates on the block labels `blk` with controls anywhere in blk + sel
    and diagonal gates allowed on the selector labels."""
    from tests.dense_ref import random_unitary
    every = list(blk) + list(sel)
    out = []
    for _ in range(count):
        kind = rng.integers(4)
        if kind == 0:   # diagonal gate over block and selector labels
            nt = int(rng.integers(1, min(3, len(every)) + 1))
            t = [int(x) for x in rng.choice(every, nt, replace=False)]
            u = np.diag(np.exp(1j * rng.uniform(-np.pi, np.pi, 1 << nt)))
        else:
            nt = int(rng.integers(1, min(3, len(blk)) + 1))
            t = [int(x) for x in rng.choice(blk, nt, replace=False)]
            u = random_unitary(1 << nt, rng)
        rest = [q for q in every if q not in t]
        nc = int(rng.integers(0, min(2, len(rest)) + 1))
        c = [int(x) for x in rng.choice(rest, nc, replace=False)] if nc else []
        cv = [int(x) for x in rng.integers(0, 2, nc)]
        out.append((t, c, cv, u))
    return out


@pytest.mark.parametrize("k,ns,seed", [(1, 0, 1), (2, 1, 2), (3, 2, 3), (4, 1, 4), (5, 0, 5),
                                       (5, 2, 6)])
def test_block_matrices_vs_dense_kronecker(qc, k, ns, seed):
    """The fuser's FP64 block products (section 3.2: a gate run on k qubits
    is the product of the gates' Kronecker-extended register operators)
    against brute-force dense operators: the register is the selector
    labels (most significant) then the block labels; its operator is block
    diagonal over the selector value, and block v is the fuser's matrix v."""
    from tests.dense_ref import dense_gate
    rng = np.random.default_rng(seed)
    labels = [int(x) for x in rng.permutation(9)[:k + ns]]
    blk, sel = labels[:k], labels[k:]
    gates = _random_block_gates(rng, blk, sel, 12)
    got = qc.block_matrices(qc.GateList(gates), blk, sel)
    order = sel + blk   # local qubit 0 = most significant
    nl = k + ns
    full = np.eye(1 << nl, dtype=np.complex128)
    for t, c, cv, u in gates:
        full = dense_gate(nl, [order.index(q) for q in t], u,
                          [order.index(q) for q in c], cv) @ full
    d = 1 << k
    for v in range(1 << ns):
        for w in range(1 << ns):
            blkvw = full[v * d:(v + 1) * d, w * d:(w + 1) * d]
            if v == w:
                assert np.max(np.abs(got[v] - blkvw)) <= 1e-14, (v, np.max(np.abs(got[v] - blkvw)))
            else:
                assert np.max(np.abs(blkvw)) == 0.0


def test_block_matrices_rejects_gates_outside_the_block(qc):
    from tests.dense_ref import random_unitary
    rng = np.random.default_rng(0)
    u = random_unitary(2, rng)
    with pytest.raises(RuntimeError):   # non-diagonal on a selector label
        qc.block_matrices(qc.GateList([([3], [], [], u)]), [0, 1], [3])
    with pytest.raises(RuntimeError):   # control outside every label
        qc.block_matrices(qc.GateList([([0], [5], [1], u)]), [0, 1], [3])
    with pytest.raises(RuntimeError):   # repeated label
        qc.block_matrices(qc.GateList([([0], [], [], u)]), [0, 1], [1])
