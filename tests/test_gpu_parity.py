"""GPU parity: every C-ABI entry point against the FP64 oracle, element by
element, on seeded inputs.

Tolerances (written per test):
* complex128: max |amplitude error| <= 1e-12 (absolute, unit-norm states).
* complex64: relative 2-norm error <= 1e-5 for circuits of depth <= 40;
  single gates and small circuits are held to tighter bounds derived from
  FP32 rounding (about 1e-7 per gate, times the number of gates).
* FP64 reductions: probabilities 1e-13 (c128) / 1e-6 (c64), expectations
  1e-11 * (number of terms) (c128) / 2 ||H|| * state error (c64).
"""
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


def check(got, ref, dtype, ngates=1):
    if dtype == torch.complex128:
        err = np.max(np.abs(got - ref))
        assert err <= 1e-12, err
    else:
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        bound = min(1e-5, 2e-7 * max(1, ngates) ** 0.5 * 4)
        assert rel <= bound, (rel, bound)


# ---------------------------------------------------------------- basics

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_init_and_copy(qc, dt):
    n = 11
    psi = qc.new_state(n, DT[dt])
    for b in (0, 1, 1234, (1 << n) - 1):
        qc.state_init(psi, b)
        ref = np.zeros(1 << n, complex)
        ref[b] = 1
        assert np.array_equal(host(psi), ref)
    src = dev(W.random_state(n, 5), torch.complex128)
    dst = qc.new_state(n, DT[dt])
    qc.state_copy(dst, src)
    want = src.to(DT[dt]).cpu().numpy().astype(np.complex128)
    assert np.array_equal(host(dst), want)


def test_same_precision_copy_sizes_and_alignment(qc):
    """The 16-byte vector copy at sizes below, at and above one 16 KiB
    chunk, and views that start 8 bytes into an allocation (the copy and the
    matrix-core block fall back to their 8-byte paths there)."""
    for dtype in (torch.complex64, torch.complex128):
        for n in (1, 2, 9, 11, 17):
            src = dev(W.random_state(n, 40 + n), dtype)
            dst = qc.new_state(n, dtype)
            qc.state_copy(dst, src)
            assert torch.equal(dst, src)
    n = 12
    base_src = torch.zeros((1 << n) + 1, dtype=torch.complex64, device="cuda")
    base_dst = torch.zeros((1 << n) + 1, dtype=torch.complex64, device="cuda")
    src, dst = base_src[1:], base_dst[1:]
    assert src.data_ptr() % 16 == 8
    psi0 = W.random_state(n, 41)
    src.copy_(torch.from_numpy(psi0).to(torch.complex64).cuda())
    qc.state_copy(dst, src)
    assert torch.equal(dst, src)
    u = random_unitary(32, np.random.default_rng(9))
    qc.apply_fused_k(dst, [0, 3, 5, 8, 11], u)
    check(host(dst), oracle.apply(host(src), [0, 3, 5, 8, 11], u), torch.complex64, ngates=8)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 7, 13])
def test_apply_1q_every_target(qc, dt, n):
    rng = np.random.default_rng(n)
    psi0 = W.random_state(n, 100 + n)
    for q in range(n):
        u = random_unitary(2, rng)
        t = dev(psi0, DT[dt])
        qc.apply_1q(t, q, u)
        check(host(t), oracle.apply(psi0, [q], u), DT[dt])


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_apply_2q_pairs(qc, dt):
    n = 9
    rng = np.random.default_rng(2)
    psi0 = W.random_state(n, 9)
    for a in range(n):
        for b in range(n):
            if a == b or (a + b) % 3:
                continue
            u = random_unitary(4, rng)
            t = dev(psi0, DT[dt])
            qc.apply_2q(t, a, b, u)
            check(host(t), oracle.apply(psi0, [a, b], u), DT[dt])


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_apply_controlled(qc, dt):
    n = 10
    rng = np.random.default_rng(3)
    psi0 = W.random_state(n, 10)
    for nc in (1, 2, 3, 5):
        for trial in range(3):
            perm = list(rng.permutation(n))
            ctrl, tgt = perm[:nc], perm[nc]
            cv = list(rng.integers(0, 2, nc))
            u = random_unitary(2, rng)
            t = dev(psi0, DT[dt])
            qc.apply_controlled(t, ctrl, cv, tgt, u)
            check(host(t), oracle.apply(psi0, [tgt], u, ctrl, cv), DT[dt])
    # diagonal with U00 == 1 takes the phase-only path (CZ, CP)
    for ph in (math.pi, 0.7):
        u = np.diag([1.0, np.exp(1j * ph)])
        t = dev(psi0, DT[dt])
        qc.apply_controlled(t, [2, 7], [1, 0], 4, u)
        check(host(t), oracle.apply(psi0, [4], u, [2, 7], [1, 0]), DT[dt])


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_apply_fused_k_random_qubits(qc, dt, k):
    n = 12
    rng = np.random.default_rng(40 + k)
    psi0 = W.random_state(n, 12)
    for trial in range(4):
        qs = list(rng.permutation(n)[:k])
        u = random_unitary(1 << k, rng)
        t = dev(psi0, DT[dt])
        qc.apply_fused_k(t, qs, u)
        check(host(t), oracle.apply(psi0, qs, u), DT[dt], ngates=4)


@pytest.mark.parametrize("tile_bits", [13, 12])
@pytest.mark.parametrize("n", [12, 13, 16, 20])
def test_fused_mfma_target_positions(qc, n, tile_bits):
    """The complex64 matrix-core path for every kind of target placement:
    all-low bits, all-high bits, mixed, reversed order, a single tile; both
    tile shapes (13: 32 x 256, used from 13 qubits; 12: 32 x 128), and
    multiplexed blocks with selectors in and above the tile."""
    old = qc.get_knob(qc.QC_KNOB_MFMA_TILE_BITS)
    qc.set_knob(qc.QC_KNOB_MFMA_TILE_BITS, tile_bits)
    try:
        rng = np.random.default_rng(n)
        psi0 = W.random_state(n, 1000 + n)
        cases = [list(range(n - 5, n)), list(range(5)), [n - 1, 0, n // 2, 2, n - 3],
                 list(reversed(range(n - 5, n))), list(rng.permutation(n)[:5])]
        for qs in cases:
            u = random_unitary(32, rng)
            t = dev(psi0, torch.complex64)
            qc.apply_fused_k(t, qs, u)
            check(host(t), oracle.apply(psi0, qs, u), torch.complex64, ngates=8)
        if n >= 14:
            layouts = [(list(range(5)), [n - 6, n - 7]),           # selectors among the columns
                       (list(range(n - 5, n)), [0, 1]),            # selectors above the tile
                       ([1, 2, 3, 4, 5], [n - 6, 0])]              # one of each
            for qs, sel in layouts:
                us = np.stack([random_unitary(32, rng) for _ in range(1 << len(sel))])
                t = dev(psi0, torch.complex64)
                qc.apply_multiplexed(t, qs, sel, us)
                check(host(t), mux_oracle(psi0, qs, sel, us), torch.complex64, ngates=8)
    finally:
        qc.set_knob(qc.QC_KNOB_MFMA_TILE_BITS, old)


@pytest.mark.parametrize("n", [12, 13, 16, 20])
def test_fused_mfma_c128_target_positions(qc, n):
    """The complex128 FP64 matrix-core path (32 x 128 tiles) for every kind
    of target placement, and multiplexed blocks with selectors in and above
    the tile, against the oracle at the complex128 tolerance."""
    rng = np.random.default_rng(500 + n)
    psi0 = W.random_state(n, 3000 + n)
    cases = [list(range(n - 5, n)), list(range(5)), [n - 1, 0, n // 2, 2, n - 3],
             list(reversed(range(n - 5, n))), list(rng.permutation(n)[:5])]
    for qs in cases:
        u = random_unitary(32, rng)
        t = dev(psi0, torch.complex128)
        qc.apply_fused_k(t, qs, u)
        check(host(t), oracle.apply(psi0, qs, u), torch.complex128, ngates=8)
    if n >= 14:
        layouts = [(list(range(5)), [n - 6, n - 7]),           # selectors among the columns
                   (list(range(n - 5, n)), [0, 1]),            # selectors above the tile
                   ([1, 2, 3, 4, 5], [n - 6, 0])]              # one of each
        for qs, sel in layouts:
            us = np.stack([random_unitary(32, rng) for _ in range(1 << len(sel))])
            t = dev(psi0, torch.complex128)
            qc.apply_multiplexed(t, qs, sel, us)
            check(host(t), mux_oracle(psi0, qs, sel, us), torch.complex128, ngates=8)


def mux_oracle(psi, qs, sel, us):
    """A multiplexed gate as 2^c controlled k-qubit gates, one per selector
    value v, each controlled on the selector qubits reading v."""
    c = len(sel)
    for v in range(1 << c):
        vals = [(v >> (c - 1 - j)) & 1 for j in range(c)]
        psi = oracle.apply(psi, qs, us[v], ctrl=sel, ctrl_val=vals)
    return psi


@pytest.mark.parametrize("dt,n,k,c", [
    ("c64", 14, 5, 2), ("c64", 16, 5, 1), ("c64", 13, 5, 2), ("c64", 11, 3, 2),
    ("c128", 12, 5, 2), ("c128", 9, 2, 1), ("c64", 12, 5, 0)])
def test_apply_multiplexed(qc, dt, n, k, c):
    """qc_apply_multiplexed on the matrix-core path (complex64, k = 5,
    n >= 12 + c) and on the vector path, with selector qubits at the lowest
    and highest bit positions and in between."""
    rng = np.random.default_rng(100 * n + 10 * k + c)
    psi0 = W.random_state(n, 2000 + n)
    layouts = [
        (list(range(k)), list(range(n - c, n))),             # selectors at the lowest bits
        (list(range(n - k, n)), list(range(c))),             # selectors at the highest bits
        ([int(x) for x in rng.permutation(n)[:k + c]][:k], None),
    ]
    for qs, sel in layouts:
        if sel is None:
            rest = [q for q in rng.permutation(n) if q not in qs]
            sel = [int(x) for x in rest[:c]]
        us = np.stack([random_unitary(1 << k, rng) for _ in range(1 << c)])
        t = dev(psi0, DT[dt])
        qc.apply_multiplexed(t, qs, sel, us)
        check(host(t), mux_oracle(psi0, qs, sel, us), DT[dt], ngates=8)


# ---------------------------------------------------------------- circuits

def _mixed_ops(n, rng, count=60):
    """Dense 1q/2q/3q gates, CZ, CP, RZ, CNOT and open-control MCX gates on
    random qubits."""
    ops = []
    for _ in range(count):
        kind = rng.integers(0, 8)
        q = [int(x) for x in rng.permutation(n)[:4]]
        if kind == 0:
            ops.append(W.Op("U", (q[0],), matrix=random_unitary(2, rng)))
        elif kind == 1:
            ops.append(W.Op("U", (q[0], q[1]), matrix=random_unitary(4, rng)))
        elif kind == 2:
            ops.append(W.Op("CZ", (q[0], q[1])))
        elif kind == 3:
            ops.append(W.Op("CP", (q[0], q[1]), angle=float(rng.uniform(0, 6))))
        elif kind == 4:
            ops.append(W.Op("RZ", (q[0],), angle=float(rng.uniform(0, 6))))
        elif kind == 5:
            ops.append(W.Op("MCX", (q[0], q[1], q[2]), ctrl_val=(int(rng.integers(0, 2)), 1)))
        elif kind == 6 and n >= 4:
            ops.append(W.Op("U", (q[0], q[1], q[2]), matrix=random_unitary(8, rng)))
        else:
            ops.append(W.Op("CNOT", (q[0], q[1])))
    return ops


@pytest.mark.parametrize("tile_bits", [13, 10, 7])
@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [6, 13, 17])
def test_tiled_runs_mixed_gates(qc, G, dt, n, tile_bits):
    """LDS tile runs: dense 1q/2q gates, diagonal gates on bits inside and
    outside the tile, controls inside and outside the tile, open controls,
    gates that cannot join a run (3-qubit), across several tiles; at the
    default tile size and two smaller ones (QC_KNOB_TILE_BITS)."""
    rng = np.random.default_rng(n)
    ops = _mixed_ops(n, rng)
    psi0 = W.random_state(n, 50 + n)
    ref = oracle.run(ops, psi0)
    t = dev(psi0, DT[dt])
    old = qc.get_knob(qc.QC_KNOB_TILE_BITS)
    qc.set_knob(qc.QC_KNOB_TILE_BITS, tile_bits)
    try:
        st = qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=2)
    finally:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, old)
    assert st["sweeps"] < len(ops)
    check(host(t), ref, DT[dt], ngates=len(ops))


@pytest.mark.parametrize("n", [21, 22])
def test_tiled_wide_complex128(qc, G, n):
    """complex128 tile runs in the wide register tiles (2^13 amplitudes, 16
    per thread; QC_KNOB_WIDE_MIN_TILES lowered to 8 so that 21 and 22 qubits
    take them): mixed gates and the QFT against the oracle, and against the
    2^12-amplitude tiles (QC_KNOB_TILE_BITS = 12) over the whole state."""
    rng = np.random.default_rng(300 + n)
    for ops in (_mixed_ops(n, rng), W.qft(n)):
        psi0 = W.random_state(n, 310 + n)
        ref = oracle.run(ops, psi0)
        gl = qc.GateList(G.gate_tuples(ops))
        t = dev(psi0, torch.complex128)
        old_wide = qc.get_knob(qc.QC_KNOB_WIDE_MIN_TILES)
        try:
            qc.set_knob(qc.QC_KNOB_WIDE_MIN_TILES, 8)
            st = qc.apply_circuit(t, gl, mode=2)
        finally:
            qc.set_knob(qc.QC_KNOB_WIDE_MIN_TILES, old_wide)
        assert st["sweeps"] < len(ops)
        check(host(t), ref, torch.complex128, ngates=len(ops))
        narrow = dev(psi0, torch.complex128)
        old = qc.get_knob(qc.QC_KNOB_TILE_BITS)
        try:
            qc.set_knob(qc.QC_KNOB_TILE_BITS, 12)
            qc.apply_circuit(narrow, gl, mode=2)
        finally:
            qc.set_knob(qc.QC_KNOB_TILE_BITS, old)
        assert np.max(np.abs(host(t) - host(narrow))) < 1e-12


def test_tiled_wide_lds_fallback(qc, G):
    """A complex128 run in wide tiles whose controlled-phase fans carry more
    lane tables than the register engine's LDS budget (24 fans, one lane
    table each) runs on the LDS-resident engine
    with 2^13-amplitude tiles (128 KiB of LDS), behind a register-tile run of
    Hadamards whose deferred factor it applies; against the oracle and
    against the same circuit in 2^12-amplitude tiles."""
    n = 21
    rng = np.random.default_rng(404)
    ops = []
    targets = [0, 1, 2, 3, 4, 5, 6, 7]          # qubits 0..7 = bits 20..13
    # first a register-tile run with Hadamards (their 1/sqrt2 factors are
    # left pending for the next run, here the LDS-engine one)
    for q in range(13, 18):
        ops.append(W.Op("H", (q,)))
        if q < 17:
            ops.append(W.Op("CP", (q + 1, q), angle=0.7))
    for r in range(24):
        q = targets[r % 8]
        ops.append(W.Op("U", (q,), matrix=random_unitary(2, rng)))
        # controls: the next two targets (the next gate then closes this
        # fan) and one low-bit qubit
        for c in (targets[(r + 1) % 8], targets[(r + 2) % 8], 16 + r % 5):
            ops.append(W.Op("CP", (int(c), q), angle=float(rng.uniform(0, 6))))
    psi0 = W.random_state(n, 405)
    ref = oracle.run(ops, psi0)
    gl = qc.GateList(G.gate_tuples(ops))
    old_wide = qc.get_knob(qc.QC_KNOB_WIDE_MIN_TILES)
    calls0, _ = qc.timing_query("tile_run_c128")
    try:
        qc.set_knob(qc.QC_KNOB_WIDE_MIN_TILES, 8)
        t = dev(psi0, torch.complex128)
        qc.timing_enable(True)
        qc.apply_circuit(t, gl, mode=2)
        torch.cuda.synchronize()
        calls, _ = qc.timing_query("tile_run_c128")
    finally:
        qc.timing_enable(False)
        qc.set_knob(qc.QC_KNOB_WIDE_MIN_TILES, old_wide)
    assert calls > calls0, "the run did not take the LDS-resident engine"
    check(host(t), ref, torch.complex128, ngates=len(ops))
    narrow = dev(psi0, torch.complex128)
    old = qc.get_knob(qc.QC_KNOB_TILE_BITS)
    try:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, 12)
        qc.apply_circuit(narrow, gl, mode=2)
    finally:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, old)
    assert np.max(np.abs(host(t) - host(narrow))) < 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_tiled_hadamard_factor_before_standalone_gates(qc, G, dt):
    """Register-tile runs of Hadamards separated by gates that no tile run
    takes (three-qubit dense gates): the 1/sqrt2 factors a run leaves out
    are applied before each such gate and at the end; against the oracle."""
    n = 21
    rng = np.random.default_rng(91)
    ops = []
    for block in range(3):
        for q in rng.permutation(n)[:7]:
            ops.append(W.Op("H", (int(q),)))
            a, b = [int(x) for x in rng.permutation(n)[:2]]
            ops.append(W.Op("CP", (a, b), angle=float(rng.uniform(0, 6))))
        q3 = [int(x) for x in rng.permutation(n)[:3]]
        ops.append(W.Op("U", tuple(q3), matrix=random_unitary(8, rng)))
    ops.append(W.Op("H", (3,)))
    psi0 = W.random_state(n, 92)
    t = dev(psi0, DT[dt])
    st = qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=2)
    assert st["sweeps"] < len(ops)
    check(host(t), oracle.run(ops, psi0), DT[dt], ngates=len(ops))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_tiled_plan_reuse(qc, G, dt):
    """A tiled circuit applied again reuses its plan: two applications of
    one gate list to fresh states, then the same list with one matrix
    changed in place (the plan must not be reused), each against the
    oracle."""
    n = 21
    rng = np.random.default_rng(77)
    ops = _mixed_ops(n, rng, count=40)
    psi0 = W.random_state(n, 78)
    gl = qc.GateList(G.gate_tuples(ops))
    ref = oracle.run(ops, psi0)
    for _ in range(2):
        t = dev(psi0, DT[dt])
        qc.apply_circuit(t, gl, mode=2)
        check(host(t), ref, DT[dt], ngates=len(ops))
    k = next(i for i, op in enumerate(ops) if op.kind == "U" and len(op.qubits) == 1)
    u = random_unitary(2, rng)
    off = sum(np.asarray(g[3]).size for g in G.gate_tuples(ops[:k]))
    gl._mats[off:off + 4] = u.reshape(-1)
    ops2 = list(ops)
    ops2[k] = W.Op("U", ops[k].qubits, matrix=u)
    t = dev(psi0, DT[dt])
    qc.apply_circuit(t, gl, mode=2)
    check(host(t), oracle.run(ops2, psi0), DT[dt], ngates=len(ops))


@pytest.mark.parametrize("tile_bits", [13, 10, 7])
@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [8, 16])
def test_tiled_dense_then_phases(qc, G, dt, n, tile_bits):
    """Tile runs where a one-qubit gate is followed by diagonal terms (the
    pattern a tile run applies in one pass): QFT, and random one-qubit gates
    each followed by 1-4 controlled phases and CZs whose qubits lie inside
    and outside the tile, including single terms with a control outside."""
    rng = np.random.default_rng(7 * n + tile_bits)
    rand_ops = []
    for _ in range(40):
        q = int(rng.integers(0, n))
        rand_ops.append(W.Op("U", (q,), matrix=random_unitary(2, rng)))
        for _ in range(int(rng.integers(1, 5))):
            a, b = [int(x) for x in rng.permutation(n)[:2]]
            if rng.integers(0, 3) == 0:
                rand_ops.append(W.Op("CZ", (a, b)))
            else:
                rand_ops.append(W.Op("CP", (a, b), angle=float(rng.uniform(0, 6))))
    old = qc.get_knob(qc.QC_KNOB_TILE_BITS)
    try:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, tile_bits)
        for ops in (W.qft(n), rand_ops):
            psi0 = W.random_state(n, 90 + n)
            ref = oracle.run(ops, psi0)
            t = dev(psi0, DT[dt])
            st = qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=2)
            assert st["sweeps"] < len(ops)
            check(host(t), ref, DT[dt], ngates=len(ops))
    finally:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, old)


def swap_ops_for(perm):
    """SWAP gates after which qubit q of the register sits at label perm[q]."""
    n = len(perm)
    at = list(range(n))      # at[label] = original qubit held there
    where = list(range(n))   # where[q] = label holding original qubit q
    ops = []
    for label in range(n):
        q = perm.index(label)
        if where[q] != label:
            other = at[label]
            ops.append(W.Op("SWAP", (label, where[q])))
            at[where[q]], at[label] = other, q
            where[other], where[q] = where[q], label
    return ops


PERMS = {
    "reverse": lambda n, rng: list(range(n))[::-1],
    "random": lambda n, rng: [int(x) for x in rng.permutation(n)],
    "cycle3": lambda n, rng: [1, 2, 0] + list(range(3, n)) if n >= 3 else list(range(n))[::-1],
    "hi_lo": lambda n, rng: [n - 1] + list(range(1, n - 1)) + [0] if n >= 2 else [0],
}


@pytest.mark.parametrize("kind", sorted(PERMS))
@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 7, 12, 17])
def test_permute_qubits(qc, dt, n, kind):
    """qc_permute_qubits against the oracle's SWAP gates (and the relabelling
    written as a transpose of the 2 x ... x 2 tensor): amplitudes move
    unchanged, so the match is exact."""
    rng = np.random.default_rng(31 * n + len(kind))
    perm = PERMS[kind](n, rng)
    psi0 = W.random_state(n, 300 + n)
    ref = oracle.run(swap_ops_for(perm), psi0)
    inv = [perm.index(axis) for axis in range(n)]
    assert np.array_equal(ref, psi0.reshape([2] * n).transpose(inv).reshape(-1))
    t = dev(psi0, DT[dt])
    qc.permute_qubits(t, perm)
    want = ref.astype(np.complex64) if dt == "c64" else ref
    assert np.array_equal(host(t), want)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("n", [10, 15])
def test_circuit_with_swaps(qc, G, dt, mode, n):
    """SWAP gates between other gates (fused and tiled modes leave them out
    and relabel the later gates): the result against the oracle."""
    rng = np.random.default_rng(n + 10 * mode)
    ops = []
    for _ in range(80):
        kind = rng.integers(0, 5)
        q = [int(x) for x in rng.permutation(n)[:2]]
        if kind == 0:
            ops.append(W.Op("SWAP", (q[0], q[1])))
        elif kind == 1:
            ops.append(W.Op("U", (q[0],), matrix=random_unitary(2, rng)))
        elif kind == 2:
            ops.append(W.Op("CP", (q[0], q[1]), angle=float(rng.uniform(0, 6))))
        elif kind == 3:
            ops.append(W.Op("CNOT", (q[0], q[1])))
        else:
            ops.append(W.Op("U", (q[0], q[1]), matrix=random_unitary(4, rng)))
    psi0 = W.random_state(n, 400 + n)
    ref = oracle.run(ops, psi0)
    t = dev(psi0, DT[dt])
    st = qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=mode, fuse_k=4)
    assert st["gates"] == len(ops)
    check(host(t), ref, DT[dt], ngates=len(ops))


@pytest.mark.parametrize("mode", [1, 2])
def test_qft_final_swaps_take_one_sweep(qc, G, mode):
    """The QFT's closing SWAP network relabels no gate (nothing follows it),
    and together it is its own inverse: one extra sweep over the state."""
    n = 16
    ops = W.qft(n)
    core = [op for op in ops if op.kind != "SWAP"]
    psi0 = W.random_state(n, 28)
    sweeps = []
    for lst in (ops, core):
        t = dev(psi0, torch.complex64)
        sweeps.append(qc.apply_circuit(t, qc.GateList(G.gate_tuples(lst)), mode=mode, fuse_k=5)["sweeps"])
    assert sweeps[0] == sweeps[1] + 1
    check(host(t), oracle.run(core, psi0), torch.complex64, ngates=len(core))   # t: the core run


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_brickwork12_config(qc, G, dt, mode):
    """12-qubit brickwork, 20 layers of Haar U(2) + CNOT (350 gates) from
    |0..0>: full state and all 4096 probabilities."""
    n, ops = W.config_brickwork12()
    ref = oracle.run(ops, oracle.basis_state(n, 0))
    t = qc.new_state(n, DT[dt])
    qc.state_init(t, 0)
    st = qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=mode, fuse_k=5)
    assert st["gates"] == len(ops)
    check(host(t), ref, DT[dt], ngates=len(ops))
    p = qc.probs(t).cpu().numpy()
    tol = 1e-13 if dt == "c128" else 1e-6
    assert np.max(np.abs(p - oracle.probs(ref))) < tol


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_qft_random_state(qc, G, dt, mode):
    n = 14
    psi0 = W.random_state(n, 28)
    ops = W.qft(n)
    ref = oracle.run(ops, psi0)
    t = dev(psi0, DT[dt])
    qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)), mode=mode, fuse_k=5)
    check(host(t), ref, DT[dt], ngates=len(ops))


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_qft24_small_tiles(qc, G, dt):
    """24-qubit QFT in tile runs of 7-bit tiles: a controlled-phase fan then
    has more than 16 controls outside the tile, so its phases span two fan
    ops.  Against the unfused complex128 run (whole state) and the oracle's
    Fourier sums (sampled amplitudes)."""
    n = 24
    ops = W.qft(n)
    psi0 = W.random_state(n, 24)
    gl = qc.GateList(G.gate_tuples(ops))
    ref = dev(psi0, torch.complex128)
    qc.apply_circuit(ref, gl, mode=0)
    t = dev(psi0, DT[dt])
    old = qc.get_knob(qc.QC_KNOB_TILE_BITS)
    try:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, 7)
        qc.apply_circuit(t, gl, mode=2)
    finally:
        qc.set_knob(qc.QC_KNOB_TILE_BITS, old)
    torch.cuda.synchronize()
    for y in (0, 1, 987654 % (1 << n), (1 << n) - 1):
        want = oracle.qft_amplitude(psi0, y)
        assert abs(complex(ref[y].item()) - want) < 1e-12, y
    d = qc.state_diff(t, ref).cpu().numpy()
    if dt == "c128":
        assert np.max(np.abs(host(t) - host(ref))) < 1e-12
    else:
        assert math.sqrt(d[0] / d[1]) < 1e-5


def test_qft28_sampled_amplitudes(qc, G):
    """28-qubit QFT on the seeded Gaussian state (4 GiB complex128): sampled
    output amplitudes against the oracle's discrete Fourier sum, and the
    complex64 run against the complex128 run."""
    n, ops, psi0 = W.config_qft28()
    gl = qc.GateList(G.gate_tuples(ops))
    t = dev(psi0, torch.complex128)
    qc.apply_circuit(t, gl, mode=0)
    t64 = dev(psi0, torch.complex64)
    qc.apply_circuit(t64, gl, mode=1, fuse_k=5)
    torch.cuda.synchronize()
    for y in (0, 1, 123456789 % (1 << n), (1 << n) - 1):
        ref = oracle.qft_amplitude(psi0, y)
        got = complex(t[y].item())
        assert abs(got - ref) < 1e-12, (y, got, ref)
    d = qc.state_diff(t64, t).cpu().numpy()
    assert math.sqrt(d[0] / d[1]) < 1e-5
    del t, t64
    torch.cuda.empty_cache()


def test_paper_examples_on_gpu(qc, G):
    """Bell, Grover and the error-correction circuit of the paper, run
    through the GPU path (the measured qubits of the error-correction
    circuit have a certain outcome, so measuring them leaves the state as
    is)."""
    # Bell: P = 0.5 / 0.5 on |00>, |11>
    t = qc.new_state(2, torch.complex128)
    qc.state_init(t, 0)
    qc.apply_circuit(t, qc.GateList(G.gate_tuples([W.Op("H", (0,)), W.Op("CNOT", (0, 1))])))
    np.testing.assert_allclose(qc.probs(t).cpu().numpy(), [0.5, 0, 0, 0.5], atol=1e-15)
    # Grover on two qubits finds |11> with probability 1
    H0, H1 = W.Op("H", (0,)), W.Op("H", (1,))
    ops = [H0, H1, W.Op("CZ", (0, 1)), H0, H1, W.Op("Z", (0,)), W.Op("Z", (1,)),
           W.Op("CZ", (0, 1)), H0, H1]
    qc.state_init(t, 0)
    qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)))
    np.testing.assert_allclose(qc.probs(t).cpu().numpy(), [0, 0, 0, 1], atol=1e-15)
    # error correction: syndrome '11' with probability 1, final state
    v = np.array([1.0, 1j]) / math.sqrt(2)
    init = np.kron(v, np.eye(16)[:, 0])
    ops = [W.Op("CNOT", (0, 1)), W.Op("CNOT", (0, 2)), W.Op("X", (0,)), W.Op("CNOT", (0, 3)),
           W.Op("CNOT", (1, 3)), W.Op("CNOT", (0, 4)), W.Op("CNOT", (2, 4)),
           W.Op("MCX", (3, 4, 2), ctrl_val=(0, 1)), W.Op("MCX", (3, 4, 1), ctrl_val=(1, 0)),
           W.Op("MCX", (3, 4, 0), ctrl_val=(1, 1))]
    t = dev(init, torch.complex128)
    qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops)))
    np.testing.assert_allclose(qc.probs(t, [3, 4]).cpu().numpy(), [0, 0, 0, 1], atol=1e-15)
    ref = np.zeros(32, complex)
    ref[0b00011], ref[0b11111] = 1 / math.sqrt(2), 1j / math.sqrt(2)
    np.testing.assert_allclose(host(t), ref, atol=1e-15)


# ---------------------------------------------------------------- reductions

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_probs_full_and_marginal(qc, dt):
    n = 13
    psi0 = W.random_state(n, 13)
    t = dev(psi0, DT[dt])
    ref_state = host(t)   # the rounded state the GPU actually holds
    tol = 1e-15
    np.testing.assert_allclose(qc.probs(t).cpu().numpy(), oracle.probs(ref_state), atol=tol)
    for qs in ([0], [12], [5, 2], [12, 0, 6], list(range(8)), list(reversed(range(n))),
               [3, 9, 1, 11, 7, 0]):
        got = qc.probs(t, qs).cpu().numpy()
        np.testing.assert_allclose(got, oracle.probs(ref_state, qs), atol=1e-14)
    assert abs(qc.probs(t, [4]).cpu().numpy().sum() - 1) < (1e-13 if dt == "c128" else 1e-6)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_expect_pauli_random_terms(qc, dt):
    n = 11
    rng = np.random.default_rng(4)
    psi0 = W.random_state(n, 21)
    t = dev(psi0, DT[dt])
    st = host(t)
    terms = [("".join(rng.choice(list("IXYZ"), n)), float(rng.normal())) for _ in range(40)]
    terms += [("I" * n, 0.5), ("X" * n, 1.0), ("Y" * n, -1.0), ("Z" * n, 2.0)]
    out = qc.expect_pauli(t, terms, per_term=True).cpu().numpy()
    ref_terms = np.array([oracle.expect_pauli(st, p).real for p, _ in terms])
    np.testing.assert_allclose(out[1:], ref_terms, atol=1e-13)
    assert abs(out[0] - sum(c * r for (_, c), r in zip(terms, ref_terms))) < 1e-12


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n", [16, 19])
def test_expect_pauli_tile_passes(qc, dt, n):
    """Registers larger than one expectation tile: Ising terms spread over
    several tile passes, X bits straddling low and high positions, Z bits
    outside the tile, Y-heavy strings, and strings with more high X bits
    than a tile holds (evaluated by the pair kernel)."""
    rng = np.random.default_rng(100 + n)
    psi0 = W.random_state(n, 22)
    t = dev(psi0, DT[dt])
    st = host(t)
    terms = list(W.tfim_terms(n))
    def one(spec):
        s = ["I"] * n
        for q, c in spec.items():
            s[q] = c
        return "".join(s)
    terms += [(one({0: "X", n - 1: "X"}), 0.7), (one({0: "Y", 1: "Y"}), -0.4),
              (one({n - 1: "Y", n - 2: "X", 0: "Z"}), 0.25), ("Z" * n, 1.5),
              (one({q: "X" for q in range(0, n, 2)}), 0.3),            # many high X bits
              (one({q: "Y" for q in range(n - 6, n)}), -0.6),          # low bits only
              (one({q: "X" for q in range(6)}), 0.9)]                  # high bits only
    for _ in range(24):
        terms.append(("".join(rng.choice(list("IIIXYZ"), n)), float(rng.normal())))
    out = qc.expect_pauli(t, terms, per_term=True).cpu().numpy()
    ref_terms = np.array([oracle.expect_pauli(st, p).real for p, _ in terms])
    np.testing.assert_allclose(out[1:], ref_terms, atol=1e-12)
    assert abs(out[0] - sum(c * r for (_, c), r in zip(terms, ref_terms))) < 1e-11
    # identical on a second call (fixed-order reductions)
    out2 = qc.expect_pauli(t, terms, per_term=True).cpu().numpy()
    assert np.array_equal(out, out2)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_tfim_energy_after_hea(qc, G, dt):
    n = 14
    theta = np.random.default_rng(5).uniform(0, 2 * math.pi, 4 * n * 2)
    ops = W.hea(n, 4)
    ref = oracle.run(ops, oracle.basis_state(n, 0), theta)
    terms = W.tfim_terms(n)
    e_ref = oracle.energy(ref, terms)
    t = qc.new_state(n, DT[dt])
    qc.state_init(t, 0)
    qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops, theta)))
    e = qc.expect_pauli(t, terms)[0].item()
    tol = 1e-11 * len(terms) if dt == "c128" else 2 * (2 * n - 1) * 1e-5
    assert abs(e - e_ref) < tol


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_state_diff(qc, dt):
    n = 12
    a0, b0 = W.random_state(n, 1), W.random_state(n, 2)
    a, b = dev(a0, DT[dt]), dev(b0, torch.complex128)
    d = qc.state_diff(a, b).cpu().numpy()
    ah = host(a)
    assert abs(d[0] - np.sum(np.abs(ah - b0) ** 2)) < 1e-12
    assert abs(d[1] - np.sum(np.abs(b0) ** 2)) < 1e-12
    assert abs(d[2] - np.max(np.abs(ah - b0))) < 1e-12


# ---------------------------------------------------------------- gradients

@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_gradient_vs_parameter_shift(qc, dt):
    n, layers = 8, 3
    ops = W.hea(n, layers)
    terms = W.tfim_terms(n)
    theta = np.random.default_rng(24).uniform(0, 2 * math.pi, layers * n * 2)
    psi0 = oracle.basis_state(n, 0)
    g_ref = oracle.param_shift_grad(ops, theta, terms, psi0)
    e_ref = oracle.energy(oracle.run(ops, psi0, theta), terms)
    psi = qc.new_state(n, DT[dt])
    lam = qc.new_state(n, DT[dt])
    qc.state_init(psi, 0)
    e, g = qc.adjoint_grad(psi, lam, ops, theta, terms)
    e, g = e.item(), g.cpu().numpy()
    if dt == "c128":
        assert abs(e - e_ref) < 1e-11
        np.testing.assert_allclose(g, g_ref, atol=1e-9)
        # the backward pass un-computes the forward pass
        back = host(psi)
        assert np.max(np.abs(back - psi0)) < 1e-12
    else:
        bound = 2 * (2 * n - 1) * 1e-5
        assert abs(e - e_ref) < bound
        assert np.max(np.abs(g - g_ref)) < bound


def test_adjoint_shared_parameters_and_all_kinds(qc):
    n = 5
    ops = [W.Op("H", (0,)), W.Op("RX", (1,), pidx=0), W.Op("RY", (2,), pidx=0),
           W.Op("CNOT", (1, 3)), W.Op("RZ", (3,), pidx=1), W.Op("Y", (4,)), W.Op("CZ", (0, 4)),
           W.Op("RY", (4,), pidx=2), W.Op("X", (2,)), W.Op("Z", (1,)), W.Op("RX", (0,), pidx=1)]
    terms = [("ZZIII", 1.0), ("IXYII", -0.5), ("YIIZX", 0.3), ("IIIIX", 2.0)]
    theta = np.array([0.3, -1.2, 2.2])
    psi0 = W.random_state(n, 77)
    g_ref = oracle.param_shift_grad(ops, theta, terms, psi0)
    psi = dev(psi0, torch.complex128)
    lam = qc.new_state(n, torch.complex128)
    e, g = qc.adjoint_grad(psi, lam, ops, theta, terms)
    np.testing.assert_allclose(g.cpu().numpy(), g_ref, atol=1e-12)
    assert abs(e.item() - oracle.energy(oracle.run(ops, psi0, theta), terms)) < 1e-12


def _dblock_case():
    n = 20
    ops = [W.Op("RY", (q,), pidx=q % 4) for q in range(n)]
    ops += [W.Op("RZ", (q,), pidx=4 + (q % 3)) for q in range(n)]
    ops += [W.Op("RZ", (7,), pidx=7)]                        # a second RZ on one qubit
    ops += [W.Op("CZ", (q, q + 1)) for q in range(0, n - 1, 2)]
    ops += [W.Op("H", (3,)), W.Op("X", (11,)), W.Op("RX", (5,), pidx=8), W.Op("CNOT", (2, 17)),
            W.Op("Y", (19,)), W.Op("Z", (0,))]
    ops += [W.Op("RZ", (q,), pidx=4 + (q % 2)) for q in range(0, n, 3)]
    ops += [W.Op("RY", (q,), pidx=q % 4) for q in range(1, n, 4)]
    terms = list(W.tfim_terms(n)) + [("XY" + "I" * (n - 4) + "ZX", 0.4)]
    theta = np.random.default_rng(5).normal(size=9)
    return n, ops, terms, theta, W.random_state(n, 91)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_register_backward_diagonal_blocks(qc, dt):
    """20 qubits, so the backward runs use register tiles: a layer's RZ
    rotations (on register slots, thread bits and bits outside the tile,
    one qubit twice) run as one block whose gradients come from the block's
    start, with fixed one-qubit gates, RX, CNOT and CZ between layers and
    shared parameters.  Against the LDS-tile backward pass (one rotation at
    a time), the oracle's energy and its central differences."""
    n, ops, terms, theta, psi0 = _dblock_case()

    def grad(engine, dtype):
        old = qc.get_knob(qc.QC_KNOB_TILE_ENGINE)
        qc.set_knob(qc.QC_KNOB_TILE_ENGINE, engine)
        try:
            psi = dev(psi0, dtype)
            lam = qc.new_state(n, dtype)
            e, g = qc.adjoint_grad(psi, lam, ops, theta, terms)
            return e.item(), g.cpu().numpy()
        finally:
            qc.set_knob(qc.QC_KNOB_TILE_ENGINE, old)

    e_rt, g_rt = grad(1, DT[dt])
    e_ref = oracle.energy(oracle.run(ops, psi0, theta), terms)
    if dt == "c128":
        e_lds, g_lds = grad(0, torch.complex128)
        np.testing.assert_allclose(g_rt, g_lds, atol=1e-12)
        assert abs(e_rt - e_ref) < 1e-12
        idx = [0, 4, 5, 7, 8]
        g_fd = oracle.fd_grad(ops, theta, terms, psi0, indices=idx)
        np.testing.assert_allclose(g_rt[idx], g_fd, atol=1e-7)
    else:
        _, g128 = grad(1, torch.complex128)
        bound = 2 * sum(abs(c) for _, c in terms) * 1e-5
        assert abs(e_rt - e_ref) < bound
        assert np.max(np.abs(g_rt - g128)) < bound


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_general_hamiltonian_register_passes(qc, dt):
    """lam = H phi on a 14-qubit register (register-tile passes): terms with
    X bits on the lanes, on one element bit, on the lanes and an element at
    once or on two element bits (the gather kernel adds those), Y phases,
    Z signs inside and outside the tile, against the oracle's energy and
    parameter-shift gradients."""
    n = 14
    ops = [W.Op("H", (q,)) for q in range(n)]
    ops += [W.Op("RY", (q,), pidx=(q // 2) % 6) for q in range(0, n, 2)]
    ops += [W.Op("CZ", (q, q + 1)) for q in range(n - 1)]
    ops += [W.Op("RX", (q,), pidx=6 + q % 3) for q in range(1, n, 3)]
    ops += [W.Op("RZ", (q,), pidx=9 + q % 2) for q in range(n)]

    def one(spec):
        s = ["I"] * n
        for q, c in spec.items():
            s[q] = c
        return "".join(s)
    terms = list(W.tfim_terms(n))
    terms += [(one({n - 1: "X", 0: "X"}), 0.7),            # lane bit + high bit
              (one({0: "Y", 1: "Y"}), -0.4),                # two high bits
              (one({n - 2: "Y", n - 3: "Z", 3: "Z"}), 0.25),
              (one({n - 1: "Y", n - 6: "X"}), 0.6),         # two lane bits, Y phase
              (one({2: "X", 5: "Z", n - 1: "Z"}), -0.35),
              (one({q: "Z" for q in range(0, n, 3)}), 0.15),
              (one({4: "Y"}), 0.5)]
    theta = np.random.default_rng(14).uniform(0, 2 * math.pi, 11)
    psi0 = oracle.basis_state(n, 0)
    g_ref = oracle.param_shift_grad(ops, theta, terms, psi0)
    e_ref = oracle.energy(oracle.run(ops, psi0, theta), terms)
    psi = qc.new_state(n, DT[dt])
    lam = qc.new_state(n, DT[dt])
    qc.state_init(psi, 0)
    e, g = qc.adjoint_grad(psi, lam, ops, theta, terms)
    e, g = e.item(), g.cpu().numpy()
    if dt == "c128":
        assert abs(e - e_ref) < 1e-11
        np.testing.assert_allclose(g, g_ref, atol=1e-10)
    else:
        norm_h = sum(abs(c) for _, c in terms)
        bound = 2 * norm_h * 1e-5
        assert abs(e - e_ref) < bound
        assert np.max(np.abs(g - g_ref)) < bound


def test_deterministic_reductions(qc):
    n = 16
    t = dev(W.random_state(n, 3), torch.complex64)
    terms = W.tfim_terms(n)
    a = qc.expect_pauli(t, terms, per_term=True).cpu().numpy()
    b = qc.expect_pauli(t, terms, per_term=True).cpu().numpy()
    assert np.array_equal(a, b)
    p1 = qc.probs(t, [3, 1]).cpu().numpy()
    p2 = qc.probs(t, [3, 1]).cpu().numpy()
    assert np.array_equal(p1, p2)


def test_adjoint_all_parameters_n10_16_layers(qc):
    """Every one of the 320 gradients of a 10-qubit, 16-layer HEA against
    the oracle's parameter-shift gradients (complex128)."""
    n, layers = 10, 16
    ops = W.hea(n, layers)
    terms = W.tfim_terms(n)
    theta = np.random.default_rng(24).uniform(0, 2 * math.pi, layers * n * 2)
    psi0 = oracle.basis_state(n, 0)
    g_ref = oracle.param_shift_grad(ops, theta, terms, psi0)
    psi = qc.new_state(n, torch.complex128)
    lam = qc.new_state(n, torch.complex128)
    qc.state_init(psi, 0)
    e, g = qc.adjoint_grad(psi, lam, ops, theta, terms)
    np.testing.assert_allclose(g.cpu().numpy(), g_ref, atol=1e-9)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_adjoint_config24_vs_central_differences(qc, G, dt):
    """24-qubit, 16-layer HEA (768 parameters), TFIM: the adjoint gradient
    against central differences (eps = 1e-4) of complex128 forward runs on a
    seeded sample of parameters (first and last layer, RY and RZ), and the
    complex64 gradient against the complex128 one."""
    n, ops, theta, terms = W.adjoint_config()
    psi = qc.new_state(n, torch.complex128)
    lam = qc.new_state(n, torch.complex128)
    qc.state_init(psi, 0)
    e128, g128 = qc.adjoint_grad(psi, lam, ops, theta, terms)
    g128 = g128.cpu().numpy()
    if dt == "c128":
        rng = np.random.default_rng(5)
        sample = [0, 1, 2 * n - 2, 2 * n - 1, len(theta) - 1, len(theta) - 2]
        sample += [int(x) for x in rng.choice(len(theta), 6, replace=False)]
        t = qc.new_state(n, torch.complex128)

        def energy(th):
            qc.state_init(t, 0)
            qc.apply_circuit(t, qc.GateList(G.gate_tuples(ops, th)), mode=2)
            return qc.expect_pauli(t, terms)[0].item()
        eps = 1e-4
        for p in sample:
            tp, tm = theta.copy(), theta.copy()
            tp[p] += eps
            tm[p] -= eps
            fd = (energy(tp) - energy(tm)) / (2 * eps)
            # FD truncation ~ eps^2/6 * ||H|| and rounding ~ 1e-15 * ||H|| / eps
            assert abs(fd - g128[p]) < 1e-6, (p, fd, g128[p])
        assert abs(energy(theta) - e128.item()) < 1e-10
    else:
        psi64 = qc.new_state(n, torch.complex64)
        lam64 = qc.new_state(n, torch.complex64)
        qc.state_init(psi64, 0)
        e64, g64 = qc.adjoint_grad(psi64, lam64, ops, theta, terms)
        bound = 2 * (2 * n - 1) * 1e-5
        assert abs(e64.item() - e128.item()) < bound
        assert np.max(np.abs(g64.cpu().numpy() - g128)) < bound


def test_autotune_picks_a_correct_fast_strategy(qc, G, tmp_path, monkeypatch):
    from paper_2503_03016_amd import autotune
    monkeypatch.setenv("QC_TUNE_CACHE", str(tmp_path / "tune.json"))
    n = 16
    ops = W.brickwork(n, 6, seed=16, entangler="CZ")
    gts = G.gate_tuples(ops)
    best = autotune.tune(n, torch.complex64, gts, family="brickwork16x6")
    table = best["table"]
    assert len(table) >= 6 and all(table[i]["ms"] <= table[i + 1]["ms"] for i in range(len(table) - 1))
    assert best["ms"] == table[0]["ms"]
    assert (tmp_path / "tune.json").exists()
    again = autotune.tune(n, torch.complex64, gts, family="brickwork16x6")
    assert again["ms"] == best["ms"]          # served from the cache
    psi = qc.new_state(n, torch.complex64)
    qc.state_init(psi, 0)
    knobs = [qc.QC_KNOB_MFMA_WG_PER_CU, qc.QC_KNOB_MFMA_TILE_BITS, qc.QC_KNOB_TILE_BITS]
    before = [qc.get_knob(k) for k in knobs]
    autotune.apply_tuned(psi, gts, family="brickwork16x6")
    # the tuned launch shape is used for that call only
    assert [qc.get_knob(k) for k in knobs] == before
    ref = oracle.run(ops, oracle.basis_state(n, 0))
    check(host(psi), ref, torch.complex64, ngates=len(ops))


def test_autograd_energy_function(qc):
    from paper_2503_03016_amd.autograd import AdjointCircuit, energy
    n, layers = 6, 2
    ops = W.hea(n, layers)
    terms = W.tfim_terms(n)
    th0 = np.random.default_rng(9).uniform(0, 2 * math.pi, layers * n * 2)
    circ = AdjointCircuit(n, ops, terms, dtype=torch.complex128)
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    e = energy(theta, circ)
    (3.0 * e).backward()
    g_ref = oracle.param_shift_grad(ops, th0, terms, oracle.basis_state(n, 0))
    e_ref = oracle.energy(oracle.run(ops, oracle.basis_state(n, 0), th0), terms)
    assert abs(e.item() - e_ref) < 1e-12
    np.testing.assert_allclose(theta.grad.numpy(), 3.0 * g_ref, atol=1e-11)
    # energy only (no gradient wanted): the forward runs without the
    # adjoint sweep and gives the same energy
    with torch.no_grad():
        e2 = energy(theta, circ)
    assert abs(e2.item() - e_ref) < 1e-12
    e3 = energy(torch.tensor(th0, dtype=torch.float64), circ)
    assert abs(e3.item() - e_ref) < 1e-12 and not e3.requires_grad


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_expect_pauli_many_terms_in_one_pass(qc, dt):
    """More terms than one tile-pass launch takes (512): 560 diagonal and
    60 low-X terms all fit the first pass's tile bits, so that pass is
    split over several launches."""
    n = 14
    rng = np.random.default_rng(314)
    psi0 = W.random_state(n, 23)
    t = dev(psi0, DT[dt])
    st = host(t)
    terms = [("".join(rng.choice(list("IZ"), n)), float(rng.normal())) for _ in range(560)]
    for _ in range(60):
        s = list(rng.choice(list("IZ"), n))
        s[n - 1 - int(rng.integers(0, 6))] = str(rng.choice(list("XY")))   # X/Y on one of the 6 lowest bits
        terms.append(("".join(s), float(rng.normal())))
    out = qc.expect_pauli(t, terms, per_term=True).cpu().numpy()
    ref_terms = np.array([oracle.expect_pauli(st, p).real for p, _ in terms])
    np.testing.assert_allclose(out[1:], ref_terms, atol=1e-12)
    assert abs(out[0] - sum(c * r for (_, c), r in zip(terms, ref_terms))) < 1e-10
