"""Circuit simulation with mid-circuit measurements and resets, as QCLAB
describes it (section 3.3): gates are applied in order; a measurement splits
every branch with a non-zero outcome probability into collapsed,
renormalised branches; X-, Y- and custom-basis measurements apply the basis
change V before the computational-basis measurement and V^dagger after it
(X: V = H; Y: V = H S^dagger; custom: a caller-given 2 x 2 unitary V,
section 2); a reset splits a branch the same way and leaves the qubit in
|0> in both (qc_reset), the outcome being recorded like a measurement's.

Branch bookkeeping is host control flow; every operation on a state is a
C-ABI call (gate kernels, qc_collapse, qc_reset, qc_state_copy).  Branches
with probability below `drop` are discarded.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np
import torch

from . import gates as G
from . import qc

_BASIS = {"z": (), "x": ("H",), "y": ("SDG", "H")}


def _basis_change(basis):
    """V applied before a measurement in `basis` ("z", "x", "y" or a 2 x 2
    matrix), None for the computational basis."""
    if isinstance(basis, str):
        seq = _BASIS[basis]
        if not seq:
            return None
        v = np.eye(2, dtype=np.complex128)
        for g in seq:
            v = G.matrix(g) @ v
        return v
    v = np.asarray(basis, dtype=np.complex128)
    if v.shape != (2, 2):
        raise ValueError("a custom measurement basis is a 2 x 2 matrix")
    return v


def simulate(n: int, items, init, dtype=torch.complex128, drop: float = 1e-12
             ) -> List[Tuple[str, float, torch.Tensor]]:
    """items: workloads.Op gates, ("M", qubit[, basis]) measurements (basis
    "z", "x", "y" or a 2 x 2 basis-change matrix) and ("R", qubit) resets.
    init: a bitstring (first character = qubit 0), a basis index, or a
    host/device vector of 2^n amplitudes.  Returns (outcome string,
    probability, device state) per branch, outcomes in lexicographic order."""
    psi = qc.new_state(n, dtype)
    if isinstance(init, str):
        idx = 0
        for ch in init:
            idx = 2 * idx + (1 if ch == "1" else 0)
        qc.state_init(psi, idx)
    elif isinstance(init, int):
        qc.state_init(psi, init)
    else:
        v = torch.as_tensor(init).to(torch.complex128)
        src = v.to("cuda")
        qc.state_copy(psi, src.contiguous())
    branches: List[Tuple[str, float, torch.Tensor]] = [("", 1.0, psi)]
    for it in items:
        if isinstance(it, tuple) and it and it[0] in ("M", "R"):
            q = int(it[1])
            is_reset = it[0] == "R"
            v = None if is_reset else _basis_change(it[2] if len(it) > 2 else "z")
            new = []
            for res, p, st in branches:
                if v is not None:
                    qc.apply_1q(st, q, v)
                for b in (0, 1):
                    post = torch.empty_like(st)
                    qc.state_copy(post, st)
                    step = qc.reset if is_reset else qc.collapse
                    pb = float(step(post, q, b).item())
                    if pb > drop:
                        if v is not None:
                            qc.apply_1q(post, q, v.conj().T)
                        new.append((res + str(b), p * pb, post))
            branches = new
        else:
            gl = qc.GateList([G.gate_tuple(it)])
            for _, _, st in branches:
                qc.apply_circuit(st, gl)
    branches.sort(key=lambda x: x[0])
    return branches
