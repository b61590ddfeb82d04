"""Circuit simulation with mid-circuit measurements, as QCLAB describes it
(section 3.3): gates are applied in order; a measurement splits every
branch with a non-zero outcome probability into collapsed, renormalised
branches; X- and Y-basis measurements apply the basis change V before the
computational-basis measurement and V^dagger after it (X: V = H; Y: V = H S^dagger).

Branch bookkeeping is host control flow; every operation on a state is a
C-ABI call (gate kernels, qc_collapse, qc_state_copy).  Branches with
probability below `drop` are discarded.
"""
from __future__ import annotations

from typing import List, Tuple

import torch

from . import gates as G
from . import qc

_BASIS = {"z": (), "x": ("H",), "y": ("SDG", "H")}


def simulate(n: int, items, init, dtype=torch.complex128, drop: float = 1e-12
             ) -> List[Tuple[str, float, torch.Tensor]]:
    """items: workloads.Op gates and ("M", qubit[, basis]) measurements.
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
        if isinstance(it, tuple) and it and it[0] == "M":
            q = int(it[1])
            pre = _BASIS[it[2] if len(it) > 2 else "z"]
            new = []
            for res, p, st in branches:
                for g in pre:
                    qc.apply_1q(st, q, G.matrix(g))
                for b in (0, 1):
                    post = torch.empty_like(st)
                    qc.state_copy(post, st)
                    pb = float(qc.collapse(post, q, b).item())
                    if pb > drop:
                        for g in reversed(pre):
                            qc.apply_1q(post, q, G.matrix(g).conj().T)
                        new.append((res + str(b), p * pb, post))
            branches = new
        else:
            gl = qc.GateList([G.gate_tuple(it)])
            for _, _, st in branches:
                qc.apply_circuit(st, gl)
    branches.sort(key=lambda x: x[0])
    return branches
