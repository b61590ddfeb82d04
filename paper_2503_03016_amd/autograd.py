"""torch.autograd.Function around qc_adjoint_grad.

Energy.apply(theta, circuit) returns E(theta) = <phi|H|phi> with
phi = U(theta)|0...0>.  When theta needs a gradient, the forward is one
qc_adjoint_grad call (forward, energy and the adjoint backward sweep
together) and the backward only scales the saved dE/dtheta by the incoming
gradient.  When it does not (torch.no_grad, or theta without
requires_grad), the forward runs the circuit and the energy alone
(qc_apply_circuit + qc_expect_pauli): no adjoint sweep is spent.
"""
from __future__ import annotations

import torch

from . import gates as G
from . import qc


class AdjointCircuit:
    """A parametrised circuit (workloads.Op list of RX/RY/RZ/H/X/Y/Z/CZ/CNOT
    with parameter indices), its Hamiltonian (Pauli strings) and the two
    device state buffers the adjoint method needs."""

    def __init__(self, n, ops, terms, dtype=torch.complex128, device="cuda"):
        self.n, self.ops, self.terms = n, list(ops), list(terms)
        self.psi = qc.new_state(n, dtype, device)
        self.lam = qc.new_state(n, dtype, device)
        qc.make_ops(self.ops)   # validate kinds early


class Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, circ: AdjointCircuit):
        th = theta.detach().to("cpu", torch.float64).numpy()
        qc.state_init(circ.psi, 0)
        if ctx.needs_input_grad[0]:
            energy, grad = qc.adjoint_grad(circ.psi, circ.lam, circ.ops, th, circ.terms)
            ctx.save_for_backward(grad.to(theta.device, theta.dtype))
        else:
            qc.apply_circuit(circ.psi, qc.GateList(G.gate_tuples(circ.ops, th)),
                             mode=qc.QC_EXEC_TILED)
            energy = qc.expect_pauli(circ.psi, circ.terms)[:1]
        return energy.reshape(()).to(theta.device, theta.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return grad_out * grad, None


def energy(theta: torch.Tensor, circ: AdjointCircuit) -> torch.Tensor:
    return Energy.apply(theta, circ)
