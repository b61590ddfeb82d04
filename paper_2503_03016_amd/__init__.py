"""Dense state-vector simulation on AMD MI355X (gfx950).

The hot path of QCLAB's circuit simulation (Keip, Camps, Van Beeumen 2025):
gate application, measurement probabilities and Pauli expectations, plus
fused 5-qubit blocks on FP32 matrix cores, a batched persistent launch and
an adjoint gradient.  All device work is in libqc.so (HIP, behind the C ABI
of include/qc.h); the Python layer only marshals arguments.

Modules: ``qc`` (the binding), ``gates`` (FP64 gate matrices),
``simulate`` (branching measurement driver), ``autograd`` (adjoint
gradient as a torch.autograd.Function), ``autotune`` (strategy tuner).
"""
from . import gates  # noqa: F401
from . import qc  # noqa: F401  (raises ImportError when libqc.so is missing)
