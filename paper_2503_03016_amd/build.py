"""Build libqc.so (HIP, gfx950 only) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqc.so")
SOURCES = ["qc_api.cpp", "qc_gates.hip", "qc_reduce.hip", "qc_fused_mfma.hip", "qc_tile.hip",
           "qc_adjoint.hip", "qc_batch.hip", "qc_measure.hip", "qc_expect_tiles.hip",
           "qc_fused_mfma_c128.hip", "qc_permute.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# The fused kernels' tile counter is taken by one lane; the atomic optimizer's
# wave-wide rewrite of it would wait on every memory operation in flight.
# The register-resident tile interpreter keeps each thread's amplitudes in
# an array indexed by compile-time element numbers only; merging the
# identical tails of its per-slot switch cases would index that array with a
# run-time value and move it to scratch memory, so common-code sinking is off.
EXTRA_FLAGS = {"qc_fused_mfma.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
               "qc_fused_mfma_c128.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
               "qc_tile.hip": ["-mllvm", "-simplifycfg-sink-common=false"],
               "qc_adjoint.hip": ["-mllvm", "-simplifycfg-sink-common=false"]}


def build(verbose: bool = False) -> str:
    objs = []
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        cmd = ([HIPCC] + FLAGS + EXTRA_FLAGS.get(src, []) +
               ["-I", os.path.join(ROOT, "include"), "-c", path, "-o", obj])
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
