"""Benchmark: 32-qubit brickwork circuit, depth 40 (Haar U(2) on every qubit
+ CZ on alternating neighbour pairs, seed 32), complex64 state (32 GiB),
gates fused into 5-qubit blocks applied on the FP32 matrix cores.

One step = one pass of the hot path over the workload: prepare |0...0>,
apply the 1900 gates as fused blocks, and take the measurement
probabilities of qubit 0.  The reference is the plain unfused complex128
run of the same circuit on the same GPU (one kernel sweep per gate); the
bench reports the speedup over it and the error of the complex64 state
against it.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--n 32] [--layers 40]
                    [--no-ref] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
PROFILES = os.path.join(ROOT, "profiles")


def log(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    p = os.path.join(ROOT, "paper_2503_03016_amd", "csrc", "qc_fused_mfma.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def load_traffic(n: int):
    """HBM bytes per launch of the fused kernel from committed rocprofv3 PMC
    counters, if they were taken on the current kernel source and size."""
    path = os.path.join(PROFILES, "fused_mfma_c64_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha") != kernel_source_hash() or d.get("n_qubits") != n:
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(n_cpu: int, layers: int, budget_s: float):
    """The FP64 oracle on the host on a bounded sample of the same circuit
    family: the first gates of the brickwork circuit at n_cpu qubits, run
    until about budget_s seconds have passed."""
    import oracle
    import workloads as W

    ops = W.brickwork(n_cpu, layers, seed=32, entangler="CZ")
    psi = oracle.basis_state(n_cpu, 0)
    sweep = 2.0 * (1 << n_cpu) * 16.0
    done = 0
    t0 = time.perf_counter()
    for op in ops:
        psi = oracle.run([op], psi)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {
        "value": round(done * sweep / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": "FP64 oracle, brickwork %d qubits (Haar U(2) + CZ, seed 32), first %d of %d "
                  "gates, complex128, one state pass per gate; %.1f s wall, %.2f gates/s"
                  % (n_cpu, done, len(ops), dt, done / dt),
        "gates_per_s": round(done / dt, 4),
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--no-ref", action="store_true", help="skip the unfused complex128 run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=24)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: the state-vector path here is single-GPU "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    import workloads as W
    from paper_2503_03016_amd import gates as G
    from paper_2503_03016_amd import qc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, layers = args.n, args.layers
    _, ops = W.config_brickwork32(n, layers)
    gl = qc.GateList(G.gate_tuples(ops))
    _, nblocks = qc.fuse_plan(n, gl, 5)
    log("workload: %d qubits, %d gates, %d fused blocks" % (n, len(ops), nblocks))

    psi = torch.empty(1 << n, dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        qc.state_init(psi, 0)
        st = qc.apply_circuit(psi, gl, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        p0 = qc.probs(psi, [0])
        return st, p0

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % i)

    qc.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    st = None
    for i in range(args.steps):
        st, p0 = step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    cnt, kms = qc.timing_query("fused_mfma_c64")
    qc.timing_enable(False)
    ms_per_step = max(gpu_ms, wall * 1e3) / args.steps
    log("timed %d steps: %.1f ms/step (events %.1f ms, wall %.1f ms)"
        % (args.steps, ms_per_step, gpu_ms / args.steps, wall * 1e3 / args.steps))

    S = float(1 << n) * 8.0
    step_bytes = S + st["state_bytes"] + S        # init write + sweeps + probs read
    value = step_bytes / (ms_per_step / 1e3) / 1e9
    gates_per_s = len(ops) / (ms_per_step / 1e3)
    avg_launch_ms = kms / cnt if cnt else float("nan")
    per_launch_bytes = 2.0 * S
    achieved = per_launch_bytes / (avg_launch_ms / 1e3) / 1e9 if cnt else None
    traffic = load_traffic(n)
    p0h = p0.cpu().tolist()

    ref = {}
    if not args.no_ref:
        ref_psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        qc.state_init(ref_psi, 0)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st128 = qc.apply_circuit(ref_psi, gl, mode=qc.QC_EXEC_UNFUSED)
        e1.record(stream)
        torch.cuda.synchronize()
        t128 = e0.elapsed_time(e1) / 1e3
        # error of the fused complex64 state against the unfused complex128 state
        qc.state_init(psi, 0)
        qc.apply_circuit(psi, gl, mode=qc.QC_EXEC_FUSED, fuse_k=5)
        d = qc.state_diff(psi, ref_psi).cpu().tolist()
        t_fused = ms_per_step / 1e3
        ref = {
            "c128_unfused_s": round(t128, 4),
            "c128_unfused_sweeps": st128["sweeps"],
            "c128_unfused_GBps": round(st128["state_bytes"] / t128 / 1e9, 1),
            "speedup_fused_c64_vs_unfused_c128": round(t128 / t_fused, 2),
            "err_rel_vs_c128": float("%.3e" % math.sqrt(d[0] / d[1])),
            "err_maxabs_vs_c128": float("%.3e" % d[2]),
        }
        log("c128 unfused: %.2f s, speedup %.2fx, rel err %.2e"
            % (t128, t128 / t_fused, math.sqrt(d[0] / d[1])))
        del ref_psi
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.cpu_n, layers, args.cpu_budget)
        log("cpu oracle: %s" % cpu["sample"])

    out = {
        "metric": "state-vector GB/s & gates/sec at 32 qubits; fused c64 vs plain c128 speedup",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "brickwork random circuit, %d qubits, depth %d (Haar U(2) + CZ), "
                        "complex64, fused 5-qubit blocks on FP32 MFMA" % (n, layers),
            "n_qubits": n, "layers": layers, "gates": len(ops), "fused_blocks": nblocks,
            "sweeps_per_step": int(st["sweeps"]) + 2, "seed": 32,
        },
        "gates_per_s": round(gates_per_s, 1),
        "prob_q0": [round(x, 9) for x in p0h],
        "roofline": {
            "bound": "hbm",
            "kernel": "k_fused_mfma_c64",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "traffic": traffic,
            "launches": cnt,
            "avg_launch_ms": round(avg_launch_ms, 4),
            "algorithmic_bytes_per_launch": per_launch_bytes,
        },
        "cpu_baseline": cpu,
    }
    out.update(ref)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
