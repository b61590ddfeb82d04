"""Benchmark: 32-qubit brickwork circuit, depth 40 (Haar U(2) on every qubit
+ CZ on alternating neighbour pairs, seed 32), complex64 state (32 GiB),
gates fused into 5-qubit blocks applied on the FP32 matrix cores.

One step = one pass of the hot path over the workload: prepare |0...0>,
apply the 1900 gates as fused blocks, and take the measurement
probabilities of qubit 0.  The reference is the plain unfused complex128
run of the same circuit on the same GPU (one kernel sweep per gate); the
bench reports the speedup over it and the error of the complex64 state
against it, and (unless --no-split) the unfused complex64 and fused
complex128 runs that separate the precision gain from the fusion gain.
Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--n 32] [--layers 40]
                    [--no-ref] [--no-split] [--no-cpu]
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
    path = os.path.join(PROFILES, "fused_mfma_c64_brickwork32_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha") != kernel_source_hash() or d.get("n_qubits") != n:
        return None
    return d.get("hbm_bytes_per_launch")


def load_mfma(n: int):
    """Matrix-core utilisation of the fused kernel from committed rocprofv3
    PMC counters, if they were taken on the current kernel source and size."""
    path = os.path.join(PROFILES, "fused_mfma_c64_brickwork32_mfma.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha") != kernel_source_hash() or d.get("n_qubits") != n:
        return None
    return {"busy_pct": d.get("mfma_busy_pct"), "fp32_tflops": d.get("fp32_matrix_tflops"),
            "frac_of_fp32_peak": round(d.get("fp32_matrix_tflops") / 157.3, 4)}


def cpu_baseline(n_cpu: int, layers: int, budget_s: float):
    """The FP64 oracle on the host on a bounded sample of the same circuit
    family: the first gates of the brickwork circuit at n_cpu qubits, run
    until about budget_s seconds have passed."""
    import oracle
    import workloads as W

    ops = W.brickwork(n_cpu, layers, seed=32, entangler="CZ")
    sweep = 2.0 * (1 << n_cpu) * 16.0

    def run(limit_s):
        psi = oracle.basis_state(n_cpu, 0)
        done = 0
        t0 = time.perf_counter()
        for op in ops:
            psi = oracle.run([op], psi)
            done += 1
            if time.perf_counter() - t0 > limit_s:
                break
        return done, time.perf_counter() - t0

    cores = oracle.threads()
    done, dt = run(budget_s)
    # the same sample on one thread (a third of the budget)
    oracle.set_threads(1)
    try:
        done1, dt1 = run(budget_s / 3.0)
    finally:
        oracle.set_threads(cores)
    return {
        "value": round(done * sweep / dt / 1e9, 3),
        "unit": "GB/s",
        "cores": cores,
        "kind": "oracle",
        "sample": "FP64 oracle, brickwork %d qubits (Haar U(2) + CZ, seed 32), first %d of %d "
                  "gates, complex128, one state pass per gate; %.1f s wall, %.2f gates/s"
                  % (n_cpu, done, len(ops), dt, done / dt),
        "gates_per_s": round(done / dt, 4),
        "one_thread": {"value": round(done1 * sweep / dt1 / 1e9, 3), "unit": "GB/s",
                       "gates_per_s": round(done1 / dt1, 4), "gates": done1,
                       "seconds": round(dt1, 2)},
    }


def _time(fn, reps: int = 3, warm: int = 1) -> float:
    """Median milliseconds of fn() over reps runs (HIP events, current stream)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    out.sort()
    return out[len(out) // 2]


def secondary_workloads() -> dict:
    """The other four synthetic configurations, timed on the GPU (state
    contents do not change the work, so QFT starts from |0...0>)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2503_03016_amd import gates as G
    from paper_2503_03016_amd import qc

    res = {}
    # 12-qubit brickwork, 20 layers, complex128: whole circuit in one LDS tile
    n, ops = W.config_brickwork12()
    gl = qc.GateList(G.gate_tuples(ops))
    psi = qc.new_state(n, torch.complex128)
    r = {}
    for name, mode in (("unfused", qc.QC_EXEC_UNFUSED), ("tiled", qc.QC_EXEC_TILED)):
        st = {}

        def run():
            qc.state_init(psi, 0)
            st.update(qc.apply_circuit(psi, gl, mode=mode))
            qc.probs(psi)
        ms = _time(run, reps=5)
        r[name] = {"us": round(ms * 1e3, 1), "sweeps": st["sweeps"],
                   "gates_per_s": round(len(ops) / (ms / 1e3), 1)}
    b = qc.Batch([(n, G.gate_tuples(ops), W.tfim_terms(n))], dtype=torch.complex128)
    ms = _time(lambda: b.run(), reps=5)
    r["one_workgroup_batch"] = {"us": round(ms * 1e3, 1),
                                "gates_per_s": round(len(ops) / (ms / 1e3), 1)}
    res["brickwork12_c128"] = r
    del psi, b
    log("secondary: brickwork12 done")

    # 28-qubit QFT, complex128 and complex64
    n = 28
    ops = W.qft(n)
    gl = qc.GateList(G.gate_tuples(ops))
    r = {}
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        psi = qc.new_state(n, dt)
        for name, mode in (("unfused", qc.QC_EXEC_UNFUSED), ("tiled", qc.QC_EXEC_TILED),
                           ("fused", qc.QC_EXEC_FUSED)):
            st = {}

            def run():
                st.update(qc.apply_circuit(psi, gl, mode=mode, fuse_k=5))
            qc.state_init(psi, 0)
            ms = _time(run, reps=1)
            r["%s_%s" % (dname, name)] = {
                "ms": round(ms, 2), "sweeps": st["sweeps"],
                "GBps": round(st["state_bytes"] / (ms / 1e3) / 1e9, 1),
                "gates_per_s": round(len(ops) / (ms / 1e3), 1)}
        del psi
        torch.cuda.empty_cache()
    res["qft28"] = r
    log("secondary: qft28 done")

    # batch of 512 circuits, one persistent launch, complex64
    cfg = W.batch_config()
    t0 = time.perf_counter()
    circuits = [(cn, G.gate_tuples(W.hea(cn, 8), th), W.tfim_terms(cn)) for cn, th in cfg]
    b = qc.Batch(circuits, dtype=torch.complex64)
    create_s = time.perf_counter() - t0
    ms = _time(lambda: b.run(), reps=3)
    gates = sum(8 * (3 * cn - 1) for cn, _ in cfg)
    res["batch512_c64"] = {"ms": round(ms, 3), "circuits_per_s": round(512 / (ms / 1e3), 1),
                           "gates_per_s": round(gates / (ms / 1e3), 1), "gates": gates,
                           "grid": b.grid, "phases": b.phases,
                           "host_plan_and_upload_s": round(create_s, 2)}
    del b
    log("secondary: batch512 done")

    # adjoint gradient, 24 qubits, 16 layers, 768 parameters
    n, ops, theta, terms = W.adjoint_config()
    r = {}
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        psi = qc.new_state(n, dt)
        lam = qc.new_state(n, dt)

        def run():
            qc.state_init(psi, 0)
            qc.adjoint_grad(psi, lam, ops, theta, terms)
        ms = _time(run, reps=3)
        r[dname] = {"ms": round(ms, 2), "ops": len(ops), "params": int(len(theta))}
        del psi, lam
    res["adjoint24"] = r
    log("secondary: adjoint24 done")
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--no-ref", action="store_true", help="skip the unfused complex128 run")
    ap.add_argument("--c128-fused-only", action="store_true",
                    help="run only the circuit fused on a complex128 state (--steps runs), "
                         "each followed by one state copy; for profiling that kernel")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the unfused complex64 and fused complex128 runs that separate the "
                         "precision gain from the fusion gain")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=24)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-copy", action="store_true",
                    help="skip the plain-copy calibration run (bandwidth ceiling)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the other four workloads")
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
    t0 = time.perf_counter()
    _, nblocks = qc.fuse_plan(n, gl, 5)
    plan_ms = (time.perf_counter() - t0) * 1e3
    log("workload: %d qubits, %d gates, %d fused blocks (plan %.1f ms)"
        % (n, len(ops), nblocks, plan_ms))

    if args.c128_fused_only:
        # the same circuit fused on a complex128 state, --steps times, each
        # run followed by one plain copy of the state (the scale of HBM byte
        # counters); for profiling the complex128 matrix-core kernel alone
        psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
        dst = torch.empty_like(psi)
        times = []
        for _ in range(max(1, args.steps)):
            qc.state_init(psi, 0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = qc.apply_circuit(psi, gl, mode=qc.QC_EXEC_FUSED, fuse_k=5)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            qc.state_copy(dst, psi)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "brickwork %d qubits, depth %d, complex128, fused 5-qubit blocks"
                          % (n, layers), "runs": len(times), "sweeps": st["sweeps"],
                          "s_per_run": [round(t, 4) for t in times]}), flush=True)
        return 0

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

    copy = None
    if not args.no_copy:
        # plain device copy of the same state: the achievable-bandwidth
        # reference for the fused sweeps (and the scale of HBM byte counters)
        dst = torch.empty_like(psi)
        qc.state_copy(dst, psi)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(3):
            qc.state_copy(dst, psi)
        c1.record(stream)
        torch.cuda.synchronize()
        cms = c0.elapsed_time(c1) / 3
        copy = {"ms": round(cms, 4), "GBps": round(2 * S / (cms / 1e3) / 1e9, 1)}
        log("copy ceiling: %.3f ms, %.1f GB/s" % (cms, copy["GBps"]))
        del dst
        torch.cuda.empty_cache()

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
        if not args.no_split:
            # separate the precision gain from the fusion gain: unfused
            # complex64 and fused complex128 on the same circuit
            def timed(state, mode):
                qc.state_init(state, 0)
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                stx = qc.apply_circuit(state, gl, mode=mode, fuse_k=5)
                b.record(stream)
                torch.cuda.synchronize()
                return a.elapsed_time(b) / 1e3, stx
            t64u, st64u = timed(psi, qc.QC_EXEC_UNFUSED)
            d64u = qc.state_diff(psi, ref_psi).cpu().tolist()
            f128 = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
            t128f, st128f = timed(f128, qc.QC_EXEC_FUSED)
            d128f = qc.state_diff(f128, ref_psi).cpu().tolist()
            del f128
            ref.update({
                "c64_unfused_s": round(t64u, 4),
                "c64_unfused_GBps": round(st64u["state_bytes"] / t64u / 1e9, 1),
                "err_rel_c64_unfused_vs_c128": float("%.3e" % math.sqrt(d64u[0] / d64u[1])),
                "c128_fused_s": round(t128f, 4),
                "c128_fused_sweeps": st128f["sweeps"],
                "c128_fused_GBps": round(st128f["state_bytes"] / t128f / 1e9, 1),
                "err_rel_c128_fused_vs_c128": float("%.3e" % math.sqrt(d128f[0] / d128f[1])),
                "speedup_precision_unfused": round(t128 / t64u, 2),
                "speedup_fusion_c128": round(t128 / t128f, 2),
                "speedup_fusion_c64": round(t64u / t_fused, 2),
            })
            log("c64 unfused: %.2f s; c128 fused: %.2f s (%d sweeps)"
                % (t64u, t128f, st128f["sweeps"]))
        del ref_psi
        torch.cuda.empty_cache()

    secondary = None
    if not args.no_secondary:
        del psi
        torch.cuda.empty_cache()
        secondary = secondary_workloads()

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
        "host_fusion_plan_ms": round(plan_ms, 2),
        "prob_q0": [round(x, 9) for x in p0h],
        "copy_ceiling": copy,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_fused_mfma_c64",
            "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
            "frac_of_copy_ceiling": (round(achieved / copy["GBps"], 4)
                                     if (achieved and copy) else None),
            "traffic": traffic,
            "mfma": load_mfma(n),
            "launches": cnt,
            "avg_launch_ms": round(avg_launch_ms, 4),
            "algorithmic_bytes_per_launch": per_launch_bytes,
        },
        "cpu_baseline": cpu,
    }
    out.update(ref)
    out["secondary_workloads"] = secondary
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
