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
                    [--no-ref] [--no-split] [--no-cpu] [--no-secondary]
                    [--only brickwork12|qft28|tfim28|batch512|adjoint24]

Every reported figure comes with its check: the headline state against the
unfused complex128 run (relative error <= 1e-5), the batch energies against
the oracle's stored values, the batch status flags, the QFT modes against
the unfused complex128 run; if a check fails, "value" is null and the exit
status is 1.
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


GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    """Stored FP64 oracle values (written by tests/golden/make_golden.py,
    which calls only the oracle); None when the file is absent."""
    path = os.path.join(GOLDEN, name)
    return json.load(open(path)) if os.path.exists(path) else None


def _diff(qc, a, ref):
    """relative 2-norm and max-abs error of state a against ref (FP64)."""
    d = qc.state_diff(a, ref).cpu().tolist()
    return {"rel": float("%.3e" % math.sqrt(d[0] / d[1])), "maxabs": float("%.3e" % d[2])}


def wl_brickwork12() -> dict:
    """12-qubit brickwork, 20 layers, complex128: unfused, one LDS tile run,
    and one workgroup of the batch kernel; states against the unfused run."""
    import torch
    import workloads as W
    from paper_2503_03016_amd import gates as G
    from paper_2503_03016_amd import qc

    n, ops = W.config_brickwork12()
    gts = G.gate_tuples(ops)
    gl = qc.GateList(gts)
    ref = qc.new_state(n, torch.complex128)
    qc.state_init(ref, 0)
    qc.apply_circuit(ref, gl, mode=qc.QC_EXEC_UNFUSED)
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
                   "gates_per_s": round(len(ops) / (ms / 1e3), 1),
                   "err_vs_unfused_c128": _diff(qc, psi, ref)}
    b = qc.Batch([(n, gts, W.tfim_terms(n))], dtype=torch.complex128, keep_states=True)
    ms = _time(lambda: b.run(), reps=5)
    r["one_workgroup_batch"] = {"us": round(ms * 1e3, 1),
                                "gates_per_s": round(len(ops) / (ms / 1e3), 1),
                                "err_vs_unfused_c128": _diff(qc, b.state(0), ref)}
    return r


def wl_qft28() -> dict:
    """28-qubit QFT of the seeded Gaussian state (seed 28), complex128 and
    complex64, every execution mode; states against the unfused complex128
    run, whose sampled amplitudes are checked against the oracle's stored
    discrete Fourier sums."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2503_03016_amd import gates as G
    from paper_2503_03016_amd import qc

    n, ops, psi0 = W.config_qft28()
    gl = qc.GateList(G.gate_tuples(ops))
    host = torch.from_numpy(psi0)
    ref = host.cuda()
    del psi0
    r = {}
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    st = qc.apply_circuit(ref, gl, mode=qc.QC_EXEC_UNFUSED)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    r["c128_unfused"] = {"ms": round(ms, 2), "sweeps": st["sweeps"],
                         "GBps": round(st["state_bytes"] / (ms / 1e3) / 1e9, 1),
                         "gates_per_s": round(len(ops) / (ms / 1e3), 1)}
    gold = _golden("qft28_amplitudes.json")
    if gold:
        idx = torch.tensor(gold["indices"], dtype=torch.int64, device="cuda")
        want = np.array([complex(a, b) for a, b in gold["amplitudes"]])
        got = ref[idx].cpu().numpy()
        r["c128_unfused"]["err_vs_oracle_sampled_maxabs"] = float(
            "%.3e" % np.max(np.abs(got - want)))
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        src = host.to(dt).cuda()
        psi = torch.empty_like(src)
        for name, mode in (("tiled", qc.QC_EXEC_TILED), ("fused", qc.QC_EXEC_FUSED)):
            st = {}

            def run():
                st.update(qc.apply_circuit(psi, gl, mode=mode, fuse_k=5))
            qc.state_copy(psi, src)
            run()                            # warm-up (and the checked run)
            err = _diff(qc, psi, ref)
            # median of five back-to-back runs, each the same transform of a
            # unit vector (the state keeps evolving; the work does not change)
            ms = _time(run, reps=5, warm=1)
            r["%s_%s" % (dname, name)] = {
                "ms": round(ms, 2), "sweeps": st["sweeps"],
                "GBps": round(st["state_bytes"] / (ms / 1e3) / 1e9, 1),
                "gates_per_s": round(len(ops) / (ms / 1e3), 1),
                "err_vs_unfused_c128": err}
        if dname == "c64":
            qc.state_copy(psi, src)
            st = qc.apply_circuit(psi, gl, mode=qc.QC_EXEC_UNFUSED)
            err = _diff(qc, psi, ref)
            qc.state_copy(psi, src)
            ms = _time(lambda: qc.apply_circuit(psi, gl, mode=qc.QC_EXEC_UNFUSED), reps=1, warm=0)
            r["c64_unfused"] = {"ms": round(ms, 2), "sweeps": st["sweeps"],
                                "GBps": round(st["state_bytes"] / (ms / 1e3) / 1e9, 1),
                                "gates_per_s": round(len(ops) / (ms / 1e3), 1),
                                "err_vs_unfused_c128": err}
        del src, psi
        torch.cuda.empty_cache()
    return r


def wl_tfim28() -> dict:
    """<H> of the 28-qubit open-chain transverse-field Ising model (55 Pauli
    terms) on the seeded Gaussian state, complex128 and complex64; per-term
    values of the complex64 run against the complex128 run."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2503_03016_amd import qc

    n = 28
    terms = W.tfim_terms(n)
    host = torch.from_numpy(W.random_state(n, seed=28))
    r = {}
    vals = {}
    S = float(1 << n)
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        psi = host.to(dt).cuda()
        v = qc.expect_pauli(psi, terms, per_term=True)
        vals[dname] = v.cpu().numpy()
        ms = _time(lambda: qc.expect_pauli(psi, terms), reps=5)
        elem = 16 if dt == torch.complex128 else 8
        r[dname] = {"ms": round(ms, 3), "terms": len(terms),
                    "state_reads_GB": round(S * elem / 1e9, 3),
                    "energy": float(vals[dname][0])}
        del psi
        torch.cuda.empty_cache()
    r["c64"]["err_vs_c128_energy"] = float("%.3e" % abs(vals["c64"][0] - vals["c128"][0]))
    r["c64"]["err_vs_c128_max_term"] = float(
        "%.3e" % np.max(np.abs(vals["c64"][1:] - vals["c128"][1:])))
    return r


def wl_batch512() -> dict:
    """512 circuits (n uniform in [10, 20], 8-layer ansatz, TFIM energy) in
    one persistent launch, complex64, eager and as a replayed HIP graph;
    every energy against the oracle's stored energies."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2503_03016_amd import gates as G
    from paper_2503_03016_amd import qc

    cfg = W.batch_config()
    t0 = time.perf_counter()
    circuits = [(cn, G.gate_tuples(W.hea(cn, 8), th), W.tfim_terms(cn)) for cn, th in cfg]
    b = qc.Batch(circuits, dtype=torch.complex64)
    create_s = time.perf_counter() - t0
    energy = torch.empty(len(cfg), dtype=torch.float64, device="cuda")
    ms = _time(lambda: b.run(energy), reps=5)
    status = b.status()
    e = energy.cpu().numpy()
    gates = sum(8 * (3 * cn - 1) for cn, _ in cfg)
    r = {"ms": round(ms, 3), "circuits_per_s": round(512 / (ms / 1e3), 1),
         "gates_per_s": round(gates / (ms / 1e3), 1), "gates": gates,
         "grid": b.grid, "phases": b.phases, "status_flags": status,
         "host_plan_and_upload_s": round(create_s, 2)}
    # the same launch captured in a HIP graph and replayed
    out = torch.empty_like(energy)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(out)
    r["graph_replay_ms"] = round(_time(lambda: g.replay(), reps=5), 3)
    r["graph_replay_bitwise_equal"] = bool(torch.equal(out, energy))
    gold = _golden("batch512_energies.json")
    if gold:
        ref = np.array(gold["energies"])
        ns = np.array([cn for cn, _ in cfg])
        err = np.abs(e - ref)
        r["err_vs_oracle_max_abs_dE"] = float("%.3e" % err.max())
        r["err_within_bound"] = bool(np.all(err < 2 * (2 * ns - 1) * 1e-5))
    del g, b
    return r


def wl_adjoint24() -> dict:
    """Adjoint gradient of the 24-qubit 16-layer ansatz (768 parameters),
    complex128 and complex64: energy and six gradients against the oracle's
    stored values, the complex64 gradient against the complex128 one."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2503_03016_amd import qc

    n, ops, theta, terms = W.adjoint_config()
    r = {}
    grads = {}
    gold = _golden("adjoint24.json")
    for dname, dt in (("c128", torch.complex128), ("c64", torch.complex64)):
        psi = qc.new_state(n, dt)
        lam = qc.new_state(n, dt)
        res = {}

        def run():
            qc.state_init(psi, 0)
            res["eg"] = qc.adjoint_grad(psi, lam, ops, theta, terms)
        ms = _time(run, reps=3)
        e, g = res["eg"]
        grads[dname] = g.cpu().numpy()
        r[dname] = {"ms": round(ms, 2), "ops": len(ops), "params": int(len(theta)),
                    "energy": float(e.item())}
        if gold:
            r[dname]["err_vs_oracle_energy"] = float("%.3e" % abs(e.item() - gold["energy"]))
            r[dname]["err_vs_oracle_param_shift_max"] = float(
                "%.3e" % np.max(np.abs(grads[dname][gold["params"]] - np.array(gold["grad"]))))
        del psi, lam
        torch.cuda.empty_cache()
    r["c64"]["err_vs_c128_max_abs_dg"] = float(
        "%.3e" % np.max(np.abs(grads["c64"] - grads["c128"])))
    return r


WORKLOADS = {"brickwork12": wl_brickwork12, "qft28": wl_qft28, "tfim28": wl_tfim28,
             "batch512": wl_batch512, "adjoint24": wl_adjoint24}


def secondary_workloads() -> dict:
    """The other synthetic configurations, timed on the GPU, each with its
    error against the oracle or against the unfused complex128 run."""
    res = {}
    for name, fn in WORKLOADS.items():
        res[name] = fn()
        log("secondary: %s done" % name)
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
                    help="skip the other workloads")
    ap.add_argument("--only", choices=sorted(WORKLOADS),
                    help="run just this one secondary workload and print its JSON line "
                         "(for profiling one kernel family)")
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
    if args.only:
        log("workload %s only" % args.only)
        res = WORKLOADS[args.only]()
        print(json.dumps({"workload": args.only, "result": res}), flush=True)
        return 0
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
    # correctness gates: a number is reported only for a correct result
    checks = {}
    if "err_rel_vs_c128" in ref:
        checks["headline_rel_err_le_1e-5"] = ref["err_rel_vs_c128"] <= 1e-5
    checks["headline_prob_sums_to_1"] = abs(sum(p0h) - 1.0) < 1e-5
    if secondary:
        b5 = secondary.get("batch512", {})
        checks["batch512_status_ok"] = b5.get("status_flags") == 0
        if "err_within_bound" in b5:
            checks["batch512_energies_vs_oracle"] = b5["err_within_bound"]
        checks["batch512_graph_replay_equal"] = b5.get("graph_replay_bitwise_equal", False)
        q = secondary.get("qft28", {})
        for k, v in q.items():
            e = v.get("err_vs_unfused_c128")
            if e:
                checks["qft28_%s" % k] = (e["maxabs"] <= 1e-12 if k.startswith("c128")
                                          else e["rel"] <= 1e-5)
        a = secondary.get("adjoint24", {})
        if "c128" in a and "err_vs_oracle_param_shift_max" in a["c128"]:
            checks["adjoint24_c128_vs_oracle"] = a["c128"]["err_vs_oracle_param_shift_max"] <= 1e-9
    out["checks"] = checks
    ok = all(checks.values())
    if not ok:
        out["value"] = None
        log("CHECK FAILED: %s" % [k for k, v in checks.items() if not v])
    print(json.dumps(out), flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
