#!/usr/bin/env python3
"""Throughput benchmark of the state-vector hot path at 30 qubits on one GPU.

One step runs the whole hot path once over the 30-qubit workload:
  reset to a seeded basis state |x>, QFT (465 gates: H and controlled-phase),
  reset to |0...0>, 20 random layers (600 Haar SU(2) + 290 CNOT),
  the FP64 norm, and the probabilities of the first 2^20 amplitudes.
The state lives in HBM the whole time (complex128: 16 GiB; complex64: 8 GiB).
Circuits run with SV_FUSE | SV_JIT: tile passes, each compiled for its own
program (compiled during the warm-up steps and kept; passes with diagonal ops
use the generic tile kernel), planned on the host inside every timed step.
`value` is gates per second over the timed steps in complex128 (the paper's
precision); the complex64 run of the same steps is reported beside it, and the
complex128 steps with the generic tile kernel alone in `generic_kernel_c128`.
Beside the steps (untimed for `value`): a Haar 2x2 gate alone on six targets
(per-gate passes against the HBM peak), a batch of 512 circuits (p50/p99
latency), serving samples at the offered rates of --serving-rates, and the
oracle on the host cores as the CPU baseline.

Printed: ONE JSON line on stdout. Diagnostics go to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# MI355X vector peaks (256 CUs at 2.4 GHz): FP64 128 flop/clock/CU. The
# published FP32 figure (157.3 TFLOP/s, 256 flop/clock/CU) counts packed FP32
# FMA; this library is built without packed FP32, so its FP32 vector rate is
# the FP64 one, and that is the roof of the complex64 vector kernels.
ALU_PEAK_TFLOPS = {"c128": 78.6, "c64": 78.6}
# Dense MFMA peaks (FP64 and FP32 matrix instructions): the compute roof of the
# dense-block kernel.
MFMA_PEAK_TFLOPS = {"c128": 78.6, "c64": 157.3}
WORKLOAD_N = 30
PROBS_COUNT = 1 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=WORKLOAD_N)
    ap.add_argument("--mode", choices=["fused", "fused-generic", "pergate", "dense", "sweep", "xl",
                                       "cpu_sweep", "graph"],
                    default="fused",
                    help="fused: SV_FUSE | SV_JIT tile passes (each pass compiled for its own "
                         "program; passes with diagonal ops keep the generic kernel); "
                         "fused-generic: SV_FUSE with the generic tile kernel only; "
                         "pergate: one launch per gate; "
                         "dense: SV_FUSE_DENSE 5-qubit blocks on the matrix cores; "
                         "sweep: per-gate timings on every qubit at 30 qubits; "
                         "xl: the 33-qubit complex128 / 34-qubit complex64 depth-10 circuit; "
                         "cpu_sweep: the oracle's per-gate cost on the host (no GPU); "
                         "graph: host cost of short circuits with and without SV_GRAPH")
    ap.add_argument("--reps", type=int, default=20, help="timed repetitions per gate (sweep)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="CPU time budget of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c64", action="store_true")
    ap.add_argument("--no-generic", action="store_true",
                    help="skip the c128 steps with the generic tile kernel (mode fused)")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the error statement (complex64 against complex128 and the oracle)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-pergate", action="store_true",
                    help="skip the per-gate 1q pass timings on six targets")
    ap.add_argument("--batched-circuits", type=int, default=512)
    ap.add_argument("--serving-arrivals", type=int, default=64,
                    help="arrivals of each serving sample (0: no serving sample)")
    ap.add_argument("--serving-rates", default="100,1000",
                    help="offered request rates (per second) of the serving samples")
    ap.add_argument("--serving-seconds", type=float, default=0.0,
                    help="if > 0, each serving sample has rate x this many arrivals (at "
                         "least 16, at most --serving-arrivals)")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a plain copy kernel of "
                         "known size, for scaling memory-traffic counters)")
    return ap.parse_args()


def workload(n):
    import qcircuits as qc
    x = qc.random_basis_index(n, 2024)
    return x, qc.qft_circuit(n), qc.layer_circuit(n, 20, 1)


def method_flops(gates, n):
    """Floating-point operations the method itself needs for a gate list on
    2^n amplitudes, gate by gate (the algorithmic work of the stride update,
    not what a fused kernel happens to execute): a dense 2x2 gate 14 per
    amplitude (28 per pair), a controlled dense 2x2 7 (half the pairs), a
    diagonal one-qubit phase 3, a controlled phase 1.5 (a quarter of the
    amplitudes, 6 each), X and CNOT 0 (pure exchanges)."""
    N = float(2 ** n)
    x = np.array([0, 0, 1, 0, 1, 0, 0, 0], dtype=np.float64)
    total = 0.0
    for g in gates:
        kind, m = int(g["kind"]), np.asarray(g["m"], dtype=np.float64)
        if kind == 2:
            total += 1.5 * N
        elif np.array_equal(m, x):
            continue
        elif kind == 0 and m[2] == m[3] == m[4] == m[5] == 0.0:
            total += 3.0 * N
        elif kind == 0:
            total += 14.0 * N
        elif kind == 1:
            total += 7.0 * N
        else:   # several controls: the pairs where all k are set, 2^-k of them
            mask = (int(g["control"]) & 0xFFFFFFFF) | ((int(g["flags"]) & 0xFFFFFFFF) << 32)
            total += 14.0 * N / 2 ** bin(mask).count("1")
    return total


def run_dtype(sv, torch, dtype, n, steps, warmup, flags):
    """Times `steps` steps; returns a result dict with per-class event timings."""
    x, qft, layers = workload(n)
    gates_per_step = len(qft) + len(layers)
    flops_per_step = method_flops(qft, n) + method_flops(layers, n)
    st = sv.StateVector(n, dtype)
    probs = torch.empty(PROBS_COUNT, dtype=torch.float64, device="cuda")
    norm_out = torch.empty(1, dtype=torch.float64, device="cuda")
    h = st.handle

    def step():
        sv.sv_reset(h, x)
        sv.sv_run_circuit(h, qft, flags)
        sv.sv_reset(h, 0)
        sv.sv_run_circuit(h, layers, flags)
        sv.sv_norm_device(h, norm_out.data_ptr())
        sv.sv_probs_device(h, 0, min(PROBS_COUNT, 1 << n), probs.data_ptr())

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    sv.sv_profile(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sv.sv_profile(h, False)
    prof = sv.sv_profile_read(h)
    norm = float(norm_out.item())
    st.close()
    del probs, norm_out
    torch.cuda.empty_cache()
    elapsed = t1 - t0
    alg_bytes = sum(v["bytes"] for v in prof.values())
    return {
        "elapsed_s": elapsed,
        "ms_per_step": 1e3 * elapsed / steps,
        "gates_per_s": gates_per_step * steps / elapsed,
        "gates_per_step": gates_per_step,
        "method_flops_per_step": flops_per_step,
        "steps": steps,
        "norm": norm,
        "profile": prof,
        "effective_hbm_frac": alg_bytes / elapsed / (HBM_PEAK_GBS * 1e9),
    }


ROOT = os.path.dirname(os.path.abspath(__file__))
GOLDEN_30Q = os.path.join(ROOT, "tests", "golden", "layers30_qft30.npz")


def precision_errors(sv, torch, n, flags):
    """The error statement of each result of the step (outside the timed
    region): for both circuits, the complex64 state against the complex128
    state of the same circuit, compared on the device in FP64 (sv_compare:
    max-abs amplitude error, relative 2-norm error, norm drift); and at 30
    qubits both states against the oracle's complex128 amplitudes at the
    sampled indices of the committed fixture."""
    x, qft, layers = workload(n)
    gold = None
    if n == 30 and os.path.exists(GOLDEN_30Q):
        with np.load(GOLDEN_30Q) as z:
            gold = {k: z[k] for k in z.files}
    out = {}
    for name, g, x0 in (("qft", qft, x), ("layers", layers, 0)):
        a = sv.StateVector(n, sv.SV_C64, basis_index=x0)
        b = sv.StateVector(n, sv.SV_C128, basis_index=x0)
        try:
            a.run(g, flags)
            b.run(g, flags)
            c = sv.sv_compare(a.handle, b.handle)
            res = {"gates": int(len(g)), "c64_vs_c128_max_abs": c["max_abs"],
                   "c64_vs_c128_rel_l2": c["rel_l2"], "c64_norm_drift": c["norm_drift"],
                   "c128_norm_drift": abs(c["norm_b"] - 1.0),
                   "c64_rel_l2_bound": 8.0 * len(g) ** 0.5 * 2.0 ** -24}
            if gold is not None:
                idx = torch.from_numpy(gold["indices"]).to(a.tensor.device)
                ref = gold[f"{name}_amp"]
                g64 = a.tensor[idx].cpu().numpy().astype(np.complex128)
                g128 = b.tensor[idx].cpu().numpy()
                res["vs_oracle_sampled"] = {
                    "indices": int(len(ref)),
                    "c128_max_abs": float(np.max(np.abs(g128 - ref))),
                    "c64_max_abs": float(np.max(np.abs(g64 - ref))),
                    "c64_rel_l2": float(np.linalg.norm(g64 - ref) / np.linalg.norm(ref))}
        finally:
            a.close()
            b.close()
            torch.cuda.empty_cache()
        out[name] = res
        log(f"[bench] {name}: c64 vs c128 max-abs {c['max_abs']:.3e} rel {c['rel_l2']:.3e}")
    return out


# The sources of each kernel class (a change in any invalidates its counters).
# The tile passes also depend on the planner, which decides what each pass
# reads and writes.
KERNEL_SOURCE = {"tile": ("kernels_tile.hip", "tile_dev.h", "jit.hip", "plan.hip"),
                 "pair": ("kernels_gate.hip",), "pair_ctrl": ("kernels_gate.hip",),
                 "swap": ("kernels_gate.hip",), "diag": ("kernels_gate.hip",),
                 "dense": ("kernels_dense.hip",)}


def measured_traffic(cls, dtype_tag):
    """HBM bytes per launch of a kernel class from the committed rocprofv3
    counter summaries (profiles/*_traffic.txt), or None when there is none or
    the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    srcs = KERNEL_SOURCE.get(cls)
    if srcs is None:
        return None
    h = hashlib.sha256()
    for src in srcs:
        with open(os.path.join(ROOT, "paper_1801_01037_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    sha = h.hexdigest()[:16]
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.txt"))):
        with open(path) as f:
            for ln in f:
                tok = ln.split()
                if len(tok) == 7 and not ln.startswith("#") and tok[0] == cls and tok[1] == dtype_tag:
                    if tok[6] != sha:
                        return None
                    return (float(tok[2]) * float(tok[4]) + float(tok[3]) * float(tok[5])) * 1024
    return None


def roofline(run, dtype_tag):
    """Roofline of the kernel class with the most device time. Its bound is
    the roof with the longer ideal time per launch at the published peaks:
    HBM (algorithmic bytes / 8 TB/s) or vector ALU (algorithmic flops / the
    dtype's vector peak); the other roof is given as `secondary`.

    Algorithmic flops of the tile passes are the method's own, gate by gate
    (method_flops: every gate of a step is applied inside some tile pass, so a
    pass is credited the step's flops divided by its passes per step); the
    flops of the fused ops the passes execute are reported beside them."""
    prof = run["profile"]
    cls, d = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = d["total_ms"] / d["launches"]
    per_launch = d["bytes"] / d["launches"]
    op_flops = d["flops"] / d["launches"]
    flops = op_flops
    if cls == "tile":
        flops = run["method_flops_per_step"] * run["steps"] / d["launches"]
    mfma = cls == "dense"
    alu_peak = (MFMA_PEAK_TFLOPS if mfma else ALU_PEAK_TFLOPS)[dtype_tag]
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4)}
    alu_ach = flops / (avg_ms * 1e-3) / 1e12
    alu = {"bound": "mfma" if mfma else "alu", "achieved": round(alu_ach, 2), "peak": alu_peak,
           "unit": "TFLOP/s", "frac": round(alu_ach / alu_peak, 4)}
    t_hbm = per_launch / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (alu_peak * 1e12)
    first, second = (alu, hbm) if t_alu > t_hbm else (hbm, alu)
    out = dict(first)
    out.update({"traffic": measured_traffic(cls, dtype_tag), "kernel": cls,
                "launches": d["launches"], "avg_ms": round(avg_ms, 4),
                "bytes_per_launch": per_launch, "flops_per_launch": flops,
                "flops_per_launch_fused_ops": op_flops,
                "flops_counted": "method, gate by gate" if cls == "tile" else "kernel ops",
                "secondary": second})
    return out


def run_batched(sv, torch, count, seed=3):
    """512 independent layered circuits, n ~ U{10..24}, depth ~ U{20..200},
    complex64, run as one batch (HIP graph) with the autotuned launch
    configuration; latency of each circuit from the device clock."""
    import qcircuits as qc
    from paper_1801_01037_amd import autotune
    specs = qc.batch_specs(seed, count, 10, 24, 20, 200)
    stream = torch.cuda.Stream()
    states, plans, gates, alg_bytes = [], [], 0, 0.0
    t0 = time.perf_counter()
    for n, d, gs in specs:
        g = qc.layer_circuit(n, d, gs)
        gates += len(g)
        st = sv.StateVector(n, sv.SV_C64, stream=stream)
        states.append(st)
        plans.append(sv.sv_plan_create(st.handle, g))
        # algorithmic bytes of the circuit: every pass reads and writes the state
        alg_bytes += sv.sv_plan_passes(plans[-1]) * 2 * 8 * 2.0 ** n
    plan_s = time.perf_counter() - t0
    tune_n = min(64, count)
    (bpc, tpt), tune_times = autotune.tune_batch(sv.SV_C64, plans[:tune_n], f"layers-{tune_n}",
                                                 stream=stream)
    b = sv.sv_batch_create(sv.SV_C64, stream.cuda_stream)
    try:
        sv.sv_batch_config(b, bpc, tpt)
        # Circuits of at most 16 tiles per pass (n <= 16) run whole in the
        # persistent launch on the batch's second stream, circuits of 4096
        # tiles per pass (n = 24) pass by pass on its third stream, both beside
        # the level launches that take the rest.
        sv.sv_batch_persist(b, 16)
        sv.sv_batch_solo(b, 4096)
        for st in states:
            st.reset(0)
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)      # capture + first replay (warm-up)
        stream.synchronize()
        for st in states:
            st.reset(0)
        stream.synchronize()
        t1 = time.perf_counter()
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)
        stream.synchronize()
        wall = time.perf_counter() - t1
        start, end = sv.sv_batch_times(b, count)
        norms = [st.norm() for st in states[:8]]
        # The same batch with level launches only.
        sv.sv_batch_persist(b, 0)
        sv.sv_batch_solo(b, 0)
        for st in states:
            st.reset(0)
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)      # capture + first replay
        stream.synchronize()
        for st in states:
            st.reset(0)
        stream.synchronize()
        t2 = time.perf_counter()
        sv.sv_batch_run(b, plans, flags=sv.SV_GRAPH)
        stream.synchronize()
        pwall = time.perf_counter() - t2
        _, pend = sv.sv_batch_times(b, count)
        levels_only = {"p50_ms": round(float(np.percentile(pend, 50)), 3),
                      "p99_ms": round(float(np.percentile(pend, 99)), 3),
                      "makespan_ms": round(float(pend.max()), 3),
                      "gates_per_s": round(gates / pwall, 1)}
    finally:
        sv.sv_batch_destroy(b)
        for p in plans:
            sv.sv_plan_destroy(p)
        for st in states:
            st.close()
        torch.cuda.empty_cache()
    return {"circuits": count, "gates": gates, "dtype": "f32",
            "workload": "layered Haar-SU(2)/CNOT circuits, n ~ U{10..24}, depth ~ U{20..200}, "
                        "complex64, one batch replayed from a HIP graph: circuits of n <= 16 in a "
                        "persistent launch on a second stream, n = 24 pass by pass on a third, "
                        "the others in level launches",
            "p50_ms": round(float(np.percentile(end, 50)), 3),
            "p99_ms": round(float(np.percentile(end, 99)), 3),
            "makespan_ms": round(float(end.max()), 3), "wall_ms": round(wall * 1e3, 3),
            "effective_GBps": round(alg_bytes / (float(end.max()) * 1e-3) / 1e9, 1),
            "effective_GBps_note": "algorithmic bytes (2 N s per tile pass) over the makespan; "
                                   "states of n <= 24 complex64 fit the 256 MiB last-level cache, "
                                   "so this is not a fraction of HBM bandwidth",
            "gates_per_s": round(gates / wall, 1), "circuits_per_s": round(count / wall, 2),
            "autotuned": {"blocks_per_cu": bpc, "tiles_per_task": tpt,
                          "candidates_ms": {k: round(v, 3) for k, v in tune_times.items()}},
            "host_planning_s": round(plan_s, 2),
            "norm_max_dev": max(abs(x - 1.0) for x in norms),
            "persistent": {"max_tiles": 16,
                           "circuits": int(sum(1 for n, _, _ in specs if max(1, 2 ** (n - 12)) <= 16))},
            "pass_by_pass": {"min_tiles": 4096,
                             "circuits": int(sum(1 for n, _, _ in specs if 2 ** (n - 12) >= 4096))},
            "levels_only": levels_only}


def _event_times(torch, stream, fn, reps, warmup=3):
    """Device times (ms) of `reps` calls of fn, each between two HIP events on
    `stream`, after `warmup` untimed calls."""
    for _ in range(warmup):
        fn()
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def _stats(ms, nbytes):
    a = np.asarray(ms)
    med = float(np.median(a))
    return {"median_ms": round(med, 4), "min_ms": round(float(a.min()), 4),
            "p90_ms": round(float(np.percentile(a, 90)), 4),
            "GBps": round(nbytes / (med * 1e-3) / 1e9, 1)}


def run_pergate_1q(sv, torch, n, reps=10, targets=(0, 5, 11, 17, 23, 29)):
    """A Haar 2x2 gate alone on each of a few targets at n qubits (one pass of
    the state per gate), per dtype: algorithmic GB/s (2 N s per gate) and its
    fraction of the 8 TB/s HBM peak, median of `reps` HIP-event timings."""
    import qcircuits as qc
    out = {}
    for dt, tag, sb in ((sv.SV_C128, "c128", 16), (sv.SV_C64, "c64", 8)):
        st = sv.StateVector(n, dt)
        try:
            u = qc.haar_su2(5, 1)[0]
            gbps = [_stats(_event_times(torch, st.stream, lambda q=q: st.apply_1q(q, u), reps),
                           2 * 2.0 ** n * sb)["GBps"] for q in targets if q < n]
        finally:
            st.close()
            torch.cuda.empty_cache()
        fr = np.asarray(gbps) / HBM_PEAK_GBS
        out[tag] = {"targets": [q for q in targets if q < n], "GBps": gbps,
                    "frac_min": round(float(fr.min()), 4), "frac_median": round(float(np.median(fr)), 4)}
    return out


def run_sweep(sv, torch, n, reps):
    """Per-gate timings at n qubits: a Haar 2x2 on every qubit, CNOT on
    neighbours and on (0, n-1) both ways, controlled phases, and general
    5-qubit gates on fixed qubit sets (one dense block on the matrix cores).
    Bytes are the algorithmic ones: 2 N s for a full pass, N s for a CNOT (the
    control-1 half), N s / 2 for a controlled phase (the quarter with both bits
    set)."""
    import qcircuits as qc
    out = {}
    for dt, tag, sb in ((sv.SV_C128, "c128", 16), (sv.SV_C64, "c64", 8)):
        N = 2.0 ** n
        st = sv.StateVector(n, dt)
        try:
            u = qc.haar_su2(5, 1)[0]
            one = {q: _stats(_event_times(torch, st.stream, lambda q=q: st.apply_1q(q, u), reps),
                             2 * N * sb) for q in range(n)}
            pairs = [(q, q + 1) for q in range(n - 1)] + [(0, n - 1), (n - 1, 0)]
            cnot = {f"{c},{t}": _stats(_event_times(torch, st.stream,
                                                    lambda c=c, t=t: st.apply_ctrl(c, t, qc.X_MATRIX), reps),
                                       N * sb) for c, t in pairs}
            cp = {f"{c},{t}": _stats(_event_times(torch, st.stream,
                                                  lambda c=c, t=t: st.apply_cphase(c, t, 0.3), reps),
                                     N * sb / 2) for c, t in ((0, n - 1), (n // 2 - 1, n // 2))}
            blocks = {}
            for qs in ((0, 1, 2, 3, 4), (12, 13, 14, 15, 16), tuple(range(n - 5, n)),
                       (0, 7, 15, 22, n - 1)):
                m = qc.random_unitary(5, sum(qs))
                blocks[",".join(map(str, qs))] = _stats(
                    _event_times(torch, st.stream, lambda qs=qs, m=m: st.apply_unitary(qs, m), reps),
                    2 * N * sb)
        finally:
            st.close()
            torch.cuda.empty_cache()
        med1 = [v["median_ms"] for v in one.values()]
        out[tag] = {"one_qubit": one, "cnot": cnot, "cphase": cp, "block5": blocks,
                    "one_qubit_gates_per_s": round(1e3 / float(np.mean(med1)), 2)}
        log(f"[bench] sweep {tag}: 1q median {min(med1):.3f}..{max(med1):.3f} ms")
    return out


def run_xl(sv, torch, reps=1):
    """The 33-qubit complex128 and 34-qubit complex64 registers (128 GiB each):
    a seeded depth-10 layered circuit with dense 5-qubit blocks
    (SV_FUSE_DENSE), with tile passes (SV_FUSE) and gate by gate; each run is
    followed by the inverse circuit in the same mode, and the distance from
    |0...0> (max-abs over sampled indices and the amplitude at 0) and the norm
    drift measure the error against exact arithmetic."""
    import qcircuits as qc
    out = {}
    for n, dt, tag in ((33, sv.SV_C128, "c128_33q"), (34, sv.SV_C64, "c64_34q")):
        g = qc.layer_circuit(n, 10, 1000 + n)
        inv = qc.inverse_circuit(g)
        st = sv.StateVector(n, dt)
        res = {"gates": int(len(g))}
        try:
            idx = np.unique((qc.splitmix64(n, 4096) >> np.uint64(64 - n)).astype(np.int64))
            idx = idx[idx != 0]
            for name, flags in (("dense", sv.SV_FUSE_DENSE), ("fused", sv.SV_FUSE), ("pergate", 0)):
                st.reset(0)
                st.synchronize()
                t0 = time.perf_counter()
                st.run(g, flags)
                st.synchronize()
                el = time.perf_counter() - t0
                st.run(inv, flags)
                nrm = st.norm()
                amp0 = complex(st.tensor[0].item())
                off = float(st.tensor[torch.as_tensor(idx, device=st.tensor.device)].abs().max().item())
                res[name] = {"ms": round(el * 1e3, 1), "gates_per_s": round(len(g) / el, 1),
                             "mirror_abs_err_at_0": abs(amp0 - 1.0), "mirror_max_abs_sampled": off,
                             "norm_drift": abs(nrm - 1.0)}
                log(f"[bench] xl {tag} {name}: {el * 1e3:.0f} ms, |psi0-1| {abs(amp0 - 1.0):.2e}")
        finally:
            st.close()
            torch.cuda.empty_cache()
        out[tag] = res
    # Side by side at 33 qubits: the complex64 state (64 GiB) against the
    # complex128 state (128 GiB) of the same circuit, compared on the device.
    n = 33
    g = qc.layer_circuit(n, 10, 1000 + n)
    a = sv.StateVector(n, sv.SV_C64)
    b = sv.StateVector(n, sv.SV_C128)
    try:
        res = {"gates": int(len(g)), "c64_rel_l2_bound": 8.0 * len(g) ** 0.5 * 2.0 ** -24}
        for name, flags in (("fused", sv.SV_FUSE), ("dense", sv.SV_FUSE_DENSE)):
            a.reset(0)
            b.reset(0)
            a.run(g, flags)
            b.run(g, flags)
            c = sv.sv_compare(a.handle, b.handle)
            res[name] = {"max_abs": c["max_abs"], "rel_l2": c["rel_l2"],
                         "c64_norm_drift": c["norm_drift"], "c128_norm_drift": abs(c["norm_b"] - 1.0)}
            log(f"[bench] xl 33q c64 vs c128 {name}: max-abs {c['max_abs']:.2e} rel {c['rel_l2']:.2e}")
    finally:
        a.close()
        b.close()
        torch.cuda.empty_cache()
    out["c64_vs_c128_33q"] = res
    return out


def run_graph_cost(sv, torch, reps=30):
    """Short circuits run again and again, with and without SV_GRAPH: the host
    time a call takes to return (planning and launches) and the time to its
    completion, median over `reps` calls after warm-up; per-pass figures divide
    by the tile passes of one call."""
    import qcircuits as qc
    out = {}
    for n, depth, dt, tag in ((10, 20, sv.SV_C64, "c64"), (14, 20, sv.SV_C64, "c64"),
                              (18, 20, sv.SV_C128, "c128"), (22, 10, sv.SV_C128, "c128")):
        g = qc.layer_circuit(n, depth, 5)
        passes = sv.sv_plan_inspect(n, dt, g, sv.SV_FUSE)[1]
        st = sv.StateVector(n, dt)
        res = {"gates": int(len(g)), "passes": int(passes)}
        try:
            for name, flags in (("direct", sv.SV_FUSE), ("graph", sv.SV_FUSE | sv.SV_GRAPH)):
                for _ in range(3):
                    st.run(g, flags)
                st.synchronize()
                host, done = [], []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    st.run(g, flags)
                    t1 = time.perf_counter()
                    st.synchronize()
                    t2 = time.perf_counter()
                    host.append(t1 - t0)
                    done.append(t2 - t0)
                h, d = float(np.median(host)) * 1e3, float(np.median(done)) * 1e3
                res[name] = {"host_ms": round(h, 4), "completion_ms": round(d, 4),
                             "host_us_per_pass": round(1e3 * h / max(passes, 1), 2)}
            log(f"[bench] graph n={n} {tag}: host {res['direct']['host_ms']:.3f} -> "
                f"{res['graph']['host_ms']:.3f} ms, done {res['direct']['completion_ms']:.3f} -> "
                f"{res['graph']['completion_ms']:.3f} ms")
        finally:
            st.close()
        out[f"n{n}_{tag}"] = res
    return out


def run_serving(arrivals, rate=100.0, seed=0):
    from paper_1801_01037_amd import serving
    reqs = serving.poisson_requests(rate, arrivals, seed)
    srv = serving.Server(chunk=8)
    try:
        stats = srv.run(reqs)
    finally:
        srv.close()
    stats["offered_rps"] = rate
    stats["workload"] = ("Poisson arrivals, n ~ U{12..28}, depth ~ U{10..100}, complex64 or "
                         "complex128 (p = 1/2), continuous batching")
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()}


def host_cpu():
    """Threads this process may run on and the host's CPU model."""
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return int(threads or 1), model


def _oracle_gates_per_s(oracle, n, gates, budget_s):
    """Whole gates of `gates`, in order from |0>, until budget_s has passed
    (at least 2); returns (gates done, seconds)."""
    psi = oracle.basis_state(n, 0)
    done, t0 = 0, time.perf_counter()
    while done < len(gates):
        oracle.run_circuit(psi, gates[done:done + 1])
        done += 1
        if done >= 2 and time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    del psi
    return done, el


def cpu_baseline(n, budget_s):
    """The oracle stepping the same 30-qubit layered circuit, whole gates in
    order, on every host thread this process may use (the OpenMP build, the
    same bits as the reference build) and on one thread (the reference
    build), each for half of `budget_s`."""
    import oracle
    _, _, layers = workload(n)
    threads, model = host_cpu()
    used = oracle.set_threads(threads)
    d_all, t_all = _oracle_gates_per_s(oracle, n, layers, budget_s / 2)
    oracle.set_threads(1)
    d_one, t_one = _oracle_gates_per_s(oracle, n, layers, budget_s / 2)
    return {"value": round(d_all / t_all, 5), "unit": "gates/s", "cores": used, "kind": "oracle",
            "sample": f"first {d_all} gates of the {n}-qubit depth-20 layered circuit "
                      f"(complex128, from |0>), {t_all:.1f} s on {used} host threads",
            "single_thread": {"value": round(d_one / t_one, 5), "cores": 1,
                              "sample": f"first {d_one} gates, {t_one:.1f} s on one host thread"},
            "host": {"threads_available": threads, "cpu_model": model}}


def run_cpu_sweep(ns=(16, 20, 24, 28, 30), min_s=1.0):
    """The oracle's per-gate cost as the paper times single gates: a Haar 2x2
    gate on qubit 0, the middle qubit and the last one, at each n, on one
    host thread and on every available thread; each figure is the mean over
    repeats that fill at least `min_s` seconds (at least one)."""
    import oracle
    import qcircuits as qc
    threads, model = host_cpu()
    u = qc.haar_su2(5, 1)[0]
    rows = []
    for n in ns:
        psi = oracle.basis_state(n, 0)
        for k in (1, threads):
            used = oracle.set_threads(k)
            for q in (0, n // 2, n - 1):
                g = qc.gate_u(q, u)
                reps, t0 = 0, time.perf_counter()
                while reps < 1 or time.perf_counter() - t0 < min_s:
                    oracle.run_circuit(psi, g)
                    reps += 1
                sec = (time.perf_counter() - t0) / reps
                rows.append({"n": n, "target": q, "threads": used, "s_per_gate": sec,
                             "GBps": round(2 * 16 * 2.0 ** n / sec / 1e9, 2)})
                log(f"[bench] cpu n={n} q={q} threads={used}: {sec * 1e3:.2f} ms/gate")
        oracle.set_threads(1)
        del psi
    return {"host": {"threads_available": threads, "cpu_model": model}, "rows": rows}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).")
        sys.exit(2)
    if args.mode == "cpu_sweep":
        extra = run_cpu_sweep()
        rows = [r for r in extra["rows"] if r["n"] == 30 and r["threads"] > 1]
        value = round(1.0 / float(np.mean([r["s_per_gate"] for r in rows])), 4) if rows else None
        print(json.dumps({"metric": "30q gates/s and % HBM peak, c64 vs c128; batched p50/p99 circuit latency",
                          "value": value, "unit": "gates/s", "n_gpus": 0, "steps": 1, "warmup": 0,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f64", "data": "synthetic",
                          "config": {"workload": "oracle per-gate cost: Haar 2x2 on qubits 0, n/2, "
                                                 "n-1 at n = 16..30, one and all host threads",
                                     "mode": args.mode},
                          "cpu_sweep": extra}))
        return
    import torch
    import paper_1801_01037_amd as sv
    if not os.path.exists(sv.LIB_PATH):
        from paper_1801_01037_amd import build
        build.build()
    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if args.calibration_copy_mib:
        src = torch.ones(args.calibration_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calibration_copy_mib} MiB done")
        del src, dst
    if args.mode in ("sweep", "xl", "graph"):
        if args.mode == "sweep":
            extra = run_sweep(sv, torch, args.qubits, args.reps)
        elif args.mode == "xl":
            extra = run_xl(sv, torch)
        else:
            extra = run_graph_cost(sv, torch)
        if args.mode == "graph":
            value = round(extra["n14_c64"]["gates"] / (extra["n14_c64"]["graph"]["completion_ms"] * 1e-3), 1)
            workload = ("short layered circuits (n = 10, 14, 18, 22) run again and again with "
                        "SV_FUSE, with and without SV_GRAPH: host time per call and completion")
        elif args.mode == "sweep":
            value = extra["c128"]["one_qubit_gates_per_s"]
            workload = (f"{args.qubits}-qubit per-gate timings: Haar 2x2 on every qubit, CNOTs, "
                        "controlled phases, general 5-qubit gates; median of "
                        f"{args.reps} HIP-event timings each")
        else:
            value = extra["c128_33q"]["dense"]["gates_per_s"]
            workload = ("33-qubit complex128 / 34-qubit complex64 seeded depth-10 layered circuit, "
                        "dense 5-qubit blocks vs tile passes vs gate by gate, with mirror error")
        print(json.dumps({"metric": "30q gates/s and % HBM peak, c64 vs c128; batched p50/p99 circuit latency",
                          "value": value, "unit": "gates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f64", "data": "synthetic",
                          "config": {"workload": workload, "mode": args.mode},
                          args.mode: extra}))
        return
    flags = {"fused": sv.SV_FUSE | sv.SV_JIT, "fused-generic": sv.SV_FUSE, "pergate": 0,
             "dense": sv.SV_FUSE_DENSE}[args.mode]
    n = args.qubits
    log(f"[bench] c128 n={n} mode={args.mode} steps={args.steps} warmup={args.warmup}")
    r128 = run_dtype(sv, torch, sv.SV_C128, n, args.steps, args.warmup, flags)
    log(f"[bench] c128 {r128['gates_per_s']:.1f} gates/s, {r128['ms_per_step']:.1f} ms/step")
    generic = None
    if args.mode == "fused" and not args.no_generic:
        # the same steps with the generic tile kernel (no pass compiled)
        rg = run_dtype(sv, torch, sv.SV_C128, n, args.steps, args.warmup, sv.SV_FUSE)
        generic = {"value": round(rg["gates_per_s"], 3), "ms_per_step": round(rg["ms_per_step"], 3),
                   "roofline": roofline(rg, "c128")}
        log(f"[bench] c128 generic kernel {rg['gates_per_s']:.1f} gates/s")
    out_c64 = None
    if not args.no_c64:
        r64 = run_dtype(sv, torch, sv.SV_C64, n, args.steps, args.warmup, flags)
        log(f"[bench] c64 {r64['gates_per_s']:.1f} gates/s, {r64['ms_per_step']:.1f} ms/step")
        out_c64 = {"value": round(r64["gates_per_s"], 3), "unit": "gates/s", "dtype": "f32",
                   "ms_per_step": round(r64["ms_per_step"], 3),
                   "effective_hbm_frac": round(r64["effective_hbm_frac"], 4),
                   "speedup_vs_c128": round(r64["gates_per_s"] / r128["gates_per_s"], 3),
                   "roofline": roofline(r64, "c64"), "norm": r64["norm"]}
        if not args.no_errors:
            log("[bench] error statement: complex64 against complex128 and the oracle")
            out_c64["errors"] = precision_errors(sv, torch, n, flags)
    pergate = None
    if not args.no_pergate and args.mode in ("fused", "fused-generic"):
        log("[bench] per-gate 1q passes")
        pergate = run_pergate_1q(sv, torch, n)
    batched = None
    if not args.no_batched:
        log(f"[bench] batched: {args.batched_circuits} circuits")
        batched = run_batched(sv, torch, args.batched_circuits)
        log(f"[bench] batched p50 {batched['p50_ms']} ms p99 {batched['p99_ms']} ms")
    serving_stats = None
    if args.serving_arrivals:
        serving_stats = []
        for rate in [float(r) for r in args.serving_rates.split(",") if r]:
            arrivals = args.serving_arrivals
            if args.serving_seconds > 0:
                arrivals = min(arrivals, max(16, int(rate * args.serving_seconds)))
            log(f"[bench] serving: {arrivals} arrivals at {rate:g}/s")
            serving_stats.append(run_serving(arrivals, rate))
            log(f"[bench] serving p50 {serving_stats[-1].get('p50_ms')} ms "
                f"p99 {serving_stats[-1].get('p99_ms')} ms")
    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline ({args.cpu_seconds:.0f} s budget)")
        cpu = cpu_baseline(n, args.cpu_seconds)
    line = {
        "metric": "30q gates/s and % HBM peak, c64 vs c128; batched p50/p99 circuit latency",
        "value": round(r128["gates_per_s"], 3),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r128["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n}-qubit QFT of a seeded basis state + {n}-qubit depth-20 "
                               "Haar-SU(2)/CNOT layers, complex128, then norm and 2^20 probs",
                   "n_qubits": n, "gates_per_step": r128["gates_per_step"],
                   "mode": args.mode, "parallelism": "single GPU"},
        "effective_hbm_frac": round(r128["effective_hbm_frac"], 4),
        "roofline": roofline(r128, "c128"),
        "cpu_baseline": cpu,
        "c64": out_c64,
        "generic_kernel_c128": generic,
        "pergate_1q": pergate,
        "batched": batched,
        "serving": serving_stats,
        "kernels_c128": {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3),
                             "GBps": round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)}
                         for k, v in r128["profile"].items()},
        "norm_c128": r128["norm"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
