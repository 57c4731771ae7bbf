#!/usr/bin/env python3
"""Benchmark of the error-injecting state-vector simulator on one MI355X.

One step = the whole hot path on one register of M = 30 qubits (complex64
state, FP64 reductions) and a seeded 1000-gate random circuit over H, Rz,
CNOT and Toffoli: reset both registers to |0...0>, run the error-free
circuit, run it again with errors injected at every step (per-gate angle
error sigma = 1e-3, bit and phase flips p = 1e-4 per qubit per step, fresh
trial key each step), renormalise every 64 gates, score the noisy register
by its fidelity against the error-free one, and read the marginal
probabilities of the 10 low qubits.  Throughput is amplitude updates per
second: 2 runs x 1000 gates x 2^30 amplitudes per step over the timed wall
time (inputs resident in device memory, no host transfers besides the
scalar fidelity and the 1024 probabilities).

Prints one JSON line.  Extra figures: the same circuit on the one-pass-per-
gate path, the roofline of the fused tile pass (HIP events around each
launch; algorithmic bytes 2 x 8 x 2^30 and algorithmic flops per launch, and
the ceiling its arithmetic intensity puts it under), the FP64 oracle timed on
a bounded sample on the host cores, batched Monte Carlo trials/s (M=14, 500
gates, 4096 trials, one launch), and the serving loop's p50/p99 latency and
throughput on a Poisson trace against the same trace served sequentially,
and the 64 GiB registers (M=33 complex64, M=32 complex128): fused-pass HBM
rate and the complex64 error against complex128.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# FP32 vector FMA ceiling without packed-FP32 instructions (the library's
# kernels are compiled without them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# per FMA x 2.4 GHz.
# The published 157.3 TFLOP/s counts packed FP32 (two FMAs per lane).
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
M = 30
GATES = 1000
CIRCUIT_SEED = 30
ERROR_SEED = 1030
SIGMA = 1e-3
P_FLIP = 1e-4
PROBS_MASK = (1 << 10) - 1
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tile_m30_c64_traffic.json")
TILE_SOURCE = os.path.join(ROOT, "paper_quant_ph_9804039_amd", "csrc", "tile_kernel.h")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def measured_traffic():
    """Per-launch HBM bytes of the fused pass from the committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(TILE_SOURCE, "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
        if rec.get("kernel_source_sha256") != h:
            return None
        return rec.get("bytes_per_launch")
    except (OSError, ValueError):
        return None


def cpu_baseline(gates, budget_s: float = 15.0, max_gates: int = 200):
    """FP64 oracle on the host cores: the first gates of the noisy run at the
    same register size, timed around the gate loop only."""
    import oracle
    oracle.build(force=False)
    em = oracle.Errors(sigma=SIGMA, p_bitflip=P_FLIP, p_phaseflip=P_FLIP, seed=ERROR_SEED, trial=0)
    psi = oracle.init(M, 0)
    done, t0 = 0, time.perf_counter()
    while done < max_gates and time.perf_counter() - t0 < budget_s:
        oracle.run(psi, M, gates[done:done + 1], em, step0=done)
        done += 1
    dt = time.perf_counter() - t0
    del psi
    return {"value": done * float(1 << M) / dt, "unit": "amplitude-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {done} gates of the noisy M={M} run (complex128, FP64), "
                      f"{dt:.1f} s on the host"}


def bench_mc(q, cg, np):
    """Batched Monte Carlo: 4096 trials of one M=14, 500-gate circuit in one
    persistent launch (complex64 registers, FP64 fidelity)."""
    Mm, Gm, T = 14, 500, 4096
    gates = cg.random_circuit(Mm, Gm, 14)
    q.qsim_run_trials(gates, Mm, q.QSIM_C64, SIGMA, P_FLIP, P_FLIP, 1014, 0, 256)  # tune
    reps = []
    for _ in range(3):
        t0 = time.perf_counter()
        F = q.qsim_run_trials(gates, Mm, q.QSIM_C64, SIGMA, P_FLIP, P_FLIP, 1014, 0, T)
        reps.append(time.perf_counter() - t0)
    dt = float(np.median(reps))
    hist, edges = np.histogram(F, bins=10, range=(0.0, 1.0))
    return {"value": T / dt, "unit": "trials/s", "trials": T, "num_qubits": Mm, "gates": Gm,
            "ms": dt * 1e3, "fidelity_mean": float(F.mean()), "fidelity_var": float(F.var()),
            "fidelity_hist_10bins": hist.tolist()}


def bench_large(q, cg, np):
    """Large registers (64 GiB): M=33 complex64 and M=32 complex128, a
    500-gate circuit with half of the targets on the top 4 qubits, sigma =
    1e-3.  Fused-pass HBM rate of each, and the complex64 register's error
    against the complex128 one at M=33 (192 GiB on the device at once)."""
    out = {"gates": 500, "top_bias": 0.5, "sigma": SIGMA}
    for Ml, dt, name in ((33, q.QSIM_C64, "m33_c64"), (32, q.QSIM_C128, "m32_c128")):
        gates = cg.random_circuit(Ml, 500, Ml, top_bias=0.5)
        try:
            with q.State(Ml, dt) as s:
                s.inject_errors(SIGMA, 0.0, 0.0, seed=1000 + Ml, trial=0)
                s.apply(gates[:20])
                s.synchronize()
                s.profile(True)
                t0 = time.perf_counter()
                s.apply(gates)
                s.synchronize()
                wall = time.perf_counter() - t0
                st = s.stats()
        except q.QsimError as e:
            out[name] = {"error": str(e)}
            continue
        gbs = st["fused_bytes"] / (st["fused_ms"] * 1e-3) / 1e9 if st["fused_ms"] > 0 else None
        out[name] = {"amplitude_updates_per_s": 500 * float(1 << Ml) / wall,
                     "fused_passes": st["fused_passes"], "fused_GBps": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS if gbs else None,
                     "ms": wall * 1e3}
    # complex64 error at M=33, measured against complex128 on the device
    gates = cg.random_circuit(33, 500, 33, top_bias=0.5)
    try:
        with q.State(33, q.QSIM_C64) as a, q.State(33, q.QSIM_C128) as b:
            for s in (a, b):
                s.inject_errors(SIGMA, 0.0, 0.0, seed=1033, trial=0)
                s.apply(gates)
            out["m33_c64_infidelity_vs_c128"] = 1.0 - a.fidelity(b)
    except q.QsimError as e:
        out["m33_c64_infidelity_vs_c128"] = {"error": str(e)}
    return out


def bench_structured(q, cg, np):
    """The f(A) = 7^A mod 15 circuit (Sec. 2.2; 5 bits of A, H/X/CNOT/Toffoli)
    on the top 9 qubits of an M=30 complex64 register, 16 times over: a
    permutation-heavy workload whose targets are all high qubits.  Error-free
    (the X-type gates are exact swaps) and with sigma = 1e-3."""
    M = 30
    one = cg.modexp15_circuit(5, qubit_map=list(range(M - 9, M)))
    gates = np.concatenate([one] * 16)
    out = {"gates": int(len(gates)), "num_qubits": M}
    for name, sigma in (("error_free", 0.0), ("sigma_1e-3", SIGMA)):
        with q.State(M, q.QSIM_C64) as s:
            if sigma > 0.0:
                s.inject_errors(sigma, 0.0, 0.0, seed=1415, trial=0)
            s.apply(gates[:24])
            s.synchronize()
            s.profile(True)
            t0 = time.perf_counter()
            s.apply(gates)
            s.synchronize()
            wall = time.perf_counter() - t0
            st = s.stats()
        gbs = st["fused_bytes"] / (st["fused_ms"] * 1e-3) / 1e9 if st["fused_ms"] > 0 else None
        out[name] = {"amplitude_updates_per_s": len(gates) * float(1 << M) / wall,
                     "fused_passes": st["fused_passes"], "fused_GBps": gbs, "ms": wall * 1e3}
    return out


def bench_serving(q, cg, np, n_req: int = 80):
    """Poisson request stream (M in [10, 28], 100-2000 gates, sigma in
    {1e-4, 1e-3, 1e-2}, complex64): continuous batching against the same
    trace served one request at a time."""
    trace = cg.poisson_trace(n_req, 0.0, 4000)
    reqs = [{"M": r["M"], "dtype": q.QSIM_C64,
             "gates": cg.random_circuit(r["M"], r["G"], r["circuit_seed"]),
             "sigma": r["sigma"], "seed": r["error_seed"], "arrival_s": 0.0} for r in trace]
    q.qsim_serve(reqs[:4], max_slots=2)  # warm-up
    t0 = time.perf_counter()
    q.qsim_serve(reqs, max_slots=1, strict_fifo=True)
    t_seq = time.perf_counter() - t0
    rate = 0.8 * n_req / t_seq
    arrivals = cg.poisson_trace(n_req, rate, 4001)
    for r, a in zip(reqs, arrivals):
        r["arrival_s"] = a["t"]

    def summary(res):
        lat = np.array([x["done_s"] - r["arrival_s"] for r, x in zip(reqs, res)])
        span = max(x["done_s"] for x in res) - min(r["arrival_s"] for r in reqs)
        upd = sum(2.0 * len(r["gates"]) * float(1 << r["M"]) for r in reqs)
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "requests_per_s": n_req / span, "amplitude_updates_per_s": upd / span}

    batched = summary(q.qsim_serve(reqs, max_slots=8))
    sequential = summary(q.qsim_serve(reqs, max_slots=1, strict_fifo=True))
    return {"requests": n_req, "offered_rate_per_s": rate,
            "sequential_capacity_per_s": n_req / t_seq,
            "continuous_batching": batched, "sequential": sequential}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-extra", action="store_true",
                    help="time the M=30 step only (for counter runs under a profiler)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 4 GiB device-to-device copy 5 times (the known-size "
                         "kernel the HBM byte counters are scaled by) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        n = 1 << 30  # 4 GiB of float32
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))
        return 0
    if args.gpus != 1:
        print("bench.py: the simulator holds one register on one GPU; --gpus must be 1 "
              "(sharding a register over several GPUs is not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import circuitgen as cg
    import paper_quant_ph_9804039_amd as q

    torch.cuda.set_device(0)
    # one explicit stream (default priority) for both registers, so the
    # kernels run back to back and the per-launch HIP events time them alone
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    gates = cg.random_circuit(M, GATES, CIRCUIT_SEED)
    opt = q.torch_options(stream=stream, renorm_period=64)
    ideal = q.State(M, q.QSIM_C64, opt)
    noisy = q.State(M, q.QSIM_C64, opt)

    def step(i: int) -> float:
        ideal.reset(0)
        noisy.reset(0)
        noisy.inject_errors(SIGMA, P_FLIP, P_FLIP, seed=ERROR_SEED, trial=i)
        ideal.apply(gates)
        noisy.apply(gates)
        F = ideal.fidelity(noisy)
        noisy.probs(PROBS_MASK)
        return F

    log(f"bench: M={M} c64, {GATES} gates, warmup {args.warmup}")
    for i in range(args.warmup):
        step(10_000 + i)
    ideal.profile(True)
    noisy.profile(True)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    Fs = [step(i) for i in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st_i, st_n = ideal.stats(), noisy.stats()
    ideal.profile(False)
    noisy.profile(False)

    upd = 2.0 * GATES * float(1 << M) * args.steps
    value = upd / wall
    fused_ms = st_i["fused_ms"] + st_n["fused_ms"]
    fused_n = st_i["fused_passes"] + st_n["fused_passes"]
    launch_bytes = 2.0 * 8.0 * float(1 << M)
    avg_ms = fused_ms / max(1, fused_n)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    launch_flops = (st_i["fused_flops"] + st_n["fused_flops"]) / max(1, fused_n)
    achieved_tf = launch_flops / (avg_ms * 1e-3) / 1e12
    # roofline: the pass is ALU-bound when its arithmetic intensity is past
    # the ridge point of the two ceilings
    intensity = launch_flops / launch_bytes
    ridge = ALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = measured_traffic()
    log(f"bench: {value:.3e} amp-upd/s, fused pass {avg_ms:.3f} ms avg, {achieved:.0f} GB/s, "
        f"{achieved_tf:.1f} TFLOP/s, {intensity:.1f} flop/B (ridge {ridge:.1f})")

    if args.skip_extra:
        print(json.dumps({"value": value, "avg_launch_ms": avg_ms, "achieved_GBps": achieved,
                          "achieved_TFLOPs": achieved_tf, "flop_per_byte": intensity}))
        return 0

    # the same circuit through the one-pass-per-gate path (context)
    plain = q.State(M, q.QSIM_C64, q.torch_options(stream=stream, exec_mode=1, renorm_period=64))
    plain.apply(gates[:20])
    torch.cuda.synchronize()
    plain.profile(True)
    tp = time.perf_counter()
    plain.apply(gates[:200])
    plain.synchronize()
    tplain = time.perf_counter() - tp
    stp = plain.stats()
    plain.close()
    plain_value = 200 * float(1 << M) / tplain
    plain_gbs = stp["pass_bytes"] / (stp["pass_ms"] * 1e-3) / 1e9
    log(f"bench: per-gate path {plain_value:.3e} amp-upd/s, {plain_gbs:.0f} GB/s algorithmic")

    ideal.close()
    noisy.close()
    del ideal, noisy
    torch.cuda.empty_cache()

    log("bench: batched Monte Carlo")
    mc = bench_mc(q, cg, np)
    log(f"bench: {mc['value']:.0f} trials/s")
    log("bench: serving")
    serving = bench_serving(q, cg, np)
    log(f"bench: serving p99 {serving['continuous_batching']['p99_ms']:.1f} ms "
        f"(sequential {serving['sequential']['p99_ms']:.1f} ms)")
    log("bench: 64 GiB registers")
    large = bench_large(q, cg, np)
    log(f"bench: large registers {json.dumps(large)}")
    log("bench: structured workload (7^A mod 15 on the top qubits)")
    structured = bench_structured(q, cg, np)
    log(f"bench: structured {json.dumps(structured)}")

    cpu = None
    if not args.no_cpu_baseline:
        log("bench: oracle sample on the host")
        cpu = cpu_baseline(gates)

    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS}
    alu = {"bound": "alu", "achieved": achieved_tf, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved_tf / ALU_PEAK_TFLOPS}
    roofline = dict(alu if intensity > ridge else hbm)
    roofline.update({
        "traffic": traffic, "kernel": "k_tile (fused tile pass)", "launches": fused_n,
        "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": launch_bytes,
        "algorithmic_flops_per_launch": launch_flops, "flop_per_byte": intensity,
        "ridge_flop_per_byte": ridge, "hbm_frac": hbm["frac"], "alu_frac": alu["frac"]})
    out = {
        "metric": "amplitude-updates/s & % HBM BW at M=30; MC trials/s at M=14; p99 latency",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded uniform random circuit, seeded error draws",
        "config": {"workload": "random-circuit-M30-c64-1000g-sigma1e-3-p1e-4",
                   "num_qubits": M, "gates": GATES, "state": "complex64 (FP64 reductions)",
                   "gate_set": "H, Rz(U[0,2pi)), CNOT, Toffoli", "sigma": SIGMA,
                   "p_bitflip": P_FLIP, "p_phaseflip": P_FLIP, "renorm_period": 64,
                   "circuit_seed": CIRCUIT_SEED, "error_seed": ERROR_SEED,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": {
            "fidelity_mean": float(np.mean(Fs)),
            "gates_per_fused_pass": (st_i["gates"] + st_n["gates"]) / max(1, fused_n),
            "flips_injected": st_n["flips"],
            "per_gate_path": {"value": plain_value, "unit": "amplitude-updates/s",
                              "algorithmic_GBps": plain_gbs, "gates": 200},
            "mc_trials": mc,
            "serving": serving,
            "large_register": large,
            "structured_modexp15": structured,
        },
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
