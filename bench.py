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
scalar fidelity and the 1024 probabilities).  The headline registers stream
every amplitude in every pass (lazy qubits off), so each fused launch moves
the same 2 x 8 x 2^30 bytes.

Prints one JSON line.  Extra figures: the same step in complex128 with its
own roofline and the complex64 result's error against it; the one-pass-per-
gate path; a measured device copy as the achievable HBM rate; batched Monte
Carlo trials/s (M=14, 500 gates, 4096 trials, one launch) beside the same
trials run one register at a time; the serving loop's p50/p99 latency and
throughput on a Poisson trace of 1000 requests against the same trace
served sequentially; the 64 GiB registers (M=33 complex64, M=32 complex128);
the structured 7^A mod 15 + quantum FFT workload with and without lazy
qubits.  The CPU leg times the FP64 oracle on all host cores and on one core,
and checks the GPU registers against it on the same gates.
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
# FP64 vector ceiling (complex128 registers): the published 78.6 TFLOP/s.
ALU_PEAK_TFLOPS_F64 = 78.6
M = 30
GATES = 1000
CIRCUIT_SEED = 30
ERROR_SEED = 1030
SIGMA = 1e-3
P_FLIP = 1e-4
PROBS_MASK = (1 << 10) - 1
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_tile_m30_c64_traffic.json")
TILE_SOURCE = os.path.join(ROOT, "paper_quant_ph_9804039_amd", "csrc", "tile_kernel.h")
SECTIONS = ("c128", "per_gate", "copy", "mc", "serving", "large", "structured", "three_state")


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


def roofline_of(stats_list, elem_bytes, alu_peak):
    """Roofline record of the fused tile pass from per-launch HIP-event times:
    algorithmic bytes 2 x elem x 2^M per launch (a read and a write of the
    register) and the operations' algorithmic flops, against the HBM peak and
    the ALU ceiling; the bound is the one the arithmetic intensity puts it
    under."""
    fused_ms = sum(s["fused_ms"] for s in stats_list)
    fused_n = sum(s["fused_passes"] for s in stats_list)
    launch_bytes = sum(s["fused_bytes"] for s in stats_list) / max(1, fused_n)
    avg_ms = fused_ms / max(1, fused_n)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    launch_flops = sum(s["fused_flops"] for s in stats_list) / max(1, fused_n)
    achieved_tf = launch_flops / (avg_ms * 1e-3) / 1e12
    intensity = launch_flops / launch_bytes
    ridge = alu_peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    hbm = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS}
    alu = {"bound": "alu", "achieved": achieved_tf, "peak": alu_peak, "unit": "TFLOP/s",
           "frac": achieved_tf / alu_peak}
    rec = dict(alu if intensity > ridge else hbm)
    rec.update({"launches": fused_n, "avg_launch_ms": avg_ms,
                "algorithmic_bytes_per_launch": launch_bytes,
                "algorithmic_flops_per_launch": launch_flops, "flop_per_byte": intensity,
                "ridge_flop_per_byte": ridge, "hbm_frac": hbm["frac"], "alu_frac": alu["frac"],
                "achieved_GBps": achieved})
    return rec


def run_steps(q, ideal, noisy, gates, steps, warmup, trial0, sync):
    def step(i):
        ideal.reset(0)
        noisy.reset(0)
        noisy.inject_errors(SIGMA, P_FLIP, P_FLIP, seed=ERROR_SEED, trial=i)
        ideal.apply(gates)
        noisy.apply(gates)
        F = ideal.fidelity(noisy)
        noisy.probs(PROBS_MASK)
        return F

    for i in range(warmup):
        step(trial0 + 10_000 + i)
    ideal.profile(True)
    noisy.profile(True)
    sync()
    t0 = time.perf_counter()
    Fs = [step(trial0 + i) for i in range(steps)]
    sync()
    wall = time.perf_counter() - t0
    st = [ideal.stats(), noisy.stats()]
    ideal.profile(False)
    noisy.profile(False)
    return wall, Fs, st


def state_error(a, b):
    """Error of register a against register b from their FP64 overlap:
    infidelity 1 - |<a|b>|^2 / (<a|a><b|b>) and the phase-aligned distance
    of the normalised states, sqrt(2 - 2 |<a|b>| / (|a| |b|))."""
    ab, aa, bb = a.overlap(b)
    c = abs(ab) / (aa * bb) ** 0.5
    return {"infidelity": 1.0 - c * c, "l2_distance": max(0.0, 2.0 - 2.0 * c) ** 0.5}


def bench_c128(q, cg, np, stream, gates, steps, sync):
    """The headline step in complex128 (same circuit, seeds and error
    model), with its own roofline, and the complex64 registers' error against
    the complex128 ones on one trial."""
    opt = q.torch_options(stream=stream, lazy_qubits=-1)
    with q.State(M, q.QSIM_C128, opt) as ideal, q.State(M, q.QSIM_C128, opt) as noisy:
        wall, Fs, st = run_steps(q, ideal, noisy, gates, steps, 1, 0, sync)
        roof = roofline_of(st, 16, ALU_PEAK_TFLOPS_F64)
        out = {"value": 2.0 * GATES * float(1 << M) * steps / wall, "unit": "amplitude-updates/s",
               "steps": steps, "ms_per_step": wall / steps * 1e3, "dtype": "f64",
               "fidelity_mean": float(np.mean(Fs)),
               "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac",
                                                 "avg_launch_ms", "launches",
                                                 "algorithmic_bytes_per_launch", "hbm_frac",
                                                 "alu_frac")},
               "kernel": "k_tile<double, 4, 256>"}
        # complex64 against complex128 on trial 0 (the step's first trial)
        opt64 = q.torch_options(stream=stream, lazy_qubits=-1, renorm_period=64)
        with q.State(M, q.QSIM_C64, opt64) as s64:
            for reg, armed in ((ideal, False), (noisy, True)):
                reg.reset(0)
                s64.reset(0)
                for s in (reg, s64):
                    if armed:
                        s.inject_errors(SIGMA, P_FLIP, P_FLIP, seed=ERROR_SEED, trial=0)
                    else:
                        s.inject_errors(None)
                    s.apply(gates)
                out["c64_vs_c128_" + ("noisy" if armed else "error_free")] = state_error(s64, reg)
    return out


def bench_copy(torch):
    """Achievable HBM rate: a 4 GiB device-to-device copy (read + write)."""
    n = 1 << 30
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    reps = 5
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": 2 * 4 * n, "ms": ms, "GBps": 2 * 4 * n / (ms * 1e-3) / 1e9}


def bench_mc(q, cg, np):
    """Batched Monte Carlo: 4096 trials of one M=14, 500-gate circuit in one
    persistent launch (complex64 registers, FP64 fidelity), beside the same
    trials run through the per-register path one at a time."""
    Mm, Gm, T = 14, 500, 4096
    gates = cg.random_circuit(Mm, Gm, 14)
    q.qsim_run_trials(gates, Mm, q.QSIM_C64, SIGMA, P_FLIP, P_FLIP, 1014, 0, 256)  # tune
    reps = []
    for _ in range(3):
        t0 = time.perf_counter()
        F = q.qsim_run_trials(gates, Mm, q.QSIM_C64, SIGMA, P_FLIP, P_FLIP, 1014, 0, T)
        reps.append(time.perf_counter() - t0)
    dt = float(np.median(reps))
    hist, _ = np.histogram(F, bins=100, range=(0.0, 1.0))
    inf = 1.0 - F
    exact = int(np.sum(inf <= 0.0))
    lhist, ledges = np.histogram(np.log10(inf[inf > 0.0]), bins=40, range=(-10.0, 0.0))
    # the same trials through the per-register path (two registers, one
    # circuit each per trial), on a sample
    S = 64
    with q.State(Mm, q.QSIM_C64) as ideal, q.State(Mm, q.QSIM_C64) as noisy:
        ideal.apply(gates)
        ideal.synchronize()
        t0 = time.perf_counter()
        Fp = []
        for t in range(S):
            noisy.reset(0)
            noisy.inject_errors(SIGMA, P_FLIP, P_FLIP, seed=1014, trial=t)
            noisy.apply(gates)
            Fp.append(ideal.fidelity(noisy))
        dtp = time.perf_counter() - t0
    Fp = np.array(Fp)
    per_reg = {"trials": S, "value": S / dtp, "unit": "trials/s",
               "batched_over_per_register": (T / dt) / (S / dtp),
               "max_abs_fidelity_diff_vs_batched": float(np.max(np.abs(Fp - F[:S])))}
    return {"value": T / dt, "unit": "trials/s", "trials": T, "num_qubits": Mm, "gates": Gm,
            "ms": dt * 1e3, "fidelity_mean": float(F.mean()), "fidelity_var": float(F.var()),
            "fidelity_hist_100bins_0_1": hist.tolist(),
            "log10_infidelity_hist": {"edges": [float(ledges[0]), float(ledges[-1])],
                                      "bins": len(lhist), "counts": lhist.tolist(),
                                      "exactly_one": exact},
            "per_register_path": per_reg}, gates, F


def bench_large(q, cg, np):
    """Large registers (64 GiB): M=33 complex64 and M=32 complex128, a
    500-gate circuit with half of the targets on the top 4 qubits, sigma =
    1e-3.  Fused-pass HBM rate of each: complex64 with the automatic qubit
    remap (the most used top qubits exchanged with low ones for the call) and
    without it, complex128 without it (its default) and with it forced; and
    the complex64 register's error against the complex128 one at M=33
    (192 GiB on the device at once)."""
    out = {"gates": 500, "top_bias": 0.5, "sigma": SIGMA}
    full = q.make_options(lazy_qubits=-1)
    runs = ((33, q.QSIM_C64, "m33_c64", 0), (33, q.QSIM_C64, "m33_c64_no_remap", -1),
            (32, q.QSIM_C128, "m32_c128", 0), (32, q.QSIM_C128, "m32_c128_remap_forced", 1))
    for Ml, dt, name, remap in runs:
        gates = cg.random_circuit(Ml, 500, Ml, top_bias=0.5)
        try:
            with q.State(Ml, dt, q.make_options(lazy_qubits=-1, remap_qubits=remap)) as s:
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
                     "remapped_qubit_pairs": st["remaps"],
                     "fused_passes": st["fused_passes"], "fused_GBps": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS if gbs else None,
                     "avg_fused_ms": st["fused_ms"] / max(1, st["fused_passes"]),
                     "ms": wall * 1e3}
    gates = cg.random_circuit(33, 500, 33, top_bias=0.5)
    try:
        with q.State(33, q.QSIM_C64, full) as a, q.State(33, q.QSIM_C128, full) as b:
            for s in (a, b):
                s.inject_errors(SIGMA, 0.0, 0.0, seed=1033, trial=0)
                s.apply(gates)
            out["m33_c64_vs_c128"] = state_error(a, b)
    except q.QsimError as e:
        out["m33_c64_vs_c128"] = {"error": str(e)}
    return out


def bench_three_state(q, cg, np):
    """The detailed three-state model (Sec. 2.0, Sec. 3.0): 19 ions, 3^19 =
    1.16e9 complex64 amplitudes (9.3 GB), 100 random gates lowered to laser
    transformations (a CNOT is five, through the auxiliary level) with angle
    errors and flips.  Fused passes (runs of transformations applied tile by
    tile in LDS, one HBM read and write per run) beside one launch per
    transformation (each rewrites the two levels it couples, 2/3 of the
    register, 2/9 when conditional), and how far apart the two are on the
    first 65536 amplitudes (rounding: FMA contraction may differ)."""
    M3, G3 = 19, 100
    gates = cg.random_circuit(M3, G3, 319, kinds=(cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT))
    pulses = q.qsim3_lower(gates, M3)
    eb = 8
    pair_amps = 2 * 3 ** (M3 - 1)
    amps = sum(pair_amps // (3 if p["cond_ion"] >= 0 else 1) for p in pulses)
    # algorithmic flops: a rotation pulse updates each amplitude of a pair as
    # c*a + v*b (2 + 6 + 2 flops), a phase pulse as one complex product (6)
    flops = sum(pair_amps // (3 if p["cond_ion"] >= 0 else 1) * (10 if p["kind"] == 0 else 6)
                for p in pulses)
    out = {"num_ions": M3, "amplitudes": 3 ** M3, "gates": G3, "transformations": len(pulses),
           "dtype": "c64"}
    results = {}
    for name, mode in (("fused", 0), ("per_transformation", 1)):
        with q.State3(M3, q.QSIM_C64, q.make_options(exec_mode=mode)) as s:
            s.apply(gates[:4])
            s.synchronize()
            walls = []
            for r in range(2):
                s.reset(0)
                s.inject_errors(SIGMA, P_FLIP, P_FLIP, seed=319, trial=r)
                s.synchronize()
                l0 = s.info()["launches"]
                t0 = time.perf_counter()
                s.apply(gates)
                s.synchronize()
                walls.append(time.perf_counter() - t0)
                launches = s.info()["launches"] - l0
            wall = min(walls)
            norm = float(np.sum(s.probs(1)))
            results[name] = s.amplitudes(0, 1 << 16)
        rec = {"seconds": wall, "transformations_per_s": len(pulses) / wall,
               "amplitude_updates_per_s": amps / wall, "norm_after": norm, "launches": launches}
        if mode == 1:
            # one launch per transformation: its algorithmic bytes are the
            # coupled levels, read and written
            gbps = 2 * amps * eb / wall / 1e9
        else:
            # a fused pass reads and writes the whole register once
            gbps = launches * 2 * 3 ** M3 * eb / wall / 1e9
        tflops = flops / wall / 1e12
        rec.update({"algorithmic_GBps": gbps, "hbm_frac": gbps / HBM_PEAK_GBS,
                    "algorithmic_TFLOPs": tflops, "alu_frac": tflops / ALU_PEAK_TFLOPS})
        out[name] = rec
    out["fused_vs_per_transformation_max_abs_diff"] = float(
        np.max(np.abs(results["fused"] - results["per_transformation"])))
    out["speedup_fused"] = out["per_transformation"]["seconds"] / out["fused"]["seconds"]
    return out


def bench_structured(q, cg, np):
    """The f(A) = 7^A mod 15 circuit (Sec. 2.2; 5 bits of A, H/X/CNOT/Toffoli)
    on the top 9 qubits of an M=30 complex64 register, 16 times over, then
    the quantum FFT on A: a permutation-heavy workload whose targets are all
    high qubits.  Lazy qubits: the 21 low qubits are never touched, so each
    pass visits one tile of 2^13 amplitudes; beside it the same circuit on a
    register that streams all 2^30 amplitudes in every pass."""
    Ms = 30
    qm = list(range(Ms - 9, Ms))
    one = cg.modexp15_circuit(5, qubit_map=qm)
    gates = np.concatenate([one] * 16 + [cg.qft_circuit(qm[:5])])
    out = {"gates": int(len(gates)), "num_qubits": Ms}
    for name, sigma, lazy in (("error_free_lazy", 0.0, 1), ("sigma_1e-3_lazy", SIGMA, 1),
                              ("error_free_full", 0.0, -1), ("sigma_1e-3_full", SIGMA, -1)):
        with q.State(Ms, q.QSIM_C64, q.make_options(lazy_qubits=lazy)) as s:
            reps = 5 if lazy > 0 else 1
            walls = []
            for r in range(reps + 1):
                s.reset(0)
                if sigma > 0:
                    s.inject_errors(sigma, 0.0, 0.0, seed=1415, trial=r)
                s.synchronize()
                if r == reps:
                    s.profile(True)
                t0 = time.perf_counter()
                s.apply(gates)
                s.synchronize()
                walls.append(time.perf_counter() - t0)
            st = s.stats()
            touched = s.touched_qubits()
            wall = float(np.median(walls[1:])) if reps > 1 else walls[-1]
        active = bin(touched).count("1")
        out[name] = {"amplitude_updates_per_s": len(gates) * float(1 << Ms) / wall,
                     "touched_qubits": active,
                     "touched_subspace_updates_per_s": len(gates) * float(1 << active) / wall,
                     "fused_passes": st["fused_passes"],
                     "fused_bytes_per_pass": st["fused_bytes"] / max(1, st["fused_passes"]),
                     "ms": wall * 1e3}
    return out


def bench_serving(q, cg, np, n_req: int = 1000, n_warm: int = 50):
    """Poisson request stream (M in [10, 28], 100-2000 gates, sigma in
    {1e-4, 1e-3, 1e-2}, complex64): 50 warm-up requests, then 1000 served
    with continuous batching against the same trace served one request at a
    time; offered load 0.8 x the measured sequential capacity."""
    trace = cg.poisson_trace(n_warm + n_req, 0.0, 4000)
    reqs = [{"M": r["M"], "dtype": q.QSIM_C64,
             "gates": cg.random_circuit(r["M"], r["G"], r["circuit_seed"]),
             "sigma": r["sigma"], "seed": r["error_seed"], "arrival_s": 0.0} for r in trace]
    warm, reqs = reqs[:n_warm], reqs[n_warm:]
    q.qsim_serve(warm, max_slots=8)
    t0 = time.perf_counter()
    q.qsim_serve(reqs, max_slots=1, strict_fifo=True)
    t_seq = time.perf_counter() - t0
    rate = 0.8 * n_req / t_seq
    arrivals = cg.poisson_trace(n_req, rate, 4001)
    for r, a in zip(reqs, arrivals):
        r["arrival_s"] = a["t"]
    buckets = ((10, 14), (15, 19), (20, 23), (24, 28))

    def summary(res):
        lat = np.array([x["done_s"] - r["arrival_s"] for r, x in zip(reqs, res)])
        Ms = np.array([r["M"] for r in reqs])
        span = max(x["done_s"] for x in res) - min(r["arrival_s"] for r in reqs)
        upd = sum(2.0 * len(r["gates"]) * float(1 << r["M"]) for r in reqs)
        per = {}
        for lo, hi in buckets:
            sel = (Ms >= lo) & (Ms <= hi)
            per[f"M{lo}-{hi}"] = {"requests": int(sel.sum()),
                                  "p50_ms": float(np.percentile(lat[sel], 50) * 1e3),
                                  "p99_ms": float(np.percentile(lat[sel], 99) * 1e3)}
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "requests_per_s": n_req / span, "amplitude_updates_per_s": upd / span,
                "per_M_bucket": per, "failed": int(sum(x["status"] != 0 for x in res))}

    batched_res = q.qsim_serve(reqs, max_slots=8)
    sequential_res = q.qsim_serve(reqs, max_slots=1, strict_fifo=True)
    same = max(abs(a["fidelity"] - b["fidelity"]) for a, b in zip(batched_res, sequential_res))
    return {"requests": n_req, "warmup_requests": n_warm, "offered_rate_per_s": rate,
            "sequential_capacity_per_s": n_req / t_seq,
            "continuous_batching": summary(batched_res), "sequential": summary(sequential_res),
            "admission": "8 slots, FIFO with backfill, at most one request with registers "
                         ">= 256 MiB in flight",
            "max_abs_fidelity_diff_batched_vs_sequential": same}


def cpu_leg(q, np, gates, mc_gates, mc_F, budget_s: float = 15.0, t1_budget_s: float = 8.0):
    """The FP64 oracle on the host: the first gates of the noisy M=30 run on
    all host cores (timed around the gate loop) and on one core; the GPU
    complex64 and complex128 registers against the oracle's state after the
    same gates; the oracle's Monte Carlo trials on the first 64 trials of the
    batched workload, against the GPU's fidelities; the three-state oracle on
    16 ions."""
    import oracle
    oracle.build(force=False)
    em = oracle.Errors(sigma=SIGMA, p_bitflip=P_FLIP, p_phaseflip=P_FLIP, seed=ERROR_SEED, trial=0)
    cores = oracle.num_threads()
    psi = oracle.init(M, 0)
    done, t0 = 0, time.perf_counter()
    while done < 200 and time.perf_counter() - t0 < budget_s:
        oracle.run(psi, M, gates[done:done + 1], em, step0=done)
        done += 1
    dt = time.perf_counter() - t0
    # one core: the first gates again, from a fresh register
    oracle.set_num_threads(1)
    psi1 = oracle.init(M, 0)
    done1, t1 = 0, time.perf_counter()
    while done1 < done and time.perf_counter() - t1 < t1_budget_s:
        oracle.run(psi1, M, gates[done1:done1 + 1], em, step0=done1)
        done1 += 1
    dt1 = time.perf_counter() - t1
    del psi1
    oracle.set_num_threads(cores)
    base = {"value": done * float(1 << M) / dt, "unit": "amplitude-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {done} gates of the noisy M={M} run (complex128, FP64), "
                      f"{dt:.1f} s on {cores} host threads",
            "t1": {"value": done1 * float(1 << M) / dt1, "cores": 1, "gates": done1,
                   "seconds": dt1}}
    # the three-state oracle on the largest register it takes (16 ions), the
    # first 10 gates of the three-state workload's kinds
    import circuitgen as cg
    Mo = 16
    go = cg.random_circuit(Mo, 10, 316, kinds=(cg.H, cg.RZ, cg.X, cg.Z, cg.CNOT))
    po = q.qsim3_lower(go, Mo)
    t3 = time.perf_counter()
    oracle.simulate3(Mo, go)
    dt3 = time.perf_counter() - t3
    ao = sum(2 * 3 ** (Mo - 1) // (3 if p["cond_ion"] >= 0 else 1) for p in po)
    base["three_state"] = {"num_ions": Mo, "transformations": len(po), "seconds": dt3,
                           "amplitude_updates_per_s": ao / dt3, "cores": cores}
    # GPU registers after the same gates, against the oracle's state
    ref = psi.view(np.complex128)
    nref = float(np.vdot(ref, ref).real)
    prec = {"gates": done}
    for dt_, name in ((q.QSIM_C64, "c64"), (q.QSIM_C128, "c128")):
        with q.State(M, dt_, q.make_options(lazy_qubits=-1)) as s:
            s.inject_errors(SIGMA, P_FLIP, P_FLIP, seed=ERROR_SEED, trial=0)
            s.apply(gates[:done])
            a = s.amplitudes()
        ov = np.vdot(ref, a)
        na = float(np.vdot(a, a).real)
        mx = 0.0
        for lo in range(0, len(a), 1 << 24):
            mx = max(mx, float(np.max(np.abs(a[lo:lo + (1 << 24)] - ref[lo:lo + (1 << 24)]))))
        prec[name] = {"infidelity": 1.0 - abs(ov) ** 2 / (na * nref), "max_abs_amp_err": mx,
                      "norm_sq": na}
        del a
    del psi, ref
    # Monte Carlo trials
    emc = oracle.Errors(sigma=SIGMA, p_bitflip=P_FLIP, p_phaseflip=P_FLIP, seed=1014, trial=0)
    t0 = time.perf_counter()
    Fo = oracle.run_trials(mc_gates, 14, emc, 64)
    dto = time.perf_counter() - t0
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.run_trials(mc_gates, 14, emc, 8)
    dto1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    mc = {"trials": 64, "value": 64 / dto, "unit": "trials/s", "cores": cores,
          "t1_value": 8 / dto1, "max_abs_fidelity_diff_gpu": float(np.max(np.abs(Fo - mc_F[:64])))}
    return base, prec, mc


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip-extra", action="store_true",
                    help="time the M=30 step only (for counter runs under a profiler)")
    ap.add_argument("--only", default="",
                    help="comma-separated extra sections to run after the step (of "
                         + ", ".join(SECTIONS) + "), without the CPU leg")
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
    only = [s for s in args.only.split(",") if s]
    for s in only:
        if s not in SECTIONS:
            print(f"bench.py: unknown section {s!r}", file=sys.stderr)
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
    opt = q.torch_options(stream=stream, renorm_period=64, lazy_qubits=-1)
    ideal = q.State(M, q.QSIM_C64, opt)
    noisy = q.State(M, q.QSIM_C64, opt)

    log(f"bench: M={M} c64, {GATES} gates, warmup {args.warmup}, timing {args.steps} steps")
    wall, Fs, st = run_steps(q, ideal, noisy, gates, args.steps, args.warmup, 0,
                             torch.cuda.synchronize)
    st_i, st_n = st
    value = 2.0 * GATES * float(1 << M) * args.steps / wall
    roof = roofline_of(st, 8, ALU_PEAK_TFLOPS)
    log(f"bench: {value:.3e} amp-upd/s, fused pass {roof['avg_launch_ms']:.3f} ms avg, "
        f"{roof['achieved_GBps']:.0f} GB/s, {roof['alu_frac'] * ALU_PEAK_TFLOPS:.1f} TFLOP/s, "
        f"{roof['flop_per_byte']:.1f} flop/B (ridge {roof['ridge_flop_per_byte']:.1f})")
    if args.skip_extra:
        print(json.dumps({"value": value, "avg_launch_ms": roof["avg_launch_ms"],
                          "achieved_GBps": roof["achieved_GBps"],
                          "flop_per_byte": roof["flop_per_byte"]}))
        return 0
    sections = only or list(SECTIONS)
    extra = {"fidelity_mean": float(np.mean(Fs)),
             "gates_per_fused_pass": (st_i["gates"] + st_n["gates"]) / max(1, roof["launches"]),
             "flips_injected": st_n["flips"]}

    if "per_gate" in sections:
        # the same circuit through the one-pass-per-gate path (context)
        plain = q.State(M, q.QSIM_C64, q.torch_options(stream=stream, exec_mode=1,
                                                       renorm_period=64))
        plain.apply(gates[:20])
        torch.cuda.synchronize()
        plain.profile(True)
        tp = time.perf_counter()
        plain.apply(gates[:200])
        plain.synchronize()
        tplain = time.perf_counter() - tp
        stp = plain.stats()
        plain.close()
        extra["per_gate_path"] = {"value": 200 * float(1 << M) / tplain,
                                  "unit": "amplitude-updates/s",
                                  "algorithmic_GBps": stp["pass_bytes"] / (stp["pass_ms"] * 1e-3) / 1e9,
                                  "gates": 200}
        log(f"bench: per-gate path {extra['per_gate_path']['value']:.3e} amp-upd/s")
    if "c128" in sections:
        log("bench: complex128 leg")
        extra["c128"] = bench_c128(q, cg, np, stream, gates, max(2, args.steps // 4),
                                   torch.cuda.synchronize)
        log(f"bench: c128 {json.dumps(extra['c128'])}")
    copy = None
    if "copy" in sections:
        copy = bench_copy(torch)
        extra["copy"] = copy
        log(f"bench: device copy {copy['GBps']:.0f} GB/s")
    ideal.close()
    noisy.close()
    del ideal, noisy
    torch.cuda.empty_cache()

    mc_gates = mc_F = None
    if "mc" in sections:
        log("bench: batched Monte Carlo")
        extra["mc_trials"], mc_gates, mc_F = bench_mc(q, cg, np)
        log(f"bench: {extra['mc_trials']['value']:.0f} trials/s")
    if "serving" in sections:
        log("bench: serving")
        extra["serving"] = bench_serving(q, cg, np)
        log(f"bench: serving p99 {extra['serving']['continuous_batching']['p99_ms']:.1f} ms "
            f"(sequential {extra['serving']['sequential']['p99_ms']:.1f} ms)")
    if "large" in sections:
        log("bench: 64 GiB registers")
        extra["large_register"] = bench_large(q, cg, np)
        log(f"bench: large registers {json.dumps(extra['large_register'])}")
    if "three_state" in sections:
        log("bench: three-state model (19 ions)")
        extra["three_state"] = bench_three_state(q, cg, np)
        log(f"bench: three-state {json.dumps(extra['three_state'])}")
    if "structured" in sections:
        log("bench: structured workload (7^A mod 15 and the quantum FFT on the top qubits)")
        extra["structured_modexp15_qft"] = bench_structured(q, cg, np)
        log(f"bench: structured {json.dumps(extra['structured_modexp15_qft'])}")

    cpu = None
    if not args.no_cpu_baseline and not only:
        log("bench: oracle on the host")
        cpu, prec, mc_oracle = cpu_leg(q, np, gates, mc_gates, mc_F)
        extra["error_vs_fp64_oracle"] = prec
        extra["mc_trials"]["oracle"] = mc_oracle

    roofline = {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roofline["traffic"] = measured_traffic()
    roofline.update({k: roof[k] for k in ("launches", "avg_launch_ms",
                                          "algorithmic_bytes_per_launch",
                                          "algorithmic_flops_per_launch", "flop_per_byte",
                                          "ridge_flop_per_byte", "hbm_frac", "alu_frac")})
    roofline["kernel"] = "k_tile<float, 4, 512> (fused tile pass)"
    if copy:
        roofline["frac_vs_measured_copy"] = roof["achieved_GBps"] / copy["GBps"]
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
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
