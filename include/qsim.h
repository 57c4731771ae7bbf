/*
 * qsim -- state-vector simulation with injected errors on one AMD Instinct
 * MI355X (gfx950), after Obenland & Despain, "A Parallel Quantum Computer
 * Simulator" (arXiv quant-ph/9804039).
 *
 * The library keeps one whole register of M qubits as a 2^M complex vector in
 * device memory (Sec. 1.2 and Fig. 1: index bit q holds the value of qubit q),
 * applies circuits of logic gates to it (Sec. 2.0: one-, two- and three-bit
 * controlled-NOTs and rotations; Sec. 2.1: every gate is a 2x2 transform on
 * the V/2 amplitude pairs that differ in the target bit), optionally injects
 * errors at every step (Sec. 1.0, 1.4, 2.0: angle deviations; Sec. 3.4 and
 * EQ 8: two extra decoherence transforms after every operation), and scores
 * the result by an inner-product fidelity against another state.
 *
 * Conventions fixed by the library (the paper leaves them open):
 *   - qubit q <-> index bit 2^q; on two qubits CNOT(control 1, target 0)
 *     swaps amplitudes 2 and 3 (Table 1, Fig. 2);
 *   - H = sqrt(1/2) [[1, 1], [1, -1]]; Rz(t) = diag(e^{-it/2}, e^{+it/2});
 *   - angle error: one eps = sigma * z per gate, z ~ N(0, 1).  Rz(t) becomes
 *     Rz(t + eps); H, X, CNOT, Toffoli and Z become i * R_n(pi + eps) about
 *     their own axis n (so eps = 0 gives the textbook gate exactly, and the
 *     unperturbed X/CNOT/Toffoli/Z are exact amplitude swaps / sign flips);
 *   - decoherence after every gate: for q = 0..M-1 in turn, a bit flip X_q
 *     with probability p_bitflip, then a phase flip Z_q with probability
 *     p_phaseflip, both exact;
 *   - draws: Philox4x64-10 (Salmon et al., SC'11), key (seed, trial),
 *     counter (step, qubit, stream, 0).  The angle of a step uses counter
 *     (step, 0, 1, 0) and Box-Muller on the high 32 bits of output words 0
 *     and 1, u = (h + 0.5) 2^-32.  The flips of qubit q use counter
 *     (step, q, 2, 0): word 0 decides the bit flip, word 1 the phase flip;
 *     each fires when its high 32 bits are below floor(p 2^32);
 *   - step = number of circuit gates applied to the state since create or
 *     reset; flips and inverse (echo) gates do not count.
 *
 * Threading: one state must not be used from two host threads at once.
 * Different states may be used concurrently.  Error messages are per thread.
 *
 * Return values: QSIM_OK (0) or a negative status.  On QSIM_EINVAL nothing
 * has been written or launched.  No function aborts or throws: host memory
 * exhaustion inside a call is reported as QSIM_ENOMEM, any other internal
 * failure as QSIM_EDEVICE, with the message in qsim_last_error().
 */
#ifndef QSIM_INCLUDE_QSIM_API_H_
#define QSIM_INCLUDE_QSIM_API_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QSIM_OK 0
#define QSIM_EINVAL (-1)   /* invalid argument: qubit, arity, sizes, dtype */
#define QSIM_ENOMEM (-2)   /* device or pinned host memory does not fit */
#define QSIM_EDEVICE (-3)  /* a HIP runtime call failed */
#define QSIM_ERANGE (-4)   /* index range out of bounds */

#define QSIM_MAX_QUBITS 34

typedef struct qsim_state qsim_state; /* opaque, owned by the library */

typedef enum { QSIM_C64 = 0, QSIM_C128 = 1 } qsim_dtype;

/* Gate kinds.  Arity: H, RZ, X, Z act on `target` alone; CNOT and CPHASE
 * add ctrl0; TOFFOLI adds ctrl0 and ctrl1.  Unused controls are -1.
 * CPHASE(theta) is the conditional phase rotation of the quantum FFT
 * (Sec. 2.2): diag(1, e^{i theta}) on the target where ctrl0 is 1, i.e. the
 * amplitudes with both bits set gain e^{i theta}; an angle error makes it
 * CPHASE(theta + eps), as Rz(theta) becomes Rz(theta + eps). */
typedef enum {
    QSIM_H = 0,
    QSIM_RZ = 1,
    QSIM_X = 2,
    QSIM_CNOT = 3,
    QSIM_TOFFOLI = 4,
    QSIM_Z = 5,
    QSIM_CPHASE = 6
} qsim_kind;

/* One gate, 24 bytes.  theta is the Rz or CPHASE angle in radians (ignored
 * otherwise). */
typedef struct {
    uint32_t kind;
    int32_t target;
    int32_t ctrl0;
    int32_t ctrl1;
    double theta;
} qsim_gate;

/* Error model (Sec. 1.4, 2.0, 3.4).  sigma >= 0 radians; p in [0, 1]. */
typedef struct {
    double sigma;
    double p_bitflip;
    double p_phaseflip;
    uint64_t seed;
    uint64_t trial;
} qsim_error_model;

/* Creation options; a zeroed struct (or NULL) gives the defaults. */
typedef struct {
    int device;          /* HIP device ordinal (default 0) */
    void *hip_stream;    /* hipStream_t the state's work goes to; NULL: the
                            library creates one at default priority */
    void *ext_buffer;    /* device memory that holds the state, borrowed (never
                            freed by the library); NULL: the library allocates */
    size_t ext_bytes;    /* size of ext_buffer, >= 2^M * element size */
    int renorm_period;   /* rescale to unit norm after every R gates.
                            0: default (64 for QSIM_C64, never for QSIM_C128);
                            -1: never */
    int exec_mode;       /* 0: fused passes, commuting operations reordered so
                            that a pass carries more of them (default);
                            1: one pass per operation, in stream order;
                            2: fused passes over runs of the stream, in order */
    int tile_bits;       /* qubits per fused tile, 9..14; 0: default (13 for
                            QSIM_C64, 12 for QSIM_C128) */
    int low_bits;        /* low qubits always in a fused tile, 1..tile_bits-1;
                            0: default (4) */
    int group_bits;      /* qubits per register quantum, 3..5, with
                            6 <= tile_bits - group_bits <= 9; 0: default (4) */
    int lazy_qubits;     /* 0 (default) or 1: a qubit no operation has yet
                            spread over both values ("untouched": after
                            create or reset it holds one definite value) costs
                            nothing, since the amplitudes with its other value
                            are zero; fused passes skip them (the flat form of
                            the dynamically allocated state vector, Sec. 3.2).
                            -1: every pass streams the whole register.  The
                            per-operation path (exec_mode 1) never skips. */
    int remap_qubits;    /* 0 (default): on complex64 registers of 31 qubits or more, a
                            call whose operations use some of the top 6
                            qubits far more often than the low qubits just
                            above the always-tiled ones first exchanges up to
                            4 such pairs (exact swaps), runs on the exchanged
                            positions and exchanges them back at its end, so
                            that its tiles read nearby memory (the one-GPU
                            form of the reorganisation of Sec. 3.1, 3.3 and
                            Fig. 8); the layout between calls never changes.
                            1: the same on every register size whenever a
                            top qubit is used more than twice as often as
                            its partner.  -1: never. */
} qsim_options;

/* Per-state counters of the work launched since the last reset of the
 * counters (qsim_profile).  Times come from HIP events around each launch and
 * are only filled while profiling is on. */
typedef struct {
    uint64_t gates;          /* circuit gates applied */
    uint64_t flips;          /* injected flips applied */
    uint64_t passes;         /* state-update kernel launches (plain + fused) */
    uint64_t fused_passes;   /* of which fused tile passes */
    uint64_t renorms;        /* renormalisations */
    double pass_ms;          /* summed duration of the state-update launches */
    double pass_bytes;       /* algorithmic HBM bytes of those launches */
    double fused_ms;         /* summed duration of the fused launches */
    double fused_bytes;      /* algorithmic HBM bytes of the fused launches */
    double other_ms;         /* reductions, init, scaling */
    double fused_flops;      /* algorithmic real flops of the fused launches
                                (see qsim_pass_info.flops) */
    uint64_t remaps;         /* qubit pairs exchanged by remaps (each pair: one
                                exchange at a call's start, one at its end) */
} qsim_stats;

/* Allocate a register of num_qubits (1..QSIM_MAX_QUBITS) in `dtype` and set it
 * to |0...0> (Fig. 1(a)).  Errors start disarmed.  EINVAL for bad arguments,
 * ENOMEM if 2^M elements do not fit (or ext_bytes is too small: EINVAL). */
int qsim_create(int num_qubits, int dtype, const qsim_options *opt, qsim_state **out);

/* Wait for the state's work, release its memory (unless borrowed) and its
 * stream (unless borrowed).  NULL is accepted. */
int qsim_destroy(qsim_state *s);

/* Set the state to the basis state |basis_index> (Sec. 1.2, Fig. 1(a): one
 * amplitude 1, every other 0) and the step counter to 0; the armed error
 * model stays armed.  ERANGE if basis_index >= 2^M.  The register memory is
 * written by the next call that touches the state: the first fused pass of
 * an apply call builds the basis state instead of loading the register, and
 * every readout, qsim_set_amplitudes, qsim_synchronize and a qsim_info that
 * asks for the device pointer write it first (on the state's stream).  Code
 * that reads the memory directly calls qsim_synchronize first. */
int qsim_reset(qsim_state *s, uint64_t basis_index);

/* Apply gates[0..n_gates) in order (Sec. 2.1), each followed by the armed
 * error model's draws for its step.  Asynchronous on the state's stream; the
 * gate array is read before returning.  EINVAL (nothing applied) if any gate
 * has a bad kind, arity, qubit, repeated qubit or a non-finite theta. */
int qsim_apply_circuit(qsim_state *s, const qsim_gate *gates, size_t n_gates);

/* Apply the exact inverse of gates[0..n_gates): the gates in reverse order,
 * Rz(t) as Rz(-t), CPHASE(t) as CPHASE(-t), the others as themselves, with
 * no errors and without advancing the step counter.  After a noisy run of a
 * circuit, this leaves
 * <0|U_ideal^dagger U_noisy|0> in amplitude 0 (the echo form of the fidelity,
 * for registers too large to hold two states). */
int qsim_apply_inverse(qsim_state *s, const qsim_gate *gates, size_t n_gates);

/* Arm the error model for later apply_circuit calls (copied), or disarm it
 * with NULL.  Errors are injected at every step (Sec. 1.0): the angle of each
 * gate deviates by eps = sigma * z (Sec. 1.4 and 2.0: operational errors are
 * deviations of the rotation angles), and after each gate every qubit takes a
 * bit flip and then a phase flip with probabilities p_bitflip and
 * p_phaseflip (Sec. 3.4 and EQ 8: two extra transformations after every
 * operation model decoherence).  Arming draws nothing: the draws of a gate
 * depend only on (seed, trial, step), so a circuit split over several
 * apply_circuit calls gets the same errors.  With sigma = 0 and both p = 0
 * the run is bit-identical to a run with errors disarmed.  EINVAL for
 * negative/non-finite sigma or p outside [0, 1]. */
int qsim_inject_errors(qsim_state *s, const qsim_error_model *em);

/* F = |<a|b>|^2 / (<a|a> <b|b>), accumulated in FP64 on the device with a
 * fixed reduction order (deterministic).  The paper tracks how errors
 * accumulate (Sec. 1.0) but defines no fidelity; this normalised squared
 * overlap is the library's choice: it equals |<a|b>|^2 for unit vectors and
 * ignores norm drift and global phase.  a and b must have the same M; their
 * dtypes may differ.  Synchronises both states' streams. */
int qsim_fidelity(const qsim_state *a, const qsim_state *b, double *out_F);

/* out = {re <a|b>, im <a|b>, <a|a>, <b|b>} in FP64 (same rules as above). */
int qsim_overlap(const qsim_state *a, const qsim_state *b, double out[4]);

/* The overlap of qsim_overlap for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the two registers are caller-owned device memory, not states.
 * a and b hold 2^num_qubits interleaved (re, im) amplitudes of dtype_a and
 * dtype_b (QSIM_C64 or QSIM_C128), 16-byte aligned, on `device`; they are
 * only read.  The work is queued on hip_stream (NULL: the null stream) and
 * the call waits for it; out (host) receives {re <a|b>, im <a|b>, <a|a>,
 * <b|b>} in FP64, bit-identical to qsim_overlap on the same amplitudes (same
 * kernels, same fixed reduction order).  No memory is allocated, host or
 * device: the reduction's per-block partials and results sit in a static
 * device array of 32.1 KiB per device (4 x 1024 partials + results, enough
 * for every num_qubits in 1..QSIM_MAX_QUBITS), held until the process ends.
 * Calls on one device share that array: they are serialised inside the
 * process, and calls on one device from several processes must not overlap.
 * EINVAL for num_qubits outside [1, QSIM_MAX_QUBITS], a bad dtype or device,
 * a NULL, misaligned or non-device pointer, or an allocation smaller than the
 * register; EDEVICE if a HIP call fails. */
int qsim_overlap_noalloc(const void *a, int dtype_a, const void *b, int dtype_b, int num_qubits,
                         int device, void *hip_stream, double out[4]);

/* Squared norm <s|s> in FP64. */
int qsim_norm(const qsim_state *s, double *out);

/* Probabilities |a_i|^2 (Sec. 1.2) in FP64 into host memory `out`.  With
 * qubit_mask covering m qubits, out_len must be 2^m; out[k] sums every index
 * whose masked bits, in ascending qubit order, spell k.  qubit_mask = 2^M - 1
 * gives the full distribution.  EINVAL for mask bits >= M or a wrong
 * out_len. */
int qsim_probs(const qsim_state *s, uint64_t qubit_mask, double *out, size_t out_len);

/* Copy amplitudes [offset, offset + count) to host memory as interleaved
 * FP64 re/im pairs (2 * count doubles).  ERANGE if out of bounds. */
int qsim_get_amplitudes(const qsim_state *s, uint64_t offset, uint64_t count, double *out);

/* Overwrite amplitudes [offset, offset + count) from interleaved FP64 host
 * memory (rounded to the state's dtype).  Does not touch the step counter. */
int qsim_set_amplitudes(qsim_state *s, uint64_t offset, uint64_t count, const double *in);

/* Batched Monte Carlo (Sec. 1.0: errors injected at each step, their
 * accumulation tracked; Sec. 1.4, 2.0 and 3.4 for the error model, as in
 * qsim_inject_errors): the error-free run of gates[0..n) from |0...0> is the
 * reference; trial t (0 <= t < n_trials) runs the same circuit from |0...0>
 * with error model `base` keyed by trial base->trial + t, and out_F[t] is its
 * fidelity against the reference (host memory, n_trials doubles; the same
 * value qsim_fidelity gives for two registers run that way).  All trials
 * run in one persistent launch, one register per workgroup, which needs the
 * register to fit the workgroup's LDS (num_qubits <= 14 for QSIM_C64,
 * <= 13 for QSIM_C128); EINVAL beyond that, and for CPHASE gates (the
 * trial kernels take the gate set H, Rz, X, CNOT, Toffoli, Z).  Synchronous.
 * Runs on `device`
 * 0 unless QSIM_DEVICE is set in the environment.  The kernel variant (one
 * LDS sweep per gate, or the register held in registers with 4 or 5 group
 * qubits) is picked by timing each on one round of trials, once per
 * (register size, dtype, gate count, error kinds) and process, optionally
 * cached in the file QSIM_TUNE_CACHE names; QSIM_TRIAL_VARIANT = 0..3 forces
 * one where it can run.  Device resources are kept per device between calls
 * and held until the process ends: a stream, the error-free register (of the
 * last shape run) and buffers grown to the largest call (about 64 bytes per
 * gate and trial of a batch, at most ~256 MiB); calls on one device are
 * serialised. */
int qsim_run_trials(const qsim_gate *gates, size_t n, int num_qubits, int dtype,
                    const qsim_error_model *base, uint64_t n_trials, double *out_F);

/* Host-only dry run of the register-group schedule qsim_run_trials uses when
 * each thread holds group_bits (4 or 5) qubits of a trial's register: the
 * circuit is cut into groups of consecutive gates whose non-diagonal targets
 * fall on at most group_bits qubits (Sec. 2.1: a gate only mixes the pairs of
 * its target, so such a run is a fixed pattern of register pairs) and that
 * hold at most 32 uncontrolled Hadamards (the kernel applies their real scale
 * at the group's end).  Writes min(cap, groups) records of 4 words to out:
 * first gate, gate count, mask of the group's qubits, uncontrolled Hadamards
 * in the group; and the group count to *n_groups (either may be NULL).  No
 * device is used.  EINVAL for a bad gate, group_bits, or a register the
 * register-group kernels cannot hold (num_qubits - group_bits outside
 * [6, 10]). */
int qsim_trial_plan(const qsim_gate *gates, size_t n, int num_qubits, int group_bits,
                    uint32_t *out, size_t cap, size_t *n_groups);

/* One pass of a fused schedule (qsim_plan). */
typedef struct {
    uint32_t fused;      /* 1: tile pass (one HBM read + write for all its
                            operations); 0: one whole-vector pass per operation */
    uint32_t first_op;   /* index into the execution order (see op_order) */
    uint32_t n_ops;
    uint32_t n_groups;   /* register groups inside a tile pass */
    uint32_t norm_after; /* 1: a renormalisation follows this pass */
    uint32_t span_qubits;/* qubits the pass's launch spans: it reads and writes
                            2^span_qubits amplitudes (M unless untouched
                            qubits are skipped, see lazy_qubits) */
    uint64_t tile_mask;  /* qubits spanned by the tile of a fused pass */
    double flops;        /* algorithmic real flops: per operation, those of its
                            2x2 on each amplitude it updates (6 for a real 2x2,
                            a perturbed X or a diagonal phase; 10 for a real
                            2x2 plus i*w on the diagonal; 0 for a swap or a
                            sign flip) on the 2^-c of the 2^span_qubits
                            amplitudes that satisfy its c controls */
    uint64_t tiles;      /* tiles (workgroup tasks) of a fused pass, else 0 */
} qsim_pass_info;

/* Host-only dry run of qsim_apply_circuit for a register created with
 * (num_qubits, dtype, opt), i.e. starting from |0...0> with every qubit
 * untouched: lower the gates (drawing the errors of em, NULL = none, starting
 * at step0) into the operation stream (each gate, then its step's flips),
 * rewrite it against the untouched qubits (lazy registers), fix the
 * execution order and partition it into passes the way the library would
 * (Sec. 2.1: a gate only mixes the amplitude pairs of its target, so gates
 * whose targets lie in one set of qubits can be applied tile by tile in one
 * pass over the state; commuting operations may be reordered for that), and
 * check every pass's kernel arguments for consistency.  Writes min(out_cap,
 * passes) entries of out, and min(order_cap, operations) entries of op_order
 * (op_order[i] = index, in the rewritten stream, of the i-th operation
 * executed; without lazy qubits the rewritten stream is the lowered one);
 * either may be NULL.  Also the pass and operation counts.  No device is
 * used.  EINVAL for bad arguments; EDEVICE if a pass fails its own
 * consistency check (a library bug). */
int qsim_plan(int num_qubits, int dtype, const qsim_options *opt, const qsim_gate *gates,
              size_t n_gates, const qsim_error_model *em, uint64_t step0, qsim_pass_info *out,
              size_t out_cap, size_t *n_passes, size_t *n_ops, uint32_t *op_order,
              size_t order_cap);

/* ---------------------------------------------------------------- serving
 *
 * A request is one simulation: the error-free run and one noisy run of a
 * circuit on a fresh register, scored by their fidelity (Sec. 1.0: errors
 * injected at each step, their accumulation tracked).  qsim_serve runs a
 * stream of requests with continuous batching: requests arrive over time,
 * each is admitted as soon as a slot (a HIP stream) and room in the HBM
 * budget for its two registers are free, its work is queued on its slot at
 * once so that admitted requests run concurrently on the device, and its
 * registers stay resident until its fidelity has come back, when slot and
 * memory go to the next waiting request.  All device memory is taken once at
 * the start; the loop itself never allocates or frees.  Results do not
 * depend on the mix: a request computes the same fidelity alone and among
 * others (same kernels, fixed reduction order). */
typedef struct {
    int num_qubits;
    int dtype;
    const qsim_gate *gates;     /* borrowed for the call */
    size_t n_gates;
    qsim_error_model errors;    /* the noisy run's error model */
    double arrival_s;           /* arrival, seconds after the call starts (>= 0) */
} qsim_request;

typedef struct {
    double fidelity;            /* F(error-free, noisy) */
    double admit_s;             /* admission time, seconds after the call starts */
    double done_s;              /* time its result was seen complete */
    int status;                 /* QSIM_OK, or QSIM_ENOMEM if its registers can never
                                   fit the budget, or the error that stopped it */
    int slot;                   /* slot it ran on (-1 if never admitted) */
} qsim_result;

typedef struct {
    int device;
    int max_slots;              /* concurrent requests, 1..64; 0: 8 */
    size_t hbm_budget;          /* bytes for resident registers; 0: the smaller of
                                   64 GiB and 80% of the free device memory */
    int strict_fifo;            /* 1: admit in arrival order only; 0: a request
                                   that fits may pass a waiting one that does not */
    int max_heavy;              /* heavy requests (see heavy_bytes) in flight at
                                   once, >= 0; 0: 1.  One register pass of a heavy
                                   request already streams HBM at full rate, so a
                                   second one would only share the bandwidth and
                                   stretch both; light requests fill the other
                                   slots (with strict_fifo a heavy request that
                                   must wait holds back everything behind it) */
    size_t heavy_bytes;         /* footprint (both registers) from which a request
                                   is heavy; 0: 256 MiB, i.e. registers that no
                                   longer fit the GPU's 256 MB last-level cache */
} qsim_serve_options;

/* Serve reqs[0..n) and write out[0..n) (same order).  Blocks until every
 * request has finished.  EINVAL (nothing run) for a malformed request (bad
 * M, dtype, gate or error model, negative or non-finite arrival) or options;
 * ENOMEM if the budget cannot be allocated. */
int qsim_serve(const qsim_request *reqs, size_t n, const qsim_serve_options *opt,
               qsim_result *out);

/* ------------------------------------------------------ three-state model
 *
 * The paper's detailed model (Sec. 2.0): each ion of the Cirac-Zoller trap
 * has its two QU-bit levels plus a temporary third level that the
 * controlled-not gate passes through, so M ions take 3^M states (Sec. 3.0)
 * and one laser transformation is 3^(M-1) independent operations on the
 * pairs of states that differ only in the transformed ion's level (Sec.
 * 3.1).  State index i = sum_q d_q 3^q with d_q in {0, 1, 2} the level of
 * ion q.  Gates are lowered to transformations (five for a CNOT, Sec. 2.0);
 * every transformation's angle deviates by eps = sigma z (Sec. 1.4); after
 * each gate the decoherence flips act on the QU-bit levels (a bit flip
 * exchanges levels 0 and 1, a phase flip negates level 1).
 *
 * Transformation on ion `ion` between levels a < b: kind 0 (rotation) is
 * exp(-i theta/2 (e^{i phi}|a><b| + e^{-i phi}|b><a|)), kind 1 (phase)
 * multiplies levels a and b by e^{-i theta/2} and e^{+i theta/2}; the third
 * level is untouched.  With cond_ion >= 0 it acts only on the states whose
 * ion cond_ion is in level cond_level.  Lowering (the paper gives no pulse
 * sequences; this is the library's reading): X = rot(01, pi, 0); H =
 * rot(01, pi/2, -pi/2), rot(01, pi, 0); Rz(t) = phase(01, t); Z =
 * phase(01, pi); CNOT(c, x) = rot_x(01, pi/2, pi/2), rot_c(12, pi, 0),
 * [c in 2] rot_x(12, 2 pi, 0), rot_c(12, pi, pi), rot_x(01, pi/2, -pi/2)
 * (exactly CNOT on the QU-bit levels); CPHASE(t) = phase_c(t/2),
 * phase_x(t/2), CNOT, phase_x(-t/2), CNOT; Toffoli = the six-CNOT circuit
 * with H on the target and phases of +-pi/4 (both up to a global phase).
 * The angle error of a gate's k-th transformation uses Philox4x64-10 at
 * counter (step, k, 3, 0), Box-Muller on the high halves of words 0 and 1;
 * the flips use the two-state model's draws. */
typedef struct qsim3_state qsim3_state; /* opaque, owned by the library */

typedef struct {
    uint32_t kind;       /* 0 rotation, 1 phase */
    int32_t ion;
    int32_t a, b;        /* levels, 0 <= a < b <= 2 */
    int32_t cond_ion;    /* -1: unconditional */
    int32_t cond_level;
    double theta, phi;
} qsim3_pulse;

/* Register of num_ions (1..20) ions in dtype, set to |0...0>; the options
 * used are device, hip_stream and exec_mode.  On registers larger than one
 * LDS tile, transformations are applied as fused passes over tiles of ions:
 * exec_mode 0 (default) lets a pass take a transformation from further down
 * the stream when it commutes with every earlier one left behind (different
 * ions, neither acting on the other's condition ion), exec_mode 2 takes runs
 * of the stream in order; exec_mode 1 launches once per transformation.
 * EINVAL / ENOMEM as qsim_create. */
int qsim3_create(int num_ions, int dtype, const qsim_options *opt, qsim3_state **out);
int qsim3_destroy(qsim3_state *s);
/* Basis state |basis_index> (0 <= basis_index < 3^M), step counter 0. */
int qsim3_reset(qsim3_state *s, uint64_t basis_index);
/* Arm (copied) or disarm (NULL) the error model, as qsim_inject_errors. */
int qsim3_inject_errors(qsim3_state *s, const qsim_error_model *em);
/* Lower gates[0..n) and apply their transformations in order, each gate
 * followed by its step's flips (Sec. 2.0, 3.4).  Asynchronous.  EINVAL for
 * a bad gate (nothing applied). */
int qsim3_apply_circuit(qsim3_state *s, const qsim_gate *gates, size_t n);
/* Apply transformations directly (no angle errors, no step).  EINVAL for a
 * malformed one (nothing applied). */
int qsim3_apply_pulses(qsim3_state *s, const qsim3_pulse *p, size_t n);
/* Host-only: the transformations gates[0..n) lower to; min(cap, count)
 * written to out (may be NULL), the count to *n_pulses. */
int qsim3_lower(const qsim_gate *gates, size_t n, int num_ions, qsim3_pulse *out, size_t cap,
                size_t *n_pulses);
/* {re <a|b>, im <a|b>, <a|a>, <b|b>} in FP64, fixed reduction order. */
int qsim3_overlap(const qsim3_state *a, const qsim3_state *b, double out[4]);
/* F = |<a|b>|^2 / (<a|a><b|b>) (the library's fidelity, see qsim_fidelity). */
int qsim3_fidelity(const qsim3_state *a, const qsim3_state *b, double *out_F);
/* Marginal probabilities of the ions in ion_mask (at most 6): out_len =
 * 3^m, entry k spells their levels in ascending ion order as base-3 digits. */
int qsim3_probs(const qsim3_state *s, uint64_t ion_mask, double *out, size_t out_len);
/* Amplitudes [offset, offset + count) as interleaved FP64 re/im pairs. */
int qsim3_get_amplitudes(const qsim3_state *s, uint64_t offset, uint64_t count, double *out);
int qsim3_synchronize(qsim3_state *s);
/* Register size, dtype, step counter, transformations applied and state
 * kernel launches (fused passes or one per transformation) since create;
 * any pointer may be NULL. */
int qsim3_info(const qsim3_state *s, int *num_ions, int *dtype, uint64_t *step,
               uint64_t *transformations, uint64_t *launches);

/* Wait for all work queued on the state's stream. */
int qsim_synchronize(qsim_state *s);

/* Register size, dtype, step counter, device pointer and byte size. */
int qsim_info(const qsim_state *s, int *num_qubits, int *dtype, uint64_t *step,
              void **device_ptr, size_t *bytes);

/* Qubits touched so far (spread over both values by some operation since
 * create or reset, Sec. 3.2's allocated part of the state): a mask over the
 * M qubits, every bit set when lazy_qubits is off.  The other qubits hold one
 * definite value each; fused passes read and write only the 2^popcount
 * amplitudes of the touched subspace (or a little more, see qsim_pass_info
 * span_qubits). */
int qsim_touched_qubits(const qsim_state *s, uint64_t *mask);

/* Turn per-launch HIP event timing on (1) or off (0); either way the
 * counters are zeroed. */
int qsim_profile(qsim_state *s, int enable);

/* Read the counters (synchronises the stream when profiling is on). */
int qsim_get_stats(qsim_state *s, qsim_stats *out);

/* Message of the last failing call on this thread ("" if none). */
const char *qsim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QSIM_INCLUDE_QSIM_API_H_ */
