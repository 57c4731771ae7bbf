// Host-side launchers of the qsim kernels (each defined next to its kernels).
// All take the element type as a template argument: float (complex64 state)
// or double (complex128 state).  Every launcher enqueues on `st` and returns
// the hipError_t of the launch.
#pragma once

#include "common.h"

namespace qsim {

// Raise `fn`'s dynamic-LDS allowance on the current device to at least
// `lds` bytes (allowances only grow; sizes up to 64 KiB need none).
// Thread-safe.
hipError_t kernel_allow_lds(const void *fn, size_t lds);
// Workgroups of `threads` threads and `lds` bytes of dynamic LDS that are
// resident on the current device at once (per-CU occupancy times CUs),
// computed once per (kernel, device, shape); 0 if the kernel cannot run so.
// Thread-safe.
int kernel_resident_blocks(const void *fn, int threads, size_t lds);

// |k>: zero the vector and set amplitude k to 1 (a fill kernel, not a memset,
// so it can sit in captured graphs).
template <typename R>
hipError_t launch_init_basis(cplx<R> *psi, int M, uint64_t k, hipStream_t st);

// One operation over the whole vector (the per-gate path).
template <typename R>
hipError_t launch_plain(const Op &op, cplx<R> *psi, int M, hipStream_t st);

// psi *= *scale (a device scalar).
template <typename R>
hipError_t launch_scale(cplx<R> *psi, int M, const double *scale, hipStream_t st);

// One fused tile pass: G group bits per register quantum, 2^(k-G) threads
// (64..512), so k - G must lie in [6, 9].  LDS (2^k elements) is only used
// when the pass has more than one group.
template <typename R>
hipError_t launch_tile(const TileArgs<R> &args, int G, hipStream_t st);
size_t tile_lds_bytes(int k, int elem_bytes);

// Deterministic FP64 reductions.  partial must hold 4 * kReduceBlocks
// doubles; out receives 4 doubles {re<a|b>, im<a|b>, <a|a>, <b|b>}.
constexpr int kReduceBlocks = 1024;
template <typename Ra, typename Rb>
hipError_t launch_overlap(const cplx<Ra> *a, const cplx<Rb> *b, int M, double *partial,
                          double *out, hipStream_t st);
// out[0] = <a|a>; partial as above.
template <typename R>
hipError_t launch_norm(const cplx<R> *a, int M, double *partial, double *out, hipStream_t st);
// Sum n per-tile partial norms in a fixed order; out[0] = sum, out[1] =
// 1/sqrt(sum).  Long sums take a first stage over chunks whose sums land in
// partial (kReduceBlocks doubles; may be NULL for n <= 16 * 256).
hipError_t launch_finish_norm(const double *tile_norms, uint64_t n, double *partial, double *out,
                              hipStream_t st);

// Probabilities.  full: out[i] = |a_i|^2.  Marginal: chunk partials, then
// out[k] summed in chunk order; `partial` holds (2^M / chunk) doubles.
template <typename R>
hipError_t launch_probs_full(const cplx<R> *psi, int M, double *out, hipStream_t st);
template <typename R>
hipError_t launch_probs_marginal(const cplx<R> *psi, int M, uint64_t mask, double *partial,
                                 uint64_t partial_len, double *out, hipStream_t st);
uint64_t probs_marginal_partial_len(int M, uint64_t mask);

// Element conversion between the state and interleaved FP64 staging.
template <typename R>
hipError_t launch_to_f64(const cplx<R> *psi, uint64_t count, double *out, hipStream_t st);
template <typename R>
hipError_t launch_from_f64(const double *in, uint64_t count, cplx<R> *psi, hipStream_t st);

// Batched Monte Carlo trials (one register per workgroup, persistent grid).
struct TrialGate {
    uint32_t kind;     // qsim_kind
    uint32_t target;
    uint32_t cmask;    // control qubits
    uint32_t pad;
    double theta;
    double pad2;
};
struct TrialLaunch {
    const TrialGate *gates;   // device array of the circuit's gates
    uint32_t ngates;
    uint32_t M;
    double sigma, p_bit, p_phase;
    uint64_t seed, trial0, n_trials;
    const void *ideal;        // device error-free register (same dtype)
    double *out_F;            // device, n_trials
    int variant;              // schedule chosen by the autotuner
    int grid;                 // persistent workgroup count
    // register-group variants: device array of nchunks chunk records
    // {first gate, gates, first group, groups} (none at present), ngroups
    // group records {first gate, gates, qubit word, 0}, then the qubit word
    // of each gate's group
    const uint32_t *sched;
    uint32_t nchunks, ngroups;
    // ...and their per-trial gates, built by a preparation kernel for
    // prep_batch trials at a time: prep_ops holds prep_batch * ngates records
    // of trial_gate_op_bytes each, prep_X prep_batch masks
    void *prep_ops;
    uint32_t *prep_X;
    uint64_t prep_batch;
};
size_t trial_gate_op_bytes(int elem_bytes);
// Register groups of the register-group variants hold at most this many
// uncontrolled Hadamards (gates the preparation kernel may turn into
// butterflies whose scale the group restores at its end).
constexpr uint32_t kMaxGroupButterflies = 32;
// LDS of the sweep variants (register plus a chunk of built gates).
size_t trial_lds_bytes(int M, int elem_bytes);
// Group qubits of a register-group variant (0 for the LDS-sweep variants).
int trial_group_bits(int variant);
template <typename R>
hipError_t launch_trials(const TrialLaunch &L, hipStream_t st);
int trial_variants();
const char *trial_variant_name(int v);
// Persistent workgroups that fit the chip at once (0 if the variant cannot
// run at this size).
int trial_grid(int variant, int M, int elem_bytes);

}  // namespace qsim
