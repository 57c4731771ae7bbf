// Batched Monte Carlo error trials for gfx950: one persistent launch, one
// register per workgroup, the register held in LDS.
//
// Each trial runs the whole circuit from |0...0> with its own error stream
// (Philox4x64-10 keyed by (seed, trial), the same draws the per-register path
// makes on the host), then scores the result against the shared error-free
// state by its FP64 fidelity.  The gate matrices of a trial are built in
// FP64 on the device, a chunk of gates at a time, from the same formulas the
// host lowering uses.
//
// Bit flips are not applied by moving data.  A workgroup keeps the trial's
// X mask: the true register is psi(i) = s(i xor X) for the stored s.  A gate
// U acting on psi is the gate X U X acting on s: on a target in X the 2x2
// swaps its rows and columns, and a control in X asks for 0 instead of 1.  A
// phase flip Z_q of psi is Z_q of s times -1 when q is in X.  The fidelity
// reads s at i xor X.  All of this is exact, so the result equals the
// flip-by-flip evolution.
#include <algorithm>

#include "launch.h"

namespace qsim {
namespace {

constexpr int kChunk = 64;  // gates whose matrices are built at a time

// A trial gate as the kernel applies it to the stored register.
template <typename R>
struct TrialOp {
    cplx<R> u[4];        // u00 u01 u10 u11; diagonal: u[0] = d0, u[3] = d1
    uint32_t type;       // OpType
    uint32_t target;
    uint32_t cmask;      // control qubits
    uint32_t cval;       // values the controls must have in the stored register
    uint32_t neg_val;    // kOpNeg: the target value whose amplitudes change sign
    uint32_t zmask;      // phase flips after the gate, on stored-register qubits
    uint32_t form;       // kOpMat: 0 real 2x2; 1 real off-diagonal, complex
                         // diagonal; 2 the same with a zero real diagonal;
                         // 3 anything else
    uint32_t pad;
};

// Matrix of one gate with angle error eps, as the host lowering builds it:
// eps == 0 gives the textbook gate; otherwise i R_n(pi + eps) about the gate's
// own axis, and Rz(t + eps).
__device__ void gate_matrix(uint32_t kind, double theta, double eps, uint32_t &type, double (&u)[8])
{
    const double h = 0.70710678118654752440084436210485;
    const double c = cos(0.5 * eps), s = sin(0.5 * eps);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        u[i] = 0.0;
    switch (kind) {
    case 0:  // H
        type = kOpMat;
        if (eps == 0.0) {
            u[0] = h; u[2] = h; u[4] = h; u[6] = -h;
        } else {
            const double ch = c * h;
            u[0] = ch; u[1] = -s; u[2] = ch; u[4] = ch; u[6] = -ch; u[7] = -s;
        }
        break;
    case 1: {  // Rz
        type = kOpDiag;
        const double phi = theta + eps;
        const double cp = cos(0.5 * phi), sp = sin(0.5 * phi);
        u[0] = cp; u[1] = -sp; u[6] = cp; u[7] = sp;
        break;
    }
    case 2: case 3: case 4:  // X, CNOT, Toffoli
        if (eps == 0.0) {
            type = kOpSwap;
            u[2] = 1.0; u[4] = 1.0;
        } else {
            type = kOpMat;
            u[1] = -s; u[2] = c; u[4] = c; u[7] = -s;
        }
        break;
    default:  // Z
        if (eps == 0.0) {
            type = kOpNeg;
            u[0] = 1.0; u[6] = -1.0;
        } else {
            type = kOpDiag;
            u[0] = c; u[1] = -s; u[6] = -c; u[7] = -s;
        }
        break;
    }
}

// A trial gate as the register-group variants read it from global memory
// (built by the preparation kernel for the group the gate sits in):
//   meta  = type | form << 4 | neg_val << 8 | P << 12 | target << 16, P =
//           the target's position among the group qubits, 15 when it is not
//           one; forms 0-3 as in TrialOp, and for an uncontrolled Hadamard 4
//           = the butterfly (a + b, a - b) and 5 = (b - a, a + b), each plus
//           i t on the diagonal with t = u[0].im;
//   scale = the real factor the butterfly forms leave out (the Hadamard's
//           h cos(eps/2)), 1 for every other form: the group multiplies its
//           quantum by the product of its gates' scales at its end, so the
//           register keeps its true norm;
//   regs  = rm | rv << 8 | rz << 16: controls on group qubits and the values
//           they need, and phase flips on group qubits, over the register
//           index;
//   lm, lv: controls on the other qubits and their values, over the thread's
//           base index; zmask: all phase flips after the gate.
// A diagonal is kept as diag(1, q) with u[3] = q: its d0 has modulus one, so
// dropping it changes the trial's state by a global phase only, which the
// fidelity does not see.
template <typename R>
struct TrialGateOp {
    cplx<R> u[4];
    R scale;
    uint32_t meta;
    uint32_t regs;
    uint32_t lm;
    uint32_t lv;
    uint32_t zmask;
    uint32_t pad[sizeof(R) == 4 ? 2 : 1];
};
static_assert(sizeof(TrialGateOp<float>) == 64 && sizeof(TrialGateOp<double>) == 96,
              "trial gate records: 64 / 96 bytes");

// A butterfly leaves out at most this much growth per gate: (B + i t I) with
// |t| <= 1 has operator norm sqrt(2 + t^2) <= sqrt(3), and the host closes a
// register group after kMaxGroupButterflies uncontrolled Hadamards, so a
// quantum grows by at most 3^16 before its group's end restores the scale.
constexpr double kMaxButterflyT = 1.0;

// Build the trial's operations for gates [c0, c0 + cn) of the circuit in
// LDS (ops), drawing the chunk's flips (one Philox block per (step, qubit))
// and tracking the X mask of bit flips across the chunk; xmask_at[g] is the
// mask before gate g of the chunk, xmask_at[cn] the mask after it.  Every
// thread of the workgroup calls it; it begins and ends with a barrier.
template <typename R, int T>
__device__ void build_chunk(const TrialGate *gates, uint32_t c0, uint32_t cn, uint32_t M,
                            double sigma, uint64_t thr_b, uint64_t thr_p, bool draws_flip,
                            uint64_t seed, uint64_t trial, uint32_t X, TrialOp<R> *ops,
                            uint32_t *bmask, uint32_t *zmask, uint32_t *xmask_at)
{
    const uint32_t tid = threadIdx.x;
    __syncthreads();
    for (uint32_t i = tid; i < cn; i += T) {
        bmask[i] = 0;
        zmask[i] = 0;
    }
    __syncthreads();
    if (draws_flip) {
        for (uint32_t i = tid; i < cn * M; i += T) {
            const uint32_t g = i / M, q = i % M;
            const u64x4 r = philox4x64_10(c0 + g, q, kStreamFlip, 0, seed, trial);
            if ((r.w[0] >> 32) < thr_b)
                atomicOr(&bmask[g], 1u << q);
            if ((r.w[1] >> 32) < thr_p)
                atomicOr(&zmask[g], 1u << q);
        }
    }
    __syncthreads();
    // X mask before each gate of the chunk (a serial scan)
    if (tid == 0) {
        uint32_t x = X;
        for (uint32_t g = 0; g < cn; ++g) {
            xmask_at[g] = x;
            x ^= bmask[g];
        }
        xmask_at[cn] = x;
    }
    __syncthreads();
    for (uint32_t g = tid; g < cn; g += T) {
        const TrialGate gd = gates[c0 + g];
        const double eps = sigma > 0.0 ? sigma * step_gaussian(seed, trial, c0 + g) : 0.0;
        uint32_t type;
        double u[8];
        gate_matrix(gd.kind, gd.theta, eps, type, u);
        const uint32_t xg = xmask_at[g];
        const bool flipped = (xg >> gd.target) & 1u;
        TrialOp<R> op;
        if (flipped) {
            // X U X: swap rows and columns
            op.u[0] = {(R)u[6], (R)u[7]};
            op.u[1] = {(R)u[4], (R)u[5]};
            op.u[2] = {(R)u[2], (R)u[3]};
            op.u[3] = {(R)u[0], (R)u[1]};
        } else {
            op.u[0] = {(R)u[0], (R)u[1]};
            op.u[1] = {(R)u[2], (R)u[3]};
            op.u[2] = {(R)u[4], (R)u[5]};
            op.u[3] = {(R)u[6], (R)u[7]};
        }
        op.type = type;
        op.target = gd.target;
        op.cmask = gd.cmask;
        op.cval = gd.cmask & ~xg;
        op.neg_val = flipped ? 0u : 1u;
        // phase flips follow this step's bit flips; Z_q on the true register
        // is Z_q on the stored one up to a global sign
        op.zmask = zmask[g];
        const bool real_off = u[3] == 0.0 && u[5] == 0.0;
        const bool real_diag = u[1] == 0.0 && u[7] == 0.0;
        const bool zero_diag = u[0] == 0.0 && u[6] == 0.0;
        op.form = !real_off ? 3u : real_diag ? 0u : zero_diag ? 2u : 1u;
        op.pad = 0;
        ops[g] = op;
    }
    __syncthreads();
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Variant 0: every operation is one sweep over the register in LDS (pairs of
// the target for matrices and swaps, single amplitudes for diagonals).
template <typename R, int T>
__global__ void __launch_bounds__(T) k_trials(const TrialGate *gates, uint32_t n, uint32_t M,
                                              double sigma, double p_bit, double p_phase,
                                              uint64_t seed, uint64_t trial0, uint64_t n_trials,
                                              const cplx<R> *ideal, double *out_F)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const uint32_t N = 1u << M;
    cplx<R> *st = reinterpret_cast<cplx<R> *>(lds);
    TrialOp<R> *ops = reinterpret_cast<TrialOp<R> *>(lds + (size_t)N * sizeof(cplx<R>));
    __shared__ uint32_t bmask[kChunk], zmask[kChunk], xmask_at[kChunk + 1];
    __shared__ double red[4][T / 64];
    const uint32_t tid = threadIdx.x;
    const bool draws_flip = p_bit > 0.0 || p_phase > 0.0;
    const uint64_t thr_b = flip_threshold(p_bit), thr_p = flip_threshold(p_phase);

    for (uint64_t t = blockIdx.x; t < n_trials; t += gridDim.x) {
        const uint64_t trial = trial0 + t;
        for (uint32_t i = tid; i < N; i += T)
            st[i] = {R(i == 0 ? 1 : 0), R(0)};
        uint32_t X = 0;  // bit flips so far (uniform)
        for (uint32_t c0 = 0; c0 < n; c0 += kChunk) {
            const uint32_t cn = min((uint32_t)kChunk, n - c0);
            build_chunk<R, T>(gates, c0, cn, M, sigma, thr_b, thr_p, draws_flip, seed, trial, X,
                              ops, bmask, zmask, xmask_at);
            for (uint32_t g = 0; g < cn; ++g) {
                const TrialOp<R> op = ops[g];
                const uint32_t tb = 1u << op.target;
                if (op.type == kOpMat || op.type == kOpSwap) {
                    for (uint32_t p = tid; p < N / 2; p += T) {
                        const uint32_t i0 = ((p >> op.target) << (op.target + 1)) | (p & (tb - 1));
                        if ((i0 & op.cmask) != op.cval)
                            continue;
                        const uint32_t i1 = i0 | tb;
                        const cplx<R> a = st[i0], b = st[i1];
                        if (op.type == kOpSwap) {
                            st[i0] = b;
                            st[i1] = a;
                        } else {
                            st[i0] = cmad2(op.u[0], a, op.u[1], b);
                            st[i1] = cmad2(op.u[2], a, op.u[3], b);
                        }
                    }
                } else if (op.type == kOpNeg) {
                    for (uint32_t i = tid; i < N; i += T)
                        if ((i & op.cmask) == op.cval && ((i >> op.target) & 1u) == op.neg_val)
                            st[i] = {-st[i].re, -st[i].im};
                } else {
                    for (uint32_t i = tid; i < N; i += T)
                        if ((i & op.cmask) == op.cval)
                            st[i] = cmul(st[i], (i & tb) ? op.u[3] : op.u[0]);
                }
                __syncthreads();
                if (op.zmask != 0) {
                    for (uint32_t i = tid; i < N; i += T)
                        if (__popc(i & op.zmask) & 1u)
                            st[i] = {-st[i].re, -st[i].im};
                    __syncthreads();
                }
            }
            X = xmask_at[cn];
        }
        // fidelity against the error-free register, reading psi(i) = s(i ^ X)
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (uint32_t i = tid; i < N; i += T) {
            const cplx<R> a = ideal[i];
            const cplx<R> b = st[i ^ X];
            const double ar = a.re, ai = a.im, br = b.re, bi = b.im;
            v[0] += ar * br + ai * bi;
            v[1] += ar * bi - ai * br;
            v[2] += ar * ar + ai * ai;
            v[3] += br * br + bi * bi;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            v[c] = wave_sum(v[c]);
        if ((tid & 63) == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                red[c][tid >> 6] = v[c];
        }
        __syncthreads();
        if (tid == 0) {
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            for (int w = 0; w < T / 64; ++w)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    s[c] += red[c][w];
            out_F[t] = (s[0] * s[0] + s[1] * s[1]) / (s[2] * s[3]);
        }
    }
}

// --------------------------------------------------------------------------
// Variants 2 and 3: the register in registers.  Each of the T = 2^(M-G)
// threads holds 2^G amplitudes of the trial's register: register r holds
// the stored amplitude whose index is the thread's base index j0 (its own
// bits on the other qubits) plus the group qubits spelling r.  The host
// splits the circuit into groups of consecutive gates whose non-diagonal
// targets fall on at most G qubits; inside a group every gate is a fixed
// pattern of register pairs (a diagonal on another qubit is a per-thread
// factor), and between groups with different qubits the register is
// re-partitioned through LDS.  Every trial's gates are built beforehand by
// a preparation kernel (below) and read with scalar loads.

// Qubit i of a group word (G <= 5 qubits < 16, four bits each, ascending).
__device__ __forceinline__ uint32_t gq(uint32_t w, int i) { return (w >> (4 * i)) & 15u; }

template <int G>
__device__ __forceinline__ void trial_layout(uint32_t w, uint32_t &j0, uint32_t &gmask)
{
    j0 = threadIdx.x;
    gmask = 0;
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const uint32_t b = gq(w, i);
        gmask |= 1u << b;
        j0 = ((j0 >> b) << (b + 1)) | (j0 & ((1u << b) - 1u));
    }
}

template <int G>
__device__ __forceinline__ uint32_t trial_index(uint32_t j0, uint32_t w, int r)
{
    uint32_t j = j0;
#pragma unroll
    for (int i = 0; i < G; ++i)
        if (r & (1 << i))
            j |= 1u << gq(w, i);
    return j;
}

// A 2x2 on group position P.  F: matrix form (see TrialOp).  C: controls on
// group qubits (mask rm over the register index, required values rv): an
// inactive pair takes the identity instead, chosen per pair by a uniform
// select of the coefficients (form 1 holds the identity), so the register
// pattern stays fixed; a general complex 2x2 (form 3) skips such pairs.
template <typename R, int G, int P, int F, bool C>
__device__ __forceinline__ void trial_pair(const cplx<R> (&u)[4], uint32_t rm, uint32_t rv,
                                           cplx<R> (&x)[1 << G])
{
#pragma unroll
    for (int r = 0; r < (1 << G); ++r) {
        if (r & (1 << P))
            continue;
        const int r1 = r | (1 << P);
        const cplx<R> a = x[r], b = x[r1];
        if (C && F == 3) {
            // a complex off-diagonal: skip the pairs that fail the controls
            if (((uint32_t)r & rm) != rv)
                continue;
            x[r] = cmad2(u[0], a, u[1], b);
            x[r1] = cmad2(u[2], a, u[3], b);
        } else if (C) {
            const bool on = ((uint32_t)r & rm) == rv;
            const R m00 = on ? u[0].re : R(1), m01 = on ? u[1].re : R(0);
            const R m10 = on ? u[2].re : R(0), m11 = on ? u[3].re : R(1);
            const R w0 = on ? u[0].im : R(0), w1 = on ? u[3].im : R(0);
            x[r] = {m00 * a.re + m01 * b.re - w0 * a.im, m00 * a.im + m01 * b.im + w0 * a.re};
            x[r1] = {m10 * a.re + m11 * b.re - w1 * b.im, m10 * a.im + m11 * b.im + w1 * b.re};
        } else if (F == 0) {
            x[r] = {u[0].re * a.re + u[1].re * b.re, u[0].re * a.im + u[1].re * b.im};
            x[r1] = {u[2].re * a.re + u[3].re * b.re, u[2].re * a.im + u[3].re * b.im};
        } else if (F == 1) {
            x[r] = {u[0].re * a.re + u[1].re * b.re - u[0].im * a.im,
                    u[0].re * a.im + u[1].re * b.im + u[0].im * a.re};
            x[r1] = {u[2].re * a.re + u[3].re * b.re - u[3].im * b.im,
                     u[2].re * a.im + u[3].re * b.im + u[3].im * b.re};
        } else if (F == 2) {
            x[r] = {u[1].re * b.re - u[0].im * a.im, u[1].re * b.im + u[0].im * a.re};
            x[r1] = {u[2].re * a.re - u[3].im * b.im, u[2].re * a.im + u[3].im * b.re};
        } else if (F == 4) {
            // a + b, a - b plus i t on the diagonal (no sum shared with F = 5)
            const R t = u[0].im;
            x[r] = {(a.re - t * a.im) + b.re, (a.im + t * a.re) + b.im};
            x[r1] = {(a.re - t * b.im) - b.re, (a.im + t * b.re) - b.im};
        } else if (F == 5) {
            // b - a, a + b plus i t on the diagonal
            const R t = u[0].im;
            x[r] = {(b.re - t * a.im) - a.re, (b.im + t * a.re) - a.im};
            x[r1] = {(b.re - t * b.im) + a.re, (b.im + t * b.re) + a.im};
        } else {
            x[r] = cmad2(u[0], a, u[1], b);
            x[r1] = cmad2(u[2], a, u[3], b);
        }
    }
}

// L: controls on lane qubits; the pair is exchanged only where `act` holds.
template <typename R, int G, int P, bool C, bool L>
__device__ __forceinline__ void trial_swap(uint32_t rm, uint32_t rv, bool act, cplx<R> (&x)[1 << G])
{
#pragma unroll
    for (int r = 0; r < (1 << G); ++r) {
        if ((r & (1 << P)) || (C && ((uint32_t)r & rm) != rv))
            continue;
        const int r1 = r | (1 << P);
        const cplx<R> a = x[r], b = x[r1];
        // selects on the components (a select of whole structs can become a
        // select of addresses, which keeps the quantum out of registers)
        const bool s = !L || act;
        x[r] = {s ? b.re : a.re, s ? b.im : a.im};
        x[r1] = {s ? a.re : b.re, s ? a.im : b.im};
    }
}

// diag(1, q) or a sign flip on group position P (registers whose bit P is
// `on`), under controls on group qubits.  A lane-controlled caller passes
// q = 1 where its controls are not met, and a sign flip as q = -1.
template <typename R, int G, int P>
__device__ __forceinline__ void trial_phase(bool neg, uint32_t on, cplx<R> q, uint32_t rm,
                                            uint32_t rv, cplx<R> (&x)[1 << G])
{
    if (!neg && rm == 0 && on == 1u) {
        // an uncontrolled phase (Rz): half of the registers move
#pragma unroll
        for (int r = 0; r < (1 << G); ++r)
            if ((r >> P) & 1)
                x[r] = cmul(x[r], q);
        return;
    }
    if (neg) {
#pragma unroll
        for (int r = 0; r < (1 << G); ++r)
            if ((((uint32_t)r >> P) & 1u) == on && ((uint32_t)r & rm) == rv)
                x[r] = {-x[r].re, -x[r].im};
        return;
    }
#pragma unroll
    for (int r = 0; r < (1 << G); ++r)
        if ((((uint32_t)r >> P) & 1u) == on && ((uint32_t)r & rm) == rv)
            x[r] = cmul(x[r], q);
}

// One gate with its target on group position P.  L: the gate has controls
// on lane qubits, met where `act` holds; it then runs on every lane with
// coefficients that are the identity where they are not met, so every
// branch here is uniform over the wave.
template <typename R, int G, int P, bool L>
__device__ __forceinline__ void trial_at(uint32_t type, uint32_t form, uint32_t neg_val,
                                         const cplx<R> (&u)[4], uint32_t rm, uint32_t rv,
                                         bool act, cplx<R> (&x)[1 << G])
{
    if (type == kOpSwap) {
        if (rm == 0)
            trial_swap<R, G, P, false, L>(rm, rv, act, x);
        else
            trial_swap<R, G, P, true, L>(rm, rv, act, x);
        return;
    }
    if (type == kOpDiag || type == kOpNeg) {
        const bool neg = type == kOpNeg;
        const uint32_t on = neg ? neg_val : 1u;
        if (!L) {
            trial_phase<R, G, P>(neg, on, u[3], rm, rv, x);
        } else {
            const cplx<R> f = neg ? cplx<R>{R(-1), R(0)} : u[3];
            const cplx<R> q = {act ? f.re : R(1), act ? f.im : R(0)};
            trial_phase<R, G, P>(false, on, q, rm, rv, x);
        }
        return;
    }
    if (L) {
        const cplx<R> v[4] = {{act ? u[0].re : R(1), act ? u[0].im : R(0)},
                              {act ? u[1].re : R(0), act ? u[1].im : R(0)},
                              {act ? u[2].re : R(0), act ? u[2].im : R(0)},
                              {act ? u[3].re : R(1), act ? u[3].im : R(0)}};
        if (form == 3) {
            if (rm != 0)
                trial_pair<R, G, P, 3, true>(v, rm, rv, x);
            else
                trial_pair<R, G, P, 3, false>(v, rm, rv, x);
        } else {
            if (rm != 0)
                trial_pair<R, G, P, 1, true>(v, rm, rv, x);
            else
                trial_pair<R, G, P, 1, false>(v, rm, rv, x);
        }
        return;
    }
    if (rm != 0) {
        if (form == 3)
            trial_pair<R, G, P, 3, true>(u, rm, rv, x);  // no gate of the set lowers to one
        else
            trial_pair<R, G, P, 1, true>(u, rm, rv, x);
        return;
    }
    switch (form) {
    case 0: trial_pair<R, G, P, 0, false>(u, rm, rv, x); break;
    case 1: trial_pair<R, G, P, 1, false>(u, rm, rv, x); break;
    case 2: trial_pair<R, G, P, 2, false>(u, rm, rv, x); break;
    case 4: trial_pair<R, G, P, 4, false>(u, rm, rv, x); break;  // never controlled
    case 5: trial_pair<R, G, P, 5, false>(u, rm, rv, x); break;
    default: trial_pair<R, G, P, 3, false>(u, rm, rv, x); break;
    }
}

template <typename R, int G, bool L>
__device__ __forceinline__ void trial_dispatch(uint32_t P, uint32_t type, uint32_t form,
                                               uint32_t neg_val, const cplx<R> (&u)[4],
                                               uint32_t rm, uint32_t rv, bool act,
                                               cplx<R> (&x)[1 << G])
{
    switch (P) {
    case 0: trial_at<R, G, 0, L>(type, form, neg_val, u, rm, rv, act, x); break;
    case 1: trial_at<R, G, 1, L>(type, form, neg_val, u, rm, rv, act, x); break;
    case 2: trial_at<R, G, 2, L>(type, form, neg_val, u, rm, rv, act, x); break;
    case 3: if constexpr (G > 3) trial_at<R, G, 3, L>(type, form, neg_val, u, rm, rv, act, x); break;
    default: if constexpr (G > 4) trial_at<R, G, 4, L>(type, form, neg_val, u, rm, rv, act, x); break;
    }
}

// One trial operation on the thread's registers (base index j0).  The
// record's fields are uniform and read with scalar loads, and every branch
// is uniform over the wave.  A diagonal or sign flip on a qubit outside the
// group, and the phase flips on lane qubits after a gate, are diagonal in
// the lane qubits: they commute with the group's other gates (whose targets
// are group qubits) and multiply the whole quantum by a per-lane factor,
// collected in F and applied once at the end of the group (useF).
template <typename R, int G>
__device__ __forceinline__ void trial_apply(const TrialGateOp<R> &op, uint32_t j0,
                                            cplx<R> (&x)[1 << G], cplx<R> &F, bool &useF)
{
    const uint32_t meta = op.meta, regs = op.regs;
    const uint32_t type = meta & 15u, form = (meta >> 4) & 15u, neg_val = (meta >> 8) & 1u;
    const uint32_t P = (meta >> 12) & 15u;
    const uint32_t rm = regs & 255u, rv = (regs >> 8) & 255u, rz = (regs >> 16) & 255u;
    const uint32_t zmask = op.zmask;
    const bool act = (j0 & op.lm) == op.lv;
    cplx<R> u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        u[k] = op.u[k];
    if (P < (uint32_t)G) {
        if (op.lm == 0)
            trial_dispatch<R, G, false>(P, type, form, neg_val, u, rm, rv, true, x);
        else
            trial_dispatch<R, G, true>(P, type, form, neg_val, u, rm, rv, act, x);
    } else {
        // the thread's bit of the target decides, for all of its registers
        const uint32_t target = (meta >> 16) & 31u;
        const bool neg = type == kOpNeg;
        const bool hit = act && ((j0 >> target) & 1u) == (neg ? neg_val : 1u);
        const cplx<R> f = neg ? cplx<R>{R(-1), R(0)} : u[3];
        const cplx<R> q = {hit ? f.re : R(1), hit ? f.im : R(0)};
        if (rm == 0) {
            F = cmul(F, q);
            useF = true;
        } else {
#pragma unroll
            for (int r = 0; r < (1 << G); ++r)
                if (((uint32_t)r & rm) == rv)
                    x[r] = cmul(x[r], q);
        }
    }
    if ((zmask | rz) != 0) {
        const bool lpar = (__popc(j0 & zmask) & 1u) != 0;
        if (rz == 0) {
            F = {lpar ? -F.re : F.re, lpar ? -F.im : F.im};
            useF = true;
        } else {
#pragma unroll
            for (int r = 0; r < (1 << G); ++r) {
                const bool s = lpar != ((__popc((uint32_t)r & rz) & 1u) != 0);
                x[r] = {s ? -x[r].re : x[r].re, s ? -x[r].im : x[r].im};
            }
        }
    }
}

// Preparation of the register-group variants: one workgroup per trial of
// the batch builds all of the trial's gates (draws, X mask, matrices in
// FP64) into global memory, and the X mask after the last gate, so that the
// trial kernel itself does no FP64 work and reads each gate with scalar
// loads.
constexpr int kPrepThreads = 256;

template <typename R>
__global__ void __launch_bounds__(kPrepThreads) k_trial_prep(const TrialLaunch L, uint64_t t0,
                                                             const uint32_t *__restrict__ gword,
                                                             TrialGateOp<R> *__restrict__ out,
                                                             uint32_t *__restrict__ out_X)
{
    __shared__ uint32_t scan[kPrepThreads];
    const uint32_t tid = threadIdx.x, n = L.ngates, M = L.M;
    const uint64_t t = t0 + blockIdx.x;  // trial index within the call
    const uint64_t trial = L.trial0 + t;
    const bool draws_flip = L.p_bit > 0.0 || L.p_phase > 0.0;
    const uint64_t thr_b = flip_threshold(L.p_bit), thr_p = flip_threshold(L.p_phase);
    const int G = L.variant == 2 ? 4 : 5;
    TrialGateOp<R> *ops = out + (uint64_t)blockIdx.x * n;
    uint32_t X = 0;  // bit flips before the current block of gates
    for (uint32_t c0 = 0; c0 < n; c0 += kPrepThreads) {
        const uint32_t g = c0 + tid;
        uint32_t bm = 0, zm = 0;
        if (g < n && draws_flip) {
            for (uint32_t q = 0; q < M; ++q) {
                const u64x4 r = philox4x64_10(g, q, kStreamFlip, 0, L.seed, trial);
                if ((r.w[0] >> 32) < thr_b)
                    bm |= 1u << q;
                if ((r.w[1] >> 32) < thr_p)
                    zm |= 1u << q;
            }
        }
        // inclusive XOR scan of the block's bit flips
        scan[tid] = bm;
        __syncthreads();
        for (uint32_t off = 1; off < kPrepThreads; off <<= 1) {
            const uint32_t v = tid >= off ? scan[tid - off] : 0u;
            __syncthreads();
            scan[tid] ^= v;
            __syncthreads();
        }
        const uint32_t xg = X ^ scan[tid] ^ bm;  // mask before gate g
        if (g < n) {
            const TrialGate gd = L.gates[g];
            const double eps = L.sigma > 0.0 ? L.sigma * step_gaussian(L.seed, trial, g) : 0.0;
            uint32_t type;
            double u[8];
            gate_matrix(gd.kind, gd.theta, eps, type, u);
            const bool flipped = (xg >> gd.target) & 1u;
            if (flipped) {
                // X U X: swap rows and columns
                for (int k = 0; k < 2; ++k) {
                    double a = u[k];
                    u[k] = u[6 + k];
                    u[6 + k] = a;
                    a = u[2 + k];
                    u[2 + k] = u[4 + k];
                    u[4 + k] = a;
                }
            }
            if (type == kOpDiag) {
                // diag(d0, d1) = d0 diag(1, d1 / d0); d0 is a global phase
                const double n0 = u[0] * u[0] + u[1] * u[1];
                const double qr = (u[6] * u[0] + u[7] * u[1]) / n0;
                const double qi = (u[7] * u[0] - u[6] * u[1]) / n0;
                u[0] = 1.0; u[1] = 0.0; u[6] = qr; u[7] = qi;
            }
            TrialGateOp<R> op;
            op.u[0] = {(R)u[0], (R)u[1]};
            op.u[1] = {(R)u[2], (R)u[3]};
            op.u[2] = {(R)u[4], (R)u[5]};
            op.u[3] = {(R)u[6], (R)u[7]};
            const bool real_off = u[3] == 0.0 && u[5] == 0.0;
            const bool real_diag = u[1] == 0.0 && u[7] == 0.0;
            const bool zero_diag = u[0] == 0.0 && u[6] == 0.0;
            uint32_t form = !real_off ? 3u : real_diag ? 0u : zero_diag ? 2u : 1u;
            op.scale = R(1);
            // an uncontrolled Hadamard, perturbed or not, is hb (B + i t) with
            // B = [[1, 1], [1, -1]], or [[-1, 1], [1, 1]] after X U X, and
            // hb = h cos(eps/2): the pair update is the butterfly B plus i t
            // on the diagonal (t in u[0].im), and hb goes to the record's
            // scale, which the group applies at its end.  Only while |t| <= 1
            // (|eps| below about 1.23), which bounds the growth inside a
            // group; beyond that the gate keeps its full coefficients.
            const double hb = u[2];
            if (type == kOpMat && gd.cmask == 0 && real_off && hb != 0.0 && u[4] == hb &&
                u[1] == u[7] && ((u[0] == hb && u[6] == -hb) || (u[0] == -hb && u[6] == hb)) &&
                fabs(u[1]) <= kMaxButterflyT * fabs(hb)) {
                form = u[0] == hb ? 4u : 5u;
                op.u[0].im = (R)(u[1] / hb);
                op.scale = (R)hb;
            }
            // positions relative to the gate's group
            const uint32_t w = gword[g];
            const uint32_t cval = gd.cmask & ~xg;
            uint32_t P = 15, rm = 0, rv = 0, rz = 0, gmask = 0;
            for (int i = 0; i < G; ++i) {
                const uint32_t b = (w >> (4 * i)) & 15u;
                gmask |= 1u << b;
                if (b == gd.target)
                    P = (uint32_t)i;
                rm |= ((gd.cmask >> b) & 1u) << i;
                rv |= ((cval >> b) & 1u) << i;
                rz |= ((zm >> b) & 1u) << i;
            }
            // a lane-space mask lists its qubits in the thread's base index,
            // which keeps the group qubits at zero: the masks are used as is
            op.meta = type | (form << 4) | ((flipped ? 0u : 1u) << 8) | (P << 12) |
                      (gd.target << 16);
            op.regs = rm | (rv << 8) | (rz << 16);
            op.lm = gd.cmask & ~gmask;
            op.lv = cval & ~gmask;
            // phase flips follow this step's bit flips; Z_q on the true
            // register is Z_q on the stored one up to a global sign
            op.zmask = zm & ~gmask;
            for (uint32_t &pw : op.pad)
                pw = 0;
            ops[g] = op;
        }
        X ^= scan[kPrepThreads - 1];
        __syncthreads();
    }
    if (tid == 0)
        out_X[blockIdx.x] = X;
}

// LDS slot of register element j: one pad slot after every 128 bytes, so
// that lanes striding over a power of two of elements spread over the banks.
template <typename R>
__device__ __forceinline__ uint32_t trial_slot(uint32_t j)
{
    return j + (j >> (sizeof(cplx<R>) == 8 ? 4 : 3));
}

template <typename R>
size_t trial_group_lds(int M)
{
    const size_t n = (size_t)1 << M;
    return (n + (n >> (sizeof(cplx<R>) == 8 ? 4 : 3))) * sizeof(cplx<R>);
}

// The gate records, the group records and the masks are read-only here and
// alias nothing the kernel writes, so their uniform reads become scalar
// loads.
template <typename R, int G, int T>
__global__ void __launch_bounds__(T) k_trials_groups(const TrialLaunch L, uint64_t t0,
                                                     uint64_t nt,
                                                     const TrialGateOp<R> *__restrict__ ops,
                                                     const uint32_t *__restrict__ Xs,
                                                     const uint32_t *__restrict__ groups,
                                                     const cplx<R> *__restrict__ ideal,
                                                     double *__restrict__ out_F)
{
    extern __shared__ __align__(16) uint8_t lds[];
    cplx<R> *buf = reinterpret_cast<cplx<R> *>(lds);
    __shared__ double red[4][T / 64];
    const uint32_t tid = threadIdx.x, n = L.ngates;

    for (uint64_t b = blockIdx.x; b < nt; b += gridDim.x) {
        const TrialGateOp<R> *tops = ops + b * n;
        uint32_t w = L.ngroups > 0 ? groups[2] : 0u;
        uint32_t j0, gmask;
        trial_layout<G>(w, j0, gmask);
        cplx<R> x[1 << G];
#pragma unroll
        for (int r = 0; r < (1 << G); ++r)
            x[r] = {R((r == 0 && j0 == 0) ? 1 : 0), R(0)};
        for (uint32_t gi = 0; gi < L.ngroups; ++gi) {
            const uint32_t first = groups[4 * gi], count = groups[4 * gi + 1];
            const uint32_t nw = groups[4 * gi + 2];
            if (nw != w) {
                // registers -> LDS in the old layout, LDS -> registers in the new one
#pragma unroll
                for (int r = 0; r < (1 << G); ++r)
                    buf[trial_slot<R>(trial_index<G>(j0, w, r))] = x[r];
                __syncthreads();
                w = nw;
                trial_layout<G>(w, j0, gmask);
#pragma unroll
                for (int r = 0; r < (1 << G); ++r)
                    x[r] = buf[trial_slot<R>(trial_index<G>(j0, w, r))];
                __syncthreads();
            }
            // two gates per trip: a gate's results land in other registers
            // than its inputs, and the second writes them back
            cplx<R> F = {R(1), R(0)};
            bool useF = false;
            R S = R(1);  // scales the butterflies of the group left out
            const uint32_t end = first + count;
            for (uint32_t g = first; g < end; g += 2) {
                trial_apply<R, G>(tops[g], j0, x, F, useF);
                S *= tops[g].scale;
                if (g + 1 >= end)
                    break;
                trial_apply<R, G>(tops[g + 1], j0, x, F, useF);
                S *= tops[g + 1].scale;
            }
            if (useF) {
                F = {F.re * S, F.im * S};
#pragma unroll
                for (int r = 0; r < (1 << G); ++r)
                    x[r] = cmul(x[r], F);
            } else if (S != R(1)) {
#pragma unroll
                for (int r = 0; r < (1 << G); ++r)
                    x[r] = {x[r].re * S, x[r].im * S};
            }
        }
        // fidelity against the error-free register, reading psi(i) = s(i ^ X)
        const uint32_t X = Xs[b];
        double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 0; r < (1 << G); ++r) {
            const uint32_t j = trial_index<G>(j0, w, r);
            const cplx<R> a = ideal[j ^ X];
            const double ar = a.re, ai = a.im, br = x[r].re, bi = x[r].im;
            v[0] += ar * br + ai * bi;
            v[1] += ar * bi - ai * br;
            v[2] += ar * ar + ai * ai;
            v[3] += br * br + bi * bi;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            v[c] = wave_sum(v[c]);
        __syncthreads();
        if ((tid & 63) == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                red[c][tid >> 6] = v[c];
        }
        __syncthreads();
        if (tid == 0) {
            double s4[4] = {0.0, 0.0, 0.0, 0.0};
            for (int wv = 0; wv < T / 64; ++wv)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    s4[c] += red[c][wv];
            out_F[t0 + b] = (s4[0] * s4[0] + s4[1] * s4[1]) / (s4[2] * s4[3]);
        }
    }
}

template <typename R, int T>
hipError_t launch_t(const TrialLaunch &L, hipStream_t st)
{
    const size_t lds = trial_lds_bytes((int)L.M, (int)sizeof(cplx<R>));
    auto fn = k_trials<R, T>;
    const hipError_t e = kernel_allow_lds(reinterpret_cast<const void *>(fn), lds);
    if (e != hipSuccess)
        return e;
    const uint64_t grid = L.n_trials < (uint64_t)L.grid ? L.n_trials : (uint64_t)L.grid;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(T), lds, st, L.gates, L.ngates, L.M,
                       L.sigma, L.p_bit, L.p_phase, L.seed, L.trial0, L.n_trials,
                       reinterpret_cast<const cplx<R> *>(L.ideal), L.out_F);
    return hipGetLastError();
}

template <typename R, int G, int T>
hipError_t launch_g(const TrialLaunch &L, hipStream_t st)
{
    const size_t lds = trial_group_lds<R>((int)L.M);
    auto fn = k_trials_groups<R, G, T>;
    const hipError_t ea = kernel_allow_lds(reinterpret_cast<const void *>(fn), lds);
    if (ea != hipSuccess)
        return ea;
    TrialGateOp<R> *ops = reinterpret_cast<TrialGateOp<R> *>(L.prep_ops);
    for (uint64_t t0 = 0; t0 < L.n_trials; t0 += L.prep_batch) {
        const uint64_t nt = std::min<uint64_t>(L.prep_batch, L.n_trials - t0);
        hipLaunchKernelGGL(k_trial_prep<R>, dim3((unsigned)nt), dim3(kPrepThreads), 0, st, L, t0,
                           L.sched + 4 * (L.nchunks + L.ngroups), ops, L.prep_X);
        const uint64_t grid = nt < (uint64_t)L.grid ? nt : (uint64_t)L.grid;
        hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(T), lds, st, L, t0, nt,
                           (const TrialGateOp<R> *)ops, (const uint32_t *)L.prep_X,
                           L.sched + 4 * L.nchunks, reinterpret_cast<const cplx<R> *>(L.ideal),
                           L.out_F);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename R, int G>
hipError_t launch_groups(const TrialLaunch &L, hipStream_t st)
{
    if (L.sched == nullptr || L.prep_ops == nullptr || L.prep_X == nullptr || L.prep_batch == 0 ||
        (int)L.M - G < 6 || (int)L.M - G > 10)
        return hipErrorInvalidValue;
    switch ((int)L.M - G) {
    case 6: return launch_g<R, G, 64>(L, st);
    case 7: return launch_g<R, G, 128>(L, st);
    case 8: return launch_g<R, G, 256>(L, st);
    case 9: return launch_g<R, G, 512>(L, st);
    default: return launch_g<R, G, 1024>(L, st);
    }
}

template <typename R, int G, int T>
int grid_g(int M)
{
    return kernel_resident_blocks(reinterpret_cast<const void *>(k_trials_groups<R, G, T>), T,
                                  trial_group_lds<R>(M));
}

template <typename R, int G>
int grid_groups(int M)
{
    switch (M - G) {
    case 6: return grid_g<R, G, 64>(M);
    case 7: return grid_g<R, G, 128>(M);
    case 8: return grid_g<R, G, 256>(M);
    case 9: return grid_g<R, G, 512>(M);
    case 10: return grid_g<R, G, 1024>(M);
    default: return 0;
    }
}

}  // namespace

size_t trial_lds_bytes(int M, int elem_bytes)
{
    const size_t op_bytes = elem_bytes == 8 ? sizeof(TrialOp<float>) : sizeof(TrialOp<double>);
    return ((size_t)1 << M) * (size_t)elem_bytes + kChunk * op_bytes;
}

// Variants the autotuner chooses from: one LDS sweep per gate with 1024 or
// 512 threads, or the register in registers with 4 or 5 group qubits.
template <typename R>
hipError_t launch_trials(const TrialLaunch &L, hipStream_t st)
{
    switch (L.variant) {
    case 0: return launch_t<R, 1024>(L, st);
    case 1: return launch_t<R, 512>(L, st);
    case 2: return launch_groups<R, 4>(L, st);
    case 3: return launch_groups<R, 5>(L, st);
    default: return hipErrorInvalidValue;
    }
}

int trial_variants() { return 4; }

int trial_group_bits(int variant) { return variant == 2 ? 4 : variant == 3 ? 5 : 0; }

size_t trial_gate_op_bytes(int elem_bytes)
{
    return elem_bytes == 8 ? sizeof(TrialGateOp<float>) : sizeof(TrialGateOp<double>);
}

template <typename R, int T>
int grid_t(int M)
{
    return kernel_resident_blocks(reinterpret_cast<const void *>(k_trials<R, T>), T,
                                  trial_lds_bytes(M, (int)sizeof(cplx<R>)));
}

int trial_grid(int variant, int M, int elem_bytes)
{
    const bool f = elem_bytes == 8;
    switch (variant) {
    case 0: return f ? grid_t<float, 1024>(M) : grid_t<double, 1024>(M);
    case 1: return f ? grid_t<float, 512>(M) : grid_t<double, 512>(M);
    case 2: return f ? grid_groups<float, 4>(M) : grid_groups<double, 4>(M);
    case 3: return f ? grid_groups<float, 5>(M) : grid_groups<double, 5>(M);
    default: return 0;
    }
}

const char *trial_variant_name(int v)
{
    switch (v) {
    case 0: return "lds-per-gate-1024";
    case 1: return "lds-per-gate-512";
    case 2: return "register-groups-4";
    case 3: return "register-groups-5";
    default: return "?";
    }
}

template hipError_t launch_trials<float>(const TrialLaunch &, hipStream_t);
template hipError_t launch_trials<double>(const TrialLaunch &, hipStream_t);

}  // namespace qsim
