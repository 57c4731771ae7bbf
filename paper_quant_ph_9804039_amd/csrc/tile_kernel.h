// Fused tile pass for gfx950: one HBM read and one HBM write of the state
// for a whole run of operations.
//
// The pair decomposition of Sec. 2.1 means a gate on target t only mixes
// amplitudes that differ in bit t.  Pick a set S of k qubits; the 2^k
// amplitudes that share all bits outside S (a "tile") are then closed under
// every gate whose target lies in S, and under every diagonal gate wherever
// its target is.  A control outside S is a constant of the tile.  So each
// workgroup takes one tile, applies the whole run of operations to it, and
// writes it back once.
//
// Inside a pass the operations come in groups whose targets (those that
// need one) fall on at most G tile bits.  For a group, each of the 2^(k-G)
// threads holds one "quantum" in registers: the 2^G amplitudes spanned by the
// group bits, register r holding the amplitude whose group bits spell r.
// Then every operation of the group is a fixed pattern of register pairs,
// and the uniform operation stream costs no data movement.  The first
// group's quanta come straight from HBM and the last group's go straight
// back; between groups the tile is re-partitioned through LDS.  Threads
// enumerate the non-group tile bits from the lowest, and the lowest tile bits
// are the low qubits, so neighbouring lanes touch neighbouring amplitudes.
#pragma once
// Included by kernels_tile_c64.hip and kernels_tile_c128.hip, one
// translation unit per precision so the two compile in parallel.
#include "launch.h"

namespace qsim {
namespace {

__device__ __forceinline__ void ld2(const cplx<float> *p, cplx<float> &a, cplx<float> &b)
{
    const float4 v = *reinterpret_cast<const float4 *>(p);
    a = {v.x, v.y};
    b = {v.z, v.w};
}
__device__ __forceinline__ void st2(cplx<float> *p, cplx<float> a, cplx<float> b)
{
    *reinterpret_cast<float4 *>(p) = make_float4(a.re, a.im, b.re, b.im);
}
__device__ __forceinline__ void ld2(const cplx<double> *p, cplx<double> &a, cplx<double> &b)
{
    const double2 v0 = reinterpret_cast<const double2 *>(p)[0];
    const double2 v1 = reinterpret_cast<const double2 *>(p)[1];
    a = {v0.x, v0.y};
    b = {v1.x, v1.y};
}
__device__ __forceinline__ void st2(cplx<double> *p, cplx<double> a, cplx<double> b)
{
    reinterpret_cast<double2 *>(p)[0] = make_double2(a.re, a.im);
    reinterpret_cast<double2 *>(p)[1] = make_double2(b.re, b.im);
}

// One amplitude at its natural alignment (8 bytes for complex64): the
// struct itself only promises 4, and the compiler then splits the access in
// two.
__device__ __forceinline__ cplx<float> ld1(const cplx<float> *p)
{
    const float2 v = *static_cast<const float2 *>(__builtin_assume_aligned(p, 8));
    return {v.x, v.y};
}
__device__ __forceinline__ void st1(cplx<float> *p, cplx<float> a)
{
    *static_cast<float2 *>(__builtin_assume_aligned(p, 8)) = make_float2(a.re, a.im);
}
__device__ __forceinline__ cplx<double> ld1(const cplx<double> *p)
{
    const double2 v = *static_cast<const double2 *>(__builtin_assume_aligned(p, 16));
    return {v.x, v.y};
}
__device__ __forceinline__ void st1(cplx<double> *p, cplx<double> a)
{
    *static_cast<double2 *>(__builtin_assume_aligned(p, 16)) = make_double2(a.re, a.im);
}

// Register-pair loops of one operation on group bit P, specialised at
// compile time.  Register r of a quantum holds the amplitude whose group bits
// spell r, so the target bit is a compile-time property of r.  C: controls
// on group bits (mask rc over the register index) are tested, with a uniform
// test per register; without them every register takes part.  F: the form
// of a kTPair, 0 = real 2x2 m, 1 = m plus i*w on the diagonal, 2 = the same
// with m00 = m11 = 0 (a perturbed X), 3 = the butterfly a + b, a - b plus
// i*w on the diagonal (a Hadamard whose scale h joined the pass's phase), 4 =
// the same with w = 0.  The coefficients are values, so a lane-controlled
// operation passes per-lane ones (the identity where the lane's controls are
// not met).
template <typename R>
struct PairCoef {
    R m00, m01, m10, m11, w0, w1;
};

template <typename R, int G, int P, int F, bool C>
__device__ __forceinline__ void pair_loop(const PairCoef<R> &m, uint32_t rc, cplx<R> (&x)[1 << G])
{
    // out0 = m00 a + m01 b + i w0 a,  out1 = m10 a + m11 b + i w1 b
#pragma unroll
    for (int r = 0; r < (1 << G); ++r) {
        if ((r & (1 << P)) || (C && ((uint32_t)r & rc) != rc))
            continue;
        const int r1 = r | (1 << P);
        const cplx<R> a = x[r], b = x[r1];
        cplx<R> na, nb;
        if (F == 4) {
            na = {a.re + b.re, a.im + b.im};
            nb = {a.re - b.re, a.im - b.im};
        } else if (F == 3) {
            // grouped so that no sum is shared with form 4: the compiler
            // would hoist a shared a +- b above the form test
            na = {(a.re - m.w0 * a.im) + b.re, (a.im + m.w0 * a.re) + b.im};
            nb = {(a.re - m.w0 * b.im) - b.re, (a.im + m.w0 * b.re) - b.im};
        } else if (F == 2) {
            na = {m.m01 * b.re - m.w0 * a.im, m.m01 * b.im + m.w0 * a.re};
            nb = {m.m10 * a.re - m.w1 * b.im, m.m10 * a.im + m.w1 * b.re};
        } else {
            na = {m.m00 * a.re + m.m01 * b.re, m.m00 * a.im + m.m01 * b.im};
            nb = {m.m10 * a.re + m.m11 * b.re, m.m10 * a.im + m.m11 * b.im};
            if (F == 1) {
                na.re -= m.w0 * a.im;
                na.im += m.w0 * a.re;
                nb.re -= m.w1 * b.im;
                nb.im += m.w1 * b.re;
            }
        }
        x[r] = na;
        x[r1] = nb;
    }
}

// L: lane-controlled, the pair is exchanged only where `act` holds.
template <typename R, int G, int P, bool C, bool L>
__device__ __forceinline__ void swap_loop(uint32_t rc, bool act, cplx<R> (&x)[1 << G])
{
#pragma unroll
    for (int r = 0; r < (1 << G); ++r) {
        if ((r & (1 << P)) || (C && ((uint32_t)r & rc) != rc))
            continue;
        const int r1 = r | (1 << P);
        const cplx<R> a = x[r], b = x[r1];
        // selects on the components: a select of whole structs can become a
        // select of their addresses, which keeps the quantum out of registers
        const bool s = !L || act;
        x[r] = {s ? b.re : a.re, s ? b.im : a.im};
        x[r1] = {s ? a.re : b.re, s ? a.im : b.im};
    }
}

template <typename R, int G, int P, bool C>
__device__ __forceinline__ void diag_loop(cplx<R> d0, cplx<R> d1, uint32_t rc, cplx<R> (&x)[1 << G])
{
#pragma unroll
    for (int r = 0; r < (1 << G); ++r) {
        if (C && ((uint32_t)r & rc) != rc)
            continue;
        x[r] = cmul(x[r], ((r >> P) & 1) ? d1 : d0);
    }
}

// diag(1, q) on group bit P: only the registers whose bit P is set move.
template <typename R, int G, int P>
__device__ __forceinline__ void phase_loop(const TileOp<R> &op, cplx<R> (&x)[1 << G])
{
    const cplx<R> q = {op.c[2], op.c[3]};
#pragma unroll
    for (int r = 0; r < (1 << G); ++r)
        if ((r >> P) & 1)
            x[r] = cmul(x[r], q);
}

template <typename R, int G, int P, bool C, bool L>
__device__ __forceinline__ void neg_loop(uint32_t rc, bool act, cplx<R> (&x)[1 << G])
{
#pragma unroll
    for (int r = 0; r < (1 << G); ++r) {
        if (!((r >> P) & 1) || (C && ((uint32_t)r & rc) != rc))
            continue;
        const bool s = !L || act;
        x[r] = {s ? -x[r].re : x[r].re, s ? -x[r].im : x[r].im};
    }
}

template <typename R>
__device__ __forceinline__ PairCoef<R> pair_coef(const TileOp<R> &op)
{
    return {op.c[0], op.c[1], op.c[2], op.c[3], op.c[4], op.c[5]};
}

// One operation on the registers of group bit P, for every lane of the
// quantum.  Operations without a control on a group bit (the common case)
// take loops with no per-register tests.
template <typename R, int G, int P>
__device__ __forceinline__ void apply_at(const TileOp<R> &op, cplx<R> (&x)[1 << G])
{
    const bool ctl = op.rc != 0;
    switch (op.kind) {
    case kTPair:
        if (ctl)
            pair_loop<R, G, P, 1, true>(pair_coef(op), op.rc, x);
        else if (op.form == 0)
            pair_loop<R, G, P, 0, false>(pair_coef(op), 0u, x);
        else if (op.form == 1)
            pair_loop<R, G, P, 1, false>(pair_coef(op), 0u, x);
        else if (op.form == 2)
            pair_loop<R, G, P, 2, false>(pair_coef(op), 0u, x);
        else if (op.form == 3)
            pair_loop<R, G, P, 3, false>(pair_coef(op), 0u, x);
        else
            pair_loop<R, G, P, 4, false>(pair_coef(op), 0u, x);
        break;
    case kTSwap:
        if (ctl)
            swap_loop<R, G, P, true, false>(op.rc, true, x);
        else
            swap_loop<R, G, P, false, false>(0u, true, x);
        break;
    case kTPhaseIn:  // never controlled
        phase_loop<R, G, P>(op, x);
        break;
    case kTDiagIn: {
        const cplx<R> d0 = {op.c[0], op.c[1]}, d1 = {op.c[2], op.c[3]};
        if (ctl)
            diag_loop<R, G, P, true>(d0, d1, op.rc, x);
        else
            diag_loop<R, G, P, false>(d0, d1, 0u, x);
        break;
    }
    default:  // kTNegIn
        if (ctl)
            neg_loop<R, G, P, true, false>(op.rc, true, x);
        else
            neg_loop<R, G, P, false, false>(0u, true, x);
        break;
    }
}

// The same for an operation with controls on lane (non-group tile) bits:
// `act` says whether this lane's controls are met.  The lanes of a wave
// differ here, so instead of branching per lane (which would make the
// compiler copy the whole quantum around every operation to keep the
// inactive lanes' values), the operation is applied everywhere with
// per-lane coefficients that are the identity where act is false.
template <typename R, int G, int P>
__device__ __forceinline__ void apply_at_lane(const TileOp<R> &op, bool act, cplx<R> (&x)[1 << G])
{
    const bool ctl = op.rc != 0;
    const R one = R(1), zero = R(0);
    switch (op.kind) {
    case kTPair: {
        const PairCoef<R> m = {act ? op.c[0] : one, act ? op.c[1] : zero, act ? op.c[2] : zero,
                               act ? op.c[3] : one, act ? op.c[4] : zero, act ? op.c[5] : zero};
        if (ctl)
            pair_loop<R, G, P, 1, true>(m, op.rc, x);
        else if (op.form == 0)
            pair_loop<R, G, P, 0, false>(m, 0u, x);
        else
            pair_loop<R, G, P, 1, false>(m, 0u, x);
        break;
    }
    case kTSwap:
        if (ctl)
            swap_loop<R, G, P, true, true>(op.rc, act, x);
        else
            swap_loop<R, G, P, false, true>(0u, act, x);
        break;
    case kTDiagIn: {
        const cplx<R> d0 = {act ? op.c[0] : one, act ? op.c[1] : zero};
        const cplx<R> d1 = {act ? op.c[2] : one, act ? op.c[3] : zero};
        if (ctl)
            diag_loop<R, G, P, true>(d0, d1, op.rc, x);
        else
            diag_loop<R, G, P, false>(d0, d1, 0u, x);
        break;
    }
    default:  // kTNegIn (kTPhaseIn is never controlled)
        if (ctl)
            neg_loop<R, G, P, true, true>(op.rc, act, x);
        else
            neg_loop<R, G, P, false, true>(0u, act, x);
        break;
    }
}

// One operation of a group on one quantum.  An uncontrolled diagonal
// reaches the kernel as diag(1, q), its d0 having been moved into the pass's
// global phase (a scalar commutes with everything).  On a bit outside the
// group it commutes with everything else in the group (those act on group
// bits only), and its factor is the same for all registers of the quantum:
// such factors are multiplied into one factor F, applied once at the end of
// the group.  Every branch here is uniform over the wave: the controls
// outside the tile are constants of the tile, and those on lane bits are
// applied through per-lane coefficients.
template <typename R, int G>
__device__ __forceinline__ void apply_op(const TileOp<R> &op, cplx<R> (&x)[1 << G], uint32_t j0,
                                         uint64_t base, cplx<R> &F, bool &useF)
{
    if ((base & op.cm_out) != op.cm_out)
        return;
    if (op.kind >= kTDiagOut) {
        // never controlled; the factor depends on the lane where the target
        // is a lane bit
        const bool bit = op.tpos != kNoPos ? ((j0 >> op.tpos) & 1u) != 0
                                           : ((base >> op.tq) & 1u) != 0;
        if (op.kind == kTNegOut) {
            F = {bit ? -F.re : F.re, bit ? -F.im : F.im};
        } else {
            const cplx<R> d = {bit ? op.c[2] : op.c[0], bit ? op.c[3] : op.c[1]};
            F = cmul(F, d);
        }
        useF = true;
        return;
    }
    // Controls on lane bits: where they fall on bits that are constant over
    // the wave (the wave bits of the thread index), every lane agrees, and
    // the wave either skips the operation or applies its plain form.
    bool act = true, mixed = false;
    if (op.qc != 0) {
        act = (j0 & op.qc) == op.qc;
        const uint64_t agree = __builtin_amdgcn_ballot_w64(act);
        if (agree == 0)
            return;
        mixed = agree != ~0ull;
    }
    if (!mixed) {
        switch (op.gpos) {
        case 0: apply_at<R, G, 0>(op, x); break;
        case 1: apply_at<R, G, 1>(op, x); break;
        case 2: apply_at<R, G, 2>(op, x); break;
        case 3: if constexpr (G > 3) apply_at<R, G, 3>(op, x); break;
        default: if constexpr (G > 4) apply_at<R, G, 4>(op, x); break;
        }
    } else {
        switch (op.gpos) {
        case 0: apply_at_lane<R, G, 0>(op, act, x); break;
        case 1: apply_at_lane<R, G, 1>(op, act, x); break;
        case 2: apply_at_lane<R, G, 2>(op, act, x); break;
        case 3: if constexpr (G > 3) apply_at_lane<R, G, 3>(op, act, x); break;
        default: if constexpr (G > 4) apply_at_lane<R, G, 4>(op, act, x); break;
        }
    }
}

// Apply the operations [first, first + cnt) of a group to one quantum; the
// last group's F starts from the pass's global phase.  An operation's
// results land in other registers than its inputs; with two operations per
// trip of the loop the second writes them back where the first read them,
// so no copy of the quantum closes each trip.
template <typename R, int G>
__device__ __forceinline__ void apply_group(const TileArgs<R> &A, uint32_t first, uint32_t cnt,
                                            cplx<R> (&x)[1 << G], uint32_t j0, uint64_t base,
                                            bool last)
{
    static_assert(G >= 3 && G <= 5, "group bits");
    const bool ph = last && A.use_phase != 0;
    cplx<R> F = ph ? cplx<R>{A.phase[0], A.phase[1]} : cplx<R>{R(1), R(0)};
    bool useF = ph;
    const uint32_t end = first + cnt;
    for (uint32_t o = first; o < end; o += 2) {
        const TileOp<R> op = A.ops[o];  // whole descriptor at once: one scalar wait
        apply_op<R, G>(op, x, j0, base, F, useF);
        if (o + 1 >= end)
            break;
        const TileOp<R> op2 = A.ops[o + 1];
        apply_op<R, G>(op2, x, j0, base, F, useF);
    }
    if (useF) {
#pragma unroll
        for (int r = 0; r < (1 << G); ++r)
            x[r] = cmul(x[r], F);
    }
}

template <int G>
__device__ __forceinline__ uint32_t elem_index(uint32_t j0, const uint32_t (&e)[G], int r)
{
    uint32_t j = j0;
#pragma unroll
    for (int i = 0; i < G; ++i)
        if (r & (1 << i))
            j |= e[i];
    return j;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Global element offset of register r: the sum of the offsets of its set
// group bits (distinct qubits, so the sums are disjoint ORs).
template <int G>
__device__ __forceinline__ uint64_t greg(const uint64_t (&o)[G], int r)
{
    uint64_t d = 0;
#pragma unroll
    for (int i = 0; i < G; ++i)
        if (r & (1 << i))
            d += o[i];
    return d;
}

// Spread the bits of v over runs of consecutive qubits (a bit deposit done
// run by run).  A run word is start | length << 8; the table is copied to
// scalar registers in one go.
__device__ __forceinline__ uint64_t spread(uint64_t v, const uint32_t (&runs)[kMaxRuns], uint32_t n)
{
    uint64_t g = 0;
    uint32_t used = 0;
#pragma unroll
    for (int i = 0; i < kMaxRuns; ++i) {
        if ((uint32_t)i < n) {
            const uint32_t start = runs[i] & 0xFFu, len = runs[i] >> 8;
            g |= ((v >> used) & ((1ull << len) - 1ull)) << start;
            used += len;
        }
    }
    return g;
}

// Register quantum <-> memory in a given layout (two adjacent registers per
// access when group bit 0 is tile bit 0).
template <typename R, int G>
__device__ __forceinline__ void load_quantum(const cplx<R> *p, const uint64_t (&o)[G], bool pair0,
                                             cplx<R> (&x)[1 << G])
{
    // the empty asm statements fence each shape in its own branch: without
    // them the compiler hoists and merges parts of both into narrow loads
    if (pair0) {
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < (1 << G); r += 2)
            ld2(p + greg<G>(o, r), x[r], x[r + 1]);
        __asm__ volatile("" ::: "memory");
    } else {
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int r = 0; r < (1 << G); ++r)
            x[r] = p[greg<G>(o, r)];
        __asm__ volatile("" ::: "memory");
    }
}

template <typename R, int G>
__device__ __forceinline__ void store_quantum(cplx<R> *p, const uint64_t (&o)[G], bool pair0,
                                              const cplx<R> (&x)[1 << G])
{
    if (pair0) {
#pragma unroll
        for (int r = 0; r < (1 << G); r += 2)
            st2(p + greg<G>(o, r), x[r], x[r + 1]);
    } else {
#pragma unroll
        for (int r = 0; r < (1 << G); ++r)
            p[greg<G>(o, r)] = x[r];
    }
}

// Layout of group gi for this thread: tile-index masks of the group bits,
// tile index of register 0, and whether registers r, r+1 are adjacent.
template <typename R, int G>
__device__ __forceinline__ void group_layout(const TileArgs<R> &A, uint32_t gi, uint32_t (&e)[G],
                                             uint32_t &j0, bool &pair0)
{
    const uint32_t gw = A.group[gi];
    j0 = threadIdx.x;
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const uint32_t p = group_bit(gw, i);
        e[i] = 1u << p;
        j0 = ((j0 >> p) << (p + 1)) | (j0 & ((1u << p) - 1u));
    }
    pair0 = e[0] == 1u;
}

// Waves per SIMD the register budget is sized for.  complex64 with G = 4 is
// the bench shape: two 512-thread workgroups per CU (LDS allows two 64 KiB
// tiles) need four waves per SIMD, i.e. at most 128 VGPRs.
template <typename R, int G>
constexpr int kTileWaves = (sizeof(R) == 4 && G == 4) ? 4 : 1;

// Fused pass, persistent: each workgroup walks one block of consecutive
// tiles.  Each of the T threads holds one quantum of 2^G amplitudes in
// registers (T * 2^G = 2^k).  HBM traffic of one workgroup overlaps the
// register and LDS work of the other workgroups on the CU.  Measured and not
// kept: a register prefetch of the next tile (with or without a two-tile
// unroll), which costs 2^G amplitudes of registers per thread and ran 5-15 %
// slower, and an XOR swizzle of the LDS re-partition, which halved the bank
// conflicts but added more VALU work than it saved.
template <typename R, int G, int T>
__global__ void __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(kTileWaves<R, G>)))
k_tile(const TileArgs<R> A)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ double wsum[T / 64];
    cplx<R> *tile = reinterpret_cast<cplx<R> *>(lds);

    uint32_t srun[kMaxRuns], crun[kMaxRuns];
#pragma unroll
    for (int i = 0; i < kMaxRuns; ++i) {
        srun[i] = A.srun[i];
        crun[i] = A.crun[i];
    }
    const uint32_t nsrun = A.nsrun, ncrun = A.ncrun;
    const uint64_t ntiles = 1ull << (A.mact - A.k);

    // the first group's layout is the same for every tile
    uint32_t e0[G], j00;
    bool pair00;
    group_layout<R, G>(A, 0, e0, j00, pair00);
    uint64_t o0[G];
#pragma unroll
    for (int i = 0; i < G; ++i)
        o0[i] = spread(e0[i], srun, nsrun);
    const uint64_t rel0 = spread(j00, srun, nsrun);
    // so is the last group's, in which the quantum goes back to HBM, and the
    // renormalisation scale
    uint32_t eL[G], jL;
    bool pairL;
    group_layout<R, G>(A, A.ngroups - 1, eL, jL, pairL);
    uint64_t oL[G];
#pragma unroll
    for (int i = 0; i < G; ++i)
        oL[i] = spread(eL[i], srun, nsrun);
    const uint64_t relL = spread(jL, srun, nsrun);
    const bool scaled = A.scale_in != nullptr;
    const R sc = scaled ? (R)*A.scale_in : R(1);

    cplx<R> x[1 << G];
    // each workgroup takes one contiguous block of tile numbers: neighbouring
    // tiles interleave their runs in memory, so one workgroup walking them in
    // order reads and writes whole stretches of HBM (6 % faster loads and
    // stores than dealing tiles round-robin over the workgroups)
    const uint64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const uint64_t t_end = (blockIdx.x + 1) * per < ntiles ? (blockIdx.x + 1) * per : ntiles;
    uint64_t tile_id = blockIdx.x * per;
    // global index of tile element 0: the tile number spread over the
    // enumerated qubits outside the tile (emask), in ascending order, plus
    // the values of the untouched qubits.  Consecutive tile numbers step
    // through the enumerated bits as a masked increment.
    const uint64_t E = A.emask;
    uint64_t ebits = spread(tile_id, crun, ncrun);

    for (; tile_id < t_end; ++tile_id) {
        const uint64_t base = ebits | A.base_or;
        ebits = ((ebits | ~E) + 1u) & E;
        if (A.gen != 0) {
            // a register just reset to a basis state: its one nonzero amplitude
            // is written here instead of by a pass of its own
            const uint64_t rel = base | rel0;
#pragma unroll
            for (int r = 0; r < (1 << G); ++r)
                x[r] = {R(rel + greg<G>(o0, r) == A.gen_index ? 1 : 0), R(0)};
        } else {
            load_quantum<R, G>(A.psi + (base | rel0), o0, pair00, x);
        }
        if (scaled) {
#pragma unroll
            for (int r = 0; r < (1 << G); ++r) {
                x[r].re *= sc;
                x[r].im *= sc;
            }
        }
        uint32_t e[G], j0 = j00;
        bool pair0 = pair00;
#pragma unroll
        for (int i = 0; i < G; ++i)
            e[i] = e0[i];
        // one call site of apply_group for all groups: its code (every
        // operation case, twice for the two slots of a trip) is most of the
        // kernel, and a second copy would double the instruction working set
        for (uint32_t gi = 0; gi < A.ngroups; ++gi) {
            if (gi > 0) {
                // registers -> LDS in the old layout, LDS -> registers in the new one
                if (pair0) {
#pragma unroll
                    for (int r = 0; r < (1 << G); r += 2)
                        st2(tile + elem_index<G>(j0, e, r), x[r], x[r + 1]);
                } else {
#pragma unroll
                    for (int r = 0; r < (1 << G); ++r)
                        st1(tile + elem_index<G>(j0, e, r), x[r]);
                }
                __syncthreads();
                group_layout<R, G>(A, gi, e, j0, pair0);
                // fenced like the HBM loads, so each layout keeps its wide reads
                if (pair0) {
                    __asm__ volatile("" ::: "memory");
#pragma unroll
                    for (int r = 0; r < (1 << G); r += 2)
                        ld2(tile + elem_index<G>(j0, e, r), x[r], x[r + 1]);
                    __asm__ volatile("" ::: "memory");
                } else {
                    __asm__ volatile("" ::: "memory");
#pragma unroll
                    for (int r = 0; r < (1 << G); ++r)
                        x[r] = ld1(tile + elem_index<G>(j0, e, r));
                    __asm__ volatile("" ::: "memory");
                }
                __syncthreads();
            }
            apply_group<R, G>(A, group_first(A.group[gi]), group_count(A.group[gi]), x, j0, base,
                              gi + 1 == A.ngroups);
        }
        // registers -> HBM in the last group's layout
        store_quantum<R, G>(A.psi + (base | relL), oL, pairL, x);
        if (A.norm_out != nullptr) {
            double nsum = 0.0;
#pragma unroll
            for (int r = 0; r < (1 << G); ++r)
                nsum += (double)x[r].re * x[r].re + (double)x[r].im * x[r].im;
            nsum = wave_sum(nsum);
            if ((threadIdx.x & 63) == 0)
                wsum[threadIdx.x >> 6] = nsum;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int w = 0; w < T / 64; ++w)
                    t += wsum[w];
                A.norm_out[tile_id] = t;
            }
            __syncthreads();
        }
    }
}

template <typename R, int G, int T>
hipError_t launch_gt(const TileArgs<R> &A, hipStream_t st)
{
    if (A.k != (uint32_t)G + (uint32_t)__builtin_ctz(T))
        return hipErrorInvalidValue;
    const size_t lds = A.ngroups > 1 ? tile_lds_bytes((int)A.k, (int)sizeof(cplx<R>)) : 0;
    const void *fn = reinterpret_cast<const void *>(k_tile<R, G, T>);
    // more than 64 KiB of dynamic LDS must be allowed per kernel first
    hipError_t e = kernel_allow_lds(fn, lds);
    if (e != hipSuccess)
        return e;
    // persistent grid: as many workgroups as fit on the chip at once (one
    // per CU of the 256 if the occupancy query fails)
    int occ = kernel_resident_blocks(fn, T, lds);
    if (occ <= 0)
        occ = 256;
    const uint64_t tiles = 1ull << (A.mact - A.k);
    const uint64_t grid = tiles < (uint64_t)occ ? tiles : (uint64_t)occ;
    hipLaunchKernelGGL((k_tile<R, G, T>), dim3((unsigned)grid), dim3(T), lds, st, A);
    return hipGetLastError();
}

template <typename R, int G>
hipError_t launch_g(const TileArgs<R> &A, hipStream_t st)
{
    switch ((int)A.k - G) {
    case 6: return launch_gt<R, G, 64>(A, st);
    case 7: return launch_gt<R, G, 128>(A, st);
    case 8: return launch_gt<R, G, 256>(A, st);
    case 9: return launch_gt<R, G, 512>(A, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

template <typename R>
hipError_t launch_tile(const TileArgs<R> &A, int G, hipStream_t st)
{
    switch (G) {
    case 3: return launch_g<R, 3>(A, st);
    case 4: return launch_g<R, 4>(A, st);
    case 5: return launch_g<R, 5>(A, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace qsim
