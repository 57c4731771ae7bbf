// The detailed three-state model on gfx950: every ion of the Cirac-Zoller
// trap has the two levels of its QU-bit plus the temporary third level the
// controlled-not gate passes through (Sec. 2.0), so M ions take 3^M states
// (Sec. 3.0) and one laser transformation is 3^(M-1) independent operations
// on the pairs of states that differ only in the transformed ion's level
// (Sec. 3.1).  State index i = sum_q d_q 3^q, d_q the level of ion q.
//
// The host lowers each gate to transformations (five for a CNOT), draws
// their angle errors and the step's flips, and applies them in order: runs
// whose ions fit one LDS tile as fused passes (k3_tile, one HBM read and
// write per run), else one launch per transformation (k3_pairs, reading and
// writing the two levels a, b of one ion, i.e. 2/3 of the register).
//
// Readings of the paper (its pulse sequences are not given):
//   - transformation on ion q between levels a < b, angle theta, phase phi:
//     exp(-i theta/2 (e^{i phi}|a><b| + e^{-i phi}|b><a|)), third level
//     untouched; a phase transformation multiplies levels a, b by
//     e^{-i theta/2}, e^{+i theta/2} (on levels 0, 1 the two-state Rz);
//   - a transformation may be conditional on another ion being in a given
//     level (the step the trap carries through its motional mode);
//   - X = rot(01, pi, 0); H = rot(01, pi/2, -pi/2) then rot(01, pi, 0);
//     Rz(t) = phase(t); Z = phase(pi); CNOT(c, x) = rot_x(01, pi/2, pi/2),
//     rot_c(12, pi, 0), [c in 2] rot_x(12, 2 pi, 0), rot_c(12, pi, pi),
//     rot_x(01, pi/2, -pi/2); CPHASE(t) on (c, x) = phase_c(t/2),
//     phase_x(t/2), CNOT, phase_x(-t/2), CNOT; Toffoli = the six-CNOT
//     circuit with H on the target and phases of +-pi/4;
//   - every transformation's angle deviates by eps = sigma z, z from
//     Philox4x64-10 keyed by (seed, trial) at counter (step, k, 3, 0) for the
//     gate's k-th transformation (Box-Muller on the high halves of words 0
//     and 1); after each gate, per ion, a bit flip exchanges levels 0 and 1
//     and a phase flip negates level 1 (counter (step, q, 2, 0)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "internal.h"
#include "lookahead.h"
#include "qsim.h"

namespace {

using qsim::cplx;

constexpr int kBlock3 = 256;
constexpr int kMaxIons = 20;      // 3^20 < 2^32: indices stay 32-bit
constexpr int kReduceBlocks3 = 1024;
constexpr int kMaxMarginalIons = 6;  // 3^6 = 729 bins per block in LDS

uint64_t pow3(int e)
{
    uint64_t p = 1;
    for (int i = 0; i < e; ++i)
        p *= 3;
    return p;
}

dim3 grid3(uint64_t work)
{
    uint64_t g = (work + kBlock3 - 1) / kBlock3;
    g = std::min<uint64_t>(std::max<uint64_t>(g, 1), 1u << 20);
    return dim3((unsigned)g);
}

// n / d for 32-bit n with d given with its reciprocal: the FP64 product is
// off by at most one, which the remainder corrects.
__device__ __forceinline__ uint32_t div_by(uint32_t n, uint32_t d, double inv)
{
    uint32_t q = (uint32_t)((double)n * inv);
    const int64_t r = (int64_t)n - (int64_t)q * (int64_t)d;
    if (r < 0)
        --q;
    else if (r >= (int64_t)d)
        ++q;
    return q;
}

// What a launch does to the pairs (level a, level b) of its ion.
enum PairMode : uint32_t { kPairMat = 0, kPairSwap = 1, kPairNegB = 2 };
// Cheaper forms of kPairMat the fused pass recognises: a rotation pulse
// (u00 = u11 = c real, u10 = -conj(u01): 12 flops per pair instead of 16)
// and a diagonal (a phase pulse: 8).
enum : uint32_t { kPairRot = 3, kPairDiag = 4 };

template <typename R>
struct RotArgs {
    cplx<R> *psi;
    uint32_t work;          // 3^(M-1) pairs
    uint32_t place;         // 3^ion
    double inv_place;
    uint32_t a, b;          // levels, a < b
    uint32_t cplace;        // 3^cond_ion (0: unconditional)
    double inv_cplace;
    uint32_t clevel;
    uint32_t mode;          // PairMode
    cplx<R> u[4];           // u00 u01 u10 u11
};

template <typename R>
__global__ void __launch_bounds__(kBlock3) k3_pairs(RotArgs<R> A)
{
    const uint32_t stride = gridDim.x * kBlock3;
    for (uint32_t w = blockIdx.x * kBlock3 + threadIdx.x; w < A.work; w += stride) {
        const uint32_t hi = div_by(w, A.place, A.inv_place);
        const uint32_t lo = w - hi * A.place;
        const uint32_t i = hi * 3u * A.place + A.a * A.place + lo;
        if (A.cplace != 0) {
            const uint32_t qd = div_by(i, A.cplace, A.inv_cplace);
            if (qd - 3u * (qd / 3u) != A.clevel)
                continue;
        }
        const uint32_t j = i + (A.b - A.a) * A.place;
        const cplx<R> x = A.psi[i], y = A.psi[j];
        if (A.mode == kPairSwap) {
            A.psi[i] = y;
            A.psi[j] = x;
        } else if (A.mode == kPairNegB) {
            A.psi[j] = {-y.re, -y.im};
        } else {
            A.psi[i] = qsim::cmad2(A.u[0], x, A.u[1], y);
            A.psi[j] = qsim::cmad2(A.u[2], x, A.u[3], y);
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock3) k3_init(cplx<R> *psi, uint32_t n, uint32_t k)
{
    const uint32_t stride = gridDim.x * kBlock3;
    for (uint32_t i = blockIdx.x * kBlock3 + threadIdx.x; i < n; i += stride)
        psi[i] = {R(i == k ? 1 : 0), R(0)};
}

// ------------------------------------------------------------ fused passes
//
// A transformation only mixes amplitudes that differ in its ion's level, so
// for a set T of k ions the 3^k amplitudes that share the levels of every
// ion outside T (a tile) are closed under every transformation on an ion of
// T, and a condition on an ion outside T is a constant of the tile.  A pass
// applies a run of transformations whose ions lie in T tile by tile: a
// workgroup loads the tile into LDS, applies the run, and writes the tile
// back: one HBM read and write for the whole run instead of one per
// transformation.  T always holds the lowest ions, so a tile is runs of
// 3^low contiguous amplitudes.
//
// Inside the tile the run comes in groups of transformations on at most two
// tile ions A, B.  For a group each thread holds one register quantum: the 9
// amplitudes that share the levels of every other tile ion, register
// ra + 3 rb holding A at level ra and B at level rb.  A transformation of the
// group is then three register pairs (one where it is conditioned on the
// other group ion), with no LDS traffic and no barrier; the tile passes
// through LDS once per group instead of once per transformation.

// Four low ions: a tile is runs of 81 contiguous amplitudes (648 bytes of
// complex64); with three, the 216-byte runs straddled cache lines that
// neighbouring tiles share, and the pass ran 5 % slower for the same number
// of passes.
constexpr uint32_t kLowIons3 = 4;
template <typename R>
constexpr int kTileIons3 = sizeof(R) == 4 ? 8 : 7;   // 3^8 x 8 B = 51 KiB, 3^7 x 16 B = 34 KiB
template <typename R>
constexpr int kMaxRun3 = sizeof(R) == 4 ? 48 : 36;   // transformations per pass (4 KiB of arguments)

__host__ __device__ constexpr uint32_t pow3c(int e) { return e <= 0 ? 1u : 3u * pow3c(e - 1); }

// One thread per register quantum: 3^(k-2) quanta (729 complex64, 243 complex128).
template <typename R>
constexpr uint32_t kTileBlock3 = sizeof(R) == 4 ? 768u : 256u;

template <typename R>
struct Run3Op {
    cplx<R> u[4];        // u00 u01 u10 u11 (kPairMat)
    uint32_t place;      // 3^(tile position of the ion)
    uint32_t a, b;       // levels, a < b
    uint32_t mode;       // PairMode
    uint32_t cplace;     // condition ion inside the tile but outside the group: 3^its position, else 0
    uint32_t oplace;     // condition ion outside the tile: 3^ion, else 0
    uint32_t clevel;
    uint32_t shape;      // in its group: ion slot (0: A, 1: B) | level pair (0: 0-1, 1: 0-2,
                         // 2: 1-2) << 1 | conditioned on the other group ion << 3
    float inv_cplace;    // 1 / cplace
};

// Group word: first transformation (6 bits), count (6 bits), tile positions
// of A and B (4 bits each).
constexpr uint32_t kGroup3Count = 6, kGroup3A = 12, kGroup3B = 16;

template <typename R>
struct Tile3Args {
    cplx<R> *psi;
    uint32_t ntiles;            // 3^(M - k)
    uint32_t nout;              // ions outside the tile
    uint32_t nops;
    uint32_t ngroups;
    uint32_t tplace[kMaxIons];  // 3^ion of tile positions 0..k-1 (positions < low: ion = position)
    uint32_t oplace[kMaxIons];  // 3^ion of the ions outside the tile, ascending
    uint32_t group[kMaxRun3<R>];
    Run3Op<R> ops[kMaxRun3<R>];
};

static_assert(sizeof(Tile3Args<float>) <= 4096 && sizeof(Tile3Args<double>) <= 4096,
              "kernel arguments must fit 4 KiB");

// The pairs of one transformation in a quantum: ion slot S, levels LA < LB.
// C: conditioned on the other group ion (only its level clevel moves);
// W: conditioned on a tile ion outside the group, which `act` holds for this
// thread (applied everywhere with the identity where act is false, so no
// lane branches).
template <typename R, int S, int LA, int LB, bool W, bool C>
__device__ __forceinline__ void quantum_pairs(const Run3Op<R> &op, bool act, cplx<R> (&x)[9])
{
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        if (C && (uint32_t)o != op.clevel)
            continue;
        const int i = S == 0 ? LA + 3 * o : o + 3 * LA;
        const int j = S == 0 ? LB + 3 * o : o + 3 * LB;
        const cplx<R> p = x[i], q = x[j];
        if (op.mode == kPairSwap) {
            const bool s = !W || act;
            x[i] = {s ? q.re : p.re, s ? q.im : p.im};
            x[j] = {s ? p.re : q.re, s ? p.im : q.im};
        } else if (op.mode == kPairNegB) {
            const bool s = !W || act;
            x[j] = {s ? -q.re : q.re, s ? -q.im : q.im};
        } else if (op.mode == kPairRot) {
            // [[c, v], [-conj(v), c]], v = (va, vb)
            const R c = !W || act ? op.u[0].re : R(1);
            const R va = !W || act ? op.u[1].re : R(0), vb = !W || act ? op.u[1].im : R(0);
            x[i] = {c * p.re + va * q.re - vb * q.im, c * p.im + va * q.im + vb * q.re};
            x[j] = {c * q.re - va * p.re - vb * p.im, c * q.im - va * p.im + vb * p.re};
        } else if (op.mode == kPairDiag) {
            const cplx<R> d0 = {!W || act ? op.u[0].re : R(1), !W || act ? op.u[0].im : R(0)};
            const cplx<R> d1 = {!W || act ? op.u[3].re : R(1), !W || act ? op.u[3].im : R(0)};
            x[i] = qsim::cmul(d0, p);
            x[j] = qsim::cmul(d1, q);
        } else if (W) {
            const R one = R(1), zero = R(0);
            const cplx<R> u0 = {act ? op.u[0].re : one, act ? op.u[0].im : zero};
            const cplx<R> u1 = {act ? op.u[1].re : zero, act ? op.u[1].im : zero};
            const cplx<R> u2 = {act ? op.u[2].re : zero, act ? op.u[2].im : zero};
            const cplx<R> u3 = {act ? op.u[3].re : one, act ? op.u[3].im : zero};
            x[i] = qsim::cmad2(u0, p, u1, q);
            x[j] = qsim::cmad2(u2, p, u3, q);
        } else {
            x[i] = qsim::cmad2(op.u[0], p, op.u[1], q);
            x[j] = qsim::cmad2(op.u[2], p, op.u[3], q);
        }
    }
}

template <typename R, bool W>
__device__ __forceinline__ void quantum_op(const Run3Op<R> &op, bool act, cplx<R> (&x)[9])
{
    // conditioned on the other group ion or not: separate code, so the
    // unconditioned pairs carry no per-pair test
    switch (op.shape & 15u) {
    case 0: quantum_pairs<R, 0, 0, 1, W, false>(op, act, x); break;
    case 1: quantum_pairs<R, 1, 0, 1, W, false>(op, act, x); break;
    case 2: quantum_pairs<R, 0, 0, 2, W, false>(op, act, x); break;
    case 3: quantum_pairs<R, 1, 0, 2, W, false>(op, act, x); break;
    case 4: quantum_pairs<R, 0, 1, 2, W, false>(op, act, x); break;
    case 5: quantum_pairs<R, 1, 1, 2, W, false>(op, act, x); break;
    case 8: quantum_pairs<R, 0, 0, 1, W, true>(op, act, x); break;
    case 9: quantum_pairs<R, 1, 0, 1, W, true>(op, act, x); break;
    case 10: quantum_pairs<R, 0, 0, 2, W, true>(op, act, x); break;
    case 11: quantum_pairs<R, 1, 0, 2, W, true>(op, act, x); break;
    case 12: quantum_pairs<R, 0, 1, 2, W, true>(op, act, x); break;
    default: quantum_pairs<R, 1, 1, 2, W, true>(op, act, x); break;
    }
}

// Powers of three, read with uniform indices (scalar loads).
__constant__ uint32_t c_pow3[16] = {1u, 3u, 9u, 27u, 81u, 243u, 729u, 2187u, 6561u, 19683u,
                                    59049u, 177147u, 531441u, 1594323u, 4782969u, 14348907u};

// One transformation of a group on the thread's quantum (bt: tile index of
// its register 0).
template <typename R>
__device__ __forceinline__ void group_op(const Run3Op<R> &desc, uint32_t base, uint32_t bt,
                                         cplx<R> (&x)[9])
{
    // the whole descriptor at once (one scalar wait), not a kernel-argument
    // load at each use
    const Run3Op<R> op = desc;
    if (op.oplace != 0 && (base / op.oplace) % 3u != op.clevel)
        return;  // uniform over the workgroup: the condition is off for this tile
    if (op.cplace == 0) {
        quantum_op<R, false>(op, true, x);
    } else {
        // bt < 3^8: the FP32 quotient is off by at most one, which the
        // remainder corrects
        uint32_t q = (uint32_t)((float)bt * op.inv_cplace);
        const int r = (int)bt - (int)(q * op.cplace);
        q = r < 0 ? q - 1u : (r >= (int)op.cplace ? q + 1u : q);
        quantum_op<R, true>(op, q - 3u * (q / 3u) == op.clevel, x);
    }
}

// One amplitude of the LDS tile at its natural alignment (the struct only
// promises that of its component, and the compiler then splits the access).
__device__ __forceinline__ cplx<float> lds_get(const cplx<float> *p)
{
    const float2 v = *static_cast<const float2 *>(__builtin_assume_aligned(p, 8));
    return {v.x, v.y};
}
__device__ __forceinline__ void lds_put(cplx<float> *p, cplx<float> a)
{
    *static_cast<float2 *>(__builtin_assume_aligned(p, 8)) = make_float2(a.re, a.im);
}
__device__ __forceinline__ cplx<double> lds_get(const cplx<double> *p)
{
    const double2 v = *static_cast<const double2 *>(__builtin_assume_aligned(p, 16));
    return {v.x, v.y};
}
__device__ __forceinline__ void lds_put(cplx<double> *p, cplx<double> a)
{
    *static_cast<double2 *>(__builtin_assume_aligned(p, 16)) = make_double2(a.re, a.im);
}

template <typename R>
__global__ void __launch_bounds__(kTileBlock3<R>) k3_tile(const Tile3Args<R> A)
{
    constexpr int K = kTileIons3<R>;
    constexpr uint32_t T = kTileBlock3<R>;
    constexpr uint32_t N = pow3c(K), L = pow3c(kLowIons3), H = pow3c(K - kLowIons3), NQ = N / 9u;
    __shared__ cplx<R> t[N];
    __shared__ uint32_t offhi[H];
    // offset of tile element e from the tile's base: e % L covers the low
    // ions (contiguous), offhi[e / L] the others
    for (uint32_t h = threadIdx.x; h < H; h += T) {
        uint32_t off = 0, v = h;
        for (int j = kLowIons3; j < K; ++j) {
            const uint32_t q = v / 3u;
            off += (v - 3u * q) * A.tplace[j];
            v = q;
        }
        offhi[h] = off;
    }
    // the thread number's base-3 digits: a group places them on the tile
    // positions other than its own two, in ascending order
    uint32_t dig[K - 2];
    {
        uint32_t v = threadIdx.x < NQ ? threadIdx.x : NQ - 1u;
#pragma unroll
        for (int j = 0; j < K - 2; ++j) {
            const uint32_t q = v / 3u;
            dig[j] = v - 3u * q;
            v = q;
        }
    }
    __syncthreads();
    const uint32_t per = (A.ntiles + gridDim.x - 1) / gridDim.x;
    const uint32_t t0 = blockIdx.x * per;
    const uint32_t t1 = t0 + per < A.ntiles ? t0 + per : A.ntiles;
    for (uint32_t tile = t0; tile < t1; ++tile) {
        uint32_t base = 0, v = tile;
        for (uint32_t m = 0; m < A.nout; ++m) {
            const uint32_t q = v / 3u;
            base += (v - 3u * q) * A.oplace[m];
            v = q;
        }
        // whole batches of loads in flight at once, then into LDS; the tail
        // element by element
        constexpr uint32_t U = 8, NB = N / (U * T) * (U * T);
        for (uint32_t e0 = 0; e0 < NB; e0 += U * T) {
            cplx<R> v[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t e = e0 + u * T + threadIdx.x;
                v[u] = A.psi[base + e % L + offhi[e / L]];
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                t[e0 + u * T + threadIdx.x] = v[u];
        }
#pragma unroll 8
        for (uint32_t e = NB + threadIdx.x; e < N; e += T)
            t[e] = A.psi[base + e % L + offhi[e / L]];
        __syncthreads();
        for (uint32_t g = 0; g < A.ngroups; ++g) {
            const uint32_t gw = A.group[g];
            const uint32_t pa = (gw >> kGroup3A) & 15u, pb = (gw >> kGroup3B) & 15u;
            const uint32_t first = gw & 63u, end = first + ((gw >> kGroup3Count) & 63u);
            {
                // tile index of register 0: digit j on the j-th tile position
                // other than pa < pb (the places are uniform)
                const uint32_t PA = c_pow3[pa], PB = c_pow3[pb];
                uint32_t bt = 0;
#pragma unroll
                for (int j = 0; j < K - 2; ++j) {
                    uint32_t p = (uint32_t)j;
                    p += p >= pa ? 1u : 0u;
                    p += p >= pb ? 1u : 0u;
                    bt += dig[j] * c_pow3[p];
                }
                cplx<R> x[9];
#pragma unroll
                for (int r = 0; r < 9; ++r)
                    x[r] = lds_get(t + bt + (uint32_t)(r % 3) * PA + (uint32_t)(r / 3) * PB);
                // two transformations per trip: the second writes its results
                // back into the registers the first read, so no copy of the
                // quantum closes each trip
                for (uint32_t o = first; o < end; o += 2) {
                    group_op<R>(A.ops[o], base, bt, x);
                    if (o + 1 >= end)
                        break;
                    group_op<R>(A.ops[o + 1], base, bt, x);
                }
                // the threads past the last quantum (complex64: 729 of 768)
                // worked on a copy of the last one and write nothing
                if (threadIdx.x < NQ) {
#pragma unroll
                    for (int r = 0; r < 9; ++r)
                        lds_put(t + bt + (uint32_t)(r % 3) * PA + (uint32_t)(r / 3) * PB, x[r]);
                }
            }
            __syncthreads();
        }
#pragma unroll 8
        for (uint32_t e = threadIdx.x; e < N; e += T)
            A.psi[base + e % L + offhi[e / L]] = t[e];
        __syncthreads();
    }
}

__device__ __forceinline__ double wave_sum3(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order block sums of NV values (lanes, then waves in order).
template <int NV>
__device__ __forceinline__ void block_sum3(double (&v)[NV], double (*scratch)[kBlock3 / 64])
{
#pragma unroll
    for (int c = 0; c < NV; ++c)
        v[c] = wave_sum3(v[c]);
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c)
            scratch[c][threadIdx.x >> 6] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0.0;
            for (int w = 0; w < kBlock3 / 64; ++w)
                s += scratch[c][w];
            v[c] = s;
        }
    }
}

// <a|b>, <a|a>, <b|b>: block b sums elements [b chunk, (b + 1) chunk).
template <typename Ra, typename Rb>
__global__ void __launch_bounds__(kBlock3) k3_overlap(const cplx<Ra> *a, const cplx<Rb> *b,
                                                      uint32_t n, uint32_t chunk, double *partial)
{
    __shared__ double scratch[4][kBlock3 / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t lo = blockIdx.x * chunk, hi = std::min(n, lo + chunk);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock3) {
        const double ar = a[i].re, ai = a[i].im, br = b[i].re, bi = b[i].im;
        v[0] += ar * br + ai * bi;
        v[1] += ar * bi - ai * br;
        v[2] += ar * ar + ai * ai;
        v[3] += br * br + bi * bi;
    }
    block_sum3<4>(v, scratch);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c)
            partial[4 * blockIdx.x + c] = v[c];
}

__global__ void __launch_bounds__(kBlock3) k3_finish(const double *partial, uint32_t nblocks,
                                                     uint32_t width, double *out)
{
    // out[c] = sum over blocks of partial[width * blk + c], c < width, in
    // block order (one thread per entry)
    for (uint32_t c = threadIdx.x; c < width; c += kBlock3) {
        double s = 0.0;
        for (uint32_t blk = 0; blk < nblocks; ++blk)
            s += partial[(uint64_t)width * blk + c];
        out[c] = s;
    }
}

// Marginal probabilities over up to six ions: block b bins elements
// [b chunk, (b + 1) chunk) into LDS, thread by thread in a fixed order, and
// writes its 3^m bins.
// The same for at most three ions (27 bins): thread t takes elements lo + t,
// lo + t + 256, ... of the block's chunk in that order into bins of its own
// in LDS, and the block then adds each bin over the threads in thread order.
constexpr uint32_t kFastMarginalBins = 27;

template <typename R>
__global__ void __launch_bounds__(kBlock3) k3_marginal_few(const cplx<R> *psi, uint32_t n,
                                                           uint32_t chunk, uint32_t m,
                                                           const uint32_t *places,
                                                           double *partial)
{
    __shared__ double tb[kFastMarginalBins * kBlock3];
    uint32_t nb = 1, pl[3] = {1, 1, 1};
    double inv[3] = {1.0, 1.0, 1.0};
    for (uint32_t j = 0; j < m; ++j) {
        nb *= 3;
        pl[j] = places[j];
        inv[j] = 1.0 / (double)pl[j];
    }
    for (uint32_t c = 0; c < nb; ++c)
        tb[c * kBlock3 + threadIdx.x] = 0.0;
    const uint32_t lo = blockIdx.x * chunk, hi = std::min(n, lo + chunk);
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock3) {
        const double p = (double)psi[i].re * psi[i].re + (double)psi[i].im * psi[i].im;
        uint32_t key = 0, kp = 1;
        for (uint32_t j = 0; j < m; ++j) {
            const uint32_t q = div_by(i, pl[j], inv[j]);
            key += (q - 3u * (q / 3u)) * kp;
            kp *= 3;
        }
        tb[key * kBlock3 + threadIdx.x] += p;
    }
    __syncthreads();
    for (uint32_t c = threadIdx.x; c < nb; c += kBlock3) {
        double s = 0.0;
        for (uint32_t t = 0; t < kBlock3; ++t)
            s += tb[c * kBlock3 + t];
        partial[(uint64_t)nb * blockIdx.x + c] = s;
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock3) k3_marginal(const cplx<R> *psi, uint32_t n,
                                                       uint32_t chunk, uint32_t m,
                                                       const uint32_t *places, double *partial)
{
    __shared__ double bins[729];
    __shared__ double tbins[kBlock3];
    __shared__ uint32_t keys[kBlock3];
    uint32_t nb = 1;
    for (uint32_t j = 0; j < m; ++j)
        nb *= 3;
    for (uint32_t c = threadIdx.x; c < nb; c += kBlock3)
        bins[c] = 0.0;
    __syncthreads();
    const uint32_t lo = blockIdx.x * chunk, hi = std::min(n, lo + chunk);
    // each pass: every thread takes one element, then thread 0 adds them in
    // thread order (deterministic, no atomics)
    for (uint32_t base = lo; base < hi; base += kBlock3) {
        const uint32_t i = base + threadIdx.x;
        uint32_t key = 0;
        double p = 0.0;
        if (i < hi) {
            p = (double)psi[i].re * psi[i].re + (double)psi[i].im * psi[i].im;
            uint32_t kp = 1;
            for (uint32_t j = 0; j < m; ++j) {
                const uint32_t d = (i / places[j]) % 3u;
                key += d * kp;
                kp *= 3;
            }
        }
        tbins[threadIdx.x] = p;
        keys[threadIdx.x] = key;
        __syncthreads();
        if (threadIdx.x == 0)
            for (int t = 0; t < kBlock3 && base + t < hi; ++t)
                bins[keys[t]] += tbins[t];
        __syncthreads();
    }
    for (uint32_t c = threadIdx.x; c < nb; c += kBlock3)
        partial[(uint64_t)nb * blockIdx.x + c] = bins[c];
}

template <typename R>
__global__ void __launch_bounds__(kBlock3) k3_to_f64(const cplx<R> *psi, uint32_t count,
                                                     double *out)
{
    const uint32_t stride = gridDim.x * kBlock3;
    for (uint32_t i = blockIdx.x * kBlock3 + threadIdx.x; i < count; i += stride) {
        out[2 * i] = psi[i].re;
        out[2 * i + 1] = psi[i].im;
    }
}

// ---------------------------------------------------------------- lowering

enum : uint32_t { kPulseRot = 0, kPulsePhase = 1 };
constexpr double kPi = 3.14159265358979323846;

struct Lowering {
    std::vector<qsim3_pulse> out;
    void rot(int ion, int a, int b, double th, double ph, int cion = -1, int clev = 0)
    {
        out.push_back({kPulseRot, ion, a, b, cion, clev, th, ph});
    }
    void phase(int ion, double th) { out.push_back({kPulsePhase, ion, 0, 1, -1, 0, th, 0.0}); }
    void cnot(int c, int x)
    {
        rot(x, 0, 1, kPi / 2, kPi / 2);
        rot(c, 1, 2, kPi, 0.0);
        rot(x, 1, 2, 2 * kPi, 0.0, c, 2);
        rot(c, 1, 2, kPi, kPi);
        rot(x, 0, 1, kPi / 2, -kPi / 2);
    }
    void h(int x)
    {
        rot(x, 0, 1, kPi / 2, -kPi / 2);
        rot(x, 0, 1, kPi, 0.0);
    }
    void gate(const qsim_gate &g)
    {
        const int x = g.target, c0 = g.ctrl0, c1 = g.ctrl1;
        switch (g.kind) {
        case QSIM_X: rot(x, 0, 1, kPi, 0.0); break;
        case QSIM_H: h(x); break;
        case QSIM_RZ: phase(x, g.theta); break;
        case QSIM_Z: phase(x, kPi); break;
        case QSIM_CNOT: cnot(c0, x); break;
        case QSIM_CPHASE:
            phase(c0, 0.5 * g.theta);
            phase(x, 0.5 * g.theta);
            cnot(c0, x);
            phase(x, -0.5 * g.theta);
            cnot(c0, x);
            break;
        default:  // Toffoli
            h(x);
            cnot(c1, x); phase(x, -kPi / 4);
            cnot(c0, x); phase(x, kPi / 4);
            cnot(c1, x); phase(x, -kPi / 4);
            cnot(c0, x); phase(c1, kPi / 4); phase(x, kPi / 4);
            h(x);
            cnot(c0, c1); phase(c0, kPi / 4); phase(c1, -kPi / 4);
            cnot(c0, c1);
            break;
        }
    }
};

// 2x2 of a transformation with its angle error, FP64, as u00 u01 u10 u11.
void pulse_matrix(const qsim3_pulse &p, double eps, double (&u)[8])
{
    const double th = p.theta + eps, c = std::cos(0.5 * th), s = std::sin(0.5 * th);
    std::memset(u, 0, sizeof(u));
    if (p.kind == kPulsePhase) {
        u[0] = c; u[1] = -s; u[6] = c; u[7] = s;
        return;
    }
    u[0] = c;
    u[2] = s * std::sin(p.phi); u[3] = -s * std::cos(p.phi);
    u[4] = -s * std::sin(p.phi); u[5] = -s * std::cos(p.phi);
    u[6] = c;
}

double pulse_eps(const qsim_error_model &em, uint64_t step, uint64_t k)
{
    const qsim::u64x4 r = qsim::philox4x64_10(step, k, 3, 0, em.seed, em.trial);
    const double u1 = ((double)(r.w[0] >> 32) + 0.5) * 0x1p-32;
    const double u2 = ((double)(r.w[1] >> 32) + 0.5) * 0x1p-32;
    return em.sigma * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586476925286766559 * u2);
}

bool pulse_valid(const qsim3_pulse &p, int M)
{
    if (p.kind > kPulsePhase || p.ion < 0 || p.ion >= M || p.a < 0 || p.b > 2 || p.a >= p.b)
        return false;
    if (p.cond_ion != -1 && (p.cond_ion < 0 || p.cond_ion >= M || p.cond_ion == p.ion ||
                             p.cond_level < 0 || p.cond_level > 2))
        return false;
    return std::isfinite(p.theta) && std::isfinite(p.phi);
}

}  // namespace

// ------------------------------------------------------------------- state

struct qsim3_state {
    int M = 0;
    int dtype = QSIM_C64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *psi = nullptr;
    uint64_t n = 0;
    uint64_t step = 0;
    bool armed = false;
    qsim_error_model em{};
    double *d_partial = nullptr;   // 729 * kReduceBlocks3 doubles
    double *d_out = nullptr;       // 729 doubles
    uint32_t *d_places = nullptr;  // marginal ions' place values
    double *d_stage = nullptr;
    size_t stage_bytes = 0;
    uint64_t pulses = 0;
    uint64_t launches = 0;   // state kernel launches (fused passes or per transformation)
    bool per_pulse = false;  // exec_mode 1: one launch per transformation
    bool in_order = false;   // exec_mode 2: fused passes over runs of the stream
};

namespace {

int fail3(int code, const char *what, hipError_t e)
{
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory)
        return qsim::set_error(QSIM_ENOMEM, "%s: out of device memory", what);
    return qsim::set_error(code, "%s: %s", what, hipGetErrorString(e));
}

#define HIP3(expr, what)                              \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess)                         \
            return fail3(QSIM_EDEVICE, what, e_);     \
    } while (0)

size_t esize(int dtype) { return dtype == QSIM_C64 ? 8 : 16; }

// One transformation (or exact flip) on the register.
template <typename R>
hipError_t launch_pairs(qsim3_state *s, int ion, int a, int b, int cion, int clev, uint32_t mode,
                        const double (&u)[8])
{
    RotArgs<R> A{};
    A.psi = static_cast<cplx<R> *>(s->psi);
    A.work = (uint32_t)(s->n / 3);
    A.place = (uint32_t)pow3(ion);
    A.inv_place = 1.0 / (double)A.place;
    A.a = (uint32_t)a;
    A.b = (uint32_t)b;
    A.cplace = cion >= 0 ? (uint32_t)pow3(cion) : 0u;
    A.inv_cplace = cion >= 0 ? 1.0 / (double)A.cplace : 0.0;
    A.clevel = (uint32_t)clev;
    A.mode = mode;
    for (int k = 0; k < 4; ++k)
        A.u[k] = {(R)u[2 * k], (R)u[2 * k + 1]};
    hipLaunchKernelGGL((k3_pairs<R>), grid3(A.work), dim3(kBlock3), 0, s->stream, A);
    return hipGetLastError();
}

hipError_t pairs(qsim3_state *s, int ion, int a, int b, int cion, int clev, uint32_t mode,
                 const double (&u)[8])
{
    return s->dtype == QSIM_C64 ? launch_pairs<float>(s, ion, a, b, cion, clev, mode, u)
                                : launch_pairs<double>(s, ion, a, b, cion, clev, mode, u);
}

// One transformation (or exact flip) with its FP64 matrix, ready to launch.
struct Xform {
    int ion, a, b, cion, clevel;
    uint32_t mode;
    double u[8];
};

Xform make_pulse(const qsim3_pulse &p, double eps)
{
    Xform x{p.ion, p.a, p.b, p.cond_ion, p.cond_level, kPairMat, {}};
    pulse_matrix(p, eps, x.u);
    return x;
}

Xform make_flip(int ion, uint32_t mode)
{
    return Xform{ion, 0, 1, -1, 0, mode, {1, 0, 0, 0, 0, 0, 1, 0}};
}

// A run of transformations as one fused pass: tile ions T (the low ions,
// then the run's ions in ascending order), the rest enumerate the tiles.
// The run is reordered into register groups of at most two tile ions:
// sweeps over the transformations left take, in order, each one that
// commutes with the ones the sweep skipped and whose ion fits the group (the
// same rule as the pass itself, so the order stays exact).
template <typename R>
hipError_t launch_run(qsim3_state *s, const Xform *x, size_t n, const std::vector<int> &T)
{
    Tile3Args<R> A{};
    A.psi = static_cast<cplx<R> *>(s->psi);
    const int M = s->M, K = kTileIons3<R>;
    if (n == 0 || n > (size_t)kMaxRun3<R>)
        return hipErrorInvalidValue;
    int pos_of[kMaxIons];
    for (int q = 0; q < M; ++q)
        pos_of[q] = -1;
    for (int j = 0; j < K; ++j) {
        A.tplace[j] = (uint32_t)pow3(T[j]);
        pos_of[T[j]] = j;
    }
    A.nout = 0;
    for (int q = 0; q < M; ++q)
        if (pos_of[q] < 0)
            A.oplace[A.nout++] = (uint32_t)pow3(q);
    A.ntiles = (uint32_t)pow3(M - K);
    A.nops = (uint32_t)n;
    A.ngroups = 0;

    std::vector<size_t> rem(n), left;
    for (size_t i = 0; i < n; ++i)
        rem[i] = i;
    uint32_t nout = 0;
    while (!rem.empty()) {
        uint32_t gpos = 0;  // tile positions of the group
        int ng = 0;
        uint64_t bx = 0, bz = 0;
        const uint32_t first = nout;
        left.clear();
        std::vector<size_t> taken;
        for (const size_t idx : rem) {
            const Xform &t = x[idx];
            if (pos_of[t.ion] < 0)
                return hipErrorInvalidValue;
            const uint64_t ux = 1ull << t.ion, uz = t.cion >= 0 ? (1ull << t.cion) : 0ull;
            const uint32_t pbit = 1u << pos_of[t.ion];
            bool ok = (ux & (bx | bz)) == 0 && (uz & bx) == 0;
            if (ok && !(gpos & pbit)) {
                if (ng == 2) {
                    ok = false;
                } else {
                    gpos |= pbit;
                    ++ng;
                }
            }
            if (ok) {
                taken.push_back(idx);
            } else {
                left.push_back(idx);
                bx |= ux;
                bz |= uz;
            }
        }
        if (ng == 1)
            gpos |= (gpos & 1u) ? 2u : 1u;  // any other tile position
        // pa < pb, as the kernel places the thread's digits around them
        const uint32_t pa = (uint32_t)__builtin_ctz(gpos);
        const uint32_t pb = (uint32_t)__builtin_ctz(gpos & (gpos - 1));
        for (const size_t idx : taken) {
            const Xform &t = x[idx];
            Run3Op<R> &op = A.ops[nout++];
            const uint32_t pos = (uint32_t)pos_of[t.ion];
            op.place = pow3c((int)pos);
            op.a = (uint32_t)t.a;
            op.b = (uint32_t)t.b;
            op.mode = t.mode;
            if (t.mode == kPairMat) {
                const cplx<R> u00 = {(R)t.u[0], (R)t.u[1]}, u01 = {(R)t.u[2], (R)t.u[3]};
                const cplx<R> u10 = {(R)t.u[4], (R)t.u[5]}, u11 = {(R)t.u[6], (R)t.u[7]};
                if (u01.re == R(0) && u01.im == R(0) && u10.re == R(0) && u10.im == R(0))
                    op.mode = kPairDiag;
                else if (u00.im == R(0) && u11.im == R(0) && u00.re == u11.re &&
                         u10.re == -u01.re && u10.im == u01.im)
                    op.mode = kPairRot;
            }
            op.cplace = 0;
            op.oplace = 0;
            op.clevel = (uint32_t)t.clevel;
            op.inv_cplace = 0.0f;
            const uint32_t lv = t.a == 0 ? (t.b == 1 ? 0u : 1u) : 2u;
            op.shape = (pos == pa ? 0u : 1u) | lv << 1;
            if (t.cion >= 0) {
                const int cp = pos_of[t.cion];
                if (cp < 0) {
                    op.oplace = (uint32_t)pow3(t.cion);
                } else if ((uint32_t)cp == pa || (uint32_t)cp == pb) {
                    op.shape |= 8u;  // the other group ion
                } else {
                    op.cplace = pow3c(cp);
                    op.inv_cplace = 1.0f / (float)op.cplace;
                }
            }
            for (int k = 0; k < 4; ++k)
                op.u[k] = {(R)t.u[2 * k], (R)t.u[2 * k + 1]};
        }
        A.group[A.ngroups++] = first | (nout - first) << kGroup3Count | pa << kGroup3A |
                               pb << kGroup3B;
        rem.swap(left);
    }
    const uint32_t grid = std::min<uint32_t>(A.ntiles, 256u * 8u);
    hipLaunchKernelGGL((k3_tile<R>), dim3(grid), dim3(kTileBlock3<R>), 0, s->stream, A);
    return hipGetLastError();
}

// Fused passes over the tile ions T (K ions, the lowest always among them).
// Two transformations commute when they act on different ions and neither
// acts on the ion the other is conditioned on (a condition only reads its
// ion's level), so a pass may take a transformation from further down the
// stream when it commutes with every earlier one left behind: exact up to
// rounding, and it lets one HBM pass carry several gates' worth of
// transformations.  T is chosen by lookahead (the same rule as the two-level
// passes); in-order mode (exec_mode 2) takes runs of the stream instead.
constexpr size_t kWindow3 = 64;
constexpr int kMaxExchanges3 = 4;

template <typename R>
int launch_ions(qsim3_state *s, const Xform *x, size_t n, uint32_t in)
{
    const int K = kTileIons3<R>;
    int nin = __builtin_popcount(in);
    // fill T to K ions with the lowest ions not yet in it
    for (int q = 0; q < s->M && nin < K; ++q)
        if (!(in & (1u << q))) {
            in |= 1u << q;
            ++nin;
        }
    std::vector<int> T;
    for (int q = 0; q < s->M; ++q)
        if (in & (1u << q))
            T.push_back(q);
    HIP3(launch_run<R>(s, x, n, T), "fused pass");
    ++s->launches;
    return QSIM_OK;
}

int launch_ions_any(qsim3_state *s, const Xform *x, size_t n, uint32_t in)
{
    return s->dtype == QSIM_C64 ? launch_ions<float>(s, x, n, in) : launch_ions<double>(s, x, n, in);
}

// Apply transformations: fused passes on registers larger than a tile
// (exec_mode other than 1), else one launch each in stream order.
int apply_xforms(qsim3_state *s, const std::vector<Xform> &xs)
{
    const int K = s->dtype == QSIM_C64 ? kTileIons3<float> : kTileIons3<double>;
    const size_t cap = s->dtype == QSIM_C64 ? (size_t)kMaxRun3<float> : (size_t)kMaxRun3<double>;
    if (s->per_pulse || s->M <= K) {
        for (const Xform &x : xs) {
            HIP3(pairs(s, x.ion, x.a, x.b, x.cion, x.clevel, x.mode, x.u), "transformation");
            ++s->launches;
        }
        return QSIM_OK;
    }
    const uint32_t low = (1u << kLowIons3) - 1;
    if (s->in_order) {
        size_t i = 0;
        while (i < xs.size()) {
            uint32_t in = low;
            int nin = (int)kLowIons3;
            size_t j = i;
            for (; j < xs.size() && j - i < cap; ++j) {
                const uint32_t bit = 1u << xs[j].ion;
                if (!(in & bit)) {
                    if (nin == K)
                        break;
                    in |= bit;
                    ++nin;
                }
            }
            const int rc = launch_ions_any(s, &xs[i], j - i, in);
            if (rc != QSIM_OK)
                return rc;
            i = j;
        }
        return QSIM_OK;
    }
    std::vector<qsim::ScanOp> all(xs.size());
    for (size_t i = 0; i < xs.size(); ++i) {
        const uint64_t t = 1ull << xs[i].ion;
        all[i] = {t, xs[i].cion >= 0 ? (1ull << xs[i].cion) : 0ull, t};
    }
    std::vector<uint32_t> rem(xs.size()), left;
    for (size_t i = 0; i < xs.size(); ++i)
        rem[i] = (uint32_t)i;
    std::vector<qsim::ScanOp> w;
    std::vector<Xform> run;
    while (!rem.empty()) {
        w.clear();
        for (size_t i = 0; i < rem.size() && i < kWindow3; ++i)
            w.push_back(all[rem[i]]);
        uint64_t in = qsim::lookahead_set(w, low, K, cap, kMaxExchanges3);
        int nin = __builtin_popcountll(in);
        uint64_t bx = 0, bz = 0;
        run.clear();
        left.clear();
        for (const uint32_t r : rem) {
            const qsim::ScanOp &u = all[r];
            bool ok = run.size() < cap && (u.x & (bx | bz)) == 0 && (u.z & bx) == 0;
            if (ok && !(in & u.t)) {
                if (nin == K) {
                    ok = false;
                } else {
                    in |= u.t;
                    ++nin;
                }
            }
            if (ok) {
                run.push_back(xs[r]);
            } else {
                left.push_back(r);
                bx |= u.x;
                bz |= u.z;
            }
        }
        // the first transformation left commutes with nothing before it and
        // the window's best set takes at least one, so every pass does work
        if (run.empty())
            return qsim::set_error(QSIM_EDEVICE, "three-state scheduler: internal error (empty pass)");
        const int rc = launch_ions_any(s, run.data(), run.size(), (uint32_t)in);
        if (rc != QSIM_OK)
            return rc;
        rem.swap(left);
    }
    return QSIM_OK;
}

void release3(qsim3_state *s)
{
    if (s == nullptr)
        return;
    (void)hipSetDevice(s->device);
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    if (s->psi)
        (void)hipFree(s->psi);
    if (s->d_partial)
        (void)hipFree(s->d_partial);
    if (s->d_out)
        (void)hipFree(s->d_out);
    if (s->d_places)
        (void)hipFree(s->d_places);
    if (s->d_stage)
        (void)hipFree(s->d_stage);
    if (s->own_stream && s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
}

int ensure_stage3(qsim3_state *s, size_t bytes)
{
    if (s->stage_bytes >= bytes)
        return QSIM_OK;
    HIP3(hipStreamSynchronize(s->stream), "stage sync");
    if (s->d_stage)
        (void)hipFree(s->d_stage);
    s->d_stage = nullptr;
    s->stage_bytes = 0;
    HIP3(hipMalloc((void **)&s->d_stage, bytes), "stage");
    s->stage_bytes = bytes;
    return QSIM_OK;
}

int validate3(const qsim3_state *s, const qsim_gate *g, size_t n)
{
    if (n > 0 && g == nullptr)
        return qsim::set_error(QSIM_EINVAL, "gates is NULL");
    char why[160];
    for (size_t k = 0; k < n; ++k)
        if (!qsim::gate_valid(g[k], s->M, why, sizeof(why)))
            return qsim::set_error(QSIM_EINVAL, "gate %zu: %s", k, why);
    return QSIM_OK;
}

}  // namespace

// ===================================================================== C ABI

extern "C" {

int qsim3_create(int num_ions, int dtype, const qsim_options *opt, qsim3_state **out)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (out == nullptr)
            return qsim::set_error(QSIM_EINVAL, "out is NULL");
        *out = nullptr;
        if (num_ions < 1 || num_ions > kMaxIons)
            return qsim::set_error(QSIM_EINVAL, "num_ions %d outside [1, %d]", num_ions, kMaxIons);
        if (dtype != QSIM_C64 && dtype != QSIM_C128)
            return qsim::set_error(QSIM_EINVAL, "dtype %d", dtype);
        qsim_options o{};
        if (opt)
            o = *opt;
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess)
            return fail3(QSIM_EDEVICE, "hipGetDeviceCount", e);
        if (o.device < 0 || o.device >= ndev)
            return qsim::set_error(QSIM_EINVAL, "device %d outside [0, %d)", o.device, ndev);
        qsim3_state *s = new (std::nothrow) qsim3_state();
        if (s == nullptr)
            return qsim::set_error(QSIM_ENOMEM, "qsim3_create: host memory exhausted");
        s->M = num_ions;
        s->dtype = dtype;
        s->device = o.device;
        s->n = pow3(num_ions);
        s->per_pulse = o.exec_mode == 1;
        s->in_order = o.exec_mode == 2;
        e = hipSetDevice(o.device);
        if (e == hipSuccess) {
            if (o.hip_stream) {
                s->stream = static_cast<hipStream_t>(o.hip_stream);
            } else {
                e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
                s->own_stream = e == hipSuccess;
            }
        }
        if (e == hipSuccess)
            e = hipMalloc(&s->psi, s->n * esize(dtype));
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->d_partial, 729 * kReduceBlocks3 * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->d_out, 729 * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->d_places, kMaxMarginalIons * sizeof(uint32_t));
        if (e == hipSuccess) {
            if (dtype == QSIM_C64)
                hipLaunchKernelGGL((k3_init<float>), grid3(s->n), dim3(kBlock3), 0, s->stream,
                                   (cplx<float> *)s->psi, (uint32_t)s->n, 0u);
            else
                hipLaunchKernelGGL((k3_init<double>), grid3(s->n), dim3(kBlock3), 0, s->stream,
                                   (cplx<double> *)s->psi, (uint32_t)s->n, 0u);
            e = hipGetLastError();
        }
        if (e != hipSuccess) {
            const int rc = fail3(QSIM_EDEVICE, "qsim3_create", e);
            release3(s);
            return rc;
        }
        *out = s;
        return QSIM_OK;
    });
}

int qsim3_destroy(qsim3_state *s)
{
    return qsim::guarded(__func__, [&]() -> int {
        release3(s);
        return QSIM_OK;
    });
}

int qsim3_reset(qsim3_state *s, uint64_t basis_index)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return qsim::set_error(QSIM_EINVAL, "state is NULL");
        if (basis_index >= s->n)
            return qsim::set_error(QSIM_ERANGE, "basis index %llu >= 3^%d",
                                   (unsigned long long)basis_index, s->M);
        HIP3(hipSetDevice(s->device), "hipSetDevice");
        if (s->dtype == QSIM_C64)
            hipLaunchKernelGGL((k3_init<float>), grid3(s->n), dim3(kBlock3), 0, s->stream,
                               (cplx<float> *)s->psi, (uint32_t)s->n, (uint32_t)basis_index);
        else
            hipLaunchKernelGGL((k3_init<double>), grid3(s->n), dim3(kBlock3), 0, s->stream,
                               (cplx<double> *)s->psi, (uint32_t)s->n, (uint32_t)basis_index);
        HIP3(hipGetLastError(), "init");
        s->step = 0;
        return QSIM_OK;
    });
}

int qsim3_inject_errors(qsim3_state *s, const qsim_error_model *em)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return qsim::set_error(QSIM_EINVAL, "state is NULL");
        if (em == nullptr) {
            s->armed = false;
            return QSIM_OK;
        }
        if (!qsim::error_model_valid(*em))
            return qsim::set_error(QSIM_EINVAL, "bad error model");
        s->em = *em;
        s->armed = true;
        return QSIM_OK;
    });
}

int qsim3_lower(const qsim_gate *gates, size_t n, int num_ions, qsim3_pulse *out, size_t cap,
                size_t *n_pulses)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (num_ions < 1 || num_ions > kMaxIons)
            return qsim::set_error(QSIM_EINVAL, "num_ions %d", num_ions);
        qsim3_state probe;
        probe.M = num_ions;
        int rc = validate3(&probe, gates, n);
        if (rc != QSIM_OK)
            return rc;
        Lowering L;
        for (size_t k = 0; k < n; ++k)
            L.gate(gates[k]);
        if (n_pulses)
            *n_pulses = L.out.size();
        for (size_t i = 0; i < L.out.size() && i < cap && out != nullptr; ++i)
            out[i] = L.out[i];
        return QSIM_OK;
    });
}

int qsim3_apply_circuit(qsim3_state *s, const qsim_gate *gates, size_t n)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return qsim::set_error(QSIM_EINVAL, "state is NULL");
        int rc = validate3(s, gates, n);
        if (rc != QSIM_OK)
            return rc;
        HIP3(hipSetDevice(s->device), "hipSetDevice");
        const bool ang = s->armed && s->em.sigma > 0.0;
        const bool flips = s->armed && (s->em.p_bitflip > 0.0 || s->em.p_phaseflip > 0.0);
        const uint64_t tb = flips ? qsim::flip_threshold(s->em.p_bitflip) : 0;
        const uint64_t tp = flips ? qsim::flip_threshold(s->em.p_phaseflip) : 0;
        std::vector<Xform> xs;
        uint64_t npulses = 0;
        for (size_t k = 0; k < n; ++k) {
            const uint64_t step = s->step + k;
            Lowering L;
            L.gate(gates[k]);
            for (size_t j = 0; j < L.out.size(); ++j)
                xs.push_back(make_pulse(L.out[j], ang ? pulse_eps(s->em, step, j) : 0.0));
            npulses += L.out.size();
            if (!flips)
                continue;
            for (int q = 0; q < s->M; ++q) {
                const qsim::u64x4 r = qsim::philox4x64_10(step, (uint64_t)q, qsim::kStreamFlip, 0,
                                                          s->em.seed, s->em.trial);
                if ((r.w[0] >> 32) < tb)
                    xs.push_back(make_flip(q, kPairSwap));
                if ((r.w[1] >> 32) < tp)
                    xs.push_back(make_flip(q, kPairNegB));
            }
        }
        rc = apply_xforms(s, xs);
        if (rc != QSIM_OK)
            return rc;
        s->pulses += npulses;
        s->step += n;
        return QSIM_OK;
    });
}

int qsim3_apply_pulses(qsim3_state *s, const qsim3_pulse *p, size_t n)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr || (n > 0 && p == nullptr))
            return qsim::set_error(QSIM_EINVAL, "NULL argument");
        for (size_t k = 0; k < n; ++k)
            if (!pulse_valid(p[k], s->M))
                return qsim::set_error(QSIM_EINVAL, "transformation %zu is malformed", k);
        HIP3(hipSetDevice(s->device), "hipSetDevice");
        std::vector<Xform> xs;
        for (size_t k = 0; k < n; ++k)
            xs.push_back(make_pulse(p[k], 0.0));
        const int rc = apply_xforms(s, xs);
        if (rc != QSIM_OK)
            return rc;
        s->pulses += n;
        return QSIM_OK;
    });
}

int qsim3_overlap(const qsim3_state *a, const qsim3_state *b, double out[4])
{
    return qsim::guarded(__func__, [&]() -> int {
        if (a == nullptr || b == nullptr || out == nullptr)
            return qsim::set_error(QSIM_EINVAL, "NULL argument");
        if (a->M != b->M || a->device != b->device)
            return qsim::set_error(QSIM_EINVAL, "registers differ in size or device");
        HIP3(hipSetDevice(a->device), "hipSetDevice");
        HIP3(hipStreamSynchronize(b->stream), "sync");
        const uint32_t n = (uint32_t)a->n;
        uint32_t chunk = kBlock3;
        while ((n + chunk - 1) / chunk > (uint32_t)kReduceBlocks3)
            chunk *= 2;
        const uint32_t g = (n + chunk - 1) / chunk;
        hipStream_t st = a->stream;
        if (a->dtype == QSIM_C64 && b->dtype == QSIM_C64)
            hipLaunchKernelGGL((k3_overlap<float, float>), dim3(g), dim3(kBlock3), 0, st,
                               (const cplx<float> *)a->psi, (const cplx<float> *)b->psi, n, chunk,
                               a->d_partial);
        else if (a->dtype == QSIM_C64)
            hipLaunchKernelGGL((k3_overlap<float, double>), dim3(g), dim3(kBlock3), 0, st,
                               (const cplx<float> *)a->psi, (const cplx<double> *)b->psi, n,
                               chunk, a->d_partial);
        else if (b->dtype == QSIM_C64)
            hipLaunchKernelGGL((k3_overlap<double, float>), dim3(g), dim3(kBlock3), 0, st,
                               (const cplx<double> *)a->psi, (const cplx<float> *)b->psi, n,
                               chunk, a->d_partial);
        else
            hipLaunchKernelGGL((k3_overlap<double, double>), dim3(g), dim3(kBlock3), 0, st,
                               (const cplx<double> *)a->psi, (const cplx<double> *)b->psi, n,
                               chunk, a->d_partial);
        hipLaunchKernelGGL(k3_finish, dim3(1), dim3(kBlock3), 0, st, a->d_partial, g, 4u,
                           a->d_out);
        HIP3(hipGetLastError(), "overlap");
        HIP3(hipMemcpyAsync(out, a->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, st),
             "overlap copy");
        HIP3(hipStreamSynchronize(st), "overlap sync");
        return QSIM_OK;
    });
}

int qsim3_fidelity(const qsim3_state *a, const qsim3_state *b, double *out_F)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (out_F == nullptr)
            return qsim::set_error(QSIM_EINVAL, "out_F is NULL");
        double o[4];
        const int rc = qsim3_overlap(a, b, o);
        if (rc != QSIM_OK)
            return rc;
        *out_F = (o[0] * o[0] + o[1] * o[1]) / (o[2] * o[3]);
        return QSIM_OK;
    });
}

int qsim3_probs(const qsim3_state *s, uint64_t ion_mask, double *out, size_t out_len)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr || out == nullptr)
            return qsim::set_error(QSIM_EINVAL, "NULL argument");
        if (ion_mask >> s->M)
            return qsim::set_error(QSIM_EINVAL, "mask has bits at or above ion %d", s->M);
        const int m = __builtin_popcountll(ion_mask);
        if (m > kMaxMarginalIons)
            return qsim::set_error(QSIM_EINVAL, "at most %d ions per marginal", kMaxMarginalIons);
        const uint64_t nb = pow3(m);
        if (out_len != nb)
            return qsim::set_error(QSIM_EINVAL, "out_len %zu != 3^%d", out_len, m);
        qsim3_state *ms = const_cast<qsim3_state *>(s);
        HIP3(hipSetDevice(s->device), "hipSetDevice");
        uint32_t places[kMaxMarginalIons] = {0};
        int j = 0;
        for (int q = 0; q < s->M; ++q)
            if ((ion_mask >> q) & 1u)
                places[j++] = (uint32_t)pow3(q);
        HIP3(hipMemcpyAsync(ms->d_places, places, sizeof(places), hipMemcpyHostToDevice,
                            s->stream), "places");
        const uint32_t n = (uint32_t)s->n;
        uint32_t chunk = kBlock3;
        while ((n + chunk - 1) / chunk > (uint32_t)kReduceBlocks3)
            chunk *= 2;
        const uint32_t g = (n + chunk - 1) / chunk;
        const bool few = nb <= kFastMarginalBins;
        if (s->dtype == QSIM_C64)
            hipLaunchKernelGGL(few ? k3_marginal_few<float> : k3_marginal<float>, dim3(g),
                               dim3(kBlock3), 0, s->stream, (const cplx<float> *)s->psi, n, chunk,
                               (uint32_t)m, ms->d_places, ms->d_partial);
        else
            hipLaunchKernelGGL(few ? k3_marginal_few<double> : k3_marginal<double>, dim3(g),
                               dim3(kBlock3), 0, s->stream, (const cplx<double> *)s->psi, n,
                               chunk, (uint32_t)m, ms->d_places, ms->d_partial);
        hipLaunchKernelGGL(k3_finish, dim3(1), dim3(kBlock3), 0, s->stream, ms->d_partial, g,
                           (uint32_t)nb, ms->d_out);
        HIP3(hipGetLastError(), "marginal");
        HIP3(hipMemcpyAsync(out, ms->d_out, nb * sizeof(double), hipMemcpyDeviceToHost,
                            s->stream), "probs copy");
        HIP3(hipStreamSynchronize(s->stream), "probs sync");
        return QSIM_OK;
    });
}

int qsim3_get_amplitudes(const qsim3_state *s, uint64_t offset, uint64_t count, double *out)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr || (out == nullptr && count > 0))
            return qsim::set_error(QSIM_EINVAL, "NULL argument");
        if (offset > s->n || count > s->n - offset)
            return qsim::set_error(QSIM_ERANGE, "range outside the 3^%d amplitudes", s->M);
        if (count == 0)
            return QSIM_OK;
        qsim3_state *ms = const_cast<qsim3_state *>(s);
        HIP3(hipSetDevice(s->device), "hipSetDevice");
        const uint64_t chunk = std::min<uint64_t>(count, 1ull << 22);
        int rc = ensure_stage3(ms, chunk * 16);
        if (rc != QSIM_OK)
            return rc;
        for (uint64_t done = 0; done < count; done += chunk) {
            const uint32_t c = (uint32_t)std::min(chunk, count - done);
            if (s->dtype == QSIM_C64)
                hipLaunchKernelGGL((k3_to_f64<float>), grid3(c), dim3(kBlock3), 0, s->stream,
                                   (const cplx<float> *)s->psi + offset + done, c, ms->d_stage);
            else
                hipLaunchKernelGGL((k3_to_f64<double>), grid3(c), dim3(kBlock3), 0, s->stream,
                                   (const cplx<double> *)s->psi + offset + done, c, ms->d_stage);
            HIP3(hipGetLastError(), "convert");
            HIP3(hipMemcpyAsync(out + 2 * done, ms->d_stage, (size_t)c * 16,
                                hipMemcpyDeviceToHost, s->stream), "amplitude copy");
            HIP3(hipStreamSynchronize(s->stream), "amplitude sync");
        }
        return QSIM_OK;
    });
}

int qsim3_synchronize(qsim3_state *s)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return qsim::set_error(QSIM_EINVAL, "state is NULL");
        HIP3(hipSetDevice(s->device), "hipSetDevice");
        HIP3(hipStreamSynchronize(s->stream), "sync");
        return QSIM_OK;
    });
}

int qsim3_info(const qsim3_state *s, int *num_ions, int *dtype, uint64_t *step,
               uint64_t *transformations, uint64_t *launches)
{
    return qsim::guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return qsim::set_error(QSIM_EINVAL, "state is NULL");
        if (num_ions) *num_ions = s->M;
        if (dtype) *dtype = s->dtype;
        if (step) *step = s->step;
        if (transformations) *transformations = s->pulses;
        if (launches) *launches = s->launches;
        return QSIM_OK;
    });
}

}  // extern "C"
