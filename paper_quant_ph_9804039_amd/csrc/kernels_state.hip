// Whole-vector kernels of the qsim library for gfx950: basis-state init, the
// per-gate pair update (one HBM pass per gate), scaling, the FP64 fidelity and
// norm reductions, probabilities and FP64 staging conversions.
//
// Every kernel streams the state with 16-byte vector accesses: a complex64
// "unit" of two adjacent amplitudes is one dwordx4, a complex128 unit is two.
// Grids are capped and walked with a grid stride so that 64-bit vectors of
// any size (up to 2^34 amplitudes) are covered.
#include "launch.h"

namespace qsim {
namespace {

constexpr int kBlock = 256;
constexpr uint64_t kMaxGrid = 1u << 20;

inline dim3 grid_for(uint64_t units)
{
    uint64_t g = (units + kBlock - 1) / kBlock;
    if (g > kMaxGrid)
        g = kMaxGrid;
    if (g == 0)
        g = 1;
    return dim3((unsigned)g);
}

// ------------------------------------------------------- vector access helpers

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

template <typename R>
__device__ __forceinline__ cplx<R> sel(bool c, cplx<R> a, cplx<R> b)
{
    return {c ? a.re : b.re, c ? a.im : b.im};
}

// --------------------------------------------------------------------- init

template <typename R>
__global__ void __launch_bounds__(kBlock) k_init_basis(cplx<R> *psi, uint64_t units, uint64_t kidx)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const cplx<R> z = {R(0), R(0)};
    for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < units; u += stride) {
        cplx<R> a = z, b = z;
        if (2 * u == kidx)
            a.re = R(1);
        if (2 * u + 1 == kidx)
            b.re = R(1);
        st2(psi + 2 * u, a, b);
    }
}

// ---------------------------------------------------- per-gate pair update
//
// Sec. 2.1: a 2x2 transform on bit t is V/2 independent transforms of the
// pairs (i, i | 2^t) with bit t of i clear.  A work unit is two pairs:
//   t == 0: the four amplitudes 4u .. 4u+3 (pairs (4u, 4u+1), (4u+2, 4u+3));
//   t >= 1: pairs (i, i + 2^t) and (i + 1, i + 1 + 2^t) where i is the pair
//           index 2u with a zero inserted at bit t; each side is one
//           contiguous two-amplitude vector.
// Controls are per pair; a unit with no active pair moves no data.

template <typename R, bool SWAP>
__global__ void __launch_bounds__(kBlock) k_pair(PlainArgs<R> A)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t tb = 1ull << A.t;
    const uint64_t cm = A.cmask;
    for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < A.n_units; u += stride) {
        uint64_t va, vb;           // first index of the two vectors
        uint64_t c0, c1;           // control-test index of the two pairs
        if (A.t == 0) {
            va = 4 * u;
            vb = 4 * u + 2;
            c0 = va;
            c1 = vb;
        } else {
            const uint64_t p = 2 * u;
            va = ((p >> A.t) << (A.t + 1)) | (p & (tb - 1));
            vb = va | tb;
            c0 = va;
            c1 = va + 1;
        }
        const bool act0 = (c0 & cm) == cm;
        const bool act1 = (c1 & cm) == cm;
        if (!act0 && !act1)
            continue;
        cplx<R> a0, a1, b0, b1;
        ld2(A.psi + va, a0, a1);
        ld2(A.psi + vb, b0, b1);
        // the two pairs as (x0, y0), (x1, y1)
        cplx<R> x0, y0, x1, y1;
        if (A.t == 0) {
            x0 = a0; y0 = a1; x1 = b0; y1 = b1;
        } else {
            x0 = a0; y0 = b0; x1 = a1; y1 = b1;
        }
        cplx<R> nx0, ny0, nx1, ny1;
        if (SWAP) {
            nx0 = y0; ny0 = x0; nx1 = y1; ny1 = x1;
        } else {
            nx0 = cmad2(A.u[0], x0, A.u[1], y0);
            ny0 = cmad2(A.u[2], x0, A.u[3], y0);
            nx1 = cmad2(A.u[0], x1, A.u[1], y1);
            ny1 = cmad2(A.u[2], x1, A.u[3], y1);
        }
        x0 = sel(act0, nx0, x0);
        y0 = sel(act0, ny0, y0);
        x1 = sel(act1, nx1, x1);
        y1 = sel(act1, ny1, y1);
        if (A.t == 0) {
            st2(A.psi + va, x0, y0);
            st2(A.psi + vb, x1, y1);
        } else {
            st2(A.psi + va, x0, x1);
            st2(A.psi + vb, y0, y1);
        }
    }
}

// Diagonal gate or exact sign flip: every amplitude is scaled by d0 or d1
// according to its target bit (only the bit-1 half moves for a sign flip).
template <typename R, bool NEG>
__global__ void __launch_bounds__(kBlock) k_diag(PlainArgs<R> A)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const uint64_t cm = A.cmask;
    const cplx<R> d0 = A.u[0], d1 = A.u[3];
    for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < A.n_units; u += stride) {
        const uint64_t i = 2 * u;
        const uint32_t bit0 = (uint32_t)((i >> A.t) & 1u);
        const uint32_t bit1 = (uint32_t)(((i + 1) >> A.t) & 1u);
        const bool act0 = (i & cm) == cm;
        const bool act1 = ((i + 1) & cm) == cm;
        if (NEG && !((act0 && bit0) || (act1 && bit1)))
            continue;
        cplx<R> a, b;
        ld2(A.psi + i, a, b);
        cplx<R> na, nb;
        if (NEG) {
            na = bit0 ? cplx<R>{-a.re, -a.im} : a;
            nb = bit1 ? cplx<R>{-b.re, -b.im} : b;
        } else {
            na = cmul(a, bit0 ? d1 : d0);
            nb = cmul(b, bit1 ? d1 : d0);
        }
        st2(A.psi + i, sel(act0, na, a), sel(act1, nb, b));
    }
}

// Scalar fallback for a one-qubit register (two amplitudes).
template <typename R>
__global__ void k_single(PlainArgs<R> A, uint32_t type)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    cplx<R> a = A.psi[0], b = A.psi[1];
    cplx<R> na, nb;
    switch (type) {
    case kOpMat: na = cmad2(A.u[0], a, A.u[1], b); nb = cmad2(A.u[2], a, A.u[3], b); break;
    case kOpSwap: na = b; nb = a; break;
    case kOpDiag: na = cmul(a, A.u[0]); nb = cmul(b, A.u[3]); break;
    default: na = a; nb = {-b.re, -b.im}; break;
    }
    A.psi[0] = na;
    A.psi[1] = nb;
}

// ---------------------------------------------------------------- scaling

template <typename R>
__global__ void __launch_bounds__(kBlock) k_scale(cplx<R> *psi, uint64_t units, const double *scale)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    const R s = (R)*scale;
    for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < units; u += stride) {
        cplx<R> a, b;
        ld2(psi + 2 * u, a, b);
        a.re *= s; a.im *= s; b.re *= s; b.im *= s;
        st2(psi + 2 * u, a, b);
    }
}

// ------------------------------------------------------- FP64 reductions
//
// Per-block partials in a fixed order (thread-strided loop, a butterfly over
// the 64 lanes of each wave, then the waves in order), then one block sums
// the kReduceBlocks partials the same way: the result does not depend on
// timing, so repeated calls agree bit for bit.

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*scratch)[kBlock / 64])
{
#pragma unroll
    for (int c = 0; c < NV; ++c)
        v[c] = wave_sum(v[c]);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c)
            scratch[c][w] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0.0;
            for (int i = 0; i < kBlock / 64; ++i)
                s += scratch[c][i];
            v[c] = s;
        }
    }
}

template <typename Ra, typename Rb, bool OVERLAP>
__global__ void __launch_bounds__(kBlock) k_reduce(const cplx<Ra> *a, const cplx<Rb> *b,
                                                   uint64_t units, double *partial)
{
    __shared__ double scratch[4][kBlock / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < units; u += stride) {
        cplx<Ra> a0, a1;
        ld2(a + 2 * u, a0, a1);
        const double ar0 = a0.re, ai0 = a0.im, ar1 = a1.re, ai1 = a1.im;
        v[2] += (ar0 * ar0 + ai0 * ai0) + (ar1 * ar1 + ai1 * ai1);
        if (OVERLAP) {
            cplx<Rb> b0, b1;
            ld2(b + 2 * u, b0, b1);
            const double br0 = b0.re, bi0 = b0.im, br1 = b1.re, bi1 = b1.im;
            v[0] += (ar0 * br0 + ai0 * bi0) + (ar1 * br1 + ai1 * bi1);
            v[1] += (ar0 * bi0 - ai0 * br0) + (ar1 * bi1 - ai1 * br1);
            v[3] += (br0 * br0 + bi0 * bi0) + (br1 * br1 + bi1 * bi1);
        }
    }
    block_sum<4>(v, scratch);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            partial[4 * (uint64_t)blockIdx.x + c] = v[c];
    }
}

__global__ void __launch_bounds__(kBlock) k_reduce_finish(const double *partial, int nblocks,
                                                          double *out)
{
    __shared__ double scratch[4][kBlock / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nblocks; i += kBlock) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            v[c] += partial[4 * i + c];
    }
    block_sum<4>(v, scratch);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            out[c] = v[c];
    }
}

// First stage of a long sum: block b adds values [b chunk, (b + 1) chunk) in
// the fixed order of block_sum.
__global__ void __launch_bounds__(kBlock) k_sum_chunks(const double *values, uint64_t n,
                                                       uint64_t chunk, double *partial)
{
    __shared__ double scratch[1][kBlock / 64];
    double v[1] = {0.0};
    const uint64_t lo = (uint64_t)blockIdx.x * chunk;
    const uint64_t hi = lo + chunk < n ? lo + chunk : n;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock)
        v[0] += values[i];
    block_sum<1>(v, scratch);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = v[0];
}

__global__ void __launch_bounds__(kBlock) k_finish_norm(const double *tile_norms, uint64_t n,
                                                        double *out)
{
    __shared__ double scratch[1][kBlock / 64];
    double v[1] = {0.0};
    for (uint64_t i = threadIdx.x; i < n; i += kBlock)
        v[0] += tile_norms[i];
    block_sum<1>(v, scratch);
    if (threadIdx.x == 0) {
        out[0] = v[0];
        out[1] = 1.0 / sqrt(v[0]);
    }
}

// ----------------------------------------------------------- probabilities

template <typename R>
__global__ void __launch_bounds__(kBlock) k_probs_full(const cplx<R> *psi, uint64_t units,
                                                       double *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t u = (uint64_t)blockIdx.x * kBlock + threadIdx.x; u < units; u += stride) {
        cplx<R> a, b;
        ld2(psi + 2 * u, a, b);
        const double pa = (double)a.re * a.re + (double)a.im * a.im;
        const double pb = (double)b.re * b.re + (double)b.im * b.im;
        reinterpret_cast<double2 *>(out)[u] = make_double2(pa, pb);
    }
}

// Marginal over a qubit mask of m bits.  The index space is (k, u): k the m
// masked bits, u the M - m others.  Work item (k, c) sums u = c*U .. c*U+U-1
// in ascending order (so ascending index order for each k); a second kernel
// adds the chunks of each k in order.  When the mask holds qubit 0, items
// with neighbouring k take neighbouring lanes (coalesced); otherwise
// neighbouring chunks do.
struct MargPlan {
    uint64_t m, U, C;
};

__host__ __device__ inline MargPlan marg_plan(int M, uint64_t mask)
{
    uint64_t m = 0;
    for (int q = 0; q < M; ++q)
        m += (mask >> q) & 1u;
    const uint64_t per_bin = 1ull << (M - m);
    uint64_t U = (M > 20) ? (1ull << (M - 20)) : 1ull;
    if (U > per_bin)
        U = per_bin;
    return {m, U, per_bin / U};
}

__device__ __forceinline__ uint64_t deposit_bits(uint64_t x, uint64_t mask)
{
    uint64_t r = 0;
    for (uint64_t bit = 1; mask != 0; bit <<= 1) {
        const uint64_t low = mask & (~mask + 1);
        if (x & bit)
            r |= low;
        mask ^= low;
    }
    return r;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_probs_chunks(const cplx<R> *psi, int M, uint64_t mask,
                                                         uint64_t U, uint64_t C, uint64_t mbits,
                                                         double *partial)
{
    const uint64_t full = (M == 64) ? ~0ull : ((1ull << M) - 1);
    const uint64_t umask = ~mask & full;
    const uint64_t items = (1ull << mbits) * C;
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t x = (uint64_t)blockIdx.x * kBlock + threadIdx.x; x < items; x += stride) {
        uint64_t kk, c;
        if (mask & 1u) {
            kk = x & ((1ull << mbits) - 1);
            c = x >> mbits;
        } else {
            c = x % C;
            kk = x / C;
        }
        const uint64_t hi = deposit_bits(kk, mask);
        uint64_t lo = deposit_bits(c * U, umask);
        double s = 0.0;
        for (uint64_t n = 0; n < U; ++n) {
            const cplx<R> a = psi[hi | lo];
            s += (double)a.re * a.re + (double)a.im * a.im;
            lo = ((lo | ~umask) + 1) & umask;  // next subset of umask, ascending
        }
        partial[kk * C + c] = s;
    }
}

__global__ void __launch_bounds__(kBlock) k_probs_finish(const double *partial, uint64_t C,
                                                         double *out)
{
    __shared__ double scratch[1][kBlock / 64];
    double v[1] = {0.0};
    const uint64_t kk = blockIdx.x;
    for (uint64_t c = threadIdx.x; c < C; c += kBlock)
        v[0] += partial[kk * C + c];
    block_sum<1>(v, scratch);
    if (threadIdx.x == 0)
        out[kk] = v[0];
}

// ------------------------------------------------------------ conversions

template <typename R>
__global__ void __launch_bounds__(kBlock) k_to_f64(const cplx<R> *psi, uint64_t count, double *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const cplx<R> a = psi[i];
        reinterpret_cast<double2 *>(out)[i] = make_double2((double)a.re, (double)a.im);
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_from_f64(const double *in, uint64_t count, cplx<R> *psi)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
        const double2 v = reinterpret_cast<const double2 *>(in)[i];
        psi[i] = {(R)v.x, (R)v.y};
    }
}

template <typename R>
PlainArgs<R> make_plain(const Op &op, cplx<R> *psi, int M)
{
    PlainArgs<R> A{};
    A.psi = psi;
    A.M = M;
    A.t = op.target;
    A.cmask = op.cmask;
    for (int c = 0; c < 4; ++c)
        A.u[c] = {(R)op.u[2 * c], (R)op.u[2 * c + 1]};
    return A;
}

}  // namespace

// ----------------------------------------------------------------- launchers

template <typename R>
hipError_t launch_init_basis(cplx<R> *psi, int M, uint64_t k, hipStream_t st)
{
    const uint64_t units = (1ull << M) / 2;
    hipLaunchKernelGGL((k_init_basis<R>), grid_for(units), dim3(kBlock), 0, st, psi, units, k);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_plain(const Op &op, cplx<R> *psi, int M, hipStream_t st)
{
    PlainArgs<R> A = make_plain<R>(op, psi, M);
    if (M < 2) {
        hipLaunchKernelGGL((k_single<R>), dim3(1), dim3(64), 0, st, A, op.type);
        return hipGetLastError();
    }
    const uint64_t n = 1ull << M;
    switch (op.type) {
    case kOpMat:
        A.n_units = n / 4;
        hipLaunchKernelGGL((k_pair<R, false>), grid_for(A.n_units), dim3(kBlock), 0, st, A);
        break;
    case kOpSwap:
        A.n_units = n / 4;
        hipLaunchKernelGGL((k_pair<R, true>), grid_for(A.n_units), dim3(kBlock), 0, st, A);
        break;
    case kOpDiag:
        A.n_units = n / 2;
        hipLaunchKernelGGL((k_diag<R, false>), grid_for(A.n_units), dim3(kBlock), 0, st, A);
        break;
    default:
        A.n_units = n / 2;
        hipLaunchKernelGGL((k_diag<R, true>), grid_for(A.n_units), dim3(kBlock), 0, st, A);
        break;
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_scale(cplx<R> *psi, int M, const double *scale, hipStream_t st)
{
    const uint64_t units = (1ull << M) / 2;
    hipLaunchKernelGGL((k_scale<R>), grid_for(units), dim3(kBlock), 0, st, psi, units, scale);
    return hipGetLastError();
}

static int reduce_grid(uint64_t units)
{
    uint64_t g = (units + kBlock - 1) / kBlock;
    return (int)(g < (uint64_t)kReduceBlocks ? g : (uint64_t)kReduceBlocks);
}

template <typename Ra, typename Rb>
hipError_t launch_overlap(const cplx<Ra> *a, const cplx<Rb> *b, int M, double *partial,
                          double *out, hipStream_t st)
{
    const uint64_t units = (1ull << M) / 2;
    const int g = reduce_grid(units);
    hipLaunchKernelGGL((k_reduce<Ra, Rb, true>), dim3(g), dim3(kBlock), 0, st, a, b, units,
                       partial);
    hipLaunchKernelGGL(k_reduce_finish, dim3(1), dim3(kBlock), 0, st, partial, g, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_norm(const cplx<R> *a, int M, double *partial, double *out, hipStream_t st)
{
    const uint64_t units = (1ull << M) / 2;
    const int g = reduce_grid(units);
    hipLaunchKernelGGL((k_reduce<R, R, false>), dim3(g), dim3(kBlock), 0, st, a, a, units,
                       partial);
    hipLaunchKernelGGL(k_reduce_finish, dim3(1), dim3(kBlock), 0, st, partial, g, out);
    return hipGetLastError();
}

hipError_t launch_finish_norm(const double *tile_norms, uint64_t n, double *partial, double *out,
                              hipStream_t st)
{
    // one block for short sums; past 16 values per thread, a first stage of
    // up to kReduceBlocks blocks over contiguous chunks (a fixed partition of
    // [0, n), so the result does not depend on timing)
    constexpr uint64_t kOneBlock = 16 * (uint64_t)kBlock;
    if (n <= kOneBlock || partial == nullptr) {
        hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(kBlock), 0, st, tile_norms, n, out);
        return hipGetLastError();
    }
    uint64_t chunk = kOneBlock;
    while ((n + chunk - 1) / chunk > (uint64_t)kReduceBlocks)
        chunk *= 2;
    const uint64_t g = (n + chunk - 1) / chunk;
    hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)g), dim3(kBlock), 0, st, tile_norms, n, chunk,
                       partial);
    hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(kBlock), 0, st, partial, g, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_probs_full(const cplx<R> *psi, int M, double *out, hipStream_t st)
{
    const uint64_t units = (1ull << M) / 2;
    hipLaunchKernelGGL((k_probs_full<R>), grid_for(units), dim3(kBlock), 0, st, psi, units, out);
    return hipGetLastError();
}

uint64_t probs_marginal_partial_len(int M, uint64_t mask)
{
    const MargPlan p = marg_plan(M, mask);
    return (1ull << p.m) * p.C;
}

template <typename R>
hipError_t launch_probs_marginal(const cplx<R> *psi, int M, uint64_t mask, double *partial,
                                 uint64_t partial_len, double *out, hipStream_t st)
{
    const MargPlan p = marg_plan(M, mask);
    if ((1ull << p.m) * p.C > partial_len)
        return hipErrorInvalidValue;
    const uint64_t items = (1ull << p.m) * p.C;
    double *dst = (p.C == 1) ? out : partial;
    hipLaunchKernelGGL((k_probs_chunks<R>), grid_for(items), dim3(kBlock), 0, st, psi, M, mask,
                       p.U, p.C, p.m, dst);
    if (p.C > 1)
        hipLaunchKernelGGL(k_probs_finish, dim3((unsigned)(1ull << p.m)), dim3(kBlock), 0, st,
                           partial, p.C, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_to_f64(const cplx<R> *psi, uint64_t count, double *out, hipStream_t st)
{
    hipLaunchKernelGGL((k_to_f64<R>), grid_for(count), dim3(kBlock), 0, st, psi, count, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_from_f64(const double *in, uint64_t count, cplx<R> *psi, hipStream_t st)
{
    hipLaunchKernelGGL((k_from_f64<R>), grid_for(count), dim3(kBlock), 0, st, in, count, psi);
    return hipGetLastError();
}

#define QSIM_INST(R)                                                                              \
    template hipError_t launch_init_basis<R>(cplx<R> *, int, uint64_t, hipStream_t);             \
    template hipError_t launch_plain<R>(const Op &, cplx<R> *, int, hipStream_t);                \
    template hipError_t launch_scale<R>(cplx<R> *, int, const double *, hipStream_t);            \
    template hipError_t launch_norm<R>(const cplx<R> *, int, double *, double *, hipStream_t);   \
    template hipError_t launch_probs_full<R>(const cplx<R> *, int, double *, hipStream_t);       \
    template hipError_t launch_probs_marginal<R>(const cplx<R> *, int, uint64_t, double *,       \
                                                 uint64_t, double *, hipStream_t);               \
    template hipError_t launch_to_f64<R>(const cplx<R> *, uint64_t, double *, hipStream_t);      \
    template hipError_t launch_from_f64<R>(const double *, uint64_t, cplx<R> *, hipStream_t);

QSIM_INST(float)
QSIM_INST(double)
template hipError_t launch_overlap<float, float>(const cplx<float> *, const cplx<float> *, int,
                                                 double *, double *, hipStream_t);
template hipError_t launch_overlap<float, double>(const cplx<float> *, const cplx<double> *, int,
                                                  double *, double *, hipStream_t);
template hipError_t launch_overlap<double, float>(const cplx<double> *, const cplx<float> *, int,
                                                  double *, double *, hipStream_t);
template hipError_t launch_overlap<double, double>(const cplx<double> *, const cplx<double> *,
                                                   int, double *, double *, hipStream_t);

}  // namespace qsim
