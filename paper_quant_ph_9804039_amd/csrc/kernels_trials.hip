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
    uint32_t pad[2];
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
    const bool draws_angle = sigma > 0.0;
    const bool draws_flip = p_bit > 0.0 || p_phase > 0.0;
    const uint64_t thr_b = flip_threshold(p_bit), thr_p = flip_threshold(p_phase);

    for (uint64_t t = blockIdx.x; t < n_trials; t += gridDim.x) {
        const uint64_t trial = trial0 + t;
        for (uint32_t i = tid; i < N; i += T)
            st[i] = {R(i == 0 ? 1 : 0), R(0)};
        uint32_t X = 0;  // bit flips so far (uniform)
        for (uint32_t c0 = 0; c0 < n; c0 += kChunk) {
            const uint32_t cn = min((uint32_t)kChunk, n - c0);
            __syncthreads();
            for (uint32_t i = tid; i < cn; i += T) {
                bmask[i] = 0;
                zmask[i] = 0;
            }
            __syncthreads();
            // flip draws of the chunk: one Philox block per (step, qubit)
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
            // the chunk's gates as applied to the stored register
            for (uint32_t g = tid; g < cn; g += T) {
                const TrialGate gd = gates[c0 + g];
                const double eps = draws_angle ? sigma * step_gaussian(seed, trial, c0 + g) : 0.0;
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
                // phase flips follow this step's bit flips; Z_q on the true
                // register is Z_q on the stored one up to a global sign
                op.zmask = zmask[g];
                ops[g] = op;
            }
            __syncthreads();
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

template <typename R, int T>
hipError_t launch_t(const TrialLaunch &L, hipStream_t st)
{
    const size_t lds = trial_lds_bytes((int)L.M, (int)sizeof(cplx<R>));
    auto fn = k_trials<R, T>;
    static size_t lds_allowed = 65536;  // per instantiation
    if (lds > lds_allowed) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e;
        }
        lds_allowed = lds;
    }
    const uint64_t grid = L.n_trials < (uint64_t)L.grid ? L.n_trials : (uint64_t)L.grid;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(T), lds, st, L.gates, L.ngates, L.M,
                       L.sigma, L.p_bit, L.p_phase, L.seed, L.trial0, L.n_trials,
                       reinterpret_cast<const cplx<R> *>(L.ideal), L.out_F);
    return hipGetLastError();
}

}  // namespace

size_t trial_lds_bytes(int M, int elem_bytes)
{
    const size_t op_bytes = elem_bytes == 8 ? sizeof(TrialOp<float>) : sizeof(TrialOp<double>);
    return ((size_t)1 << M) * (size_t)elem_bytes + kChunk * op_bytes;
}

// Variants the autotuner chooses from: workgroup size 1024 or 512.
template <typename R>
hipError_t launch_trials(const TrialLaunch &L, hipStream_t st)
{
    switch (L.variant) {
    case 0: return launch_t<R, 1024>(L, st);
    case 1: return launch_t<R, 512>(L, st);
    default: return hipErrorInvalidValue;
    }
}

int trial_variants() { return 2; }

template <typename R, int T>
int grid_t(int M)
{
    const size_t lds = trial_lds_bytes(M, (int)sizeof(cplx<R>));
    auto fn = k_trials<R, T>;
    if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, T, lds) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}

int trial_grid(int variant, int M, int elem_bytes)
{
    if (elem_bytes == 8)
        return variant == 0 ? grid_t<float, 1024>(M) : grid_t<float, 512>(M);
    return variant == 0 ? grid_t<double, 1024>(M) : grid_t<double, 512>(M);
}

const char *trial_variant_name(int v)
{
    return v == 0 ? "lds-per-gate-1024" : v == 1 ? "lds-per-gate-512" : "?";
}

template hipError_t launch_trials<float>(const TrialLaunch &, hipStream_t);
template hipError_t launch_trials<double>(const TrialLaunch &, hipStream_t);

}  // namespace qsim
