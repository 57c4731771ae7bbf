// Shared definitions of the qsim HIP library: amplitude types, the random
// number generator, lowered operations and the argument blocks of the
// kernels.  Everything here is specific to gfx950 (wave64, 64 KiB+ LDS).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qsim {

// ---------------------------------------------------------------- amplitudes

template <typename R>
struct cplx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename R>
__device__ __forceinline__ cplx<R> cmad2(cplx<R> u0, cplx<R> a, cplx<R> u1, cplx<R> b)
{
    // u0 * a + u1 * b
    return {(u0.re * a.re - u0.im * a.im) + (u1.re * b.re - u1.im * b.im),
            (u0.re * a.im + u0.im * a.re) + (u1.re * b.im + u1.im * b.re)};
}

// ------------------------------------------------------------ random draws
//
// Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128
// multiplies; the key advances by the two Weyl increments between rounds.
// The simulator keys it by (seed, trial) and counts (step, qubit, stream, 0),
// so any draw can be made by any thread in any order.

struct u64x4 {
    uint64_t w[4];
};

__host__ __device__ inline void mul_wide(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
}

__host__ __device__ inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t hA, lA, hB, lB;
        mul_wide(kMulA, c0, hA, lA);
        mul_wide(kMulB, c2, hB, lB);
        const uint64_t n0 = hB ^ c1 ^ k0;
        const uint64_t n2 = hA ^ c3 ^ k1;
        c0 = n0;
        c1 = lB;
        c2 = n2;
        c3 = lA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {{c0, c1, c2, c3}};
}

enum : uint64_t { kStreamAngle = 1, kStreamFlip = 2 };

// Threshold of a Bernoulli(p) draw on a 32-bit uniform integer.
__host__ __device__ inline uint64_t flip_threshold(double p)
{
    return (uint64_t)floor(p * 4294967296.0);
}

// z ~ N(0, 1) of one step by Box-Muller on the high halves of words 0 and 1.
__host__ __device__ inline double step_gaussian(uint64_t seed, uint64_t trial, uint64_t step)
{
    const u64x4 r = philox4x64_10(step, 0, kStreamAngle, 0, seed, trial);
    const double u1 = ((double)(r.w[0] >> 32) + 0.5) * 0x1p-32;
    const double u2 = ((double)(r.w[1] >> 32) + 0.5) * 0x1p-32;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

// ------------------------------------------------------- lowered operations

enum OpType : uint32_t {
    kOpMat = 0,   // general 2x2 on the target pairs
    kOpDiag = 1,  // diag(d0, d1): d0 on target bit 0, d1 on target bit 1
    kOpSwap = 2,  // exact exchange of the pair (unperturbed X / CNOT / Toffoli, bit flip)
    kOpNeg = 3,   // exact sign flip where the target bit is 1 (unperturbed Z, phase flip)
};

// Host-side lowered operation, FP64 coefficients.
struct Op {
    uint32_t type;
    int32_t target;
    uint64_t cmask;   // global control mask (all bits must be 1)
    double u[8];      // kOpMat: u00 u01 u10 u11 as re,im; kOpDiag: d0 = u[0..1], d1 = u[6..7]
    uint64_t step;    // circuit step the operation belongs to
    uint64_t zdep;    // untouched qubits whose definite value the operation was
                      // specialised on (kept as ordering dependencies)
    bool is_flip;     // injected by the error model
    bool step_end;    // last operation of its step
    bool norm_mark;   // a renormalisation boundary follows this operation
    bool activates;   // spreads its (untouched) target over both values
    bool relocate;    // moves an untouched qubit's amplitudes to its other value
};

// ------------------------------------------------------ kernel argument blocks

template <typename R>
struct PlainArgs {
    cplx<R> *psi;
    uint64_t n_units;      // work units (see the kernel)
    int M;
    int t;                 // target qubit
    uint64_t cmask;        // global control mask
    cplx<R> u[4];          // u00 u01 u10 u11 (kOpDiag: u[0] = d0, u[3] = d1)
};

constexpr int kMaxTileBits = 14;
// Operations per fused pass: they travel in the kernel arguments (at most
// 4 KiB), so complex64 passes take more than complex128 ones.
template <typename R>
constexpr int kPassOps = sizeof(R) == 4 ? 63 : 40;
constexpr int kMaxPassOps = 63;
constexpr int kMaxGroups = 32;
constexpr uint32_t kNoPos = 0xFFu;
constexpr int kMaxRuns = 16;  // runs of consecutive qubits in a tile set or its complement

// How a fused pass applies one operation to a register quantum (2^G
// amplitudes spanned by the group bits; see the tile kernel).
enum TileOpKind : uint8_t {
    kTPair = 0,     // real 2x2 m plus i*w on the diagonal (H, perturbed H / X)
    kTPhaseIn = 1,  // uncontrolled diag(1, q) on a group bit (the diagonal's d0 is global)
    kTSwap = 2,     // exact exchange
    kTDiagIn = 3,   // controlled diag(d0, d1) on a group bit
    kTNegIn = 4,    // exact sign flip on a group bit
    kTDiagOut = 5,  // uncontrolled diag(1, q) on a bit outside the group: one factor per quantum
    kTNegOut = 6,   // uncontrolled sign flip on a bit outside the group
};

template <typename R>
struct TileOp {
    uint8_t kind;       // TileOpKind
    uint8_t gpos;       // target's index among the group bits (kinds 0..4)
    uint8_t rc;         // controls on group bits, as a mask over the register index
    uint8_t form;       // kTPair: 0 real m; 1 m + i*w on the diagonal; 2 the same, m00 = m11 = 0;
                        // 3 (never controlled) h*([[1,1],[1,-1]] + i*t) with h in the pass phase,
                        // t = c[4]; 4 the same with t = 0
    uint32_t qc;        // controls on tile bits outside the group, as a tile-index mask
    uint64_t cm_out;    // controls on qubits outside the tile, as a global mask
    uint32_t tpos;      // kinds 5, 6: tile bit of the target, kNoPos if outside the tile
    uint32_t tq;        // target qubit (global)
    R c[8];             // kTPair: m00 m01 m10 m11 w0 w1; diagonal kinds: d0, d1 (re, im)
};

// Group word of a fused pass: first op (6 bits), op count (6 bits), then the
// G <= 5 sorted tile bits of the group, 4 bits each (32 bits in all).
constexpr uint32_t kGroupCountShift = 6;
constexpr uint32_t kGroupBitsShift = 12;
static_assert(kMaxPassOps <= 63 && kMaxTileBits <= 16, "group word field widths");
__host__ __device__ inline uint32_t group_first(uint32_t w) { return w & 63u; }
__host__ __device__ inline uint32_t group_count(uint32_t w) { return (w >> kGroupCountShift) & 63u; }
__host__ __device__ inline uint32_t group_bit(uint32_t w, int i)
{
    return (w >> (kGroupBitsShift + 4 * i)) & 15u;
}

// A fused pass: tiles of 2^k amplitudes spanned by qubits spos[0..k), the
// first `low` of which are qubits 0..low-1 (contiguous runs in memory).  The
// 2^(mact-k) tiles enumerate the qubits of emask; every other qubit of the
// register is untouched and holds the value base_or gives it (its other
// value's amplitudes are zero and are not visited).
template <typename R>
struct TileArgs {
    cplx<R> *psi;
    const double *scale_in;   // if set, multiply every amplitude by *scale_in on load
    double *norm_out;         // if set, per-tile sum of |a|^2 after the pass
    uint64_t smask;           // global mask of the tile qubits
    uint64_t emask;           // qubits the tile number enumerates, = the crun runs
    uint64_t base_or;         // values of the untouched qubits outside the pass
    uint32_t mact;            // qubits the pass spans: tile qubits + enumerated ones
    uint32_t M;
    uint32_t k;
    uint32_t low;
    uint32_t nops;
    uint32_t ngroups;
    uint8_t spos[kMaxTileBits];        // qubit of each tile bit (host-side checks)
    uint32_t nsrun, ncrun;             // runs of consecutive qubits, as words
    uint32_t srun[kMaxRuns];           //   start | length << 8: tile index bits ->
    uint32_t crun[kMaxRuns];           //   tile qubits; tile number bits -> the rest
    uint32_t group[kMaxGroups];        // see group_first / group_count / group_bit
    R phase[2];                        // global phase of the pass's uncontrolled diagonals
    uint32_t use_phase;                // phase != 1
    uint32_t gen;                      // the register is basis state gen_index: the first
    uint64_t gen_index;                //   group builds its quanta instead of loading them
    TileOp<R> ops[kPassOps<R>];
};

static_assert(sizeof(TileArgs<float>) <= 4096 && sizeof(TileArgs<double>) <= 4096,
              "kernel arguments must fit 4 KiB");
static_assert(kPassOps<float> <= kMaxPassOps && kPassOps<double> <= kMaxPassOps, "op caps");

}  // namespace qsim
