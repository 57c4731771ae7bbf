// C-ABI of the qsim library: state management, gate lowering with error
// injection, the pass scheduler, and the FP64 readouts.  All device work goes
// to the state's HIP stream; nothing here computes amplitudes on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "internal.h"
#include "launch.h"
#include "lookahead.h"
#include "qsim.h"

using namespace qsim;

// ------------------------------------------------------------------ errors

namespace {

// Message of the last failing call, per thread (a fixed buffer, so that
// recording an error never allocates).
thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory)
        return fail(QSIM_ENOMEM, "%s: out of device memory", what);
    return fail(QSIM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                     \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess)                   \
            return hip_fail(e_, what);          \
    } while (0)

struct PendingTiming {
    hipEvent_t start, stop;
    int kind;      // 0 plain pass, 1 fused pass, 2 other
    double bytes;
    double flops;
};

}  // namespace

namespace qsim {

int set_error(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace qsim

// ------------------------------------------------------------------- state

struct qsim_state {
    int M = 0;
    int dtype = QSIM_C64;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *psi = nullptr;
    size_t bytes = 0;
    bool own_mem = false;
    uint64_t step = 0;
    bool armed = false;
    qsim_error_model em{};
    int renorm_period = 0;   // 0 = never
    int exec_mode = 0;
    bool lazy = false;       // fused passes visit the touched qubits only
    int remap = 0;           // qubit remap: 0 automatic, 1 eager, -1 never
    uint64_t active = 0;     // touched qubits: amplitudes spread over both values
    uint64_t fixed = 0;      // the value of every untouched qubit
    bool init_pending = false;  // reset to basis state init_index, not yet written
    uint64_t init_index = 0;
    int tile_bits = 13;
    int low_bits = 5;
    int group_bits = 5;
    double *d_partial = nullptr;   // reduction partials
    size_t partial_len = 0;
    double *d_tile_norm = nullptr; // per-tile norms of a fused pass
    double *d_scalars = nullptr;   // [0..3] overlap / norm, [4] norm sum, [5] scale
    double *h_pinned = nullptr;    // 16 doubles
    void *d_stage = nullptr;
    size_t stage_bytes = 0;
    bool profiling = false;
    qsim_stats stats{};
    std::vector<PendingTiming> pending;
    std::vector<hipEvent_t> free_events;
};

namespace {

size_t elem_bytes(int dtype) { return dtype == QSIM_C64 ? 8 : 16; }

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    if (v == nullptr || *v == 0)
        return dflt;
    return atoi(v);
}

// ------------------------------------------------------------ profiling

hipEvent_t take_event(qsim_state *s)
{
    if (!s->free_events.empty()) {
        hipEvent_t e = s->free_events.back();
        s->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

int flush_timings(qsim_state *s)
{
    if (s->pending.empty())
        return QSIM_OK;
    HIP_TRY(hipStreamSynchronize(s->stream), "timing sync");
    for (const PendingTiming &p : s->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
            if (p.kind == 0 || p.kind == 1) {
                s->stats.pass_ms += ms;
                s->stats.pass_bytes += p.bytes;
            }
            if (p.kind == 1) {
                s->stats.fused_ms += ms;
                s->stats.fused_bytes += p.bytes;
                s->stats.fused_flops += p.flops;
            }
            if (p.kind == 2)
                s->stats.other_ms += ms;
        }
        s->free_events.push_back(p.start);
        s->free_events.push_back(p.stop);
    }
    s->pending.clear();
    return QSIM_OK;
}

// Wraps one launch with events when profiling.
struct Timed {
    qsim_state *s;
    hipEvent_t a = nullptr;
    int kind;
    double bytes;
    double flops;
    Timed(qsim_state *st, int kd, double by, double fl = 0.0)
        : s(st), kind(kd), bytes(by), flops(fl)
    {
        if (s->profiling) {
            a = take_event(s);
            if (a)
                (void)hipEventRecord(a, s->stream);
        }
    }
    void done()
    {
        if (!s->profiling || a == nullptr)
            return;
        hipEvent_t b = take_event(s);
        if (b == nullptr)
            return;
        (void)hipEventRecord(b, s->stream);
        s->pending.push_back({a, b, kind, bytes, flops});
        if (s->pending.size() > 8192)
            flush_timings(s);
    }
};

// ---------------------------------------------------------------- lowering

constexpr size_t kMaxLdsBytes = 160 * 1024;  // gfx950 LDS per workgroup

constexpr double kSqrtHalf = 0.70710678118654752440084436210485;

}  // namespace

bool qsim::gate_valid(const qsim_gate &g, int M, char *why, size_t n)
{
    int need;
    switch (g.kind) {
    case QSIM_H: case QSIM_RZ: case QSIM_X: case QSIM_Z: need = 0; break;
    case QSIM_CNOT: case QSIM_CPHASE: need = 1; break;
    case QSIM_TOFFOLI: need = 2; break;
    default: snprintf(why, n, "unknown gate kind %u", g.kind); return false;
    }
    if (g.target < 0 || g.target >= M) {
        snprintf(why, n, "target %d outside [0, %d)", g.target, M);
        return false;
    }
    const int c[2] = {g.ctrl0, g.ctrl1};
    for (int i = 0; i < 2; ++i) {
        const bool used = i < need;
        if (!used && c[i] != -1) {
            snprintf(why, n, "gate kind %u takes %d control(s)", g.kind, need);
            return false;
        }
        if (used && (c[i] < 0 || c[i] >= M)) {
            snprintf(why, n, "control %d outside [0, %d)", c[i], M);
            return false;
        }
        if (used && c[i] == g.target) {
            snprintf(why, n, "control %d equals the target", c[i]);
            return false;
        }
    }
    if (need == 2 && g.ctrl0 == g.ctrl1) {
        snprintf(why, n, "repeated control %d", g.ctrl0);
        return false;
    }
    if (!std::isfinite(g.theta)) {
        snprintf(why, n, "non-finite theta");
        return false;
    }
    return true;
}

bool qsim::error_model_valid(const qsim_error_model &em)
{
    return em.sigma >= 0.0 && std::isfinite(em.sigma) && em.p_bitflip >= 0.0 &&
           em.p_bitflip <= 1.0 && em.p_phaseflip >= 0.0 && em.p_phaseflip <= 1.0;
}

namespace {

// The 2x2 of a gate with angle error eps (FP64).  eps == 0 gives the textbook
// gate; otherwise the gate is i R_n(pi + eps) about its own axis n, and Rz(t)
// and CPHASE(t) take t + eps.
Op lower_gate(const qsim_gate &g, double eps, bool inverse)
{
    Op op{};
    op.target = g.target;
    op.cmask = 0;
    if (g.ctrl0 >= 0)
        op.cmask |= 1ull << g.ctrl0;
    if (g.ctrl1 >= 0)
        op.cmask |= 1ull << g.ctrl1;
    const double c = std::cos(0.5 * eps), sn = std::sin(0.5 * eps);
    auto set = [&](int idx, double re, double im) {
        op.u[2 * idx] = re;
        op.u[2 * idx + 1] = im;
    };
    switch (g.kind) {
    case QSIM_H: {
        op.type = kOpMat;
        if (eps == 0.0) {
            set(0, kSqrtHalf, 0); set(1, kSqrtHalf, 0); set(2, kSqrtHalf, 0); set(3, -kSqrtHalf, 0);
        } else {
            const double ch = c * kSqrtHalf;
            set(0, ch, -sn); set(1, ch, 0); set(2, ch, 0); set(3, -ch, -sn);
        }
        break;
    }
    case QSIM_RZ: {
        op.type = kOpDiag;
        const double phi = (inverse ? -g.theta : g.theta) + eps;
        const double cp = std::cos(0.5 * phi), sp = std::sin(0.5 * phi);
        set(0, cp, -sp); set(3, cp, sp);
        break;
    }
    case QSIM_CPHASE: {
        // diag(1, e^{i phi}) on the target where the control is set (the
        // conditional rotations of the quantum FFT, Sec. 2.2)
        op.type = kOpDiag;
        const double phi = (inverse ? -g.theta : g.theta) + eps;
        set(0, 1, 0); set(3, std::cos(phi), std::sin(phi));
        break;
    }
    case QSIM_X: case QSIM_CNOT: case QSIM_TOFFOLI:
        if (eps == 0.0) {
            op.type = kOpSwap;
            set(1, 1, 0); set(2, 1, 0);
        } else {
            op.type = kOpMat;
            set(0, 0, -sn); set(1, c, 0); set(2, c, 0); set(3, 0, -sn);
        }
        break;
    default:  // QSIM_Z
        if (eps == 0.0) {
            op.type = kOpNeg;
            set(0, 1, 0); set(3, -1, 0);
        } else {
            op.type = kOpDiag;
            set(0, c, -sn); set(3, -c, -sn);
        }
        break;
    }
    return op;
}

// Gates plus the armed error model's draws -> operations (Sec. 2.0: angle
// deviation per gate; Sec. 3.4: two extra transforms after every operation).
void lower_circuit(const qsim_state *s, const qsim_gate *gates, size_t n, std::vector<Op> &ops)
{
    const bool ang = s->armed && s->em.sigma > 0.0;
    const bool flips = s->armed && (s->em.p_bitflip > 0.0 || s->em.p_phaseflip > 0.0);
    const uint64_t thr_b = flips ? flip_threshold(s->em.p_bitflip) : 0;
    const uint64_t thr_p = flips ? flip_threshold(s->em.p_phaseflip) : 0;
    ops.reserve(ops.size() + n);
    for (size_t k = 0; k < n; ++k) {
        const uint64_t step = s->step + k;
        const double eps = ang ? s->em.sigma * step_gaussian(s->em.seed, s->em.trial, step) : 0.0;
        Op op = lower_gate(gates[k], eps, false);
        op.step = step;
        op.is_flip = false;
        op.step_end = true;
        ops.push_back(op);
        if (!flips)
            continue;
        for (int q = 0; q < s->M; ++q) {
            const u64x4 r = philox4x64_10(step, (uint64_t)q, kStreamFlip, 0, s->em.seed, s->em.trial);
            const bool bf = (r.w[0] >> 32) < thr_b;
            const bool pf = (r.w[1] >> 32) < thr_p;
            if (!bf && !pf)
                continue;
            ops.back().step_end = false;
            if (bf) {
                Op x{};
                x.type = kOpSwap;
                x.target = q;
                x.u[2] = 1; x.u[4] = 1;
                x.step = step;
                x.is_flip = true;
                x.step_end = true;
                ops.push_back(x);
            }
            if (pf) {
                if (bf)
                    ops.back().step_end = false;
                Op z{};
                z.type = kOpNeg;
                z.target = q;
                z.u[0] = 1; z.u[6] = -1;
                z.step = step;
                z.is_flip = true;
                z.step_end = true;
                ops.push_back(z);
            }
        }
    }
}

// Algorithmic HBM bytes of one operation done as its own pass.
double plain_bytes(const qsim_state *s, const Op &op)
{
    const double full = 2.0 * (double)(1ull << s->M) * (double)elem_bytes(s->dtype);
    const int nc = __builtin_popcountll(op.cmask);
    double frac = 1.0 / (double)(1ull << nc);
    if (op.type == kOpNeg)
        frac *= 0.5;
    return full * frac;
}

// Algorithmic real flops of one operation over a 2^M register: the flops of
// its 2x2 per amplitude it updates (a real 2x2, or a perturbed X with its
// zero diagonal: 6; a real 2x2 plus i*w on the diagonal: 10; a diagonal
// phase: 6; a swap or sign flip: 0), on the 2^-c of the register that
// satisfies its c controls.
double op_flops(const Op &op, int M)
{
    double per = 0.0;
    const double *u = op.u;
    if (op.type == kOpMat)
        per = (u[1] != 0.0 || u[7] != 0.0) && (u[0] != 0.0 || u[6] != 0.0) ? 10.0 : 6.0;
    else if (op.type == kOpDiag)
        per = 6.0;
    return per * std::ldexp(1.0, M - __builtin_popcountll(op.cmask));
}

// ------------------------------------------------------------- scheduling

struct PassPlan {
    bool fused;
    size_t first, count;
    bool norm_after;   // compute the norm after this pass (renorm boundary)
};

// Operations whose target must be a tile qubit of a fused pass (and a group
// bit inside it): everything but uncontrolled diagonals.
bool needs_tile_target(const Op &op)
{
    return op.type == kOpMat || op.type == kOpSwap || op.cmask != 0;
}

// Operations a fused pass can carry: everything but a 2x2 with complex
// off-diagonal entries (no gate of the set lowers to one; such an operation
// gets a pass of its own).
bool fusable(const Op &op)
{
    return !(op.type == kOpMat && (op.u[3] != 0.0 || op.u[5] != 0.0));
}

bool renorm_due(const qsim_state *s, const Op &op)
{
    return s->renorm_period > 0 && op.step_end && ((op.step + 1) % (uint64_t)s->renorm_period) == 0;
}

// Mark the operations after which a renormalisation boundary falls, before
// the stream is rewritten or reordered.
void mark_norms(const qsim_state *s, std::vector<Op> &ops)
{
    for (Op &op : ops) {
        op.norm_mark = renorm_due(s, op);
        op.zdep = 0;
        op.activates = false;
        op.relocate = false;
    }
}

uint64_t full_mask(int M) { return M >= 64 ? ~0ull : ((1ull << M) - 1); }

Op exact_swap(int q, uint64_t step)
{
    Op x{};
    x.type = kOpSwap;
    x.target = q;
    x.u[2] = 1;
    x.u[4] = 1;
    x.step = step;
    return x;
}

// ------------------------------------------------------------ lazy qubits
//
// The flat form of the dynamically allocated state vector of Sec. 3.2: until
// an operation spreads a qubit over both of its values, the qubit has one
// definite value, every amplitude with the other value is exactly zero, and
// those need not be read, written or transformed.  The state records the
// qubits already spread ("touched", s->active) and the value of every other
// one (s->fixed); a fused pass walks only the tiles whose untouched qubits
// hold their values.  Before scheduling, the operation stream of a call is
// rewritten against that knowledge, in stream order:
//   - a control on an untouched qubit is decided: value 0 drops the
//     operation, value 1 drops the control (the operation keeps the qubit as
//     an ordering dependency, so the scheduler never moves it across the
//     qubit's first spreading operation);
//   - a diagonal (Rz, Z, CPHASE, a phase flip) whose target is untouched is a
//     scalar: without controls it joins a global phase, applied once at the
//     end of the call; with controls it becomes that phase on one of them;
//   - an exact uncontrolled X (a bit flip, an unperturbed X) on an untouched
//     qubit flips its logical value without moving data;
//   - every other operation on an untouched qubit spreads it (an exact swap
//     first moves its amplitudes to its logical value if that was flipped);
//   - at the end of the call, every untouched qubit whose value was flipped
//     gets one exact swap (its amplitudes move to the new value, and the qubit
//     stays untouched), and the global phase is applied as one scalar
//     operation: between calls the register holds the plain state vector.
// Every step is exact except the phase products, which round as the gates'
// own products would.
void lazy_rewrite(const qsim_state *s, std::vector<Op> &stream)
{
    std::vector<Op> out;
    out.reserve(stream.size() + 8);
    uint64_t act = s->active;
    uint64_t flipped = 0;              // untouched qubits whose value was flipped
    double ph_re = 1.0, ph_im = 0.0;   // global phase gathered so far
    const uint64_t last_step = stream.empty() ? 0 : stream.back().step;
    auto value = [&](int q) { return (((s->fixed ^ flipped) >> q) & 1ull) != 0; };
    // a dropped operation hands its renormalisation boundary to the one before
    auto dropped = [&](const Op &op) {
        if (op.norm_mark && !out.empty())
            out.back().norm_mark = true;
    };
    for (Op op : stream) {
        const uint64_t quiet = op.cmask & ~act;  // controls on untouched qubits
        bool met = true;
        for (uint64_t m = quiet; m != 0; m &= m - 1)
            met = met && value(__builtin_ctzll(m));
        if (!met) {
            dropped(op);
            continue;
        }
        op.cmask &= act;
        op.zdep = quiet;
        const uint64_t tb = 1ull << op.target;
        if (act & tb) {
            out.push_back(op);
            continue;
        }
        const bool v = value(op.target);
        if (op.type == kOpDiag || op.type == kOpNeg) {
            double fr = 1.0, fi = 0.0;  // the factor the target's value picks
            if (op.type == kOpNeg) {
                fr = v ? -1.0 : 1.0;
            } else {
                fr = v ? op.u[6] : op.u[0];
                fi = v ? op.u[7] : op.u[1];
            }
            if (fr == 1.0 && fi == 0.0) {
                dropped(op);
                continue;
            }
            if (op.cmask == 0) {
                const double r = ph_re * fr - ph_im * fi;
                ph_im = ph_re * fi + ph_im * fr;
                ph_re = r;
                dropped(op);
                continue;
            }
            // the factor where the touched controls are met: a diagonal on one
            // of them, controlled by the others
            Op d = op;
            const int c = __builtin_ctzll(op.cmask);
            d.target = c;
            d.cmask = op.cmask & ~(1ull << c);
            d.zdep |= tb;
            std::memset(d.u, 0, sizeof(d.u));
            d.u[0] = 1.0;
            if (fr == -1.0 && fi == 0.0) {
                d.type = kOpNeg;
                d.u[6] = -1.0;
            } else {
                d.type = kOpDiag;
                d.u[6] = fr;
                d.u[7] = fi;
            }
            out.push_back(d);
            continue;
        }
        if (op.type == kOpSwap && op.cmask == 0) {
            flipped ^= tb;
            dropped(op);
            continue;
        }
        // spreads its target
        if (flipped & tb) {
            Op x = exact_swap(op.target, op.step);
            x.activates = true;
            out.push_back(x);
            flipped &= ~tb;
        }
        op.activates = true;
        act |= tb;
        out.push_back(op);
    }
    for (uint64_t m = flipped; m != 0; m &= m - 1) {
        Op x = exact_swap(__builtin_ctzll(m), last_step);
        x.relocate = true;
        out.push_back(x);
    }
    if (ph_re != 1.0 || ph_im != 0.0) {
        Op p{};
        p.type = kOpDiag;
        p.target = 0;
        p.u[0] = ph_re; p.u[1] = ph_im;
        p.u[6] = ph_re; p.u[7] = ph_im;
        p.step = last_step;
        out.push_back(p);
    }
    stream.swap(out);
}

// Shape of the fused passes of a state: k tile qubits, G group bits per
// register quantum, 2^(k-G) threads per workgroup with 6 <= k - G <= 9.
// False when the register is too small for a fused pass (M < 9).
bool tile_shape(const qsim_state *s, int &k, int &G)
{
    k = std::min(s->tile_bits, s->M);
    G = std::min(std::max(s->group_bits, k - 9), k - 6);
    return G >= 3 && G <= 5;
}

// Qubits an operation acts on as the target of a non-diagonal transform
// (x), and as a control or the target of a diagonal one (z).  Two operations
// commute when neither one's x qubits meet the other's x or z qubits: they
// then act on disjoint qubits, or share only qubits on which both are
// diagonal in the computational basis.
struct OpUse {
    uint64_t x, z;
};

OpUse op_use(const Op &op)
{
    const uint64_t t = 1ull << op.target;
    const bool diag = op.type == kOpDiag || op.type == kOpNeg;
    return {diag ? 0ull : t, op.cmask | op.zdep | (diag ? t : 0ull)};
}

// Lookahead of the tile-set and group choices: the next kWindow operations,
// up to kMaxExchanges exchanges.
constexpr size_t kWindow = 64;
constexpr int kMaxExchanges = 4;

// Reorder the operations of one fused pass, order[first, first + count), so
// that they fall into few register groups (each group is one LDS
// re-partition of the tile): repeatedly take, in order, every operation that
// commutes with the operations left behind and whose target fits a set of at
// most G qubits (uncontrolled diagonals fit any set).
void cluster_pass(const std::vector<Op> &ops, std::vector<uint32_t> &order, size_t first,
                  size_t count, int G)
{
    std::vector<uint32_t> rem(order.begin() + (std::ptrdiff_t)first,
                              order.begin() + (std::ptrdiff_t)(first + count));
    std::vector<uint32_t> left, out;
    out.reserve(count);
    std::vector<ScanOp> w;
    while (!rem.empty()) {
        // the group's target bits by the same lookahead as a pass's tile set
        w.clear();
        for (const uint32_t idx : rem) {
            const Op &op = ops[idx];
            const OpUse u = op_use(op);
            w.push_back({u.x, u.z, needs_tile_target(op) ? (1ull << op.target) : 0ull});
        }
        uint64_t cur = lookahead_set(w, 0, G, w.size(), kMaxExchanges), bx = 0, bz = 0;
        int ncur = __builtin_popcountll(cur);
        left.clear();
        for (const uint32_t idx : rem) {
            const Op &op = ops[idx];
            const OpUse u = op_use(op);
            bool ok = (u.x & (bx | bz)) == 0 && (u.z & bx) == 0;
            if (ok && needs_tile_target(op)) {
                const uint64_t tb = 1ull << op.target;
                if (!(cur & tb)) {
                    if (ncur == G) {
                        ok = false;
                    } else {
                        cur |= tb;
                        ++ncur;
                    }
                }
            }
            if (ok) {
                out.push_back(idx);
            } else {
                left.push_back(idx);
                bx |= u.x;
                bz |= u.z;
            }
        }
        rem.swap(left);
    }
    std::copy(out.begin(), out.end(), order.begin() + (std::ptrdiff_t)first);
}

// Tile set of the next fused pass in reorder mode, by lookahead over the
// next kWindow operations with up to kMaxExchanges exchanges (the 1000-gate
// random circuits at 30 qubits: 30-33 passes instead of 36-39 with sets
// filled first come, first served; with the group lookahead about 5 ms of
// host time per 1000 gates).

uint64_t choose_tile_set(const std::vector<Op> &ops, const std::vector<uint32_t> &rem,
                         uint64_t S0, int k, size_t cap)
{
    const size_t W = std::min(rem.size(), kWindow);
    std::vector<ScanOp> w(W);
    for (size_t i = 0; i < W; ++i) {
        const Op &op = ops[rem[i]];
        const OpUse u = op_use(op);
        w[i] = {u.x, u.z, needs_tile_target(op) ? (1ull << op.target) : 0ull};
    }
    return lookahead_set(w, S0, k, cap, kMaxExchanges);
}

// One fused pass taken from the operations `rem` not yet placed (stream
// indices, in stream order; what the pass leaves behind stays in `rem`),
// appending its operations to `order`.  A pass starts with the low qubits in
// its tile set (plus, in reorder mode, the qubits choose_tile_set picks) and
// scans the operations not yet placed, in stream order: it takes an
// operation when the operation commutes with every earlier one still left
// behind and its target is in the tile set or the set has room for it
// (diagonal operations without controls never constrain the set).  In-order
// mode stops the scan at the first operation it cannot take instead, so
// passes are runs of the stream.  Every pass takes at least one operation:
// the first one left commutes with nothing earlier, and either the set has
// room for its target or the set was chosen to take something from the
// window.
PassPlan fused_pass(const qsim_state *s, const std::vector<Op> &ops, std::vector<uint32_t> &rem,
                    std::vector<uint32_t> &left, int k, int G, bool reorder,
                    std::vector<uint32_t> &order)
{
    const int low = std::min(s->low_bits, k);
    const size_t cap = s->dtype == QSIM_C64 ? (size_t)kPassOps<float> : (size_t)kPassOps<double>;
    uint64_t S = (low >= 64) ? ~0ull : ((1ull << low) - 1);
    if (reorder)
        S = choose_tile_set(ops, rem, S, k, cap);
    int size = __builtin_popcountll(S);
    uint64_t bx = 0, bz = 0;  // qubits held by operations left behind
    const size_t first = order.size();
    size_t taken = 0;
    left.clear();
    for (size_t r = 0; r < rem.size(); ++r) {
        const Op &op = ops[rem[r]];
        const OpUse u = op_use(op);
        bool ok = taken < cap && (u.x & (bx | bz)) == 0 && (u.z & bx) == 0;
        if (ok && needs_tile_target(op)) {
            const uint64_t tb = 1ull << op.target;
            if (!(S & tb)) {
                if (size == k) {
                    ok = false;
                } else {
                    S |= tb;
                    ++size;
                }
            }
        }
        if (ok) {
            order.push_back(rem[r]);
            ++taken;
            continue;
        }
        if (!reorder || taken == cap) {
            left.insert(left.end(), rem.begin() + (std::ptrdiff_t)r, rem.end());
            break;
        }
        left.push_back(rem[r]);
        bx |= u.x;
        bz |= u.z;
    }
    if (reorder)
        cluster_pass(ops, order, first, taken, G);
    rem.swap(left);
    return {true, first, taken, false};
}

// Partition the operation stream into passes and fix the order in which the
// operations run (order[i] = stream index of the i-th operation to run), one
// pass at a time, so that a caller can launch each pass while the next one is
// planned.  An operation a fused pass cannot carry gets a pass of its own,
// and no operation moves across it.  Plain mode, and registers too small for
// a tile (M < 9), run one pass per operation in stream order.
//
// Renormalisation is a scaling of the whole state, which commutes with every
// operation, so it does not pin the order: the norm is taken after the first
// pass by which every operation up to a renormalisation boundary has run
// (several boundaries may share one), and the next pass applies the scale.
class PassScheduler {
public:
    PassScheduler(const qsim_state *s, const std::vector<Op> &ops)
        : s_(s), ops_(ops), n_(ops.size()), ran_(ops.size(), false)
    {
        plain_ = s->exec_mode == 1 || !tile_shape(s, k_, G_);
        reorder_ = s->exec_mode == 0;
        if (!plain_)
            open_segment(0);
    }

    // The next pass (its operations appended to order); false when done.
    bool next(std::vector<uint32_t> &order, PassPlan &p)
    {
        if (plain_) {
            if (i_ >= n_)
                return false;
            order.push_back((uint32_t)i_);
            p = {false, order.size() - 1, 1, false};
            ++i_;
        } else if (!rem_.empty()) {
            p = fused_pass(s_, ops_, rem_, left_, k_, G_, reorder_, order);
        } else if (seg_end_ < n_) {
            // the operation that ended the segment, then the next segment
            order.push_back((uint32_t)seg_end_);
            p = {false, order.size() - 1, 1, false};
            open_segment(seg_end_ + 1);
        } else {
            return false;
        }
        for (size_t i = p.first; i < p.first + p.count; ++i)
            ran_[order[i]] = true;
        while (prefix_ < n_ && ran_[prefix_])
            ++prefix_;
        for (; next_ < prefix_; ++next_)
            if (ops_[next_].norm_mark)
                p.norm_after = true;
        return true;
    }

private:
    // operations [lo, first operation a fused pass cannot carry) become rem_
    void open_segment(size_t lo)
    {
        seg_end_ = lo;
        while (seg_end_ < n_ && fusable(ops_[seg_end_]))
            ++seg_end_;
        rem_.clear();
        for (size_t i = lo; i < seg_end_; ++i)
            rem_.push_back((uint32_t)i);
    }

    const qsim_state *s_;
    const std::vector<Op> &ops_;
    size_t n_;
    int k_ = 0, G_ = 0;
    bool plain_ = true, reorder_ = false;
    size_t i_ = 0;                   // plain mode: next operation
    size_t seg_end_ = 0;             // fused mode: end of the current segment
    std::vector<uint32_t> rem_, left_;
    std::vector<bool> ran_;
    size_t prefix_ = 0;  // every stream index below it has run
    size_t next_ = 0;    // next operation to check for a boundary
};

void schedule(const qsim_state *s, const std::vector<Op> &ops, std::vector<uint32_t> &order,
              std::vector<PassPlan> &plan)
{
    order.clear();
    order.reserve(ops.size());
    PassScheduler sched(s, ops);
    PassPlan p;
    while (sched.next(order, p))
        plan.push_back(p);
}

// Runs of consecutive qubits in `mask` (below qubit M).
int count_runs(uint64_t mask, int M)
{
    int n = 0;
    for (int q = 0; q < M; ++q)
        if (((mask >> q) & 1u) && (q == 0 || !((mask >> (q - 1)) & 1u)))
            ++n;
    return n;
}

// Qubits the tiles of a pass over tile set S enumerate: the touched qubits
// outside S.  Where they fall into more runs than the kernel's run table
// holds, the untouched qubits of the narrowest gaps between runs are
// enumerated too (their other value's tiles are zero and stay zero); gaps that
// hold a tile qubit cannot close, but there are at most |S| + 1 of them.
uint64_t pass_enumerated(uint64_t act, uint64_t S, int M)
{
    uint64_t E = act & full_mask(M) & ~S;
    while (count_runs(E, M) > kMaxRuns) {
        int best_lo = -1, best_len = 0;
        for (int q = 0; q < M;) {
            if ((E >> q) & 1u) {
                ++q;
                continue;
            }
            int e = q;
            while (e < M && !((E >> e) & 1u))
                ++e;
            const bool inner = q > 0 && e < M;
            const uint64_t gap = full_mask(e - q) << q;
            if (inner && (gap & S) == 0 && (best_lo < 0 || e - q < best_len)) {
                best_lo = q;
                best_len = e - q;
            }
            q = e;
        }
        if (best_lo < 0)
            break;
        E |= full_mask(best_len) << best_lo;
    }
    return E;
}

// Build the kernel arguments of one fused pass.  act: qubits touched when the
// pass runs; fixed: the values of the others.
template <typename R>
void build_tile_args(const qsim_state *s, const std::vector<Op> &ops, const PassPlan &p,
                     uint64_t act, uint64_t fixed, TileArgs<R> &A, int &G)
{
    const int M = s->M;
    int k;
    tile_shape(s, k, G);
    const int low = std::min(s->low_bits, k);
    // tile qubit set: low qubits, then the pass's targets, then the lowest free
    // qubits (touched ones first)
    uint64_t S = (1ull << low) - 1;
    for (size_t o = p.first; o < p.first + p.count; ++o)
        if (needs_tile_target(ops[o]))
            S |= 1ull << ops[o].target;
    for (int q = 0; q < M && __builtin_popcountll(S) < k; ++q)
        if ((act >> q) & 1u)
            S |= 1ull << q;
    for (int q = 0; q < M && __builtin_popcountll(S) < k; ++q)
        S |= 1ull << q;
    const uint64_t E = pass_enumerated(act, S, M);
    std::memset(&A, 0, sizeof(A));
    A.M = (uint32_t)M;
    A.k = (uint32_t)k;
    A.low = (uint32_t)low;
    A.smask = S;
    A.emask = E;
    A.base_or = fixed & full_mask(M) & ~S & ~E;
    A.mact = (uint32_t)__builtin_popcountll(S | E);
    int tpos_of[64];
    int m = 0;
    for (int q = 0; q < M; ++q) {
        if (S & (1ull << q)) {
            A.spos[m] = (uint8_t)q;
            tpos_of[q] = m++;
        } else {
            tpos_of[q] = -1;
        }
    }
    // runs of consecutive qubits of S and of E, ascending (untouched qubits
    // outside both are skipped: base_or holds their values)
    for (int q = 0; q < M;) {
        const int kind = ((S >> q) & 1u) ? 1 : ((E >> q) & 1u) ? 2 : 0;
        int e = q + 1;
        while (e < M && (((S >> e) & 1u) ? 1 : ((E >> e) & 1u) ? 2 : 0) == kind)
            ++e;
        if (kind != 0) {
            uint32_t &n = kind == 1 ? A.nsrun : A.ncrun;
            if (n < (uint32_t)kMaxRuns)
                (kind == 1 ? A.srun : A.crun)[n] = (uint32_t)q | ((uint32_t)(e - q) << 8);
            ++n;  // past kMaxRuns the consistency check rejects the pass
        }
        q = e;
    }
    // operations, grouped so that the targets that need a group bit span at
    // most G tile bits per group
    A.nops = (uint32_t)p.count;
    std::vector<uint32_t> cur;  // tile bits of the current group
    uint32_t gfirst = 0;
    std::vector<std::pair<uint32_t, std::vector<uint32_t>>> groups;  // (first | count, bits)
    auto close_group = [&](uint32_t end) {
        if (end == gfirst)
            return;
        groups.push_back({gfirst | ((end - gfirst) << kGroupCountShift), cur});
        cur.clear();
        gfirst = end;
    };
    for (uint32_t o = 0; o < A.nops; ++o) {
        const Op &op = ops[p.first + o];
        if (needs_tile_target(op)) {
            const uint32_t tp = (uint32_t)tpos_of[op.target];
            if (std::find(cur.begin(), cur.end(), tp) == cur.end()) {
                if ((int)cur.size() == G)
                    close_group(o);
                cur.push_back(tp);
            }
        }
    }
    close_group(A.nops);
    A.ngroups = (uint32_t)groups.size();
    double phase_re = 1.0, phase_im = 0.0;  // global phase of the pass's diagonals
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        std::vector<uint32_t> bits = groups[gi].second;
        auto absent = [&](uint32_t b) {
            return std::find(bits.begin(), bits.end(), b) == bits.end();
        };
        // pad first with the tile bits that the group's uncontrolled
        // diagonal operations act on, most used first (on a group bit such
        // an operation scales half of the registers; on any other bit it
        // costs a factor on all of them), then with the highest free tile
        // bits (keeps tile bit 0 outside the group, so neighbouring threads
        // touch neighbouring LDS words)
        {
            const uint32_t gf = group_first(groups[gi].first), gc = group_count(groups[gi].first);
            int uses[64] = {0};
            for (uint32_t o = gf; o < gf + gc; ++o) {
                const Op &op = ops[p.first + o];
                if (!needs_tile_target(op) && tpos_of[op.target] >= 0)
                    ++uses[tpos_of[op.target]];
            }
            while ((int)bits.size() < G) {
                int best = -1;
                for (int b = 0; b < k; ++b)
                    if (uses[b] > 0 && absent((uint32_t)b) && (best < 0 || uses[b] > uses[best]))
                        best = b;
                if (best < 0)
                    break;
                bits.push_back((uint32_t)best);
            }
        }
        for (int b = k - 1; b >= 0 && (int)bits.size() < G; --b)
            if (absent((uint32_t)b))
                bits.push_back((uint32_t)b);
        std::sort(bits.begin(), bits.end());
        uint32_t w = groups[gi].first;
        for (int i = 0; i < G; ++i)
            w |= bits[i] << (kGroupBitsShift + 4 * i);
        A.group[gi] = w;
        auto gidx = [&](int q) -> int {
            if (tpos_of[q] < 0)
                return -1;
            const auto it = std::find(bits.begin(), bits.end(), (uint32_t)tpos_of[q]);
            return it == bits.end() ? -1 : (int)(it - bits.begin());
        };
        const uint32_t first = group_first(w), cnt = group_count(w);
        for (uint32_t o = first; o < first + cnt && o < A.nops; ++o) {
            const Op &op = ops[p.first + o];
            TileOp<R> &t = A.ops[o];
            std::memset(&t, 0, sizeof(t));
            t.tq = (uint32_t)op.target;
            t.tpos = tpos_of[op.target] >= 0 ? (uint32_t)tpos_of[op.target] : kNoPos;
            const int gp = gidx(op.target);
            t.gpos = gp >= 0 ? (uint8_t)gp : (uint8_t)0;
            for (int q = 0; q < M; ++q) {
                if (!(op.cmask & (1ull << q)))
                    continue;
                const int cg = gidx(q);
                if (tpos_of[q] < 0)
                    t.cm_out |= 1ull << q;
                else if (cg >= 0)
                    t.rc |= (uint8_t)(1u << cg);
                else
                    t.qc |= 1u << tpos_of[q];
            }
            const double *u = op.u;
            switch (op.type) {
            case kOpMat:
                // real off-diagonal (fusable() admits no other matrix): real
                // 2x2 plus i*w on the diagonal
                t.kind = kTPair;
                if (op.cmask == 0 && u[0] != 0.0 && u[2] == u[0] && u[4] == u[0] &&
                    u[6] == -u[0] && u[7] == u[1]) {
                    // h [[1, 1], [1, -1]] + i w (a Hadamard, perturbed or
                    // not) = h ([[1, 1], [1, -1]] + i w/h): the real scalar h
                    // joins the pass's global phase and the pair becomes a
                    // butterfly, a +- b plus i (w/h) on the diagonal
                    const double h = u[0], tw = u[1] / h;
                    phase_re *= h;
                    phase_im *= h;
                    t.c[4] = (R)tw; t.c[5] = (R)tw;
                    t.form = tw != 0.0 ? 3 : 4;
                    break;
                }
                t.c[0] = (R)u[0]; t.c[1] = (R)u[2]; t.c[2] = (R)u[4]; t.c[3] = (R)u[6];
                t.c[4] = (R)u[1]; t.c[5] = (R)u[7];
                t.form = (u[1] != 0.0 || u[7] != 0.0) ? (u[0] == 0.0 && u[6] == 0.0 ? 2 : 1) : 0;
                break;
            case kOpSwap:
                t.kind = kTSwap;
                break;
            case kOpDiag:
                if (op.cmask == 0) {
                    // diag(d0, d1) = d0 diag(1, d1/d0): d0 multiplies the
                    // whole register and joins the pass's global phase
                    const double d0r = u[0], d0i = u[1], d1r = u[6], d1i = u[7];
                    const double n0 = d0r * d0r + d0i * d0i;
                    const double qr = (d1r * d0r + d1i * d0i) / n0;
                    const double qi = (d1i * d0r - d1r * d0i) / n0;
                    const double pr = phase_re * d0r - phase_im * d0i;
                    phase_im = phase_re * d0i + phase_im * d0r;
                    phase_re = pr;
                    t.kind = gp >= 0 ? kTPhaseIn : kTDiagOut;
                    t.c[0] = R(1); t.c[1] = R(0); t.c[2] = (R)qr; t.c[3] = (R)qi;
                } else {
                    t.kind = kTDiagIn;
                    t.c[0] = (R)u[0]; t.c[1] = (R)u[1]; t.c[2] = (R)u[6]; t.c[3] = (R)u[7];
                }
                break;
            default:
                t.kind = gp >= 0 ? kTNegIn : kTNegOut;
                break;
            }
        }
    }
    A.phase[0] = (R)phase_re;
    A.phase[1] = (R)phase_im;
    A.use_phase = (phase_re != 1.0 || phase_im != 0.0) ? 1u : 0u;
}

// Internal consistency of a fused pass's arguments (used by qsim_plan).
template <typename R>
bool tile_args_consistent(const TileArgs<R> &A, int G, const std::vector<Op> &ops,
                          const PassPlan &p, char *why, size_t n)
{
    if (A.nops != p.count || A.nops == 0 || A.nops > (uint32_t)kPassOps<R>) {
        snprintf(why, n, "op count %u", A.nops);
        return false;
    }
    if (A.ngroups == 0 || A.ngroups > (uint32_t)kMaxGroups) {
        snprintf(why, n, "group count %u", A.ngroups);
        return false;
    }
    if ((uint64_t)__builtin_popcountll(A.smask) != A.k || A.k - (uint32_t)G < 6 || A.k - (uint32_t)G > 9) {
        snprintf(why, n, "tile set / shape");
        return false;
    }
    // the run tables must spell the tile set and its complement, in order
    uint64_t sm = 0, cm = 0;
    uint32_t sl = 0, cl = 0;
    for (uint32_t i = 0; i < A.nsrun && i < (uint32_t)kMaxRuns; ++i) {
        sm |= ((1ull << (A.srun[i] >> 8)) - 1) << (A.srun[i] & 0xFFu);
        sl += A.srun[i] >> 8;
        if (i > 0 && (A.srun[i] & 0xFFu) <= (A.srun[i - 1] & 0xFFu))
            sm = 0;
    }
    for (uint32_t i = 0; i < A.ncrun && i < (uint32_t)kMaxRuns; ++i) {
        cm |= ((1ull << (A.crun[i] >> 8)) - 1) << (A.crun[i] & 0xFFu);
        cl += A.crun[i] >> 8;
        if (i > 0 && (A.crun[i] & 0xFFu) <= (A.crun[i - 1] & 0xFFu))
            cm = 0;
    }
    const uint64_t full = full_mask((int)A.M);
    if (A.nsrun > (uint32_t)kMaxRuns || A.ncrun > (uint32_t)kMaxRuns || sm != A.smask ||
        cm != A.emask || (A.emask & A.smask) != 0 || (A.emask & ~full) != 0 || sl != A.k ||
        A.mact != A.k + (uint32_t)__builtin_popcountll(A.emask) || cl != A.mact - A.k ||
        (A.base_or & (A.smask | A.emask | ~full)) != 0) {
        snprintf(why, n, "run tables");
        return false;
    }
    uint32_t next = 0;
    for (uint32_t gi = 0; gi < A.ngroups; ++gi) {
        const uint32_t w = A.group[gi];
        if (group_first(w) != next || group_count(w) == 0) {
            snprintf(why, n, "group %u does not continue at op %u", gi, next);
            return false;
        }
        next += group_count(w);
        uint32_t seen = 0;
        for (int i = 0; i < G; ++i) {
            const uint32_t b = group_bit(w, i);
            if (b >= A.k || (seen >> b) & 1u || (i > 0 && b <= group_bit(w, i - 1))) {
                snprintf(why, n, "group %u bits", gi);
                return false;
            }
            seen |= 1u << b;
        }
        for (uint32_t o = group_first(w); o < next; ++o) {
            const Op &op = ops[p.first + o];
            const TileOp<R> &t = A.ops[o];
            const bool in_tile = (A.smask >> op.target) & 1u;
            if ((t.kind == kTPhaseIn || t.kind >= kTDiagOut) && op.cmask != 0) {
                snprintf(why, n, "op %u: controlled diagonal taken as a phase", o);
                return false;
            }
            if (t.kind <= kTNegIn) {
                if (!in_tile || t.gpos >= (uint32_t)G || group_bit(w, t.gpos) != t.tpos) {
                    snprintf(why, n, "op %u target not on its group bit", o);
                    return false;
                }
            } else if (op.cmask != 0) {
                snprintf(why, n, "op %u: controlled diagonal folded", o);
                return false;
            }
            // controls and diagonal targets outside the tile must be qubits
            // the tile number enumerates (untouched ones were decided)
            if ((t.cm_out & ~A.emask) != 0 ||
                (t.kind >= kTDiagOut && t.tpos == kNoPos && !((A.emask >> op.target) & 1u))) {
                snprintf(why, n, "op %u reads an untouched qubit outside the tile", o);
                return false;
            }
            // the three control masks must rebuild the op's control set
            uint64_t back = t.cm_out;
            for (int i = 0; i < G; ++i)
                if ((t.rc >> i) & 1u)
                    back |= 1ull << A.spos[group_bit(w, i)];
            for (uint32_t m = 0; m < A.k; ++m)
                if ((t.qc >> m) & 1u)
                    back |= 1ull << A.spos[m];
            if (back != op.cmask) {
                snprintf(why, n, "op %u control masks", o);
                return false;
            }
        }
    }
    if (next != A.nops) {
        snprintf(why, n, "groups cover %u of %u ops", next, A.nops);
        return false;
    }
    return true;
}

// ------------------------------------------------------------ qubit remap
//
// The one-GPU form of the paper's reorganisation of the state (Sec. 3.1,
// Sec. 3.3 and Fig. 8: work on a chosen set of qubits, move the data when
// the set must change, and do that rarely).  A fused pass reads each tile as
// runs of 2^low contiguous amplitudes; a tile that spans the top qubits of a
// large register gathers its runs from addresses 2^(M-1) elements apart,
// which the memory system serves more slowly (at M = 33 the same pass runs
// about a tenth faster once those qubits are low).  When a call's operations
// use a few top qubits much more often than the low ones just above the
// always-tiled qubits, the call exchanges each such pair first (an exact
// swap: three CNOT exchanges, fused into the first pass like any other
// operation), applies every operation to the exchanged positions, and
// exchanges them back at its end, so between calls the register keeps its
// plain layout and every readout is unchanged.
constexpr int kRemapMinQubits = 31;  // automatic remap from this register size
constexpr int kRemapWindow = 6;      // top qubits that may move, low ones that may take them
constexpr int kRemapPairs = 4;

void choose_remap(const qsim_state *s, const std::vector<Op> &ops,
                  std::vector<std::pair<int, int>> &pairs)
{
    pairs.clear();
    int k, G;
    if (s->remap < 0 || s->exec_mode == 1 || !tile_shape(s, k, G))
        return;
    const int M = s->M, low = std::min(s->low_bits, k);
    // automatic only for complex64: a complex128 tile's runs are twice as
    // long, and there the exchange passes cost more than they save (measured
    // at M = 32: 3 % slower over 500 gates; complex64 at M = 33: 1 % faster)
    if ((s->remap == 0 && (M < kRemapMinQubits || s->dtype != QSIM_C64)) ||
        M - low < 2 * kRemapWindow)
        return;
    int uses[64] = {0};
    for (const Op &op : ops)
        if (needs_tile_target(op))
            ++uses[op.target];
    std::vector<int> hot, cold;
    for (int i = 0; i < kRemapWindow; ++i) {
        hot.push_back(M - 1 - i);
        cold.push_back(low + i);
    }
    std::stable_sort(hot.begin(), hot.end(), [&](int a, int b) { return uses[a] > uses[b]; });
    std::stable_sort(cold.begin(), cold.end(), [&](int a, int b) { return uses[a] < uses[b]; });
    // automatic: a top qubit must carry at least 1/50 of the operations (8 at
    // least) and twice its partner's count plus that margin
    const int margin = s->remap > 0 ? 1 : std::max(8, (int)(ops.size() / 50));
    for (int i = 0; i < kRemapPairs; ++i)
        if (uses[hot[i]] >= margin && uses[hot[i]] >= 2 * uses[cold[i]] + margin)
            pairs.push_back({hot[i], cold[i]});
}

void apply_remap(const std::vector<std::pair<int, int>> &pairs, std::vector<Op> &stream)
{
    if (pairs.empty())
        return;
    int perm[64];
    for (int q = 0; q < 64; ++q)
        perm[q] = q;
    for (const auto &pr : pairs) {
        perm[pr.first] = pr.second;
        perm[pr.second] = pr.first;
    }
    auto move_mask = [&](uint64_t m) {
        uint64_t r = 0;
        for (; m != 0; m &= m - 1)
            r |= 1ull << perm[__builtin_ctzll(m)];
        return r;
    };
    const uint64_t step0 = stream.empty() ? 0 : stream.front().step;
    const uint64_t step1 = stream.empty() ? 0 : stream.back().step;
    auto exchange = [&](std::vector<Op> &out, uint64_t step) {
        for (const auto &pr : pairs) {
            const int a = pr.first, b = pr.second;
            const int seq[3][2] = {{b, a}, {a, b}, {b, a}};  // (target, control)
            for (const auto &tc : seq) {
                Op x = exact_swap(tc[0], step);
                x.cmask = 1ull << tc[1];
                out.push_back(x);
            }
        }
    };
    std::vector<Op> out;
    out.reserve(stream.size() + 6 * pairs.size());
    exchange(out, step0);
    for (Op op : stream) {
        op.target = perm[op.target];
        op.cmask = move_mask(op.cmask);
        out.push_back(op);
    }
    exchange(out, step1);
    stream.swap(out);
}

// A call's operation stream made ready for scheduling: renormalisation
// boundaries marked, the qubit remap chosen and applied, then (lazy states)
// the stream rewritten against the untouched qubits.  Returns the number of
// exchanged qubit pairs.
int prepare_stream(const qsim_state *s, std::vector<Op> &stream)
{
    mark_norms(s, stream);
    std::vector<std::pair<int, int>> pairs;
    choose_remap(s, stream, pairs);
    apply_remap(pairs, stream);
    if (s->lazy)
        lazy_rewrite(s, stream);
    return (int)pairs.size();
}

// Touched qubits and untouched values after a pass has run.
void track_pass(const std::vector<Op> &ops, const PassPlan &p, uint64_t &act, uint64_t &fixed)
{
    for (size_t i = p.first; i < p.first + p.count; ++i) {
        if (ops[i].activates)
            act |= 1ull << ops[i].target;
        if (ops[i].relocate)
            fixed ^= 1ull << ops[i].target;
    }
}

// Write a reset that is still pending (readouts, direct access to the
// memory).  The state's contents are unchanged by it, so const callers may
// settle too.
int settle(const qsim_state *cs)
{
    qsim_state *s = const_cast<qsim_state *>(cs);
    if (!s->init_pending)
        return QSIM_OK;
    HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
    HIP_TRY(s->dtype == QSIM_C64
                ? launch_init_basis<float>((cplx<float> *)s->psi, s->M, s->init_index, s->stream)
                : launch_init_basis<double>((cplx<double> *)s->psi, s->M, s->init_index, s->stream),
            "init launch");
    s->init_pending = false;
    return QSIM_OK;
}

#define SETTLE(st)                       \
    do {                                 \
        const int rc_ = settle(st);      \
        if (rc_ != QSIM_OK)              \
            return rc_;                  \
    } while (0)

template <typename R>
int run_ops(qsim_state *s, std::vector<Op> &stream)
{
    // a reset still pending is written by the first pass when that pass is a
    // fused one over the whole register (it builds its quanta instead of
    // loading them), else by an initialisation pass first
    bool gen_first = s->init_pending;
    s->stats.remaps += (uint64_t)prepare_stream(s, stream);
    // passes are planned one at a time and launched at once, so the host
    // plans the next pass while the device runs the previous ones
    std::vector<uint32_t> order;
    order.reserve(stream.size());
    std::vector<Op> ops;
    ops.reserve(stream.size());
    PassScheduler sched(s, stream);
    PassPlan p;
    cplx<R> *psi = reinterpret_cast<cplx<R> *>(s->psi);
    const double full = 2.0 * (double)(1ull << s->M) * (double)elem_bytes(s->dtype);
    bool scale_pending = false;
    double *norm_sum = s->d_scalars + 4;   // [4] = sum, [5] = 1/sqrt(sum)
    uint64_t act = s->active, fixed = s->fixed;
    while (sched.next(order, p)) {
        for (size_t i = ops.size(); i < order.size(); ++i)
            ops.push_back(stream[order[i]]);
        if (p.fused) {
            TileArgs<R> A;
            int G = 0;
            build_tile_args<R>(s, ops, p, act, fixed, A, G);
            if (A.nsrun > (uint32_t)kMaxRuns || A.ncrun > (uint32_t)kMaxRuns ||
                A.mact < A.k || A.mact > (uint32_t)s->M)
                return fail(QSIM_EDEVICE, "internal: fused pass tables out of range");
            A.gen = 0;
            A.gen_index = 0;
            if (gen_first) {
                if (A.mact == (uint32_t)s->M && A.base_or == 0) {
                    A.gen = 1;
                    A.gen_index = s->init_index;
                } else {
                    HIP_TRY(launch_init_basis<R>(psi, s->M, s->init_index, s->stream), "init launch");
                }
                gen_first = false;
                s->init_pending = false;
            }
            A.psi = psi;
            A.scale_in = scale_pending ? norm_sum + 1 : nullptr;
            A.norm_out = p.norm_after ? s->d_tile_norm : nullptr;
            double flops = 0.0;
            for (size_t i = p.first; i < p.first + p.count; ++i)
                flops += op_flops(ops[i], (int)A.mact);
            const double bytes = 2.0 * std::ldexp((double)elem_bytes(s->dtype), (int)A.mact);
            Timed t(s, 1, bytes, flops);
            HIP_TRY(launch_tile<R>(A, G, s->stream), "fused pass launch");
            t.done();
            scale_pending = false;
            s->stats.fused_passes++;
            if (p.norm_after) {
                Timed t2(s, 2, 0);
                HIP_TRY(launch_finish_norm(s->d_tile_norm, 1ull << (A.mact - A.k), s->d_partial,
                                           norm_sum, s->stream), "norm launch");
                t2.done();
                scale_pending = true;
                s->stats.renorms++;
            }
        } else {
            if (gen_first) {
                HIP_TRY(launch_init_basis<R>(psi, s->M, s->init_index, s->stream), "init launch");
                gen_first = false;
                s->init_pending = false;
            }
            if (scale_pending) {
                Timed t0(s, 2, full);
                HIP_TRY(launch_scale<R>(psi, s->M, norm_sum + 1, s->stream), "scale launch");
                t0.done();
                scale_pending = false;
            }
            const Op &op = ops[p.first];
            Timed t(s, 0, plain_bytes(s, op));
            HIP_TRY(launch_plain<R>(op, psi, s->M, s->stream), "pass launch");
            t.done();
            if (p.norm_after) {
                Timed t2(s, 2, full / 2);
                HIP_TRY(launch_norm<R>(psi, s->M, s->d_partial, s->d_scalars, s->stream), "norm");
                HIP_TRY(launch_finish_norm(s->d_scalars + 2, 1, nullptr, norm_sum, s->stream), "norm");
                t2.done();
                scale_pending = true;
                s->stats.renorms++;
            }
        }
        track_pass(ops, p, act, fixed);
        s->stats.passes++;
    }
    if (gen_first) {  // an empty call
        HIP_TRY(launch_init_basis<R>(psi, s->M, s->init_index, s->stream), "init launch");
        s->init_pending = false;
    }
    if (scale_pending) {
        Timed t0(s, 2, full);
        HIP_TRY(launch_scale<R>(psi, s->M, norm_sum + 1, s->stream), "scale launch");
        t0.done();
    }
    s->active = act;
    s->fixed = fixed & ~act;
    return QSIM_OK;
}

int validate_gates(const qsim_state *s, const qsim_gate *gates, size_t n)
{
    if (n > 0 && gates == nullptr)
        return fail(QSIM_EINVAL, "gates is NULL");
    char why[160];
    for (size_t k = 0; k < n; ++k)
        if (!gate_valid(gates[k], s->M, why, sizeof(why)))
            return fail(QSIM_EINVAL, "gate %zu: %s", k, why);
    return QSIM_OK;
}

int ensure_stage(qsim_state *s, size_t bytes)
{
    if (s->stage_bytes >= bytes)
        return QSIM_OK;
    HIP_TRY(hipStreamSynchronize(s->stream), "stage sync");
    if (s->d_stage)
        (void)hipFree(s->d_stage);
    s->d_stage = nullptr;
    s->stage_bytes = 0;
    HIP_TRY(hipMalloc(&s->d_stage, bytes), "stage alloc");
    s->stage_bytes = bytes;
    return QSIM_OK;
}

// Options -> state fields (no device calls).
int configure(qsim_state *s, int num_qubits, int dtype, const qsim_options &o)
{
    if (num_qubits < 1 || num_qubits > QSIM_MAX_QUBITS)
        return fail(QSIM_EINVAL, "num_qubits %d outside [1, %d]", num_qubits, QSIM_MAX_QUBITS);
    if (dtype != QSIM_C64 && dtype != QSIM_C128)
        return fail(QSIM_EINVAL, "dtype %d is neither QSIM_C64 nor QSIM_C128", dtype);
    if (o.exec_mode < 0 || o.exec_mode > 2)
        return fail(QSIM_EINVAL, "exec_mode %d", o.exec_mode);
    if (o.renorm_period < -1)
        return fail(QSIM_EINVAL, "renorm_period %d", o.renorm_period);
    if (o.lazy_qubits < -1 || o.lazy_qubits > 1)
        return fail(QSIM_EINVAL, "lazy_qubits %d is not -1, 0 or 1", o.lazy_qubits);
    if (o.remap_qubits < -1 || o.remap_qubits > 1)
        return fail(QSIM_EINVAL, "remap_qubits %d is not -1, 0 or 1", o.remap_qubits);
    const size_t eb = elem_bytes(dtype);
    const size_t bytes = ((size_t)1 << num_qubits) * eb;
    if (o.ext_buffer && o.ext_bytes < bytes)
        return fail(QSIM_EINVAL, "ext_bytes %zu < %zu needed", o.ext_bytes, bytes);
    if (o.ext_buffer && (reinterpret_cast<uintptr_t>(o.ext_buffer) % 32) != 0)
        return fail(QSIM_EINVAL, "ext_buffer must be 32-byte aligned");
    const int dflt_k = dtype == QSIM_C64 ? 13 : 12;
    const int dflt_g = 4;
    int k = o.tile_bits > 0 ? o.tile_bits : env_int("QSIM_TILE_BITS", dflt_k);
    int low = o.low_bits > 0 ? o.low_bits : env_int("QSIM_LOW_BITS", 4);
    int G = o.group_bits > 0 ? o.group_bits : env_int("QSIM_GROUP_BITS", dflt_g);
    if (k < 9 || k > kMaxTileBits || low < 1 || low >= k || G < 3 || G > 5 || k - G < 6 ||
        k - G > 9)
        return fail(QSIM_EINVAL,
                    "tile_bits %d / low_bits %d / group bits %d out of range (9 <= tile_bits "
                    "<= %d, 1 <= low_bits < tile_bits, 6 <= tile_bits - group bits <= 9)",
                    k, low, G, kMaxTileBits);
    if (tile_lds_bytes(k, (int)eb) > kMaxLdsBytes)
        return fail(QSIM_EINVAL, "a %d-qubit tile of this dtype does not fit the 160 KiB LDS", k);
    s->M = num_qubits;
    s->dtype = dtype;
    s->device = o.device;
    s->exec_mode = o.exec_mode;
    s->tile_bits = k;
    s->low_bits = low;
    s->group_bits = G;
    s->renorm_period = o.renorm_period == 0 ? (dtype == QSIM_C64 ? 64 : 0)
                       : (o.renorm_period < 0 ? 0 : o.renorm_period);
    s->bytes = bytes;
    // the per-operation path always streams the whole register
    s->lazy = o.lazy_qubits >= 0 && o.exec_mode != 1;
    s->remap = o.remap_qubits;
    s->active = s->lazy ? 0 : full_mask(num_qubits);
    s->fixed = 0;  // the register starts (or is rebound) at |0...0>
    return QSIM_OK;
}

void release(qsim_state *s)
{
    if (s == nullptr)
        return;
    (void)hipSetDevice(s->device);
    if (s->stream)
        (void)hipStreamSynchronize(s->stream);
    for (PendingTiming &p : s->pending) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    for (hipEvent_t e : s->free_events)
        (void)hipEventDestroy(e);
    if (s->own_mem && s->psi)
        (void)hipFree(s->psi);
    if (s->d_partial)
        (void)hipFree(s->d_partial);
    if (s->d_tile_norm)
        (void)hipFree(s->d_tile_norm);
    if (s->d_scalars)
        (void)hipFree(s->d_scalars);
    if (s->d_stage)
        (void)hipFree(s->d_stage);
    if (s->h_pinned)
        (void)hipHostFree(s->h_pinned);
    if (s->own_stream && s->stream)
        (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // namespace

// ============================================================ serving slots

namespace qsim {

int slot_state_create(int device, hipStream_t st, int max_qubits, qsim_state **out)
{
    *out = nullptr;
    qsim_state *s = new (std::nothrow) qsim_state();
    if (s == nullptr)
        return fail(QSIM_ENOMEM, "slot state: host memory exhausted");
    s->device = device;
    s->stream = st;
    s->own_stream = false;
    s->own_mem = false;
    const uint64_t tiles = 1ull << std::max(0, max_qubits - 9);  // smallest tile: 9 qubits
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess)
        e = hipMalloc((void **)&s->d_partial, 4 * kReduceBlocks * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&s->d_tile_norm, tiles * sizeof(double));
    if (e == hipSuccess)
        e = hipMalloc((void **)&s->d_scalars, 16 * sizeof(double));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&s->h_pinned, 16 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "slot state");
        release(s);
        return rc;
    }
    *out = s;
    return QSIM_OK;
}

int slot_state_bind(qsim_state *s, int num_qubits, int dtype, void *psi)
{
    qsim_options o{};
    o.device = s->device;
    int rc = configure(s, num_qubits, dtype, o);
    if (rc != QSIM_OK)
        return rc;
    s->psi = psi;
    s->step = 0;
    s->armed = false;
    HIP_TRY(dtype == QSIM_C64
                ? launch_init_basis<float>((cplx<float> *)psi, num_qubits, 0, s->stream)
                : launch_init_basis<double>((cplx<double> *)psi, num_qubits, 0, s->stream),
            "init launch");
    return QSIM_OK;
}

int overlap_enqueue(const qsim_state *a, const qsim_state *b, double *host_out4)
{
    SETTLE(a);
    SETTLE(b);
    hipError_t e;
    if (a->dtype == QSIM_C64 && b->dtype == QSIM_C64)
        e = launch_overlap<float, float>((const cplx<float> *)a->psi, (const cplx<float> *)b->psi,
                                         a->M, a->d_partial, a->d_scalars, a->stream);
    else if (a->dtype == QSIM_C64)
        e = launch_overlap<float, double>((const cplx<float> *)a->psi,
                                          (const cplx<double> *)b->psi, a->M, a->d_partial,
                                          a->d_scalars, a->stream);
    else if (b->dtype == QSIM_C64)
        e = launch_overlap<double, float>((const cplx<double> *)a->psi,
                                          (const cplx<float> *)b->psi, a->M, a->d_partial,
                                          a->d_scalars, a->stream);
    else
        e = launch_overlap<double, double>((const cplx<double> *)a->psi,
                                           (const cplx<double> *)b->psi, a->M, a->d_partial,
                                           a->d_scalars, a->stream);
    HIP_TRY(e, "overlap launch");
    HIP_TRY(hipMemcpyAsync(host_out4, a->d_scalars, 4 * sizeof(double), hipMemcpyDeviceToHost,
                           a->stream), "overlap copy");
    return QSIM_OK;
}

void slot_state_destroy(qsim_state *s) { release(s); }

}  // namespace qsim

// ===================================================================== C ABI

extern "C" {

const char *qsim_last_error(void) { return g_err; }

int qsim_create(int num_qubits, int dtype, const qsim_options *opt, qsim_state **out)
{
    return guarded(__func__, [&]() -> int {
        if (out == nullptr)
            return fail(QSIM_EINVAL, "out is NULL");
        *out = nullptr;
        qsim_options o{};
        if (opt)
            o = *opt;
        qsim_state *s = new (std::nothrow) qsim_state();
        if (s == nullptr)
            return fail(QSIM_ENOMEM, "qsim_create: host memory exhausted");
        int rc = configure(s, num_qubits, dtype, o);
        if (rc != QSIM_OK) {
            delete s;
            return rc;
        }
        const size_t bytes = s->bytes;
        const int k = s->tile_bits;
        int ndev = 0;
        hipError_t e0 = hipGetDeviceCount(&ndev);
        if (e0 != hipSuccess) {
            delete s;
            return hip_fail(e0, "hipGetDeviceCount");
        }
        if (o.device < 0 || o.device >= ndev) {
            delete s;
            return fail(QSIM_EINVAL, "device %d outside [0, %d)", o.device, ndev);
        }
        hipError_t e = hipSetDevice(o.device);
        if (e == hipSuccess) {
            if (o.hip_stream) {
                s->stream = reinterpret_cast<hipStream_t>(o.hip_stream);
            } else {
                e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
                s->own_stream = e == hipSuccess;
            }
        }
        if (e == hipSuccess) {
            if (o.ext_buffer) {
                s->psi = o.ext_buffer;
            } else {
                e = hipMalloc(&s->psi, bytes);
                s->own_mem = e == hipSuccess;
            }
        }
        const int kk = std::min(k, num_qubits);
        const uint64_t tiles = 1ull << (num_qubits - kk);
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->d_partial, 4 * kReduceBlocks * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->d_tile_norm, tiles * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc((void **)&s->d_scalars, 16 * sizeof(double));
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&s->h_pinned, 16 * sizeof(double), hipHostMallocDefault);
        if (e == hipSuccess)
            e = (dtype == QSIM_C64)
                    ? launch_init_basis<float>((cplx<float> *)s->psi, num_qubits, 0, s->stream)
                    : launch_init_basis<double>((cplx<double> *)s->psi, num_qubits, 0, s->stream);
        if (e != hipSuccess) {
            rc = hip_fail(e, "qsim_create");
            release(s);
            return rc;
        }
        *out = s;
        return QSIM_OK;
    });
}

int qsim_destroy(qsim_state *s)
{
    return guarded(__func__, [&]() -> int {
        release(s);
        return QSIM_OK;
    });
}

int qsim_reset(qsim_state *s, uint64_t basis_index)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        if (basis_index >= (1ull << s->M))
            return fail(QSIM_ERANGE, "basis index %llu >= 2^%d", (unsigned long long)basis_index, s->M);
        // written by the first pass of the next call that applies gates (or
        // before anything reads the register), not by a pass of its own
        s->init_pending = true;
        s->init_index = basis_index;
        s->step = 0;
        s->active = s->lazy ? 0 : full_mask(s->M);
        s->fixed = basis_index & ~s->active;
        return QSIM_OK;
    });
}

int qsim_inject_errors(qsim_state *s, const qsim_error_model *em)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        if (em == nullptr) {
            s->armed = false;
            return QSIM_OK;
        }
        if (!error_model_valid(*em))
            return fail(QSIM_EINVAL, "sigma must be finite and >= 0, flip probabilities in [0, 1]");
        s->em = *em;
        s->armed = true;
        return QSIM_OK;
    });
}

int qsim_apply_circuit(qsim_state *s, const qsim_gate *gates, size_t n_gates)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        int rc = validate_gates(s, gates, n_gates);
        if (rc != QSIM_OK)
            return rc;
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        std::vector<Op> ops;
        lower_circuit(s, gates, n_gates, ops);
        const size_t flips = ops.size() - n_gates;
        rc = s->dtype == QSIM_C64 ? run_ops<float>(s, ops) : run_ops<double>(s, ops);
        if (rc != QSIM_OK)
            return rc;
        s->step += n_gates;
        s->stats.gates += n_gates;
        s->stats.flips += flips;
        return QSIM_OK;
    });
}

int qsim_apply_inverse(qsim_state *s, const qsim_gate *gates, size_t n_gates)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        int rc = validate_gates(s, gates, n_gates);
        if (rc != QSIM_OK)
            return rc;
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        std::vector<Op> ops;
        ops.reserve(n_gates);
        for (size_t k = 0; k < n_gates; ++k) {
            Op op = lower_gate(gates[n_gates - 1 - k], 0.0, true);
            op.step = k;
            op.is_flip = false;
            op.step_end = true;
            ops.push_back(op);
        }
        const int saved = s->renorm_period;
        s->renorm_period = 0;
        rc = s->dtype == QSIM_C64 ? run_ops<float>(s, ops) : run_ops<double>(s, ops);
        s->renorm_period = saved;
        return rc;
    });
}

int qsim_synchronize(qsim_state *s)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        SETTLE(s);
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        HIP_TRY(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
        return QSIM_OK;
    });
}

int qsim_overlap(const qsim_state *a, const qsim_state *b, double out[4])
{
    return guarded(__func__, [&]() -> int {
        if (a == nullptr || b == nullptr || out == nullptr)
            return fail(QSIM_EINVAL, "NULL argument");
        if (a->M != b->M)
            return fail(QSIM_EINVAL, "register sizes differ (%d vs %d)", a->M, b->M);
        if (a->device != b->device)
            return fail(QSIM_EINVAL, "states live on different devices");
        qsim_state *sa = const_cast<qsim_state *>(a);
        SETTLE(a);
        SETTLE(b);
        HIP_TRY(hipSetDevice(a->device), "hipSetDevice");
        if (a->stream != b->stream) {
            hipEvent_t ev;
            HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
            HIP_TRY(hipEventRecord(ev, b->stream), "event record");
            HIP_TRY(hipStreamWaitEvent(a->stream, ev, 0), "stream wait");
            (void)hipEventDestroy(ev);
        }
        Timed t(sa, 2, 0);
        hipError_t e;
        if (a->dtype == QSIM_C64 && b->dtype == QSIM_C64)
            e = launch_overlap<float, float>((const cplx<float> *)a->psi, (const cplx<float> *)b->psi,
                                             a->M, a->d_partial, a->d_scalars, a->stream);
        else if (a->dtype == QSIM_C64)
            e = launch_overlap<float, double>((const cplx<float> *)a->psi,
                                              (const cplx<double> *)b->psi, a->M, a->d_partial,
                                              a->d_scalars, a->stream);
        else if (b->dtype == QSIM_C64)
            e = launch_overlap<double, float>((const cplx<double> *)a->psi,
                                              (const cplx<float> *)b->psi, a->M, a->d_partial,
                                              a->d_scalars, a->stream);
        else
            e = launch_overlap<double, double>((const cplx<double> *)a->psi,
                                               (const cplx<double> *)b->psi, a->M, a->d_partial,
                                               a->d_scalars, a->stream);
        HIP_TRY(e, "overlap launch");
        t.done();
        HIP_TRY(hipMemcpyAsync(a->h_pinned, a->d_scalars, 4 * sizeof(double), hipMemcpyDeviceToHost,
                               a->stream), "overlap copy");
        HIP_TRY(hipStreamSynchronize(a->stream), "overlap sync");
        if (a->stream != b->stream)
            HIP_TRY(hipStreamSynchronize(b->stream), "overlap sync");
        std::memcpy(out, a->h_pinned, 4 * sizeof(double));
        return QSIM_OK;
    });
}

int qsim_fidelity(const qsim_state *a, const qsim_state *b, double *out_F)
{
    return guarded(__func__, [&]() -> int {
        if (out_F == nullptr)
            return fail(QSIM_EINVAL, "out_F is NULL");
        double o[4];
        int rc = qsim_overlap(a, b, o);
        if (rc != QSIM_OK)
            return rc;
        *out_F = (o[0] * o[0] + o[1] * o[1]) / (o[2] * o[3]);
        return QSIM_OK;
    });
}

int qsim_norm(const qsim_state *s, double *out)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr || out == nullptr)
            return fail(QSIM_EINVAL, "NULL argument");
        qsim_state *m = const_cast<qsim_state *>(s);
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        SETTLE(s);
        Timed t(m, 2, 0);
        HIP_TRY(s->dtype == QSIM_C64
                    ? launch_norm<float>((const cplx<float> *)s->psi, s->M, s->d_partial,
                                         s->d_scalars, s->stream)
                    : launch_norm<double>((const cplx<double> *)s->psi, s->M, s->d_partial,
                                          s->d_scalars, s->stream),
                "norm launch");
        t.done();
        HIP_TRY(hipMemcpyAsync(s->h_pinned, s->d_scalars, 4 * sizeof(double), hipMemcpyDeviceToHost,
                               s->stream), "norm copy");
        HIP_TRY(hipStreamSynchronize(s->stream), "norm sync");
        *out = s->h_pinned[2];
        return QSIM_OK;
    });
}

int qsim_probs(const qsim_state *s, uint64_t qubit_mask, double *out, size_t out_len)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr || out == nullptr)
            return fail(QSIM_EINVAL, "NULL argument");
        const uint64_t full = (1ull << s->M) - 1;
        if (qubit_mask & ~full)
            return fail(QSIM_EINVAL, "mask has bits at or above qubit %d", s->M);
        const int m = __builtin_popcountll(qubit_mask);
        if (out_len != (1ull << m))
            return fail(QSIM_EINVAL, "out_len %zu != 2^%d", out_len, m);
        qsim_state *ms = const_cast<qsim_state *>(s);
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        SETTLE(s);
        const size_t out_bytes = out_len * sizeof(double);
        if (qubit_mask == full) {
            int rc = ensure_stage(ms, out_bytes);
            if (rc != QSIM_OK)
                return rc;
            Timed t(ms, 2, 0);
            HIP_TRY(s->dtype == QSIM_C64
                        ? launch_probs_full<float>((const cplx<float> *)s->psi, s->M,
                                                   (double *)s->d_stage, s->stream)
                        : launch_probs_full<double>((const cplx<double> *)s->psi, s->M,
                                                    (double *)s->d_stage, s->stream),
                    "probs launch");
            t.done();
        } else {
            const uint64_t plen = probs_marginal_partial_len(s->M, qubit_mask);
            const size_t out_off = (plen * sizeof(double) + 255) & ~(size_t)255;
            int rc = ensure_stage(ms, out_off + out_bytes);
            if (rc != QSIM_OK)
                return rc;
            double *partial = (double *)s->d_stage;
            double *dout = (double *)((char *)s->d_stage + out_off);
            Timed t(ms, 2, 0);
            HIP_TRY(s->dtype == QSIM_C64
                        ? launch_probs_marginal<float>((const cplx<float> *)s->psi, s->M, qubit_mask,
                                                       partial, plen, dout, s->stream)
                        : launch_probs_marginal<double>((const cplx<double> *)s->psi, s->M,
                                                        qubit_mask, partial, plen, dout, s->stream),
                    "marginal launch");
            t.done();
            HIP_TRY(hipMemcpyAsync(out, dout, out_bytes, hipMemcpyDeviceToHost, s->stream),
                    "probs copy");
            HIP_TRY(hipStreamSynchronize(s->stream), "probs sync");
            return QSIM_OK;
        }
        HIP_TRY(hipMemcpyAsync(out, s->d_stage, out_bytes, hipMemcpyDeviceToHost, s->stream),
                "probs copy");
        HIP_TRY(hipStreamSynchronize(s->stream), "probs sync");
        return QSIM_OK;
    });
}

int qsim_get_amplitudes(const qsim_state *s, uint64_t offset, uint64_t count, double *out)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr || (out == nullptr && count > 0))
            return fail(QSIM_EINVAL, "NULL argument");
        const uint64_t n = 1ull << s->M;
        if (offset > n || count > n - offset)
            return fail(QSIM_ERANGE, "range [%llu, +%llu) outside 2^%d amplitudes",
                        (unsigned long long)offset, (unsigned long long)count, s->M);
        qsim_state *ms = const_cast<qsim_state *>(s);
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        SETTLE(s);
        const uint64_t chunk = std::min<uint64_t>(count, 1ull << 22);
        if (count == 0)
            return QSIM_OK;
        int rc = ensure_stage(ms, chunk * 16);
        if (rc != QSIM_OK)
            return rc;
        for (uint64_t done = 0; done < count; done += chunk) {
            const uint64_t c = std::min(chunk, count - done);
            HIP_TRY(s->dtype == QSIM_C64
                        ? launch_to_f64<float>((const cplx<float> *)s->psi + offset + done, c,
                                               (double *)s->d_stage, s->stream)
                        : launch_to_f64<double>((const cplx<double> *)s->psi + offset + done, c,
                                                (double *)s->d_stage, s->stream),
                    "convert launch");
            HIP_TRY(hipMemcpyAsync(out + 2 * done, s->d_stage, c * 16, hipMemcpyDeviceToHost,
                                   s->stream), "amplitude copy");
            HIP_TRY(hipStreamSynchronize(s->stream), "amplitude sync");
        }
        return QSIM_OK;
    });
}

int qsim_set_amplitudes(qsim_state *s, uint64_t offset, uint64_t count, const double *in)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr || (in == nullptr && count > 0))
            return fail(QSIM_EINVAL, "NULL argument");
        const uint64_t n = 1ull << s->M;
        if (offset > n || count > n - offset)
            return fail(QSIM_ERANGE, "range outside the register");
        for (uint64_t i = 0; i < 2 * count; ++i)
            if (!std::isfinite(in[i]))
                return fail(QSIM_EINVAL, "non-finite input at %llu", (unsigned long long)i);
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        SETTLE(s);
        if (count == 0)
            return QSIM_OK;
        const uint64_t chunk = std::min<uint64_t>(count, 1ull << 22);
        int rc = ensure_stage(s, chunk * 16);
        if (rc != QSIM_OK)
            return rc;
        // arbitrary amplitudes: no qubit is known to hold one value any more
        s->active = full_mask(s->M);
        for (uint64_t done = 0; done < count; done += chunk) {
            const uint64_t c = std::min(chunk, count - done);
            HIP_TRY(hipMemcpyAsync(s->d_stage, in + 2 * done, c * 16, hipMemcpyHostToDevice,
                                   s->stream), "amplitude copy");
            HIP_TRY(s->dtype == QSIM_C64
                        ? launch_from_f64<float>((const double *)s->d_stage, c,
                                                 (cplx<float> *)s->psi + offset + done, s->stream)
                        : launch_from_f64<double>((const double *)s->d_stage, c,
                                                  (cplx<double> *)s->psi + offset + done, s->stream),
                    "convert launch");
            HIP_TRY(hipStreamSynchronize(s->stream), "amplitude sync");
        }
        return QSIM_OK;
    });
}

int qsim_plan(int num_qubits, int dtype, const qsim_options *opt, const qsim_gate *gates,
              size_t n_gates, const qsim_error_model *em, uint64_t step0, qsim_pass_info *out,
              size_t out_cap, size_t *n_passes, size_t *n_ops, uint32_t *op_order,
              size_t order_cap)
{
    return guarded(__func__, [&]() -> int {
        qsim_options o{};
        if (opt)
            o = *opt;
        qsim_state st;
        int rc = configure(&st, num_qubits, dtype, o);
        if (rc != QSIM_OK)
            return rc;
        rc = validate_gates(&st, gates, n_gates);
        if (rc != QSIM_OK)
            return rc;
        if (em) {
            if (!error_model_valid(*em))
                return fail(QSIM_EINVAL, "bad error model");
            st.em = *em;
            st.armed = true;
        }
        st.step = step0;
        std::vector<Op> stream;
        lower_circuit(&st, gates, n_gates, stream);
        prepare_stream(&st, stream);
        std::vector<PassPlan> plan;
        std::vector<uint32_t> order;
        schedule(&st, stream, order, plan);
        uint64_t act = st.active, fixed = st.fixed;
        std::vector<Op> ops(order.size());
        for (size_t i = 0; i < order.size(); ++i)
            ops[i] = stream[order[i]];
        if (n_passes)
            *n_passes = plan.size();
        if (n_ops)
            *n_ops = ops.size();
        if (op_order)
            for (size_t i = 0; i < order.size() && i < order_cap; ++i)
                op_order[i] = order[i];
        for (size_t i = 0; i < plan.size(); ++i) {
            qsim_pass_info info{};
            info.fused = plan[i].fused ? 1u : 0u;
            info.first_op = (uint32_t)plan[i].first;
            info.n_ops = (uint32_t)plan[i].count;
            info.norm_after = plan[i].norm_after ? 1u : 0u;
            int span = num_qubits;  // qubits the pass's launch spans
            if (plan[i].fused) {
                char why[160];
                int G = 0;
                bool ok;
                if (dtype == QSIM_C64) {
                    TileArgs<float> A;
                    build_tile_args<float>(&st, ops, plan[i], act, fixed, A, G);
                    ok = tile_args_consistent<float>(A, G, ops, plan[i], why, sizeof(why));
                    info.n_groups = A.ngroups;
                    info.tile_mask = A.smask;
                    span = (int)A.mact;
                    info.tiles = 1ull << (A.mact - A.k);
                } else {
                    TileArgs<double> A;
                    build_tile_args<double>(&st, ops, plan[i], act, fixed, A, G);
                    ok = tile_args_consistent<double>(A, G, ops, plan[i], why, sizeof(why));
                    info.n_groups = A.ngroups;
                    info.tile_mask = A.smask;
                    span = (int)A.mact;
                    info.tiles = 1ull << (A.mact - A.k);
                }
                if (!ok)
                    return fail(QSIM_EDEVICE, "internal: pass %zu inconsistent: %s", i, why);
            }
            for (size_t j = plan[i].first; j < plan[i].first + plan[i].count; ++j)
                info.flops += op_flops(ops[j], span);
            info.span_qubits = (uint32_t)span;
            track_pass(ops, plan[i], act, fixed);
            if (out && i < out_cap)
                out[i] = info;
        }
        return QSIM_OK;
    });
}

int qsim_touched_qubits(const qsim_state *s, uint64_t *mask)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr || mask == nullptr)
            return fail(QSIM_EINVAL, "NULL argument");
        *mask = s->active;
        return QSIM_OK;
    });
}

int qsim_info(const qsim_state *s, int *num_qubits, int *dtype, uint64_t *step, void **device_ptr,
              size_t *bytes)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        if (num_qubits) *num_qubits = s->M;
        if (dtype) *dtype = s->dtype;
        if (step) *step = s->step;
        if (device_ptr) {
            SETTLE(s);  // whoever reads the memory sees the state
            *device_ptr = s->psi;
        }
        if (bytes) *bytes = s->bytes;
        return QSIM_OK;
    });
}

int qsim_profile(qsim_state *s, int enable)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr)
            return fail(QSIM_EINVAL, "state is NULL");
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        int rc = flush_timings(s);
        if (rc != QSIM_OK)
            return rc;
        s->stats = qsim_stats{};
        s->profiling = enable != 0;
        return QSIM_OK;
    });
}

int qsim_get_stats(qsim_state *s, qsim_stats *out)
{
    return guarded(__func__, [&]() -> int {
        if (s == nullptr || out == nullptr)
            return fail(QSIM_EINVAL, "NULL argument");
        HIP_TRY(hipSetDevice(s->device), "hipSetDevice");
        int rc = flush_timings(s);
        if (rc != QSIM_OK)
            return rc;
        *out = s->stats;
        return QSIM_OK;
    });
}

}  // extern "C"
