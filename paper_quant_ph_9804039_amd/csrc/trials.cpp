// qsim_run_trials: batched Monte Carlo error trials in one persistent launch,
// with a small autotuner that picks the kernel variant per problem shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"
#include "internal.h"
#include "launch.h"
#include "qsim.h"

using namespace qsim;

namespace {

int hip_err(hipError_t e, const char *what)
{
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? QSIM_ENOMEM : QSIM_EDEVICE, "%s: %s", what,
                     hipGetErrorString(e));
}

// ------------------------------------------------------------------ autotuner
//
// Key: register size, dtype, gate count and whether angle errors and flips
// are drawn.  The choice is kept for the process, and in the file named by
// QSIM_TUNE_CACHE (one "M dtype gates angle flips variant" line per key) if
// that is set.

using TuneKey = std::tuple<int, int, uint32_t, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
bool g_tune_loaded = false;

void tune_load()
{
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    const char *path = getenv("QSIM_TUNE_CACHE");
    if (path == nullptr || *path == 0)
        return;
    FILE *f = fopen(path, "r");
    if (f == nullptr)
        return;
    int M, dt, a, fl, v;
    unsigned n;
    while (fscanf(f, "%d %d %u %d %d %d", &M, &dt, &n, &a, &fl, &v) == 6)
        if (v >= 0 && v < trial_variants())
            g_tune[TuneKey(M, dt, n, a, fl)] = v;
    fclose(f);
}

void tune_store(const TuneKey &k, int v)
{
    g_tune[k] = v;
    const char *path = getenv("QSIM_TUNE_CACHE");
    if (path == nullptr || *path == 0)
        return;
    FILE *f = fopen(path, "a");
    if (f == nullptr)
        return;
    fprintf(f, "%d %d %u %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
            std::get<3>(k), std::get<4>(k), v);
    fclose(f);
}

// Gates the preparation kernel may turn into a butterfly: the uncontrolled
// Hadamards.
bool trial_butterfly_candidate(const qsim_gate &g)
{
    return g.kind == QSIM_H && g.ctrl0 < 0 && g.ctrl1 < 0;
}

// Register-group schedule of a circuit (variants with G group qubits):
// groups of consecutive gates whose non-diagonal targets (every kind but Rz
// and Z) span at most G qubits and that hold at most kMaxGroupButterflies
// uncontrolled Hadamards (the kernel applies their scales at the group's
// end), each padded to G qubits with the qubits its diagonal gates act on
// (most used first; on a group qubit a diagonal is a per-register factor)
// and then the highest free qubits.  out = the group records (see
// TrialLaunch; no chunk records), then each gate's group word.
void group_schedule(const qsim_gate *gates, size_t n, int M, int G, std::vector<uint32_t> &out,
                    uint32_t &nchunks, uint32_t &ngroups)
{
    auto diagonal = [](const qsim_gate &g) { return g.kind == QSIM_RZ || g.kind == QSIM_Z; };
    out.clear();
    ngroups = 0;
    size_t i = 0;
    while (i < n) {
        uint32_t cur = 0;  // qubit mask of the group's non-diagonal targets
        uint32_t nbf = 0;  // uncontrolled Hadamards in the group
        size_t j = i;
        while (j < n) {
            if (trial_butterfly_candidate(gates[j]) && nbf == kMaxGroupButterflies)
                break;
            if (!diagonal(gates[j])) {
                const uint32_t tb = 1u << gates[j].target;
                if (!(cur & tb)) {
                    if (__builtin_popcount(cur) == G)
                        break;
                    cur |= tb;
                }
            }
            if (trial_butterfly_candidate(gates[j]))
                ++nbf;
            ++j;
        }
        int uses[32] = {0};
        for (size_t k = i; k < j; ++k)
            if (diagonal(gates[k]))
                ++uses[gates[k].target];
        while (__builtin_popcount(cur) < G) {
            int best = -1;
            for (int q = 0; q < M; ++q)
                if (uses[q] > 0 && !((cur >> q) & 1u) && (best < 0 || uses[q] > uses[best]))
                    best = q;
            if (best < 0)
                break;
            cur |= 1u << best;
        }
        for (int q = M - 1; q >= 0 && __builtin_popcount(cur) < G; --q)
            cur |= 1u << q;
        uint32_t word = 0;
        int slot = 0;
        for (int q = 0; q < M; ++q)
            if ((cur >> q) & 1u)
                word |= (uint32_t)q << (4 * slot++);
        out.insert(out.end(), {(uint32_t)i, (uint32_t)(j - i), word, nbf});
        ++ngroups;
        i = j;
    }
    for (uint32_t gi = 0; gi < ngroups; ++gi)
        for (uint32_t k = 0; k < out[4 * gi + 1]; ++k)
            out.push_back(out[4 * gi + 2]);
    nchunks = 0;
}

// The register-group schedules on the device, one per group size.
struct GroupSched {
    void *buf[2] = {nullptr, nullptr};  // G = 4, 5 (device, not owned)
    uint32_t nchunks[2] = {0, 0}, ngroups[2] = {0, 0};
    void apply(TrialLaunch &L, int variant) const
    {
        const int G = trial_group_bits(variant);
        if (G < 4 || G > 5 || buf[G - 4] == nullptr) {
            L.sched = nullptr;
            L.nchunks = L.ngroups = 0;
            return;
        }
        L.sched = reinterpret_cast<const uint32_t *>(buf[G - 4]);
        L.nchunks = nchunks[G - 4];
        L.ngroups = ngroups[G - 4];
    }
};

hipError_t launch(int dtype, const TrialLaunch &L, hipStream_t st)
{
    return dtype == QSIM_C64 ? launch_trials<float>(L, st) : launch_trials<double>(L, st);
}

// Time every variant on one round of trials (one trial per workgroup) and
// keep the fastest.  The timing runs write to a scratch output of
// kTuneTrials doubles.
constexpr int kTuneTrials = 4096;

int autotune(int dtype, TrialLaunch L, const GroupSched &gs, hipStream_t st, double *scratch,
             int &best)
{
    best = -1;
    float best_ms = 0.f;
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess)
        return hip_err(e, "tune event");
    e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_err(e, "tune event");
    }
    const int elem = dtype == QSIM_C64 ? 8 : 16;
    for (int v = 0; v < trial_variants(); ++v) {
        const int grid = trial_grid(v, (int)L.M, elem);
        if (grid <= 0)
            continue;
        L.variant = v;
        L.grid = grid;
        L.n_trials = (uint64_t)std::min(grid, kTuneTrials);
        gs.apply(L, v);
        if (trial_group_bits(v) > 0 && L.sched == nullptr)
            continue;
        L.out_F = scratch;
        // once to warm up, once timed
        e = launch(dtype, L, st);
        if (e == hipSuccess)
            e = hipEventRecord(a, st);
        if (e == hipSuccess)
            e = launch(dtype, L, st);
        if (e == hipSuccess)
            e = hipEventRecord(b, st);
        if (e == hipSuccess)
            e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            continue;
        }
        if (best < 0 || ms < best_ms) {
            best = v;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (best < 0)
        return set_error(QSIM_EDEVICE, "no trial kernel variant could run this register");
    return QSIM_OK;
}

// Device resources that qsim_run_trials keeps between calls, per device:
// a stream, the error-free register's state, and buffers that grow to the
// largest call seen.  They are held until the process ends (never freed at
// exit, when the runtime may already be gone); calls on one device are
// serialised by the workspace's mutex.
struct Workspace {
    std::mutex mu;
    hipStream_t st = nullptr;
    struct Buf {
        void *p = nullptr;
        size_t cap = 0;
    };
    Buf gates, out, sched[2], prep, prepx, tune;
    qsim_state *ideal = nullptr;
    int ideal_m = 0, ideal_dtype = -1;
};

hipError_t grow(Workspace::Buf &b, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 1);
    if (b.cap >= bytes)
        return hipSuccess;
    if (b.p != nullptr) {
        // the previous call on this workspace ended with a stream sync
        const hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess)
            return e;
    }
    const hipError_t e = hipMalloc(&b.p, bytes);
    if (e == hipSuccess)
        b.cap = bytes;
    else
        b.p = nullptr;
    return e;
}

Workspace &workspace(int device)
{
    static std::mutex mu;
    static auto *all = new std::map<int, Workspace *>();  // never destroyed
    std::lock_guard<std::mutex> lk(mu);
    Workspace *&w = (*all)[device];
    if (w == nullptr)
        w = new Workspace();
    return *w;
}

}  // namespace

extern "C" int qsim_run_trials(const qsim_gate *gates, size_t n, int num_qubits, int dtype,
                               const qsim_error_model *base, uint64_t n_trials, double *out_F)
{
    return guarded(__func__, [&]() -> int {
        if (dtype != QSIM_C64 && dtype != QSIM_C128)
            return set_error(QSIM_EINVAL, "dtype %d is neither QSIM_C64 nor QSIM_C128", dtype);
        const int max_m = dtype == QSIM_C64 ? 14 : 13;
        if (num_qubits < 1 || num_qubits > max_m)
            return set_error(QSIM_EINVAL,
                             "num_qubits %d outside [1, %d]: a trial's register must fit the "
                             "workgroup's LDS", num_qubits, max_m);
        if (base == nullptr || !error_model_valid(*base))
            return set_error(QSIM_EINVAL, "error model missing or invalid");
        if (n_trials > 0 && out_F == nullptr)
            return set_error(QSIM_EINVAL, "out_F is NULL");
        if (n > 0 && gates == nullptr)
            return set_error(QSIM_EINVAL, "gates is NULL");
        if (n > (size_t)UINT32_MAX)
            return set_error(QSIM_EINVAL, "too many gates");
        char why[160];
        for (size_t k = 0; k < n; ++k) {
            if (!gate_valid(gates[k], num_qubits, why, sizeof(why)))
                return set_error(QSIM_EINVAL, "gate %zu: %s", k, why);
            if (gates[k].kind == QSIM_CPHASE)
                return set_error(QSIM_EINVAL, "gate %zu: the trial kernels do not take "
                                 "controlled phases", k);
        }
        if (n_trials == 0)
            return QSIM_OK;

        int device = 0;
        if (const char *d = getenv("QSIM_DEVICE"))
            device = atoi(d);
        Workspace &ws = workspace(device);
        std::lock_guard<std::mutex> ws_lock(ws.mu);
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess)
            return hip_err(e, "hipSetDevice");
        if (ws.st == nullptr && (e = hipStreamCreateWithFlags(&ws.st, hipStreamNonBlocking)) != hipSuccess) {
            ws.st = nullptr;
            return hip_err(e, "stream");
        }
        hipStream_t st = ws.st;

        // the error-free register, kept between calls of the same shape
        int rc = QSIM_OK;
        if (ws.ideal != nullptr && (ws.ideal_m != num_qubits || ws.ideal_dtype != dtype)) {
            qsim_destroy(ws.ideal);
            ws.ideal = nullptr;
        }
        if (ws.ideal == nullptr) {
            qsim_options o{};
            o.device = device;
            o.renorm_period = -1;
            rc = qsim_create(num_qubits, dtype, &o, &ws.ideal);
            if (rc != QSIM_OK) {
                ws.ideal = nullptr;
                return rc;
            }
            ws.ideal_m = num_qubits;
            ws.ideal_dtype = dtype;
        } else if ((rc = qsim_reset(ws.ideal, 0)) != QSIM_OK) {
            return rc;
        }
        rc = qsim_apply_circuit(ws.ideal, gates, n);
        if (rc != QSIM_OK)
            return rc;
        rc = qsim_synchronize(ws.ideal);
        if (rc != QSIM_OK)
            return rc;
        void *ideal_ptr = nullptr;
        rc = qsim_info(ws.ideal, nullptr, nullptr, nullptr, &ideal_ptr, nullptr);
        if (rc != QSIM_OK)
            return rc;

        std::vector<TrialGate> hg(n);
        for (size_t k = 0; k < n; ++k) {
            TrialGate t{};
            t.kind = gates[k].kind;
            t.target = (uint32_t)gates[k].target;
            t.cmask = 0;
            if (gates[k].ctrl0 >= 0)
                t.cmask |= 1u << gates[k].ctrl0;
            if (gates[k].ctrl1 >= 0)
                t.cmask |= 1u << gates[k].ctrl1;
            t.theta = gates[k].theta;
            hg[k] = t;
        }
        if ((e = grow(ws.gates, n * sizeof(TrialGate))) != hipSuccess)
            return hip_err(e, "gate buffer");
        if ((e = grow(ws.out, n_trials * sizeof(double))) != hipSuccess)
            return hip_err(e, "output buffer");
        if (n > 0 && (e = hipMemcpyAsync(ws.gates.p, hg.data(), n * sizeof(TrialGate),
                                         hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_err(e, "gate upload");
        // register-group schedules (variants 2 and 3), where the register fits
        GroupSched gs;
        std::vector<uint32_t> sched[2];
        for (int G = 4; G <= 5; ++G) {
            if (n == 0 || num_qubits - G < 6 || num_qubits - G > 10)
                continue;
            group_schedule(gates, n, num_qubits, G, sched[G - 4], gs.nchunks[G - 4],
                           gs.ngroups[G - 4]);
            const size_t bytes = sched[G - 4].size() * sizeof(uint32_t);
            if ((e = grow(ws.sched[G - 4], bytes)) != hipSuccess)
                return hip_err(e, "schedule buffer");
            gs.buf[G - 4] = ws.sched[G - 4].p;
            if ((e = hipMemcpyAsync(gs.buf[G - 4], sched[G - 4].data(), bytes,
                                    hipMemcpyHostToDevice, st)) != hipSuccess)
                return hip_err(e, "schedule upload");
        }

        // per-trial gate records of the register-group variants, a batch of
        // trials at a time (at most ~256 MiB)
        uint64_t batch = 0;
        void *prep = nullptr, *prepx = nullptr;
        if (gs.buf[0] != nullptr || gs.buf[1] != nullptr) {
            const size_t per_trial = n * trial_gate_op_bytes(dtype == QSIM_C64 ? 8 : 16);
            const uint64_t cap = std::max<uint64_t>(1, ((size_t)256 << 20) / per_trial);
            batch = std::min<uint64_t>(cap, std::max<uint64_t>(n_trials, (uint64_t)kTuneTrials));
            if ((e = grow(ws.prep, batch * per_trial)) != hipSuccess)
                return hip_err(e, "trial gate buffer");
            if ((e = grow(ws.prepx, batch * sizeof(uint32_t))) != hipSuccess)
                return hip_err(e, "trial mask buffer");
            prep = ws.prep.p;
            prepx = ws.prepx.p;
        }

        TrialLaunch L{};
        L.prep_ops = prep;
        L.prep_X = reinterpret_cast<uint32_t *>(prepx);
        L.prep_batch = batch;
        L.gates = reinterpret_cast<const TrialGate *>(ws.gates.p);
        L.ngates = (uint32_t)n;
        L.M = (uint32_t)num_qubits;
        L.sigma = base->sigma;
        L.p_bit = base->p_bitflip;
        L.p_phase = base->p_phaseflip;
        L.seed = base->seed;
        L.trial0 = base->trial;
        L.ideal = ideal_ptr;

        const TuneKey key(num_qubits, dtype, (uint32_t)n, base->sigma > 0.0 ? 1 : 0,
                          (base->p_bitflip > 0.0 || base->p_phaseflip > 0.0) ? 1 : 0);
        int variant = -1;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_load();
            auto it = g_tune.find(key);
            if (it != g_tune.end())
                variant = it->second;
        }
        const int elem = dtype == QSIM_C64 ? 8 : 16;
        // QSIM_TRIAL_VARIANT forces a variant (when it can run this register)
        if (const char *v = getenv("QSIM_TRIAL_VARIANT")) {
            const int forced = atoi(v);
            TrialLaunch probe = L;
            gs.apply(probe, forced);
            if (forced >= 0 && forced < trial_variants() && trial_grid(forced, num_qubits, elem) > 0 &&
                (trial_group_bits(forced) == 0 || probe.sched != nullptr))
                variant = forced;
        }
        if (variant < 0 || trial_grid(variant, num_qubits, elem) <= 0) {
            if ((e = grow(ws.tune, kTuneTrials * sizeof(double))) != hipSuccess)
                return hip_err(e, "tune buffer");
            TrialLaunch T = L;
            T.n_trials = 1;  // grid set per variant inside
            rc = autotune(dtype, T, gs, st, reinterpret_cast<double *>(ws.tune.p), variant);
            if (rc != QSIM_OK)
                return rc;
            std::lock_guard<std::mutex> lk(g_tune_mu);
            tune_store(key, variant);
        }
        L.variant = variant;
        L.grid = trial_grid(variant, num_qubits, elem);
        gs.apply(L, variant);
        if (L.grid <= 0)
            return set_error(QSIM_EDEVICE, "trial kernel cannot run this register");
        L.n_trials = n_trials;
        L.out_F = reinterpret_cast<double *>(ws.out.p);
        if ((e = launch(dtype, L, st)) != hipSuccess)
            return hip_err(e, "trial launch");
        if ((e = hipMemcpyAsync(out_F, ws.out.p, n_trials * sizeof(double), hipMemcpyDeviceToHost,
                                st)) != hipSuccess)
            return hip_err(e, "result copy");
        if ((e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_err(e, "trial sync");
        return QSIM_OK;
    });
}


extern "C" int qsim_trial_plan(const qsim_gate *gates, size_t n, int num_qubits, int group_bits,
                               uint32_t *out, size_t cap, size_t *n_groups)
{
    return guarded(__func__, [&]() -> int {
        if (group_bits != 4 && group_bits != 5)
            return set_error(QSIM_EINVAL, "group_bits %d is neither 4 nor 5", group_bits);
        if (num_qubits - group_bits < 6 || num_qubits - group_bits > 10)
            return set_error(QSIM_EINVAL,
                             "num_qubits %d: the register-group kernels need 6 <= num_qubits - "
                             "group_bits <= 10", num_qubits);
        if (n > 0 && gates == nullptr)
            return set_error(QSIM_EINVAL, "gates is NULL");
        if (n > (size_t)UINT32_MAX)
            return set_error(QSIM_EINVAL, "too many gates");
        char why[160];
        for (size_t k = 0; k < n; ++k) {
            if (!gate_valid(gates[k], num_qubits, why, sizeof(why)))
                return set_error(QSIM_EINVAL, "gate %zu: %s", k, why);
            if (gates[k].kind == QSIM_CPHASE)
                return set_error(QSIM_EINVAL, "gate %zu: the trial kernels do not take "
                                 "controlled phases", k);
        }
        std::vector<uint32_t> sched;
        uint32_t nchunks = 0, ngroups = 0;
        group_schedule(gates, n, num_qubits, group_bits, sched, nchunks, ngroups);
        if (n_groups != nullptr)
            *n_groups = ngroups;
        for (size_t g = 0; g < ngroups && g < cap && out != nullptr; ++g) {
            const uint32_t word = sched[4 * g + 2];
            uint32_t mask = 0;
            for (int i = 0; i < group_bits; ++i)
                mask |= 1u << ((word >> (4 * i)) & 15u);
            out[4 * g] = sched[4 * g];
            out[4 * g + 1] = sched[4 * g + 1];
            out[4 * g + 2] = mask;
            out[4 * g + 3] = sched[4 * g + 3];
        }
        return QSIM_OK;
    });
}
