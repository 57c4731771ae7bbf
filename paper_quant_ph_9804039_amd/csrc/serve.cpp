// qsim_serve: continuous batching of simulation requests on one GPU.
//
// One host thread runs an event loop: arrivals join a waiting list; a waiting
// request is admitted when a slot (HIP stream) is idle, the arena has room
// for its two registers and, if its registers stream from HBM ("heavy"),
// fewer than max_heavy heavy requests are in flight (a heavy request alone
// keeps the HBM busy; light ones overlap with it almost for free); admission
// queues all of its work on the slot's stream (error-free run, noisy run,
// fidelity, a copy of four doubles into pinned memory, an event), so
// admitted requests overlap on the device; the
// loop polls the events and, when one completes, takes the fidelity and
// returns slot and memory.  The arena is one allocation made before the
// loop, split first-fit; registers are bound to slot states whose scratch
// buffers were also sized beforehand.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <thread>
#include <vector>

#include "common.h"
#include "internal.h"
#include "qsim.h"

using namespace qsim;

namespace {

int hip_err(hipError_t e, const char *what)
{
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? QSIM_ENOMEM : QSIM_EDEVICE, "%s: %s", what,
                     hipGetErrorString(e));
}

// First-fit allocator over [0, size) with coalescing of freed neighbours.
class Arena {
  public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0)
                    free_[off + bytes] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + kAlign - 1) & ~(kAlign - 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }

  private:
    static constexpr size_t kAlign = 256;
    std::map<size_t, size_t> free_;
    size_t used_ = 0;
};

size_t elem_bytes(int dtype) { return dtype == QSIM_C64 ? 8 : 16; }

size_t footprint(const qsim_request &r)
{
    const size_t one = ((size_t)1 << r.num_qubits) * elem_bytes(r.dtype);
    return 2 * ((one + 255) & ~(size_t)255);
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    qsim_state *ideal = nullptr;
    qsim_state *noisy = nullptr;
    double *result = nullptr;  // pinned, 4 doubles
    bool busy = false;
    size_t req = 0;
    size_t off = 0, bytes = 0;
};

struct Loop {
    std::vector<Slot> slots;
    void *arena_mem = nullptr;
    ~Loop()
    {
        for (Slot &s : slots) {
            if (s.stream)
                (void)hipStreamSynchronize(s.stream);
            slot_state_destroy(s.ideal);
            slot_state_destroy(s.noisy);
            if (s.result)
                (void)hipHostFree(s.result);
            if (s.done)
                (void)hipEventDestroy(s.done);
            if (s.stream)
                (void)hipStreamDestroy(s.stream);
        }
        if (arena_mem)
            (void)hipFree(arena_mem);
    }
};

// Queue all of a request's work on its slot.
int admit(Slot &sl, const qsim_request &r, char *base)
{
    const size_t half = sl.bytes / 2;
    int rc = slot_state_bind(sl.ideal, r.num_qubits, r.dtype, base + sl.off);
    if (rc == QSIM_OK)
        rc = slot_state_bind(sl.noisy, r.num_qubits, r.dtype, base + sl.off + half);
    if (rc == QSIM_OK)
        rc = qsim_apply_circuit(sl.ideal, r.gates, r.n_gates);
    if (rc == QSIM_OK)
        rc = qsim_inject_errors(sl.noisy, &r.errors);
    if (rc == QSIM_OK)
        rc = qsim_apply_circuit(sl.noisy, r.gates, r.n_gates);
    if (rc == QSIM_OK)
        rc = overlap_enqueue(sl.ideal, sl.noisy, sl.result);
    if (rc == QSIM_OK) {
        hipError_t e = hipEventRecord(sl.done, sl.stream);
        if (e != hipSuccess)
            rc = hip_err(e, "completion event");
    }
    return rc;
}

}  // namespace

extern "C" int qsim_serve(const qsim_request *reqs, size_t n, const qsim_serve_options *opt,
                          qsim_result *out)
{
    return guarded(__func__, [&]() -> int {
        if (n > 0 && (reqs == nullptr || out == nullptr))
            return set_error(QSIM_EINVAL, "NULL argument");
        qsim_serve_options o{};
        if (opt)
            o = *opt;
        const int nslots = o.max_slots == 0 ? 8 : o.max_slots;
        if (nslots < 1 || nslots > 64)
            return set_error(QSIM_EINVAL, "max_slots %d outside [1, 64]", o.max_slots);
        if (o.max_heavy < 0)
            return set_error(QSIM_EINVAL, "max_heavy %d is negative", o.max_heavy);
        const int max_heavy = o.max_heavy == 0 ? 1 : o.max_heavy;
        const size_t heavy_bytes = o.heavy_bytes == 0 ? ((size_t)256 << 20) : o.heavy_bytes;
        int max_m = 1;
        char why[160];
        for (size_t i = 0; i < n; ++i) {
            const qsim_request &r = reqs[i];
            if (r.num_qubits < 1 || r.num_qubits > QSIM_MAX_QUBITS)
                return set_error(QSIM_EINVAL, "request %zu: num_qubits %d", i, r.num_qubits);
            if (r.dtype != QSIM_C64 && r.dtype != QSIM_C128)
                return set_error(QSIM_EINVAL, "request %zu: dtype %d", i, r.dtype);
            if (!(r.arrival_s >= 0.0) || !std::isfinite(r.arrival_s))
                return set_error(QSIM_EINVAL, "request %zu: arrival time", i);
            if (!error_model_valid(r.errors))
                return set_error(QSIM_EINVAL, "request %zu: error model", i);
            if (r.n_gates > 0 && r.gates == nullptr)
                return set_error(QSIM_EINVAL, "request %zu: gates is NULL", i);
            for (size_t k = 0; k < r.n_gates; ++k)
                if (!gate_valid(r.gates[k], r.num_qubits, why, sizeof(why)))
                    return set_error(QSIM_EINVAL, "request %zu gate %zu: %s", i, k, why);
            max_m = std::max(max_m, r.num_qubits);
        }
        for (size_t i = 0; i < n; ++i)
            out[i] = qsim_result{0.0, -1.0, -1.0, QSIM_OK, -1};
        if (n == 0)
            return QSIM_OK;

        hipError_t e = hipSetDevice(o.device);
        if (e != hipSuccess)
            return hip_err(e, "hipSetDevice");
        size_t budget = o.hbm_budget;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess)
                return hip_err(e, "hipMemGetInfo");
            budget = std::min((size_t)64 << 30, (size_t)(0.8 * (double)fr));
        }
        Loop L;
        if ((e = hipMalloc(&L.arena_mem, budget)) != hipSuccess)
            return hip_err(e, "arena");
        Arena arena(budget);
        L.slots.resize(nslots);
        for (Slot &sl : L.slots) {
            if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess)
                return hip_err(e, "slot stream");
            if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
                return hip_err(e, "slot event");
            if ((e = hipHostMalloc((void **)&sl.result, 4 * sizeof(double), hipHostMallocDefault)) !=
                hipSuccess)
                return hip_err(e, "slot result");
            int rc = slot_state_create(o.device, sl.stream, max_m, &sl.ideal);
            if (rc == QSIM_OK)
                rc = slot_state_create(o.device, sl.stream, max_m, &sl.noisy);
            if (rc != QSIM_OK)
                return rc;
        }

        std::vector<size_t> order(n);
        for (size_t i = 0; i < n; ++i)
            order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
        std::deque<size_t> waiting;
        size_t next = 0, finished = 0;
        char *base = reinterpret_cast<char *>(L.arena_mem);
        const auto t0 = std::chrono::steady_clock::now();
        auto now = [&] {
            return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        };
        while (finished < n) {
            bool progress = false;
            const double t = now();
            while (next < n && reqs[order[next]].arrival_s <= t) {
                const size_t i = order[next++];
                if (footprint(reqs[i]) > budget) {
                    out[i].status = QSIM_ENOMEM;
                    out[i].done_s = t;
                    ++finished;
                } else {
                    waiting.push_back(i);
                }
                progress = true;
            }
            // completions
            for (size_t si = 0; si < L.slots.size(); ++si) {
                Slot &sl = L.slots[si];
                if (!sl.busy)
                    continue;
                e = hipEventQuery(sl.done);
                if (e == hipErrorNotReady)
                    continue;
                qsim_result &res = out[sl.req];
                if (e == hipSuccess) {
                    const double *v = sl.result;
                    res.fidelity = (v[0] * v[0] + v[1] * v[1]) / (v[2] * v[3]);
                } else {
                    res.status = hip_err(e, "request work");
                }
                res.done_s = now();
                arena.release(sl.off, sl.bytes);
                sl.busy = false;
                ++finished;
                progress = true;
            }
            // admissions, in arrival order; at most max_heavy heavy requests
            // in flight
            int heavy_now = 0;
            for (const Slot &s : L.slots)
                if (s.busy && s.bytes >= heavy_bytes)
                    ++heavy_now;
            for (auto it = waiting.begin(); it != waiting.end();) {
                auto free_slot = std::find_if(L.slots.begin(), L.slots.end(),
                                              [](const Slot &s) { return !s.busy; });
                if (free_slot == L.slots.end())
                    break;
                const size_t i = *it;
                size_t off = 0;
                const size_t bytes = footprint(reqs[i]);
                const bool heavy = bytes >= heavy_bytes;
                if (heavy && heavy_now >= max_heavy) {
                    if (o.strict_fifo)
                        break;
                    ++it;
                    continue;
                }
                if (!arena.alloc(bytes, off)) {
                    if (o.strict_fifo)
                        break;
                    ++it;
                    continue;
                }
                Slot &sl = *free_slot;
                sl.off = off;
                sl.bytes = bytes;
                sl.req = i;
                out[i].admit_s = now();
                out[i].slot = (int)(free_slot - L.slots.begin());
                const int rc = admit(sl, reqs[i], base);
                if (rc != QSIM_OK) {
                    (void)hipStreamSynchronize(sl.stream);
                    arena.release(off, bytes);
                    out[i].status = rc;
                    out[i].done_s = now();
                    ++finished;
                } else {
                    sl.busy = true;
                    if (heavy)
                        ++heavy_now;
                }
                it = waiting.erase(it);
                progress = true;
            }
            if (!progress)
                std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        return QSIM_OK;
    });
}
