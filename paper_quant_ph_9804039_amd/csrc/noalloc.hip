// qsim_overlap_noalloc: the overlap readout of two caller-owned registers
// with its reduction scratch in a static device array, so the call allocates
// no memory at all (host or device).
//
// The array lives in this translation unit.  Host code never passes its name
// to a kernel: the name is a host-side stand-in, not a device address.  Its
// address on each device is looked up once, with that device current, by
// hipGetSymbolAddress and kept per device.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "internal.h"
#include "launch.h"
#include "qsim.h"

// Per-block FP64 partials of the overlap reduction (4 per block, at most
// kReduceBlocks blocks whatever the register size) plus its 4 results:
// 32.1 KiB per device, held until the process ends.
constexpr size_t kScratchDoubles = 4 * (size_t)qsim::kReduceBlocks + 8;
constexpr size_t kResultOffset = 4 * (size_t)qsim::kReduceBlocks;

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    std::mutex lock;       // held for a whole call: calls on one device do not overlap
    double *ptr = nullptr; // device address of `scratch` on this device
};

DeviceScratch g_dev[kMaxDevices];

// Device address of the scratch array on `device` (the current device),
// looked up on the first call there.  Called with g_dev[device].lock held.
int scratch_on(int device, double **out)
{
    DeviceScratch &d = g_dev[device];
    if (d.ptr == nullptr) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return qsim::set_error(QSIM_EDEVICE, "qsim_overlap_noalloc: scratch address on "
                                   "device %d: %s", device, hipGetErrorString(e));
        d.ptr = static_cast<double *>(p);
    }
    *out = d.ptr;
    return QSIM_OK;
}

// A register argument must be device memory on `device` holding at least
// `bytes` from `p` on.
int check_register(const void *p, size_t bytes, int device, const char *name)
{
    if (p == nullptr)
        return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: %s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0)
        return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: %s must be 16-byte aligned",
                               name);
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != device) {
        (void)hipGetLastError();
        return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: %s is not device memory "
                               "of device %d", name, device);
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess) {
        (void)hipGetLastError();
        return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: %s: no allocation found",
                               name);
    }
    const uintptr_t b = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
    if (q < b || q - b > size || size - (q - b) < bytes)
        return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: %s holds fewer than the "
                               "%zu bytes of the register", name, bytes);
    return QSIM_OK;
}

template <typename Ra, typename Rb>
hipError_t enqueue(const void *a, const void *b, int M, double *s, hipStream_t st)
{
    return qsim::launch_overlap<Ra, Rb>(static_cast<const qsim::cplx<Ra> *>(a),
                                        static_cast<const qsim::cplx<Rb> *>(b), M, s,
                                        s + kResultOffset, st);
}

}  // namespace

extern "C" int qsim_overlap_noalloc(const void *a, int dtype_a, const void *b, int dtype_b,
                                    int num_qubits, int device, void *hip_stream, double out[4])
{
    return qsim::guarded(__func__, [&]() -> int {
        if (out == nullptr)
            return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: out is NULL");
        if (num_qubits < 1 || num_qubits > QSIM_MAX_QUBITS)
            return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: num_qubits %d outside "
                                   "[1, %d]", num_qubits, QSIM_MAX_QUBITS);
        const bool ok_a = dtype_a == QSIM_C64 || dtype_a == QSIM_C128;
        const bool ok_b = dtype_b == QSIM_C64 || dtype_b == QSIM_C128;
        if (!ok_a || !ok_b)
            return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: dtype must be "
                                   "QSIM_C64 or QSIM_C128");
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess)
            return qsim::set_error(QSIM_EDEVICE, "qsim_overlap_noalloc: hipGetDeviceCount: %s",
                                   hipGetErrorString(e));
        if (device < 0 || device >= ndev || device >= kMaxDevices)
            return qsim::set_error(QSIM_EINVAL, "qsim_overlap_noalloc: device %d outside "
                                   "[0, %d)", device, ndev < kMaxDevices ? ndev : kMaxDevices);
        e = hipSetDevice(device);
        if (e != hipSuccess)
            return qsim::set_error(QSIM_EDEVICE, "qsim_overlap_noalloc: hipSetDevice: %s",
                                   hipGetErrorString(e));
        const size_t n = (size_t)1 << num_qubits;
        int rc = check_register(a, n * (dtype_a == QSIM_C64 ? 8 : 16), device, "a");
        if (rc == QSIM_OK)
            rc = check_register(b, n * (dtype_b == QSIM_C64 ? 8 : 16), device, "b");
        if (rc != QSIM_OK)
            return rc;
        hipStream_t st = static_cast<hipStream_t>(hip_stream);
        std::lock_guard<std::mutex> hold(g_dev[device].lock);
        double *s = nullptr;
        rc = scratch_on(device, &s);
        if (rc != QSIM_OK)
            return rc;
        // every partial the finishing block reads is written by this call's
        // first kernel, so nothing needs clearing between calls
        if (dtype_a == QSIM_C64 && dtype_b == QSIM_C64)
            e = enqueue<float, float>(a, b, num_qubits, s, st);
        else if (dtype_a == QSIM_C64)
            e = enqueue<float, double>(a, b, num_qubits, s, st);
        else if (dtype_b == QSIM_C64)
            e = enqueue<double, float>(a, b, num_qubits, s, st);
        else
            e = enqueue<double, double>(a, b, num_qubits, s, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, s + kResultOffset, 4 * sizeof(double), hipMemcpyDeviceToHost,
                               st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return qsim::set_error(QSIM_EDEVICE, "qsim_overlap_noalloc: %s", hipGetErrorString(e));
        return QSIM_OK;
    });
}
