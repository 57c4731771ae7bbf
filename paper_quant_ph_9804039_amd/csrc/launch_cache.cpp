// Per-kernel, per-device launch facts (dynamic-LDS allowance, resident
// workgroups), computed once and shared by every host thread.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "launch.h"

namespace qsim {
namespace {

struct Cache {
    std::mutex mu;
    std::map<std::pair<const void *, int>, size_t> lds;                 // (kernel, device)
    std::map<std::tuple<const void *, int, int, size_t>, int> resident;  // + threads, lds
};

Cache &cache()
{
    static Cache *c = new Cache();  // never destroyed: kernels may launch during exit
    return *c;
}

}  // namespace

hipError_t kernel_allow_lds(const void *fn, size_t lds)
{
    if (lds <= 65536)
        return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t &allowed = c.lds[{fn, dev}];
    if (lds <= allowed)
        return hipSuccess;
    // the allowance only grows, so a launch sized below it stays valid
    // whatever another thread asks for at the same time
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    allowed = lds;
    return hipSuccess;
}

int kernel_resident_blocks(const void *fn, int threads, size_t lds)
{
    if (kernel_allow_lds(fn, lds) != hipSuccess)
        return 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    Cache &c = cache();
    std::lock_guard<std::mutex> lk(c.mu);
    const auto key = std::make_tuple(fn, dev, threads, lds);
    const auto it = c.resident.find(key);
    if (it != c.resident.end())
        return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int n = per_cu * cus;
    c.resident[key] = n;
    return n;
}

}  // namespace qsim
