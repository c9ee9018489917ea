// Library-owned device scratch for the entry points that allocate nothing
// (lrx_solve_dev_noalloc).  One static array per device, held until the
// process ends; its device address is looked up once per device with that
// device current and kept, because in host code the array's name is only a
// host-side stand-in.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace lrx {

namespace {

static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int dev, void** ptr) {
    *ptr = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev) return hipErrorInvalidDevice;        // the caller makes dev current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}

}  // namespace lrx
