// Fixed device scratch for the entry point that allocates nothing
// (pm_decode_specific_noalloc in capi.cpp).
//
// The array lives in the library's code object, so HIP reserves it on every
// device the code object is loaded on, and keeps it until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address on the current device comes from hipGetSymbolAddress, once
// per device, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>

#include "noalloc.hpp"

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

extern "C" hipError_t pmk_noalloc_scratch(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *ptr = g_ptr[dev];
    return hipSuccess;
}
