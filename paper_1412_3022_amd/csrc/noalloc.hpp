// The fixed device scratch of the no-allocation entry point (noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

// Bytes of the static scratch array, per device.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;

// Device address of the scratch array on the current device, looked up with
// hipGetSymbolAddress on the first call for that device and kept.
extern "C" hipError_t pmk_noalloc_scratch(void **ptr);
