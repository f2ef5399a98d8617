// Small device writes through kernel arguments (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

// Words one pm_put_words launch carries (its arguments stay under 4 KiB).
constexpr uint32_t kPutWords = 960;

// Write n <= kPutWords words to device memory dst, in order on stream st.
extern "C" hipError_t pmk_put(uint32_t *dst, const uint32_t *words, uint32_t n, hipStream_t st);
