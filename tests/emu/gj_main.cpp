// Host driver for the batched Gauss-Jordan kernel (gj.hip): the kernel's own
// source, with the host stand-ins below, runs one problem at a time with one
// OS thread per GPU thread; __syncthreads is a std::barrier and the LDS block
// is a heap buffer of exactly the kernel's LDS size, so AddressSanitizer
// sees any access outside it.
//
//   gj_main IN OUT
// IN: u64 count, B, nrows, nsets, alpha, nnodes, src_ld, src_stride, d_ld,
//     d_stride, has_sets, src_bytes; src bytes; count*nsets u32 node ids
//     when has_sets.  OUT: count*d_stride bytes of D, count*B u32 kept,
//     count i32 status.
#include <atomic>
#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

struct Dim3 { uint32_t x = 0; };
static thread_local Dim3 threadIdx, blockIdx;
static Dim3 blockDim;
static std::barrier<> *g_bar = nullptr;
static unsigned char *g_sm = nullptr;

typedef int hipError_t;
typedef void *hipStream_t;
#define hipSuccess 0
#define __global__
#define __launch_bounds__(n)
#define __device__
#define __host__
#define __constant__
#define __forceinline__ inline
#define __syncthreads() g_bar->arrive_and_wait()
#define hipFuncAttributeMaxDynamicSharedMemorySize 0
#define hipFuncSetAttribute(...) 0
#define hipLaunchKernelGGL(...) (void)0
#define hipGetLastError() 0

static inline uint32_t atomicOr(uint32_t *p, uint32_t v) { return std::atomic_ref<uint32_t>(*p).fetch_or(v); }
// v_bitop3_b32: bit i of the result is bit (a_i << 2 | b_i << 1 | c_i) of imm
static inline uint32_t __builtin_amdgcn_bitop3_b32(uint32_t a, uint32_t b, uint32_t c, unsigned imm) {
    uint32_t r = 0;
    for (unsigned k = 0; k < 8; ++k)
        if ((imm >> k) & 1u) r |= ((k & 4u) ? a : ~a) & ((k & 2u) ? b : ~b) & ((k & 1u) ? c : ~c);
    return r;
}
static inline uint32_t atomicMin(uint32_t *p, uint32_t v) {
    std::atomic_ref<uint32_t> r(*p);
    uint32_t o = r.load();
    while (v < o && !r.compare_exchange_weak(o, v)) {
    }
    return o;
}

#include "gj_kernel.inc"

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint64_t h[12];
    if (fread(h, sizeof h, 1, f) != 1) return 2;
    const uint64_t count = h[0], B = h[1], nrows = h[2], nsets = h[3], alpha = h[4], nnodes = h[5];
    const uint64_t src_ld = h[6], src_stride = h[7], d_ld = h[8], d_stride = h[9], has_sets = h[10], sb = h[11];
    std::vector<uint8_t> src(sb);
    if (sb && fread(src.data(), 1, sb, f) != sb) return 2;
    std::vector<uint32_t> sets(has_sets ? count * nsets : 0);
    if (!sets.empty() && fread(sets.data(), 4, sets.size(), f) != sets.size()) return 2;
    fclose(f);
    std::vector<uint8_t> D(count * d_stride, 0x5A);
    std::vector<uint32_t> kept(count * B, 0xFFFFFFFFu);
    std::vector<int32_t> status(count, 99);
    const PmkGj a{src.data(), src_ld, src_stride, has_sets ? sets.data() : nullptr,
                  static_cast<uint32_t>(nsets), static_cast<uint32_t>(alpha), static_cast<uint32_t>(nnodes),
                  static_cast<uint32_t>(nrows), static_cast<uint32_t>(B), D.data(), d_ld, d_stride,
                  kept.data(), status.data()};
    const uint32_t T = B <= 64 ? 256u : 1024u;   // the block size pmk_gj launches
    const size_t lds = pmk_gj_lds_bytes(static_cast<uint32_t>(B), static_cast<uint32_t>(nrows),
                                        has_sets ? static_cast<uint32_t>(nsets) : 0u);
    for (uint64_t p = 0; p < count; ++p) {
        g_sm = static_cast<unsigned char *>(malloc(lds));
        memset(g_sm, 0xA5, lds);   // LDS starts with garbage
        std::barrier<> bar(T);
        g_bar = &bar;
        blockDim.x = T;
        std::vector<std::thread> th;
        th.reserve(T);
        for (uint32_t t = 0; t < T; ++t)
            th.emplace_back([&a, t, p] {
                threadIdx.x = t;
                blockIdx.x = static_cast<uint32_t>(p);
                pm_gj(a);
            });
        for (auto &x : th) x.join();
        free(g_sm);
    }
    f = fopen(argv[2], "wb");
    if (!f) return 2;
    fwrite(D.data(), 1, D.size(), f);
    fwrite(kept.data(), 4, kept.size(), f);
    fwrite(status.data(), 4, status.size(), f);
    fclose(f);
    return 0;
}
