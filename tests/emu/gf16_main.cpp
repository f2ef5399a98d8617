// Host driver for the GF(2^16) region kernel (gf16.hip): the kernel's own
// source, with the host stand-ins below, runs every lane of every wave of
// the launch in turn.  Inputs, outputs, program and tables are heap buffers
// of exactly their sizes, so AddressSanitizer sees any access outside them.
//
//   gf16_main IN OUT
// IN: u64 in_n, out_n, s, in_ld, out_ld, nwords, ngroups; in_n*in_ld input
//     bytes; nwords u32 program words; 65536*32 u32 table words.
// OUT: out_n*out_ld bytes (0x5A where the kernel does not write).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

struct Dim3 { uint32_t x = 0; };
static Dim3 threadIdx, blockIdx, gridDim;
struct uint2 { uint32_t x, y; };
static inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }

typedef int hipError_t;
typedef void *hipStream_t;
#define hipSuccess 0
#define hipErrorInvalidValue 1
#define __global__
#define __launch_bounds__(n)
#define __device__
#define __host__
#define __forceinline__ inline
#define hipLaunchKernelGGL(...) (void)0
#define hipGetLastError() 0
struct dim3 { dim3(uint32_t) {} };

// v_perm_b32: byte i of the result is byte sel_i of the 8 bytes {a:b}, b the
// low dword (selector values 0..7 only; the kernel uses no other)
static inline uint32_t __builtin_amdgcn_perm(uint32_t a, uint32_t b, uint32_t sel) {
    const uint64_t v = (static_cast<uint64_t>(a) << 32) | b;
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t s = (sel >> (8 * i)) & 0xFFu;
        if (s > 7) abort();
        r |= static_cast<uint32_t>((v >> (8 * s)) & 0xFFu) << (8 * i);
    }
    return r;
}
// every lane of a wave holds the same value where the kernel reads the first lane's
static inline uint32_t __builtin_amdgcn_readfirstlane(uint32_t v) { return v; }
// v_bitop3_b32: bit i of the result is bit (a_i << 2 | b_i << 1 | c_i) of imm
static inline uint32_t __builtin_amdgcn_bitop3_b32(uint32_t a, uint32_t b, uint32_t c, unsigned imm) {
    uint32_t r = 0;
    for (unsigned k = 0; k < 8; ++k)
        if ((imm >> k) & 1u) r |= ((k & 4u) ? a : ~a) & ((k & 2u) ? b : ~b) & ((k & 1u) ? c : ~c);
    return r;
}

#include "gf16_kernel.inc"

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint64_t h[7];
    if (fread(h, sizeof h, 1, f) != 1) return 2;
    const uint64_t in_n = h[0], out_n = h[1], s = h[2], in_ld = h[3], out_ld = h[4], nwords = h[5], ngroups = h[6];
    std::vector<uint8_t> in(in_n * in_ld);
    std::vector<uint32_t> prog(nwords), tab(static_cast<size_t>(65536) * kPm16TableWords);
    if (fread(in.data(), 1, in.size(), f) != in.size()) return 2;
    if (fread(prog.data(), 4, prog.size(), f) != prog.size()) return 2;
    if (fread(tab.data(), 4, tab.size(), f) != tab.size()) return 2;
    fclose(f);
    std::vector<uint8_t> out(out_n * out_ld, 0x5A);
    const uint64_t ntiles = (s + kPm16TileBytes - 1) / kPm16TileBytes;
    const PmkApply16 a{in.data(), in_ld, out.data(), out_ld, s, prog.data(), tab.data(),
                       static_cast<uint32_t>(ngroups), static_cast<uint32_t>(ntiles)};
    const uint64_t items = ngroups * ntiles, nwg = (items + kWaves - 1) / kWaves;   // the grid pmk_apply16 launches
    gridDim.x = static_cast<uint32_t>(nwg);
    for (uint32_t b = 0; b < nwg; ++b)
        for (uint32_t t = 0; t < 64 * kWaves; ++t) {
            blockIdx.x = b;
            threadIdx.x = t;
            pm_apply16<kPm16Rows, kPm16Units>(a);
        }
    FILE *g = fopen(argv[2], "wb");
    if (!g || fwrite(out.data(), 1, out.size(), g) != out.size()) return 2;
    fclose(g);
    return 0;
}
