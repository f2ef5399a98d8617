// Host stand-ins that let a generated bit-sliced kernel source compile as
// plain C++ (clang, for the ext_vector_type loads): the kernels share nothing
// between threads (no LDS, no barriers; cross-lane reads only of wave-uniform
// values), so running every (block, thread) in turn gives the GPU's bytes.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>
struct EmuDim { unsigned x; };
static EmuDim threadIdx, blockIdx;
#define __device__
#define __global__
#define __constant__ static const
#define __launch_bounds__(x)
#define __noinline__ __attribute__((noinline))
#define __forceinline__ inline
// v_bitop3_b32: bit i of the result is bit (a_i << 2 | b_i << 1 | c_i) of imm
// (the kernels use 0x96, a ^ b ^ c, and 0xD8, c ? b : a)
static inline unsigned __builtin_amdgcn_bitop3_b32(unsigned a, unsigned b, unsigned c, unsigned imm) {
    if (imm == 0x96) return a ^ b ^ c;          // the two tables the kernels use, without the loop
    if (imm == 0xD8) return (a & ~c) | (b & c);
    unsigned r = 0;
    for (unsigned k = 0; k < 8; ++k)
        if ((imm >> k) & 1u) r |= ((k & 4u) ? a : ~a) & ((k & 2u) ? b : ~b) & ((k & 1u) ? c : ~c);
    return r;
}
// Like the builtin, returns int (a caller that widens it without going
// through an unsigned type sign-extends, as on the GPU).
#define __builtin_amdgcn_readfirstlane(x) ((int)(x))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
// v_perm_b32 for byte selectors 0..7: bytes 0..3 from b, 4..7 from a
static inline unsigned __builtin_amdgcn_perm(unsigned a, unsigned b, unsigned sel) {
    const unsigned long long v = (static_cast<unsigned long long>(a) << 32) | b;
    unsigned r = 0;
    for (int i = 0; i < 4; ++i) {
        const unsigned s = (sel >> (8 * i)) & 0xFF;
        if (s > 7) abort();
        r |= static_cast<unsigned>((v >> (8 * s)) & 0xFF) << (8 * i);
    }
    return r;
}
#ifndef EMU_TILE
#define EMU_TILE 2048
#endif
#ifndef EMU_KERNEL
#define EMU_KERNEL pmbs
#endif
