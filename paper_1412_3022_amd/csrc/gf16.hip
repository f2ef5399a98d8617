// GF(2^16) region matrix multiplication: out[r] = sum_c A[r][c] * in[c] over
// blocks of 16-bit symbols (symbol p in bytes 2p, low, and 2p + 1, high).
//
// Section 3.3 takes the sparse PM-MSR construction to GF(2^16) for k up to
// 64; every operation of such a code is still a region matrix product
// (Sections 2 and 4), now with 16-bit coefficients.  The matrices of those
// codes are large (B = k(k - 1) up to 4032 columns), so the kernel reads the
// matrix as data, like the split-table kernels of the byte field, instead of
// compiling it.
//
// Multiplication by a constant c is linear over GF(2).  Each byte of a
// symbol x is split into pieces of 3, 3 and 2 bits, x = sum_p v_p x^(e_p)
// with e_p = 0, 3, 6, 8, 11, 14, and c*x is the sum of c*(v_p x^(e_p)).  A
// piece has at most 8 values, so each of those products is one v_perm_b32
// lookup per output byte in an 8-byte table.  The tables of every field
// element sit in one 8 MiB array (32 dwords per element) that the host fills
// once per device.
//
// Data layout per lane: 8 bytes (4 symbols) per unit, U units 512 bytes
// apart, so one load instruction of a wave covers 512 contiguous bytes and a
// wave tile is U * 512 bytes.  The low bytes of the 4 symbols are gathered
// into one dword and the high bytes into another (one v_perm_b32 each), so
// every lookup acts on 4 symbols at once; the results are interleaved back
// before the store.
//
// Work: a work item is (row group, tile); a wave takes one.  A row group is
// up to R output rows that share the list of columns any of them reads;
// each column record holds the R coefficients (0 where a row does not read
// it).  Items are numbered tile-major, so the groups of one tile run side by
// side and share its source columns in L2, and consecutive work-groups are
// placed on the same XCD.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gf16k.hpp"

namespace {

constexpr uint32_t kWaves = 4;

// 8 bytes at byte offset pos of a block of s bytes (s even, pos % 8 == 0):
// the symbols past s read as zero.
__device__ __forceinline__ uint2 load_unit(const uint8_t *p, uint64_t pos, uint64_t s) {
    if (pos + 8u <= s) return *reinterpret_cast<const uint2 *>(p + pos);
    uint32_t w[2] = {0u, 0u};
    for (uint32_t t = 0; t < 4u; ++t)
        if (pos + 2u * t < s) w[t / 2u] |= static_cast<uint32_t>(*reinterpret_cast<const uint16_t *>(p + pos + 2u * t))
                                           << (16u * (t % 2u));
    return make_uint2(w[0], w[1]);
}

__device__ __forceinline__ void store_unit(uint8_t *p, uint64_t pos, uint64_t s, uint2 v) {
    if (pos + 8u <= s) {
        *reinterpret_cast<uint2 *>(p + pos) = v;
        return;
    }
    const uint32_t w[2] = {v.x, v.y};
    for (uint32_t t = 0; t < 4u; ++t)
        if (pos + 2u * t < s)
            *reinterpret_cast<uint16_t *>(p + pos + 2u * t) = static_cast<uint16_t>(w[t / 2u] >> (16u * (t % 2u)));
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

template <int R, int U>
__global__ __launch_bounds__(64 * kWaves) void pm_apply16(PmkApply16 a) {
    // the wave index is the same in all lanes: made a scalar, so the work
    // item, the program words and the coefficient tables are read with
    // scalar loads into SGPRs
    const uint32_t lane = threadIdx.x % 64u, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    const uint32_t nwg = gridDim.x, b = blockIdx.x, per = nwg / 8u;
    const uint32_t wg = b < per * 8u ? (b % 8u) * per + b / 8u : b;
    const uint64_t item = static_cast<uint64_t>(wg) * kWaves + wave;
    if (item >= static_cast<uint64_t>(a.ngroups) * a.ntiles) return;
    const uint32_t tile = static_cast<uint32_t>(item / a.ngroups), g = static_cast<uint32_t>(item % a.ngroups);
    const uint32_t *gd = a.prog + kPm16Header + g * (2u + R);
    const uint32_t off = gd[0], ncols = gd[1];
    const uint64_t base = static_cast<uint64_t>(tile) * (U * 512u) + lane * 8u;

    if (ncols == kPm16CopyGroup) {   // rows that are input blocks as they are
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t row = gd[2 + r];
            if (row == kPm16NoRow) continue;
            const uint8_t *src = a.in + static_cast<uint64_t>(a.prog[off + r]) * a.in_ld;
            uint8_t *dst = a.out + static_cast<uint64_t>(row) * a.out_ld;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t pos = base + u * 512u;
                if (pos < a.s) store_unit(dst, pos, a.s, load_unit(src, pos, a.s));
            }
        }
        return;
    }

    uint32_t accL[R][U], accH[R][U];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int u = 0; u < U; ++u) accL[r][u] = accH[r][u] = 0u;

    for (uint32_t j = 0; j < ncols; ++j) {
        const uint32_t *rec = a.prog + off + j * (1u + R / 2);
        const uint8_t *src = a.in + static_cast<uint64_t>(rec[0]) * a.in_ld;
        // the six 3/3/2-bit pieces of the 4 symbols of each unit, as byte selectors
        uint32_t sel[6][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint2 v = load_unit(src, base + u * 512u, a.s);
            const uint32_t lo = __builtin_amdgcn_perm(v.y, v.x, 0x06040200u);   // low bytes of 4 symbols
            const uint32_t hi = __builtin_amdgcn_perm(v.y, v.x, 0x07050301u);   // high bytes
            sel[0][u] = lo & 0x07070707u;
            sel[1][u] = (lo >> 3) & 0x07070707u;
            sel[2][u] = (lo >> 6) & 0x03030303u;
            sel[3][u] = hi & 0x07070707u;
            sel[4][u] = (hi >> 3) & 0x07070707u;
            sel[5][u] = (hi >> 6) & 0x03030303u;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t c = (rec[1 + r / 2] >> (16 * (r % 2))) & 0xFFFFu;
            if (!c) continue;
            const uint32_t *t = a.tables + static_cast<uint64_t>(c) * kPm16TableWords;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // piece p, output byte h: table dwords 4p + 2h, 4p + 2h + 1
                uint32_t l = accL[r][u], h = accH[r][u];
                l = xor3(l, __builtin_amdgcn_perm(t[1], t[0], sel[0][u]), __builtin_amdgcn_perm(t[5], t[4], sel[1][u]));
                l = xor3(l, __builtin_amdgcn_perm(t[9], t[8], sel[2][u]), __builtin_amdgcn_perm(t[13], t[12], sel[3][u]));
                l = xor3(l, __builtin_amdgcn_perm(t[17], t[16], sel[4][u]),
                         __builtin_amdgcn_perm(t[21], t[20], sel[5][u]));
                h = xor3(h, __builtin_amdgcn_perm(t[3], t[2], sel[0][u]), __builtin_amdgcn_perm(t[7], t[6], sel[1][u]));
                h = xor3(h, __builtin_amdgcn_perm(t[11], t[10], sel[2][u]),
                         __builtin_amdgcn_perm(t[15], t[14], sel[3][u]));
                h = xor3(h, __builtin_amdgcn_perm(t[19], t[18], sel[4][u]),
                         __builtin_amdgcn_perm(t[23], t[22], sel[5][u]));
                accL[r][u] = l;
                accH[r][u] = h;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t row = gd[2 + r];
        if (row == kPm16NoRow) continue;
        uint8_t *dst = a.out + static_cast<uint64_t>(row) * a.out_ld;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t pos = base + u * 512u;
            if (pos >= a.s) continue;
            const uint2 v = make_uint2(__builtin_amdgcn_perm(accH[r][u], accL[r][u], 0x05010400u),
                                       __builtin_amdgcn_perm(accH[r][u], accL[r][u], 0x07030602u));
            store_unit(dst, pos, a.s, v);
        }
    }
}

}  // namespace

extern "C" hipError_t pmk_apply16(const PmkApply16 *h, hipStream_t st) {
    const uint64_t items = static_cast<uint64_t>(h->ngroups) * h->ntiles;
    if (items == 0) return hipSuccess;
    const uint64_t nwg = (items + kWaves - 1) / kWaves;
    if (nwg > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((pm_apply16<kPm16Rows, kPm16Units>), dim3(static_cast<uint32_t>(nwg)), dim3(64 * kWaves), 0,
                       st, *h);
    return hipGetLastError();
}
