// GF(2^8) region matrix kernels for gfx950 (CDNA4).
//
// out[r][p] = XOR_c A[r][c] * in[c][p] for every byte p of the regions: the
// data phase of encode (Y = G X), repair and decode (Section 2 of the paper).
// The paper multiplies a region by a constant with SIMD split tables
// (Section 4); here every lane owns 8 or 16 contiguous bytes of a byte tile,
// splits each source byte into 3 + 3 + 2 bit fields once, and looks the three
// partial products up with v_perm_b32 (an 8-entry byte table per selector
// byte).  One table half rides in an SGPR, the other in a VGPR.  Partial
// products are folded into per-row register accumulators three at a time with
// v_bitop3_b32.  Each work-group handles one (byte tile, row group) pair; the
// row group's coefficient tables are wave-uniform and come in through the
// scalar cache.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kTabWords = 5;
constexpr int kGroupWords = 8;
constexpr int kHeaderWords = 4;
constexpr int kWaves = 4;          // waves per work-group
constexpr int kThreads = 64 * kWaves;

struct ApplyArgs {
    const uint8_t *in;
    uint64_t in_ld;
    uint8_t *out;
    uint64_t out_ld;
    uint64_t s;            // bytes per block
    const uint32_t *prog;  // device program blob
    uint32_t ngroups;
    uint32_t nwork;        // tiles * groups
    uint32_t per_xcd;      // grid / 8
    uint32_t pad;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// ---- chunk I/O: VEC dwords per lane, full or clipped at the block end -----
template <int VEC, bool FULL>
__device__ __forceinline__ void load_chunk(const uint8_t *p, uint32_t avail, uint32_t (&x)[VEC]) {
    if constexpr (FULL) {
        if constexpr (VEC == 4) {
            const u32x4 v = *reinterpret_cast<const u32x4 *>(p);
            x[0] = v.x; x[1] = v.y; x[2] = v.z; x[3] = v.w;
        } else {
            const u32x2 v = *reinterpret_cast<const u32x2 *>(p);
            x[0] = v.x; x[1] = v.y;
        }
    } else {
#pragma unroll
        for (int w = 0; w < VEC; ++w) x[w] = 0;
#pragma unroll
        for (uint32_t b = 0; b < 4u * VEC; ++b)
            if (b < avail) x[b >> 2] |= static_cast<uint32_t>(p[b]) << (8 * (b & 3));
    }
}

template <int VEC, bool FULL>
__device__ __forceinline__ void store_chunk(uint8_t *p, uint32_t avail, const uint32_t (&x)[VEC]) {
    if constexpr (FULL) {
        if constexpr (VEC == 4) {
            const u32x4 v = {x[0], x[1], x[2], x[3]};
            __builtin_nontemporal_store(v, reinterpret_cast<u32x4 *>(p));
        } else {
            const u32x2 v = {x[0], x[1]};
            __builtin_nontemporal_store(v, reinterpret_cast<u32x2 *>(p));
        }
    } else {
#pragma unroll
        for (uint32_t b = 0; b < 4u * VEC; ++b)
            if (b < avail) p[b] = static_cast<uint8_t>(x[b >> 2] >> (8 * (b & 3)));
    }
}

// One lane's share of one row group: RG accumulators of VEC dwords.
template <int RG, int VEC, bool FULL>
__device__ __forceinline__ void table_group(const uint32_t *__restrict__ prog, const uint32_t *grec,
                                            const uint8_t *__restrict__ in, uint64_t in_ld,
                                            uint8_t *__restrict__ out, uint64_t out_ld,
                                            uint64_t off, uint32_t avail) {
    const uint32_t nrows = grec[1], ncols = grec[2];
    const uint32_t *cols = prog + grec[3];
    const uint32_t *tab = prog + grec[4];
    const uint32_t *rows = prog + grec[5];
    uint32_t acc[RG][VEC];
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[r][v] = 0;

    const uint8_t *inb = in + off;
    uint32_t x0[VEC], x1[VEC], n0[VEC], n1[VEC];
    if (ncols) {
        load_chunk<VEC, FULL>(inb + static_cast<uint64_t>(cols[0]) * in_ld, avail, n0);
        load_chunk<VEC, FULL>(inb + static_cast<uint64_t>(cols[1]) * in_ld, avail, n1);
    }
    for (uint32_t ci = 0; ci < ncols; ci += 2) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) { x0[v] = n0[v]; x1[v] = n1[v]; }
        if (ci + 2 < ncols) {   // prefetch the next column pair
            load_chunk<VEC, FULL>(inb + static_cast<uint64_t>(cols[ci + 2]) * in_ld, avail, n0);
            load_chunk<VEC, FULL>(inb + static_cast<uint64_t>(cols[ci + 3]) * in_ld, avail, n1);
        }
        uint32_t a0[VEC], b0[VEC], c0[VEC], a1[VEC], b1[VEC], c1[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            a0[v] = x0[v] & 0x07070707u;
            b0[v] = (x0[v] >> 3) & 0x07070707u;
            c0[v] = (x0[v] >> 6) & 0x03030303u;
            a1[v] = x1[v] & 0x07070707u;
            b1[v] = (x1[v] >> 3) & 0x07070707u;
            c1[v] = (x1[v] >> 6) & 0x03030303u;
        }
        const uint32_t *t0 = tab + ci * (RG * kTabWords);
        const uint32_t *t1 = t0 + RG * kTabWords;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const uint32_t *p = t0 + r * kTabWords;
            const uint32_t *q = t1 + r * kTabWords;
            const uint32_t p0 = p[0], p1 = p[1], p2 = p[2], p3 = p[3], p4 = p[4];
            const uint32_t q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4];
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                const uint32_t l0 = perm(p1, p0, a0[v]);
                const uint32_t m0 = perm(p3, p2, b0[v]);
                const uint32_t h0 = perm(p4, p4, c0[v]);
                const uint32_t l1 = perm(q1, q0, a1[v]);
                const uint32_t m1 = perm(q3, q2, b1[v]);
                const uint32_t h1 = perm(q4, q4, c1[v]);
                acc[r][v] = xor3(xor3(xor3(acc[r][v], l0, m0), h0, l1), m1, h1);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RG; ++r)
        if (static_cast<uint32_t>(r) < nrows)
            store_chunk<VEC, FULL>(out + static_cast<uint64_t>(rows[r]) * out_ld + off, avail, acc[r]);
}

template <int VEC, bool FULL>
__device__ __forceinline__ void copy_group(const uint32_t *__restrict__ prog, const uint32_t *grec,
                                           const uint8_t *__restrict__ in, uint64_t in_ld,
                                           uint8_t *__restrict__ out, uint64_t out_ld,
                                           uint64_t off, uint32_t avail) {
    const uint32_t nrows = grec[1];
    const uint32_t *cols = prog + grec[3];
    const uint32_t *rows = prog + grec[5];
    for (uint32_t r = 0; r < nrows; ++r) {
        uint32_t x[VEC];
        load_chunk<VEC, FULL>(in + static_cast<uint64_t>(cols[r]) * in_ld + off, avail, x);
        store_chunk<VEC, FULL>(out + static_cast<uint64_t>(rows[r]) * out_ld + off, avail, x);
    }
}

template <int RG, int VEC>
__device__ __forceinline__ void run_unit(const uint32_t *__restrict__ prog, uint32_t grp, uint64_t tile_off,
                                         const uint8_t *__restrict__ in, uint64_t in_ld,
                                         uint8_t *__restrict__ out, uint64_t out_ld, uint64_t s) {
    constexpr uint32_t kLaneBytes = 4 * VEC;
    constexpr uint32_t kWaveBytes = 64 * kLaneBytes;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const uint32_t lane = threadIdx.x % 64;
    const uint64_t wave_off = tile_off + static_cast<uint64_t>(wave) * kWaveBytes;
    if (wave_off >= s) return;
    const uint64_t off = wave_off + static_cast<uint64_t>(lane) * kLaneBytes;
    const uint32_t *grec = prog + kHeaderWords + grp * kGroupWords;
    const bool full = wave_off + kWaveBytes <= s;   // wave-uniform
    const uint32_t avail = off < s ? static_cast<uint32_t>(s - off < kLaneBytes ? s - off : kLaneBytes) : 0u;
    if (grec[0] == 0) {
        if (full) table_group<RG, VEC, true>(prog, grec, in, in_ld, out, out_ld, off, kLaneBytes);
        else table_group<RG, VEC, false>(prog, grec, in, in_ld, out, out_ld, off, avail);
    } else {
        if (full) copy_group<VEC, true>(prog, grec, in, in_ld, out, out_ld, off, kLaneBytes);
        else copy_group<VEC, false>(prog, grec, in, in_ld, out, out_ld, off, avail);
    }
}

// Plain launch: one work-group per (byte tile, row group).  Work-groups are
// dealt to the 8 XCDs round-robin by the hardware, so the linear work index
// is remapped to give each XCD a contiguous run: all row groups of a tile then
// meet in one L2, and their input re-reads hit there.
template <int RG, int VEC>
__global__ __launch_bounds__(kThreads) void pm_apply_kernel(ApplyArgs a) {
    const uint32_t b = blockIdx.x;
    const uint32_t lin = (b % 8u) * a.per_xcd + b / 8u;
    if (lin >= a.nwork) return;
    const uint32_t tile = lin / a.ngroups;
    const uint32_t grp = lin - tile * a.ngroups;
    constexpr uint64_t kTile = static_cast<uint64_t>(kThreads) * 4 * VEC;
    run_unit<RG, VEC>(a.prog, grp, tile * kTile, a.in, a.in_ld, a.out, a.out_ld, a.s);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side launchers (C linkage inside the library only).
struct PmkApply {
    const uint8_t *in;
    uint64_t in_ld;
    uint8_t *out;
    uint64_t out_ld;
    uint64_t s;
    const uint32_t *prog;
    uint32_t ngroups;
};

template <int RG, int VEC>
static hipError_t launch_apply(const PmkApply &h, hipStream_t st) {
    constexpr uint64_t kTile = static_cast<uint64_t>(kThreads) * 4 * VEC;
    const uint64_t ntiles = (h.s + kTile - 1) / kTile;
    const uint64_t nwork = ntiles * h.ngroups;
    if (nwork == 0) return hipSuccess;
    if (nwork > 0x7fffff00ull) return hipErrorInvalidValue;
    const uint32_t grid = static_cast<uint32_t>((nwork + 7) / 8 * 8);
    ApplyArgs a{h.in, h.in_ld, h.out, h.out_ld, h.s, h.prog, h.ngroups,
                static_cast<uint32_t>(nwork), grid / 8u, 0u};
    hipLaunchKernelGGL((pm_apply_kernel<RG, VEC>), dim3(grid), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

extern "C" int pmk_tile_bytes(int vec) { return kThreads * 4 * vec; }

extern "C" hipError_t pmk_apply(int rg, int vec, const PmkApply *h, hipStream_t st) {
    switch (rg * 10 + vec) {
        case 42: return launch_apply<4, 2>(*h, st);
        case 44: return launch_apply<4, 4>(*h, st);
        case 82: return launch_apply<8, 2>(*h, st);
        case 84: return launch_apply<8, 4>(*h, st);
        case 162: return launch_apply<16, 2>(*h, st);
        case 164: return launch_apply<16, 4>(*h, st);
        default: return hipErrorInvalidValue;
    }
}
