// GF(2^8) region matrix kernels for gfx950 (CDNA4).
//
// out[r][p] = XOR_c A[r][c] * in[c][p] for every byte p of the regions: the
// data phase of encode (Y = G X), repair and decode (Section 2 of the paper).
// The paper multiplies a region by a constant with SIMD split tables
// (Section 4).  Here every lane owns 8 or 16 contiguous bytes of a byte tile,
// splits each source byte into 3 + 3 + 2 bit fields once, and looks the three
// partial products up with v_perm_b32 (an 8-entry byte table per selector
// byte).  Partial products are folded into per-row register accumulators
// three at a time with v_bitop3_b32.  A work unit is one (byte tile, row
// group) pair; the row group's coefficient tables are wave-uniform.
//
// Two table paths:
//  - scalar: tables come in through the scalar cache (s_load); one half of
//    each byte-permute table must then be copied into a VGPR.
//  - LDS: the work-group stages the group's tables in LDS once per unit and
//    every wave reads them as VGPRs; no scalar-cache misses, no copies.
#include <hip/hip_runtime.h>

#include "put.hpp"

#include <map>
#include <mutex>
#include <utility>
#include <stdint.h>

namespace {

constexpr int kGroupWords = 8;
constexpr int kHeaderWords = 4;
constexpr int kWaves = 4;          // waves per work-group
constexpr int kThreads = 64 * kWaves;
constexpr uint32_t kLdsSlots = 2048;   // table slots staged at once (40 KiB)

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
    uint32_t lds_slots;    // LDS path: slots staged per chunk
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// Kernel programs are read-only for the whole launch: reading them through
// the constant address space keeps wave-uniform loads on the scalar unit
// (s_load) even though the kernel also stores to global memory.
typedef const __attribute__((address_space(4))) uint32_t *cptr;

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

template <int VEC>
struct Fields {
    uint32_t a[VEC], b[VEC], c[VEC];
};

template <int VEC>
__device__ __forceinline__ void split(const uint32_t (&x)[VEC], Fields<VEC> &f) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        f.a[v] = x[v] & 0x07070707u;          // bits 0..2 of every byte
        f.b[v] = (x[v] >> 3) & 0x07070707u;   // bits 3..5
        f.c[v] = (x[v] >> 6) & 0x03030303u;   // bits 6..7
    }
}

// acc ^= c0 * x0 ^ c1 * x1 for one row: table words {lo3 0..3, lo3 4..7,
// mid3 0..3, mid3 4..7, top2 0..3} of the pair's two coefficients.
template <int VEC>
__device__ __forceinline__ void row_pair(uint32_t (&acc)[VEC], const Fields<VEC> &f0, const Fields<VEC> &f1,
                                         uint32_t p0, uint32_t p1, uint32_t p2, uint32_t p3, uint32_t p4,
                                         uint32_t q0, uint32_t q1, uint32_t q2, uint32_t q3, uint32_t q4) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        const uint32_t l0 = perm(p1, p0, f0.a[v]);
        const uint32_t m0 = perm(p3, p2, f0.b[v]);
        const uint32_t h0 = perm(p4, p4, f0.c[v]);
        const uint32_t l1 = perm(q1, q0, f1.a[v]);
        const uint32_t m1 = perm(q3, q2, f1.b[v]);
        const uint32_t h1 = perm(q4, q4, f1.c[v]);
        acc[v] = xor3(xor3(xor3(acc[v], l0, m0), h0, l1), m1, h1);
    }
}

template <int VEC, bool FULL>
__device__ __forceinline__ void load_pair(const uint8_t *inb, cptr cols, uint32_t ci, uint64_t in_ld,
                                          uint32_t avail, uint32_t (&x0)[VEC], uint32_t (&x1)[VEC]) {
    load_chunk<VEC, FULL>(inb + static_cast<uint64_t>(cols[ci]) * in_ld, avail, x0);
    load_chunk<VEC, FULL>(inb + static_cast<uint64_t>(cols[ci + 1]) * in_ld, avail, x1);
}

// Where the coefficient tables of the current pair come from.
struct ScalarTables {
    cptr t4, t1;   // group's 4-word and 1-word table parts
    template <int RG, int VEC>
    __device__ __forceinline__ void pair(uint32_t (&acc)[RG][VEC], const Fields<VEC> &f0, const Fields<VEC> &f1,
                                         uint32_t ci) const {
        cptr a4 = t4 + ci * RG * 4, b4 = a4 + RG * 4;
        cptr a1 = t1 + ci * RG, b1 = a1 + RG;
#pragma unroll
        for (int r = 0; r < RG; ++r)
            row_pair<VEC>(acc[r], f0, f1, a4[4 * r], a4[4 * r + 1], a4[4 * r + 2], a4[4 * r + 3], a1[r],
                          b4[4 * r], b4[4 * r + 1], b4[4 * r + 2], b4[4 * r + 3], b1[r]);
    }
};

struct LdsTables {
    const u32x4 *t4;       // staged 4-word parts, slot = column * RG + row
    const uint32_t *t1;    // staged 1-word parts
    uint32_t c0;           // first column of the staged chunk
    template <int RG, int VEC>
    __device__ __forceinline__ void pair(uint32_t (&acc)[RG][VEC], const Fields<VEC> &f0, const Fields<VEC> &f1,
                                         uint32_t ci) const {
        const uint32_t base = (ci - c0) * RG;
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            const u32x4 p = t4[base + r], q = t4[base + RG + r];
            row_pair<VEC>(acc[r], f0, f1, p.x, p.y, p.z, p.w, t1[base + r], q.x, q.y, q.z, q.w,
                          t1[base + RG + r]);
        }
    }
};

// Columns [cb, ce) of a row group for one lane, one pair prefetched ahead.
template <int RG, int VEC, bool FULL, class Tabs>
__device__ __forceinline__ void run_columns(uint32_t (&acc)[RG][VEC], const Tabs &tabs, cptr cols, uint32_t cb,
                                            uint32_t ce, const uint8_t *inb, uint64_t in_ld, uint32_t avail) {
    uint32_t x0[VEC], x1[VEC], n0[VEC], n1[VEC];
    if (cb < ce) load_pair<VEC, FULL>(inb, cols, cb, in_ld, avail, n0, n1);
    for (uint32_t ci = cb; ci < ce; ci += 2) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) { x0[v] = n0[v]; x1[v] = n1[v]; }
        if (ci + 2 < ce) load_pair<VEC, FULL>(inb, cols, ci + 2, in_ld, avail, n0, n1);
        Fields<VEC> f0, f1;
        split<VEC>(x0, f0);
        split<VEC>(x1, f1);
        tabs.template pair<RG, VEC>(acc, f0, f1, ci);
    }
}

template <int RG, int VEC, bool FULL>
__device__ __forceinline__ void store_rows(const uint32_t (&acc)[RG][VEC], cptr rows, uint32_t nrows,
                                           uint8_t *out, uint64_t out_ld, uint64_t off, uint32_t avail) {
#pragma unroll
    for (int r = 0; r < RG; ++r)
        if (static_cast<uint32_t>(r) < nrows)
            store_chunk<VEC, FULL>(out + static_cast<uint64_t>(rows[r]) * out_ld + off, avail, acc[r]);
}

template <int VEC, bool FULL>
__device__ __forceinline__ void copy_rows(cptr cols, cptr rows, uint32_t nrows, const uint8_t *in, uint64_t in_ld,
                                          uint8_t *out, uint64_t out_ld, uint64_t off, uint32_t avail) {
    for (uint32_t r = 0; r < nrows; ++r) {
        uint32_t x[VEC];
        load_chunk<VEC, FULL>(in + static_cast<uint64_t>(cols[r]) * in_ld + off, avail, x);
        store_chunk<VEC, FULL>(out + static_cast<uint64_t>(rows[r]) * out_ld + off, avail, x);
    }
}

// Lane geometry of a unit: each wave owns 64 * 4 * VEC contiguous bytes.
template <int VEC>
struct Lane {
    uint64_t off;
    uint32_t avail;
    bool active, full;
    __device__ __forceinline__ Lane(uint64_t tile_off, uint64_t s) {
        constexpr uint32_t kLaneBytes = 4 * VEC;
        constexpr uint32_t kWaveBytes = 64 * kLaneBytes;
        const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
        const uint64_t wave_off = tile_off + static_cast<uint64_t>(wave) * kWaveBytes;
        active = wave_off < s;                  // wave-uniform
        full = wave_off + kWaveBytes <= s;      // wave-uniform
        off = wave_off + static_cast<uint64_t>(threadIdx.x % 64) * kLaneBytes;
        avail = off < s ? static_cast<uint32_t>(s - off < kLaneBytes ? s - off : kLaneBytes) : 0u;
    }
};

// Units of this work-group: the (tile, group) units are cut into 8 contiguous
// ranges, one per XCD (work-groups are dealt to XCDs round-robin), and the
// work-groups of an XCD stride through their range, so all row groups of a
// tile run side by side in one L2, where re-reads of shared columns hit.
struct UnitRange {
    uint32_t u, end, step;
    __device__ __forceinline__ UnitRange(uint32_t nwork, uint32_t per_xcd) {
        const uint32_t xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;
        const uint32_t per = (nwork + 7u) / 8u;
        const uint32_t u0 = xcd * per;
        end = u0 + per < nwork ? u0 + per : nwork;
        u = u0 + slot;
        step = per_xcd;
    }
};

// ---- scalar-table kernel ---------------------------------------------------
template <int RG, int VEC>
__global__ __launch_bounds__(kThreads) void pm_apply_scalar(ApplyArgs a) {
    constexpr uint64_t kTile = static_cast<uint64_t>(kThreads) * 4 * VEC;
    const cptr prog = (cptr)(a.prog);
    for (UnitRange ur(a.nwork, a.per_xcd); ur.u < ur.end; ur.u += ur.step) {
        const uint32_t tile = ur.u / a.ngroups;
        const uint32_t grp = ur.u - tile * a.ngroups;
        const Lane<VEC> ln(tile * kTile, a.s);
        if (!ln.active) continue;
        const cptr g = prog + kHeaderWords + grp * kGroupWords;
        const cptr cols = prog + g[3], rows = prog + g[5];
        if (g[0] == 0) {
            const ScalarTables tabs{prog + g[4], prog + g[6]};
            uint32_t acc[RG][VEC] = {};
            if (ln.full) {
                run_columns<RG, VEC, true>(acc, tabs, cols, 0, g[2], a.in + ln.off, a.in_ld, 4 * VEC);
                store_rows<RG, VEC, true>(acc, rows, g[1], a.out, a.out_ld, ln.off, 4 * VEC);
            } else {
                run_columns<RG, VEC, false>(acc, tabs, cols, 0, g[2], a.in + ln.off, a.in_ld, ln.avail);
                store_rows<RG, VEC, false>(acc, rows, g[1], a.out, a.out_ld, ln.off, ln.avail);
            }
        } else if (ln.full) {
            copy_rows<VEC, true>(cols, rows, g[1], a.in, a.in_ld, a.out, a.out_ld, ln.off, 4 * VEC);
        } else {
            copy_rows<VEC, false>(cols, rows, g[1], a.in, a.in_ld, a.out, a.out_ld, ln.off, ln.avail);
        }
    }
}

// ---- software-pipelined kernel ----------------------------------------------
// For row groups of at most MAXC columns: while a wave multiplies one unit,
// the loads of every column of its next unit are already in flight (two
// register buffers, used alternately), so each wave keeps MAXC * 64 * 4 * VEC
// bytes of loads outstanding instead of one column pair.  The loads of a
// unit are issued unconditionally (columns past the group's end re-read its
// first column) so the compiler can wait on exactly the older unit's loads.
// Units that do not fit (partial tiles, copy groups, wider groups) take the
// plain path.
template <int RG, int VEC, int MAXC>
struct Pipe {
    static constexpr uint64_t kTile = static_cast<uint64_t>(kThreads) * 4 * VEC;

    // Issue all loads of unit u into x when it can take the fast path.
    static __device__ __forceinline__ bool prefetch(const ApplyArgs &a, cptr prog, uint32_t u,
                                                    uint32_t (&x)[MAXC][VEC]) {
        const uint32_t tile = u / a.ngroups;
        const uint32_t grp = u - tile * a.ngroups;
        const Lane<VEC> ln(tile * kTile, a.s);
        const cptr g = prog + kHeaderWords + grp * kGroupWords;
        const uint32_t ncols = g[2];
        if (!ln.full || g[0] != 0 || ncols > MAXC) return false;
        const cptr cols = prog + g[3];
        const uint8_t *inb = a.in + ln.off;
        // One scalar fetch of MAXC column ids (the program pads the id list),
        // then branch-free selects: every load issues back to back.
        uint32_t cw[MAXC];
#pragma unroll
        for (int c = 0; c < MAXC; ++c) cw[c] = cols[c];
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const uint32_t col = static_cast<uint32_t>(c) < ncols ? cw[c] : cw[0];
            load_chunk<VEC, true>(inb + static_cast<uint64_t>(col) * a.in_ld, 4 * VEC, x[c]);
        }
        return true;
    }

    static __device__ __forceinline__ void compute(const ApplyArgs &a, cptr prog, uint32_t u,
                                                   const uint32_t (&x)[MAXC][VEC]) {
        const uint32_t tile = u / a.ngroups;
        const uint32_t grp = u - tile * a.ngroups;
        const Lane<VEC> ln(tile * kTile, a.s);
        const cptr g = prog + kHeaderWords + grp * kGroupWords;
        const uint32_t ncols = g[2];
        const ScalarTables tabs{prog + g[4], prog + g[6]};
        uint32_t acc[RG][VEC] = {};
#pragma unroll
        for (int c = 0; c < MAXC; c += 2) {
            if (static_cast<uint32_t>(c) < ncols) {
                Fields<VEC> f0, f1;
                split<VEC>(x[c], f0);
                split<VEC>(x[c + 1], f1);
                tabs.template pair<RG, VEC>(acc, f0, f1, static_cast<uint32_t>(c));
            }
        }
        store_rows<RG, VEC, true>(acc, prog + g[5], g[1], a.out, a.out_ld, ln.off, 4 * VEC);
    }

    // The plain path for a unit that cannot be pipelined.
    static __device__ __forceinline__ void plain(const ApplyArgs &a, cptr prog, uint32_t u) {
        const uint32_t tile = u / a.ngroups;
        const uint32_t grp = u - tile * a.ngroups;
        const Lane<VEC> ln(tile * kTile, a.s);
        if (!ln.active) return;
        const cptr g = prog + kHeaderWords + grp * kGroupWords;
        const cptr cols = prog + g[3], rows = prog + g[5];
        if (g[0] == 0) {
            const ScalarTables tabs{prog + g[4], prog + g[6]};
            uint32_t acc[RG][VEC] = {};
            if (ln.full) {
                run_columns<RG, VEC, true>(acc, tabs, cols, 0, g[2], a.in + ln.off, a.in_ld, 4 * VEC);
                store_rows<RG, VEC, true>(acc, rows, g[1], a.out, a.out_ld, ln.off, 4 * VEC);
            } else {
                run_columns<RG, VEC, false>(acc, tabs, cols, 0, g[2], a.in + ln.off, a.in_ld, ln.avail);
                store_rows<RG, VEC, false>(acc, rows, g[1], a.out, a.out_ld, ln.off, ln.avail);
            }
        } else if (ln.full) {
            copy_rows<VEC, true>(cols, rows, g[1], a.in, a.in_ld, a.out, a.out_ld, ln.off, 4 * VEC);
        } else {
            copy_rows<VEC, false>(cols, rows, g[1], a.in, a.in_ld, a.out, a.out_ld, ln.off, ln.avail);
        }
    }
};

template <int RG, int VEC, int MAXC>
__global__ __launch_bounds__(kThreads) void pm_apply_pipe(ApplyArgs a) {
    using P = Pipe<RG, VEC, MAXC>;
    const cptr prog = (cptr)(a.prog);
    const UnitRange ur(a.nwork, a.per_xcd);
    uint32_t xa[MAXC][VEC], xb[MAXC][VEC];
    uint32_t u = ur.u;
    if (u >= ur.end) return;
    bool fa = P::prefetch(a, prog, u, xa), fb = false;
    while (true) {
        const uint32_t u2 = u + ur.step;
        fb = u2 < ur.end && P::prefetch(a, prog, u2, xb);
        if (fa) P::compute(a, prog, u, xa);
        else P::plain(a, prog, u);
        u = u2;
        if (u >= ur.end) break;
        const uint32_t u3 = u + ur.step;
        fa = u3 < ur.end && P::prefetch(a, prog, u3, xa);
        if (fb) P::compute(a, prog, u, xb);
        else P::plain(a, prog, u);
        u = u3;
        if (u >= ur.end) break;
    }
}

// ---- LDS-table kernel --------------------------------------------------------
// Every wave of the work-group reaches every barrier: waves past the block
// end skip only their loads, arithmetic and stores, and the unit sequence and
// all barrier conditions are uniform across the work-group.
template <int RG, int VEC>
__global__ __launch_bounds__(kThreads) void pm_apply_lds(ApplyArgs a) {
    constexpr uint64_t kTile = static_cast<uint64_t>(kThreads) * 4 * VEC;
    __shared__ u32x4 s4[kLdsSlots];
    __shared__ uint32_t s1[kLdsSlots];
    const cptr prog = (cptr)(a.prog);
    const uint32_t chunk_cols = (kLdsSlots / RG) & ~1u;   // even
    uint32_t staged_grp = 0xffffffffu, staged_c0 = 0;
    for (UnitRange ur(a.nwork, a.per_xcd); ur.u < ur.end; ur.u += ur.step) {
        const uint32_t tile = ur.u / a.ngroups;
        const uint32_t grp = ur.u - tile * a.ngroups;
        const Lane<VEC> ln(tile * kTile, a.s);
        const cptr g = prog + kHeaderWords + grp * kGroupWords;
        const cptr cols = prog + g[3], rows = prog + g[5];
        const uint32_t ncols = g[2];
        if (g[0] != 0) {
            if (ln.active) {
                if (ln.full) copy_rows<VEC, true>(cols, rows, g[1], a.in, a.in_ld, a.out, a.out_ld, ln.off, 4 * VEC);
                else copy_rows<VEC, false>(cols, rows, g[1], a.in, a.in_ld, a.out, a.out_ld, ln.off, ln.avail);
            }
            continue;
        }
        uint32_t acc[RG][VEC] = {};
        for (uint32_t c0 = 0; c0 < ncols; c0 += chunk_cols) {
            const uint32_t c1 = c0 + chunk_cols < ncols ? c0 + chunk_cols : ncols;
            if (grp != staged_grp || c0 != staged_c0) {
                __syncthreads();   // every wave is done with the previous tables
                const uint32_t nslot = (c1 - c0) * RG;
                const uint32_t *g4 = (const uint32_t *)(prog + g[4]) + c0 * RG * 4;
                const uint32_t *g1 = (const uint32_t *)(prog + g[6]) + c0 * RG;
                for (uint32_t i = threadIdx.x; i < nslot; i += kThreads) {
                    s4[i] = *reinterpret_cast<const u32x4 *>(g4 + 4 * i);
                    s1[i] = g1[i];
                }
                __syncthreads();
                staged_grp = grp;
                staged_c0 = c0;
            }
            if (ln.active) {
                const LdsTables tabs{s4, s1, c0};
                if (ln.full) run_columns<RG, VEC, true>(acc, tabs, cols, c0, c1, a.in + ln.off, a.in_ld, 4 * VEC);
                else run_columns<RG, VEC, false>(acc, tabs, cols, c0, c1, a.in + ln.off, a.in_ld, ln.avail);
            }
        }
        if (ln.active) {
            if (ln.full) store_rows<RG, VEC, true>(acc, rows, g[1], a.out, a.out_ld, ln.off, 4 * VEC);
            else store_rows<RG, VEC, false>(acc, rows, g[1], a.out, a.out_ld, ln.off, ln.avail);
        }
    }
}

// ---- batched work-list kernel ---------------------------------------------
// Many independent region products (objects of different sizes and codes,
// encode / repair / decode mixed) in one persistent launch.  Every wave is a
// worker: it takes the next unit -- (item, row group, wave tile) -- from its
// XCD's queue with one atomic add, and when that queue is empty it steals
// from the other seven.  Units are numbered item by item, tile by tile, group
// by group, so the row groups of a tile are taken back to back inside one
// XCD and share its L2.  Items are ordered by their first unit; a wave finds
// its item by binary search, starting from the item it worked on last.
struct BatchItem {
    const uint32_t *prog;
    const uint8_t *in;
    uint8_t *out;
    uint64_t in_ld, out_ld, s;
    uint32_t ngroups, ntiles;   // ntiles counts wave tiles
    uint32_t unit0, pad;
};

struct BatchArgs {
    const BatchItem *items;
    uint32_t nitems, nunits;
    uint32_t *counters;   // 8 queue heads, 64 bytes apart, and the finished-wave count
};

constexpr uint32_t kCounterStride = 16;
constexpr uint32_t kDoneWord = 8;   // waves of the launch that have left the queues

template <int RG, int VEC>
__global__ __launch_bounds__(kThreads) void pm_batch_kernel(BatchArgs a) {
    constexpr uint32_t kLaneBytes = 4 * VEC;
    constexpr uint32_t kWaveBytes = 64 * kLaneBytes;
    typedef const __attribute__((address_space(4))) BatchItem *citem;
    const citem items = (citem)(a.items);
    const uint32_t lane = threadIdx.x % 64;
    const uint32_t xcd = blockIdx.x % 8u;
    const uint32_t per = (a.nunits + 7u) / 8u;
    uint32_t cur = 0;   // item searched from
    for (uint32_t q = 0; q < 8u; ++q) {
        const uint32_t x = (xcd + q) % 8u;
        const uint32_t r0 = x * per;
        const uint32_t r1 = r0 + per < a.nunits ? r0 + per : a.nunits;
        if (r0 >= r1) continue;
        while (true) {
            uint32_t k = 0;
            if (lane == 0) k = atomicAdd(a.counters + x * kCounterStride, 1u);
            k = __builtin_amdgcn_readfirstlane(k);
            const uint32_t u = r0 + k;
            if (u >= r1) break;
            // item with unit0 <= u < next unit0
            if (!(items[cur].unit0 <= u && (cur + 1 == a.nitems || u < items[cur + 1].unit0))) {
                uint32_t lo = 0, hi = a.nitems;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) / 2;
                    if (items[mid].unit0 <= u) lo = mid;
                    else hi = mid;
                }
                cur = lo;
            }
            const citem it = items + cur;
            const uint32_t local = u - it->unit0;
            const uint32_t ng = it->ngroups;
            const uint32_t tile = local / ng;
            const uint32_t grp = local - tile * ng;
            const uint64_t s = it->s;
            const uint64_t wave_off = static_cast<uint64_t>(tile) * kWaveBytes;
            const bool full = wave_off + kWaveBytes <= s;
            const uint64_t off = wave_off + static_cast<uint64_t>(lane) * kLaneBytes;
            const uint32_t avail =
                off < s ? static_cast<uint32_t>(s - off < kLaneBytes ? s - off : kLaneBytes) : 0u;
            const cptr prog = (cptr)(it->prog);
            const cptr g = prog + kHeaderWords + grp * kGroupWords;
            const cptr cols = prog + g[3], rows = prog + g[5];
            const uint8_t *in = it->in;
            uint8_t *out = it->out;
            const uint64_t in_ld = it->in_ld, out_ld = it->out_ld;
            if (g[0] == 0) {
                const ScalarTables tabs{prog + g[4], prog + g[6]};
                uint32_t acc[RG][VEC] = {};
                if (full) {
                    run_columns<RG, VEC, true>(acc, tabs, cols, 0, g[2], in + off, in_ld, kLaneBytes);
                    store_rows<RG, VEC, true>(acc, rows, g[1], out, out_ld, off, kLaneBytes);
                } else {
                    run_columns<RG, VEC, false>(acc, tabs, cols, 0, g[2], in + off, in_ld, avail);
                    store_rows<RG, VEC, false>(acc, rows, g[1], out, out_ld, off, avail);
                }
            } else if (full) {
                copy_rows<VEC, true>(cols, rows, g[1], in, in_ld, out, out_ld, off, kLaneBytes);
            } else {
                copy_rows<VEC, false>(cols, rows, g[1], in, in_ld, out, out_ld, off, avail);
            }
        }
    }
    // The counters start every launch at zero: the last wave to leave the
    // queues resets them, so no reset launch precedes each batch kernel.
    // Every other wave's last queue-head update has returned (the loop
    // read its value) before that wave's own count is added.  No fence: an
    // agent-scope release would write back the XCD's L2 for every wave.
    if (lane == 0) {
        const uint32_t waves = gridDim.x * (blockDim.x / 64u);
        if (atomicAdd(a.counters + kDoneWord, 1u) == waves - 1u) {
            for (uint32_t x = 0; x < 8u; ++x) atomicExch(a.counters + x * kCounterStride, 0u);
            atomicExch(a.counters + kDoneWord, 0u);
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host-side launchers.
struct PmkApply {
    const uint8_t *in;
    uint64_t in_ld;
    uint8_t *out;
    uint64_t out_ld;
    uint64_t s;
    const uint32_t *prog;
    uint32_t ngroups;
};

// Resident work-groups per CU of one kernel, and the CU count, per device:
// measured once per (kernel, device) and kept under a lock (kernels of the
// same signature differ in occupancy, and launches come from user threads
// and the server's scheduler at once).
static std::mutex g_resident_mu;
static std::map<std::pair<const void *, int>, std::pair<int, int>> &g_resident =
    *new std::map<std::pair<const void *, int>, std::pair<int, int>>();

template <class K>
static uint32_t resident_groups(K kernel, int *ncu_out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const auto key = std::make_pair(reinterpret_cast<const void *>(kernel), dev);
    std::lock_guard<std::mutex> lk(g_resident_mu);
    auto it = g_resident.find(key);
    if (it == g_resident.end()) {
        int b = 0, n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, kThreads, 0) != hipSuccess || b < 1) b = 1;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        it = g_resident.emplace(key, std::make_pair(b, n)).first;
    }
    *ncu_out = it->second.second;
    return static_cast<uint32_t>(it->second.first);
}

template <int RG, int VEC, int KIND>   // KIND: 0 scalar, 1 LDS, 2 pipelined (<= 16 columns)
static hipError_t launch_apply(const PmkApply &h, hipStream_t st) {
    constexpr bool LDS = KIND == 1;
    constexpr uint64_t kTile = static_cast<uint64_t>(kThreads) * 4 * VEC;
    const uint64_t ntiles = (h.s + kTile - 1) / kTile;
    const uint64_t nwork = ntiles * h.ngroups;
    if (nwork == 0) return hipSuccess;
    if (nwork > 0x7fffff00ull) return hipErrorInvalidValue;
    int ncu = 0;
    uint32_t per_cu;
    if constexpr (KIND == 1) per_cu = resident_groups(pm_apply_lds<RG, VEC>, &ncu);
    else if constexpr (KIND == 2) per_cu = resident_groups(pm_apply_pipe<RG, VEC, 16>, &ncu);
    else per_cu = resident_groups(pm_apply_scalar<RG, VEC>, &ncu);
    const uint64_t resident = static_cast<uint64_t>(per_cu) * static_cast<uint64_t>(ncu);
    uint64_t grid = nwork < resident ? nwork : resident;
    grid = (grid + 7) / 8 * 8;
    ApplyArgs a{h.in, h.in_ld, h.out, h.out_ld, h.s, h.prog, h.ngroups,
                static_cast<uint32_t>(nwork), static_cast<uint32_t>(grid / 8u), kLdsSlots};
    if constexpr (KIND == 1)
        hipLaunchKernelGGL((pm_apply_lds<RG, VEC>), dim3(static_cast<uint32_t>(grid)), dim3(kThreads), 0, st, a);
    else if constexpr (KIND == 2)
        hipLaunchKernelGGL((pm_apply_pipe<RG, VEC, 16>), dim3(static_cast<uint32_t>(grid)), dim3(kThreads), 0, st,
                           a);
    else
        hipLaunchKernelGGL((pm_apply_scalar<RG, VEC>), dim3(static_cast<uint32_t>(grid)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

struct PmkBatch {
    const void *items;     // device BatchItem array
    uint32_t nitems, nunits;
    uint32_t *counters;    // device, 8 * 16 words, zero before the first launch on them (each
                           // launch leaves them at zero)
};

extern "C" int pmk_batch_item_bytes() { return static_cast<int>(sizeof(BatchItem)); }
extern "C" int pmk_wave_bytes(int vec) { return 64 * 4 * vec; }

template <int RG, int VEC>
static hipError_t launch_batch(const PmkBatch &h, hipStream_t st) {
    if (h.nunits == 0) return hipSuccess;
    int ncu = 0;
    const uint32_t per_cu = resident_groups(pm_batch_kernel<RG, VEC>, &ncu);
    const uint64_t waves = (static_cast<uint64_t>(h.nunits) + kWaves - 1) / kWaves;
    const uint64_t resident = static_cast<uint64_t>(per_cu) * static_cast<uint64_t>(ncu);
    uint64_t grid = waves < resident ? waves : resident;
    grid = (grid + 7) / 8 * 8;
    BatchArgs a{static_cast<const BatchItem *>(h.items), h.nitems, h.nunits, h.counters};
    hipLaunchKernelGGL((pm_batch_kernel<RG, VEC>), dim3(static_cast<uint32_t>(grid)), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

// Batch launch for items whose programs all have rg rows per group; vec is
// the dwords per lane (2 or 4).
extern "C" hipError_t pmk_batch(int rg, int vec, const PmkBatch *h, hipStream_t st) {
    switch (rg * 100 + vec) {
        case 402: return launch_batch<4, 2>(*h, st);
        case 404: return launch_batch<4, 4>(*h, st);
        case 802: return launch_batch<8, 2>(*h, st);
        case 804: return launch_batch<8, 4>(*h, st);
        case 1602: return launch_batch<16, 2>(*h, st);
        case 1604: return launch_batch<16, 4>(*h, st);
        default: return hipErrorInvalidValue;
    }
}

extern "C" int pmk_tile_bytes(int vec) { return kThreads * 4 * (vec % 10); }

// vec: dwords per lane (2 or 4) with scalar tables; 12 or 14 for the same
// widths with LDS-staged tables; 22 or 24 for the software-pipelined kernel.
extern "C" hipError_t pmk_apply(int rg, int vec, const PmkApply *h, hipStream_t st) {
    switch (rg * 100 + vec) {
        case 402: return launch_apply<4, 2, 0>(*h, st);
        case 404: return launch_apply<4, 4, 0>(*h, st);
        case 802: return launch_apply<8, 2, 0>(*h, st);
        case 804: return launch_apply<8, 4, 0>(*h, st);
        case 1602: return launch_apply<16, 2, 0>(*h, st);
        case 1604: return launch_apply<16, 4, 0>(*h, st);
        case 412: return launch_apply<4, 2, 1>(*h, st);
        case 414: return launch_apply<4, 4, 1>(*h, st);
        case 812: return launch_apply<8, 2, 1>(*h, st);
        case 814: return launch_apply<8, 4, 1>(*h, st);
        case 1612: return launch_apply<16, 2, 1>(*h, st);
        case 1614: return launch_apply<16, 4, 1>(*h, st);
        case 422: return launch_apply<4, 2, 2>(*h, st);
        case 424: return launch_apply<4, 4, 2>(*h, st);
        case 822: return launch_apply<8, 2, 2>(*h, st);
        case 824: return launch_apply<8, 4, 2>(*h, st);
        case 1622: return launch_apply<16, 2, 2>(*h, st);
        case 1624: return launch_apply<16, 4, 2>(*h, st);
        default: return hipErrorInvalidValue;
    }
}

// Small device writes as a kernel: the words travel in the kernel arguments
// (copied at launch, also under graph capture), so a launch list can be
// placed in a caller's workspace in stream order with no host staging.
struct PutArgs {
    uint32_t *dst;
    uint32_t n, pad;
    uint32_t w[kPutWords];
};

extern "C" __global__ __launch_bounds__(256) void pm_put_words(PutArgs a) {
    for (uint32_t i = threadIdx.x; i < a.n; i += 256u) a.dst[i] = a.w[i];
}

extern "C" hipError_t pmk_put(uint32_t *dst, const uint32_t *words, uint32_t n, hipStream_t st) {
    if (n > kPutWords) return hipErrorInvalidValue;
    PutArgs a{dst, n, 0, {}};
    for (uint32_t i = 0; i < n; ++i) a.w[i] = words[i];
    hipLaunchKernelGGL(pm_put_words, dim3(1), dim3(256), 0, st, a);
    return hipGetLastError();
}
