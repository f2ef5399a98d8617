// Dense GF(2^8) region products on the matrix cores (gfx950).
//
// Multiplying by a constant is linear over GF(2) (Section 4.1's note on
// bit matrices): with the input bytes of 8 blocks at one position as 64
// bits, the 64 x 32 block of the GF(2) expansion of the matrix (see
// mfma.hpp) maps them to 32 output bits, and over all chunks of 8 input
// blocks an output bit is the parity of a count of products of set bits.
// v_mfma_scale_f32_32x32x64_f8f6f4 with 4-bit float operands computes those
// counts exactly: every product of two set bits is 1.0 (the operand values
// are in mfma.cpp).  Accumulator register i of a lane holds bit b = i % 8
// of an output byte, and starts at 2^(23 - b): the ulp there is 2^-b, so
// after adding an integer count c the encoding's mantissa is c << b, and
// bit b of the encoding is the parity of c (counts stay below 2^13, far
// from changing the exponent).  So the output byte is the OR of the 8
// encodings each masked to its own bit: one operation per accumulator.
// The first chunk's instructions take those start values as their C
// operand, so no accumulator is initialized separately.
//
// Work: a work-group of 8 waves (one per CU, two waves per SIMD) holds T M
// tiles (4 T output rows).  It first copies their A operands for every K
// chunk (T KiB per chunk, from the precomputed expansion) and the chunks'
// input block offsets into LDS; then each wave takes position blocks of
// 32 U bytes, the 8 waves on adjacent blocks, pq of them each, so that the
// grid is a single round of work-groups.  A position block is U sub-tiles
// of 32 positions: sub-tile u holds positions U n + u, so one U-byte load
// per lane and input block serves all of them, and one U-byte store per
// lane and output row writes them back.  Per chunk a lane loads 4 U-byte
// words (its K half's 4 blocks), gathers them into U dwords of one byte per
// block with byte permutes, masks each into the 4 operand dwords of its
// sub-tile and issues T U matrix instructions.  T = 4, U = 2 while the
// operands of 4 tiles fit in LDS (up to 39 chunks): every gathered and
// masked operand then serves 4 instructions.  Beyond that T = 2, U = 4.
// Input loads run kDepth chunks ahead, LDS reads of the A operands one
// chunk.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "mfma.hpp"

namespace {

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr uint32_t kWaves = 8;
constexpr uint32_t kDepth = 4;   // chunks of input loads in flight
constexpr uint32_t kLdsMax = 160u * 1024u;

// LDS of a work-group: the input block offsets of every chunk (block id x
// in_ld, 32-bit: the launch requires every input byte within 4 GiB of in;
// 8 per chunk, kMfMaxChunks chunks), then the A operands, [chunk][tile]
// [lane] 16 bytes each, for one chunk more than the matrix has.
constexpr uint32_t kOffsBytes = kMfMaxChunks * kMfColsPerChunk * 4u;
extern __shared__ uint4 pm_mf_lds[];

template <uint32_t U>
struct Word;
template <>
struct Word<2> { typedef uint16_t type; };
template <>
struct Word<4> { typedef uint32_t type; };

// U bytes at p[off ..]; bytes at or past rem read as zero.
template <uint32_t U, bool TAIL>
__device__ __forceinline__ uint32_t loadU(const uint8_t *p, uint32_t off, uint64_t rem) {
    typedef typename Word<U>::type W;
    if (!TAIL || off + U <= rem) return *reinterpret_cast<const W *>(p + off);
    uint32_t w = 0u;
    for (uint32_t b = 0; b < U; ++b)
        if (off + b < rem) w |= static_cast<uint32_t>(p[off + b]) << (8u * b);
    return w;
}

template <uint32_t U, bool TAIL>
__device__ __forceinline__ void storeU(uint8_t *p, uint32_t off, uint64_t rem, uint32_t w) {
    typedef typename Word<U>::type W;
    if (!TAIL || off + U <= rem) {
        __builtin_nontemporal_store(static_cast<W>(w), reinterpret_cast<W *>(p + off));
        return;
    }
    for (uint32_t b = 0; b < U; ++b)
        if (off + b < rem) p[off + b] = static_cast<uint8_t>(w >> (8u * b));
}

// The output byte of accumulators base .. base + 7 (register i holds bit
// i - base at that bit of its encoding).
__device__ __forceinline__ uint32_t pack8(const v16f &a, int base) {
    uint32_t b = 0u;
#pragma unroll
    for (int i = 0; i < 8; ++i) b |= __float_as_uint(a[base + i]) & (1u << i);
    return b;
}

// The lane's 4 input words of chunk kc at position block base: blocks
// 4 kb .. 4 kb + 3 of the chunk, whose offsets (block id x in_ld) the
// work-group keeps in LDS.  p = in + base, the same for the whole wave, so
// an address is p plus a 32-bit lane offset.
template <uint32_t U, bool TAIL>
__device__ __forceinline__ void load_chunk(const uint32_t *offs, uint32_t kc, const uint8_t *p, uint32_t off,
                                           uint32_t kb, uint64_t rem, uint32_t (&w)[4]) {
    typedef typename Word<U>::type W;
    const uint4 o = *reinterpret_cast<const uint4 *>(offs + kc * kMfColsPerChunk + 4u * kb);
    const uint32_t oj[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
        w[j] = TAIL ? loadU<U, true>(p + oj[j], off, rem) : *reinterpret_cast<const W *>(p + (oj[j] + off));
}

// One position block: the work-group's T M tiles over the 32 U positions
// from base.  TAIL: the block ends inside them, so loads and stores check
// each byte.
template <uint32_t T, uint32_t U, bool TAIL>
__device__ __forceinline__ void run_block(const PmkMfma &a, const uint32_t *offs, const uint4 *abits, uint32_t mt0,
                                          uint64_t base, uint32_t lane) {
    const uint32_t kb = lane / 32u, off = U * (lane % 32u);
    const bool hi = kb != 0u;
    const uint32_t nc = a.nchunks, last = nc - 1u;
    const uint8_t *pin = a.in + base;
    const uint64_t rem = a.s - base;
    v16f start;
#pragma unroll
    for (int i = 0; i < 16; ++i) start[i] = __uint_as_float(static_cast<uint32_t>(150 - i % 8) << 23);   // 2^(23 - i % 8)
    v16f acc[T][U];

    uint32_t w[kDepth][4];
#pragma unroll
    for (uint32_t d = 0; d < kDepth; ++d)
        load_chunk<U, TAIL>(offs, d < last ? d : last, pin, off, kb, rem, w[d]);
    // A operands, double-buffered by chunk parity
    uint4 abuf[2][T];
#pragma unroll
    for (uint32_t t = 0; t < T; ++t) abuf[0][t] = abits[t * 64u + lane];

    // one chunk kc from slot wd: gather and mask the input bits, refill the
    // slot with chunk kc + kDepth (past the last chunk the last one is read
    // again, in bounds and unused), read the next chunk's A operands and
    // multiply (the first chunk from the start values)
    auto step = [&](uint32_t kc, uint32_t(&wd)[4], uint4(&acur)[T], uint4(&anext)[T], bool first) {
        uint32_t D[U];   // D_u: byte j = byte u of wd[j] (the 4 blocks at position base + off + u)
        const uint32_t e01 = __builtin_amdgcn_perm(wd[1], wd[0], 0x05010400u);   // w0.0 w1.0 w0.1 w1.1
        const uint32_t e23 = __builtin_amdgcn_perm(wd[3], wd[2], 0x05010400u);
        D[0] = __builtin_amdgcn_perm(e23, e01, 0x05040100u);
        D[1] = __builtin_amdgcn_perm(e23, e01, 0x07060302u);
        if (U == 4) {
            const uint32_t f01 = __builtin_amdgcn_perm(wd[1], wd[0], 0x07030602u);   // w0.2 w1.2 w0.3 w1.3
            const uint32_t f23 = __builtin_amdgcn_perm(wd[3], wd[2], 0x07030602u);
            D[U > 2 ? 2 : 0] = __builtin_amdgcn_perm(f23, f01, 0x05040100u);
            D[U > 2 ? 3 : 1] = __builtin_amdgcn_perm(f23, f01, 0x07060302u);
        }
        const uint32_t nk = kc + kDepth;
        load_chunk<U, TAIL>(offs, nk < last ? nk : last, pin, off, kb, rem, wd);
        // the LDS holds one more chunk of A operands, so the read after the
        // last chunk stays in the allocation (and is unused)
#pragma unroll
        for (uint32_t t = 0; t < T; ++t) anext[t] = abits[((kc + 1u) * T + t) * 64u + lane];
        // keep the refill loads here: under register pressure the scheduler
        // sinks them to the end of the unrolled round, and the next round
        // then waits for all of them at its first chunk
        __builtin_amdgcn_sched_barrier(0);
        v8i B[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t D2 = D[u] >> 2;
            B[u][0] = static_cast<int>(D[u] & 0x11111111u);
            B[u][1] = static_cast<int>(D[u] & 0x22222222u);
            B[u][2] = static_cast<int>(D2 & 0x11111111u);
            B[u][3] = static_cast<int>(D2 & 0x22222222u);
#pragma unroll
            for (int q = 4; q < 8; ++q) B[u][q] = 0;
        }
#pragma unroll
        for (uint32_t t = 0; t < T; ++t) {
            const uint4 av = acur[t];
            const v8i A = {static_cast<int>(av.x), static_cast<int>(av.y), static_cast<int>(av.z),
                           static_cast<int>(av.w), 0, 0, 0, 0};
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                acc[t][u] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(A, B[u], first ? start : acc[t][u], 4, 4,
                                                                            0, 127, 0, 127);
        }
    };
    // chunk 0, then whole rounds of the kDepth slots from chunk 1 (no exit
    // inside a round, so the compiler's load waits stay exact across the
    // loop edge; chunk k sits in slot k % kDepth and A buffer k % 2), then
    // the rest
    step(0u, w[0], abuf[0], abuf[1], true);
    uint32_t k0 = 1;
    for (; k0 + kDepth <= nc; k0 += kDepth) {
#pragma unroll
        for (uint32_t d = 0; d < kDepth; ++d)
            step(k0 + d, w[(1 + d) % kDepth], abuf[(1 + d) % 2], abuf[d % 2], false);
    }
#pragma unroll
    for (uint32_t d = 0; d < kDepth - 1u; ++d)
        if (k0 + d < nc) step(k0 + d, w[(1 + d) % kDepth], abuf[(1 + d) % 2], abuf[d % 2], false);
    // accumulators 0..7 are bits 0..7 of output row 2 kb of the tile, 8..15
    // those of row 2 kb + 1; sub-tile u is byte u of the word
#pragma unroll
    for (uint32_t t = 0; t < T; ++t) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const uint32_t *rp = a.rows + (mt0 + t) * kMfRowsPerTile + half;
            const uint32_t row = hi ? rp[2] : rp[0];
            uint32_t v = 0u;
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) v |= pack8(acc[t][u], 8 * half) << (8u * u);
            if (row == kMfNoRow) continue;
            storeU<U, TAIL>(a.out + static_cast<uint64_t>(row) * a.out_ld + base, off, rem, v);
        }
    }
}

template <uint32_t T, uint32_t U>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(2, 2))) void pm_mfma(PmkMfma a) {
    const uint32_t lane = threadIdx.x % 64u, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
    // work-groups reach the XCDs round-robin: give each XCD a contiguous
    // range of logical indices, all M blocks of a few position groups, so
    // the blocks' input bytes are read into one L2 (the last nwg % 8
    // work-groups keep their own index, so the mapping is one to one)
    const uint32_t nwg = gridDim.x, per = nwg / 8u, b = blockIdx.x;
    const uint32_t wg = b < per * 8u ? (b % 8u) * per + b / 8u : b;
    const uint32_t mb = wg % a.nmblocks, pg = wg / a.nmblocks;
    // the input block offsets of every chunk, then the A operands of tiles
    // T mb .. T mb + T - 1 for every chunk (in abits [tile][chunk][lane],
    // in LDS [chunk][tile][lane], so that a chunk's T reads differ by
    // constant offsets)
    uint32_t *offs = reinterpret_cast<uint32_t *>(pm_mf_lds);
    uint4 *abits = pm_mf_lds + kOffsBytes / 16u;
    const uint32_t nc = a.nchunks;
    for (uint32_t i = threadIdx.x; i < nc * kMfColsPerChunk; i += 64u * kWaves)
        offs[i] = static_cast<uint32_t>(a.cols[i] * a.in_ld);
    const uint4 *src = reinterpret_cast<const uint4 *>(a.abits) + static_cast<uint64_t>(mb) * T * nc * 64u;
    for (uint32_t i = threadIdx.x; i < T * nc * 64u; i += 64u * kWaves) {
        const uint32_t l = i % 64u, kc = (i / 64u) % nc, t = i / (64u * nc);
        abits[(kc * T + t) * 64u + l] = src[i];
    }
    __syncthreads();
    const uint32_t p0 = pg * kWaves * a.pq;
    for (uint32_t j = 0; j < a.pq; ++j) {
        const uint32_t pb = p0 + j * kWaves + wave;
        if (pb >= a.npblocks) break;
        const uint64_t base = static_cast<uint64_t>(pb) * (32u * U);
        if (base + 32u * U <= a.s) run_block<T, U, false>(a, offs, abits, mb * T, base, lane);
        else run_block<T, U, true>(a, offs, abits, mb * T, base, lane);
    }
}

// Launch plan for h (its first 10 fields set) on a device of ncu compute
// units: the tiles per work-group T (4 when their operands fit in LDS, else
// 2; U = 8 / T), and in h the M blocks, position blocks (32 U bytes) and
// position blocks per wave; nwg work-groups of lds bytes of LDS each.  One
// work-group fits per CU (its LDS), so the position blocks are split into
// as many groups as leave every M block one work-group per group and the
// grid a single round.  False for a shape the kernel does not take.
bool mf_plan(PmkMfma &h, uint32_t ncu, uint32_t &T, uint32_t &nwg, size_t &lds) {
    if (h.nchunks == 0 || h.nchunks > kMfMaxChunks || h.nmtiles == 0 || h.nmtiles % kMfTilePad != 0 || ncu == 0)
        return false;
    T = kOffsBytes + 4u * (h.nchunks + 1u) * 1024u <= kLdsMax ? 4u : 2u;
    const uint32_t U = 8u / T;
    const uint64_t npb = (h.s + 32u * U - 1) / (32u * U);
    if (npb == 0 || npb > 0xFFFFFFFFull) return false;
    h.nmblocks = h.nmtiles / T;
    h.npblocks = static_cast<uint32_t>(npb);
    const uint64_t groups = ncu >= h.nmblocks ? ncu / h.nmblocks : 1u;
    const uint64_t pq = (npb + kWaves * groups - 1) / (kWaves * groups);
    h.pq = static_cast<uint32_t>(pq);
    const uint64_t npg = (npb + kWaves * pq - 1) / (kWaves * pq);
    const uint64_t n = npg * h.nmblocks;
    if (n > 0x7fffffffull) return false;
    nwg = static_cast<uint32_t>(n);
    lds = kOffsBytes + static_cast<size_t>(T) * (h.nchunks + 1u) * 1024u;
    return true;
}

}  // namespace

extern "C" hipError_t pmk_mfma(const PmkMfma *hp, hipStream_t st) {
    PmkMfma h = *hp;
    if (h.s == 0) return hipSuccess;
    // compute units of the current device, looked up once per device, and
    // the dynamic LDS limit raised so far per kernel and device
    static std::mutex mu;
    static std::map<int, uint32_t> cus;
    static std::map<std::pair<int, const void *>, size_t> lds_set;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    uint32_t ncu = 0;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cus.find(dev);
        if (it == cus.end()) {
            int n = 0;
            e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            it = cus.emplace(dev, static_cast<uint32_t>(n)).first;
        }
        ncu = it->second;
    }
    uint32_t T = 0, nwg = 0;
    size_t lds = 0;
    if (!mf_plan(h, ncu, T, nwg, lds)) return hipErrorInvalidValue;
    const void *fn = T == 4 ? reinterpret_cast<const void *>(&pm_mfma<4, 2>)
                            : reinterpret_cast<const void *>(&pm_mfma<2, 4>);
    if (lds > 64u * 1024u) {   // past the default limit of dynamic LDS
        std::lock_guard<std::mutex> lk(mu);
        size_t &cur = lds_set[{dev, fn}];
        if (cur < lds) {
            e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
            if (e != hipSuccess) return e;
            cur = lds;
        }
    }
    if (T == 4)
        hipLaunchKernelGGL((pm_mfma<4, 2>), dim3(nwg), dim3(64 * kWaves), lds, st, h);
    else
        hipLaunchKernelGGL((pm_mfma<2, 4>), dim3(nwg), dim3(64 * kWaves), lds, st, h);
    return hipGetLastError();
}
