// Batched GF(2^8) Gauss-Jordan elimination on the device: the init phase of
// decode (and any other per-failure-pattern inverse), many patterns at once.
//
// The paper splits each operation into an initialization that builds or
// inverts small matrices and a data phase that applies them (Section 4),
// and notes that the initialization dominates for small objects.  Decoding
// from a node set K inverts the rows of the generator that K's blocks
// follow (Section 2: X = inverse(G~) Y~); for MBR the k d received rows have
// rank B and the first independent ones, in order, are used.
//
// One work-group per problem.  All m candidate rows sit in LDS as
// [g_i | e_i] (B generator columns, then m columns that start as the
// identity), and columns are eliminated in order: the pivot of column c is
// the lowest-index candidate not yet a pivot with a nonzero in c, which is
// scaled to 1 there and cleared from every other row.  After B columns the
// g parts of the pivot rows are unit vectors and their e parts are the rows
// of the inverse of the pivot candidates.  That set is the set of the first
// B independent candidates in order: were the pivot r_i of column c in the
// span of r_0 .. r_{i-1}, then (the non-pivot rows below index i being zero
// on columns 0..c, the pivot rows independent on the pivot columns) its
// current value would be a combination of those non-pivot rows alone and
// zero at c.  So the result is the (unique) inverse of the same rows as any
// exact elimination that keeps the first independent rows.
//
// Each update row_i ^= f_i * P (P the scaled pivot row) XORs the eight
// multiples x^t P, formed once per pivot, selected by the bits of f_i: a
// thread holds them for its dword column in registers, so an update costs
// one LDS read-modify-write per 4 bytes and no table lookups.
//
// Field: x^8 + x^4 + x^3 + x^2 + 1 with generator 2; the pivot inverse and
// the scaling through exponent and logarithm tables built in LDS.
#include "gj.hpp"

namespace {

constexpr uint8_t kZeroLog = 0xFF;   // log of 0

// exp[t] = 2^t twice over (so a sum of two logs indexes it), log[2^t] = t,
// log[0] = kZeroLog; built by the compiler
struct GfTables {
    uint8_t ex[512];
    uint8_t lg[256];
};
constexpr GfTables gf_tables() {
    GfTables t{};
    uint32_t e = 1;
    for (uint32_t i = 0; i < 255u; ++i) {
        t.ex[i] = t.ex[i + 255u] = static_cast<uint8_t>(e);
        t.lg[e] = static_cast<uint8_t>(i);
        e = ((e << 1) ^ ((e & 0x80u) ? 0x11Du : 0u)) & 0xFFu;
    }
    t.lg[0] = kZeroLog;
    return t;
}
__constant__ GfTables kGf = gf_tables();

// x times four packed field elements
__device__ __forceinline__ uint32_t xtime4(uint32_t v) {
    const uint32_t hi = (v >> 7) & 0x01010101u;
    return ((v & 0x7F7F7F7Fu) << 1) ^ (hi * 0x1Du);
}

}  // namespace

extern "C" __global__ __launch_bounds__(1024) void pm_gj(PmkGj a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const uint32_t B = a.B, m = a.nrows, T = blockDim.x, tid = threadIdx.x, p = blockIdx.x;
    const uint32_t W = pmk_gj_width(B, m), W4 = W / 4u;
    const uint32_t lane = tid % 64u, wave = tid / 64u, nwaves = T / 64u;
    // 2-D map of the row updates: cols threads along a row, G row groups
    const uint32_t cols = W4 < T ? W4 : T, G = T / cols, j0 = tid % cols, g0 = tid / cols;
    // LDS: u32 pivrow[B], kept[B], slot[4], setv[nsets], pw[8][W4];
    // u8 rows[m][W], exp[512], log[256], used[m], fcol[m]
    uint32_t *pivrow = reinterpret_cast<uint32_t *>(sm);
    uint32_t *kept = pivrow + B;
    uint32_t *slot = kept + B;
    uint32_t *setv = slot + 4;
    uint32_t *pw = setv + a.nsets;
    uint8_t *rows = reinterpret_cast<uint8_t *>(pw + 8u * W4);
    uint32_t *rows4 = reinterpret_cast<uint32_t *>(rows);
    uint8_t *ex = rows + static_cast<size_t>(m) * W;
    uint8_t *lg = ex + 512;
    uint8_t *used = lg + 256;
    uint8_t *fcol = used + m;

    for (uint32_t t = tid; t < 512u; t += T) ex[t] = kGf.ex[t];
    for (uint32_t t = tid; t < 256u; t += T) lg[t] = kGf.lg[t];
    if (a.sets)
        for (uint32_t i = tid; i < a.nsets; i += T) setv[i] = a.sets[static_cast<uint64_t>(p) * a.nsets + i];
    if (tid == 0) slot[1] = 0;
    __syncthreads();
    // node ids of a set: in range and distinct, else nothing is read
    if (a.sets)
        for (uint32_t i = tid; i < a.nsets; i += T) {
            uint32_t bad = setv[i] >= a.nnodes;
            for (uint32_t j = 0; j < i; ++j) bad |= setv[j] == setv[i];
            if (bad) atomicOr(&slot[1], 1u);
        }
    __syncthreads();
    const bool bad = slot[1] != 0u;
    if (!bad) {
        // candidate i: [its generator row | e_i | zero padding], a wave per row
        for (uint32_t i = wave; i < m; i += nwaves) {
            const uint64_t idx = a.sets ? static_cast<uint64_t>(setv[i / a.alpha]) * a.alpha + i % a.alpha : i;
            const uint8_t *src = a.src + static_cast<uint64_t>(p) * a.src_stride + idx * a.src_ld;
            for (uint32_t j = lane; j < W; j += 64u) rows[i * W + j] = j < B ? src[j] : (j == B + i ? 1 : 0);
        }
        for (uint32_t i = tid; i < m; i += T) used[i] = 0;
    }
    uint32_t np = 0;   // pivots found
    for (uint32_t c = 0; c < B && !bad; ++c) {
        if (tid == 0) slot[0] = m;
        __syncthreads();
        for (uint32_t i = tid; i < m; i += T)
            if (!used[i] && rows[i * W + c]) atomicMin(&slot[0], i);
        __syncthreads();
        const uint32_t pr = slot[0];
        if (pr == m) break;   // rank < B
        // scale the pivot row to 1 at c and form its multiples x^t P (the
        // row is zero before column c, so dwords before c / 4 stay zero);
        // keep column c of every row for the updates
        const uint32_t linv = (255u - lg[rows[pr * W + c]]) % 255u;
        for (uint32_t i = tid; i < m; i += T) fcol[i] = i == pr ? 0 : rows[i * W + c];
        for (uint32_t j4 = c / 4u + tid; j4 < W4; j4 += T) {
            const uint32_t x = rows4[pr * W4 + j4];
            uint32_t y = 0;
            for (uint32_t b = 0; b < 4; ++b) {
                const uint32_t v = (x >> (8u * b)) & 0xFFu;
                if (v) {
                    uint32_t l = lg[v] + linv;
                    if (l >= 255u) l -= 255u;
                    y |= static_cast<uint32_t>(ex[l]) << (8u * b);
                }
            }
            for (uint32_t t = 0; t < 8; ++t) {
                pw[t * W4 + j4] = y;
                y = xtime4(y);
            }
        }
        __syncthreads();
        // clear column c from every other row (f of the pivot row is 0);
        // the pivot row becomes P.  A thread owns dword column j4 of rows
        // g, g + G, ...: it holds the eight multiples of P there and selects
        // them by the bits of f_i, acc ^ (mask & P) in one three-input op.
        if (g0 < G)
            for (uint32_t j4 = j0; j4 < W4; j4 += cols) {
                if (j4 < c / 4u) continue;
                uint32_t P[8];
                for (uint32_t t = 0; t < 8; ++t) P[t] = pw[t * W4 + j4];
                if (pr % G == g0) rows4[pr * W4 + j4] = P[0];
                for (uint32_t i = g0; i < m; i += G) {
                    const uint32_t f = fcol[i];
                    if (!f) continue;
                    uint32_t acc = rows4[i * W4 + j4];
                    for (uint32_t t = 0; t < 8; ++t)
                        acc = __builtin_amdgcn_bitop3_b32(acc, static_cast<uint32_t>(-static_cast<int32_t>((f >> t) & 1u)),
                                                          P[t], 0x78);
                    rows4[i * W4 + j4] = acc;
                }
            }
        if (tid == 0) {
            used[pr] = 1;
            pivrow[c] = pr;
        }
        ++np;
    }
    __syncthreads();
    const int32_t st = bad ? -1 : (np == B ? 0 : -3);
    if (tid == 0) a.status[p] = st;
    uint8_t *D = a.D + static_cast<uint64_t>(p) * a.d_stride;
    if (st != 0) {
        for (uint32_t t = tid; t < B * B; t += T) D[static_cast<uint64_t>(t / B) * a.d_ld + t % B] = 0;
        return;
    }
    // the pivot candidates in increasing order: kept[q]
    for (uint32_t c = tid; c < B; c += T) {
        uint32_t rank = 0;
        for (uint32_t c2 = 0; c2 < B; ++c2) rank += pivrow[c2] < pivrow[c];
        kept[rank] = pivrow[c];
    }
    __syncthreads();
    // row c of the inverse: the e part of column c's pivot row, read at the
    // pivot candidates in increasing order
    for (uint32_t t = tid; t < B * B; t += T) {
        const uint32_t c = t / B, q = t - c * B;
        D[static_cast<uint64_t>(c) * a.d_ld + q] = rows[pivrow[c] * W + B + kept[q]];
    }
    if (a.kept)
        for (uint32_t q = tid; q < B; q += T) a.kept[static_cast<uint64_t>(p) * B + q] = kept[q];
}

// Row width (bytes) of the elimination state: B generator columns and m
// identity columns, rounded to whole dwords.
extern "C" __host__ __device__ uint32_t pmk_gj_width(uint32_t B, uint32_t m) { return (B + m + 3u) & ~3u; }

// Bytes of LDS one problem of m candidates, B columns and nsets node ids needs.
extern "C" size_t pmk_gj_lds_bytes(uint32_t B, uint32_t m, uint32_t nsets) {
    const size_t W = pmk_gj_width(B, m);
    return (2u * static_cast<size_t>(B) + 4u + nsets) * 4u + 8u * W + static_cast<size_t>(m) * W + 512u + 256u +
           2u * m;
}

extern "C" hipError_t pmk_gj(const PmkGj *h, uint32_t count, hipStream_t st) {
    const size_t lds = pmk_gj_lds_bytes(h->B, h->nrows, h->sets ? h->nsets : 0u);
    const uint32_t threads = h->B <= 64 ? 256u : 1024u;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(pm_gj),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(pm_gj, dim3(count), dim3(threads), lds, st, *h);
    return hipGetLastError();
}
