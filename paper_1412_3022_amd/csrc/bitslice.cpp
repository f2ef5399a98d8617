// Bit-sliced region kernels specialized per matrix (compiled with hipRTC).
//
// Multiplying a byte by a constant c in GF(2^8) is linear over GF(2): bit i
// of c*x is the XOR of the bits j of x for which bit i of c*2^j is set.  Once
// 32 bytes of a lane are transposed into 8 bit planes (plane j = bit j of
// every byte), c*x for all 32 bytes is a fixed XOR network over the planes,
// and a whole row group is a fixed network over its columns' planes.  This is
// the GPU counterpart of the paper's bit-matrix XOR schedules (Section 4.1,
// the encode paragraph's note on bit matrices).
//
// The network is emitted as straight-line HIP source for one matrix,
// compiled once with hipRTC and cached (per matrix and device).  Per source
// column the generator forms the XOR combinations of planes 0-3 and of
// planes 4-7 that the group's rows need (the "four Russians" table), so every
// output plane costs one three-input XOR per column.  The 8x8 bit transposes
// in and out cost 12 masked swaps each.  Rows of a group number at most 8
// (64 plane accumulators), or 16 for a matrix of at most 16 x 16 that is
// then one group; copy groups move bytes without transposing.
//
// Launch geometry: each lane owns 32 bytes of a wave tile (two 16-byte
// pieces 1 KiB apart, so every load instruction is one contiguous KiB).
// Work-groups of 4 waves are dealt to the 8 XCDs round-robin; on each XCD
// every slot (work-group) is bound to one row group and the slots of a group
// stride over that XCD's range of tiles.  All groups of a tile therefore run
// at about the same time in one L2 (shared source columns are mostly read
// from HBM once), while each work-group executes only one group's code (the
// instruction cache holds it).  A wave loads the two columns after the one
// it multiplies (the k=8 encode then needs 125 VGPRs: 4 waves per SIMD), and
// the outputs leave with streaming (nontemporal) stores.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "bitslice.hpp"
#include "construct.hpp"
#include "engine.hpp"
#include "gf256.hpp"
#include "program.hpp"

namespace pmrc {
namespace {

constexpr int kGroupWords = 8;
constexpr size_t kPrefetch = 2;   // columns loaded ahead of the one being multiplied
// First statement of every group function: an empty asm that makes the two
// strides opaque for each call.  Without it the compiler hoists every
// group's column bases (in + column * ld) out of the tile loop, and the
// hundreds of 64-bit scalars that produces spill into VGPR lanes (k = 16
// encode: 903 SGPR spills and 176 VGPRs, against none and 151 with it).
const char *kOpaqueStrides = "  asm volatile(\"\" : \"+s\"(ld), \"+s\"(old));\n";
constexpr int kWaves = 4;         // waves per work-group
constexpr int kHeaderWords = 4;

const char *kPrelude = R"(
typedef unsigned int u32;
typedef unsigned long long u64;
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
#define X3(a, b, c) __builtin_amdgcn_bitop3_b32((a), (b), (c), 0x96)
// outputs are written once and not read back by the kernel: streaming stores
__device__ __forceinline__ void ST(unsigned char *d, u32x4 v) { __builtin_nontemporal_store(v, (u32x4 *)d); }
// delta swap of the bits of b under mask m with those of a under m << sh,
// as two selects (v_bitop3 truth table 0xD8: c ? b : a)
#define SEL(a, b, m) __builtin_amdgcn_bitop3_b32((a), (b), (m), 0xD8)
#define DS(a, b, sh, m) { const u32 a_ = (a), b_ = (b); (a) = SEL(a_, b_ << (sh), (m) << (sh)); (b) = SEL(b_, a_ >> (sh), (m)); }
#define TR8(A0, A1, A2, A3, A4, A5, A6, A7) { \
  DS(A0, A4, 4, 0x0F0F0F0Fu) DS(A1, A5, 4, 0x0F0F0F0Fu) DS(A2, A6, 4, 0x0F0F0F0Fu) DS(A3, A7, 4, 0x0F0F0F0Fu) \
  DS(A0, A2, 2, 0x33333333u) DS(A1, A3, 2, 0x33333333u) DS(A4, A6, 2, 0x33333333u) DS(A5, A7, 2, 0x33333333u) \
  DS(A0, A1, 1, 0x55555555u) DS(A2, A3, 1, 0x55555555u) DS(A4, A5, 1, 0x55555555u) DS(A6, A7, 1, 0x55555555u) }
// One region set: tile0 = its first tile in the launch's tile numbering.
struct BsItem { const unsigned char *in; u64 ld; unsigned char *out; u64 old; u64 s; u32 nfull, ntiles, tile0, pad; };
// Arguments of the single-set kernel.
struct BsArgs { const unsigned char *in; u64 ld; unsigned char *out; u64 old; u64 s; u32 nfull, ntiles, P; };
// Arguments of the multi-set kernel: `items` in device memory, sorted by tile0.
struct BsMultiArgs { const BsItem *items; u32 nitems, ntiles, P, pad; };
// A wave-uniform 64-bit value, made a scalar for the compiler.  The builtin
// returns int: each half goes through u32 so the low half is not
// sign-extended into the high one.
__device__ __forceinline__ u64 rfl64(u64 x) {
  const u32 hi = (u32)__builtin_amdgcn_readfirstlane((u32)(x >> 32));
  const u32 lo = (u32)__builtin_amdgcn_readfirstlane((u32)x);
  return ((u64)hi << 32) | (u64)lo;
}
// Index of the item that holds tile t, searched in [lo, hi).
__device__ __forceinline__ u32 find_item(const BsItem *items, u32 lo, u32 hi, u32 t) {
  while (hi - lo > 1u) {
    const u32 mid = (lo + hi) / 2u;
    if (items[mid].tile0 <= t) lo = mid; else hi = mid;
  }
  return lo;
}
// Product in GF(2^8) by shift and add (used only for the last s mod 16 bytes).
__device__ __forceinline__ u32 gm(u32 c, u32 x) {
  u32 p = 0u;
#pragma unroll 1
  for (; c; c >>= 1) {
    if (c & 1u) p ^= x;
    x = (x << 1) ^ ((x & 0x80u) ? POLY : 0u);
  }
  return p;
}
)";

struct Grp {
    uint32_t kind;
    std::vector<uint32_t> rows, cols;           // output rows; input blocks
    std::vector<std::vector<uint8_t>> coef;     // [row][col]
};

std::vector<Grp> read_groups(const Program &p) {
    std::vector<Grp> out;
    const uint32_t *b = p.blob.data();
    for (int g = 0; g < p.ngroups; ++g) {
        const uint32_t *r = b + kHeaderWords + g * kGroupWords;
        Grp G;
        G.kind = r[0];
        const uint32_t nrows = r[1], ncols = r[2];
        for (uint32_t i = 0; i < nrows; ++i) G.rows.push_back(b[r[5] + i]);
        if (G.kind == GROUP_COPY) {
            for (uint32_t i = 0; i < nrows; ++i) G.cols.push_back(b[r[3] + i]);
        } else {
            for (uint32_t c = 0; c < ncols; ++c) G.cols.push_back(b[r[3] + c]);
            G.coef.assign(nrows, std::vector<uint8_t>(ncols, 0));
            for (uint32_t c = 0; c < ncols; ++c)
                for (uint32_t i = 0; i < nrows; ++i)   // slot (c, i): word 0 byte 1 = coef * 1
                    G.coef[i][c] = static_cast<uint8_t>((b[r[4] + (c * p.rg + i) * 4] >> 8) & 0xFF);
        }
        out.push_back(std::move(G));
    }
    return out;
}

int popc(unsigned m) { return __builtin_popcount(m); }

// A load step for every column, the same in every table group that reads
// it: the groups of a tile run at about the same pace, so a column shared
// by several groups is then fetched by all of them within a short window
// and the later fetches hit L2.  Greedy: columns read by most groups first,
// each at the first step still free in all its groups.
std::map<uint32_t, int> column_steps(const std::vector<Grp> &gs) {
    std::map<uint32_t, std::vector<int>> users;
    for (size_t g = 0; g < gs.size(); ++g) {
        if (gs[g].kind == GROUP_COPY) continue;
        for (size_t ci = 0; ci < gs[g].cols.size(); ++ci) {
            bool any = false;
            for (size_t r = 0; r < gs[g].rows.size(); ++r) any |= gs[g].coef[r][ci] != 0;
            if (any) users[gs[g].cols[ci]].push_back(static_cast<int>(g));
        }
    }
    std::vector<uint32_t> order;
    for (auto &kv : users) order.push_back(kv.first);
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return users[a].size() > users[b].size(); });
    std::vector<std::set<int>> taken(gs.size());
    std::map<uint32_t, int> step;
    for (uint32_t c : order) {
        int s = 0;
        for (;; ++s) {
            bool free = true;
            for (int g : users[c]) free &= !taken[g].count(s);
            if (free) break;
        }
        step[c] = s;
        for (int g : users[c]) taken[g].insert(s);
    }
    return step;
}

// Straight-line code of one table group.
void emit_table_group(std::ostringstream &o, int gi, const Grp &G, const std::map<uint32_t, int> &steps) {
    const int n = static_cast<int>(G.rows.size());
    o << "__device__ __forceinline__ void g" << gi
      << "(const unsigned char *in, u64 ld, unsigned char *out, u64 old, u64 off) {\n" << kOpaqueStrides;
    for (int r = 0; r < n; ++r) {
        o << "  u32";
        for (int i = 0; i < 8; ++i) o << (i ? "," : "") << " q" << r << "_" << i << " = 0u";
        o << ";\n";
    }
    // Columns with a nonzero coefficient (padding columns are skipped).  The
    // loads of column j + kPrefetch are issued before column j is multiplied,
    // so every wave keeps several columns in flight.
    std::vector<size_t> used;
    for (size_t ci = 0; ci < G.cols.size(); ++ci) {
        bool any = false;
        for (int r = 0; r < n; ++r) any |= G.coef[r][ci] != 0;
        if (any) used.push_back(ci);
    }
    std::stable_sort(used.begin(), used.end(),
                     [&](size_t a, size_t b) { return steps.at(G.cols[a]) < steps.at(G.cols[b]); });
    auto load = [&](size_t j) {
        o << "  const u32x4 x" << j << "l = *(const u32x4 *)(in + (u64)" << G.cols[used[j]] << "u * ld + off), x" << j
          << "h = *(const u32x4 *)(in + (u64)" << G.cols[used[j]] << "u * ld + off + 1024);\n";
    };
    for (size_t j = 0; j < used.size() && j < kPrefetch; ++j) load(j);
    for (size_t j = 0; j < used.size(); ++j) {
        const size_t ci = used[j];
        if (j + kPrefetch < used.size()) load(j + kPrefetch);
        o << "  {\n    const u32x4 lo = x" << j << "l, hi = x" << j << "h;\n"
          << "    u32 P0 = lo.x, P1 = lo.y, P2 = lo.z, P3 = lo.w, P4 = hi.x, P5 = hi.y, P6 = hi.z, P7 = hi.w;\n"
          << "    TR8(P0, P1, P2, P3, P4, P5, P6, P7)\n";
        struct Eq { int r, i; unsigned lo, hi; };
        std::vector<Eq> eqs;
        std::set<std::pair<int, unsigned>> need;   // (half, mask)
        for (int r = 0; r < n; ++r) {
            const uint8_t a = G.coef[r][ci];
            if (!a) continue;
            uint8_t colbits[8];
            for (int j = 0; j < 8; ++j) colbits[j] = gmul(a, static_cast<uint8_t>(1u << j));
            for (int i = 0; i < 8; ++i) {
                unsigned lo = 0, hi = 0;
                for (int j = 0; j < 8; ++j)
                    if ((colbits[j] >> i) & 1) {
                        if (j < 4) lo |= 1u << j;
                        else hi |= 1u << (j - 4);
                    }
                eqs.push_back({r, i, lo, hi});
                if (lo) need.insert({0, lo});
                if (hi) need.insert({1, hi});
            }
        }
        auto name = [](int half, unsigned m) {
            std::ostringstream s;
            if (popc(m) == 1) s << "P" << (__builtin_ctz(m) + 4 * half);
            else s << (half ? "H" : "L") << m;
            return s.str();
        };
        std::set<std::pair<int, unsigned>> made;
        // each combination = (combination without its lowest plane) ^ that plane
        std::vector<std::pair<int, unsigned>> order(need.begin(), need.end());
        std::sort(order.begin(), order.end(), [](auto a, auto b) {
            return popc(a.second) != popc(b.second) ? popc(a.second) < popc(b.second) : a < b;
        });
        for (auto want : order) {
            std::vector<unsigned> chain;
            for (unsigned m = want.second; popc(m) > 1 && !made.count({want.first, m}); m &= m - 1) chain.push_back(m);
            for (auto it = chain.rbegin(); it != chain.rend(); ++it) {
                const unsigned m = *it, low = m & (~m + 1);
                o << "    const u32 " << name(want.first, m) << " = " << name(want.first, m ^ low) << " ^ "
                  << name(want.first, low) << ";\n";
                made.insert({want.first, m});
            }
        }
        for (const Eq &e : eqs) {
            const std::string q = "q" + std::to_string(e.r) + "_" + std::to_string(e.i);
            if (e.lo && e.hi) o << "    " << q << " = X3(" << q << ", " << name(0, e.lo) << ", " << name(1, e.hi) << ");\n";
            else if (e.lo) o << "    " << q << " ^= " << name(0, e.lo) << ";\n";
            else if (e.hi) o << "    " << q << " ^= " << name(1, e.hi) << ";\n";
        }
        o << "  }\n";
    }
    for (int r = 0; r < n; ++r) {
        o << "  TR8(";
        for (int i = 0; i < 8; ++i) o << (i ? ", " : "") << "q" << r << "_" << i;
        o << ")\n  { unsigned char *d = out + (u64)" << G.rows[r] << "u * old + off;\n"
          << "    ST(d, u32x4{q" << r << "_0, q" << r << "_1, q" << r << "_2, q" << r << "_3});\n"
          << "    ST(d + 1024, u32x4{q" << r << "_4, q" << r << "_5, q" << r << "_6, q" << r << "_7}); }\n";
    }
    o << "}\n";
}

void emit_copy_group(std::ostringstream &o, int gi, const Grp &G) {
    o << "__device__ __forceinline__ void g" << gi
      << "(const unsigned char *in, u64 ld, unsigned char *out, u64 old, u64 off) {\n" << kOpaqueStrides;
    for (size_t i = 0; i < G.rows.size(); ++i)
        o << "  { const unsigned char *p = in + (u64)" << G.cols[i] << "u * ld + off;\n"
          << "    unsigned char *d = out + (u64)" << G.rows[i] << "u * old + off;\n"
          << "    const u32x4 lo = *(const u32x4 *)p, hi = *(const u32x4 *)(p + 1024);\n"
          << "    ST(d, lo); ST(d + 1024, hi); }\n";
    o << "}\n";
}

// The last s mod 16 bytes of every row: one lane per byte position, each
// output byte the sum over the group's columns of coefficient times input
// byte, with the group's rows, columns and coefficients in constant tables.
void emit_byte_tail(std::ostringstream &o, int gi, const Grp &G) {
    const size_t nr = G.rows.size(), nc = G.kind == GROUP_COPY ? 1 : G.cols.size();
    o << "__constant__ u32 tr" << gi << "[" << nr << "] = {";
    for (size_t r = 0; r < nr; ++r) o << (r ? ", " : "") << G.rows[r] << "u";
    o << "};\n__constant__ u32 tc" << gi << "[" << nr * nc << "] = {";
    for (size_t r = 0; r < nr; ++r)
        for (size_t c = 0; c < nc; ++c) {
            // per (row, column): input block | coefficient << 24
            const uint32_t col = G.kind == GROUP_COPY ? G.cols[r] : G.cols[c];
            const uint32_t coef = G.kind == GROUP_COPY ? 1u : G.coef[r][c];
            o << (r + c ? ", " : "") << (col | coef << 24) << "u";
        }
    o << "};\n__device__ __noinline__ void b" << gi
      << "(const unsigned char *in, u64 ld, unsigned char *out, u64 old, u64 pos) {\n"
      << "#pragma unroll 1\n  for (u32 r = 0; r < " << nr << "u; ++r) {\n    u32 acc = 0u;\n"
      << "#pragma unroll 1\n    for (u32 c = 0; c < " << nc << "u; ++c) {\n"
      << "      const u32 e = tc" << gi << "[r * " << nc << "u + c];\n"
      << "      acc ^= gm(e >> 24, in[(u64)(e & 0xFFFFFFu) * ld + pos]);\n    }\n"
      << "    out[(u64)tr" << gi << "[r] * old + pos] = (unsigned char)acc;\n  }\n}\n";
}

// Straight-line operations per lane chunk: per emitted column (nonzero
// somewhere in the group) its transpose, combinations and one three-input XOR
// per row plane; per row the output transpose.
long estimate_ops(const std::vector<Grp> &gs) {
    long ops = 0;
    for (const Grp &G : gs) {
        if (G.kind == GROUP_COPY) continue;
        long cols = 0;
        for (size_t ci = 0; ci < G.cols.size(); ++ci) {
            bool any = false;
            for (size_t r = 0; r < G.rows.size(); ++r) any |= G.coef[r][ci] != 0;
            cols += any;
        }
        ops += cols * (60 + 24 + 8 * static_cast<long>(G.rows.size()));
        ops += 60 * static_cast<long>(G.rows.size());
    }
    return ops;
}


}  // namespace

std::unique_ptr<BsProgram> bs_generate(const Program &p8) {
    std::vector<Grp> gs = read_groups(p8);
    auto bp = std::make_unique<BsProgram>();
    bp->ngroups = static_cast<int>(gs.size());
    bp->est_ops = estimate_ops(gs);
    if (bp->est_ops > kBsMaxOps) return bp;   // left to the table kernels: no source
    std::ostringstream o;
    // reduction polynomial of the field: x^8 = x * x^7
    o << "#define POLY " << (0x100u | gmul(0x80, 2)) << "u\n" << kPrelude;
    const std::map<uint32_t, int> steps = column_steps(gs);
    for (size_t g = 0; g < gs.size(); ++g) {
        if (gs[g].kind == GROUP_COPY) emit_copy_group(o, static_cast<int>(g), gs[g]);
        else emit_table_group(o, static_cast<int>(g), gs[g], steps);
        emit_byte_tail(o, static_cast<int>(g), gs[g]);
    }
    const int G = bp->ngroups;
    const std::string body = o.str();
    // Tiles 0 .. nfull-1 of a region set are the full 2048-byte tiles; when
    // s16 (s rounded down to 16) is not a multiple of 2048, tile nfull is the
    // window [s16 - 2048, s16), which overlaps tile nfull-1 and stores the
    // same bytes it does.  The s - s16 bytes after s16 are done byte by byte
    // by the lanes of the wave that takes the last tile.
    auto group_calls = [&](std::ostringstream &k, const char *pre, const char *ind) {
        k << ind << "switch (g) {\n";
        for (int g = 0; g < G; ++g)
            k << ind << "  case " << g << ": g" << g << "(" << pre << "in, " << pre << "ld, " << pre << "out, " << pre
              << "old, tile + lane * 16u); break;\n";
        k << ind << "}\n" << ind << "if (lt == " << pre << "ntiles - 1u && s16 + lane < " << pre << "s) {\n"
          << ind << "  switch (g) {\n";
        for (int g = 0; g < G; ++g)
            k << ind << "    case " << g << ": b" << g << "(" << pre << "in, " << pre << "ld, " << pre << "out, " << pre
              << "old, s16 + lane); break;\n";
        k << ind << "  }\n" << ind << "}\n";
    };
    auto head = [&](std::ostringstream &k, const char *name, const char *args) {
        k << "extern \"C\" __global__ __launch_bounds__(" << 64 * kWaves << ") void " << name << "(" << args
          << " a) {\n"
          << "  const u32 wave = threadIdx.x / 64, lane = threadIdx.x % 64;\n"
          << "  const u32 xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;\n"
          << "  const u32 per = (a.ntiles + 7u) / 8u, t0 = xcd * per;\n"
          << "  const u32 t1 = t0 + per < a.ntiles ? t0 + per : a.ntiles;\n"
          << "  const u32 G = " << G << "u;\n"
          << "  // slots of one group stride over this XCD's tiles; with fewer slots\n"
          << "  // than groups a slot takes groups slot, slot + P, ...\n"
          << "  for (u32 g = slot % G; g < G; g += a.P) {\n"
          << "    const u32 R = a.P >= G ? (a.P - 1u - g) / G + 1u : 1u;\n"
          << "    const u32 r = a.P >= G ? slot / G : 0u;\n";
    };
    {
        std::ostringstream k;
        head(k, "pmbs", "BsArgs");
        k << "    const u64 s16 = a.s & ~15ull;\n"
          << "    for (u32 t = t0 + r * " << kWaves << "u + wave; t < t1; t += R * " << kWaves << "u) {\n"
          << "      const u32 lt = t;\n"
          << "      const u64 tile = t < a.nfull ? (u64)t * 2048u : s16 - 2048u;\n";
        group_calls(k, "a.", "      ");
        k << "    }\n    if (a.P >= G) break;\n  }\n}\n";
        bp->k[BS_SINGLE].source = body + k.str();
    }
    {
        // The tiles of all sets are numbered back to back; a wave walks its
        // tiles in rising order and finds each one's set by a search bounded
        // by its stride (every set has at least one tile).
        std::ostringstream k;
        head(k, "pmbs_multi", "BsMultiArgs");
        k << "    const u32 step = R * " << kWaves << "u;\n"
          << "    u32 it = 0u, prev = 0u;\n"
          << "    bool first = true;\n"
          << "    for (u32 t = t0 + r * " << kWaves << "u + wave; t < t1; t += step) {\n"
          << "      const u32 lim = first ? a.nitems : (it + (t - prev) + 1u < a.nitems ? it + (t - prev) + 1u : a.nitems);\n"
          << "      it = find_item(a.items, first ? 0u : it, lim, t);\n"
          << "      first = false;\n"
          << "      prev = t;\n"
          << "      BsItem I = a.items[it];\n"
          << "      // the set is the same for the whole wave\n"
          << "      I.in = (const unsigned char *)rfl64((u64)I.in);\n"
          << "      I.out = (unsigned char *)rfl64((u64)I.out);\n"
          << "      I.ld = rfl64(I.ld);\n"
          << "      I.old = rfl64(I.old);\n"
          << "      I.s = rfl64(I.s);\n"
          << "      const u32 lt = t - I.tile0;\n"
          << "      const u64 s16 = I.s & ~15ull;\n"
          << "      const u64 tile = lt < I.nfull ? (u64)lt * 2048u : s16 - 2048u;\n";
        group_calls(k, "I.", "      ");
        k << "    }\n    if (a.P >= G) break;\n  }\n}\n";
        bp->k[BS_MULTI].source = body + k.str();
    }
    if (const char *dump = getenv("PMRC_BS_DUMP")) {   // debugging aid: keep the generated sources
        for (int kind = 0; kind < 2; ++kind) {
            const std::string path = std::string(dump) + (kind == BS_MULTI ? ".multi" : "");
            if (FILE *f = fopen(path.c_str(), "w")) {
                fputs(bp->k[kind].source.c_str(), f);
                fclose(f);
            }
        }
    }
    return bp;
}

static int bs_compile_locked(BsKernel &bk);

int bs_compile(BsProgram &bp, BsKind kind) {
    std::lock_guard<std::mutex> lk(bp.mu);
    BsKernel &bk = bp.k[kind];
    if (bk.compiled) return bk.compile_status;
    bk.compiled = true;
    bk.compile_status = bs_compile_locked(bk);
    bk.state.store(bk.compile_status == ST_OK ? BS_READY : BS_FAILED, std::memory_order_release);
    return bk.compile_status;
}

// Code objects by generated source, for the life of the process: the same
// matrix met again (another code object with the same parameters, or a
// failure pattern seen before) reuses its code instead of running hipRTC.
static std::mutex g_code_mu;
static std::map<std::string, std::vector<char>> &g_code_cache = *new std::map<std::string, std::vector<char>>();

static int bs_compile_locked(BsKernel &bk) {
    {
        std::lock_guard<std::mutex> lk(g_code_mu);
        auto it = g_code_cache.find(bk.source);
        if (it != g_code_cache.end()) {
            bk.code = it->second;
            return ST_OK;
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, bk.source.c_str(), "pm_bitslice.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
        return ST_EHIP;
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17"};
    hiprtcResult r = hiprtcCompileProgram(prog, 3, opts);
    if (r != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        g_hip_msg = "hipRTC: " + log.substr(0, 2000);
        hiprtcDestroyProgram(&prog);
        return ST_EHIP;
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    bk.code.resize(cs);
    hiprtcGetCode(prog, bk.code.data());
    hiprtcDestroyProgram(&prog);
    std::lock_guard<std::mutex> lk(g_code_mu);
    g_code_cache.emplace(bk.source, bk.code);
    return ST_OK;
}

BsProgram::~BsProgram() {
    for (BsKernel &bk : k)
        for (auto &kv : bk.dev)
            if (kv.second.mod) (void)hipModuleUnload(kv.second.mod);
}

// The module of a compiled kernel on the current device (loaded on first
// use there), with its work-group slots per XCD.  resident_only: neither
// compile nor load; ST_ENOTREADY unless the kernel is already loaded here.
static int bs_module(BsProgram &bp, BsKind kind, BsModule **out, bool resident_only = false) {
    if (resident_only) {
        if (!bs_ready(bp, kind)) return ST_ENOTREADY;
    } else {
        int st_c = bs_compile(bp, kind);
        if (st_c != ST_OK) return st_c;
    }
    int devid = 0;
    hipError_t e = hipGetDevice(&devid);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lk(bp.mu);
    BsKernel &bk = bp.k[kind];
    if (resident_only) {
        auto it = bk.dev.find(devid);
        if (it == bk.dev.end() || !it->second.fn) return ST_ENOTREADY;
        *out = &it->second;
        return ST_OK;
    }
    BsModule *m = &bk.dev[devid];
    if (!m->fn) {
        if (!m->mod && (e = hipModuleLoadData(&m->mod, bk.code.data())) != hipSuccess) {
            m->mod = nullptr;
            return hip_fail(e);
        }
        hipFunction_t fn = nullptr;
        if ((e = hipModuleGetFunction(&fn, m->mod, bp.fn_name[kind])) != hipSuccess)
            return hip_fail(e);
        int per_cu = 0, ncu = 0;
        if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * kWaves, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, devid) != hipSuccess || ncu < 8)
            ncu = 256;
        const int p0 = std::max(1, per_cu * ncu / 8);
        m->P = bp.ngroups <= p0 ? (p0 / bp.ngroups) * bp.ngroups : p0;
        m->fn = fn;
    }
    *out = m;
    return ST_OK;
}

BsItem bs_item(const uint8_t *in, uint64_t in_ld, uint8_t *out, uint64_t out_ld, uint64_t s, uint32_t tile0) {
    const uint64_t s16 = s & ~uint64_t(15), nfull = s16 / kBsTileBytes;
    return BsItem{in, in_ld, out, out_ld, s, static_cast<uint32_t>(nfull),
                  static_cast<uint32_t>(nfull + (s16 % kBsTileBytes ? 1 : 0)), tile0, 0};
}

int bs_load(BsProgram &bp, BsKind kind) {
    BsModule *m;
    return bs_module(bp, kind, &m);
}

// The kernel's one (struct) parameter goes through kernelParams, whose
// values the runtime copies at the launch call, also when the stream is
// being captured into a graph (a pointer to a caller's buffer passed in
// `extra` would have to outlive the graph).
template <class Args>
static int bs_go(Args &args, hipFunction_t fn, uint32_t P, hipStream_t st) {
    void *params[] = {&args};
    hipError_t e = hipModuleLaunchKernel(fn, 8u * P, 1, 1, 64 * kWaves, 1, 1, 0, st, params, nullptr);
    return e == hipSuccess ? ST_OK : hip_fail(e);
}

// Work-group slots per XCD for ntiles tiles: at least enough that every wave
// takes at most one tile of its group.  Slots past the resident ones start
// as the first work-groups finish, so the hardware dispatcher balances the
// last round instead of a few waves running a second tile after all others
// are done (64 MiB k = 8 encode: 30.4 -> 29.4 us; four times that object:
// 114 -> 106 us).
static uint32_t slots_for(const BsModule *m, int ngroups, uint64_t ntiles) {
    const uint64_t per = (ntiles + 7) / 8;
    const uint64_t one_shot = static_cast<uint64_t>(ngroups) * ((per + kWaves - 1) / kWaves);
    return static_cast<uint32_t>(std::max<uint64_t>(static_cast<uint64_t>(m->P), std::min<uint64_t>(one_shot, 1u << 24)));
}

int bs_launch(BsProgram &bp, const uint8_t *in, uint64_t in_ld, uint8_t *out, uint64_t out_ld, uint64_t s,
              hipStream_t st, bool resident_only) {
    // the window tile needs one full tile before it; shorter blocks are
    // refused here and left to the table kernels by the caller
    const uint64_t tb = bp.tile_bytes;
    if (s < tb) return ST_EINVAL;
    if (s / tb + 1 > 0xffffffffull) return ST_EINVAL;
    BsModule *m;
    int rc = bs_module(bp, BS_SINGLE, &m, resident_only);
    if (rc != ST_OK) return rc;
    const uint64_t s16 = s & ~uint64_t(15), nfull = s16 / tb;
    const BsItem it{in, in_ld, out, out_ld, s, static_cast<uint32_t>(nfull),
                    static_cast<uint32_t>(nfull + (s16 % tb ? 1 : 0)), 0, 0};
    struct {
        const uint8_t *in;
        uint64_t ld;
        uint8_t *out;
        uint64_t old, s;
        uint32_t nfull, ntiles, P;
    } args{in, in_ld, out, out_ld, s, it.nfull, it.ntiles, slots_for(m, bp.ngroups, it.ntiles)};
    return bs_go(args, m->fn, args.P, st);
}

int bs_launch_items(BsProgram &bp, const BsItem *d_items, uint32_t nitems, uint32_t ntiles, hipStream_t st,
                    uint32_t slots) {
    if (nitems == 0 || ntiles == 0) return ST_OK;
    BsModule *m;
    int rc = bs_module(bp, BS_MULTI, &m);
    if (rc != ST_OK) return rc;
    struct {
        const BsItem *items;
        uint32_t nitems, ntiles, P, pad;
    // persistent: each wave walks several tiles, which amortizes the search
    // for their items
    } args{d_items, nitems, ntiles, slots ? slots : static_cast<uint32_t>(m->P), 0};
    return bs_go(args, m->fn, args.P, st);
}

uint32_t bs_default_slots(BsProgram &bp) {
    BsModule *m;
    return bs_module(bp, BS_MULTI, &m) == ST_OK ? static_cast<uint32_t>(m->P) : 0u;
}

}  // namespace pmrc
