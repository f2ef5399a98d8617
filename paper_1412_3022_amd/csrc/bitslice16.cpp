// Bit-sliced region kernels for GF(2^16) matrices, specialized per matrix and
// compiled with hipRTC like the GF(2^8) ones (bitslice.cpp).
//
// Multiplying a 16-bit symbol by a constant c is linear over GF(2): bit i of
// c*x is the XOR of the bits j of x for which bit i of c*x^j is set, a 16 x 16
// bit matrix.  A lane holds 32 symbols of a block (four 16-byte pieces 1 KiB
// apart: a wave tile is 4 KiB).  Their low bytes, gathered into 8 dwords by
// byte permutes, and their high bytes are each transposed into 8 bit planes
// (the same 8 x 8 transposes as the byte field's), giving 16 planes; per
// source column the generator forms the XOR combinations of planes that the
// group's rows need within each nibble of planes (0-3, 4-7, 8-11, 12-15) and
// each output plane costs at most two three-input XORs.  The output planes
// go back through the same transposes and permutes.  A row group holds 4
// rows (64 plane accumulators).  Rows that are one input block times 1 are
// copied.  There are no tables: the matrix is in the code, so the kernel
// reads only the blocks (the table kernel also reads 24 table dwords per
// coefficient and row, which for matrices with many distinct coefficients
// come from beyond L2).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "bitslice.hpp"
#include "gf16.hpp"

namespace pmrc {
namespace w16 {
namespace {

constexpr int kRows = 4;          // rows per table group
constexpr int kCopyRows = 8;      // rows per copy group
constexpr int kWaves = 4;
constexpr uint32_t kTile = 4096;  // bytes of a block per wave tile

const char *kPrelude16 = R"(
typedef unsigned int u32;
typedef unsigned long long u64;
typedef u32 u32x4 __attribute__((ext_vector_type(4)));
#define X3(a, b, c) __builtin_amdgcn_bitop3_b32((a), (b), (c), 0x96)
__device__ __forceinline__ void ST(unsigned char *d, u32x4 v) { __builtin_nontemporal_store(v, (u32x4 *)d); }
// delta swap of the bits of b under mask m with those of a under m << sh,
// as two selects (v_bitop3 truth table 0xD8: c ? b : a)
#define SEL(a, b, m) __builtin_amdgcn_bitop3_b32((a), (b), (m), 0xD8)
#define DS(a, b, sh, m) { const u32 a_ = (a), b_ = (b); (a) = SEL(a_, b_ << (sh), (m) << (sh)); (b) = SEL(b_, a_ >> (sh), (m)); }
#define TR8(A0, A1, A2, A3, A4, A5, A6, A7) { \
  DS(A0, A4, 4, 0x0F0F0F0Fu) DS(A1, A5, 4, 0x0F0F0F0Fu) DS(A2, A6, 4, 0x0F0F0F0Fu) DS(A3, A7, 4, 0x0F0F0F0Fu) \
  DS(A0, A2, 2, 0x33333333u) DS(A1, A3, 2, 0x33333333u) DS(A4, A6, 2, 0x33333333u) DS(A5, A7, 2, 0x33333333u) \
  DS(A0, A1, 1, 0x55555555u) DS(A2, A3, 1, 0x55555555u) DS(A4, A5, 1, 0x55555555u) DS(A6, A7, 1, 0x55555555u) }
// low (LOB) or high (HIB) bytes of the 4 symbols in dwords a (symbols 0, 1)
// and b (2, 3), and back (MLO: symbols 0, 1 from low bytes L and high bytes
// H of 4 symbols; MHI: symbols 2, 3)
#define LOB(b, a) __builtin_amdgcn_perm((b), (a), 0x06040200u)
#define HIB(b, a) __builtin_amdgcn_perm((b), (a), 0x07050301u)
#define MLO(H, L) __builtin_amdgcn_perm((H), (L), 0x05010400u)
#define MHI(H, L) __builtin_amdgcn_perm((H), (L), 0x07030602u)
struct BsArgs { const unsigned char *in; u64 ld; unsigned char *out; u64 old; u64 s; u32 nfull, ntiles, P; };
// Product in GF(2^16) by shift and add (used only for the last s mod 16 bytes).
__device__ __forceinline__ u32 gm16(u32 c, u32 x) {
  u32 p = 0u;
#pragma unroll 1
  for (; c; c >>= 1) {
    if (c & 1u) p ^= x;
    x = ((x << 1) & 0xFFFFu) ^ ((x & 0x8000u) ? POLY16 : 0u);
  }
  return p;
}
)";

struct Grp {
    bool copy = false;
    std::vector<uint32_t> rows, cols;            // output rows; input blocks
    std::vector<std::vector<uint16_t>> coef;     // [row][col]
};

int popc(unsigned m) { return __builtin_popcount(m); }

// Load order of each table group's columns.  The groups of a tile run on one
// XCD at about the same pace, so a column that several groups read is given
// the same load step in all of them: the first fetch brings it into L2 and
// the others hit there instead of reading it from HBM again.  Greedy, columns
// read by most groups first, each at the first step free in all its groups;
// a group then loads its columns in step order (coefficients permuted along).
void order_columns(std::vector<Grp> &gs) {
    std::map<uint32_t, std::vector<size_t>> users;
    for (size_t g = 0; g < gs.size(); ++g)
        for (uint32_t c : gs[g].cols) users[c].push_back(g);
    std::vector<uint32_t> cols;
    for (auto &kv : users) cols.push_back(kv.first);
    std::stable_sort(cols.begin(), cols.end(),
                     [&](uint32_t a, uint32_t b) { return users[a].size() > users[b].size(); });
    std::vector<std::set<int>> taken(gs.size());
    std::map<uint32_t, int> step;
    for (uint32_t c : cols) {
        int s = 0;
        for (;; ++s) {
            bool free = true;
            for (size_t g : users[c]) free &= !taken[g].count(s);
            if (free) break;
        }
        step[c] = s;
        for (size_t g : users[c]) taken[g].insert(s);
    }
    for (Grp &g : gs) {
        std::vector<size_t> idx(g.cols.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(),
                         [&](size_t a, size_t b) { return step[g.cols[a]] < step[g.cols[b]]; });
        Grp h;
        h.rows = g.rows;
        for (size_t i : idx) h.cols.push_back(g.cols[i]);
        for (auto &row : g.coef) {
            std::vector<uint16_t> v;
            for (size_t i : idx) v.push_back(row[i]);
            h.coef.push_back(std::move(v));
        }
        g = std::move(h);
    }
}

std::vector<Grp> make_groups(const Mat16 &A) {
    std::vector<std::vector<int>> sup(A.rows);
    std::vector<int> order, copies;
    for (int r = 0; r < A.rows; ++r) {
        for (int c = 0; c < A.cols; ++c)
            if (A.at(r, c)) sup[r].push_back(c);
        // rows with no coefficient join the table groups and are written as zeros
        if (sup[r].size() == 1 && A.at(r, sup[r][0]) == 1) copies.push_back(r);
        else order.push_back(r);
    }
    // rows with the same support side by side: a group reads few columns
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sup[a] < sup[b]; });
    std::vector<Grp> gs;
    for (size_t i = 0; i < order.size(); i += kRows) {
        Grp g;
        std::set<int> cs;
        for (size_t j = i; j < order.size() && j < i + kRows; ++j) {
            g.rows.push_back(static_cast<uint32_t>(order[j]));
            cs.insert(sup[order[j]].begin(), sup[order[j]].end());
        }
        g.cols.assign(cs.begin(), cs.end());
        for (uint32_t r : g.rows) {
            std::vector<uint16_t> v;
            for (uint32_t c : g.cols) v.push_back(A.at(static_cast<int>(r), static_cast<int>(c)));
            g.coef.push_back(std::move(v));
        }
        gs.push_back(std::move(g));
    }
    order_columns(gs);
    for (size_t i = 0; i < copies.size(); i += kCopyRows) {
        Grp g;
        g.copy = true;
        for (size_t j = i; j < copies.size() && j < i + kCopyRows; ++j) {
            g.rows.push_back(static_cast<uint32_t>(copies[j]));
            g.cols.push_back(static_cast<uint32_t>(sup[copies[j]][0]));
        }
        gs.push_back(std::move(g));
    }
    return gs;
}

// Operations per lane chunk of 32 symbols: per column its permutes and
// transposes, combinations and two XORs per row plane; per row the output.
long group_ops(const Grp &g) {
    if (g.copy) return 0;
    return static_cast<long>(g.cols.size()) * (16 + 72 + 44 + 32 * static_cast<long>(g.rows.size())) +
           static_cast<long>(g.rows.size()) * (72 + 16);
}

long estimate_ops(const std::vector<Grp> &gs) {
    long ops = 0;
    for (const Grp &g : gs) ops += group_ops(g);
    return ops;
}

void emit_load(std::ostringstream &o, size_t j, uint32_t col) {
    o << "  const u32x4";
    for (int k = 0; k < 4; ++k)
        o << (k ? "," : "") << " x" << j << "_" << k << " = *(const u32x4 *)(in + (u64)" << col << "u * ld + off + "
          << 1024 * k << "u)";
    o << ";\n";
}

void emit_table_group(std::ostringstream &o, int gi, const Grp &G) {
    const int n = static_cast<int>(G.rows.size());
    o << "__device__ __forceinline__ void g" << gi
      << "(const unsigned char *in, u64 ld, unsigned char *out, u64 old, u64 off) {\n"
      << "  asm volatile(\"\" : \"+s\"(ld), \"+s\"(old));\n";
    for (int r = 0; r < n; ++r) {
        o << "  u32";
        for (int i = 0; i < 16; ++i) o << (i ? "," : "") << " q" << r << "_" << i << " = 0u";
        o << ";\n";
    }
    const size_t nc = G.cols.size();
    if (nc) emit_load(o, 0, G.cols[0]);
    for (size_t j = 0; j < nc; ++j) {
        if (j + 1 < nc) emit_load(o, j + 1, G.cols[j + 1]);
        o << "  {\n";
        // planes 0-7 from the low bytes, 8-15 from the high bytes
        for (int h = 0; h < 2; ++h) {
            o << "    u32";
            for (int i = 0; i < 8; ++i) {
                const int k = i / 2;   // piece
                const char *a = i % 2 ? ".z" : ".x", *b = i % 2 ? ".w" : ".y";
                o << (i ? "," : "") << " P" << (8 * h + i) << " = " << (h ? "HIB(" : "LOB(") << "x" << j << "_" << k
                  << b << ", x" << j << "_" << k << a << ")";
            }
            o << ";\n";
        }
        o << "    TR8(P0, P1, P2, P3, P4, P5, P6, P7)\n    TR8(P8, P9, P10, P11, P12, P13, P14, P15)\n";
        // output plane i of row r: XOR over nibbles g of the combination
        // mask_g of planes 4g .. 4g + 3
        struct Eq { int r, i; std::vector<std::pair<int, unsigned>> terms; };
        std::vector<Eq> eqs;
        std::set<std::pair<int, unsigned>> need;
        for (int r = 0; r < n; ++r) {
            const uint16_t c = G.coef[r][j];
            if (!c) continue;
            uint16_t colbits[16];
            for (int t = 0; t < 16; ++t) colbits[t] = mul(c, static_cast<uint16_t>(1u << t));
            for (int i = 0; i < 16; ++i) {
                Eq e{r, i, {}};
                for (int g = 0; g < 4; ++g) {
                    unsigned m = 0;
                    for (int t = 0; t < 4; ++t)
                        if ((colbits[4 * g + t] >> i) & 1) m |= 1u << t;
                    if (m) {
                        e.terms.push_back({g, m});
                        need.insert({g, m});
                    }
                }
                if (!e.terms.empty()) eqs.push_back(std::move(e));
            }
        }
        auto name = [](int g, unsigned m) {
            std::ostringstream s;
            if (popc(m) == 1) s << "P" << (4 * g + __builtin_ctz(m));
            else s << "C" << g << "_" << m;
            return s.str();
        };
        std::set<std::pair<int, unsigned>> made;
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
            size_t t = 0;
            for (; t + 1 < e.terms.size(); t += 2)
                o << "    " << q << " = X3(" << q << ", " << name(e.terms[t].first, e.terms[t].second) << ", "
                  << name(e.terms[t + 1].first, e.terms[t + 1].second) << ");\n";
            if (t < e.terms.size()) o << "    " << q << " ^= " << name(e.terms[t].first, e.terms[t].second) << ";\n";
        }
        o << "  }\n";
    }
    for (int r = 0; r < n; ++r) {
        o << "  {\n    TR8(";
        for (int i = 0; i < 8; ++i) o << (i ? ", " : "") << "q" << r << "_" << i;
        o << ")\n    TR8(";
        for (int i = 8; i < 16; ++i) o << (i > 8 ? ", " : "") << "q" << r << "_" << i;
        o << ")\n    unsigned char *d = out + (u64)" << G.rows[r] << "u * old + off;\n";
        for (int k = 0; k < 4; ++k) {
            // piece k: symbols 8k .. 8k + 7 = low / high byte dwords 2k, 2k + 1
            o << "    ST(d + " << 1024 * k << "u, u32x4{";
            for (int h = 0; h < 2; ++h) {
                const int i = 2 * k + h;
                o << (h ? ", " : "") << "MLO(q" << r << "_" << (8 + i) << ", q" << r << "_" << i << "), MHI(q" << r
                  << "_" << (8 + i) << ", q" << r << "_" << i << ")";
            }
            o << "});\n";
        }
        o << "  }\n";
    }
    o << "}\n";
}

void emit_copy_group(std::ostringstream &o, int gi, const Grp &G) {
    o << "__device__ __forceinline__ void g" << gi
      << "(const unsigned char *in, u64 ld, unsigned char *out, u64 old, u64 off) {\n"
      << "  asm volatile(\"\" : \"+s\"(ld), \"+s\"(old));\n";
    for (size_t i = 0; i < G.rows.size(); ++i) {
        o << "  { const unsigned char *p = in + (u64)" << G.cols[i] << "u * ld + off;\n"
          << "    unsigned char *d = out + (u64)" << G.rows[i] << "u * old + off;\n";
        for (int k = 0; k < 4; ++k)
            o << "    const u32x4 v" << k << " = *(const u32x4 *)(p + " << 1024 * k << "u);\n";
        for (int k = 0; k < 4; ++k) o << "    ST(d + " << 1024 * k << "u, v" << k << ");\n";
        o << "  }\n";
    }
    o << "}\n";
}

// The last s mod 16 bytes of every row: one lane per symbol.
void emit_tail(std::ostringstream &o, int gi, const Grp &G) {
    const size_t nr = G.rows.size(), nc = G.copy ? 1 : G.cols.size();
    o << "__constant__ u32 tr" << gi << "[" << nr << "] = {";
    for (size_t r = 0; r < nr; ++r) o << (r ? ", " : "") << G.rows[r] << "u";
    o << "};\n__constant__ u32 tc" << gi << "[" << nr * nc << "] = {";
    for (size_t r = 0; r < nr; ++r)
        for (size_t c = 0; c < nc; ++c) {
            // per (row, column): input block | coefficient << 16
            const uint32_t col = G.copy ? G.cols[r] : G.cols[c];
            const uint32_t coef = G.copy ? 1u : G.coef[r][c];
            o << (r + c ? ", " : "") << (col | coef << 16) << "u";
        }
    o << "};\n__device__ __noinline__ void b" << gi
      << "(const unsigned char *in, u64 ld, unsigned char *out, u64 old, u64 pos) {\n"
      << "#pragma unroll 1\n  for (u32 r = 0; r < " << nr << "u; ++r) {\n    u32 acc = 0u;\n"
      << "#pragma unroll 1\n    for (u32 c = 0; c < " << nc << "u; ++c) {\n"
      << "      const u32 e = tc" << gi << "[r * " << nc << "u + c];\n"
      << "      acc ^= gm16(e >> 16, *(const unsigned short *)(in + (u64)(e & 0xFFFFu) * ld + pos));\n    }\n"
      << "    *(unsigned short *)(out + (u64)tr" << gi << "[r] * old + pos) = (unsigned short)acc;\n  }\n}\n";
}

}  // namespace

namespace {

// The kernel source over the row groups gs (their functions, byte tails and
// the tile loop).
std::string emit_source(const std::vector<Grp> &gs) {
    std::ostringstream o;
    // x^16 reduced: x^12 + x^3 + x + 1
    o << "#define POLY16 " << mul(0x8000, 2) << "u\n" << kPrelude16;
    for (size_t g = 0; g < gs.size(); ++g) {
        if (gs[g].copy) emit_copy_group(o, static_cast<int>(g), gs[g]);
        else emit_table_group(o, static_cast<int>(g), gs[g]);
        emit_tail(o, static_cast<int>(g), gs[g]);
    }
    const int G = static_cast<int>(gs.size());
    // Tiles 0 .. nfull-1 are the full 4096-byte tiles; when s16 (s rounded
    // down to 16) is not a multiple of 4096, tile nfull is the window
    // [s16 - 4096, s16) overlapping the one before.  The (s - s16) / 2
    // symbols after s16 are done one per lane by the wave of the last tile.
    o << "extern \"C\" __global__ __launch_bounds__(" << 64 * kWaves << ") void pmbs16(BsArgs a) {\n"
      << "  const u32 wave = threadIdx.x / 64, lane = threadIdx.x % 64;\n"
      << "  const u32 xcd = blockIdx.x % 8u, slot = blockIdx.x / 8u;\n"
      << "  const u32 per = (a.ntiles + 7u) / 8u, t0 = xcd * per;\n"
      << "  const u32 t1 = t0 + per < a.ntiles ? t0 + per : a.ntiles;\n"
      << "  const u32 G = " << G << "u;\n"
      << "  for (u32 g = slot % G; g < G; g += a.P) {\n"
      << "    const u32 R = a.P >= G ? (a.P - 1u - g) / G + 1u : 1u;\n"
      << "    const u32 r = a.P >= G ? slot / G : 0u;\n"
      << "    const u64 s16 = a.s & ~15ull;\n"
      << "    for (u32 t = t0 + r * " << kWaves << "u + wave; t < t1; t += R * " << kWaves << "u) {\n"
      << "      const u64 tile = t < a.nfull ? (u64)t * " << kTile << "u : s16 - " << kTile << "u;\n"
      << "      switch (g) {\n";
    for (int g = 0; g < G; ++g) o << "        case " << g << ": g" << g << "(a.in, a.ld, a.out, a.old, tile + lane * 16u); break;\n";
    o << "      }\n      if (t == a.ntiles - 1u && s16 + 2u * lane < a.s) {\n        switch (g) {\n";
    for (int g = 0; g < G; ++g)
        o << "          case " << g << ": b" << g << "(a.in, a.ld, a.out, a.old, s16 + 2u * lane); break;\n";
    o << "        }\n      }\n    }\n    if (a.P >= G) break;\n  }\n}\n";
    return o.str();
}

std::unique_ptr<BsProgram> make_part(std::vector<Grp> gs) {
    auto bp = std::make_unique<BsProgram>();
    bp->ngroups = static_cast<int>(gs.size());
    bp->tile_bytes = kTile;
    bp->fn_name[BS_SINGLE] = "pmbs16";
    bp->est_ops = estimate_ops(gs);
    bp->k[BS_SINGLE].source = emit_source(gs);
    return bp;
}

}  // namespace

std::vector<std::unique_ptr<BsProgram>> bs16_generate_parts(const Mat16 &A) {
    std::vector<Grp> gs = make_groups(A);
    const long est = estimate_ops(gs);
    std::vector<std::unique_ptr<BsProgram>> parts;
    if (gs.empty() || est > kBs16MaxParts * kBs16PartOps) return parts;   // left to the table kernel
    // consecutive groups (rows in support order, so groups that read the
    // same columns stay in one part) of about est / np operations each
    const long np = est <= kBsMaxOps ? 1 : kBs16MaxParts;
    std::vector<Grp> cur;
    long done = 0;
    for (size_t g = 0; g < gs.size(); ++g) {
        done += group_ops(gs[g]);
        cur.push_back(std::move(gs[g]));
        const long cut = est * (static_cast<long>(parts.size()) + 1) / np;
        if (static_cast<long>(parts.size()) + 1 < np && done >= cut) {
            parts.push_back(make_part(std::move(cur)));
            cur.clear();
        }
    }
    if (!cur.empty()) parts.push_back(make_part(std::move(cur)));
    if (const char *dump = getenv("PMRC_BS_DUMP")) {   // debugging aid: keep the generated sources
        for (size_t i = 0; i < parts.size(); ++i) {
            const std::string path = parts.size() == 1 ? std::string(dump) : std::string(dump) + ".part" + std::to_string(i);
            if (FILE *f = fopen(path.c_str(), "w")) {
                fputs(parts[i]->k[BS_SINGLE].source.c_str(), f);
                fclose(f);
            }
        }
    }
    return parts;
}

std::unique_ptr<BsProgram> bs16_generate(const Mat16 &A) {
    std::vector<std::unique_ptr<BsProgram>> parts = bs16_generate_parts(A);
    if (parts.size() == 1) return std::move(parts[0]);
    // no single kernel: the whole matrix's group count and size, no source
    std::vector<Grp> gs = make_groups(A);
    auto bp = std::make_unique<BsProgram>();
    bp->ngroups = static_cast<int>(gs.size());
    bp->tile_bytes = kTile;
    bp->fn_name[BS_SINGLE] = "pmbs16";
    bp->est_ops = estimate_ops(gs);
    return bp;
}

}  // namespace w16
}  // namespace pmrc
