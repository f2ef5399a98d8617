#include "program.hpp"

#include <algorithm>
#include <array>
#include <map>

namespace pmrc {
namespace {

struct Support {
    std::vector<uint64_t> bits;
    explicit Support(int ncols = 0) : bits((ncols + 63) / 64, 0) {}
    void set(int c) { bits[c >> 6] |= 1ull << (c & 63); }
    bool test(int c) const { return (bits[c >> 6] >> (c & 63)) & 1; }
    int count() const {
        int s = 0;
        for (uint64_t b : bits) s += __builtin_popcountll(b);
        return s;
    }
    int union_count(const Support &o) const {
        int s = 0;
        for (size_t i = 0; i < bits.size(); ++i) s += __builtin_popcountll(bits[i] | o.bits[i]);
        return s;
    }
    void merge(const Support &o) {
        for (size_t i = 0; i < bits.size(); ++i) bits[i] |= o.bits[i];
    }
    bool operator<(const Support &o) const { return bits < o.bits; }
};

struct Grp {
    uint32_t kind;
    std::vector<int> rows;
    Support sup;
};

}  // namespace

void pack_tables(uint8_t c, uint32_t out[kTabWords]) {
    auto word = [&](int e0, int e1, int e2, int e3) {
        return static_cast<uint32_t>(gmul(c, e0)) | static_cast<uint32_t>(gmul(c, e1)) << 8 |
               static_cast<uint32_t>(gmul(c, e2)) << 16 | static_cast<uint32_t>(gmul(c, e3)) << 24;
    };
    out[0] = word(0, 1, 2, 3);        // low 3 bits, entries 0..3
    out[1] = word(4, 5, 6, 7);        // low 3 bits, entries 4..7
    out[2] = word(0, 8, 16, 24);      // middle 3 bits, entries 0..3
    out[3] = word(32, 40, 48, 56);    // middle 3 bits, entries 4..7
    out[4] = word(0, 64, 128, 192);   // top 2 bits
}

Program build_program(const Mat &A, int rg, const std::vector<int> &in_map, const std::vector<char> *skip) {
    Program P;
    P.rg = rg;
    P.rows = A.rows;
    P.cols = A.cols;
    std::vector<Grp> groups;
    std::map<Support, std::vector<int>> buckets;
    std::vector<int> copy_rows;
    for (int r = 0; r < A.rows; ++r) {
        if (skip && (*skip)[static_cast<size_t>(r)]) continue;   // a row another kernel writes
        Support s(A.cols);
        int nz = 0, last = -1;
        for (int c = 0; c < A.cols; ++c)
            if (A.at(r, c)) { s.set(c); ++nz; last = c; }
        P.nnz += nz;
        if (nz == 1 && A.at(r, last) == 1) { copy_rows.push_back(r); continue; }
        buckets[s].push_back(r);
    }
    // Rows with identical support share a group (PM codes give whole classes
    // of such rows: one per position j inside the parity nodes).
    for (auto &kv : buckets) {
        const std::vector<int> &rows = kv.second;
        for (size_t i = 0; i < rows.size(); i += rg) {
            Grp g{GROUP_TABLE, {}, kv.first};
            for (size_t j = i; j < rows.size() && j < i + rg; ++j) g.rows.push_back(rows[j]);
            groups.push_back(std::move(g));
        }
    }
    // Greedy merge of partly filled groups when the union of their columns is
    // smaller than the columns they read apart (kernel cost ~ columns x RG).
    if (groups.size() <= 256) {
        while (true) {
            long best_gain = 0;
            size_t bi = 0, bj = 0;
            for (size_t i = 0; i < groups.size(); ++i)
                for (size_t j = i + 1; j < groups.size(); ++j) {
                    if (groups[i].rows.size() + groups[j].rows.size() > static_cast<size_t>(rg)) continue;
                    long gain = groups[i].sup.count() + groups[j].sup.count() - groups[i].sup.union_count(groups[j].sup);
                    if (gain > best_gain) { best_gain = gain; bi = i; bj = j; }
                }
            if (best_gain <= 0) break;
            groups[bi].rows.insert(groups[bi].rows.end(), groups[bj].rows.begin(), groups[bj].rows.end());
            groups[bi].sup.merge(groups[bj].sup);
            groups.erase(groups.begin() + static_cast<long>(bj));
        }
    }
    for (size_t i = 0; i < copy_rows.size(); i += rg) {
        Grp g{GROUP_COPY, {}, Support(A.cols)};
        for (size_t j = i; j < copy_rows.size() && j < i + rg; ++j) g.rows.push_back(copy_rows[j]);
        P.copies += static_cast<long>(g.rows.size());
        groups.push_back(std::move(g));
    }
    P.ngroups = static_cast<int>(groups.size());

    // Layout.  The tables of every coefficient value, packed once.
    static const std::vector<std::array<uint32_t, kTabWords>> packed = [] {
        std::vector<std::array<uint32_t, kTabWords>> t(256);
        for (int c = 0; c < 256; ++c) pack_tables(static_cast<uint8_t>(c), t[c].data());
        return t;
    }();
    std::vector<uint32_t> rec, rowids, colids, tab4, tab1;
    auto in_col = [&](int c) { return static_cast<uint32_t>(in_map.empty() ? c : in_map[c]); };
    for (const Grp &g : groups) {
        uint32_t row_off = static_cast<uint32_t>(rowids.size());
        for (int r : g.rows) rowids.push_back(static_cast<uint32_t>(r));
        uint32_t col_off = static_cast<uint32_t>(colids.size());
        uint32_t tab4_off = static_cast<uint32_t>(tab4.size());
        uint32_t tab1_off = static_cast<uint32_t>(tab1.size());
        uint32_t ncols = 0;
        if (g.kind == GROUP_COPY) {
            for (int r : g.rows) {
                int c = 0;
                while (!A.at(r, c)) ++c;
                colids.push_back(in_col(c));
            }
            ncols = static_cast<uint32_t>(g.rows.size());
        } else {
            std::vector<int> cols;
            for (int c = 0; c < A.cols; ++c)
                if (g.sup.test(c)) cols.push_back(c);
            // The kernel consumes columns in pairs; pad with a zero-coefficient
            // slot that rereads the last column.
            bool pad = cols.size() % 2 == 1;
            for (size_t ci = 0; ci < cols.size(); ++ci) {
                colids.push_back(in_col(cols[ci]));
                for (int r = 0; r < rg; ++r) {
                    uint8_t coef = r < static_cast<int>(g.rows.size()) ? A.at(g.rows[r], cols[ci]) : 0;
                    const uint32_t *t = packed[coef].data();
                    tab4.insert(tab4.end(), t, t + 4);
                    tab1.push_back(t[4]);
                }
            }
            if (pad) {
                colids.push_back(in_col(cols.back()));
                tab4.insert(tab4.end(), static_cast<size_t>(rg) * 4, 0u);
                tab1.insert(tab1.end(), static_cast<size_t>(rg), 0u);
            }
            ncols = static_cast<uint32_t>(cols.size() + (pad ? 1 : 0));
            P.slots += static_cast<long>(ncols) * rg;
            P.max_group_slots = std::max(P.max_group_slots, static_cast<long>(ncols) * rg);
            P.col_reads += ncols;
        }
        uint32_t r8[kGroupWords] = {g.kind, static_cast<uint32_t>(g.rows.size()), ncols, col_off,
                                    tab4_off, row_off, tab1_off, 0};
        rec.insert(rec.end(), r8, r8 + kGroupWords);
    }
    // Absolute word offsets.
    const uint32_t base_rows = kHeaderWords + static_cast<uint32_t>(rec.size());
    const uint32_t base_cols = base_rows + static_cast<uint32_t>(rowids.size());
    // 16 spare words after the column ids: kernels may fetch a fixed 16 ids.
    uint32_t base_tab4 = base_cols + static_cast<uint32_t>(colids.size()) + 16u;
    base_tab4 = (base_tab4 + 15u) & ~15u;  // 64-byte aligned tables
    uint32_t base_tab1 = base_tab4 + static_cast<uint32_t>(tab4.size());
    for (size_t g = 0; g < groups.size(); ++g) {
        rec[g * kGroupWords + 3] += base_cols;
        rec[g * kGroupWords + 4] += base_tab4;
        rec[g * kGroupWords + 5] += base_rows;
        rec[g * kGroupWords + 6] += base_tab1;
    }
    P.blob.assign(base_tab1 + tab1.size(), 0u);
    P.blob[0] = static_cast<uint32_t>(P.ngroups);
    P.blob[1] = static_cast<uint32_t>(rg);
    P.blob[2] = static_cast<uint32_t>(A.rows);
    P.blob[3] = static_cast<uint32_t>(A.cols);
    std::copy(rec.begin(), rec.end(), P.blob.begin() + kHeaderWords);
    std::copy(rowids.begin(), rowids.end(), P.blob.begin() + base_rows);
    std::copy(colids.begin(), colids.end(), P.blob.begin() + base_cols);
    std::copy(tab4.begin(), tab4.end(), P.blob.begin() + base_tab4);
    std::copy(tab1.begin(), tab1.end(), P.blob.begin() + base_tab1);
    return P;
}

}  // namespace pmrc
