// A "program" is a small GF(2^8) matrix A (R x C) laid out for the region
// kernel: output rows are packed into groups of at most RG rows that read the
// same input columns, so the kernel can keep one accumulator per group row in
// registers and loop over the group's columns with no per-coefficient branch.
// Group record: kind, rows, columns, then word offsets of the column ids, of
// the 4-word table part, of the row ids and of the 1-word table part.
// Each (group, column, row) slot carries the split product tables of its
// coefficient: c*{0..7} (low 3 bits), c*{0,8,..,56} (middle 3 bits) and
// c*{0,64,128,192} (top 2 bits), packed so that a byte-permute lookup with the
// 3-, 3- and 2-bit fields of a source byte as selectors returns the three
// partial products (the split-table multiply of the paper's Section 4).
// Unit rows become plain copies and all-zero rows become zero fills.
#pragma once
#include <cstdint>
#include <vector>

#include "gf256.hpp"

namespace pmrc {

enum GroupKind : uint32_t { GROUP_TABLE = 0, GROUP_COPY = 1 };

constexpr int kTabWords = 5;       // words per coefficient slot
constexpr int kGroupWords = 8;     // words per group record
constexpr int kHeaderWords = 4;    // ngroups, rg, nrows_out, ncols_in

struct Program {
    int rg = 0;
    int rows = 0, cols = 0;      // matrix shape
    int ngroups = 0;
    long nnz = 0;                // nonzero coefficients of A
    long slots = 0;              // (group column x RG) slots the kernel evaluates
    long copies = 0;             // unit rows served by copy
    long col_reads = 0;          // sum over groups of columns read (input re-reads)
    long max_group_slots = 0;    // largest (columns x RG) of one group: its table footprint
    std::vector<uint32_t> blob;  // header | groups | row ids | column ids | tables
};

// in_map: input block index of each matrix column (empty = identity).
// skip: rows left out of every group (written by another kernel), or null.
Program build_program(const Mat &A, int rg, const std::vector<int> &in_map = {},
                      const std::vector<char> *skip = nullptr);

// Pack the tables of one coefficient (5 words) -- exposed for tests.
void pack_tables(uint8_t c, uint32_t out[kTabWords]);

}  // namespace pmrc
