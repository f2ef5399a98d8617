// Dense region products on the matrix cores (mfma.hip, host side in
// mfma.cpp): a GF(2^8) matrix A (R x C) becomes its GF(2) expansion, the
// 8R x 8C bit matrix whose entry ((r, i), (c, j)) is bit i of A[r][c] * 2^j,
// and out = A in is, bit plane by bit plane, the parity of an integer
// product of that bit matrix with the bits of the input bytes.  The integer
// product runs on v_mfma_scale_f32_32x32x64_f8f6f4 with 4-bit float
// operands, exact in f32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

// One M tile is 32 rows of the bit matrix: 4 output rows of 8 bits.  One K
// chunk is 64 of its columns: 8 input blocks of 8 bits.
constexpr uint32_t kMfRowsPerTile = 4;
constexpr uint32_t kMfColsPerChunk = 8;
constexpr uint32_t kMfTileWords = 64 * 4;   // A operand of one (M tile, K chunk): 4 dwords per lane
constexpr uint32_t kMfNoRow = 0xFFFFFFFFu;
// The tile count is padded to a multiple of this (the most M tiles a
// work-group holds).
constexpr uint32_t kMfTilePad = 4;
// A work-group stages the A operands of its M tiles for every K chunk in
// LDS (1 KiB per tile and chunk): 4 tiles up to 39 chunks, 2 tiles up to
// 64 chunks (512 input blocks, 128 KiB).
constexpr uint32_t kMfMaxChunks = 64;

struct PmkMfma {
    const uint8_t *in;       // input block c at in + c * in_ld
    uint64_t in_ld;
    uint8_t *out;            // output row r at out + r * out_ld
    uint64_t out_ld;
    uint64_t s;              // bytes per block
    const uint32_t *abits;   // [nmtiles][nchunks][64 lanes][4 dwords]
    const uint32_t *cols;    // nchunks * 8 input block ids (padding: any valid id)
    const uint32_t *rows;    // nmtiles * 4 output row ids (kMfNoRow: not written)
    uint32_t nmtiles, nchunks;
    // set by pmk_mfma: M blocks (the tiles of one work-group), position
    // blocks (the bytes of one wave), position blocks per wave
    uint32_t nmblocks, npblocks, pq, pad;
};

// The kernel addresses input bytes as in plus a 32-bit offset: all in_n
// input blocks must end within 4 GiB of in (the caller checks).
inline bool mf_span_ok(uint64_t in_ld, uint64_t s, uint64_t in_n) {
    return in_n > 0 && s < (uint64_t(1) << 32) && (in_n - 1) * in_ld < (uint64_t(1) << 32) - s;
}

// Launches the kernel for h (the first 10 fields set, the input within
// mf_span_ok); hipErrorInvalidValue for more than kMfMaxChunks chunks, a
// tile count not a multiple of kMfTilePad or a grid past the launch
// limits.
extern "C" hipError_t pmk_mfma(const PmkMfma *h, hipStream_t st);

namespace pmrc {

struct Mat;

// The operand layout of a matrix for pmk_mfma: words = abits, then cols,
// then rows (offsets in words).
struct MfmaProgram {
    uint32_t nmtiles = 0, nchunks = 0;
    uint32_t cols_off = 0, rows_off = 0;
    std::vector<uint32_t> words;
};

// in_map: input block of each matrix column (empty = identity).  rows: the
// matrix rows to compute, each written to its own output row (empty = all;
// the other rows are left to the caller).
MfmaProgram build_mfma_program(const Mat &A, const std::vector<int> &in_map, const std::vector<int> &rows = {});

}  // namespace pmrc
