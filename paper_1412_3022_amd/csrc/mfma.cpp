// Host side of the matrix-core region product: the GF(2) expansion of a
// GF(2^8) matrix, laid out as the A operands of the kernel in mfma.hip.
#include "mfma.hpp"

#include "gf256.hpp"

namespace pmrc {

// Operand layout (both operands of v_mfma_scale_f32_32x32x64_f8f6f4 with
// 4-bit elements): lane l holds row (A) or column (B) l % 32 and the 32
// elements of K half kb = l / 32, 8 per dword, element 8q + t in nibble t of
// dword q.  The kernel builds B from a dword D whose byte j is input block
// 4 kb + j of the chunk (all at one byte position): dword q is D masked to
// bit q % 2 of every nibble (q = 0, 1) or D >> 2 masked the same way (q = 2,
// 3).  So element (q, t) is bit 4t + q of D, block 4 kb + (4t + q) / 8, bit
// (4t + q) % 8, and it reads 0.5 (even q) or 1.0 (odd q) when the bit is
// set.  A uses the same correspondence with entries 2.0 (even q) or 1.0
// (odd q), so every product of two set bits is exactly 1.0.
//
// Result layout: lane l holds column l % 32 and, in accumulator i, row
// 8 (i / 4) + 4 (l / 32) + i % 4.  Bit-matrix row m of a tile is therefore
// given to output row 2 h + q / 2 and bit 4 (q % 2) + t of that row, with
// q = m / 8, h = (m / 4) % 2, t = m % 4, so that accumulators 0..7 of a lane
// are bits 0..7 of output row 2 h and 8..15 those of row 2 h + 1.
MfmaProgram build_mfma_program(const Mat &A, const std::vector<int> &in_map, const std::vector<int> &rows) {
    MfmaProgram P;
    const uint32_t R = static_cast<uint32_t>(rows.empty() ? A.rows : static_cast<int>(rows.size()));
    const uint32_t C = static_cast<uint32_t>(A.cols);
    auto mrow = [&](uint32_t r) { return rows.empty() ? static_cast<int>(r) : rows[r]; };   // tile row -> matrix row
    // whole M blocks: the kernel runs every tile of a block without a check
    P.nmtiles = (R + kMfRowsPerTile - 1) / kMfRowsPerTile;
    P.nmtiles = (P.nmtiles + kMfTilePad - 1) / kMfTilePad * kMfTilePad;
    P.nchunks = (C + kMfColsPerChunk - 1) / kMfColsPerChunk;
    const size_t abits = static_cast<size_t>(P.nmtiles) * P.nchunks * kMfTileWords;
    P.cols_off = static_cast<uint32_t>(abits);
    P.rows_off = P.cols_off + P.nchunks * kMfColsPerChunk;
    P.words.assign(P.rows_off + P.nmtiles * kMfRowsPerTile, 0u);
    // bit i of c * 2^j, per coefficient value
    for (uint32_t mt = 0; mt < P.nmtiles; ++mt)
        for (uint32_t kc = 0; kc < P.nchunks; ++kc) {
            uint32_t *tile = &P.words[(static_cast<size_t>(mt) * P.nchunks + kc) * kMfTileWords];
            for (uint32_t l = 0; l < 64; ++l) {
                const uint32_t m = l % 32, kb = l / 32;
                const uint32_t qm = m / 8, h = (m / 4) % 2, tm = m % 4;
                const uint32_t r = mt * kMfRowsPerTile + 2 * h + qm / 2, bit = 4 * (qm % 2) + tm;
                if (r >= R) continue;
                for (uint32_t q = 0; q < 4; ++q)
                    for (uint32_t t = 0; t < 8; ++t) {
                        const uint32_t beta = 4 * t + q;
                        const uint32_t c = kc * kMfColsPerChunk + 4 * kb + beta / 8, j = beta % 8;
                        if (c >= C) continue;
                        const uint8_t a = A.at(mrow(r), static_cast<int>(c));
                        if (!a) continue;
                        if ((gmul(a, static_cast<uint8_t>(1u << j)) >> bit) & 1u)
                            tile[l * 4 + q] |= (q % 2 ? 0x2u : 0x4u) << (4 * t);   // 1.0 or 2.0 in e2m1
                    }
            }
        }
    for (uint32_t c = 0; c < P.nchunks * kMfColsPerChunk; ++c)
        P.words[P.cols_off + c] = c < C ? static_cast<uint32_t>(in_map.empty() ? c : in_map[c]) : 0u;
    for (uint32_t r = 0; r < P.nmtiles * kMfRowsPerTile; ++r)
        P.words[P.rows_off + r] = r < R ? static_cast<uint32_t>(mrow(r)) : kMfNoRow;
    return P;
}

}  // namespace pmrc
