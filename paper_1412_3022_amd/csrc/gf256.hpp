// GF(2^8) arithmetic and small dense matrices for the host (init) phase.
//
// Field: polynomial x^8 + x^4 + x^3 + x^2 + 1 (0x11D), generator g = 2, the
// default GF(2^8) of GF-Complete that the paper's implementation uses
// (Section 3.3, paragraph on the computational check; Section 4).
// Products come from a full 256 x 256 table filled by carry-less
// multiplication with reduction; inverses from a search of that table.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace pmrc {

struct GF {
    uint8_t mul_t[256][256];
    uint8_t inv_t[256];
    uint8_t pow_t[255];   // g^e, e in [0, 255)
    GF();
    static const GF &get();
};

inline uint8_t gmul(uint8_t a, uint8_t b) { return GF::get().mul_t[a][b]; }
inline uint8_t ginv(uint8_t a) { return GF::get().inv_t[a]; }
inline uint8_t gdiv(uint8_t a, uint8_t b) { return gmul(a, ginv(b)); }
uint8_t gpow(long e);

// Row-major dense matrix over GF(2^8).
struct Mat {
    int rows = 0, cols = 0;
    std::vector<uint8_t> v;
    Mat() = default;
    Mat(int r, int c) : rows(r), cols(c), v(static_cast<size_t>(r) * c, 0) {}
    uint8_t &at(int r, int c) { return v[static_cast<size_t>(r) * cols + c]; }
    uint8_t at(int r, int c) const { return v[static_cast<size_t>(r) * cols + c]; }
    const uint8_t *row(int r) const { return v.data() + static_cast<size_t>(r) * cols; }
    uint8_t *row(int r) { return v.data() + static_cast<size_t>(r) * cols; }
    static Mat identity(int n);
};

Mat matmul(const Mat &A, const Mat &B);
// Inverse of a square matrix; false when singular.
bool invert(const Mat &A, Mat &out);
// Rows of A (by index, in order) picked greedily: a row is kept when it is
// independent of the rows kept before it.  Stops after `want` rows.
std::vector<int> independent_rows(const Mat &A, int want);
Mat select_rows(const Mat &A, const std::vector<int> &idx);

}  // namespace pmrc
