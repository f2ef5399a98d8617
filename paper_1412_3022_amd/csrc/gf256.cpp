#include "gf256.hpp"

#include <algorithm>

namespace pmrc {

static uint8_t clmul_reduce(unsigned a, unsigned b) {
    unsigned r = 0;
    for (int i = 0; i < 8; ++i)
        if (b & (1u << i)) r ^= a << i;
    for (int i = 14; i >= 8; --i)
        if (r & (1u << i)) r ^= 0x11Du << (i - 8);
    return static_cast<uint8_t>(r);
}

GF::GF() {
    for (int a = 0; a < 256; ++a)
        for (int b = 0; b < 256; ++b) mul_t[a][b] = clmul_reduce(a, b);
    inv_t[0] = 0;
    for (int a = 1; a < 256; ++a)
        for (int b = 1; b < 256; ++b)
            if (mul_t[a][b] == 1) { inv_t[a] = static_cast<uint8_t>(b); break; }
    uint8_t p = 1;
    for (int e = 0; e < 255; ++e) { pow_t[e] = p; p = mul_t[p][2]; }
}

const GF &GF::get() {
    static const GF gf;
    return gf;
}

uint8_t gpow(long e) {
    long r = e % 255;
    if (r < 0) r += 255;
    return GF::get().pow_t[r];
}

Mat Mat::identity(int n) {
    Mat I(n, n);
    for (int i = 0; i < n; ++i) I.at(i, i) = 1;
    return I;
}

Mat matmul(const Mat &A, const Mat &B) {
    Mat C(A.rows, B.cols);
    const GF &gf = GF::get();
    for (int i = 0; i < A.rows; ++i)
        for (int t = 0; t < A.cols; ++t) {
            uint8_t a = A.at(i, t);
            if (!a) continue;
            const uint8_t *mrow = gf.mul_t[a];
            const uint8_t *brow = B.row(t);
            uint8_t *crow = &C.v[static_cast<size_t>(i) * C.cols];
            for (int j = 0; j < B.cols; ++j) crow[j] ^= mrow[brow[j]];
        }
    return C;
}

bool invert(const Mat &A, Mat &out) {
    const int n = A.rows;
    if (A.cols != n) return false;
    Mat W = A;
    out = Mat::identity(n);
    const GF &gf = GF::get();
    for (int c = 0; c < n; ++c) {
        int p = c;
        while (p < n && W.at(p, c) == 0) ++p;
        if (p == n) return false;
        if (p != c) {
            std::swap_ranges(W.v.begin() + static_cast<long>(p) * n, W.v.begin() + static_cast<long>(p + 1) * n,
                             W.v.begin() + static_cast<long>(c) * n);
            std::swap_ranges(out.v.begin() + static_cast<long>(p) * n, out.v.begin() + static_cast<long>(p + 1) * n,
                             out.v.begin() + static_cast<long>(c) * n);
        }
        // columns left of c of W are already unit columns: only j >= c change
        const uint8_t *scale = gf.mul_t[gf.inv_t[W.at(c, c)]];
        uint8_t *wc = W.row(c), *oc = out.row(c);
        for (int j = c; j < n; ++j) wc[j] = scale[wc[j]];
        for (int j = 0; j < n; ++j) oc[j] = scale[oc[j]];
        for (int r = 0; r < n; ++r) {
            uint8_t *wr = W.row(r), *orow = out.row(r);
            const uint8_t f = wr[c];
            if (r == c || !f) continue;
            const uint8_t *fm = gf.mul_t[f];
            for (int j = c; j < n; ++j) wr[j] ^= fm[wc[j]];
            for (int j = 0; j < n; ++j) orow[j] ^= fm[oc[j]];
        }
    }
    return true;
}

std::vector<int> independent_rows(const Mat &A, int want) {
    // Keep an echelon basis; reduce each candidate against it.
    const GF &gf = GF::get();
    std::vector<std::vector<uint8_t>> basis;
    std::vector<int> lead, kept;
    for (int r = 0; r < A.rows && static_cast<int>(kept.size()) < want; ++r) {
        std::vector<uint8_t> v(A.row(r), A.row(r) + A.cols);
        for (size_t b = 0; b < basis.size(); ++b) {
            uint8_t f = v[lead[b]];
            if (!f) continue;
            const uint8_t *fm = gf.mul_t[f];
            for (int j = 0; j < A.cols; ++j) v[j] ^= fm[basis[b][j]];
        }
        int l = 0;
        while (l < A.cols && v[l] == 0) ++l;
        if (l == A.cols) continue;
        const uint8_t *sm = gf.mul_t[gf.inv_t[v[l]]];
        for (int j = 0; j < A.cols; ++j) v[j] = sm[v[j]];
        // keep the basis reduced in column l
        for (size_t b = 0; b < basis.size(); ++b) {
            uint8_t f = basis[b][l];
            if (!f) continue;
            const uint8_t *fm = gf.mul_t[f];
            for (int j = 0; j < A.cols; ++j) basis[b][j] ^= fm[v[j]];
        }
        basis.push_back(std::move(v));
        lead.push_back(l);
        kept.push_back(r);
    }
    return kept;
}

Mat select_rows(const Mat &A, const std::vector<int> &idx) {
    Mat S(static_cast<int>(idx.size()), A.cols);
    for (size_t i = 0; i < idx.size(); ++i)
        std::copy(A.row(idx[i]), A.row(idx[i]) + A.cols, S.v.begin() + static_cast<long>(i) * A.cols);
    return S;
}

}  // namespace pmrc
