// GF(2^16) codes (Section 3.3): field, construction, per-operation matrices,
// and the host side of the GF(2^16) region kernel (gf16.hip).
#include "gf16.hpp"

#include <algorithm>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <thread>

#include "gf16k.hpp"

namespace pmrc {
namespace w16 {
namespace {

constexpr uint32_t kPoly = 0x1100Bu;
constexpr int kOrder = 65535;

// exp[e] = g^e for e in [0, 2 * 65535) (so a sum of two logs indexes it),
// lg[a] = log_g a for a != 0
struct Field {
    std::vector<uint16_t> ex;
    std::vector<int32_t> lg;
    Field() : ex(2 * kOrder), lg(65536, -1) {
        uint32_t a = 1;
        for (int e = 0; e < kOrder; ++e) {
            ex[e] = ex[e + kOrder] = static_cast<uint16_t>(a);
            lg[a] = e;
            a <<= 1;
            if (a & 0x10000u) a ^= kPoly;
        }
    }
};

const Field &field() {
    static const Field f;
    return f;
}

// Gauss-Jordan on [A | I] in place; rows of the right half become the
// inverse.  Row updates run in the log domain: the pivot row's logarithms
// are taken once per pivot.
bool gauss_jordan(std::vector<uint16_t> &M, int n, int w) {
    const Field &F = field();
    std::vector<int32_t> plog(w);
    for (int c = 0; c < n; ++c) {
        int p = c;
        while (p < n && M[static_cast<size_t>(p) * w + c] == 0) ++p;
        if (p == n) return false;
        if (p != c)
            std::swap_ranges(M.begin() + static_cast<long>(p) * w, M.begin() + static_cast<long>(p + 1) * w,
                             M.begin() + static_cast<long>(c) * w);
        uint16_t *pr = M.data() + static_cast<size_t>(c) * w;
        const int32_t linv = (kOrder - F.lg[pr[c]]) % kOrder;
        for (int j = 0; j < w; ++j) {
            if (pr[j]) {
                plog[j] = F.lg[pr[j]] + linv;
                if (plog[j] >= kOrder) plog[j] -= kOrder;
                pr[j] = F.ex[plog[j]];
            } else {
                plog[j] = -1;
            }
        }
        for (int r = 0; r < n; ++r) {
            uint16_t *row = M.data() + static_cast<size_t>(r) * w;
            if (r == c || row[c] == 0) continue;
            const int32_t lf = F.lg[row[c]];
            for (int j = c; j < w; ++j)
                if (plog[j] >= 0) row[j] ^= F.ex[lf + plog[j]];
        }
    }
    return true;
}

bool subsets_invertible(const Mat16 &psi, int must) {
    const int n = psi.rows, d = psi.cols;
    std::vector<int> idx(d);
    std::iota(idx.begin(), idx.end(), 0);
    Mat16 S(d, d), Si;
    while (true) {
        if (must < 0 || std::find(idx.begin(), idx.end(), must) != idx.end()) {
            for (int i = 0; i < d; ++i)
                std::copy(psi.v.begin() + static_cast<long>(idx[i]) * d,
                          psi.v.begin() + static_cast<long>(idx[i] + 1) * d, S.v.begin() + static_cast<long>(i) * d);
            if (!invert(S, Si)) return false;
        }
        int i = d - 1;
        while (i >= 0 && idx[i] == n - d + i) --i;
        if (i < 0) return true;
        ++idx[i];
        for (int j = i + 1; j < d; ++j) idx[j] = idx[j - 1] + 1;
    }
}

bool distinct(std::vector<uint16_t> v) {
    std::sort(v.begin(), v.end());
    return std::adjacent_find(v.begin(), v.end()) == v.end();
}

// Sparse construction (Section 3.3) over GF(2^16): Phi = identity on top of
// the Cauchy rows 1 / (g^(i + alpha) + g^(j - 1)), Lambda_i = (g^(i + alpha)
// + 1) / (g^(i + alpha) + g^alpha) (1-based i, j).  At n = 2k the last node's
// Lambda becomes the first power of g that is new and keeps every helper
// set holding that node invertible.
int msr_sparse(int k, int n, Mat16 &psi, std::vector<uint16_t> &lam) {
    const int alpha = k - 1, d = 2 * alpha;
    if (n != 2 * k - 1 && n != 2 * k) return ST_EUNSUPPORTED;
    psi = Mat16(n, d);
    lam.assign(n, 0);
    const uint16_t ga = gpow(alpha);
    for (int i1 = 1; i1 <= n; ++i1) {
        const uint16_t xi = gpow(i1 + alpha);
        for (int j1 = 1; j1 <= alpha; ++j1) {
            uint16_t v = 0;
            if (i1 <= alpha) {
                v = i1 == j1 ? 1 : 0;
            } else {
                const uint16_t den = xi ^ gpow(j1 - 1);
                if (!den) return ST_EUNSUPPORTED;
                v = inv(den);
            }
            psi.at(i1 - 1, j1 - 1) = v;
        }
        if (!(xi ^ ga)) return ST_EUNSUPPORTED;
        lam[i1 - 1] = mul(xi ^ 1, inv(xi ^ ga));
        for (int j = 0; j < alpha; ++j) psi.at(i1 - 1, alpha + j) = mul(lam[i1 - 1], psi.at(i1 - 1, j));
    }
    if (n == 2 * k) {
        const int last = n - 1;
        bool found = false;
        for (int t = 0; t < kOrder && !found; ++t) {
            const uint16_t cand = gpow(t);
            if (std::find(lam.begin(), lam.begin() + last, cand) != lam.begin() + last) continue;
            lam[last] = cand;
            for (int j = 0; j < alpha; ++j) psi.at(last, alpha + j) = mul(cand, psi.at(last, j));
            found = subsets_invertible(psi, last);
        }
        if (!found) return ST_EUNSUPPORTED;
    }
    if (!distinct(lam) || !subsets_invertible(psi, -1)) return ST_EUNSUPPORTED;
    return ST_OK;
}

}  // namespace

uint16_t mul(uint16_t a, uint16_t b) {
    if (!a || !b) return 0;
    const Field &F = field();
    return F.ex[F.lg[a] + F.lg[b]];
}

uint16_t inv(uint16_t a) {
    if (!a) return 0;
    const Field &F = field();
    return F.ex[(kOrder - F.lg[a]) % kOrder];
}

uint16_t gpow(long e) {
    long r = e % kOrder;
    if (r < 0) r += kOrder;
    return field().ex[r];
}

Mat16 matmul(const Mat16 &A, const Mat16 &B) {
    Mat16 C(A.rows, B.cols);
    for (int i = 0; i < A.rows; ++i)
        for (int t = 0; t < A.cols; ++t) {
            const uint16_t a = A.at(i, t);
            if (!a) continue;
            for (int j = 0; j < B.cols; ++j) C.at(i, j) ^= mul(a, B.at(t, j));
        }
    return C;
}

bool invert(const Mat16 &A, Mat16 &out) {
    const int n = A.rows, w = 2 * n;
    if (A.cols != n) return false;
    std::vector<uint16_t> M(static_cast<size_t>(n) * w, 0);
    for (int i = 0; i < n; ++i) {
        std::copy(A.v.begin() + static_cast<long>(i) * n, A.v.begin() + static_cast<long>(i + 1) * n,
                  M.begin() + static_cast<long>(i) * w);
        M[static_cast<size_t>(i) * w + n + i] = 1;
    }
    if (!gauss_jordan(M, n, w)) return false;
    out = Mat16(n, n);
    for (int i = 0; i < n; ++i)
        std::copy(M.begin() + static_cast<long>(i) * w + n, M.begin() + static_cast<long>(i + 1) * w,
                  out.v.begin() + static_cast<long>(i) * n);
    return true;
}

int build_code(const CodeSpec &s, Code16 &c) {
    c = Code16();
    if (s.kind != KIND_MSR || s.construction != CONS_SPARSE || !s.x.empty()) return ST_EUNSUPPORTED;
    if (s.k < 2 || s.n < s.d + 1 || s.n > 65535) return ST_EINVAL;
    if (s.d != 2 * s.k - 2) return ST_EUNSUPPORTED;
    c.k = s.k; c.d = s.d; c.n = s.n;
    c.alpha = s.k - 1;
    c.B = s.k * c.alpha;
    c.systematic = s.systematic ? 1 : 0;
    int st = msr_sparse(s.k, s.n, c.psi, c.lambda);
    if (st != ST_OK) return st;
    c.L = index_msr(c.alpha);
    // linearization (Section 3.1): G[alpha i + j][L[l][j]] = Psi[i][l]
    c.G = Mat16(c.n * c.alpha, c.B);
    for (int i = 0; i < c.n; ++i)
        for (int j = 0; j < c.alpha; ++j)
            for (int l = 0; l < c.d; ++l) c.G.at(c.alpha * i + j, c.L[l * c.alpha + j]) ^= c.psi.at(i, l);
    if (c.systematic) {
        // G' = G inverse(G~), G~ the first B rows (Section 3.2)
        Mat16 top(c.B, c.B), topinv;
        std::copy(c.G.v.begin(), c.G.v.begin() + static_cast<long>(c.B) * c.B, top.v.begin());
        if (!invert(top, topinv)) return ST_ESINGULAR;
        c.Gsys = matmul(c.G, topinv);
        c.enc = Mat16(c.n * c.alpha - c.B, c.B);
        std::copy(c.Gsys.v.begin() + static_cast<long>(c.B) * c.B, c.Gsys.v.end(), c.enc.v.begin());
        for (int t = 0; t < c.n * c.alpha; ++t) c.node_map.push_back(t);
    } else {
        c.Gsys = c.G;
        c.enc = c.G;
        for (int t = 0; t < c.n * c.alpha; ++t) c.node_map.push_back(c.B + t);
    }
    return ST_OK;
}

Mat16 helper_row(const Code16 &c, int f) {
    Mat16 r(1, c.alpha);
    for (int a = 0; a < c.alpha; ++a) r.at(0, a) = c.psi.at(f, a);
    return r;
}

// [I | lambda_f I] inverse(Psi_H): the newcomer's alpha x d matrix (Section 2).
int newcomer_matrix(const Code16 &c, int f, const std::vector<int> &H, Mat16 &R) {
    const int d = c.d;
    if (static_cast<int>(H.size()) != d) return ST_EINVAL;
    Mat16 PH(d, d), PHinv;
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) PH.at(i, j) = c.psi.at(H[i], j);
    if (!invert(PH, PHinv)) return ST_ESINGULAR;
    R = Mat16(c.alpha, d);
    for (int a = 0; a < c.alpha; ++a)
        for (int j = 0; j < d; ++j) R.at(a, j) = PHinv.at(a, j) ^ mul(c.lambda[f], PHinv.at(c.alpha + a, j));
    return ST_OK;
}

// The inverse of the k alpha = B generator rows of the nodes K, node-major.
int decode_matrix(const Code16 &c, const std::vector<int> &K, Mat16 &D) {
    Mat16 rows(c.B, c.B);
    for (size_t i = 0; i < K.size(); ++i)
        for (int j = 0; j < c.alpha; ++j)
            std::copy(c.Gsys.v.begin() + static_cast<long>(K[i] * c.alpha + j) * c.B,
                      c.Gsys.v.begin() + static_cast<long>(K[i] * c.alpha + j + 1) * c.B,
                      rows.v.begin() + static_cast<long>(i * c.alpha + j) * c.B);
    return invert(rows, D) ? ST_OK : ST_ESINGULAR;
}

// The specific PM-MSR decode from the k nodes K as five factors over
// GF(2^16), the same factorization as for GF(2^8) (construct.hpp):
//   F[0] (k(k-1) x k alpha): Z_ij = y_i . phi_j, i != j, rows i-major;
//   F[1] (B x k(k-1)): P_ij, then Q_ij, of every pair i < j;
//   F[2] (2 alpha^2 x B): phi_i^t S1 and phi_i^t S2 for the first alpha nodes;
//   F[3] (B x 2 alpha^2): the message symbols from inverse(Phi_A);
//   F[4] (B x B): systematic codes only, X = G~ Z.
int specific_factors(const Code16 &c, const std::vector<int> &K, Mat16 F[kSpecificPasses]) {
    const int k = c.k, a = c.alpha, d = c.d, B = c.B;
    if (static_cast<int>(K.size()) != k) return ST_EINVAL;
    auto phi = [&](int i, int t) { return c.psi.at(K[i], t); };
    auto lam = [&](int i) { return c.lambda[K[i]]; };
    const int npairs = k * (k - 1) / 2;
    std::vector<std::vector<int>> zrow(k, std::vector<int>(k, -1)), pair_of(k, std::vector<int>(k, -1));
    Mat16 Zm(k * (k - 1), k * a);
    int zr = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            if (j == i) continue;
            zrow[i][j] = zr;
            for (int t = 0; t < a; ++t) Zm.at(zr, i * a + t) = phi(j, t);
            ++zr;
        }
    // Q_ij = cc (Z_ij + Z_ji), P_ij = lambda_j cc Z_ij + lambda_i cc Z_ji,
    // cc = 1 / (lambda_i + lambda_j)
    Mat16 A(B, k * (k - 1));
    int q = 0;
    for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j, ++q) {
            const uint16_t sum = lam(i) ^ lam(j);
            if (!sum) return ST_ESINGULAR;
            const uint16_t cc = inv(sum);
            pair_of[i][j] = pair_of[j][i] = q;
            A.at(q, zrow[i][j]) = mul(lam(j), cc);
            A.at(q, zrow[j][i]) = mul(lam(i), cc);
            A.at(npairs + q, zrow[i][j]) = cc;
            A.at(npairs + q, zrow[j][i]) = cc;
        }
    // phi_i^t S1 (S2) from the alpha values P_ij (Q_ij), j != i in order
    Mat16 Bm(2 * a * a, B);
    for (int i = 0; i < a; ++i) {
        Mat16 Fi(a, a), Fi_inv;
        std::vector<int> js;
        for (int j = 0; j < k; ++j)
            if (j != i) js.push_back(j);
        for (int r = 0; r < a; ++r)
            for (int t = 0; t < a; ++t) Fi.at(r, t) = phi(js[r], t);
        if (!invert(Fi, Fi_inv)) return ST_ESINGULAR;
        for (int b = 0; b < a; ++b)
            for (int r = 0; r < a; ++r) {
                const int qp = pair_of[i][js[r]];
                Bm.at(i * a + b, qp) = Fi_inv.at(b, r);
                Bm.at(a * a + i * a + b, npairs + qp) = Fi_inv.at(b, r);
            }
    }
    // S1 = inverse(Phi_A) U, S2 = inverse(Phi_A) V; symbol L[l][j] = M[l][j]
    Mat16 PhiA(a, a), PhiA_inv;
    for (int i = 0; i < a; ++i)
        for (int t = 0; t < a; ++t) PhiA.at(i, t) = phi(i, t);
    if (!invert(PhiA, PhiA_inv)) return ST_ESINGULAR;
    Mat16 Cm(B, 2 * a * a);
    std::vector<char> done(B, 0);
    for (int l = 0; l < d; ++l)
        for (int j = 0; j < a; ++j) {
            const int m = c.L[l * a + j];
            if (done[m]) continue;
            done[m] = 1;
            const int half = l < a ? 0 : 1, row = l % a;
            for (int i = 0; i < a; ++i) Cm.at(m, half * a * a + i * a + j) = PhiA_inv.at(row, i);
        }
    F[0] = std::move(Zm);
    F[1] = std::move(A);
    F[2] = std::move(Bm);
    F[3] = std::move(Cm);
    if (c.systematic) {
        Mat16 Gt(B, B);
        std::copy(c.G.v.begin(), c.G.v.begin() + static_cast<long>(B) * B, Gt.v.begin());
        F[4] = std::move(Gt);
    } else {
        F[4] = Mat16();
    }
    return ST_OK;
}

// Rows that are one input block times 1 (a decode's blocks that the nodes
// hold as they are: only the lost blocks are computed) form copy groups.
// The other rows form groups of kPm16Rows, each with the columns any of its
// rows reads (in the load order given below).  Rows are taken in the order of their
// supports (the sorted lists of columns they read), so rows that read the
// same columns share a group and its column records: in the linearized
// generator, the rows alpha i + j of all nodes i read the message symbols of
// column j of M.  This cuts the records of the k = 8 systematic encode from
// 392 to 98, and of the k = 64 non-systematic one from 487 760 to 75 612.
std::vector<std::shared_ptr<BsProgram>> Prog16::bitslice() {
    std::lock_guard<std::mutex> lk(mu);
    if (!bs_tried) {
        bs_tried = true;
        std::vector<std::unique_ptr<BsProgram>> parts = bs16_generate_parts(A);
        if (static_cast<int>(parts.size()) <= max_parts)
            for (std::unique_ptr<BsProgram> &b : parts) bs.push_back(std::move(b));
    }
    return bs;
}

Prog16::Prog16(const Mat16 &A_) : rows(A_.rows), cols(A_.cols), A(A_) {
    const int R = static_cast<int>(kPm16Rows);
    std::vector<std::vector<int>> sup(A.rows);
    std::vector<int> order, copies;
    for (int r = 0; r < A.rows; ++r) {
        for (int c = 0; c < A.cols; ++c)
            if (A.at(r, c)) sup[r].push_back(c);
        if (sup[r].size() == 1 && A.at(r, sup[r][0]) == 1) copies.push_back(r);
        else order.push_back(r);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return sup[a] < sup[b]; });
    const int nt = static_cast<int>(order.size()), nc = static_cast<int>(copies.size());
    const uint32_t ntable = static_cast<uint32_t>((nt + R - 1) / R), ncopy = static_cast<uint32_t>((nc + R - 1) / R);
    ngroups = ntable + ncopy;
    words.assign(kPm16Header + static_cast<size_t>(ngroups) * (2 + R), 0);
    words[0] = ngroups;
    std::vector<std::vector<int>> gcols(ntable);
    for (uint32_t g = 0; g < ntable; ++g) {
        const int i0 = static_cast<int>(g) * R, i1 = std::min(nt, i0 + R);
        std::vector<int> &cols_of = gcols[g];
        for (int i = i0; i < i1; ++i) cols_of.insert(cols_of.end(), sup[order[i]].begin(), sup[order[i]].end());
        std::sort(cols_of.begin(), cols_of.end());
        cols_of.erase(std::unique(cols_of.begin(), cols_of.end()), cols_of.end());
    }
    // A column that several groups read gets one position in all of their
    // record lists where it can (greedy, columns read by most groups first,
    // each at the first position free in all its groups; a group then reads
    // its columns in that order).  The groups of a tile run side by side on
    // one XCD, so the first read brings the column's tile into L2 and the
    // others find it there.
    {
        std::map<int, std::vector<uint32_t>> users;
        for (uint32_t g = 0; g < ntable; ++g)
            for (int c : gcols[g]) users[c].push_back(g);
        std::vector<int> byuse;
        for (auto &kv : users) byuse.push_back(kv.first);
        std::stable_sort(byuse.begin(), byuse.end(),
                         [&](int a, int b) { return users[a].size() > users[b].size(); });
        std::vector<std::set<int>> taken(ntable);
        std::map<int, int> step;
        for (int c : byuse) {
            int st = 0;
            for (;; ++st) {
                bool free = true;
                for (uint32_t g : users[c]) free &= !taken[g].count(st);
                if (free) break;
            }
            step[c] = st;
            for (uint32_t g : users[c]) taken[g].insert(st);
        }
        for (auto &cl : gcols)
            std::stable_sort(cl.begin(), cl.end(), [&](int a, int b) { return step[a] < step[b]; });
    }
    for (uint32_t g = 0; g < ntable; ++g) {
        const int i0 = static_cast<int>(g) * R, i1 = std::min(nt, i0 + R);
        const std::vector<int> &cols_of = gcols[g];
        const size_t first = words.size();
        for (int c : cols_of) {
            words.push_back(static_cast<uint32_t>(c));
            for (int i = 0; i < R; i += 2) {
                const uint32_t lo = i0 + i < i1 ? A.at(order[i0 + i], c) : 0;
                const uint32_t hi = i0 + i + 1 < i1 ? A.at(order[i0 + i + 1], c) : 0;
                words.push_back(lo | hi << 16);
            }
        }
        uint32_t *gd = &words[kPm16Header + static_cast<size_t>(g) * (2 + R)];
        gd[0] = static_cast<uint32_t>(first);
        gd[1] = static_cast<uint32_t>(cols_of.size());
        for (int i = 0; i < R; ++i) gd[2 + i] = i0 + i < i1 ? static_cast<uint32_t>(order[i0 + i]) : kPm16NoRow;
    }
    for (uint32_t q = 0; q < ncopy; ++q) {
        const int i0 = static_cast<int>(q) * R, i1 = std::min(nc, i0 + R);
        const size_t first = words.size();
        for (int i = 0; i < R; ++i) words.push_back(i0 + i < i1 ? static_cast<uint32_t>(sup[copies[i0 + i]][0]) : 0u);
        uint32_t *gd = &words[kPm16Header + static_cast<size_t>(ntable + q) * (2 + R)];
        gd[0] = static_cast<uint32_t>(first);
        gd[1] = kPm16CopyGroup;
        for (int i = 0; i < R; ++i) gd[2 + i] = i0 + i < i1 ? static_cast<uint32_t>(copies[i0 + i]) : kPm16NoRow;
    }
}

namespace {

// The split tables of every field element (layout in gf16k.hpp).
const std::vector<uint32_t> &tables() {
    static const std::vector<uint32_t> t = [] {
        static const uint32_t shift[6] = {0, 3, 6, 8, 11, 14}, values[6] = {8, 8, 4, 8, 8, 4};
        std::vector<uint32_t> w(static_cast<size_t>(65536) * kPm16TableWords, 0);
        for (uint32_t c = 0; c < 65536u; ++c) {
            uint32_t *e = &w[static_cast<size_t>(c) * kPm16TableWords];
            for (uint32_t p = 0; p < 6; ++p)
                for (uint32_t h = 0; h < 2; ++h)
                    for (uint32_t v = 0; v < values[p]; ++v) {
                        const uint32_t prod = mul(static_cast<uint16_t>(c), static_cast<uint16_t>(v << shift[p]));
                        e[4 * p + 2 * h + v / 4] |= ((prod >> (8 * h)) & 0xFFu) << (8 * (v % 4));
                    }
        }
        return w;
    }();
    return t;
}

std::mutex g_tab_mu;
std::map<int, DevCopy> &g_tab_dev = *new std::map<int, DevCopy>();

int table_ptr(hipStream_t user, const uint32_t **out) {
    const std::vector<uint32_t> &t = tables();
    const void *p = nullptr;
    int st = device_copy(g_tab_mu, g_tab_dev, t.data(), t.size() * sizeof(uint32_t), user, &p, false);
    if (st == ST_OK) *out = static_cast<const uint32_t *>(p);
    return st;
}

int prog_ptr(Prog16 &p, hipStream_t user, const uint32_t **out) {
    const void *d = nullptr;
    int st = device_copy(p.mu, p.dev, p.words.data(), p.words.size() * sizeof(uint32_t), user, &d);
    if (st == ST_OK) *out = static_cast<const uint32_t *>(d);
    return st;
}

}  // namespace

int resolve16(Ctx16 &c, int op, uint32_t failed, const uint32_t *ids, Prog16 **pe, size_t *in_n, size_t *out_n) {
    const Code16 &m = c.m;
    if ((op == OPK_HELPER || op == OPK_NEWCOMER) && failed >= static_cast<uint32_t>(m.n)) return ST_EINVAL;
    std::vector<int> list;
    if (op == OPK_NEWCOMER || op == OPK_DECODE) {
        if (!ids) return ST_EINVAL;
        list.assign(ids, ids + (op == OPK_NEWCOMER ? m.d : m.k));
        std::vector<int> sorted = list;
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return ST_EINVAL;
        for (int v : list)
            if (v < 0 || v >= m.n || (op == OPK_NEWCOMER && v == static_cast<int>(failed))) return ST_EINVAL;
    }
    std::lock_guard<std::mutex> lk(c.mu);
    switch (op) {
        case OPK_ENCODE:
            if (!c.enc) c.enc = std::make_unique<Prog16>(m.enc);
            *pe = c.enc.get();
            *in_n = static_cast<size_t>(m.B);
            *out_n = static_cast<size_t>(m.enc.rows);
            return ST_OK;
        case OPK_HELPER: {
            auto &p = c.helper[static_cast<int>(failed)];
            if (!p) p = std::make_unique<Prog16>(helper_row(m, static_cast<int>(failed)));
            *pe = p.get();
            *in_n = static_cast<size_t>(m.alpha);
            *out_n = 1;
            return ST_OK;
        }
        case OPK_NEWCOMER: {
            auto &p = c.newcomer[std::make_pair(static_cast<int>(failed), list)];
            if (!p) {
                Mat16 R;
                int st = newcomer_matrix(m, static_cast<int>(failed), list, R);
                if (st != ST_OK) return st;
                p = std::make_unique<Prog16>(R);
            }
            *pe = p.get();
            *in_n = static_cast<size_t>(m.d);
            *out_n = static_cast<size_t>(m.alpha);
            return ST_OK;
        }
        case OPK_DECODE: {
            auto &p = c.decode[list];
            if (!p) {
                Mat16 D;
                int st = decode_matrix(m, list, D);
                if (st != ST_OK) return st;
                p = std::make_unique<Prog16>(D);
            }
            *pe = p.get();
            *in_n = static_cast<size_t>(m.B);
            *out_n = static_cast<size_t>(m.B);
            return ST_OK;
        }
        default:
            return ST_EINVAL;
    }
}

int resolve_specific16(Ctx16 &c, const uint32_t *ids, Prog16 *pe[kSpecificPasses], int rows[kSpecificPasses],
                       int *npass) {
    const Code16 &m = c.m;
    if (!ids) return ST_EINVAL;
    std::vector<int> list(ids, ids + m.k), sorted = list;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return ST_EINVAL;
    for (int v : list)
        if (v < 0 || v >= m.n) return ST_EINVAL;
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.specific.find(list);
    if (it == c.specific.end()) {
        Mat16 F[kSpecificPasses];
        int st = specific_factors(m, list, F);
        if (st != ST_OK) return st;
        Ctx16::Specific sp;
        for (int p = 0; p < kSpecificPasses; ++p) {
            sp.F[p] = std::move(F[p]);
            if (sp.F[p].rows) {
                sp.prog[p] = std::make_unique<Prog16>(sp.F[p]);
                // one kernel at most: split kernels would cost minutes of
                // init per node set for passes that are short already
                sp.prog[p]->max_parts = 1;
            }
        }
        it = c.specific.emplace(list, std::move(sp)).first;
    }
    *npass = 0;
    while (*npass < kSpecificPasses && it->second.F[*npass].rows) {
        pe[*npass] = it->second.prog[*npass].get();
        rows[*npass] = it->second.F[*npass].rows;
        ++*npass;
    }
    return ST_OK;
}

const Mat16 *specific_factor16(Ctx16 &c, const uint32_t *ids, int which) {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.specific.find(std::vector<int>(ids, ids + c.m.k));
    return it == c.specific.end() ? nullptr : &it->second.F[which];
}

namespace {

// Side streams of the split kernels on one device, with the events that
// fork them from the caller's stream and join them back.
struct SideStreams {
    hipStream_t st[kBs16MaxParts - 1] = {};
    hipEvent_t fork = nullptr, join[kBs16MaxParts - 1] = {};
};
std::mutex g_side_mu;   // guards g_side and every fork / join sequence
std::map<int, SideStreams> &g_side = *new std::map<int, SideStreams>();   // kept to process exit

// The parts of a split kernel write disjoint rows from the same inputs, and
// each alone fills only part of the GPU (its row groups times the tiles), so
// they run side by side: part 0 on the caller's stream, the others on side
// streams that wait for everything the caller enqueued before, and the
// caller's stream then waits for them.  The enqueue sequence holds a lock,
// so concurrent calls never interleave their records and waits of the
// shared events.
int launch_parts(const std::vector<std::shared_ptr<BsProgram>> &parts, const uint8_t *in, size_t in_ld,
                 uint8_t *out, size_t out_ld, size_t s, hipStream_t stream) {
    if (parts.size() == 1) return bs_launch(*parts[0], in, in_ld, out, out_ld, s, stream);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideStreams &sd = g_side[dev];
    if (!sd.fork) {
        if ((e = hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming)) != hipSuccess) {
            sd.fork = nullptr;
            return hip_fail(e);
        }
        for (int i = 0; i < kBs16MaxParts - 1; ++i)
            if ((e = hipStreamCreateWithFlags(&sd.st[i], hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&sd.join[i], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e);
    }
    if ((e = hipEventRecord(sd.fork, stream)) != hipSuccess) return hip_fail(e);
    int st = ST_OK;
    for (size_t i = 1; i < parts.size() && st == ST_OK; ++i) {
        hipStream_t side = sd.st[i - 1];
        if ((e = hipStreamWaitEvent(side, sd.fork, 0)) != hipSuccess) return hip_fail(e);
        st = bs_launch(*parts[i], in, in_ld, out, out_ld, s, side);
        if ((e = hipEventRecord(sd.join[i - 1], side)) != hipSuccess) return hip_fail(e);
    }
    if (st == ST_OK) st = bs_launch(*parts[0], in, in_ld, out, out_ld, s, stream);
    // the caller's stream waits for every side stream that was forked,
    // also when a launch failed
    for (size_t i = 1; i < parts.size(); ++i)
        if ((e = hipStreamWaitEvent(stream, sd.join[i - 1], 0)) != hipSuccess) return hip_fail(e);
    return st;
}

}  // namespace

int stage16(Prog16 &p) {
    const std::vector<uint32_t> &t = tables();
    const void *d = nullptr;
    int st = device_copy_sync(g_tab_mu, g_tab_dev, t.data(), t.size() * sizeof(uint32_t), &d, false);
    if (st == ST_OK) st = device_copy_sync(p.mu, p.dev, p.words.data(), p.words.size() * sizeof(uint32_t), &d);
    std::vector<std::shared_ptr<BsProgram>> parts;
    {
        std::lock_guard<std::mutex> lk(p.mu);
        parts = p.bs;
    }
    for (const std::shared_ptr<BsProgram> &bp : parts)
        if (st == ST_OK && bs_ready(*bp, BS_SINGLE)) st = bs_load(*bp, BS_SINGLE);
    return st;
}

int compile16(Prog16 &p, int *specialized) {
    std::vector<std::shared_ptr<BsProgram>> parts = p.bitslice();
    if (specialized) *specialized = 0;
    if (parts.empty()) return ST_OK;
    // the parts compile side by side (hipRTC runs on the calling threads;
    // every thread is joined before this returns)
    std::vector<int> st(parts.size(), ST_OK);
    std::vector<std::string> msg(parts.size());
    std::vector<std::thread> th;
    for (size_t i = 1; i < parts.size(); ++i)
        th.emplace_back([&, i] {
            st[i] = bs_compile(*parts[i], BS_SINGLE);
            if (st[i] != ST_OK) msg[i] = g_hip_msg;
        });
    st[0] = bs_compile(*parts[0], BS_SINGLE);
    for (std::thread &t : th) t.join();
    for (size_t i = 0; i < parts.size(); ++i)
        if (st[i] != ST_OK) {
            if (i) g_hip_msg = msg[i];
            return st[i];
        }
    if (specialized) *specialized = 1;
    return ST_OK;
}

int launch16(Prog16 &p, const uint8_t *in, size_t in_ld, size_t in_n, uint8_t *out, size_t out_ld, size_t out_n,
             size_t s, hipStream_t stream) {
    if (s == 0 || s % 2 != 0) return ST_EINVAL;
    int st;
    if ((st = check_regions(in, in_ld, in_n, s)) != ST_OK) return st;
    if ((st = check_regions(out, out_ld, out_n, s)) != ST_OK) return st;
    if (overlaps(in, in_ld, in_n, out, out_ld, out_n, s)) return ST_EINVAL;
    if (p.ngroups == 0) return ST_OK;
    // the bit-sliced kernel once compiled (init phase), for blocks of at
    // least one of its tiles (its parts side by side)
    std::vector<std::shared_ptr<BsProgram>> parts;
    {
        std::lock_guard<std::mutex> lk(p.mu);
        parts = p.bs;
    }
    bool ready = !parts.empty() && s >= parts[0]->tile_bytes;
    for (const std::shared_ptr<BsProgram> &bp : parts) ready = ready && bs_ready(*bp, BS_SINGLE);
    if (ready) return launch_parts(parts, in, in_ld, out, out_ld, s, stream);
    const uint64_t ntiles = (s + kPm16TileBytes - 1) / kPm16TileBytes;
    // tile numbers are 32-bit and the grid holds at most 2^31 - 1 work-groups of 4 items
    if (ntiles > 0xFFFFFFFFull || ntiles * p.ngroups > 0x1FFFFFFFCull) return ST_EINVAL;
    const uint32_t *dt = nullptr, *dp = nullptr;
    if ((st = table_ptr(stream, &dt)) != ST_OK) return st;
    if ((st = prog_ptr(p, stream, &dp)) != ST_OK) return st;
    PmkApply16 a{in, in_ld, out, out_ld, s, dp, dt, p.ngroups, static_cast<uint32_t>(ntiles)};
    hipError_t e = pmk_apply16(&a, stream);
    return e == hipSuccess ? ST_OK : hip_fail(e);
}

}  // namespace w16
}  // namespace pmrc
