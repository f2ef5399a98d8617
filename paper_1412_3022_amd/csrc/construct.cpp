#include "construct.hpp"

#include <algorithm>
#include <numeric>

namespace pmrc {
namespace {

// Visit every m-subset of {0..n-1} that contains `must` (all when must < 0);
// stop early when fn returns false.  Returns false if stopped.
template <class Fn>
bool for_each_subset(int n, int m, int must, Fn fn) {
    std::vector<int> idx(m);
    std::iota(idx.begin(), idx.end(), 0);
    while (true) {
        if (must < 0 || std::find(idx.begin(), idx.end(), must) != idx.end())
            if (!fn(idx)) return false;
        int i = m - 1;
        while (i >= 0 && idx[i] == n - m + i) --i;
        if (i < 0) return true;
        ++idx[i];
        for (int j = i + 1; j < m; ++j) idx[j] = idx[j - 1] + 1;
    }
}

bool all_square_subsets_invertible(const Mat &psi, int must) {
    const int d = psi.cols;
    Mat inv;
    return for_each_subset(psi.rows, d, must, [&](const std::vector<int> &rows) {
        return invert(select_rows(psi, rows), inv);
    });
}

bool distinct(const std::vector<uint8_t> &v) {
    std::vector<uint8_t> s = v;
    std::sort(s.begin(), s.end());
    return std::adjacent_find(s.begin(), s.end()) == s.end();
}

// ---- PM-MSR encoding matrices (Section 3.3) -------------------------------
// Psi = [Phi | Lambda Phi], n x 2 alpha.
void assemble_msr(Mat &psi, const std::vector<uint8_t> &lam, int alpha) {
    for (int i = 0; i < psi.rows; ++i)
        for (int j = 0; j < alpha; ++j) psi.at(i, alpha + j) = gmul(lam[i], psi.at(i, j));
}

// Vandermonde: Phi[i][j] = x_i^j, Lambda_i = x_i^alpha (x_i = g^i by default).
int msr_vanilla(const CodeSpec &s, int alpha, Mat &psi, std::vector<uint8_t> &lam) {
    std::vector<uint8_t> x(s.n);
    for (int i = 0; i < s.n; ++i) x[i] = s.x.empty() ? gpow(i) : s.x[i];
    if (!distinct(x)) return ST_EINVAL;
    psi = Mat(s.n, 2 * alpha);
    lam.assign(s.n, 0);
    for (int i = 0; i < s.n; ++i) {
        uint8_t p = 1;
        for (int j = 0; j < alpha; ++j) { psi.at(i, j) = p; p = gmul(p, x[i]); }
        lam[i] = p;
    }
    assemble_msr(psi, lam, alpha);
    // Distinct x makes every d rows of Psi and every alpha rows of Phi
    // independent (Vandermonde); Lambda must still be distinct.
    return distinct(lam) ? ST_OK : ST_EUNSUPPORTED;
}

// Sparse construction of the paper: identity on top of a Cauchy matrix,
// node i (1-based) evaluated at g^(i + alpha), Lambda a Moebius map of it.
// At n = 2k the last node's Lambda is moved to the first power of g that is
// unused and keeps every helper set containing that node invertible.
int msr_sparse(const CodeSpec &s, int alpha, Mat &psi, std::vector<uint8_t> &lam) {
    const int n = s.n, k = s.k;
    if (n != 2 * k - 1 && n != 2 * k) return ST_EUNSUPPORTED;
    psi = Mat(n, 2 * alpha);
    lam.assign(n, 0);
    const uint8_t ga = gpow(alpha);
    for (int i1 = 1; i1 <= n; ++i1) {
        const uint8_t xi = gpow(i1 + alpha);
        for (int j1 = 1; j1 <= alpha; ++j1) {
            uint8_t v;
            if (i1 <= alpha) {
                v = (i1 == j1) ? 1 : 0;
            } else {
                const uint8_t diff = xi ^ gpow(j1 - 1);
                if (!diff) return ST_EUNSUPPORTED;
                v = ginv(diff);
            }
            psi.at(i1 - 1, j1 - 1) = v;
        }
        if (!(xi ^ ga)) return ST_EUNSUPPORTED;
        lam[i1 - 1] = gdiv(xi ^ 1, xi ^ ga);
    }
    assemble_msr(psi, lam, alpha);
    if (n == 2 * k) {
        const int last = n - 1;
        bool found = false;
        for (int t = 0; t < 255 && !found; ++t) {
            const uint8_t cand = gpow(t);
            if (std::find(lam.begin(), lam.begin() + last, cand) != lam.begin() + last) continue;
            lam[last] = cand;
            for (int j = 0; j < alpha; ++j) psi.at(last, alpha + j) = gmul(cand, psi.at(last, j));
            found = all_square_subsets_invertible(psi, last);
        }
        if (!found) return ST_EUNSUPPORTED;
    }
    if (!distinct(lam)) return ST_EUNSUPPORTED;
    if (!all_square_subsets_invertible(psi, -1)) return ST_EUNSUPPORTED;
    return ST_OK;
}

}  // namespace

// Index matrix of PM-MSR: M = [S1; S2], both symmetric alpha x alpha, upper
// triangles numbered row by row, S1 first (Section 3.1 example).
std::vector<int> index_msr(int alpha) {
    std::vector<int> L(static_cast<size_t>(2 * alpha) * alpha);
    int next = 0;
    for (int blk = 0; blk < 2; ++blk) {
        const int off = blk * alpha;
        for (int r = 0; r < alpha; ++r)
            for (int c = r; c < alpha; ++c) {
                L[(off + r) * alpha + c] = next;
                L[(off + c) * alpha + r] = next;
                ++next;
            }
    }
    return L;
}

namespace {

// Index matrix of PM-MBR: M = [[S, T], [T^t, 0]], S symmetric k x k then T
// k x (d-k), each numbered row by row.
std::vector<int> index_mbr(int k, int d) {
    std::vector<int> L(static_cast<size_t>(d) * d, -1);
    int next = 0;
    for (int r = 0; r < k; ++r)
        for (int c = r; c < k; ++c) { L[r * d + c] = L[c * d + r] = next++; }
    for (int r = 0; r < k; ++r)
        for (int c = k; c < d; ++c) { L[r * d + c] = L[c * d + r] = next++; }
    return L;
}

// Systematic PM-MBR Psi: a Vandermonde base right-multiplied by
// [[P^-1, P^-1 D], [0, I]] (P, D = top k rows of its first k and last d-k
// columns), which makes the first k rows [I_k | 0].
int mbr_psi(int k, int d, int n, Mat &psi) {
    Mat base(n, d);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < d; ++c) base.at(i, c) = gpow(static_cast<long>(i) * c);
    Mat P(k, k), Pinv;
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < k; ++c) P.at(r, c) = base.at(r, c);
    if (!invert(P, Pinv)) return ST_EUNSUPPORTED;
    Mat T = Mat::identity(d);
    Mat Dtop(k, d - k);
    for (int r = 0; r < k; ++r)
        for (int c = k; c < d; ++c) Dtop.at(r, c - k) = base.at(r, c);
    Mat PD = matmul(Pinv, Dtop);
    for (int r = 0; r < k; ++r) {
        for (int c = 0; c < k; ++c) T.at(r, c) = Pinv.at(r, c);
        for (int c = k; c < d; ++c) T.at(r, c) = PD.at(r, c - k);
    }
    psi = matmul(base, T);
    return ST_OK;
}

// Linearization (Section 3.1): row alpha*i + j of G holds Psi[i][l] in the
// column of the message symbol M[l][j].
Mat linearize(const Mat &psi, const std::vector<int> &L, int alpha, int B) {
    const int n = psi.rows, d = psi.cols;
    Mat G(n * alpha, B);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < alpha; ++j)
            for (int l = 0; l < d; ++l) {
                const int sym = L[l * alpha + j];
                if (sym >= 0) G.at(alpha * i + j, sym) ^= psi.at(i, l);
            }
    return G;
}

}  // namespace

int build_code(const CodeSpec &s, CodeMats &c) {
    c = CodeMats();
    c.kind = s.kind; c.construction = s.construction; c.systematic = s.systematic ? 1 : 0;
    c.k = s.k; c.d = s.d; c.n = s.n;
    if (s.n > 255 || s.k < 1 || s.n <= s.k) return ST_EINVAL;
    if (!s.x.empty() && static_cast<int>(s.x.size()) != s.n) return ST_EINVAL;
    if (s.kind == KIND_MSR) {
        if (s.k < 2 || s.n < s.d + 1) return ST_EINVAL;
        if (s.d != 2 * s.k - 2) return ST_EUNSUPPORTED;  // basic PM-MSR regime only
        c.alpha = s.k - 1;
        c.B = s.k * c.alpha;
        int st = (s.construction == CONS_VANILLA) ? msr_vanilla(s, c.alpha, c.psi, c.lambda)
                                                  : (s.construction == CONS_SPARSE
                                                         ? msr_sparse(s, c.alpha, c.psi, c.lambda)
                                                         : ST_EINVAL);
        if (st != ST_OK) return st;
        c.L = index_msr(c.alpha);
        c.G = linearize(c.psi, c.L, c.alpha, c.B);
        if (c.systematic) {
            Mat top(c.B, c.B), topinv;
            std::copy(c.G.v.begin(), c.G.v.begin() + static_cast<long>(c.B) * c.B, top.v.begin());
            if (!invert(top, topinv)) return ST_ESINGULAR;
            c.Gsys = matmul(c.G, topinv);
            c.enc = Mat(c.n * c.alpha - c.B, c.B);
            std::copy(c.Gsys.v.begin() + static_cast<long>(c.B) * c.B, c.Gsys.v.end(), c.enc.v.begin());
            for (int t = 0; t < c.n * c.alpha; ++t) c.node_map.push_back(t);
        } else {
            c.Gsys = c.G;
            c.enc = c.G;
            for (int t = 0; t < c.n * c.alpha; ++t) c.node_map.push_back(c.B + t);
        }
    } else if (s.kind == KIND_MBR) {
        if (s.d < s.k || s.n < s.d + 1) return ST_EINVAL;
        c.alpha = s.d;
        c.B = s.k * s.d - s.k * (s.k - 1) / 2;
        int st = mbr_psi(s.k, s.d, s.n, c.psi);
        if (st != ST_OK) return st;
        c.L = index_mbr(s.k, s.d);
        c.G = linearize(c.psi, c.L, c.alpha, c.B);
        c.Gsys = c.G;
        const int kd = s.k * s.d;
        c.enc = Mat(c.n * c.alpha - kd, c.B);
        std::copy(c.G.v.begin() + static_cast<long>(kd) * c.B, c.G.v.end(), c.enc.v.begin());
        for (int t = 0; t < c.n * c.alpha; ++t) {
            if (t < kd) {
                int sym = -1, cnt = 0;
                for (int m = 0; m < c.B; ++m)
                    if (c.G.at(t, m)) { sym = m; ++cnt; }
                if (cnt != 1 || c.G.at(t, sym) != 1) return ST_ESINGULAR;
                c.node_map.push_back(sym);
            } else {
                c.node_map.push_back(c.B + (t - kd));
            }
        }
    } else if (s.kind == KIND_RS) {
        c.d = s.k;
        c.alpha = 1;
        c.B = s.k;
        Mat V(s.n, s.k), top(s.k, s.k), topinv;
        for (int i = 0; i < s.n; ++i)
            for (int j = 0; j < s.k; ++j) V.at(i, j) = gpow(static_cast<long>(i) * j);
        std::copy(V.v.begin(), V.v.begin() + static_cast<long>(s.k) * s.k, top.v.begin());
        if (!invert(top, topinv)) return ST_ESINGULAR;
        c.G = matmul(V, topinv);
        c.Gsys = c.G;
        c.psi = c.G;
        c.enc = Mat(s.n - s.k, s.k);
        std::copy(c.G.v.begin() + static_cast<long>(s.k) * s.k, c.G.v.end(), c.enc.v.begin());
        for (int t = 0; t < s.n; ++t) c.node_map.push_back(t);
    } else {
        return ST_EINVAL;
    }
    return ST_OK;
}

Mat helper_row(const CodeMats &c, int f) {
    if (c.kind == KIND_RS) {
        Mat r(1, 1);
        r.at(0, 0) = 1;
        return r;
    }
    // MSR sends phi_f (first alpha entries of psi_f); MBR sends psi_f (d = alpha).
    Mat r(1, c.alpha);
    for (int a = 0; a < c.alpha; ++a) r.at(0, a) = c.psi.at(f, a);
    return r;
}

int newcomer_matrix(const CodeMats &c, int f, const std::vector<int> &H, Mat &R) {
    const int d = c.d;
    if (static_cast<int>(H.size()) != d) return ST_EINVAL;
    Mat PH = select_rows(c.psi, H), PHinv;
    if (!invert(PH, PHinv)) return ST_ESINGULAR;
    if (c.kind == KIND_MBR) {
        R = PHinv;
    } else if (c.kind == KIND_MSR) {
        // The newcomer recovers (S1 phi_f; S2 phi_f); by symmetry its blocks
        // are phi_f^T S1 + lambda_f phi_f^T S2.
        R = Mat(c.alpha, d);
        for (int a = 0; a < c.alpha; ++a)
            for (int j = 0; j < d; ++j)
                R.at(a, j) = PHinv.at(a, j) ^ gmul(c.lambda[f], PHinv.at(c.alpha + a, j));
    } else {
        Mat gf(1, c.k);
        for (int j = 0; j < c.k; ++j) gf.at(0, j) = c.G.at(f, j);
        R = matmul(gf, PHinv);
    }
    return ST_OK;
}

int decode_matrix(const CodeMats &c, const std::vector<int> &K, Mat &D, std::vector<int> &used) {
    const int a = c.alpha;
    Mat rows(static_cast<int>(K.size()) * a, c.B);
    for (size_t i = 0; i < K.size(); ++i)
        for (int j = 0; j < a; ++j)
            std::copy(c.Gsys.row(K[i] * a + j), c.Gsys.row(K[i] * a + j) + c.B,
                      rows.v.begin() + static_cast<long>(i * a + j) * c.B);
    if (rows.rows == c.B) {   // MSR and RS: exactly B received blocks, all of them used
        used.resize(c.B);
        for (int r = 0; r < c.B; ++r) used[r] = r;
        return invert(rows, D) ? ST_OK : ST_ESINGULAR;
    }
    used = independent_rows(rows, c.B);
    if (static_cast<int>(used.size()) != c.B) return ST_ESINGULAR;
    if (!invert(select_rows(rows, used), D)) return ST_ESINGULAR;
    return ST_OK;
}

// The data collector of the product-matrix MSR code (Section 2: Psi =
// [Phi, Lambda Phi], node i holds phi_i^t S1 + lambda_i phi_i^t S2), with
// every step a matrix over blocks.  Node blocks i*alpha + a of K give
// Z_ij = sum_a y_i[a] phi_j[a] = P_ij + lambda_i Q_ij; a pair i < j yields
// Q_ij = c (Z_ij + Z_ji) and P_ij = Z_ij + lambda_i Q_ij with c = 1 /
// (lambda_i + lambda_j); as lambda_i c + 1 = lambda_j c, P_ij = lambda_j c
// Z_ij + lambda_i c Z_ji.
// The data collector of the product-matrix MBR code (Section 2: M =
// [[S, T], [T^t, 0]], Psi = [Phi, Delta]; the k nodes of K hold
// [Phi_K S + Delta_K T^t, Phi_K T]) in two passes over blocks.  With
// Phinv = inverse(Phi_K) and E = Phinv Delta_K:
//   T[l][t] = sum_i Phinv[l][i] y_i[k + t],
//   S[l][j] = sum_i Phinv[l][i] y_i[j] + sum_t E[l][t] T[j][t].
// S is symmetric, so each of its symbols is taken from the side (l, j) or
// (j, l) with fewer terms; for a node l < k of K (a row [I_k, 0] of Psi)
// row l of Phinv is a unit vector and row l of E is zero, so its T and S
// symbols become plain copies.
static int mbr_specific_factors(const CodeMats &c, const std::vector<int> &K, Mat F[kSpecificPasses]) {
    const int k = c.k, d = c.d, dk = d - k, B = c.B;
    Mat Phi(k, k), Phinv;
    for (int i = 0; i < k; ++i)
        for (int t = 0; t < k; ++t) Phi.at(i, t) = c.psi.at(K[i], t);
    if (!invert(Phi, Phinv)) return ST_ESINGULAR;
    std::vector<uint8_t> E(static_cast<size_t>(k) * dk, 0);
    for (int l = 0; l < k; ++l)
        for (int t = 0; t < dk; ++t) {
            uint8_t acc = 0;
            for (int i = 0; i < k; ++i) acc ^= gmul(Phinv.at(l, i), c.psi.at(K[i], k + t));
            E[static_cast<size_t>(l) * dk + t] = acc;
        }
    // second-pass inputs: T[l][t] at l*dk + t, then copies of y_i[j] at
    // k*dk + i*k + j (renumbered below to the copies actually read)
    const int nT = k * dk, nv = nT + k * k;
    Mat F1(B, nv);
    // terms of an S symbol taken from side l (row l of Phinv and of E)
    auto s_terms = [&](int l) {
        int cnt = 0;
        for (int i = 0; i < k; ++i) cnt += Phinv.at(l, i) != 0;
        for (int t = 0; t < dk; ++t) cnt += E[static_cast<size_t>(l) * dk + t] != 0;
        return cnt;
    };
    for (int a = 0; a < k; ++a) {
        for (int b = a; b < k; ++b) {
            const int l = s_terms(a) <= s_terms(b) ? a : b, j = l == a ? b : a;
            const int m = c.L[a * d + b];
            for (int i = 0; i < k; ++i) F1.at(m, nT + i * k + j) ^= Phinv.at(l, i);
            for (int t = 0; t < dk; ++t) F1.at(m, j * dk + t) ^= E[static_cast<size_t>(l) * dk + t];
        }
        for (int t = 0; t < dk; ++t) F1.at(c.L[a * d + k + t], a * dk + t) = 1;
    }
    std::vector<int> wrow(nv, -1);
    int nw = nT;
    for (int v = 0; v < nT; ++v) wrow[v] = v;
    for (int v = nT; v < nv; ++v) {
        bool used = false;
        for (int m = 0; m < B && !used; ++m) used = F1.at(m, v) != 0;
        if (used) wrow[v] = nw++;
    }
    Mat F0(nw, k * d), W1(B, nw);
    for (int l = 0; l < k; ++l)
        for (int t = 0; t < dk; ++t)
            for (int i = 0; i < k; ++i) F0.at(l * dk + t, i * d + k + t) = Phinv.at(l, i);
    for (int v = nT; v < nv; ++v)
        if (wrow[v] >= 0) {
            const int i = (v - nT) / k, j = (v - nT) % k;
            F0.at(wrow[v], i * d + j) = 1;
        }
    for (int m = 0; m < B; ++m)
        for (int v = 0; v < nv; ++v)
            if (F1.at(m, v)) W1.at(m, wrow[v]) = F1.at(m, v);
    F[0] = std::move(F0);
    F[1] = std::move(W1);
    for (int p = 2; p < kSpecificPasses; ++p) F[p] = Mat();
    return ST_OK;
}

int specific_decode_factors(const CodeMats &c, const std::vector<int> &K, Mat F[kSpecificPasses]) {
    if (c.kind == KIND_MBR) {
        if (static_cast<int>(K.size()) != c.k) return ST_EINVAL;
        return mbr_specific_factors(c, K, F);
    }
    if (c.kind != KIND_MSR) return ST_EUNSUPPORTED;
    const int k = c.k, a = c.alpha, d = c.d, B = c.B;
    if (static_cast<int>(K.size()) != k || d != 2 * a) return ST_EINVAL;
    auto phi = [&](int i, int t) { return c.psi.at(K[i], t); };
    auto lam = [&](int i) { return c.lambda[K[i]]; };
    for (int i = 0; i < k; ++i)
        for (int t = 0; t < a; ++t)
            if (c.psi.at(K[i], a + t) != gmul(lam(i), phi(i, t))) return ST_EUNSUPPORTED;
    const int npairs = k * (k - 1) / 2;   // = B / 2
    // Z_ij for i != j, rows i-major: row zrow[i][j]
    std::vector<std::vector<int>> zrow(k, std::vector<int>(k, -1)), pair_of(k, std::vector<int>(k, -1));
    Mat Zm(k * (k - 1), k * a);
    int zr = 0;
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            if (j == i) continue;
            zrow[i][j] = zr;
            for (int t = 0; t < a; ++t) Zm.at(zr, i * a + t) = phi(j, t);
            ++zr;
        }
    Mat A(B, k * (k - 1));
    int q = 0;
    for (int i = 0; i < k; ++i)
        for (int j = i + 1; j < k; ++j, ++q) {
            const uint8_t sum = lam(i) ^ lam(j);
            if (!sum) return ST_ESINGULAR;
            const uint8_t cc = ginv(sum);
            pair_of[i][j] = pair_of[j][i] = q;
            A.at(q, zrow[i][j]) = gmul(lam(j), cc);            // P_ij
            A.at(q, zrow[j][i]) = gmul(lam(i), cc);
            A.at(npairs + q, zrow[i][j]) = cc;                 // Q_ij
            A.at(npairs + q, zrow[j][i]) = cc;
        }
    // phi_i^t S1 from the alpha values P_ij (j != i, increasing j): rows
    // phi_j^t of the system, solved by its inverse
    Mat Bm(2 * a * a, B);
    for (int i = 0; i < a; ++i) {
        Mat Fi(a, a), Fi_inv;
        std::vector<int> js;
        for (int j = 0; j < k; ++j)
            if (j != i) js.push_back(j);
        for (int r = 0; r < a; ++r)
            for (int t = 0; t < a; ++t) Fi.at(r, t) = phi(js[r], t);
        if (!invert(Fi, Fi_inv)) return ST_ESINGULAR;
        for (int b = 0; b < a; ++b)
            for (int r = 0; r < a; ++r) {
                const int qp = pair_of[i][js[r]];
                Bm.at(i * a + b, qp) = Fi_inv.at(b, r);                    // U[i][b] from P
                Bm.at(a * a + i * a + b, npairs + qp) = Fi_inv.at(b, r);   // V[i][b] from Q
            }
    }
    // S1 = inverse(Phi_A) U, S2 = inverse(Phi_A) V; message symbol L[l][j]
    Mat PhiA(a, a), PhiA_inv;
    for (int i = 0; i < a; ++i)
        for (int t = 0; t < a; ++t) PhiA.at(i, t) = phi(i, t);
    if (!invert(PhiA, PhiA_inv)) return ST_ESINGULAR;
    Mat Cm(B, 2 * a * a);
    std::vector<char> done(B, 0);
    for (int l = 0; l < d; ++l)
        for (int j = 0; j < a; ++j) {
            const int msym = c.L[l * a + j];
            if (msym < 0 || done[msym]) continue;
            done[msym] = 1;
            const int half = l < a ? 0 : 1, row = l % a;
            for (int i = 0; i < a; ++i) Cm.at(msym, half * a * a + i * a + j) = PhiA_inv.at(row, i);
        }
    for (int m = 0; m < B; ++m)
        if (!done[m]) return ST_EINVAL;
    F[0] = std::move(Zm);
    F[1] = std::move(A);
    F[2] = std::move(Bm);
    F[3] = std::move(Cm);
    if (c.systematic) {
        Mat Gt(B, B);   // the first B rows of the linearized generator
        std::copy(c.G.v.begin(), c.G.v.begin() + static_cast<long>(B) * B, Gt.v.begin());
        F[4] = std::move(Gt);
    } else {
        F[4] = Mat();
    }
    return ST_OK;
}

}  // namespace pmrc
