/*
 * oracle16.c -- the GF(2^16) part of the CPU oracle for "Fast Product-Matrix
 * Regenerating Codes" (Le Scouarnec, arXiv 1412.3022).
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: nothing in the product may include,
 * link or call it.  It shares no code with the library.
 *
 * Section 3.3 states that the sparse PM-MSR construction, valid for k up to 39
 * in GF(2^8), is valid for k up to 64 in GF(2^16).  This file holds that
 * construction and the data phase of the resulting codes over GF(2^16):
 * the field, dense linear algebra, the sparse Psi and Lambda with their
 * computational validity check, linearization, the systematic form, region
 * multiplication, repair and decode matrices, and the specific PM-MSR decoder.
 *
 * Conventions: matrices are row-major uint16_t arrays; a region holds 16-bit
 * symbols, symbol p in bytes 2p (low byte) and 2p + 1 (high byte).
 * Reading: the paper gives no byte order for GF(2^16) regions; little-endian
 * (the order of the machines it runs on) is taken.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Field GF(2^16).  Reading: the paper uses GF-Complete's default fields; for
 * w = 16 that is the polynomial x^16 + x^12 + x^3 + x + 1 (0x1100B), with
 * generator g = 2 (x is primitive for it: tested).  add = sub = XOR; mul and
 * div through exponent and logarithm tables, the exponent table doubled so a
 * sum of two logarithms indexes it directly.                                */
static uint16_t EXP16[2 * 65535];
static int LOG16[65536];
static int ready16 = 0;

void or16_init(void)
{
    if (ready16) return;
    unsigned a = 1;
    for (int i = 0; i < 65535; i++) {
        EXP16[i] = EXP16[i + 65535] = (uint16_t)a;
        LOG16[a] = i;
        a <<= 1;                         /* multiply by g = x */
        if (a & 0x10000) a ^= 0x1100B;   /* reduce modulo the field polynomial */
    }
    LOG16[0] = -1;
    ready16 = 1;
}

uint16_t or16_mul(uint16_t a, uint16_t b)
{
    if (a == 0 || b == 0) return 0;
    return EXP16[LOG16[a] + LOG16[b]];
}

/* multiplicative inverse; 0 for a == 0 */
uint16_t or16_inv(uint16_t a)
{
    if (a == 0) return 0;
    return EXP16[(65535 - LOG16[a]) % 65535];
}

uint16_t or16_div(uint16_t a, uint16_t b) { return or16_mul(a, or16_inv(b)); }

/* g^e for any integer e */
uint16_t or16_gpow(long e)
{
    long r = e % 65535;
    if (r < 0) r += 65535;
    return EXP16[r];
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra over GF(2^16).                                       */

/* C (m x n) = A (m x k) * B (k x n) */
void or16_matmul(const uint16_t *A, const uint16_t *B, uint16_t *C, int m, int k, int n)
{
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) {
            uint16_t acc = 0;
            for (int t = 0; t < k; t++) acc ^= or16_mul(A[(size_t)i * k + t], B[(size_t)t * n + j]);
            C[(size_t)i * n + j] = acc;
        }
}

/* Gauss-Jordan on [A | I]: pivot = first row at or below the diagonal with a
 * nonzero entry.  Returns 0 and fills Ainv, or -1 when A is singular. */
int or16_invert(const uint16_t *A, uint16_t *Ainv, int n)
{
    size_t w = (size_t)2 * n;
    uint16_t *M = (uint16_t *)malloc(sizeof(uint16_t) * n * w);
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++) {
            M[i * w + j] = A[(size_t)i * n + j];
            M[i * w + n + j] = (uint16_t)(i == j);
        }
    }
    int rc = 0;
    for (int c = 0; c < n && rc == 0; c++) {
        int p = c;
        while (p < n && M[p * w + c] == 0) p++;
        if (p == n) { rc = -1; break; }
        if (p != c)
            for (size_t j = 0; j < w; j++) { uint16_t t = M[p * w + j]; M[p * w + j] = M[c * w + j]; M[c * w + j] = t; }
        uint16_t s = or16_inv(M[c * w + c]);
        for (size_t j = 0; j < w; j++) M[c * w + j] = or16_mul(s, M[c * w + j]);
        for (int r = 0; r < n; r++) {
            uint16_t f = M[r * w + c];
            if (r == c || f == 0) continue;
            for (size_t j = 0; j < w; j++) M[r * w + j] ^= or16_mul(f, M[c * w + j]);
        }
    }
    if (rc == 0)
        for (int i = 0; i < n; i++) memcpy(Ainv + (size_t)i * n, M + i * w + n, sizeof(uint16_t) * n);
    free(M);
    return rc;
}

/* rank of an m x n matrix by row reduction */
int or16_rank(const uint16_t *A, int m, int n)
{
    uint16_t *M = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)m * n);
    memcpy(M, A, sizeof(uint16_t) * (size_t)m * n);
    int r = 0;
    for (int c = 0; c < n && r < m; c++) {
        int p = r;
        while (p < m && M[(size_t)p * n + c] == 0) p++;
        if (p == m) continue;
        for (int j = 0; j < n; j++) { uint16_t t = M[(size_t)p * n + j]; M[(size_t)p * n + j] = M[(size_t)r * n + j]; M[(size_t)r * n + j] = t; }
        uint16_t s = or16_inv(M[(size_t)r * n + c]);
        for (int i = r + 1; i < m; i++) {
            uint16_t f = or16_mul(M[(size_t)i * n + c], s);
            if (!f) continue;
            for (int j = 0; j < n; j++) M[(size_t)i * n + j] ^= or16_mul(f, M[(size_t)r * n + j]);
        }
        r++;
    }
    free(M);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Sparse PM-MSR encoding matrix (Section 3.3), as printed, over GF(2^16):
 *   Phi_{i,j} = [i == j]                          for i <= alpha,
 *   Phi_{i,j} = 1 / (g^(i+alpha) - g^(j-1))        for i >  alpha,
 *   Lambda_{i,i} = (g^(i+alpha) - g^0) / (g^(i+alpha) - g^alpha),
 *   Psi = [Phi, Lambda Phi]   (1-based i, j; "-" is XOR). */
int or16_msr_sparse_printed(int k, int n, uint16_t *psi, uint16_t *lam)
{
    int alpha = k - 1, d = 2 * alpha;
    for (int t = 0; t < n; t++) {
        int i = t + 1;
        uint16_t xi = or16_gpow(i + alpha);
        for (int j = 1; j <= alpha; j++) {
            uint16_t phi;
            if (i <= alpha) phi = (uint16_t)(i == j);
            else {
                uint16_t den = xi ^ or16_gpow(j - 1);
                if (!den) return -1;
                phi = or16_inv(den);
            }
            psi[t * d + (j - 1)] = phi;
        }
        uint16_t den = xi ^ or16_gpow(alpha);
        if (!den) return -1;
        lam[t] = or16_div(xi ^ 1, den);
        for (int j = 0; j < alpha; j++) psi[t * d + alpha + j] = or16_mul(lam[t], psi[t * d + j]);
    }
    return 0;
}

static int next_subset16(int *idx, int m, int n)
{
    int i = m - 1;
    while (i >= 0 && idx[i] == n - m + i) i--;
    if (i < 0) return 0;
    idx[i]++;
    for (int j = i + 1; j < m; j++) idx[j] = idx[j - 1] + 1;
    return 1;
}

/* Every d x d submatrix of Psi (n x d) whose rows include `must` (all when
 * must < 0) is invertible: the computational check of Section 3.3. */
int or16_all_dsubsets_invertible(const uint16_t *psi, int n, int d, int must)
{
    int *idx = (int *)malloc(sizeof(int) * (size_t)d);
    uint16_t *S = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)d * d);
    uint16_t *Si = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)d * d);
    for (int i = 0; i < d; i++) idx[i] = i;
    int ok = 1;
    do {
        int has = (must < 0);
        for (int i = 0; i < d; i++) if (idx[i] == must) has = 1;
        if (!has) continue;
        for (int i = 0; i < d; i++) memcpy(S + (size_t)i * d, psi + (size_t)idx[i] * d, sizeof(uint16_t) * d);
        if (or16_invert(S, Si, d) != 0) { ok = 0; break; }
    } while (next_subset16(idx, d, n));
    free(idx); free(S); free(Si);
    return ok;
}

/* Validity (Section 3.3): Lambda entries distinct and every d rows of Psi
 * independent.  1 when valid. */
int or16_msr_valid(const uint16_t *psi, const uint16_t *lam, int n, int d)
{
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (lam[i] == lam[j]) return 0;
    return or16_all_dsubsets_invertible(psi, n, d, -1);
}

/* The construction the library uses: as printed for n = 2k - 1; at n = 2k the
 * last node takes Lambda = g^t for the smallest t whose value is new and keeps
 * every d-subset holding that node invertible (the same reading as over
 * GF(2^8): the printed last row makes such subsets singular). */
int or16_msr_sparse(int k, int n, uint16_t *psi, uint16_t *lam)
{
    int alpha = k - 1, d = 2 * alpha;
    if (n != 2 * k - 1 && n != 2 * k) return -1;
    if (or16_msr_sparse_printed(k, n, psi, lam) != 0) return -1;
    if (n == 2 * k - 1) return 0;
    int last = n - 1;
    for (int t = 0; t < 65535; t++) {
        uint16_t cand = or16_gpow(t);
        int clash = 0;
        for (int i = 0; i < last; i++) if (lam[i] == cand) clash = 1;
        if (clash) continue;
        lam[last] = cand;
        for (int j = 0; j < alpha; j++) psi[last * d + alpha + j] = or16_mul(cand, psi[last * d + j]);
        if (or16_all_dsubsets_invertible(psi, n, d, last)) return 0;
    }
    return -1;
}

/* Linearization (Section 3.1): G[alpha i + j][L[l][j]] = Psi[i][l]. */
void or16_linearize(const uint16_t *psi, const int *L, int n, int d, int alpha, int B, uint16_t *G)
{
    memset(G, 0, sizeof(uint16_t) * (size_t)n * alpha * B);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < alpha; j++)
            for (int l = 0; l < d; l++) {
                int m = L[l * alpha + j];
                if (m >= 0) G[(size_t)(alpha * i + j) * B + m] ^= psi[i * d + l];
            }
}

static uint16_t sym_get(const uint8_t *r, size_t p) { return (uint16_t)(r[2 * p] | (r[2 * p + 1] << 8)); }
static void sym_put(uint8_t *r, size_t p, uint16_t v) { r[2 * p] = (uint8_t)v; r[2 * p + 1] = (uint8_t)(v >> 8); }

/* Product-matrix encoding (Section 2; Section 3.1): node i, block j is
 * sum_l Psi[i][l] M[l][j] with M[l][j] = X[L[l][j]], symbol by symbol.  Used
 * only to check the linearized generator. */
void or16_specific_encode(const uint16_t *psi, const int *L, int n, int d, int alpha,
                          const uint8_t *const *X, uint8_t *const *C, size_t nsym)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < alpha; j++) {
            uint8_t *out = C[i * alpha + j];
            memset(out, 0, 2 * nsym);
            for (int l = 0; l < d; l++) {
                int m = L[l * alpha + j];
                if (m < 0) continue;
                uint16_t coef = psi[i * d + l];
                for (size_t p = 0; p < nsym; p++) sym_put(out, p, sym_get(out, p) ^ or16_mul(coef, sym_get(X[m], p)));
            }
        }
}

/* Systematic form (Section 3.2): G' = G * inverse(first B rows of G). */
int or16_systematic(const uint16_t *G, int rows, int B, uint16_t *Gp)
{
    uint16_t *Gti = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)B * B);
    int rc = or16_invert(G, Gti, B);
    if (rc == 0) or16_matmul(G, Gti, Gp, rows, B, B);
    free(Gti);
    return rc;
}

/* Region matrix multiply: out[r] = sum_c A[r][c] * in[c], symbol by symbol. */
void or16_apply(const uint16_t *A, int rows, int cols, const uint8_t *const *in, uint8_t *const *out, size_t nsym)
{
    for (int r = 0; r < rows; r++) {
        memset(out[r], 0, 2 * nsym);
        for (int c = 0; c < cols; c++) {
            uint16_t a = A[(size_t)r * cols + c];
            if (!a) continue;
            for (size_t p = 0; p < nsym; p++) sym_put(out[r], p, sym_get(out[r], p) ^ or16_mul(a, sym_get(in[c], p)));
        }
    }
}

/* Repair of node f from helpers H (Section 2): the newcomer's alpha x d
 * matrix [I | lambda_f I] inverse(Psi_H); the helper sends phi_f^T times its
 * alpha blocks.  -1 when Psi_H is singular. */
int or16_newcomer_matrix(const uint16_t *psi, const uint16_t *lam, int d, int alpha, int f, const int *H,
                         uint16_t *R)
{
    uint16_t *S = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)d * d);
    uint16_t *Si = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)d * d);
    for (int i = 0; i < d; i++) memcpy(S + (size_t)i * d, psi + (size_t)H[i] * d, sizeof(uint16_t) * d);
    int rc = or16_invert(S, Si, d);
    if (rc == 0)
        for (int a = 0; a < alpha; a++)
            for (int c = 0; c < d; c++)
                R[a * d + c] = Si[a * d + c] ^ or16_mul(lam[f], Si[(alpha + a) * d + c]);
    free(S); free(Si);
    return rc;
}

/* Decode from the k nodes K (Section 2: X = inverse(G~) Y~): the k alpha rows
 * of the generator the nodes follow, node-major, inverted.  For PM-MSR they
 * are exactly B rows.  -1 when singular. */
int or16_decode_matrix(const uint16_t *Gsys, int B, int alpha, const int *K, int k, uint16_t *D)
{
    if (k * alpha != B) return -1;
    uint16_t *Sel = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)B * B);
    for (int t = 0; t < B; t++)
        memcpy(Sel + (size_t)t * B, Gsys + (size_t)(K[t / alpha] * alpha + t % alpha) * B, sizeof(uint16_t) * B);
    int rc = or16_invert(Sel, D, B);
    free(Sel);
    return rc;
}

/* Specific PM-MSR decoding over GF(2^16): the data collector of the
 * product-matrix MSR code that Section 4.1 (decoding paragraph) compares with
 * the linearized decode, symbol by symbol.  Reading (as for GF(2^8): the steps
 * follow from Psi = [Phi, Lambda Phi], M = [S1; S2] with S1, S2 symmetric,
 * node i storing phi_i^t S1 + lambda_i phi_i^t S2):
 *  1. Z[i][j] = y_i . phi_j = P_ij + lambda_i Q_ij for the k nodes of K;
 *  2. a pair i < j gives Q_ij = (Z[i][j] + Z[j][i]) / (lambda_i + lambda_j)
 *     and P_ij = Z[i][j] + lambda_i Q_ij;
 *  3. for each of the first alpha nodes i of K, the alpha values P_ij (j != i)
 *     are phi_i^t S1 phi_j: an alpha x alpha system with rows phi_j^t gives
 *     phi_i^t S1 (and phi_i^t S2 from Q);
 *  4. those rows are Phi_A S1 and Phi_A S2: S1, S2 follow from inverse(Phi_A);
 *  5. message symbol L[l][j] = M[l][j]; a systematic code stored G Z with
 *     Z = inverse(G~) X, so X = G~ Z, the product-matrix encoding of Z by the
 *     first k nodes.
 * Y: the k alpha blocks of K, node-major; X receives B blocks of nsym symbols.
 * Returns -1 when a system is singular or two lambda of K are equal, -2 when
 * Psi does not have the [Phi, Lambda Phi] form. */
int or16_msr_specific_decode(const uint16_t *psi, const uint16_t *lam, const int *L, int k, const int *K,
                             const uint8_t *const *Y, int systematic, uint8_t *const *X, size_t nsym)
{
    const int alpha = k - 1, d = 2 * alpha, B = alpha * (alpha + 1);
    for (int i = 0; i < k; i++)
        for (int a = 0; a < alpha; a++)
            if (psi[K[i] * d + alpha + a] != or16_mul(lam[K[i]], psi[K[i] * d + a])) return -2;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (lam[K[i]] == lam[K[j]]) return -1;
    size_t aa = (size_t)alpha * alpha;
    uint16_t *Finv = (uint16_t *)malloc(sizeof(uint16_t) * aa * alpha), *F = (uint16_t *)malloc(sizeof(uint16_t) * aa);
    uint16_t *PhiA = (uint16_t *)malloc(sizeof(uint16_t) * aa), *PhiAinv = (uint16_t *)malloc(sizeof(uint16_t) * aa);
    int rc = 0;
    for (int i = 0; i < alpha && rc == 0; i++) {
        int r = 0;
        for (int j = 0; j < k; j++) {
            if (j == i) continue;
            memcpy(F + (size_t)r * alpha, psi + (size_t)K[j] * d, sizeof(uint16_t) * alpha);
            r++;
        }
        rc = or16_invert(F, Finv + (size_t)i * aa, alpha);
    }
    for (int i = 0; i < alpha; i++) memcpy(PhiA + (size_t)i * alpha, psi + (size_t)K[i] * d, sizeof(uint16_t) * alpha);
    if (rc == 0) rc = or16_invert(PhiA, PhiAinv, alpha);
    uint16_t *y = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)k * alpha);
    uint16_t *z = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)k * k);
    uint16_t *P = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)k * k), *Q = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)k * k);
    uint16_t *U = (uint16_t *)malloc(sizeof(uint16_t) * aa), *V = (uint16_t *)malloc(sizeof(uint16_t) * aa);
    uint16_t *S1 = (uint16_t *)malloc(sizeof(uint16_t) * aa), *S2 = (uint16_t *)malloc(sizeof(uint16_t) * aa);
    uint16_t *Zm = (uint16_t *)malloc(sizeof(uint16_t) * (size_t)B);
    uint16_t *pv = (uint16_t *)malloc(sizeof(uint16_t) * alpha), *qv = (uint16_t *)malloc(sizeof(uint16_t) * alpha);
    for (size_t p = 0; p < nsym && rc == 0; p++) {
        for (int t = 0; t < k * alpha; t++) y[t] = sym_get(Y[t], p);
        for (int i = 0; i < k; i++)                                   /* step 1 */
            for (int j = 0; j < k; j++) {
                uint16_t acc = 0;
                for (int a = 0; a < alpha; a++) acc ^= or16_mul(y[i * alpha + a], psi[K[j] * d + a]);
                z[i * k + j] = acc;
            }
        for (int i = 0; i < k; i++)                                   /* step 2 */
            for (int j = i + 1; j < k; j++) {
                uint16_t q = or16_div(z[i * k + j] ^ z[j * k + i], lam[K[i]] ^ lam[K[j]]);
                uint16_t pp = z[i * k + j] ^ or16_mul(lam[K[i]], q);
                P[i * k + j] = P[j * k + i] = pp;
                Q[i * k + j] = Q[j * k + i] = q;
            }
        for (int i = 0; i < alpha; i++) {                             /* step 3 */
            int r = 0;
            for (int j = 0; j < k; j++) {
                if (j == i) continue;
                pv[r] = P[i * k + j];
                qv[r] = Q[i * k + j];
                r++;
            }
            or16_matmul(Finv + (size_t)i * aa, pv, U + (size_t)i * alpha, alpha, alpha, 1);
            or16_matmul(Finv + (size_t)i * aa, qv, V + (size_t)i * alpha, alpha, alpha, 1);
        }
        or16_matmul(PhiAinv, U, S1, alpha, alpha, alpha);             /* step 4 */
        or16_matmul(PhiAinv, V, S2, alpha, alpha, alpha);
        for (int l = 0; l < d; l++)                                   /* step 5 */
            for (int j = 0; j < alpha; j++)
                Zm[L[l * alpha + j]] = l < alpha ? S1[l * alpha + j] : S2[(l - alpha) * alpha + j];
        if (!systematic) {
            for (int m = 0; m < B; m++) sym_put(X[m], p, Zm[m]);
        } else {
            for (int i = 0; i < k; i++)
                for (int j = 0; j < alpha; j++) {
                    uint16_t acc = 0;
                    for (int l = 0; l < d; l++) acc ^= or16_mul(psi[i * d + l], Zm[L[l * alpha + j]]);
                    sym_put(X[i * alpha + j], p, acc);
                }
        }
    }
    free(Finv); free(F); free(PhiA); free(PhiAinv); free(y); free(z); free(P); free(Q);
    free(U); free(V); free(S1); free(S2); free(Zm); free(pv); free(qv);
    return rc == 0 ? 0 : -1;
}
