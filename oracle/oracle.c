/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the
 * product-matrix (PM) regenerating-code data path of "Fast Product-Matrix
 * Regenerating Codes" (Le Scouarnec, arXiv 1412.3022).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its
 * Python binding) may include, link or call this file.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
 * code with the library: its own field tables, its own linear algebra, its
 * own constructions.
 *
 * Every function follows a passage of the paper (cited by section, equation
 * or table) or, where the paper defers to the seminal product-matrix paper
 * (Rashmi, Shah, Kumar 2011), the standard PM-MSR / PM-MBR definitions that
 * the paper restates in Section 2 and Section 3.3.  Readings of ambiguous
 * passages are marked "Reading:".
 *
 * Conventions: nodes are 0-based (paper's i is i+1 here); matrices are
 * row-major uint8_t arrays; a byte region is a plain host pointer.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ------------------------------------------------------------------------ */
/* Field GF(2^8): the default field of GF-Complete (Section 3.3, the paragraph
 * on computational validity).  Reading: polynomial x^8+x^4+x^3+x^2+1 (0x11D)
 * with generator g = 2; this choice reproduces the paper's validity range
 * k in {2..39} for the sparse construction (tested).
 * add = sub = XOR; mul/div through exponent and logarithm tables.          */
static uint8_t EXP_T[255];
static int LOG_T[256];
static int field_ready = 0;

void or_init(void)
{
    if (field_ready) return;
    unsigned a = 1;
    for (int i = 0; i < 255; i++) {
        EXP_T[i] = (uint8_t)a;
        LOG_T[a] = i;
        a <<= 1;                       /* multiply by g = x */
        if (a & 0x100) a ^= 0x11D;     /* reduce modulo the field polynomial */
    }
    LOG_T[0] = -1;
    field_ready = 1;
}

uint8_t or_mul(uint8_t a, uint8_t b)
{
    if (a == 0 || b == 0) return 0;
    return EXP_T[(LOG_T[a] + LOG_T[b]) % 255];
}

/* multiplicative inverse; a must be nonzero (returns 0 for a == 0) */
uint8_t or_inv(uint8_t a)
{
    if (a == 0) return 0;
    return EXP_T[(255 - LOG_T[a]) % 255];
}

uint8_t or_div(uint8_t a, uint8_t b) { return or_mul(a, or_inv(b)); }

/* g^e for any integer e */
uint8_t or_gpow(long e)
{
    long r = e % 255;
    if (r < 0) r += 255;
    return EXP_T[r];
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra over GF(2^8) on small row-major matrices.            */

/* C (m x n) = A (m x k) * B (k x n) */
void or_matmul(const uint8_t *A, const uint8_t *B, uint8_t *C, int m, int k, int n)
{
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) {
            uint8_t acc = 0;
            for (int t = 0; t < k; t++) acc ^= or_mul(A[i * k + t], B[t * n + j]);
            C[i * n + j] = acc;
        }
}

/* Gauss-Jordan elimination on [A | I].  Returns 0 and fills Ainv (n x n), or
 * -1 when A is singular.  The inverse is unique, so the pivot order chosen
 * here does not matter for any result. */
int or_invert(const uint8_t *A, uint8_t *Ainv, int n)
{
    uint8_t *W = (uint8_t *)malloc((size_t)n * 2 * n);
    if (!W) return -2;
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++) {
            W[i * 2 * n + j] = A[i * n + j];
            W[i * 2 * n + n + j] = (uint8_t)(i == j);
        }
    }
    for (int col = 0; col < n; col++) {
        int piv = -1;
        for (int r = col; r < n; r++)
            if (W[r * 2 * n + col]) { piv = r; break; }
        if (piv < 0) { free(W); return -1; }
        if (piv != col)
            for (int j = 0; j < 2 * n; j++) {
                uint8_t t = W[piv * 2 * n + j];
                W[piv * 2 * n + j] = W[col * 2 * n + j];
                W[col * 2 * n + j] = t;
            }
        uint8_t s = or_inv(W[col * 2 * n + col]);
        for (int j = 0; j < 2 * n; j++) W[col * 2 * n + j] = or_mul(W[col * 2 * n + j], s);
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            uint8_t f = W[r * 2 * n + col];
            if (!f) continue;
            for (int j = 0; j < 2 * n; j++) W[r * 2 * n + j] ^= or_mul(f, W[col * 2 * n + j]);
        }
    }
    for (int i = 0; i < n; i++) memcpy(Ainv + i * n, W + i * 2 * n + n, (size_t)n);
    free(W);
    return 0;
}

/* rank of an m x n matrix */
int or_rank(const uint8_t *A, int m, int n)
{
    uint8_t *W = (uint8_t *)malloc((size_t)m * n + 1);
    memcpy(W, A, (size_t)m * n);
    int rank = 0;
    for (int col = 0; col < n && rank < m; col++) {
        int piv = -1;
        for (int r = rank; r < m; r++)
            if (W[r * n + col]) { piv = r; break; }
        if (piv < 0) continue;
        for (int j = 0; j < n; j++) {
            uint8_t t = W[piv * n + j]; W[piv * n + j] = W[rank * n + j]; W[rank * n + j] = t;
        }
        uint8_t s = or_inv(W[rank * n + col]);
        for (int r = 0; r < m; r++) {
            if (r == rank) continue;
            uint8_t f = or_mul(W[r * n + col], s);
            if (!f) continue;
            for (int j = 0; j < n; j++) W[r * n + j] ^= or_mul(f, W[rank * n + j]);
        }
        rank++;
    }
    free(W);
    return rank;
}

/* ------------------------------------------------------------------------ */
/* Code parameters (Section 2, the paragraph on MSR and MBR codes):
 *   MSR: alpha = Delta = d - k + 1, B = k * Delta; the PM-MSR construction
 *        works at d = 2k - 2, so alpha = k - 1 and B = k (k - 1).
 *   MBR: alpha = d, Delta = (2d - k + 1) / 2, B = k d - k (k - 1) / 2.
 *   beta = 1 (one block downloaded from each of the d helpers).
 * kind: 0 = MSR, 1 = MBR, 2 = Reed-Solomon baseline (alpha = 1, B = k).   */
int or_dims(int kind, int k, int d, int n, int *alpha, int *B)
{
    if (k < 1 || n < k || n > 255) return -1;
    if (kind == 0) {
        if (k < 2 || d != 2 * k - 2 || n < d + 1) return -1;
        *alpha = k - 1; *B = k * (k - 1);
    } else if (kind == 1) {
        if (d < k || n < d + 1) return -1;
        *alpha = d; *B = k * d - k * (k - 1) / 2;
    } else if (kind == 2) {
        *alpha = 1; *B = k;
    } else return -1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Encoding matrix Psi (n x d) and the diagonal Lambda of PM-MSR.            */

/* Vanilla PM-MSR (Section 3.3, the Vandermonde construction and its n=5,
 * k=3 example): Phi[i][j] = x_i^j (j < alpha), Lambda_i = x_i^alpha, so
 * Psi = [Phi, Lambda Phi] has Psi[i][c] = x_i^c for c < 2 alpha.  The paper
 * takes x_i = g^(i-1) (1-based), i.e. g^i here; x may override it. */
int or_msr_vanilla(int k, int n, const uint8_t *x, uint8_t *psi, uint8_t *lam)
{
    int alpha = k - 1, d = 2 * alpha;
    for (int i = 0; i < n; i++) {
        uint8_t xi = x ? x[i] : or_gpow(i);
        uint8_t p = 1;
        for (int c = 0; c < d; c++) { psi[i * d + c] = p; p = or_mul(p, xi); }
        lam[i] = psi[i * d + alpha];            /* x_i^alpha */
    }
    return 0;
}

/* Sparse PM-MSR exactly as printed (Section 3.3, the construction proposed
 * by the paper and its n=5, k=3 example), with 1-based i, j:
 *   Phi_{i,j} = [i == j]                          for i <= alpha,
 *   Phi_{i,j} = 1 / (g^(i+alpha) - g^(j-1))        for i >  alpha,
 *   Lambda_{i,i} = (g^(i+alpha) - g^0) / (g^(i+alpha) - g^alpha),
 *   Psi = [Phi, Lambda Phi].   In characteristic 2, "-" is XOR. */
int or_msr_sparse_printed(int k, int n, uint8_t *psi, uint8_t *lam)
{
    int alpha = k - 1, d = 2 * alpha;
    for (int t = 0; t < n; t++) {
        int i = t + 1;                           /* paper's 1-based row index */
        uint8_t xi = or_gpow(i + alpha);
        for (int j = 1; j <= alpha; j++) {
            uint8_t phi;
            if (i <= alpha) phi = (uint8_t)(i == j);
            else {
                uint8_t den = xi ^ or_gpow(j - 1);
                if (!den) return -1;
                phi = or_inv(den);
            }
            psi[t * d + (j - 1)] = phi;
        }
        uint8_t den = xi ^ or_gpow(alpha);
        if (!den) return -1;
        lam[t] = or_div(xi ^ 1, den);
        for (int j = 0; j < alpha; j++) psi[t * d + alpha + j] = or_mul(lam[t], psi[t * d + j]);
    }
    return 0;
}

/* Every d x d submatrix of Psi whose rows include `must` (or all of them when
 * must < 0) is invertible.  This is the computational check of Section 3.3
 * (validity paragraph). */
static int next_subset(int *idx, int m, int n)
{
    int i = m - 1;
    while (i >= 0 && idx[i] == n - m + i) i--;
    if (i < 0) return 0;
    idx[i]++;
    for (int j = i + 1; j < m; j++) idx[j] = idx[j - 1] + 1;
    return 1;
}

int or_all_dsubsets_invertible(const uint8_t *psi, int n, int d, int must)
{
    int *idx = (int *)malloc(sizeof(int) * (size_t)d);
    uint8_t *S = (uint8_t *)malloc((size_t)d * d), *Si = (uint8_t *)malloc((size_t)d * d);
    for (int i = 0; i < d; i++) idx[i] = i;
    int ok = 1;
    do {
        int has = (must < 0);
        for (int i = 0; i < d; i++) if (idx[i] == must) has = 1;
        if (!has) continue;
        for (int i = 0; i < d; i++) memcpy(S + i * d, psi + idx[i] * d, (size_t)d);
        if (or_invert(S, Si, d) != 0) { ok = 0; break; }
    } while (next_subset(idx, d, n));
    free(idx); free(S); free(Si);
    return ok;
}

static int lambda_distinct(const uint8_t *lam, int n)
{
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (lam[i] == lam[j]) return 0;
    return 1;
}

/* Validity of an MSR encoding matrix (Section 3.3, the constraint list and
 * the validity paragraph): Lambda entries distinct and every d rows of Psi
 * linearly independent.  (Any alpha rows of Phi are independent by
 * construction for both constructions: Vandermonde, resp. identity over a
 * Cauchy matrix.)  Returns 1 when valid. */
int or_msr_valid(const uint8_t *psi, const uint8_t *lam, int n, int d)
{
    if (!lambda_distinct(lam, n)) return 0;
    return or_all_dsubsets_invertible(psi, n, d, -1);
}

/* Sparse PM-MSR used by the library and the configurations.
 * Reading (the paper is silent beyond n = d + 1 = 2k - 1, where it checks
 * "all n possible d x d sub-matrices"): at n = 2k the printed construction has
 * alpha + 2 Cauchy rows, and its Lambda*Phi block on those rows has rank at
 * most alpha + 1 (partial fractions), so helper sets holding every Cauchy row
 * are singular.  Rows 1..2k-1 are kept exactly as printed and the last node
 * keeps its printed Phi row but takes Lambda = g^t for the smallest t >= 0
 * such that g^t differs from every other Lambda entry and every d-subset of
 * Psi containing that node is invertible.  n must be 2k-1 or 2k. */
int or_msr_sparse(int k, int n, uint8_t *psi, uint8_t *lam)
{
    int alpha = k - 1, d = 2 * alpha;
    if (n != 2 * k - 1 && n != 2 * k) return -1;
    if (or_msr_sparse_printed(k, n, psi, lam) != 0) return -1;
    if (n == 2 * k - 1) return 0;
    int last = n - 1;
    for (int t = 0; t < 255; t++) {
        uint8_t cand = or_gpow(t);
        int clash = 0;
        for (int i = 0; i < last; i++) if (lam[i] == cand) clash = 1;
        if (clash) continue;
        lam[last] = cand;
        for (int j = 0; j < alpha; j++) psi[last * d + alpha + j] = or_mul(cand, psi[last * d + j]);
        if (or_all_dsubsets_invertible(psi, n, d, last)) return 0;
    }
    return -1;
}

/* PM-MBR systematic encoding matrix.  The paper (Section 3.2) only says the
 * seminal paper gives a systematic Psi whose first rows are the identity;
 * PM-MBR needs Psi = [Phi, Delta] (n x d, Phi n x k) with any d rows of Psi
 * and any k rows of Phi independent.
 * Reading: start from the Vandermonde Psi0[i][c] = g^(i c) (c < d) and right-
 * multiply by the invertible block upper-triangular T = [[P^-1, P^-1 D],[0, I]]
 * with P, D the top k rows of Phi0, Delta0.  Both properties survive, and the
 * first k rows become [I_k | 0]. */
int or_mbr_psi(int k, int d, int n, uint8_t *psi)
{
    uint8_t *P0 = (uint8_t *)malloc((size_t)n * d);
    for (int i = 0; i < n; i++)
        for (int c = 0; c < d; c++) P0[i * d + c] = or_gpow((long)i * c);
    uint8_t *T = (uint8_t *)calloc((size_t)d * d, 1);
    uint8_t *P = (uint8_t *)malloc((size_t)k * k), *Pi = (uint8_t *)malloc((size_t)k * k);
    for (int r = 0; r < k; r++) memcpy(P + r * k, P0 + r * d, (size_t)k);
    if (or_invert(P, Pi, k) != 0) { free(P0); free(T); free(P); free(Pi); return -1; }
    /* T top-left = P^-1 ; top-right = P^-1 * D ; bottom-right = I */
    for (int r = 0; r < k; r++)
        for (int c = 0; c < k; c++) T[r * d + c] = Pi[r * k + c];
    for (int r = 0; r < k; r++)
        for (int c = k; c < d; c++) {
            uint8_t acc = 0;
            for (int t = 0; t < k; t++) acc ^= or_mul(Pi[r * k + t], P0[t * d + c]);
            T[r * d + c] = acc;
        }
    for (int c = k; c < d; c++) T[c * d + c] = 1;
    or_matmul(P0, T, psi, n, d, d);
    free(P0); free(T); free(P); free(Pi);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Index matrix L with M[l][j] = X[L[l][j]] (Section 3.1, first paragraph and
 * its k = 3 example).  -1 marks a structural zero of M.                     */

/* MSR: M = [S1; S2] with S1, S2 symmetric alpha x alpha.  Each upper triangle
 * is numbered row by row, S1 before S2; for alpha = 2 this is the printed
 * example.  Reading for alpha >= 3: row-major (the systematic generator does
 * not depend on the order, tested). L is d x alpha. */
int or_index_msr(int k, int *L)
{
    int alpha = k - 1, idx = 0;
    for (int s = 0; s < 2; s++)
        for (int r = 0; r < alpha; r++)
            for (int c = r; c < alpha; c++) {
                L[(s * alpha + r) * alpha + c] = idx;
                L[(s * alpha + c) * alpha + r] = idx;
                idx++;
            }
    return idx;
}

/* MBR: M = [[S, T], [T^t, 0]] (d x d) with S k x k symmetric (upper triangle
 * numbered row by row) followed by T k x (d-k) numbered row by row. */
int or_index_mbr(int k, int d, int *L)
{
    int idx = 0;
    for (int i = 0; i < d * d; i++) L[i] = -1;
    for (int r = 0; r < k; r++)
        for (int c = r; c < k; c++) { L[r * d + c] = idx; L[c * d + r] = idx; idx++; }
    for (int r = 0; r < k; r++)
        for (int c = k; c < d; c++) { L[r * d + c] = idx; L[c * d + r] = idx; idx++; }
    return idx;
}

/* Linearization (Section 3.1): G[alpha i + j][L[l][j]] = Psi[i][l], zero
 * elsewhere.  G is (n alpha) x B. */
void or_linearize(const uint8_t *psi, const int *L, int n, int d, int alpha, int B, uint8_t *G)
{
    memset(G, 0, (size_t)n * alpha * B);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < alpha; j++)
            for (int l = 0; l < d; l++) {
                int m = L[l * alpha + j];
                if (m >= 0) G[(size_t)(alpha * i + j) * B + m] ^= psi[i * d + l];
            }
}

/* Product-matrix encoding as the seminal paper defines it (Section 2, last
 * paragraphs; Section 3.1): C = Psi M with M[l][j] = X[L[l][j]].  Node i,
 * block j gets sum_l Psi[i][l] * X[L[l][j]] byte by byte.  Used only to check
 * the linearized generator. */
void or_specific_encode(const uint8_t *psi, const int *L, int n, int d, int alpha,
                        const uint8_t *const *X, uint8_t *const *C, size_t s)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < alpha; j++) {
            uint8_t *out = C[i * alpha + j];
            memset(out, 0, s);
            for (int l = 0; l < d; l++) {
                int m = L[l * alpha + j];
                if (m < 0) continue;
                uint8_t coef = psi[i * d + l];
                for (size_t p = 0; p < s; p++) out[p] ^= or_mul(coef, X[m][p]);
            }
        }
}

/* Systematic form (Section 3.2): G' = G * inverse(first B rows of G).
 * Returns -1 when those rows are singular. */
int or_systematic(const uint8_t *G, int rows, int B, uint8_t *Gp)
{
    uint8_t *Gt = (uint8_t *)malloc((size_t)B * B), *Gti = (uint8_t *)malloc((size_t)B * B);
    memcpy(Gt, G, (size_t)B * B);
    int rc = or_invert(Gt, Gti, B);
    if (rc == 0) or_matmul(G, Gti, Gp, rows, B, B);
    free(Gt); free(Gti);
    return rc;
}

/* Reed-Solomon baseline (Section 4, the list of evaluated codes): the
 * systematic Vandermonde code, V[i][c] = g^(i c), G = V * inverse(V[0:k]).
 * Writes all n x k rows of G. */
int or_rs_generator(int k, int n, uint8_t *G)
{
    uint8_t *V = (uint8_t *)malloc((size_t)n * k);
    for (int i = 0; i < n; i++)
        for (int c = 0; c < k; c++) V[i * k + c] = or_gpow((long)i * c);
    int rc = or_systematic(V, n, k, G);
    free(V);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Data phase: the region matrix product out[r] = sum_c A[r][c] * in[c],
 * byte by byte (Section 2: Y = G X; Section 4: Jerasure applies the matrix
 * to the blocks).  Threads split the byte range only, for timing. */
typedef struct {
    const uint8_t *A; int rows, cols;
    const uint8_t *const *in; uint8_t *const *out;
    size_t p0, p1;
} apply_job;

static void apply_range(const apply_job *j)
{
    for (int r = 0; r < j->rows; r++) {
        uint8_t *o = j->out[r];
        for (size_t p = j->p0; p < j->p1; p++) {
            uint8_t acc = 0;
            for (int c = 0; c < j->cols; c++) acc ^= or_mul(j->A[r * j->cols + c], j->in[c][p]);
            o[p] = acc;
        }
    }
}

static void *apply_thread(void *arg) { apply_range((const apply_job *)arg); return NULL; }

void or_apply(const uint8_t *A, int rows, int cols, const uint8_t *const *in,
              uint8_t *const *out, size_t s, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    apply_job jobs[256];
    pthread_t th[256];
    size_t chunk = (s + (size_t)nthreads - 1) / (size_t)nthreads;
    for (int t = 0; t < nthreads; t++) {
        jobs[t].A = A; jobs[t].rows = rows; jobs[t].cols = cols;
        jobs[t].in = in; jobs[t].out = out;
        jobs[t].p0 = (size_t)t * chunk < s ? (size_t)t * chunk : s;
        jobs[t].p1 = jobs[t].p0 + chunk < s ? jobs[t].p0 + chunk : s;
    }
    if (nthreads == 1) { apply_range(&jobs[0]); return; }
    int ok[256];
    for (int t = 0; t < nthreads; t++) {
        ok[t] = pthread_create(&th[t], NULL, apply_thread, &jobs[t]) == 0;
        if (!ok[t]) apply_range(&jobs[t]);
    }
    for (int t = 0; t < nthreads; t++) if (ok[t]) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------ */
/* Repair (Section 2, the paragraph on repair with d helpers and its
 * footnote; the algorithm is the seminal paper's).  Failed node f, helpers H
 * (d distinct nodes, given order).
 *   helper row:  MSR  phi_f (the first alpha entries of Psi[f]);
 *                MBR  psi_f (all d entries);   RS: [1].
 *   newcomer:    MSR  R = [I_alpha | lambda_f I_alpha] * inverse(Psi_H);
 *                MBR  R = inverse(Psi_H);
 *                RS   R = G[f] * inverse(G_H)   (decode then re-encode).
 * Psi_H stacks the rows of Psi (or, for RS, of G) of the helpers in order.
 * Why: helper h sends psi_h^T M phi_f, so the newcomer receives
 * Psi_H (M phi_f); M's blocks are symmetric, so node f's content is
 * phi_f^T S1 + lambda_f phi_f^T S2 (MSR) or psi_f^T M (MBR).            */
void or_helper_row(int kind, const uint8_t *psi, int d, int alpha, int f, uint8_t *row)
{
    if (kind == 2) { row[0] = 1; return; }
    for (int a = 0; a < alpha; a++) row[a] = psi[f * d + a];
}

/* R has alpha rows and d columns (RS: 1 x k).  Returns -1 when Psi_H is singular. */
int or_newcomer_matrix(int kind, const uint8_t *psi_or_g, const uint8_t *lam, int d, int alpha,
                       int f, const int *H, uint8_t *R)
{
    int m = d;   /* Psi_H is d x d (RS: G_H is k x k with d = k) */
    uint8_t *S = (uint8_t *)malloc((size_t)m * m), *Si = (uint8_t *)malloc((size_t)m * m);
    for (int i = 0; i < m; i++) memcpy(S + i * m, psi_or_g + H[i] * m, (size_t)m);
    if (or_invert(S, Si, m) != 0) { free(S); free(Si); return -1; }
    if (kind == 1) {
        memcpy(R, Si, (size_t)m * m);
    } else if (kind == 0) {
        /* [I | lambda_f I] * Si : row a = Si[a] + lambda_f * Si[alpha + a] */
        for (int a = 0; a < alpha; a++)
            for (int c = 0; c < d; c++)
                R[a * d + c] = Si[a * d + c] ^ or_mul(lam[f], Si[(alpha + a) * d + c]);
    } else {
        /* RS: row f of G times inverse(G_H) */
        or_matmul(psi_or_g + f * m, Si, R, 1, m, m);
    }
    free(S); free(Si);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Specific PM-MSR decoding: the data-collector algorithm of the seminal
 * product-matrix paper, which the paper's Section 2 refers to and whose cost
 * Section 4.1 (decoding paragraph) compares with the linearized decode.
 * Reading (the paper does not restate its steps; they follow from the MSR
 * structure it gives in Section 2: Psi = [Phi, Lambda Phi], M = [S1; S2] with
 * S1, S2 symmetric alpha x alpha, node i storing phi_i^t S1 + lambda_i phi_i^t S2):
 *  1. Z = Y_DC Phi_DC^t, so Z[i][j] = P_ij + lambda_i Q_ij with
 *     P = Phi_DC S1 Phi_DC^t and Q = Phi_DC S2 Phi_DC^t, both symmetric;
 *  2. for i < j, the pair Z[i][j], Z[j][i] gives Q_ij = (Z[i][j] + Z[j][i]) /
 *     (lambda_i + lambda_j) and P_ij = Z[i][j] + lambda_i Q_ij;
 *  3. for each of the first alpha connected nodes i, the alpha values P_ij
 *     (j != i) equal phi_i^t S1 phi_j, so phi_i^t S1 solves an alpha x alpha
 *     system with rows phi_j^t (likewise phi_i^t S2 from Q);
 *  4. those alpha rows form Phi_A S1 (Phi_A S2), inverted for S1 (S2);
 *  5. M gives the message Z_m = M[l][j] at m = L[l][j]; a systematic code
 *     (Section 3.2) stored G Z with Z = inverse(G~) X, so X = G~ Z is the
 *     product-matrix encoding of Z for the first k nodes.
 * The matrices of steps 3-4 do not depend on the data and are inverted once;
 * the rest runs byte position by byte position.  K lists k distinct nodes,
 * Y their k alpha blocks node-major, X receives B blocks.  Returns -1 when a
 * system is singular or the lambda_i of K are not distinct, -2 when Psi does
 * not have the [Phi, Lambda Phi] form. */
int or_msr_specific_decode(const uint8_t *psi, const uint8_t *lam, const int *L, int k, int n,
                           const int *K, const uint8_t *const *Y, int systematic,
                           uint8_t *const *X, size_t s)
{
    const int alpha = k - 1, d = 2 * alpha, B = alpha * (alpha + 1);
    (void)n;
    for (int i = 0; i < k; i++)
        for (int a = 0; a < alpha; a++)
            if (psi[K[i] * d + alpha + a] != or_mul(lam[K[i]], psi[K[i] * d + a])) return -2;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            if (lam[K[i]] == lam[K[j]]) return -1;
    /* step 3 systems: Finv[i] inverts the rows phi_j^t, j != i (i < alpha) */
    uint8_t *Finv = (uint8_t *)malloc((size_t)alpha * alpha * alpha);
    uint8_t *F = (uint8_t *)malloc((size_t)alpha * alpha);
    uint8_t *PhiA = (uint8_t *)malloc((size_t)alpha * alpha), *PhiAinv = (uint8_t *)malloc((size_t)alpha * alpha);
    int rc = 0;
    for (int i = 0; i < alpha && rc == 0; i++) {
        int r = 0;
        for (int j = 0; j < k; j++) {
            if (j == i) continue;
            memcpy(F + r * alpha, psi + K[j] * d, (size_t)alpha);
            r++;
        }
        rc = or_invert(F, Finv + (size_t)i * alpha * alpha, alpha);
    }
    for (int i = 0; i < alpha; i++) memcpy(PhiA + i * alpha, psi + K[i] * d, (size_t)alpha);
    if (rc == 0) rc = or_invert(PhiA, PhiAinv, alpha);
    uint8_t *y = (uint8_t *)malloc((size_t)k * alpha), *z = (uint8_t *)malloc((size_t)k * k);
    uint8_t *P = (uint8_t *)malloc((size_t)k * k), *Q = (uint8_t *)malloc((size_t)k * k);
    uint8_t *U = (uint8_t *)malloc((size_t)alpha * alpha), *V = (uint8_t *)malloc((size_t)alpha * alpha);
    uint8_t *S1 = (uint8_t *)malloc((size_t)alpha * alpha), *S2 = (uint8_t *)malloc((size_t)alpha * alpha);
    uint8_t *Zm = (uint8_t *)malloc((size_t)B), *pv = (uint8_t *)malloc((size_t)alpha), *qv = (uint8_t *)malloc((size_t)alpha);
    for (size_t p = 0; p < s && rc == 0; p++) {
        for (int t = 0; t < k * alpha; t++) y[t] = Y[t][p];
        /* step 1 */
        for (int i = 0; i < k; i++)
            for (int j = 0; j < k; j++) {
                uint8_t acc = 0;
                for (int a = 0; a < alpha; a++) acc ^= or_mul(y[i * alpha + a], psi[K[j] * d + a]);
                z[i * k + j] = acc;
            }
        /* step 2 */
        for (int i = 0; i < k; i++)
            for (int j = i + 1; j < k; j++) {
                uint8_t q = or_div(z[i * k + j] ^ z[j * k + i], lam[K[i]] ^ lam[K[j]]);
                uint8_t pp = z[i * k + j] ^ or_mul(lam[K[i]], q);
                P[i * k + j] = P[j * k + i] = pp;
                Q[i * k + j] = Q[j * k + i] = q;
            }
        /* step 3: U[i] = phi_i^t S1, V[i] = phi_i^t S2 for the first alpha nodes */
        for (int i = 0; i < alpha; i++) {
            int r = 0;
            for (int j = 0; j < k; j++) {
                if (j == i) continue;
                pv[r] = P[i * k + j];
                qv[r] = Q[i * k + j];
                r++;
            }
            or_matmul(Finv + (size_t)i * alpha * alpha, pv, U + i * alpha, alpha, alpha, 1);
            or_matmul(Finv + (size_t)i * alpha * alpha, qv, V + i * alpha, alpha, alpha, 1);
        }
        /* step 4 */
        or_matmul(PhiAinv, U, S1, alpha, alpha, alpha);
        or_matmul(PhiAinv, V, S2, alpha, alpha, alpha);
        /* step 5: message symbols, then the data */
        for (int l = 0; l < d; l++)
            for (int j = 0; j < alpha; j++)
                Zm[L[l * alpha + j]] = l < alpha ? S1[l * alpha + j] : S2[(l - alpha) * alpha + j];
        if (!systematic) {
            for (int m = 0; m < B; m++) X[m][p] = Zm[m];
        } else {
            for (int i = 0; i < k; i++)
                for (int j = 0; j < alpha; j++) {
                    uint8_t acc = 0;
                    for (int l = 0; l < d; l++) acc ^= or_mul(psi[i * d + l], Zm[L[l * alpha + j]]);
                    X[i * alpha + j][p] = acc;
                }
        }
    }
    free(Finv); free(F); free(PhiA); free(PhiAinv); free(y); free(z); free(P); free(Q);
    free(U); free(V); free(S1); free(S2); free(Zm); free(pv); free(qv);
    return rc == 0 ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Specific PM-MBR decoding: the data-collector algorithm of the seminal
 * product-matrix paper for MBR, which the paper's Section 2 refers to and
 * whose cost its MBR subsection of Section 4 (decoding paragraph) compares
 * with the linearized decode.  Reading (the paper does not restate the
 * steps; they follow from the MBR structure: M = [[S, T], [T^t, 0]] with S
 * symmetric k x k and T k x (d-k), Psi = [Phi, Delta] with Phi n x k and
 * Delta n x (d-k), node i storing psi_i^t M):
 *  1. the k connected nodes hold Psi_DC M = [Phi_DC S + Delta_DC T^t,
 *     Phi_DC T], so T = inverse(Phi_DC) times their last d-k blocks;
 *  2. S = inverse(Phi_DC) (their first k blocks + Delta_DC T^t) (minus is
 *     plus in characteristic 2);
 *  3. the message symbol m = L[l][j] is M[l][j].  This code is systematic
 *     through Psi itself (its first k rows are [I_k, 0], Section 3.2), so
 *     the data are the message symbols.
 * K lists k distinct nodes, Y their k d blocks node-major, X receives B
 * blocks.  Returns -1 when Phi_DC is singular. */
int or_mbr_specific_decode(const uint8_t *psi, const int *L, int k, int d, const int *K,
                           const uint8_t *const *Y, uint8_t *const *X, size_t s)
{
    const int dk = d - k;
    uint8_t *Phi = (uint8_t *)malloc((size_t)k * k), *Phinv = (uint8_t *)malloc((size_t)k * k);
    for (int i = 0; i < k; i++) memcpy(Phi + i * k, psi + K[i] * d, (size_t)k);
    int rc = or_invert(Phi, Phinv, k);
    uint8_t *yl = (uint8_t *)malloc((size_t)k * (dk ? dk : 1)), *T = (uint8_t *)malloc((size_t)k * (dk ? dk : 1));
    uint8_t *R = (uint8_t *)malloc((size_t)k * k), *S = (uint8_t *)malloc((size_t)k * k);
    for (size_t p = 0; p < s && rc == 0; p++) {
        /* step 1 */
        for (int i = 0; i < k; i++)
            for (int t = 0; t < dk; t++) yl[i * dk + t] = Y[i * d + k + t][p];
        if (dk) or_matmul(Phinv, yl, T, k, k, dk);
        /* step 2: R[i][j] = y_i[j] + sum_t Delta[i][t] T[j][t] */
        for (int i = 0; i < k; i++)
            for (int j = 0; j < k; j++) {
                uint8_t acc = Y[i * d + j][p];
                for (int t = 0; t < dk; t++) acc ^= or_mul(psi[K[i] * d + k + t], T[j * dk + t]);
                R[i * k + j] = acc;
            }
        or_matmul(Phinv, R, S, k, k, k);
        /* step 3 */
        for (int l = 0; l < d; l++)
            for (int j = 0; j < d; j++) {
                const int m = L[l * d + j];
                if (m < 0) continue;
                X[m][p] = l < k ? (j < k ? S[l * k + j] : T[l * dk + (j - k)]) : T[j * dk + (l - k)];
            }
    }
    free(Phi); free(Phinv); free(yl); free(T); free(R); free(S);
    return rc == 0 ? 0 : -1;
}

/* ------------------------------------------------------------------------ */
/* Decode (Section 2: X = inverse(G~) Y~ over the rows of the surviving
 * blocks).  Gsys is the generator the nodes were encoded with (systematic or
 * not), (n alpha) x B.  K lists k nodes; their k alpha rows are scanned in
 * order and each row independent of the rows kept so far is kept until B are
 * kept (for MSR and RS exactly B rows exist; for MBR the k d rows have rank B:
 * reading, first-found).  kept[] receives the indices (into the k alpha
 * received blocks) of the rows used; D (B x B) is the inverse of those rows.
 * Returns -1 when fewer than B independent rows exist. */
int or_decode_matrix(const uint8_t *Gsys, int B, int alpha, const int *K, int k,
                     uint8_t *D, int *kept)
{
    int total = k * alpha, nk = 0;
    uint8_t *Sel = (uint8_t *)malloc((size_t)B * B);
    for (int t = 0; t < total && nk < B; t++) {
        int node = K[t / alpha], j = t % alpha;
        memcpy(Sel + (size_t)nk * B, Gsys + (size_t)(node * alpha + j) * B, (size_t)B);
        if (or_rank(Sel, nk + 1, B) == nk + 1) kept[nk++] = t;
    }
    int rc = -1;
    if (nk == B) rc = or_invert(Sel, D, B);
    free(Sel);
    return rc;
}
