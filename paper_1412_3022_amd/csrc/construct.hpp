// Host construction of PM-MSR / PM-MBR codes (the "initialization" phase of
// the paper's Section 4): encoding matrix Psi, index matrix L, linearized
// generator G (Section 3.1), systematic generator G' = [I; G''] (Section 3.2),
// and the per-failure-pattern repair and decode matrices.
#pragma once
#include <cstdint>
#include <vector>

#include "gf256.hpp"

namespace pmrc {

enum Kind { KIND_MSR = 0, KIND_MBR = 1, KIND_RS = 2 };
enum Construction { CONS_VANILLA = 0, CONS_SPARSE = 1 };

struct CodeSpec {
    int kind = KIND_MSR, construction = CONS_SPARSE, systematic = 1;
    int k = 0, d = 0, n = 0;
    std::vector<uint8_t> x;  // optional vanilla evaluation points (n entries)
};

struct CodeMats {
    int kind = 0, construction = 0, systematic = 1;
    int k = 0, d = 0, n = 0, alpha = 0, B = 0;
    Mat psi;                      // n x d (RS: the n x k generator)
    std::vector<uint8_t> lambda;  // MSR only, n entries
    std::vector<int> L;           // index matrix (MSR d x alpha, MBR d x d), -1 = zero
    Mat G;                        // linearized generator, (n alpha) x B
    Mat Gsys;                     // generator the node contents follow
    Mat enc;                      // rows written by encode
    std::vector<int32_t> node_map;  // per node block: < B -> X block, >= B -> enc row + B
};

// Status codes shared with the C ABI.
enum {
    ST_OK = 0, ST_EINVAL = -1, ST_EUNSUPPORTED = -2, ST_ESINGULAR = -3,
    ST_ENOMEM = -4, ST_EHIP = -5, ST_EBUSY = -6, ST_ENOTREADY = -7, ST_ELIMIT = -8,
};

int build_code(const CodeSpec &spec, CodeMats &out);

// Index matrix of PM-MSR (2 alpha x alpha, row-major): M = [S1; S2] with the
// upper triangles of S1 then S2 numbered row by row (Section 3.1).
std::vector<int> index_msr(int alpha);

// Repair: the helper's projection row (1 x alpha; RS 1 x 1).
Mat helper_row(const CodeMats &c, int failed);
// Repair: the newcomer's matrix for helpers H (alpha x d; RS 1 x k).
int newcomer_matrix(const CodeMats &c, int failed, const std::vector<int> &helpers, Mat &R);
// Decode from nodes K: D (B x B) and the received block indices it reads.
int decode_matrix(const CodeMats &c, const std::vector<int> &nodes, Mat &D, std::vector<int> &used);

// Specific PM-MSR decoding from the k nodes K, as five sparse factors whose
// product is the linearized decode matrix:
//   F[0] (k(k-1) x k alpha): Z_ij = y_i . phi_j for i != j, from node i's
//        blocks only (rows i-major);
//   F[1] (B x k(k-1)): P_ij and Q_ij of every node pair i < j (pairs in
//        order, all P rows then all Q rows) from Z_ij and Z_ji;
//   F[2] (2 alpha^2 x B): phi_i^t S1 and phi_i^t S2 for the first alpha
//        nodes of K (alpha x alpha solves);
//   F[3] (B x 2 alpha^2): the message symbols, S1 = inverse(Phi_A) U and
//        S2 = inverse(Phi_A) V;
//   F[4] (B x B): systematic codes only, X = G~ Z (rows 0 otherwise).
// Specific PM-MBR decoding from the k nodes K, as two factors:
//   F[0] (w x k d): T = inverse(Phi_K) times the last d - k blocks of each
//        node (k (d-k) rows), then copies of the first-k node blocks that
//        F[1] reads;
//   F[1] (B x w): the message symbols, T copied and S from the first-k
//        blocks and T; F[2..4] are empty.
// The passes run in order while F[p] has rows.  ST_EUNSUPPORTED for RS,
// ST_ESINGULAR for a singular system.
constexpr int kSpecificPasses = 5;
int specific_decode_factors(const CodeMats &c, const std::vector<int> &K, Mat F[kSpecificPasses]);

}  // namespace pmrc
