// GF(2^16) codes: the sparse PM-MSR construction over GF(2^16) (Section 3.3:
// valid there for k up to 64, against 39 in GF(2^8)), its matrices, and the
// host side of the GF(2^16) region kernel.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "construct.hpp"
#include "engine.hpp"

namespace pmrc {
namespace w16 {

// Field: x^16 + x^12 + x^3 + x + 1 (0x1100B), generator g = 2: GF-Complete's
// default GF(2^16).
uint16_t mul(uint16_t a, uint16_t b);
uint16_t inv(uint16_t a);
uint16_t gpow(long e);

// Row-major dense matrix over GF(2^16).
struct Mat16 {
    int rows = 0, cols = 0;
    std::vector<uint16_t> v;
    Mat16() = default;
    Mat16(int r, int c) : rows(r), cols(c), v(static_cast<size_t>(r) * c, 0) {}
    uint16_t &at(int r, int c) { return v[static_cast<size_t>(r) * cols + c]; }
    uint16_t at(int r, int c) const { return v[static_cast<size_t>(r) * cols + c]; }
};

Mat16 matmul(const Mat16 &A, const Mat16 &B);
bool invert(const Mat16 &A, Mat16 &out);

struct Code16 {
    int k = 0, d = 0, n = 0, alpha = 0, B = 0, systematic = 1;
    Mat16 psi;                      // n x d
    std::vector<uint16_t> lambda;   // n
    std::vector<int> L;             // d x alpha index matrix
    Mat16 G, Gsys, enc;
    std::vector<int32_t> node_map;  // as CodeMats::node_map
};

// Sparse PM-MSR only (d = 2k - 2, n = 2k - 1 or 2k); other kinds and
// constructions: ST_EUNSUPPORTED.
int build_code(const CodeSpec &spec, Code16 &out);
Mat16 helper_row(const Code16 &c, int failed);
int newcomer_matrix(const Code16 &c, int failed, const std::vector<int> &helpers, Mat16 &R);
int decode_matrix(const Code16 &c, const std::vector<int> &nodes, Mat16 &D);

// A GF(2^16) matrix past one bit-sliced kernel's limit (kBsMaxOps) and
// within kBs16MaxParts kernels of at most kBs16PartOps operations is split
// into that many kernels (parts).  They compile side by side, and a data
// call runs them side by side on two hardware queues: more parts would share
// the process's few queues, and each part alone fills only part of the GPU.
constexpr long kBs16MaxParts = 2;
constexpr long kBs16PartOps = 256000;

// A matrix packed for the kernel, with its per-device copies, and its
// bit-sliced specialization (bitslice16.cpp) when it is small enough.
struct Prog16 {
    std::vector<uint32_t> words;
    uint32_t ngroups = 0;
    int rows = 0, cols = 0;
    Mat16 A;
    std::mutex mu;
    std::map<int, DevCopy> dev;
    bool bs_tried = false;
    int max_parts = static_cast<int>(kBs16MaxParts);   // more parts than this: the table kernel
    std::vector<std::shared_ptr<BsProgram>> bs;   // the bit-sliced kernel's parts
    explicit Prog16(const Mat16 &A);
    ~Prog16() { free_device_copies(dev); }
    // The bit-sliced kernel's parts, generated on first use (none when the
    // matrix is over the size limit).
    std::vector<std::shared_ptr<BsProgram>> bitslice();
};

// Straight-line bit-sliced kernel source for a GF(2^16) matrix (not
// compiled); est_ops over kBsMaxOps means no source.
std::unique_ptr<BsProgram> bs16_generate(const Mat16 &A);
// The bit-sliced form as kernels over consecutive row groups of about equal
// size: one when the matrix is within kBsMaxOps, kBs16MaxParts up to
// kBs16MaxParts x kBs16PartOps operations, none past that (the table kernel
// runs).
std::vector<std::unique_ptr<BsProgram>> bs16_generate_parts(const Mat16 &A);

// The specific PM-MSR decode from the k nodes K as five factors (the
// GF(2^16) counterpart of specific_decode_factors; F[4] empty for a
// non-systematic code).
int specific_factors(const Code16 &c, const std::vector<int> &K, Mat16 F[kSpecificPasses]);

// Everything a GF(2^16) code object holds besides its parameters.
struct Ctx16 {
    Code16 m;
    std::mutex mu;
    struct Specific {
        Mat16 F[kSpecificPasses];
        std::unique_ptr<Prog16> prog[kSpecificPasses];
    };
    std::map<std::vector<int>, Specific> specific;
    std::unique_ptr<Prog16> enc;
    std::map<int, std::unique_ptr<Prog16>> helper;
    std::map<std::pair<int, std::vector<int>>, std::unique_ptr<Prog16>> newcomer;
    std::map<std::vector<int>, std::unique_ptr<Prog16>> decode;
};

// The program of one operation (OPK_*), built on first use.  in_n / out_n:
// the input and output block counts.
int resolve16(Ctx16 &c, int op, uint32_t failed, const uint32_t *ids, Prog16 **pe, size_t *in_n, size_t *out_n);
// The passes of the specific decode from the k nodes ids (factors and
// programs built on first use): npass programs and their output rows.
int resolve_specific16(Ctx16 &c, const uint32_t *ids, Prog16 *pe[kSpecificPasses], int rows[kSpecificPasses],
                       int *npass);
// Factor `which` of a node list already resolved, or nullptr.
const Mat16 *specific_factor16(Ctx16 &c, const uint32_t *ids, int which);
// Upload the program (and the field tables) to the current device and wait
// for those copies (no other work is waited for); with a GPU present also
// loads the bit-sliced kernel if compile16 compiled one.
int stage16(Prog16 &p);
// Init phase: generate and compile the bit-sliced kernel (hipRTC, no GPU
// needed); *specialized = 1 when it is ready.
int compile16(Prog16 &p, int *specialized);
// out (out_n blocks) = A in (in_n blocks), s bytes per block (even).
int launch16(Prog16 &p, const uint8_t *in, size_t in_ld, size_t in_n, uint8_t *out, size_t out_ld, size_t out_n,
             size_t s, hipStream_t stream);

}  // namespace w16
}  // namespace pmrc
