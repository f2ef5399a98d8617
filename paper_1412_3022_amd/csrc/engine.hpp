// Internal interfaces shared by the C ABI, the batch planner and the server:
// device copies of kernel programs and the region-kernel launcher.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>

#include "bitslice.hpp"
#include "gf256.hpp"
#include "program.hpp"

// Arguments of one plain region-kernel launch (defined in kernels.hip).
struct PmkApply {
    const uint8_t *in;
    uint64_t in_ld;
    uint8_t *out;
    uint64_t out_ld;
    uint64_t s;
    const uint32_t *prog;
    uint32_t ngroups;
};
extern "C" hipError_t pmk_apply(int rg, int vec, const PmkApply *h, hipStream_t st);
extern "C" int pmk_tile_bytes(int vec);

struct pm_code;

namespace pmrc {

extern thread_local std::string g_hip_msg;
int hip_fail(hipError_t e);

struct DevCopy {
    void *ptr = nullptr;
    hipEvent_t ready = nullptr;
    bool done = false;
};

// The copy of `bytes` host bytes on the current device in `dev` (guarded by
// mu), uploaded on first use there on an internal stream; `user` is made to
// wait for the upload until it is known to be complete.
int device_copy(std::mutex &mu, std::map<int, DevCopy> &dev, const void *host, size_t bytes, hipStream_t user,
                const void **out);
// Same, but returns only once the copy has landed (for plans, graphs and
// pm_prepare); no stream is made to wait.
int device_copy_sync(std::mutex &mu, std::map<int, DevCopy> &dev, const void *host, size_t bytes,
                     const void **out);
void free_device_copies(std::map<int, DevCopy> &dev);

// A program plus its per-device copies.  device_ptr() uploads on first use
// on the current device (on an internal stream) and makes `user` wait for
// the upload until it is known to be complete.
struct ProgEntry {
    Program prog;
    Mat A;                      // the matrix (for specialized kernels)
    std::vector<int> in_map;
    std::mutex mu;
    std::map<int, DevCopy> dev;
    bool bs_tried = false;
    std::shared_ptr<BsProgram> bs;   // bit-sliced specialization, if eligible
    ~ProgEntry();
    // The bit-sliced specialization, generated (not compiled) on first use;
    // nullptr when the matrix is too large to specialize.
    std::shared_ptr<BsProgram> bitslice();
    // The specialization if its kernel of this BsKind has been compiled, else
    // nullptr (never generates or compiles).
    std::shared_ptr<BsProgram> bitslice_if_compiled(int kind);
    int device_ptr(hipStream_t user, const uint32_t **out);
    // Same, but returns only once the copy has landed (for plans and graphs).
    int device_ptr_sync(const uint32_t **out);
};

constexpr int kVecBitslice = 32;   // variant code of the bit-sliced specialization
// Default variant: the bit-sliced kernel when the matrix's kernel has been
// compiled (by pm_prepare, the autotuner or an explicit bit-sliced call) and
// the block is at least one tile long, else the table kernel with kVecTable
// dwords per lane.
constexpr int kVecAuto = 0;
constexpr int kVecTable = 2;

struct Variant {
    int rg = 0;   // 0 = cost model
    int vec = 0;  // kVecAuto or an explicit variant code
    static int pick_rg(const Mat &A);
};

int check_regions(const void *base, size_t ld, size_t nblocks, size_t s);
// Whether two region sets (a_n blocks at a with stride a_ld, b_n at b) of s
// bytes per block share a byte range.
bool overlaps(const void *a, size_t a_ld, size_t a_n, const void *b, size_t b_ld, size_t b_n, size_t s);
int launch_program(ProgEntry &pe, int vec, const uint8_t *in, size_t in_ld, size_t in_n, uint8_t *out,
                   size_t out_ld, size_t out_n, size_t s, hipStream_t stream);

ProgEntry *apply_program(const Mat &A, int *vec);
void set_apply_variant(int rg, int vec);

enum OpKind { OPK_ENCODE = 0, OPK_HELPER = 1, OPK_NEWCOMER = 2, OPK_DECODE = 3 };

// Program and region counts of one operation of a code.  ids: d helper ids
// (newcomer) or k node ids (decode); failed: the failed node (repair).
struct Resolved {
    ProgEntry *pe = nullptr;
    size_t in_n = 0, out_n = 0;
    int vec = kVecAuto;
};
int resolve_op(pm_code *c, int op, uint32_t failed, const uint32_t *ids, Resolved *r);

}  // namespace pmrc
