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
    size_t bytes = 0;
    hipEvent_t ready = nullptr;
    bool done = false;
    bool counted = true;   // included in device_table_bytes()
};

// Device bytes held by per-matrix table copies (all codes, devices and
// caches, evicted entries that still wait to be freed included; not the
// fixed GF(2^16) field table, which nothing can evict).
size_t device_table_bytes();
// Test hook: the next n table uploads fail with ST_ENOMEM before allocating.
void fail_next_uploads(uint32_t n);

// The copy of `bytes` host bytes on the current device in `dev` (guarded by
// mu), uploaded on first use there on an internal stream; `user` is made to
// wait for the upload until it is known to be complete.
// counted: whether the copy counts in device_table_bytes().
int device_copy(std::mutex &mu, std::map<int, DevCopy> &dev, const void *host, size_t bytes, hipStream_t user,
                const void **out, bool counted = true);
// Same, but returns only once the copy has landed (for plans, graphs and
// pm_prepare); no stream is made to wait.
int device_copy_sync(std::mutex &mu, std::map<int, DevCopy> &dev, const void *host, size_t bytes,
                     const void **out, bool counted = true);
void free_device_copies(std::map<int, DevCopy> &dev);

// A program plus its per-device copies.  device_ptr() uploads on first use
// on the current device (on an internal stream) and makes `user` wait for
// the upload until it is known to be complete.
struct ProgEntry {
    uint64_t tick = 0;          // last use, for the least-recently-used caches
    Program prog;
    Mat A;                      // the matrix (for specialized kernels)
    std::vector<int> in_map;
    std::mutex mu;
    std::map<int, DevCopy> dev;
    bool bs_tried = false;
    std::shared_ptr<BsProgram> bs;   // bit-sliced specialization, if eligible
    // matrix-core form (dense matrices too large to specialize), built on
    // first use, with its per-device copies
    bool mf_tried = false;
    bool mf_ok = false;
    std::vector<uint32_t> mf_words;
    uint32_t mf_nmtiles = 0, mf_nchunks = 0, mf_cols_off = 0, mf_rows_off = 0;
    std::map<int, DevCopy> mf_dev;
    // rows that are one input block times 1 (a decode's blocks that K's
    // systematic nodes hold) are not computed on the matrix cores: a table
    // kernel launch of copy groups writes them first (ngroups 0: none)
    Program mf_copy;
    std::map<int, DevCopy> mf_copy_dev;
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
    // The copy on the current device if it has already been made (`user`
    // then waits for its upload if that may still be in flight); allocates
    // and uploads nothing: ST_ENOTREADY when there is no copy yet.
    int device_ptr_resident(hipStream_t user, const uint32_t **out);
    // Bytes a device_ptr call would upload on the current device (0 when
    // the copy is there).
    size_t upload_bytes();
    // Whether the matrix is dense and too large for a specialized kernel:
    // then the matrix-core kernel runs instead of the table kernel.  Dense
    // counts the rows that are not copies: at least a third of their
    // coefficients nonzero.
    bool mfma_eligible();
    // Enqueue the matrix-core product (builds and uploads its operands on
    // first use; resident_only: ST_ENOTREADY unless they are on the device).
    int launch_mfma(const uint8_t *in, size_t in_ld, uint8_t *out, size_t out_ld, size_t s, hipStream_t stream,
                    bool resident_only = false);
    // Build and upload the matrix-core operands now (init phase; waits for
    // the upload).
    int stage_mfma();
    // Bytes stage_mfma would upload on the current device.
    size_t mfma_upload_bytes();
    void build_mfma_locked();
};

constexpr int kVecBitslice = 32;   // variant code of the bit-sliced specialization
// Default variant: the bit-sliced kernel when the matrix's kernel has been
// compiled (by pm_prepare, the autotuner or an explicit bit-sliced call) and
// the block is at least one tile long, else the table kernel with kVecTable
// dwords per lane.
constexpr int kVecAuto = 0;
constexpr int kVecTable = 2;
constexpr int kVecMfma = 40;      // variant code of the matrix-core kernel

struct Variant {
    int rg = 0;   // 0 = cost model
    int vec = 0;  // kVecAuto or an explicit variant code
    static int pick_rg(const Mat &A);
};

int check_regions(const void *base, size_t ld, size_t nblocks, size_t s);
// Whether two region sets (a_n blocks at a with stride a_ld, b_n at b) of s
// bytes per block share a byte range.
bool overlaps(const void *a, size_t a_ld, size_t a_n, const void *b, size_t b_ld, size_t b_n, size_t s);
// resident_only: use only kernels and tables already on the device (compile,
// load, allocate and upload nothing); ST_ENOTREADY otherwise.
int launch_program(ProgEntry &pe, int vec, const uint8_t *in, size_t in_ld, size_t in_n, uint8_t *out,
                   size_t out_ld, size_t out_n, size_t s, hipStream_t stream, bool resident_only = false);

std::shared_ptr<ProgEntry> apply_program(const Mat &A, int *vec);

// Evicted cache entries.  An entry leaves its cache at once but keeps its
// device memory (tables, loaded kernels) until no launch can still read it:
// retired entries are freed after a device-wide synchronization, and only
// when nothing else (a batch plan, a queued request, a call in progress)
// holds them.  That happens when retired entries hold more than a few MiB
// of device memory (not from a thread whose stream is being captured), in
// pm_cache_trim and at pm_code_destroy.
void retire(std::shared_ptr<ProgEntry> pe);
// Free what can be freed now.  sync: synchronize the device first (else
// only entries without device memory go).
void reap_retired(bool sync);
// Evict least recently used per-pattern entries of every live code (and of
// the pm_apply cache) and free them until the device bytes of tables are at
// most `target` or nothing more can go.  Synchronizes the device.
void trim_tables(size_t target);
void set_apply_variant(int rg, int vec);

enum OpKind { OPK_ENCODE = 0, OPK_HELPER = 1, OPK_NEWCOMER = 2, OPK_DECODE = 3 };

// Program and region counts of one operation of a code.  ids: d helper ids
// (newcomer) or k node ids (decode); failed: the failed node (repair).
struct Resolved {
    std::shared_ptr<ProgEntry> pe;
    size_t in_n = 0, out_n = 0;
    int vec = kVecAuto;
};
int resolve_op(pm_code *c, int op, uint32_t failed, const uint32_t *ids, Resolved *r);

}  // namespace pmrc
