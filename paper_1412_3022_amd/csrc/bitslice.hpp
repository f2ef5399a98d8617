// Bit-sliced region kernels specialized per matrix (see bitslice.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace pmrc {

struct Program;

struct BsModule {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int P = 0;   // work-group slots per XCD
};

// Compile state of one kernel of a BsProgram, readable without its mutex.
enum BsState { BS_NONE = 0, BS_READY = 2, BS_FAILED = 3 };
// The two kernels generated for a matrix: one region set per launch (plain
// calls), or a device array of region sets (batches and the server).  They
// share the group code but are separate programs, compiled on demand: the
// register allocation of the single-set kernel must not depend on the other.
enum BsKind { BS_SINGLE = 0, BS_MULTI = 1 };

struct BsKernel {
    std::string source;
    bool compiled = false;
    int compile_status = 0;
    std::atomic<int> state{BS_NONE};
    std::vector<char> code;           // gfx950 code object
    std::map<int, BsModule> dev;      // per device
};

struct BsProgram {
    int ngroups = 0;
    long est_ops = 0;   // straight-line VALU operations per lane chunk
    uint32_t tile_bytes = 2048;   // bytes of a block per wave tile (4096 for GF(2^16))
    const char *fn_name[2] = {"pmbs", "pmbs_multi"};   // kernel names, by BsKind
    std::mutex mu;
    BsKernel k[2];      // by BsKind
    ~BsProgram();
};

// Programs whose generated code would exceed this many operations are left
// to the table kernels (compile time and instruction-cache footprint).  The
// k = 16 sparse encode (about 148 000) is inside; its hipRTC compile takes
// about 30 s.  Dense k = 16 decode matrices (about a million) are not.
constexpr long kBsMaxOps = 160000;
constexpr uint64_t kBsTileBytes = 2048;   // bytes per wave tile

// Generate the source for a program built with 8 rows per group.
std::unique_ptr<BsProgram> bs_generate(const Program &p8);
// Compile one kernel now (blocks for the hipRTC run; a no-op once compiled).
// Nothing compiles in the background: no compile can be in flight at exit.
int bs_compile(BsProgram &bp, BsKind kind);
inline bool bs_ready(const BsProgram &bp, BsKind kind) {
    return bp.k[kind].state.load(std::memory_order_acquire) == BS_READY;
}
// One region set of a multi-item launch (layout shared with the generated
// kernel's BsItem): tile0 = its first tile in the launch's numbering.
struct BsItem {
    const uint8_t *in;
    uint64_t ld;
    uint8_t *out;
    uint64_t old, s;
    uint32_t nfull, ntiles, tile0, pad;
};
static_assert(sizeof(BsItem) == 56, "BsItem layout");
// The item for bytes [0, s) of a region pair, s >= kBsTileBytes.
BsItem bs_item(const uint8_t *in, uint64_t in_ld, uint8_t *out, uint64_t out_ld, uint64_t s, uint32_t tile0);

// Compile (if needed) and load one kernel on the current device.
int bs_load(BsProgram &bp, BsKind kind);
// Run the kernel over bytes [0, s) of every block, s >= kBsTileBytes (else
// ST_EINVAL).  Bases 16-byte aligned, ld multiples of 16 (as checked by the
// entry points).  resident_only: compile and load nothing; ST_ENOTREADY
// unless the kernel is already loaded on the current device.
int bs_launch(BsProgram &bp, const uint8_t *in, uint64_t in_ld, uint8_t *out, uint64_t out_ld, uint64_t s,
              hipStream_t st, bool resident_only = false);
// One launch of the multi-set kernel over nitems items in device memory
// (d_items, sorted by tile0, tiles numbered back to back, ntiles in all,
// every item s >= kBsTileBytes), all for this program.
// slots: work-group slots per XCD (0 = the resident count, bs_default_slots).
int bs_launch_items(BsProgram &bp, const BsItem *d_items, uint32_t nitems, uint32_t ntiles, hipStream_t st,
                    uint32_t slots = 0);
// The resident work-group slots per XCD of the multi-set kernel on the
// current device (compiles and loads it if needed); 0 on failure.
uint32_t bs_default_slots(BsProgram &bp);

}  // namespace pmrc
