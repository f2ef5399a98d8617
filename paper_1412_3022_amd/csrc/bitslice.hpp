// Bit-sliced region kernels specialized per matrix (see bitslice.cpp).
#pragma once
#include <hip/hip_runtime.h>

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

// Compile state of a BsProgram, readable without its mutex.
enum BsState { BS_NONE = 0, BS_READY = 2, BS_FAILED = 3 };

struct BsProgram {
    std::string source;
    int ngroups = 0;
    long est_ops = 0;   // straight-line VALU operations per 32-byte lane chunk
    std::mutex mu;
    bool compiled = false;
    int compile_status = 0;
    std::atomic<int> state{BS_NONE};
    std::vector<char> code;   // gfx950 code object
    std::map<int, BsModule> dev;
    ~BsProgram();
};

// Programs whose generated code would exceed this many operations are left
// to the table kernels (compile time and instruction-cache footprint).
constexpr long kBsMaxOps = 60000;
constexpr uint64_t kBsTileBytes = 2048;   // bytes per wave tile

// Generate the source for a program built with 8 rows per group.
std::unique_ptr<BsProgram> bs_generate(const Program &p8);
// Compile now (blocks for the hipRTC run; a no-op once compiled).  Nothing
// compiles in the background: no compile can be in flight at process exit.
int bs_compile(BsProgram &bp);
// Run the kernel over bytes [0, s) of every block, s >= kBsTileBytes (else
// ST_EINVAL).  Bases 16-byte aligned, ld multiples of 16 (as checked by the
// entry points).
int bs_launch(BsProgram &bp, const uint8_t *in, uint64_t in_ld, uint8_t *out, uint64_t out_ld, uint64_t s,
              hipStream_t st);

}  // namespace pmrc
