// Launch interface of the GF(2^16) region kernel (gf16.hip), shared by the
// kernel file and the host code.
//
// Program (uint32 words, device memory): word 0 = number of row groups;
// then per group 2 + kPm16Rows words: the offset of its first column
// record, its column count, and the output row of each of its kPm16Rows
// slots (kPm16NoRow for an unused slot).  A column record is 1 +
// kPm16Rows / 2 words: the input block, then the slots' 16-bit
// coefficients, two per word (slot 2i in the low half).  A copy group
// (rows that are one input block times 1) has kPm16CopyGroup for its column
// count and one record of kPm16Rows words: the input block of each slot.
//
// Tables (device memory): kPm16TableWords dwords per field element c, in
// element order.  A symbol's bits are cut into six pieces starting at bits
// e_p = 0, 3, 6, 8, 11, 14 (3, 3, 2, 3, 3, 2 bits).  For piece p and output
// byte h, the two dwords at 4p + 2h hold byte h of c * (v x^(e_p)) for
// v = 0..7 (zero for v >= 4 in the 2-bit pieces); dwords 24..31 are zero.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

constexpr uint32_t kPm16Rows = 8;
constexpr uint32_t kPm16Units = 4;                       // 8-byte units per lane
constexpr uint32_t kPm16TileBytes = kPm16Units * 512u;   // bytes of a block per wave tile
constexpr uint32_t kPm16Header = 1;
constexpr uint32_t kPm16TableWords = 32;
constexpr uint32_t kPm16NoRow = 0xFFFFFFFFu;
constexpr uint32_t kPm16CopyGroup = 0xFFFFFFFFu;

struct PmkApply16 {
    const uint8_t *in;    // input block c at in + c * in_ld
    uint64_t in_ld;
    uint8_t *out;         // output row r at out + r * out_ld
    uint64_t out_ld;
    uint64_t s;           // bytes per block (even)
    const uint32_t *prog;
    const uint32_t *tables;
    uint32_t ngroups, ntiles;   // ntiles = ceil(s / kPm16TileBytes)
};

extern "C" hipError_t pmk_apply16(const PmkApply16 *h, hipStream_t st);
