// Launch interface of the batched GF(2^8) Gauss-Jordan kernel (gj.hip),
// shared by the kernel file and the host code.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct PmkGj {
    const uint8_t *src;     // candidate row idx of problem p: src + p*src_stride + idx*src_ld (B bytes)
    uint64_t src_ld, src_stride;
    const uint32_t *sets;   // per problem, nsets node ids (candidate rows node*alpha .. +alpha-1),
                            // or nullptr: candidate r is row r
    uint32_t nsets, alpha, nnodes;
    uint32_t nrows, B;      // candidates per problem, columns (= rank wanted)
    uint8_t *D;             // problem p: row i at D + p*d_stride + i*d_ld, B bytes
    uint64_t d_ld, d_stride;
    uint32_t *kept;         // problem p: B candidate indices at kept + p*B, or nullptr
    int32_t *status;        // problem p: 0, -1 (bad node id or repeated node), -3 (rank < B)
};

// Row width of the elimination state and LDS bytes of one problem with m
// candidate rows, B columns and nsets node ids (0 without sets).
extern "C" __host__ __device__ uint32_t pmk_gj_width(uint32_t B, uint32_t m);
extern "C" size_t pmk_gj_lds_bytes(uint32_t B, uint32_t m, uint32_t nsets);
// One work-group per problem, count problems.
extern "C" hipError_t pmk_gj(const PmkGj *h, uint32_t count, hipStream_t st);
