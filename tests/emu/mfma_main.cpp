// Host run of the matrix-core kernel (csrc/mfma.hip) with its own source,
// launched by its own launch plan.  Every GPU thread is an OS thread; the
// work-group's LDS is a buffer of the planned size and its barrier a
// barrier of the 256 threads; the wave-wide matrix instruction is a
// stand-in that exchanges the 64 lanes' operands through memory between two
// barriers of the wave and computes the product in the register layout the
// library assumes (lane l: row / column l % 32, K half l / 32, element 8q + t
// in nibble t of operand dword q; result register i of lane l: row
// 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32), with 4-bit floats decoded
// from their e2m1 encoding.  Input and output blocks sit right before an
// inaccessible page (and the run uses AddressSanitizer), so an access past
// a block end faults.
//
// EMU_NCU=n in the environment plans the launch for n compute units (256 by
// default; fewer give each wave several position blocks at small sizes).
// argv: in_file out_file.  in_file: R C nin s ld (uint64 each), then A (R x C
// bytes), in_map (C uint32), then nin x s input bytes.  out_file: R x s bytes.
#include <sys/mman.h>
#include <unistd.h>

#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#include "gf256.hpp"
#include "mfma.hpp"

struct EmuDim { unsigned x; };
static thread_local EmuDim threadIdx, blockIdx;
static EmuDim gridDim;
struct alignas(16) uint4 { uint32_t x, y, z, w; };
#define __device__
#define __global__
#define __launch_bounds__(x)
#define __forceinline__ inline
#define __shared__
static thread_local uint4 *pm_mf_lds;                 // the work-group's LDS
static thread_local std::barrier<> *t_wg;             // its barrier
#define __syncthreads() t_wg->arrive_and_wait()
#define __builtin_amdgcn_readfirstlane(x) ((int)(x))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
#define __builtin_amdgcn_sched_barrier(mask) ((void)(mask))   // a compiler scheduling fence
static inline uint32_t __float_as_uint(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static inline float __uint_as_float(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

// v_perm_b32 for byte selectors 0..7: bytes 0..3 from b, 4..7 from a
static inline uint32_t __builtin_amdgcn_perm(uint32_t a, uint32_t b, uint32_t sel) {
    const uint64_t v = (static_cast<uint64_t>(a) << 32) | b;
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) {
        const uint32_t s = (sel >> (8 * i)) & 0xFF;
        if (s > 7) { fprintf(stderr, "perm selector %u not emulated\n", s); abort(); }
        r |= static_cast<uint32_t>((v >> (8 * s)) & 0xFF) << (8 * i);
    }
    return r;
}

typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

// one wave's exchange area and barrier
struct Wave {
    std::barrier<> bar{64};
    uint32_t a[64][4], b[64][4];
};
static thread_local Wave *t_wave;
static thread_local unsigned t_lane;

static float e2m1(uint32_t nib) {
    const uint32_t s = nib >> 3, e = (nib >> 1) & 3, m = nib & 1;
    const float v = e == 0 ? 0.5f * m : std::ldexp(1.0f + 0.5f * m, static_cast<int>(e) - 1);
    return s ? -v : v;
}

static v16f __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(v8i A, v8i B, v16f C, int cbsz, int blgp, int, int sa,
                                                            int, int sb) {
    if (cbsz != 4 || blgp != 4 || sa != 127 || sb != 127) { fprintf(stderr, "mfma form not emulated\n"); abort(); }
    Wave &w = *t_wave;
    const unsigned l = t_lane;
    for (int q = 0; q < 4; ++q) { w.a[l][q] = static_cast<uint32_t>(A[q]); w.b[l][q] = static_cast<uint32_t>(B[q]); }
    w.bar.arrive_and_wait();
    v16f D = C;
    for (int i = 0; i < 16; ++i) {
        const unsigned m = 8 * (i / 4) + 4 * (l / 32) + i % 4, n = l % 32;
        float acc = 0.0f;
        for (unsigned kb = 0; kb < 2; ++kb)
            for (int q = 0; q < 4; ++q)
                for (int t = 0; t < 8; ++t)
                    acc += e2m1((w.a[m + 32 * kb][q] >> (4 * t)) & 15) * e2m1((w.b[n + 32 * kb][q] >> (4 * t)) & 15);
        D[i] += acc;
    }
    w.bar.arrive_and_wait();
    return D;
}

#include "mfma_kernel.inc"

// A region right before an inaccessible page.
static uint8_t *guarded(size_t bytes) {
    const size_t page = static_cast<size_t>(sysconf(_SC_PAGESIZE));
    const size_t span = (bytes + page - 1) / page * page + page;
    uint8_t *p = static_cast<uint8_t *>(mmap(nullptr, span, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0));
    if (p == MAP_FAILED) { perror("mmap"); exit(3); }
    mprotect(p + span - page, page, PROT_NONE);
    return p + span - page - bytes;
}

int main(int argc, char **argv) {
    if (argc != 3) return 1;
    FILE *f = fopen(argv[1], "rb");
    uint64_t hdr[5];
    if (!f || fread(hdr, 8, 5, f) != 5) return 2;
    const uint64_t R = hdr[0], C = hdr[1], nin = hdr[2], s = hdr[3], ld = hdr[4];
    pmrc::Mat A(static_cast<int>(R), static_cast<int>(C));
    std::vector<uint32_t> imap(C);
    if (fread(A.v.data(), 1, R * C, f) != R * C || fread(imap.data(), 4, C, f) != C) return 2;
    uint8_t *in = guarded((nin - 1) * ld + s);
    for (uint64_t r = 0; r < nin; ++r)
        if (fread(in + r * ld, 1, s, f) != s) return 2;
    fclose(f);
    uint8_t *out = guarded((R - 1) * ld + s);
    std::vector<int> in_map(imap.begin(), imap.end());
    // EMU_SUBSET: the program computes only the rows that are not one input
    // block times 1 (the library copies those with another kernel)
    std::vector<int> rows;
    if (getenv("EMU_SUBSET"))
        for (int r = 0; r < A.rows; ++r) {
            int nz = 0, last = -1;
            for (int c = 0; c < A.cols; ++c)
                if (A.at(r, c)) { ++nz; last = c; }
            if (!(nz == 1 && A.at(r, last) == 1)) rows.push_back(r);
        }
    pmrc::MfmaProgram P = pmrc::build_mfma_program(A, in_map, rows);
    const uint32_t *w = P.words.data();
    PmkMfma h{in, ld, out, ld, s, w, w + P.cols_off, w + P.rows_off, P.nmtiles, P.nchunks, 0, 0, 0, 0};
    uint32_t T = 0, nwg = 0;
    size_t lds = 0;
    const char *ncu = getenv("EMU_NCU");   // compute units of the planned device
    if (!mf_plan(h, ncu ? static_cast<uint32_t>(atoi(ncu)) : 256u, T, nwg, lds)) return 6;
    printf("T %u nwg %u pq %u lds %zu\n", T, nwg, h.pq, lds);
    gridDim.x = nwg;
    for (unsigned b = 0; b < nwg; ++b) {
        auto waves = std::make_unique<Wave[]>(kWaves);
        std::barrier<> wg(64 * kWaves);
        std::vector<uint4> mem(lds / sizeof(uint4));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < 64 * kWaves; ++t)
            th.emplace_back([&, b, t] {
                blockIdx.x = b;
                threadIdx.x = t;
                t_wave = &waves[t / 64];
                t_lane = t % 64;
                t_wg = &wg;
                pm_mf_lds = mem.data();
                if (T == 4) pm_mfma<4, 2>(h);
                else pm_mfma<2, 4>(h);
            });
        for (auto &x : th) x.join();
    }
    FILE *o = fopen(argv[2], "wb");
    for (uint64_t r = 0; r < R; ++r) fwrite(out + r * ld, 1, s, o);
    fclose(o);
    return 0;
}
