// C ABI of the engine (declared in include/pm.h): code objects, per-failure
// pattern matrix caches, device copies of the kernel tables, and dispatch of
// the region kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "construct.hpp"
#include "engine.hpp"
#include "gf16.hpp"
#include "gj.hpp"
#include "mfma.hpp"
#include "noalloc.hpp"
#include "put.hpp"
#include "pm.h"
#include "program.hpp"

using namespace pmrc;

namespace pmrc {

thread_local std::string g_hip_msg;

int hip_fail(hipError_t e) {
    g_hip_msg = hipGetErrorString(e);
    return ST_EHIP;
}

// ---- device copies of programs ---------------------------------------------
// Process-lifetime objects are heap allocated and never destroyed, so no HIP
// call runs from a static destructor after the runtime has shut down.
static std::mutex g_dev_mu;
static std::map<int, hipStream_t> &g_upload_stream = *new std::map<int, hipStream_t>();

static int upload_stream(int dev, hipStream_t *out) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_upload_stream.find(dev);
    if (it != g_upload_stream.end()) { *out = it->second; return ST_OK; }
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e);
    g_upload_stream[dev] = s;
    *out = s;
    return ST_OK;
}

ProgEntry::~ProgEntry() {
    free_device_copies(dev);
    free_device_copies(mf_dev);
    free_device_copies(mf_copy_dev);
}

// Rows that are one input block times 1: copies, not products.
static bool unit_row(const Mat &A, int r, int *nnz) {
    int nz = 0, last = -1;
    for (int c = 0; c < A.cols; ++c)
        if (A.at(r, c)) {
            ++nz;
            last = c;
        }
    *nnz = nz;
    return nz == 1 && A.at(r, last) == 1;
}

static std::atomic<size_t> g_table_bytes{0};
static std::atomic<uint32_t> g_fail_uploads{0};

size_t device_table_bytes() { return g_table_bytes.load(); }
void fail_next_uploads(uint32_t n) { g_fail_uploads.store(n); }

// Undo a partly made copy (the upload failed after the allocation).
static void drop_copy(DevCopy &dc) {
    if (dc.ready) (void)hipEventDestroy(dc.ready);
    if (dc.ptr) {
        (void)hipFree(dc.ptr);
        if (dc.counted) g_table_bytes -= dc.bytes;
    }
    dc = DevCopy{};
}

int device_copy(std::mutex &mu, std::map<int, DevCopy> &dev, const void *host, size_t bytes, hipStream_t user,
                const void **out, bool counted) {
    int devid = 0;
    hipError_t e = hipGetDevice(&devid);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lk(mu);
    DevCopy &dc = dev[devid];
    if (!dc.ptr) {
        for (uint32_t n = g_fail_uploads.load(); n > 0;)
            if (g_fail_uploads.compare_exchange_weak(n, n - 1)) return ST_ENOMEM;
        hipStream_t up = nullptr;
        int st = upload_stream(devid, &up);
        if (st != ST_OK) return st;
        if ((e = hipMalloc(&dc.ptr, bytes)) != hipSuccess) {
            dc.ptr = nullptr;
            return e == hipErrorOutOfMemory ? ST_ENOMEM : hip_fail(e);
        }
        dc.bytes = bytes;
        dc.counted = counted;
        if (counted) g_table_bytes += bytes;
        if ((e = hipMemcpyAsync(dc.ptr, host, bytes, hipMemcpyHostToDevice, up)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&dc.ready, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventRecord(dc.ready, up)) != hipSuccess) {
            // a failed copy must not be taken for a good one by the next call;
            // the upload stream is drained so the memory is not freed under it
            (void)hipStreamSynchronize(up);
            drop_copy(dc);
            return hip_fail(e);
        }
    }
    if (!dc.done) {
        e = hipEventQuery(dc.ready);
        if (e == hipSuccess) {
            dc.done = true;
        } else if (e == hipErrorNotReady) {
            if ((e = hipStreamWaitEvent(user, dc.ready, 0)) != hipSuccess) return hip_fail(e);
        } else {
            return hip_fail(e);
        }
    }
    *out = dc.ptr;
    return ST_OK;
}

void free_device_copies(std::map<int, DevCopy> &dev) {
    for (auto &kv : dev) drop_copy(kv.second);
    dev.clear();
}

int ProgEntry::device_ptr(hipStream_t user, const uint32_t **out) {
    const void *p = nullptr;
    int st = device_copy(mu, dev, prog.blob.data(), prog.blob.size() * sizeof(uint32_t), user, &p);
    if (st == ST_OK) *out = static_cast<const uint32_t *>(p);
    return st;
}

int device_copy_sync(std::mutex &mu, std::map<int, DevCopy> &dev, const void *host, size_t bytes,
                     const void **out, bool counted) {
    int st = device_copy(mu, dev, host, bytes, nullptr, out, counted);
    if (st != ST_OK) return st;
    int devid = 0;
    hipError_t e = hipGetDevice(&devid);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lk(mu);
    DevCopy &dc = dev[devid];
    if (!dc.done) {
        if ((e = hipEventSynchronize(dc.ready)) != hipSuccess) return hip_fail(e);
        dc.done = true;
    }
    return ST_OK;
}

size_t ProgEntry::upload_bytes() {
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    auto it = dev.find(devid);
    return it != dev.end() && it->second.ptr ? 0 : prog.blob.size() * sizeof(uint32_t);
}

int ProgEntry::device_ptr_resident(hipStream_t user, const uint32_t **out) {
    int devid = 0;
    hipError_t e = hipGetDevice(&devid);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> lk(mu);
    auto it = dev.find(devid);
    if (it == dev.end() || !it->second.ptr) return ST_ENOTREADY;
    DevCopy &dc = it->second;
    if (!dc.done) {
        e = hipEventQuery(dc.ready);
        if (e == hipSuccess) {
            dc.done = true;
        } else if (e == hipErrorNotReady) {
            if ((e = hipStreamWaitEvent(user, dc.ready, 0)) != hipSuccess) return hip_fail(e);
        } else {
            return hip_fail(e);
        }
    }
    *out = static_cast<const uint32_t *>(dc.ptr);
    return ST_OK;
}

int ProgEntry::device_ptr_sync(const uint32_t **out) {
    const void *p = nullptr;
    int st = device_copy_sync(mu, dev, prog.blob.data(), prog.blob.size() * sizeof(uint32_t), &p);
    if (st == ST_OK) *out = static_cast<const uint32_t *>(p);
    return st;
}

// A dense matrix beyond the specialization limit: at most 512 columns (the
// kernel's operands of one M tile in LDS), and rows other than copies
// spanning at least 64 x 64 cells, a third of them nonzero.
bool ProgEntry::mfma_eligible() {
    if (A.rows == 0 || A.cols == 0) return false;
    if (static_cast<uint32_t>(A.cols) > kMfMaxChunks * kMfColsPerChunk) return false;
    // the rows that are computed (copies aside): at least 64 x 64 cells and
    // a third of them nonzero.  (The table kernels' cost grows with the
    // nonzeros, the matrix cores' with the cells; on a decode of the
    // (16,30,32) code from 9 systematic and 7 parity nodes, 105 computed rows
    // 47 % nonzero, the table kernel took 329 us and the matrix cores 272 us
    // computing all 240 rows.)
    long nt = 0, nnz = 0;
    for (int r = 0; r < A.rows; ++r) {
        int nz = 0;
        if (unit_row(A, r, &nz)) continue;
        ++nt;
        nnz += nz;
    }
    const long cells = nt * A.cols;
    if (cells < 64 * 64 || nnz * 3 < cells) return false;
    std::shared_ptr<BsProgram> b = bitslice();
    return !b;
}

void ProgEntry::build_mfma_locked() {
    if (mf_tried) return;
    mf_tried = true;
    std::vector<int> rows;
    std::vector<char> computed(static_cast<size_t>(A.rows), 0);
    for (int r = 0; r < A.rows; ++r) {
        int nz = 0;
        if (!unit_row(A, r, &nz)) {
            rows.push_back(r);
            computed[static_cast<size_t>(r)] = 1;
        }
    }
    if (static_cast<int>(rows.size()) < A.rows) {
        mf_copy = build_program(A, prog.rg, in_map, &computed);   // the copy rows alone
    } else {
        rows.clear();   // every row on the matrix cores
    }
    MfmaProgram P = build_mfma_program(A, in_map, rows);
    mf_words = std::move(P.words);
    mf_nmtiles = P.nmtiles;
    mf_nchunks = P.nchunks;
    mf_cols_off = P.cols_off;
    mf_rows_off = P.rows_off;
    mf_ok = true;
}

size_t ProgEntry::mfma_upload_bytes() {
    int devid = 0;
    if (hipGetDevice(&devid) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    build_mfma_locked();
    size_t b = 0;
    auto it = mf_dev.find(devid);
    if (it == mf_dev.end() || !it->second.ptr) b += mf_words.size() * sizeof(uint32_t);
    auto ic = mf_copy_dev.find(devid);
    if (mf_copy.ngroups && (ic == mf_copy_dev.end() || !ic->second.ptr)) b += mf_copy.blob.size() * sizeof(uint32_t);
    return b;
}

int ProgEntry::stage_mfma() {
    {
        std::lock_guard<std::mutex> lk(mu);
        build_mfma_locked();
    }
    const void *d = nullptr;
    int st = device_copy_sync(mu, mf_dev, mf_words.data(), mf_words.size() * sizeof(uint32_t), &d);
    if (st == ST_OK && mf_copy.ngroups)
        st = device_copy_sync(mu, mf_copy_dev, mf_copy.blob.data(), mf_copy.blob.size() * sizeof(uint32_t), &d);
    return st;
}

int ProgEntry::launch_mfma(const uint8_t *in, size_t in_ld, uint8_t *out, size_t out_ld, size_t s,
                           hipStream_t stream, bool resident_only) {
    {
        std::lock_guard<std::mutex> lk(mu);
        if (!mf_tried && resident_only) return ST_ENOTREADY;
        build_mfma_locked();
    }
    if (!mf_ok) return ST_EINVAL;
    const void *d = nullptr, *dc = nullptr;
    int st;
    if (resident_only) {
        int devid = 0;
        hipError_t e = hipGetDevice(&devid);
        if (e != hipSuccess) return hip_fail(e);
        std::lock_guard<std::mutex> lk(mu);
        auto it = mf_dev.find(devid);
        if (it == mf_dev.end() || !it->second.ptr || !it->second.done) return ST_ENOTREADY;
        d = it->second.ptr;
        if (mf_copy.ngroups) {
            auto ic = mf_copy_dev.find(devid);
            if (ic == mf_copy_dev.end() || !ic->second.ptr || !ic->second.done) return ST_ENOTREADY;
            dc = ic->second.ptr;
        }
    } else if ((st = device_copy(mu, mf_dev, mf_words.data(), mf_words.size() * sizeof(uint32_t), stream, &d)) !=
                   ST_OK ||
               (mf_copy.ngroups && (st = device_copy(mu, mf_copy_dev, mf_copy.blob.data(),
                                                     mf_copy.blob.size() * sizeof(uint32_t), stream, &dc)) != ST_OK)) {
        return st;
    }
    if (mf_copy.ngroups) {   // the copy rows, on the table kernel's copy groups
        PmkApply a{in, in_ld, out, out_ld, s, static_cast<const uint32_t *>(dc), static_cast<uint32_t>(mf_copy.ngroups)};
        hipError_t e = pmk_apply(mf_copy.rg, kVecTable, &a, stream);
        if (e != hipSuccess) return hip_fail(e);
    }
    const uint32_t *w = static_cast<const uint32_t *>(d);
    PmkMfma h{in, in_ld, out, out_ld, s, w, w + mf_cols_off, w + mf_rows_off, mf_nmtiles, mf_nchunks, 0, 0, 0, 0};
    hipError_t e = pmk_mfma(&h, stream);
    return e == hipSuccess ? ST_OK : hip_fail(e);
}

std::shared_ptr<BsProgram> ProgEntry::bitslice() {
    std::lock_guard<std::mutex> lk(mu);
    if (!bs_tried) {
        bs_tried = true;
        // One group for a matrix of at most 16 x 16: every column is then
        // transposed once (the k = 4 encode and decode run 13-18 % faster);
        // with more columns the 16-row groups' register use (2 waves per
        // SIMD) costs more than the transposes they save.
        const int rg = A.rows <= 16 && A.cols <= 16 ? 16 : 8;
        Program p8 = build_program(A, rg, in_map);
        std::unique_ptr<BsProgram> b = bs_generate(p8);
        if (b->est_ops <= kBsMaxOps) bs = std::move(b);
    }
    return bs;
}

std::shared_ptr<BsProgram> ProgEntry::bitslice_if_compiled(int kind) {
    std::lock_guard<std::mutex> lk(mu);
    if (bs && bs_ready(*bs, static_cast<BsKind>(kind))) return bs;
    return nullptr;
}

// ---- variant choice ----------------------------------------------------------
// VALU cost per lane dword of a program: each evaluated slot costs three
// byte-permutes and 1.5 three-input XORs plus its share of table moves; each
// group column costs its source-field extraction and a load.
static double program_cost(const Program &p) {
    return static_cast<double>(p.slots) * 4.8 + static_cast<double>(p.col_reads) * 7.0 +
           static_cast<double>(p.copies) * 2.0;
}

int Variant::pick_rg(const Mat &A) {
    double best = 1e300;
    int best_rg = 8;
    for (int rg : {4, 8, 16}) {
        Program p = build_program(A, rg);
        double c = program_cost(p);
        if (c < best - 1e-9) { best = c; best_rg = rg; }
    }
    return best_rg;
}

// ---- launching -----------------------------------------------------------------
static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_regions(const void *base, size_t ld, size_t nblocks, size_t s) {
    if (nblocks == 0) return ST_OK;
    if (!base || !aligned16(base) || ld % 16 != 0 || ld < s) return ST_EINVAL;
    return ST_OK;
}

bool overlaps(const void *a, size_t a_ld, size_t a_n, const void *b, size_t b_ld, size_t b_n,
                     size_t s) {
    if (!a_n || !b_n) return false;
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), a1 = a0 + (a_n - 1) * a_ld + s;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(b), b1 = b0 + (b_n - 1) * b_ld + s;
    return a0 < b1 && b0 < a1;
}

int launch_program(ProgEntry &pe, int vec, const uint8_t *in, size_t in_ld, size_t in_n, uint8_t *out,
                   size_t out_ld, size_t out_n, size_t s, hipStream_t stream, bool resident_only) {
    if (s == 0) return ST_EINVAL;
    int st;
    if ((st = check_regions(in, in_ld, in_n, s)) != ST_OK) return st;
    if ((st = check_regions(out, out_ld, out_n, s)) != ST_OK) return st;
    if (overlaps(in, in_ld, in_n, out, out_ld, out_n, s)) return ST_EINVAL;
    if (pe.prog.ngroups == 0) return ST_OK;
    // the matrix cores take up to 512 columns and address the input within
    // 4 GiB of its first block; past that the table kernel gives the same
    // bytes
    const bool mf_span =
        static_cast<uint32_t>(pe.A.cols) <= kMfMaxChunks * kMfColsPerChunk && mf_span_ok(in_ld, s, in_n);
    if (vec == kVecMfma) {
        if (mf_span) return pe.launch_mfma(in, in_ld, out, out_ld, s, stream, resident_only);
        vec = 4;
    } else if (vec == kVecBitslice && !resident_only) {
        // blocks shorter than one tile, and matrices too large for a
        // specialized kernel, run on the table kernel
        if (s >= kBsTileBytes)
            if (std::shared_ptr<BsProgram> bp = pe.bitslice()) return bs_launch(*bp, in, in_ld, out, out_ld, s, stream);
        vec = 4;
    } else if (vec == kVecAuto || vec == kVecBitslice) {
        if (s >= kBsTileBytes)
            if (std::shared_ptr<BsProgram> bp = pe.bitslice_if_compiled(BS_SINGLE)) {
                st = bs_launch(*bp, in, in_ld, out, out_ld, s, stream, resident_only);
                // compiled but not loaded on this device: the table kernel
                // may still be resident
                if (st != ST_ENOTREADY) return st;
            }
        // dense matrices over the specialization limit: the matrix cores
        if (vec == kVecAuto && mf_span && pe.mfma_eligible()) {
            st = pe.launch_mfma(in, in_ld, out, out_ld, s, stream, resident_only);
            if (st != ST_ENOTREADY) return st;
        }
        vec = vec == kVecBitslice ? 4 : kVecTable;
    }
    const uint32_t *dprog = nullptr;
    if ((st = resident_only ? pe.device_ptr_resident(stream, &dprog) : pe.device_ptr(stream, &dprog)) != ST_OK)
        return st;
    PmkApply a{in, in_ld, out, out_ld, s, dprog, static_cast<uint32_t>(pe.prog.ngroups)};
    hipError_t e = pmk_apply(pe.prog.rg, vec, &a, stream);
    if (e != hipSuccess) return hip_fail(e);
    return ST_OK;
}

// ---- retired cache entries ---------------------------------------------------------
static std::mutex g_grave_mu;
static std::vector<std::shared_ptr<ProgEntry>> &g_grave = *new std::vector<std::shared_ptr<ProgEntry>>();
constexpr size_t kGraveBytes = size_t(64) << 20;   // device bytes of retired entries before a reap
constexpr size_t kGraveEntries = 256;

static size_t entry_device_bytes(ProgEntry &pe) {
    std::lock_guard<std::mutex> lk(pe.mu);
    size_t b = 0;
    for (auto &kv : pe.dev) b += kv.second.bytes;
    for (auto &kv : pe.mf_dev) b += kv.second.bytes;
    for (auto &kv : pe.mf_copy_dev) b += kv.second.bytes;
    if (pe.bs) b += 1;   // a loaded kernel module: device memory of unknown size
    return b;
}

void reap_retired(bool sync) {
    std::vector<std::shared_ptr<ProgEntry>> go;
    {
        std::lock_guard<std::mutex> lk(g_grave_mu);
        // entries nobody else holds can no longer be launched again; those
        // with device memory still wait for the launches already enqueued
        for (auto it = g_grave.begin(); it != g_grave.end();) {
            if (it->use_count() == 1 && (sync || entry_device_bytes(**it) == 0)) {
                go.push_back(std::move(*it));
                it = g_grave.erase(it);
            } else {
                ++it;
            }
        }
    }
    if (go.empty()) return;
    if (sync) {
        int n = 0;
        if (hipGetDeviceCount(&n) == hipSuccess && n > 0) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            // another thread's stream capture must not forbid this wait
            hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
            (void)hipThreadExchangeStreamCaptureMode(&mode);
            for (int d = 0; d < n; ++d)
                if (hipSetDevice(d) == hipSuccess) (void)hipDeviceSynchronize();
            (void)hipSetDevice(cur);
            (void)hipThreadExchangeStreamCaptureMode(&mode);
        } else {
            (void)hipGetLastError();
        }
    }
    go.clear();   // frees device copies and unloads kernels
}

void retire(std::shared_ptr<ProgEntry> pe) {
    if (!pe) return;
    size_t bytes = 0, entries = 0;
    {
        std::lock_guard<std::mutex> lk(g_grave_mu);
        g_grave.push_back(std::move(pe));
        for (auto &e : g_grave) bytes += entry_device_bytes(*e);
        entries = g_grave.size();
    }
    if (bytes == 0 || entries > kGraveEntries) reap_retired(false);
    if (bytes > kGraveBytes || entries > kGraveEntries) reap_retired(true);
}

// Drop the least recently used entries of a cache once it holds more than
// cap: a quarter of cap at a time, entries for which busy() holds kept.
// Each dropped value goes to drop().
template <class Map, class Tick, class Busy, class Drop>
void lru_trim(Map &m, size_t cap, Tick tick, Busy busy, Drop drop) {
    if (m.size() <= cap) return;
    std::vector<std::pair<uint64_t, typename Map::iterator>> order;
    for (auto it = m.begin(); it != m.end(); ++it)
        if (!busy(it->second)) order.emplace_back(tick(it->second), it);
    std::sort(order.begin(), order.end(),
              [](const auto &a, const auto &b) { return a.first < b.first; });
    const size_t target = cap - cap / 4;
    for (auto &o : order) {
        if (m.size() <= target) break;
        drop(o.second->second);
        m.erase(o.second);
    }
}

// ---- pm_apply: programs cached by matrix content ----------------------------------
constexpr size_t kApplyCap = 256;
static std::mutex g_apply_mu;
static uint64_t g_apply_tick = 0;
static std::map<std::tuple<int, int, std::vector<uint8_t>, int>, std::shared_ptr<ProgEntry>> &g_apply =
    *new std::map<std::tuple<int, int, std::vector<uint8_t>, int>, std::shared_ptr<ProgEntry>>();
static Variant g_apply_var;

void set_apply_variant(int rg, int vec) {
    std::lock_guard<std::mutex> lk(g_apply_mu);
    g_apply_var.rg = rg;
    g_apply_var.vec = vec;
}

std::shared_ptr<ProgEntry> apply_program(const Mat &A, int *vec) {
    std::vector<std::shared_ptr<ProgEntry>> evicted;
    std::shared_ptr<ProgEntry> out;
    {
        std::lock_guard<std::mutex> lk(g_apply_mu);
        const int rg = g_apply_var.rg ? g_apply_var.rg : Variant::pick_rg(A);
        *vec = g_apply_var.vec;
        auto key = std::make_tuple(A.rows, A.cols, A.v, rg);
        auto it = g_apply.find(key);
        if (it == g_apply.end()) {
            auto pe = std::make_shared<ProgEntry>();
            pe->prog = build_program(A, rg);
            pe->A = A;
            it = g_apply.emplace(std::move(key), std::move(pe)).first;
        }
        it->second->tick = ++g_apply_tick;
        out = it->second;
        lru_trim(
            g_apply, kApplyCap, [](const std::shared_ptr<ProgEntry> &p) { return p->tick; },
            [&](const std::shared_ptr<ProgEntry> &p) { return p == out; },
            [&](std::shared_ptr<ProgEntry> &p) { evicted.push_back(std::move(p)); });
    }
    for (auto &p : evicted) retire(std::move(p));
    return out;
}

}  // namespace pmrc

// ---- the code object -------------------------------------------------------------
// Per-failure-pattern caches hold at most this many entries each (helper,
// newcomer and decode patterns, specific-decode node lists) unless
// pm_code_set_cache_limit says otherwise; beyond it the least recently used
// are evicted (and their device memory retired).
constexpr size_t kPatternCap = 256;

template <class V>
struct Aged {
    V v;
    uint64_t tick = 0;
};

struct pm_code {
    CodeMats m;
    // GF(2^16) codes keep everything here (m holds only k, d, n, alpha, B)
    std::unique_ptr<w16::Ctx16> w16;
    std::mutex mu;
    Variant var[4];
    uint64_t tick = 0;            // use counter of the caches below
    size_t cap = kPatternCap;     // entries per per-pattern cache
    std::map<std::tuple<int>, std::shared_ptr<ProgEntry>> enc;                      // rg
    std::map<std::pair<int, int>, std::shared_ptr<ProgEntry>> helper;              // failed, rg
    std::map<std::tuple<int, std::vector<int>, int>, std::shared_ptr<ProgEntry>> newcomer;
    std::map<std::pair<std::vector<int>, int>, std::shared_ptr<ProgEntry>> decode;  // nodes, rg
    std::map<int, Aged<Mat>> helper_mat;
    std::map<std::pair<int, std::vector<int>>, Aged<Mat>> newcomer_mat;
    std::map<std::vector<int>, Aged<std::pair<Mat, std::vector<int>>>> decode_mat;
    // specific PM-MSR decode per node list: its factors and their programs
    struct Specific {
        Mat F[kSpecificPasses];
        std::map<int, std::shared_ptr<ProgEntry>> progs[kSpecificPasses];   // by rg
        uint64_t tick = 0;
    };
    std::map<std::vector<int>, Specific> specific;
    // device copies of the generator the node contents follow (Gsys), for
    // the batched decode-matrix init
    std::mutex dev_mu;
    std::map<int, DevCopy> gsys_dev;
    ~pm_code() { free_device_copies(gsys_dev); }
};

namespace {

// Find or build the program for matrix A (key ends with the row-group size),
// marked used now; evicts the map's least recently used entries beyond the
// code's cap into `evicted`.  Caller holds code->mu.
template <class Map, class Key>
std::shared_ptr<ProgEntry> get_prog(pm_code *c, Map &map, const Key &key_prefix_rg, const Mat &A,
                                    const std::vector<int> &in_map,
                                    std::vector<std::shared_ptr<ProgEntry>> &evicted) {
    auto it = map.find(key_prefix_rg);
    if (it == map.end()) {
        auto pe = std::make_shared<ProgEntry>();
        int rg = std::get<std::tuple_size<Key>::value - 1>(key_prefix_rg);
        pe->prog = build_program(A, rg, in_map);
        pe->A = A;
        pe->in_map = in_map;
        it = map.emplace(key_prefix_rg, std::move(pe)).first;
    }
    it->second->tick = ++c->tick;
    std::shared_ptr<ProgEntry> out = it->second;
    lru_trim(
        map, c->cap, [](const std::shared_ptr<ProgEntry> &p) { return p->tick; },
        // held by a batch plan, a queued request or a call in progress
        [](const std::shared_ptr<ProgEntry> &p) { return p.use_count() > 1; },
        [&](std::shared_ptr<ProgEntry> &p) { evicted.push_back(std::move(p)); });
    return out;
}

// Find or build a per-pattern matrix, marked used now; trims the map.
template <class Map, class Key, class Build>
int get_mat(pm_code *c, Map &map, const Key &key, Build build, typename Map::mapped_type **out) {
    auto it = map.find(key);
    if (it == map.end()) {
        typename Map::mapped_type a;
        int st = build(a.v);
        if (st != ST_OK) return st;
        it = map.emplace(key, std::move(a)).first;
    }
    it->second.tick = ++c->tick;
    lru_trim(
        map, c->cap, [](const typename Map::mapped_type &a) { return a.tick; },
        [&](const typename Map::mapped_type &a) { return &a == &it->second; }, [](typename Map::mapped_type &) {});
    *out = &it->second;
    return ST_OK;
}

int resolve_rg(Variant &v, const Mat &A, std::map<std::vector<uint8_t>, int> *memo = nullptr) {
    if (v.rg) return v.rg;
    if (memo) {
        auto it = memo->find(A.v);
        if (it != memo->end()) return it->second;
    }
    int rg = Variant::pick_rg(A);
    if (memo) {
        if (memo->size() >= 4096) memo->clear();   // a cost-model memo: cheap to rebuild
        (*memo)[A.v] = rg;
    }
    return rg;
}

std::map<std::vector<uint8_t>, int> &rg_memo() {
    static std::map<std::vector<uint8_t>, int> m;
    return m;
}
std::mutex g_memo_mu;

int pick_rg_cached(Variant &v, const Mat &A) {
    if (v.rg) return v.rg;
    std::lock_guard<std::mutex> lk(g_memo_mu);
    return resolve_rg(v, A, &rg_memo());
}

}  // namespace

namespace pmrc {

// Matrix, program and region counts of one operation of a code; builds and
// caches the per-failure-pattern matrices (the initialization phase).
int resolve_op(pm_code *c, int op, uint32_t failed, const uint32_t *ids, Resolved *r) {
    if (!c) return ST_EINVAL;
    if (c->w16) return ST_EUNSUPPORTED;   // batches and the server take GF(2^8) codes
    const CodeMats &m = c->m;
    if ((op == OPK_HELPER || op == OPK_NEWCOMER) && failed >= static_cast<uint32_t>(m.n)) return ST_EINVAL;
    std::vector<int> list;
    if (op == OPK_NEWCOMER || op == OPK_DECODE) {
        if (!ids) return ST_EINVAL;
        const int cnt = op == OPK_NEWCOMER ? m.d : m.k;
        list.assign(ids, ids + cnt);
        std::vector<int> sorted = list;
        std::sort(sorted.begin(), sorted.end());
        if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return ST_EINVAL;
        for (int v : list)
            if (v < 0 || v >= m.n || (op == OPK_NEWCOMER && v == static_cast<int>(failed))) return ST_EINVAL;
    }
    std::vector<std::shared_ptr<ProgEntry>> evicted;
    int st = ST_OK;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        const Variant &var = c->var[op];
        r->vec = var.vec;
        switch (op) {
            case OPK_ENCODE: {
                const int rg = pick_rg_cached(c->var[0], m.enc);
                r->pe = get_prog(c, c->enc, std::make_tuple(rg), m.enc, {}, evicted);
                r->in_n = static_cast<size_t>(m.B);
                r->out_n = static_cast<size_t>(m.enc.rows);
                break;
            }
            case OPK_HELPER: {
                Aged<Mat> *hm = nullptr;
                st = get_mat(c, c->helper_mat, static_cast<int>(failed),
                             [&](Mat &out) { out = helper_row(m, static_cast<int>(failed)); return ST_OK; }, &hm);
                if (st != ST_OK) break;
                const int rg = var.rg ? var.rg : 4;
                r->pe = get_prog(c, c->helper, std::make_pair(static_cast<int>(failed), rg), hm->v, {}, evicted);
                r->in_n = static_cast<size_t>(m.kind == KIND_RS ? 1 : m.alpha);
                r->out_n = 1;
                break;
            }
            case OPK_NEWCOMER: {
                Aged<Mat> *nm = nullptr;
                st = get_mat(c, c->newcomer_mat, std::make_pair(static_cast<int>(failed), list),
                             [&](Mat &out) { return newcomer_matrix(m, static_cast<int>(failed), list, out); }, &nm);
                if (st != ST_OK) break;
                const int rg = pick_rg_cached(c->var[2], nm->v);
                r->pe = get_prog(c, c->newcomer, std::make_tuple(static_cast<int>(failed), list, rg), nm->v, {},
                                 evicted);
                r->in_n = static_cast<size_t>(m.d);
                r->out_n = static_cast<size_t>(nm->v.rows);
                break;
            }
            case OPK_DECODE: {
                Aged<std::pair<Mat, std::vector<int>>> *dm = nullptr;
                st = get_mat(c, c->decode_mat, list,
                             [&](std::pair<Mat, std::vector<int>> &out) {
                                 return decode_matrix(m, list, out.first, out.second);
                             },
                             &dm);
                if (st != ST_OK) break;
                const int rg = pick_rg_cached(c->var[3], dm->v.first);
                r->pe = get_prog(c, c->decode, std::make_pair(list, rg), dm->v.first, dm->v.second, evicted);
                r->in_n = static_cast<size_t>(m.k) * static_cast<size_t>(m.alpha);
                r->out_n = static_cast<size_t>(m.B);
                break;
            }
            default:
                st = ST_EINVAL;
        }
    }
    for (auto &p : evicted) retire(std::move(p));
    return st;
}

}  // namespace pmrc

namespace {

// The specific decode of node list ids: factors (built once) and the
// program of each pass.  The passes are the leading factors with rows: all
// five for systematic PM-MSR, four without the re-encoding, two for PM-MBR.
struct SpecificOps {
    std::shared_ptr<ProgEntry> pe[kSpecificPasses];
    int npass = 0;
    int rows[kSpecificPasses] = {};
};

// lookup_only: build nothing (no factors, no programs); ST_ENOTREADY when the
// node list has not been resolved before.
int resolve_specific(pm_code *c, const uint32_t *ids, SpecificOps *out, bool lookup_only = false) {
    if (!c || !ids) return ST_EINVAL;
    if (c->w16) return ST_EUNSUPPORTED;
    const CodeMats &m = c->m;
    if (m.kind != KIND_MSR && m.kind != KIND_MBR) return ST_EUNSUPPORTED;
    std::vector<int> list(ids, ids + m.k), sorted;
    sorted = list;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return ST_EINVAL;
    for (int v : list)
        if (v < 0 || v >= m.n) return ST_EINVAL;
    std::vector<std::shared_ptr<ProgEntry>> evicted;
    int st = ST_OK;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->specific.find(list);
        if (it == c->specific.end()) {
            if (lookup_only) return ST_ENOTREADY;
            pm_code::Specific sp;
            st = specific_decode_factors(m, list, sp.F);
            if (st != ST_OK) return st;
            it = c->specific.emplace(list, std::move(sp)).first;
        }
        pm_code::Specific &sp = it->second;
        sp.tick = ++c->tick;
        out->npass = 0;
        while (out->npass < kSpecificPasses && sp.F[out->npass].rows) ++out->npass;
        for (int p = 0; p < out->npass && st == ST_OK; ++p) {
            const Mat &F = sp.F[p];
            const int rg = pick_rg_cached(c->var[3], F);
            auto &map = sp.progs[p];
            auto pit = map.find(rg);
            if (pit == map.end()) {
                if (lookup_only) {
                    st = ST_ENOTREADY;
                    break;
                }
                auto pe = std::make_shared<ProgEntry>();
                pe->prog = build_program(F, rg);
                pe->A = F;
                pit = map.emplace(rg, std::move(pe)).first;
            }
            out->pe[p] = pit->second;
            out->rows[p] = F.rows;
        }
        const pm_code::Specific *cur = &it->second;
        lru_trim(
            c->specific, c->cap, [](const pm_code::Specific &x) { return x.tick; },
            [&](const pm_code::Specific &x) {
                if (&x == cur) return true;
                for (auto &mp : x.progs)
                    for (auto &kv : mp)
                        if (kv.second.use_count() > 1) return true;
                return false;
            },
            [&](pm_code::Specific &x) {
                for (auto &mp : x.progs)
                    for (auto &kv : mp) evicted.push_back(std::move(kv.second));
            });
    }
    for (auto &p : evicted) retire(std::move(p));
    return st;
}

// Live GF(2^8) codes, for trims of the table caches across codes.
std::mutex g_codes_mu;
std::set<pm_code *> &g_codes = *new std::set<pm_code *>();

void register_code(pm_code *c) {
    std::lock_guard<std::mutex> lk(g_codes_mu);
    g_codes.insert(c);
}

void unregister_code(pm_code *c) {
    std::lock_guard<std::mutex> lk(g_codes_mu);
    g_codes.erase(c);
}

// Evict the least recently used per-pattern entries of a code beyond `keep`
// per cache (entries in use stay).  Caller holds c->mu.
void trim_code_locked(pm_code *c, size_t keep, std::vector<std::shared_ptr<ProgEntry>> &evicted) {
    auto tick = [](const std::shared_ptr<ProgEntry> &p) { return p->tick; };
    auto busy = [](const std::shared_ptr<ProgEntry> &p) { return p.use_count() > 1; };
    auto drop = [&](std::shared_ptr<ProgEntry> &p) { evicted.push_back(std::move(p)); };
    lru_trim(c->helper, keep, tick, busy, drop);
    lru_trim(c->newcomer, keep, tick, busy, drop);
    lru_trim(c->decode, keep, tick, busy, drop);
    auto none = [](auto &) {};
    auto mtick = [](const auto &a) { return a.tick; };
    auto mbusy = [](const auto &) { return false; };
    lru_trim(c->helper_mat, keep, mtick, mbusy, none);
    lru_trim(c->newcomer_mat, keep, mtick, mbusy, none);
    lru_trim(c->decode_mat, keep, mtick, mbusy, none);
    lru_trim(
        c->specific, keep, [](const pm_code::Specific &x) { return x.tick; },
        [](const pm_code::Specific &x) {
            for (auto &mp : x.progs)
                for (auto &kv : mp)
                    if (kv.second.use_count() > 1) return true;
            return false;
        },
        [&](pm_code::Specific &x) {
            for (auto &mp : x.progs)
                for (auto &kv : mp) evicted.push_back(std::move(kv.second));
        });
}

}  // namespace

namespace pmrc {

void trim_tables(size_t target) {
    for (int round = 0; round < 6 && device_table_bytes() > target; ++round) {
        std::vector<std::shared_ptr<ProgEntry>> evicted;
        {
            std::lock_guard<std::mutex> lk(g_codes_mu);
            for (pm_code *c : g_codes) {
                std::lock_guard<std::mutex> lc(c->mu);
                // halve every per-pattern cache, oldest entries first
                size_t most = std::max({c->helper.size(), c->newcomer.size(), c->decode.size(),
                                        c->specific.size()});
                trim_code_locked(c, most / 2, evicted);
            }
        }
        for (auto &p : evicted) retire(std::move(p));
        reap_retired(true);
        {
            std::lock_guard<std::mutex> lk(g_apply_mu);
            if (round >= 2) {   // the pm_apply cache last
                std::vector<std::shared_ptr<ProgEntry>> ev2;
                lru_trim(
                    g_apply, g_apply.size() / 2, [](const std::shared_ptr<ProgEntry> &p) { return p->tick; },
                    [](const std::shared_ptr<ProgEntry> &p) { return p.use_count() > 1; },
                    [&](std::shared_ptr<ProgEntry> &p) { ev2.push_back(std::move(p)); });
                evicted.swap(ev2);
            }
        }
        for (auto &p : evicted) retire(std::move(p));
    }
    reap_retired(true);
}

}  // namespace pmrc

namespace {

// Workspace of pm_repair: the d helper blocks (what the helpers send), then
// the launch list of the projections (d multi-set items), 16-byte aligned.
size_t repair_ws_bytes(const CodeMats &m, size_t s) {
    const size_t d = static_cast<size_t>(m.kind == KIND_RS ? m.k : m.d);
    const size_t ld = (s + 15) / 16 * 16;
    return d * ld + (d * sizeof(BsItem) + 15) / 16 * 16;
}

// Workspace blocks of a specific decode: the outputs of every pass but the
// last, back to back.  PM-MSR: Z: k(k-1), pairs: B, phi_i^t S: 2 alpha^2,
// and for systematic codes the B message symbols.  PM-MBR: T and the copied
// node blocks, at most k d.
size_t specific_ws_blocks(const CodeMats &m) {
    if (m.kind == KIND_MBR) return static_cast<size_t>(m.k) * m.d;
    return static_cast<size_t>(m.k) * (m.k - 1) + static_cast<size_t>(m.B) +
           2u * static_cast<size_t>(m.alpha) * m.alpha + (m.systematic ? m.B : 0);
}

}  // namespace

extern "C" {

const char *pm_status_string(pm_status st) {
    switch (st) {
        case PM_OK: return "ok";
        case PM_EINVAL: return "invalid argument";
        case PM_EUNSUPPORTED: return "unsupported parameters";
        case PM_ESINGULAR: return "singular matrix (node set cannot repair or decode)";
        case PM_ENOMEM: return "out of memory";
        case PM_EHIP: return "HIP runtime error";
        case PM_EBUSY: return "busy";
        case PM_ENOTREADY: return "not prepared on this device (call pm_prepare first)";
        case PM_ELIMIT: return "exceeds the fixed scratch of the no-allocation entry point";
    }
    return "unknown status";
}

const char *pm_last_hip_error(void) { return g_hip_msg.c_str(); }

pm_status pm_code_create(const pm_params *p, pm_code **out) {
    if (!p || !out) return PM_EINVAL;
    *out = nullptr;
    if (p->w != 8 && p->w != 16) return PM_EUNSUPPORTED;
    if (p->kind < 0 || p->kind > 2) return PM_EINVAL;
    CodeSpec spec;
    spec.kind = p->kind;
    spec.construction = p->construction;
    spec.systematic = (p->kind == PM_MSR) ? (p->systematic ? 1 : 0) : 1;
    spec.k = static_cast<int>(p->k);
    spec.d = static_cast<int>(p->d);
    spec.n = static_cast<int>(p->n);
    if (p->kind == PM_MSR && p->construction != PM_VANILLA && p->construction != PM_SPARSE) return PM_EINVAL;
    if (p->x) {
        if (p->kind != PM_MSR || p->construction != PM_VANILLA || p->n > 255) return PM_EINVAL;
        spec.x.assign(p->x, p->x + p->n);
    }
    try {
        std::unique_ptr<pm_code> c(new pm_code());
        if (p->w == 16) {
            c->w16 = std::make_unique<w16::Ctx16>();
            int st = w16::build_code(spec, c->w16->m);
            if (st != ST_OK) return static_cast<pm_status>(st);
            const w16::Code16 &m = c->w16->m;
            c->m.kind = KIND_MSR;
            c->m.construction = CONS_SPARSE;
            c->m.systematic = m.systematic;
            c->m.k = m.k; c->m.d = m.d; c->m.n = m.n; c->m.alpha = m.alpha; c->m.B = m.B;
            *out = c.release();
            return PM_OK;
        }
        int st = build_code(spec, c->m);
        if (st != ST_OK) return static_cast<pm_status>(st);
        register_code(c.get());
        *out = c.release();
        return PM_OK;
    } catch (const std::bad_alloc &) {
        return PM_ENOMEM;
    }
}

void pm_code_destroy(pm_code *code) {
    if (!code) return;
    unregister_code(code);
    delete code;
    reap_retired(false);
}

pm_status pm_code_set_cache_limit(pm_code *c, uint32_t entries) {
    if (!c || entries == 0) return PM_EINVAL;
    std::vector<std::shared_ptr<ProgEntry>> evicted;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->cap = entries;
        trim_code_locked(c, entries, evicted);
    }
    for (auto &p : evicted) retire(std::move(p));
    return PM_OK;
}

pm_status pm_cache_release(void) {
    reap_retired(true);
    return PM_OK;
}

size_t pm_table_bytes(void) { return device_table_bytes(); }

pm_status pm_debug_fail_uploads(uint32_t count) {
    fail_next_uploads(count);
    return PM_OK;
}

pm_status pm_code_dims(const pm_code *c, uint32_t *alpha, uint32_t *beta, uint32_t *B, uint32_t *enc_rows) {
    if (!c) return PM_EINVAL;
    if (alpha) *alpha = static_cast<uint32_t>(c->m.alpha);
    if (beta) *beta = 1;
    if (B) *B = static_cast<uint32_t>(c->m.B);
    if (enc_rows) *enc_rows = static_cast<uint32_t>(c->w16 ? c->w16->m.enc.rows : c->m.enc.rows);
    return PM_OK;
}

pm_status pm_code_matrix(const pm_code *c, int which, uint8_t *dst, size_t cap, uint32_t *rows, uint32_t *cols) {
    if (!c) return PM_EINVAL;
    if (c->w16) {   // two bytes per entry, little-endian
        const w16::Code16 &m = c->w16->m;
        w16::Mat16 lam;
        const w16::Mat16 *M = nullptr;
        switch (which) {
            case 0: M = &m.psi; break;
            case 1:
                lam = w16::Mat16(1, m.n);
                std::copy(m.lambda.begin(), m.lambda.end(), lam.v.begin());
                M = &lam;
                break;
            case 2: M = &m.G; break;
            case 3: M = &m.Gsys; break;
            case 4: M = &m.enc; break;
            default: return PM_EINVAL;
        }
        if (rows) *rows = static_cast<uint32_t>(M->rows);
        if (cols) *cols = static_cast<uint32_t>(M->cols);
        if (!dst) return PM_OK;
        if (cap < 2 * M->v.size()) return PM_EINVAL;
        for (size_t i = 0; i < M->v.size(); ++i) {
            dst[2 * i] = static_cast<uint8_t>(M->v[i]);
            dst[2 * i + 1] = static_cast<uint8_t>(M->v[i] >> 8);
        }
        return PM_OK;
    }
    const Mat *M = nullptr;
    Mat lam;
    switch (which) {
        case 0: M = &c->m.psi; break;
        case 1:
            if (c->m.kind != KIND_MSR) return PM_EINVAL;
            lam = Mat(1, c->m.n);
            std::copy(c->m.lambda.begin(), c->m.lambda.end(), lam.v.begin());
            M = &lam;
            break;
        case 2: M = &c->m.G; break;
        case 3: M = &c->m.Gsys; break;
        case 4: M = &c->m.enc; break;
        default: return PM_EINVAL;
    }
    if (rows) *rows = static_cast<uint32_t>(M->rows);
    if (cols) *cols = static_cast<uint32_t>(M->cols);
    if (!dst) return PM_OK;
    if (cap < M->v.size()) return PM_EINVAL;
    std::memcpy(dst, M->v.data(), M->v.size());
    return PM_OK;
}

pm_status pm_code_node_map(const pm_code *c, int32_t *map, size_t cap) {
    if (!c || !map) return PM_EINVAL;
    const std::vector<int32_t> &nm = c->w16 ? c->w16->m.node_map : c->m.node_map;
    if (cap < nm.size()) return PM_EINVAL;
    std::copy(nm.begin(), nm.end(), map);
    return PM_OK;
}

pm_status pm_set_variant(pm_code *c, int op, uint32_t rg, uint32_t vec) {
    const bool reset = rg == 0 && vec == 0;
    if (!reset && ((rg != 4 && rg != 8 && rg != 16) ||
                   (vec != 2 && vec != 4 && vec != 12 && vec != 14 && vec != 22 && vec != 24 &&
                    vec != kVecBitslice && vec != kVecMfma) ||
                   ((vec == kVecBitslice || vec == kVecMfma) && rg != 8)))
        return PM_EINVAL;
    if (op == 4) {
        set_apply_variant(static_cast<int>(rg), static_cast<int>(vec));
        return PM_OK;
    }
    if (!c || op < 0 || op > 3) return PM_EINVAL;
    if (c->w16) return PM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(c->mu);
    c->var[op].rg = static_cast<int>(rg);
    c->var[op].vec = reset ? 0 : static_cast<int>(vec);
    return PM_OK;
}


pm_status pm_decode_specific_workspace(const pm_code *c, size_t s, size_t *bytes) {
    if (!c || !bytes || s == 0) return PM_EINVAL;
    if (c->m.kind != KIND_MSR && c->m.kind != KIND_MBR) return PM_EUNSUPPORTED;
    *bytes = specific_ws_blocks(c->m) * ((s + 15) / 16 * 16);
    return PM_OK;
}

}  // extern "C"

namespace {

// The passes of a specific decode over a workspace of at least
// specific_ws_blocks(m) blocks of ld bytes (checked by the callers).
// resident_only: launch only kernels and tables already on the device.
pm_status run_specific(pm_code *c, const SpecificOps &ops, w16::Prog16 *const *pe16, const uint8_t *Y, size_t y_ld,
                       uint8_t *X, size_t x_ld, size_t s, uint8_t *workspace, hipStream_t h, bool resident_only) {
    const CodeMats &m = c->m;
    const size_t ld = (s + 15) / 16 * 16;
    // the workspace must not overlap the caller's regions
    const uintptr_t w0 = reinterpret_cast<uintptr_t>(workspace), w1 = w0 + specific_ws_blocks(m) * ld;
    auto clear = [&](const uint8_t *base, size_t rld, size_t rows) {
        const uintptr_t b0 = reinterpret_cast<uintptr_t>(base), b1 = b0 + (rows - 1) * rld + s;
        return b1 <= w0 || w1 <= b0;
    };
    if (!clear(Y, y_ld, static_cast<size_t>(m.k) * m.alpha) || !clear(X, x_ld, static_cast<size_t>(m.B)))
        return PM_EINVAL;
    // pass p reads the previous pass's output (the node blocks for p = 0) and
    // writes the next workspace slice (X for the last pass)
    const uint8_t *in = Y;
    size_t in_ld = y_ld, in_n = static_cast<size_t>(m.k) * m.alpha;
    uint8_t *slice = workspace;
    for (int p = 0; p < ops.npass; ++p) {
        const bool last = p == ops.npass - 1;
        uint8_t *out = last ? X : slice;
        const size_t out_ld = last ? x_ld : ld;
        const int st = c->w16 ? w16::launch16(*pe16[p], in, in_ld, in_n, out, out_ld, ops.rows[p], s, h)
                              : launch_program(*ops.pe[p], kVecAuto, in, in_ld, in_n, out, out_ld, ops.rows[p], s, h,
                                               resident_only);
        if (st != ST_OK) return static_cast<pm_status>(st);
        in = out;
        in_ld = out_ld;
        in_n = static_cast<size_t>(ops.rows[p]);
        slice += static_cast<size_t>(ops.rows[p]) * ld;
    }
    return PM_OK;
}

}  // namespace

extern "C" {

pm_status pm_decode_specific(const pm_code *cc, const uint32_t *nodes, const uint8_t *Y, size_t y_ld, uint8_t *X,
                             size_t x_ld, size_t s, uint8_t *workspace, size_t workspace_bytes, pm_stream stream) {
    if (s == 0 || !cc) return PM_EINVAL;
    pm_code *c = const_cast<pm_code *>(cc);
    // GF(2^8): programs of the region engine; GF(2^16): of the GF(2^16) kernel
    SpecificOps ops;
    w16::Prog16 *pe16[kSpecificPasses] = {};
    int st = c->w16 ? w16::resolve_specific16(*c->w16, nodes, pe16, ops.rows, &ops.npass)
                    : resolve_specific(c, nodes, &ops);
    if (st != ST_OK) return static_cast<pm_status>(st);
    const size_t ld = (s + 15) / 16 * 16;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 15u) ||
        workspace_bytes < specific_ws_blocks(c->m) * ld)
        return PM_EINVAL;
    return run_specific(c, ops, pe16, Y, y_ld, X, x_ld, s, workspace, reinterpret_cast<hipStream_t>(stream), false);
}

pm_status pm_decode_specific_noalloc(const pm_code *cc, const uint32_t *nodes, const uint8_t *Y, size_t y_ld,
                                     uint8_t *X, size_t x_ld, size_t s, pm_stream stream) {
    if (s == 0 || !cc) return PM_EINVAL;
    pm_code *c = const_cast<pm_code *>(cc);
    if (c->w16) return PM_EUNSUPPORTED;
    if (c->m.kind != KIND_MSR && c->m.kind != KIND_MBR) return PM_EUNSUPPORTED;
    const size_t ld = (s + 15) / 16 * 16;
    if (specific_ws_blocks(c->m) * ld > kNoAllocScratchBytes) return PM_ELIMIT;
    SpecificOps ops;
    int st = resolve_specific(c, nodes, &ops, true);
    if (st != ST_OK) return static_cast<pm_status>(st);
    void *scratch = nullptr;
    hipError_t e = pmk_noalloc_scratch(&scratch);
    if (e != hipSuccess) return static_cast<pm_status>(hip_fail(e));
    return run_specific(c, ops, nullptr, Y, y_ld, X, x_ld, s, static_cast<uint8_t *>(scratch),
                        reinterpret_cast<hipStream_t>(stream), true);
}

pm_status pm_decode_specific_factor(const pm_code *cc, const uint32_t *nodes, int which, uint8_t *dst, size_t cap,
                                    uint32_t *rows, uint32_t *cols) {
    if (which < 0 || which >= kSpecificPasses || !cc) return PM_EINVAL;
    pm_code *c = const_cast<pm_code *>(cc);
    if (c->w16) {   // two bytes per entry, little-endian
        w16::Prog16 *pe16[kSpecificPasses];
        int rows16[kSpecificPasses], npass = 0;
        int st = w16::resolve_specific16(*c->w16, nodes, pe16, rows16, &npass);
        if (st != ST_OK) return static_cast<pm_status>(st);
        const w16::Mat16 *F = w16::specific_factor16(*c->w16, nodes, which);
        if (!F) return PM_EINVAL;
        if (rows) *rows = static_cast<uint32_t>(F->rows);
        if (cols) *cols = static_cast<uint32_t>(F->cols);
        if (dst) {
            if (cap < 2 * F->v.size()) return PM_EINVAL;
            for (size_t i = 0; i < F->v.size(); ++i) {
                dst[2 * i] = static_cast<uint8_t>(F->v[i]);
                dst[2 * i + 1] = static_cast<uint8_t>(F->v[i] >> 8);
            }
        }
        return PM_OK;
    }
    // resolve, then read the factor under the lock; another thread's use
    // of the cache may evict the entry in between, hence the retry
    Mat F;
    for (int attempt = 0;; ++attempt) {
        SpecificOps ops;
        int st = resolve_specific(c, nodes, &ops);
        if (st != ST_OK) return static_cast<pm_status>(st);
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->specific.find(std::vector<int>(nodes, nodes + c->m.k));
        if (it != c->specific.end()) {
            F = it->second.F[which];
            break;
        }
        if (attempt >= 8) return PM_EBUSY;
    }
    if (rows) *rows = static_cast<uint32_t>(F.rows);
    if (cols) *cols = static_cast<uint32_t>(F.cols);
    if (dst) {
        if (cap < F.v.size()) return PM_EINVAL;
        std::copy(F.v.begin(), F.v.end(), dst);
    }
    return PM_OK;
}


}  // extern "C"

namespace {

// Whether one problem of m candidates, B columns and nsets node ids fits
// one work-group's LDS on the current device.
int gj_check(uint32_t B, uint32_t m, uint32_t nsets) {
    if (B == 0 || m < B) return ST_EINVAL;
    int dev = 0, maxlds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if ((e = hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev)) != hipSuccess)
        return hip_fail(e);
    return pmk_gj_lds_bytes(B, m, nsets) <= static_cast<size_t>(maxlds) ? ST_OK : ST_EUNSUPPORTED;
}

}  // namespace

extern "C" {

pm_status pm_decode_matrix(const pm_code *cc, const uint32_t *nodes, uint8_t *D, size_t cap, uint32_t *kept) {
    if (!cc || !nodes) return PM_EINVAL;
    if (cc->w16) return PM_EUNSUPPORTED;
    pm_code *c = const_cast<pm_code *>(cc);
    const CodeMats &m = c->m;
    std::vector<int> list(nodes, nodes + m.k), sorted = list;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) return PM_EINVAL;
    for (int v : list)
        if (v < 0 || v >= m.n) return PM_EINVAL;
    if (D && cap < static_cast<size_t>(m.B) * m.B) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    Aged<std::pair<Mat, std::vector<int>>> *dm = nullptr;
    int st = get_mat(c, c->decode_mat, list,
                     [&](std::pair<Mat, std::vector<int>> &out) { return decode_matrix(m, list, out.first, out.second); },
                     &dm);
    if (st != ST_OK) return static_cast<pm_status>(st);
    if (D) std::copy(dm->v.first.v.begin(), dm->v.first.v.end(), D);
    if (kept)
        for (size_t q = 0; q < dm->v.second.size(); ++q) kept[q] = static_cast<uint32_t>(dm->v.second[q]);
    return PM_OK;
}

pm_status pm_decode_matrices(const pm_code *cc, const uint32_t *node_sets, uint32_t count, uint8_t *D,
                             size_t d_stride, uint32_t *kept, int32_t *status, pm_stream stream) {
    if (!cc || !node_sets || !D || !status) return PM_EINVAL;
    if (cc->w16) return PM_EUNSUPPORTED;
    pm_code *c = const_cast<pm_code *>(cc);
    const CodeMats &m = c->m;
    const uint32_t B = static_cast<uint32_t>(m.B);
    if (d_stride < static_cast<size_t>(B) * B) return PM_EINVAL;
    if (count == 0) return PM_OK;
    int st = gj_check(B, static_cast<uint32_t>(m.k * m.alpha), static_cast<uint32_t>(m.k));
    if (st != ST_OK) return static_cast<pm_status>(st);
    hipStream_t h = reinterpret_cast<hipStream_t>(stream);
    const void *g = nullptr;
    if ((st = device_copy(c->dev_mu, c->gsys_dev, m.Gsys.v.data(), m.Gsys.v.size(), h, &g)) != ST_OK)
        return static_cast<pm_status>(st);
    const PmkGj a{static_cast<const uint8_t *>(g), B, 0, node_sets, static_cast<uint32_t>(m.k),
                  static_cast<uint32_t>(m.alpha), static_cast<uint32_t>(m.n),
                  static_cast<uint32_t>(m.k * m.alpha), B, D, B, d_stride, kept, status};
    hipError_t e = pmk_gj(&a, count, h);
    return e == hipSuccess ? PM_OK : static_cast<pm_status>(hip_fail(e));
}

pm_status pm_gf_invert_batch(const uint8_t *A, size_t a_ld, size_t a_stride, uint32_t m, uint32_t count,
                             uint8_t *Ainv, size_t inv_ld, size_t inv_stride, int32_t *status, pm_stream stream) {
    if (!A || !Ainv || !status || m == 0 || a_ld < m || inv_ld < m) return PM_EINVAL;
    if (count > 1 && (a_stride < (m - 1) * a_ld + m || inv_stride < (m - 1) * inv_ld + m)) return PM_EINVAL;
    if (count == 0) return PM_OK;
    int st = gj_check(m, m, 0);
    if (st != ST_OK) return static_cast<pm_status>(st);
    const PmkGj a{A, a_ld, a_stride, nullptr, 0, 1, 0, m, m, Ainv, inv_ld, inv_stride, nullptr, status};
    hipError_t e = pmk_gj(&a, count, reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? PM_OK : static_cast<pm_status>(hip_fail(e));
}

}  // extern "C"

namespace {

// With a GPU present, the init phase also uploads the table program and
// loads the compiled kernel (if any) on the current device, so that the
// first data call after pm_prepare does neither; with none it only compiles.
int stage_on_device(ProgEntry &pe, BsProgram *bp, BsKind kind) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return ST_OK;
    }
    // a dense matrix on the matrix cores needs only their operands there
    if (!bp && pe.mfma_eligible()) return pe.stage_mfma();
    const uint32_t *d = nullptr;
    int st = pe.device_ptr_sync(&d);
    if (st == ST_OK && bp) st = bs_load(*bp, kind);
    return st;
}

}  // namespace

namespace {

// One data-phase operation of a GF(2^16) code on the GF(2^16) region kernel.
pm_status run16(const pm_code *cc, int op, uint32_t failed, const uint32_t *ids, const uint8_t *in, size_t in_ld,
                uint8_t *out, size_t out_ld, size_t s, pm_stream stream) {
    w16::Prog16 *pe = nullptr;
    size_t in_n = 0, out_n = 0;
    int st = w16::resolve16(*const_cast<pm_code *>(cc)->w16, op, failed, ids, &pe, &in_n, &out_n);
    if (st != ST_OK) return static_cast<pm_status>(st);
    return static_cast<pm_status>(
        w16::launch16(*pe, in, in_ld, in_n, out, out_ld, out_n, s, reinterpret_cast<hipStream_t>(stream)));
}

}  // namespace

extern "C" {

pm_status pm_prepare(pm_code *c, int op, uint32_t failed, const uint32_t *ids, uint32_t flags, int *specialized) {
    if (specialized) *specialized = 0;
    if (!c || op < 0 || op > 5 || (flags & ~static_cast<uint32_t>(PM_PREPARE_BATCHED))) return PM_EINVAL;
    if (op == 5) {   // pm_repair: the projections as one multi-set launch, then the newcomer
        if (c->w16) return pm_prepare(c, 2, failed, ids, 0, specialized);
        int s1 = 0, s2 = 0;
        pm_status st = pm_prepare(c, 1, failed, nullptr, PM_PREPARE_BATCHED, &s1);
        if (st == PM_OK) st = pm_prepare(c, 2, failed, ids, flags, &s2);
        if (specialized) *specialized = s1 && s2;
        return st;
    }
    if (c->w16) {   // the matrices, their programs and bit-sliced kernels, staged on the device
        if (flags & PM_PREPARE_BATCHED) return PM_EUNSUPPORTED;
        w16::Prog16 *pe[kSpecificPasses] = {};
        int rows[kSpecificPasses], npass = 1;
        size_t in_n = 0, out_n = 0;
        int st = op == 4 ? w16::resolve_specific16(*c->w16, ids, pe, rows, &npass)
                         : w16::resolve16(*c->w16, op, failed, ids, &pe[0], &in_n, &out_n);
        int all = 1;
        for (int p = 0; p < npass && st == ST_OK; ++p) {
            int sp = 0;
            st = w16::compile16(*pe[p], &sp);
            all &= sp;
        }
        int ndev = 0;
        if (st == ST_OK && hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0)
            for (int p = 0; p < npass && st == ST_OK; ++p) st = w16::stage16(*pe[p]);
        else
            (void)hipGetLastError();
        if (specialized && st == ST_OK) *specialized = all;
        return static_cast<pm_status>(st);
    }
    if (op == 4) {   // the passes of the specific decode
        SpecificOps ops;
        int st = resolve_specific(c, ids, &ops);
        if (st != ST_OK) return static_cast<pm_status>(st);
        const BsKind kind = (flags & PM_PREPARE_BATCHED) ? BS_MULTI : BS_SINGLE;
        int all = 1;
        for (int p = 0; p < ops.npass; ++p) {
            std::shared_ptr<BsProgram> bp = ops.pe[p]->bitslice();
            if (!bp) all = 0;
            else if ((st = bs_compile(*bp, kind)) != ST_OK) return static_cast<pm_status>(st);
            if ((st = stage_on_device(*ops.pe[p], bp.get(), kind)) != ST_OK) return static_cast<pm_status>(st);
        }
        // set-up of pm_decode_specific_noalloc: its scratch address on this
        // device (the first lookup may load the library's code object)
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
            void *scratch = nullptr;
            hipError_t e = pmk_noalloc_scratch(&scratch);
            if (e != hipSuccess) return static_cast<pm_status>(hip_fail(e));
        } else {
            (void)hipGetLastError();
        }
        if (specialized) *specialized = all;
        return PM_OK;
    }
    Resolved r;
    int st = resolve_op(c, op, failed, ids, &r);
    if (st != ST_OK) return static_cast<pm_status>(st);
    const BsKind kind = (flags & PM_PREPARE_BATCHED) ? BS_MULTI : BS_SINGLE;
    std::shared_ptr<BsProgram> bp;
    if (r.vec == kVecAuto || r.vec == kVecBitslice) bp = r.pe->bitslice();   // else an explicit table variant
    if (bp && (st = bs_compile(*bp, kind)) != ST_OK) return static_cast<pm_status>(st);
    if ((st = stage_on_device(*r.pe, bp.get(), kind)) != ST_OK) return static_cast<pm_status>(st);
    if (specialized) *specialized = bp ? 1 : 0;
    return PM_OK;
}

pm_status pm_encode(const pm_code *cc, const uint8_t *X, size_t x_ld, uint8_t *out, size_t out_ld,
                    size_t s, pm_stream stream) {
    if (s == 0) return PM_EINVAL;
    if (cc && cc->w16) return run16(cc, OPK_ENCODE, 0, nullptr, X, x_ld, out, out_ld, s, stream);
    Resolved r;
    int st = resolve_op(const_cast<pm_code *>(cc), OPK_ENCODE, 0, nullptr, &r);
    if (st != ST_OK) return static_cast<pm_status>(st);
    return static_cast<pm_status>(launch_program(*r.pe, r.vec, X, x_ld, r.in_n, out, out_ld, r.out_n, s,
                                                 reinterpret_cast<hipStream_t>(stream)));
}

pm_status pm_repair_helper(const pm_code *cc, uint32_t failed, const uint8_t *node, size_t node_ld,
                           uint8_t *out, size_t s, pm_stream stream) {
    if (s == 0) return PM_EINVAL;
    if (cc && cc->w16) return run16(cc, OPK_HELPER, failed, nullptr, node, node_ld, out, (s + 15) / 16 * 16, s, stream);
    Resolved r;
    int st = resolve_op(const_cast<pm_code *>(cc), OPK_HELPER, failed, nullptr, &r);
    if (st != ST_OK) return static_cast<pm_status>(st);
    const size_t out_ld = (s + 15) / 16 * 16;   // one output block: ld only has to be valid
    return static_cast<pm_status>(launch_program(*r.pe, r.vec, node, node_ld, r.in_n, out, out_ld, 1, s,
                                                 reinterpret_cast<hipStream_t>(stream)));
}

pm_status pm_repair_workspace(const pm_code *c, size_t s, size_t *bytes) {
    if (!c || !bytes || s == 0) return PM_EINVAL;
    *bytes = repair_ws_bytes(c->m, s);
    return PM_OK;
}

pm_status pm_repair(const pm_code *cc, uint32_t failed, const uint32_t *helpers, const uint8_t *const *helper_nodes,
                    size_t node_ld, uint8_t *workspace, size_t workspace_bytes, uint8_t *out, size_t out_ld, size_t s,
                    pm_stream stream) {
    if (!cc || s == 0 || !helpers || !helper_nodes) return PM_EINVAL;
    pm_code *c = const_cast<pm_code *>(cc);
    const CodeMats &m = c->m;
    const size_t d = static_cast<size_t>(m.kind == KIND_RS ? m.k : m.d);
    const size_t ld = (s + 15) / 16 * 16;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 15u) || workspace_bytes < repair_ws_bytes(m, s))
        return PM_EINVAL;
    hipStream_t h = reinterpret_cast<hipStream_t>(stream);
    uint8_t *recv = workspace;
    const size_t node_blocks = static_cast<size_t>(m.kind == KIND_RS ? 1 : m.alpha);
    // no output may overlap an input or the other output
    for (size_t j = 0; j < d; ++j) {
        int st = check_regions(helper_nodes[j], node_ld, node_blocks, s);
        if (st != ST_OK) return static_cast<pm_status>(st);
        if (overlaps(helper_nodes[j], node_ld, node_blocks, recv, ld, d, s) ||
            overlaps(helper_nodes[j], node_ld, node_blocks, out, out_ld, static_cast<size_t>(m.alpha), s))
            return PM_EINVAL;
    }
    if (overlaps(recv, ld, d, out, out_ld, static_cast<size_t>(m.alpha), s)) return PM_EINVAL;
    if (c->w16) {   // the GF(2^16) kernel: one projection call per helper
        for (size_t j = 0; j < d; ++j) {
            pm_status st = run16(cc, OPK_HELPER, failed, nullptr, helper_nodes[j], node_ld, recv + j * ld, ld, s, stream);
            if (st != PM_OK) return st;
        }
        return run16(cc, OPK_NEWCOMER, failed, helpers, recv, ld, out, out_ld, s, stream);
    }
    Resolved hr, nr;
    int st = resolve_op(c, OPK_HELPER, failed, nullptr, &hr);
    if (st == ST_OK) st = resolve_op(c, OPK_NEWCOMER, failed, helpers, &nr);
    if (st != ST_OK) return static_cast<pm_status>(st);
    // 1. the d projections, one launch of the multi-set kernel when the
    // helper vector's is compiled (its launch list goes to the workspace
    // tail in stream order), else one launch per helper
    std::shared_ptr<BsProgram> bp;
    if (s >= kBsTileBytes && (hr.vec == kVecAuto || hr.vec == kVecBitslice) && hr.pe->prog.ngroups > 0)
        bp = hr.pe->bitslice_if_compiled(BS_MULTI);
    if (bp && d * sizeof(BsItem) / 4 > kPutWords) bp = nullptr;   // d > 68: list too long for one put
    if (bp) {
        std::vector<BsItem> items;
        uint32_t tile = 0;
        for (size_t j = 0; j < d; ++j) {
            items.push_back(bs_item(helper_nodes[j], node_ld, recv + j * ld, ld, s, tile));
            tile += items.back().ntiles;
        }
        uint32_t *list = reinterpret_cast<uint32_t *>(workspace + d * ld);
        const uint32_t words = static_cast<uint32_t>(items.size() * sizeof(BsItem) / 4);
        hipError_t e = pmk_put(list, reinterpret_cast<const uint32_t *>(items.data()), words, h);
        if (e != hipSuccess) return static_cast<pm_status>(hip_fail(e));
        st = bs_launch_items(*bp, reinterpret_cast<const BsItem *>(list), static_cast<uint32_t>(d), tile, h);
    } else {
        for (size_t j = 0; j < d && st == ST_OK; ++j)
            st = launch_program(*hr.pe, hr.vec, helper_nodes[j], node_ld, hr.in_n, recv + j * ld, ld, 1, s, h);
    }
    if (st != ST_OK) return static_cast<pm_status>(st);
    // 2. the newcomer's solve over the d received blocks
    return static_cast<pm_status>(launch_program(*nr.pe, nr.vec, recv, ld, nr.in_n, out, out_ld, nr.out_n, s, h));
}

pm_status pm_repair_newcomer(const pm_code *cc, uint32_t failed, const uint32_t *helpers, const uint8_t *recv,
                             size_t recv_ld, uint8_t *out, size_t out_ld, size_t s, pm_stream stream) {
    if (s == 0) return PM_EINVAL;
    if (cc && cc->w16) return run16(cc, OPK_NEWCOMER, failed, helpers, recv, recv_ld, out, out_ld, s, stream);
    Resolved r;
    int st = resolve_op(const_cast<pm_code *>(cc), OPK_NEWCOMER, failed, helpers, &r);
    if (st != ST_OK) return static_cast<pm_status>(st);
    return static_cast<pm_status>(launch_program(*r.pe, r.vec, recv, recv_ld, r.in_n, out, out_ld, r.out_n, s,
                                                 reinterpret_cast<hipStream_t>(stream)));
}

pm_status pm_decode(const pm_code *cc, const uint32_t *nodes, const uint8_t *Y, size_t y_ld, uint8_t *X,
                    size_t x_ld, size_t s, pm_stream stream) {
    if (s == 0) return PM_EINVAL;
    if (cc && cc->w16) return run16(cc, OPK_DECODE, 0, nodes, Y, y_ld, X, x_ld, s, stream);
    Resolved r;
    int st = resolve_op(const_cast<pm_code *>(cc), OPK_DECODE, 0, nodes, &r);
    if (st != ST_OK) return static_cast<pm_status>(st);
    return static_cast<pm_status>(launch_program(*r.pe, r.vec, Y, y_ld, r.in_n, X, x_ld, r.out_n, s,
                                                 reinterpret_cast<hipStream_t>(stream)));
}

pm_status pm_apply(const uint8_t *A, uint32_t rows, uint32_t cols, const uint8_t *in, size_t in_ld, uint8_t *out,
                   size_t out_ld, size_t s, pm_stream stream) {
    if (!A || rows == 0 || cols == 0 || s == 0) return PM_EINVAL;
    Mat M(static_cast<int>(rows), static_cast<int>(cols));
    std::memcpy(M.v.data(), A, M.v.size());
    int vec = 0;
    std::shared_ptr<ProgEntry> pe = apply_program(M, &vec);
    return static_cast<pm_status>(launch_program(*pe, vec, in, in_ld, cols, out, out_ld, rows, s,
                                                 reinterpret_cast<hipStream_t>(stream)));
}

pm_status pm_autotune_encode(pm_code *c, const uint8_t *X, size_t x_ld, uint8_t *out, size_t out_ld, size_t s,
                             uint32_t reps, pm_stream stream, uint32_t *best_rg, uint32_t *best_vec) {
    if (!c || s == 0 || reps == 0) return PM_EINVAL;
    if (c->w16) return PM_EUNSUPPORTED;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return static_cast<pm_status>(hip_fail(e));
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return static_cast<pm_status>(hip_fail(e));
    }
    float best = 1e30f;
    int brg = 0, bvec = 0;
    pm_status rc = PM_OK;
    for (int rg : {4, 8, 16}) {
        for (int vec : {2, 4, 12, 14, 22, 24, kVecBitslice, kVecMfma}) {
            // one specialization per matrix; the matrix cores for dense ones
            if ((vec == kVecBitslice || vec == kVecMfma) && rg != 8) continue;
            pm_set_variant(c, 0, static_cast<uint32_t>(rg), static_cast<uint32_t>(vec));
            rc = pm_encode(c, X, x_ld, out, out_ld, s, stream);   // warm-up (and upload)
            if (rc != PM_OK) break;
            (void)hipEventRecord(e0, st);
            for (uint32_t i = 0; i < reps && rc == PM_OK; ++i) rc = pm_encode(c, X, x_ld, out, out_ld, s, stream);
            (void)hipEventRecord(e1, st);
            if (rc != PM_OK) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) { rc = static_cast<pm_status>(hip_fail(e)); break; }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; brg = rg; bvec = vec; }
        }
        if (rc != PM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != PM_OK) {
        pm_set_variant(c, 0, 0, 0);
        return rc;
    }
    pm_set_variant(c, 0, static_cast<uint32_t>(brg), static_cast<uint32_t>(bvec));
    if (best_rg) *best_rg = static_cast<uint32_t>(brg);
    if (best_vec) *best_vec = static_cast<uint32_t>(bvec);
    return PM_OK;
}

}  // extern "C"
