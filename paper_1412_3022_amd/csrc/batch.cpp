// Batched launches (C ABI in include/pm.h): a plan resolves every item to
// its kernel program once, lays the items out as a device work list per row
// group size, and runs them as one persistent work-list launch per size, all
// captured in a HIP graph on first use.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "construct.hpp"
#include "engine.hpp"
#include "pm.h"

using namespace pmrc;

struct PmkBatch {
    const void *items;
    uint32_t nitems, nunits;
    uint32_t *counters;
};
extern "C" hipError_t pmk_batch(int rg, int vec, const PmkBatch *h, hipStream_t st);
extern "C" int pmk_batch_item_bytes();
extern "C" int pmk_wave_bytes(int vec);

namespace {

// Host image of the device work-list entry (layout fixed by the kernel).
struct HostItem {
    const uint32_t *prog;
    const uint8_t *in;
    uint8_t *out;
    uint64_t in_ld, out_ld, s;
    uint32_t ngroups, ntiles;
    uint32_t unit0, pad;
};
static_assert(sizeof(HostItem) == 64, "work-list entry layout");

struct Member {
    const uint32_t *prog;
    int ngroups;
    const uint8_t *in;
    uint8_t *out;
    uint64_t in_ld, out_ld, s;
};

struct SizeClass {
    int rg = 0;
    int vec = 2;
    std::vector<Member> members;
    void *d_items = nullptr;
    uint32_t nitems = 0, nunits = 0;
};

// Items whose matrix has a compiled multi-set bit-sliced kernel: one launch
// of that kernel over all of them.
struct BsClass {
    std::shared_ptr<BsProgram> bp;
    std::vector<BsItem> items;
    BsItem *d_items = nullptr;
    uint32_t ntiles = 0;
    uint32_t slots = 0;   // work-group slots per XCD of its launch (0 = resident count; the autotuner sets it)
};

}  // namespace

struct pm_batch {
    // programs whose device tables the work lists point to: kept alive (and
    // out of reach of cache eviction) for the life of the plan
    std::vector<std::shared_ptr<ProgEntry>> keep;
    std::vector<SizeClass> classes;
    std::vector<BsClass> bs_classes;
    uint32_t *d_counters = nullptr;   // 8 queue heads per class, 64 B apart
    uint32_t flags = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~pm_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto &c : classes)
            if (c.d_items) (void)hipFree(c.d_items);
        for (auto &c : bs_classes)
            if (c.d_items) (void)hipFree(c.d_items);
        if (d_counters) (void)hipFree(d_counters);
    }
};

namespace {

bool overlap(const void *a, uint64_t a_ld, size_t a_n, const void *b, uint64_t b_ld, size_t b_n, uint64_t s) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), a1 = a0 + (a_n - 1) * a_ld + s;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(b), b1 = b0 + (b_n - 1) * b_ld + s;
    return a0 < b1 && b0 < a1;
}

// Lay out one class's work list for `vec` dwords per lane and upload it.
int build_class(SizeClass &c, int vec) {
    const uint64_t wave_bytes = static_cast<uint64_t>(pmk_wave_bytes(vec));
    std::vector<HostItem> items;
    uint64_t unit = 0;
    for (const Member &m : c.members) {
        const uint64_t ntiles = (m.s + wave_bytes - 1) / wave_bytes;
        const uint64_t units = ntiles * static_cast<uint64_t>(m.ngroups);
        if (units == 0) continue;
        HostItem h{m.prog, m.in, m.out, m.in_ld, m.out_ld, m.s, static_cast<uint32_t>(m.ngroups),
                   static_cast<uint32_t>(ntiles), static_cast<uint32_t>(unit), 0};
        items.push_back(h);
        unit += units;
        if (unit > 0xffffff00ull) return ST_EINVAL;
    }
    if (c.d_items) {
        // A previous work list may still be read by a launch in flight.
        (void)hipDeviceSynchronize();
        (void)hipFree(c.d_items);
        c.d_items = nullptr;
    }
    c.vec = vec;
    c.nitems = static_cast<uint32_t>(items.size());
    c.nunits = static_cast<uint32_t>(unit);
    if (items.empty()) return ST_OK;
    hipError_t e = hipMalloc(&c.d_items, items.size() * sizeof(HostItem));
    if (e != hipSuccess) {
        c.d_items = nullptr;
        return hip_fail(e);
    }
    e = hipMemcpy(c.d_items, items.data(), items.size() * sizeof(HostItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e);
    return ST_OK;
}

// Number the tiles of a bit-sliced class back to back and upload it.
int build_bs_class(BsClass &c) {
    uint64_t tile = 0;
    for (BsItem &it : c.items) {
        it.tile0 = static_cast<uint32_t>(tile);
        tile += it.ntiles;
        if (tile > 0xffffff00ull) return ST_EINVAL;
    }
    c.ntiles = static_cast<uint32_t>(tile);
    const size_t bytes = c.items.size() * sizeof(BsItem);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&c.d_items), bytes);
    if (e != hipSuccess) {
        c.d_items = nullptr;
        return hip_fail(e);
    }
    if ((e = hipMemcpy(c.d_items, c.items.data(), bytes, hipMemcpyHostToDevice)) != hipSuccess) return hip_fail(e);
    // compile (if needed) and load the module now, not inside a graph capture
    return bs_load(*c.bp, BS_MULTI);
}

int launch_all(pm_batch *b, hipStream_t st) {
    for (BsClass &c : b->bs_classes) {
        int rc = bs_launch_items(*c.bp, c.d_items, static_cast<uint32_t>(c.items.size()), c.ntiles, st, c.slots);
        if (rc != ST_OK) return rc;
    }
    for (size_t i = 0; i < b->classes.size(); ++i) {
        SizeClass &c = b->classes[i];
        if (!c.nunits) continue;
        PmkBatch h{c.d_items, c.nitems, c.nunits, b->d_counters + i * 8 * 16};
        hipError_t e = pmk_batch(c.rg, c.vec, &h, st);
        if (e != hipSuccess) return hip_fail(e);
    }
    return ST_OK;
}

void drop_graph(pm_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

}  // namespace

extern "C" {

pm_status pm_batch_plan(const pm_batch_item *items, size_t n, uint32_t flags, pm_batch **out) {
    if (!out || (!items && n)) return PM_EINVAL;
    *out = nullptr;
    if (hipInit(0) != hipSuccess) return PM_EHIP;
    std::unique_ptr<pm_batch> b(new pm_batch());
    b->flags = flags;
    std::map<int, size_t> by_rg;
    std::map<BsProgram *, size_t> by_bs;
    for (size_t i = 0; i < n; ++i) {
        const pm_batch_item &it = items[i];
        if (!it.code || it.block_bytes == 0 || it.op < 0 || it.op > 3) return PM_EINVAL;
        Resolved r;
        int st = resolve_op(const_cast<pm_code *>(it.code), it.op, it.failed, it.ids, &r);
        if (st != ST_OK) return static_cast<pm_status>(st);
        const uint64_t out_ld = it.op == 1 ? (it.block_bytes + 15) / 16 * 16 : it.out_ld;
        if ((st = check_regions(it.in, it.in_ld, r.in_n, it.block_bytes)) != ST_OK) return static_cast<pm_status>(st);
        if ((st = check_regions(it.out, out_ld, r.out_n, it.block_bytes)) != ST_OK)
            return static_cast<pm_status>(st);
        if (overlap(it.in, it.in_ld, r.in_n, it.out, out_ld, r.out_n, it.block_bytes)) return PM_EINVAL;
        if (r.pe->prog.ngroups == 0) continue;
        if (it.block_bytes >= kBsTileBytes && (r.vec == kVecAuto || r.vec == kVecBitslice)) {
            std::shared_ptr<BsProgram> bp;
            if (flags & PM_BATCH_SPECIALIZE) {
                if ((bp = r.pe->bitslice()) && (st = bs_compile(*bp, BS_MULTI)) != ST_OK)
                    return static_cast<pm_status>(st);
            } else {
                bp = r.pe->bitslice_if_compiled(BS_MULTI);
            }
            if (bp) {
                auto cls = by_bs.find(bp.get());
                if (cls == by_bs.end()) {
                    cls = by_bs.emplace(bp.get(), b->bs_classes.size()).first;
                    b->bs_classes.emplace_back();
                    b->bs_classes.back().bp = bp;
                }
                b->bs_classes[cls->second].items.push_back(
                    bs_item(it.in, it.in_ld, it.out, out_ld, it.block_bytes, 0));
                continue;
            }
        }
        const uint32_t *dprog = nullptr;
        if ((st = r.pe->device_ptr_sync(&dprog)) != ST_OK) return static_cast<pm_status>(st);
        if (b->keep.empty() || b->keep.back() != r.pe) b->keep.push_back(r.pe);
        auto cls = by_rg.find(r.pe->prog.rg);
        if (cls == by_rg.end()) {
            cls = by_rg.emplace(r.pe->prog.rg, b->classes.size()).first;
            b->classes.emplace_back();
            b->classes.back().rg = r.pe->prog.rg;
        }
        b->classes[cls->second].members.push_back(
            Member{dprog, r.pe->prog.ngroups, it.in, it.out, it.in_ld, out_ld, it.block_bytes});
    }
    for (SizeClass &c : b->classes) {
        int st = build_class(c, 2);
        if (st != ST_OK) return static_cast<pm_status>(st);
    }
    for (BsClass &c : b->bs_classes) {
        int st = build_bs_class(c);
        if (st != ST_OK) return static_cast<pm_status>(st);
    }
    const size_t cbytes = std::max<size_t>(1, b->classes.size()) * 8 * 16 * sizeof(uint32_t);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&b->d_counters), cbytes);
    if (e != hipSuccess) {
        b->d_counters = nullptr;
        return static_cast<pm_status>(hip_fail(e));
    }
    // the work-list kernels leave their counters at zero: only the first launch needs this
    if ((e = hipMemset(b->d_counters, 0, cbytes)) != hipSuccess) return static_cast<pm_status>(hip_fail(e));
    *out = b.release();
    return PM_OK;
}

pm_status pm_batch_set_variant(pm_batch *b, uint32_t rows_per_group, uint32_t dwords_per_lane) {
    if (!b || (dwords_per_lane != 2 && dwords_per_lane != 4)) return PM_EINVAL;
    for (SizeClass &c : b->classes) {
        if (rows_per_group && static_cast<int>(rows_per_group) != c.rg) continue;
        int st = build_class(c, static_cast<int>(dwords_per_lane));
        if (st != ST_OK) return static_cast<pm_status>(st);
    }
    drop_graph(b);
    return PM_OK;
}

pm_status pm_batch_run(pm_batch *b, pm_stream stream) {
    if (!b) return PM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(b->flags & PM_BATCH_GRAPH)) return static_cast<pm_status>(launch_all(b, st));
    hipError_t e;
    if (!b->exec) {
        // Capture the reset + work-list launches once; later runs replay them.
        hipStream_t cap;
        if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
            return static_cast<pm_status>(hip_fail(e));
        if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
            (void)hipStreamDestroy(cap);
            return static_cast<pm_status>(hip_fail(e));
        }
        int rc = launch_all(b, cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cap, &g);
        (void)hipStreamDestroy(cap);
        if (rc != ST_OK) {
            if (g) (void)hipGraphDestroy(g);
            return static_cast<pm_status>(rc);
        }
        if (e != hipSuccess) return static_cast<pm_status>(hip_fail(e));
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            b->exec = nullptr;
            return static_cast<pm_status>(hip_fail(e));
        }
    }
    if ((e = hipGraphLaunch(b->exec, st)) != hipSuccess) return static_cast<pm_status>(hip_fail(e));
    return PM_OK;
}

pm_status pm_batch_autotune(pm_batch *b, uint32_t reps, pm_stream stream, uint32_t *best_dwords_per_lane) {
    if (!b || reps == 0) return PM_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return static_cast<pm_status>(hip_fail(e));
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return static_cast<pm_status>(hip_fail(e));
    }
    const uint32_t saved = b->flags;
    b->flags &= ~static_cast<uint32_t>(PM_BATCH_GRAPH);
    int rc = ST_OK;
    uint32_t best_vec = 2;
    // Each size class is tuned on its own: its tile width changes only its
    // own work list.
    for (SizeClass &c : b->classes) {
        float best = 1e30f;
        for (int vec : {2, 4}) {
            if ((rc = build_class(c, vec)) != ST_OK) break;
            PmkBatch h{c.d_items, c.nitems, c.nunits,
                       b->d_counters + static_cast<size_t>(&c - b->classes.data()) * 8 * 16};
            if ((e = pmk_batch(c.rg, vec, &h, st)) != hipSuccess) { rc = hip_fail(e); break; }
            (void)hipEventRecord(e0, st);
            for (uint32_t i = 0; i < reps; ++i)
                if ((e = pmk_batch(c.rg, vec, &h, st)) != hipSuccess) { rc = hip_fail(e); break; }
            (void)hipEventRecord(e1, st);
            if (rc != ST_OK) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) { rc = hip_fail(e); break; }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; best_vec = static_cast<uint32_t>(vec); }
        }
        if (rc != ST_OK) break;
        if ((rc = build_class(c, static_cast<int>(best_vec))) != ST_OK) break;
    }
    // The bit-sliced launches carry most bytes: each matrix's persistent
    // grid is timed at half, all and twice its resident work-group slots
    // (fewer waves leave more of L2 to each; more let the dispatcher fill
    // the gaps that waves finishing early leave), and keeps the fastest.
    for (BsClass &c : b->bs_classes) {
        if (rc != ST_OK) break;
        const uint32_t p0 = bs_default_slots(*c.bp);
        if (!p0) {
            rc = ST_EHIP;
            break;
        }
        float best = 1e30f;
        uint32_t best_p = p0;
        const uint32_t n = static_cast<uint32_t>(c.items.size());
        for (uint32_t p : {std::max(1u, p0 / 2), p0, 2 * p0}) {
            if ((rc = bs_launch_items(*c.bp, c.d_items, n, c.ntiles, st, p)) != ST_OK) break;
            (void)hipEventRecord(e0, st);
            for (uint32_t i = 0; i < reps && rc == ST_OK; ++i) rc = bs_launch_items(*c.bp, c.d_items, n, c.ntiles, st, p);
            (void)hipEventRecord(e1, st);
            if (rc != ST_OK) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) { rc = hip_fail(e); break; }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; best_p = p; }
        }
        c.slots = best_p;
    }
    b->flags = saved;
    drop_graph(b);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_dwords_per_lane) *best_dwords_per_lane = best_vec;
    return static_cast<pm_status>(rc);
}

pm_status pm_batch_info(const pm_batch *b, uint64_t *units, uint32_t *size_classes) {
    if (!b) return PM_EINVAL;
    uint64_t u = 0;
    for (const SizeClass &c : b->classes) u += c.nunits;
    for (const BsClass &c : b->bs_classes) u += static_cast<uint64_t>(c.ntiles) * c.bp->ngroups;
    if (units) *units = u;
    if (size_classes) *size_classes = static_cast<uint32_t>(b->classes.size() + b->bs_classes.size());
    return PM_OK;
}

void pm_batch_destroy(pm_batch *b) { delete b; }

}  // extern "C"
