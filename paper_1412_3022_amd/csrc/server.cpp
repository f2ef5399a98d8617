// Served mode (C ABI in include/pm.h): continuous batching of encode, repair
// and decode requests under an HBM budget.
//
// A scheduler thread admits queued requests in arrival order while the
// arena (one device allocation of the budget's size) can hold their outputs
// and repair scratch, packs the admitted ones into a micro-batch, and runs it
// on one of several streams as work-list launches: phase 1 holds encodes,
// decodes and the helper projections of repairs, phase 2 the newcomer
// solves (stream order makes phase 2 see phase 1's scratch).  Requests that
// arrive while earlier micro-batches are on the GPU are admitted into the
// next free stream slot, so their work overlaps on the device.  Results stay
// in the arena until the client releases them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "construct.hpp"
#include "engine.hpp"
#include "mfma.hpp"
#include "pm.h"

using namespace pmrc;

struct PmkBatch {
    const void *items;
    uint32_t nitems, nunits;
    uint32_t *counters;
};
extern "C" hipError_t pmk_batch(int rg, int vec, const PmkBatch *h, hipStream_t st);
extern "C" int pmk_wave_bytes(int vec);

namespace {

uint64_t now_ns() {
    return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                     std::chrono::steady_clock::now().time_since_epoch())
                                     .count());
}

struct HostItem {   // device work-list entry (layout fixed by the kernel)
    const uint32_t *prog;
    const uint8_t *in;
    uint8_t *out;
    uint64_t in_ld, out_ld, s;
    uint32_t ngroups, ntiles;
    uint32_t unit0, pad;
};
static_assert(sizeof(HostItem) == 64, "work-list entry layout");

constexpr int kClasses = 3;        // row-group sizes 4, 8, 16
constexpr int kPhases = 2;
constexpr uint64_t kAlign = 256;

int class_of(int rg) { return rg == 4 ? 0 : (rg == 8 ? 1 : 2); }
int rg_of(int cls) { return cls == 0 ? 4 : (cls == 1 ? 8 : 16); }

// First-fit allocator over the arena's byte range.
struct Arena {
    uint64_t size = 0, used = 0, high = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    void init(uint64_t n) {
        size = n;
        free_.clear();
        free_[0] = n;
    }
    bool alloc(uint64_t n, uint64_t *off) {
        n = (n + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const uint64_t rest = it->second - n, start = it->first + n;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used += n;
            high = std::max(high, used);
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = (n + kAlign - 1) / kAlign * kAlign;
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Req {
    uint64_t ticket = 0;
    pm_request r{};
    std::vector<uint32_t> ids;
    std::vector<const uint8_t *> helpers;
    Resolved main, helper;
    uint64_t out_off = 0, bytes = 0, out_ld = 0;
    uint32_t out_blocks = 0;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = PM_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    HostItem *h_items = nullptr;   // pinned staging of the work lists
    void *d_items = nullptr;
    BsItem *h_bs = nullptr;        // pinned staging of the bit-sliced item lists
    BsItem *d_bs = nullptr;
    uint32_t *d_counters = nullptr;
    std::vector<Req *> reqs;
    bool busy = false;
};

}  // namespace

struct pm_server {
    pm_server_cfg cfg{};
    uint8_t *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    uint32_t item_cap = 0;
    std::mutex mu;                    // pending, done, releases, stats
    std::condition_variable cv;
    std::deque<Req *> pending;
    std::deque<pm_completion> done;
    std::vector<std::pair<uint64_t, uint64_t>> releases;   // (offset, bytes)
    std::map<uint64_t, std::pair<uint64_t, uint64_t>> live;  // ticket -> arena (offset, bytes)
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread sched;
    uint64_t launch_ns = 0;           // host time in launch(), under mu
    int device = 0;
    // statistics
    uint64_t batches = 0, completed = 0, failed = 0, table_high = 0;
    uint64_t reserve = 0;             // budget part for kernel tables
    uint32_t max_busy = 0;
    int error = PM_OK;

    ~pm_server() {
        stop = true;
        cv.notify_all();
        if (sched.joinable()) sched.join();
        for (Slot &s : slots) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.h_items) (void)hipHostFree(s.h_items);
            if (s.d_items) (void)hipFree(s.d_items);
            if (s.h_bs) (void)hipHostFree(s.h_bs);
            if (s.d_bs) (void)hipFree(s.d_bs);
            if (s.d_counters) (void)hipFree(s.d_counters);
        }
        if (arena_base) (void)hipFree(arena_base);
        for (Req *r : pending) delete r;
        for (Slot &sl : slots)
            for (Req *r : sl.reqs) delete r;
    }

    // Reserve arena space for a request's result (and repair scratch).
    // Arena bytes of a request: its result blocks and, for a repair, the d
    // received blocks.
    static uint64_t request_bytes(const Req *q) {
        const uint64_t ld = (q->r.block_bytes + 15) / 16 * 16;
        const uint64_t scratch = q->r.op == PM_REQ_REPAIR ? q->main.in_n : 0;
        return (q->main.out_n + scratch) * ld;
    }

    bool admit(Req *q) {
        const uint64_t s = q->r.block_bytes;
        const uint64_t ld = (s + 15) / 16 * 16;
        const uint64_t out_blocks = q->main.out_n;
        q->bytes = request_bytes(q);
        if (!arena.alloc(q->bytes, &q->out_off)) return false;
        q->out_ld = ld;
        q->out_blocks = static_cast<uint32_t>(out_blocks);
        q->t_admit = now_ns();
        return true;
    }

    // Pack the slot's requests into per-phase, per-class work lists, upload
    // them and launch.  Everything that can fail on the host (resolving
    // device tables, list capacity) happens before anything is enqueued; if
    // an enqueue fails part way, the stream is drained before returning, so
    // no kernel of a failed micro-batch is still running when its requests
    // are completed with the error.
    int launch(Slot &sl) {
        std::vector<HostItem> lists[kPhases][kClasses];
        // items whose matrix has a compiled multi-set bit-sliced kernel, per
        // phase and matrix
        std::map<BsProgram *, std::pair<std::shared_ptr<BsProgram>, std::vector<BsItem>>> bs_lists[kPhases];
        // items on the matrix cores, per phase
        struct MfItem {
            std::shared_ptr<ProgEntry> pe;
            const uint8_t *in;
            uint64_t in_ld;
            uint8_t *out;
            uint64_t out_ld, s;
        };
        std::vector<MfItem> mf_lists[kPhases];
        const int vec = static_cast<int>(cfg.dwords_per_lane ? cfg.dwords_per_lane : 2);
        const uint64_t wave_bytes = static_cast<uint64_t>(pmk_wave_bytes(vec));
        auto add = [&](int phase, const Resolved &rs, const uint8_t *in, uint64_t in_ld, uint8_t *out,
                       uint64_t out_ld, uint64_t s) -> int {
            const Program &p = rs.pe->prog;
            if (p.ngroups == 0) return ST_OK;
            if (s >= kBsTileBytes && (rs.vec == kVecAuto || rs.vec == kVecBitslice))
                if (std::shared_ptr<BsProgram> bp = rs.pe->bitslice_if_compiled(BS_MULTI)) {
                    auto &e = bs_lists[phase][bp.get()];
                    e.first = bp;
                    e.second.push_back(bs_item(in, in_ld, out, out_ld, s, 0));
                    return ST_OK;
                }
            // dense matrices over the specialization limit: the matrix
            // cores, one launch per item in the phase
            if (rs.vec == kVecAuto && mf_span_ok(in_ld, s, rs.in_n) && rs.pe->mfma_eligible()) {
                const size_t need = rs.pe->mfma_upload_bytes();
                if (need && device_table_bytes() + need > reserve) {
                    trim_tables(reserve > need ? reserve - need : 0);
                    if (device_table_bytes() + need > reserve) return ST_ENOMEM;
                }
                const int st = rs.pe->stage_mfma();
                if (st != ST_OK) return st;
                mf_lists[phase].push_back(MfItem{rs.pe, in, in_ld, out, out_ld, s});
                return ST_OK;
            }
            // a table not yet on the device counts against the reserve
            const size_t need = rs.pe->upload_bytes();
            if (need && device_table_bytes() + need > reserve) {
                trim_tables(reserve > need ? reserve - need : 0);
                if (device_table_bytes() + need > reserve) return ST_ENOMEM;
            }
            const uint32_t *dprog = nullptr;
            const int st = rs.pe->device_ptr_sync(&dprog);
            if (st != ST_OK) return st;
            const uint64_t ntiles = (s + wave_bytes - 1) / wave_bytes;
            lists[phase][class_of(p.rg)].push_back(HostItem{dprog, in, out, in_ld, out_ld, s,
                                                            static_cast<uint32_t>(p.ngroups),
                                                            static_cast<uint32_t>(ntiles), 0, 0});
            return ST_OK;
        };
        for (Req *q : sl.reqs) {
            const pm_request &r = q->r;
            uint8_t *out = arena_base + q->out_off;
            const uint64_t s = r.block_bytes;
            int st = ST_OK;
            if (r.op == PM_REQ_REPAIR) {
                uint8_t *scratch = out + static_cast<uint64_t>(q->out_blocks) * q->out_ld;
                for (size_t j = 0; j < q->helpers.size() && st == ST_OK; ++j)
                    st = add(0, q->helper, q->helpers[j], r.node_ld, scratch + j * q->out_ld, q->out_ld, s);
                if (st == ST_OK) st = add(1, q->main, scratch, q->out_ld, out, q->out_ld, s);
            } else {
                st = add(0, q->main, r.in, r.in_ld, out, q->out_ld, s);
            }
            if (st != ST_OK) return st;   // nothing enqueued yet
        }
        // Number units and stage [phase][class] lists back to back.
        uint32_t pos = 0;
        uint32_t start[kPhases][kClasses], units[kPhases][kClasses];
        for (int ph = 0; ph < kPhases; ++ph)
            for (int c = 0; c < kClasses; ++c) {
                start[ph][c] = pos;
                uint64_t u = 0;
                for (HostItem &h : lists[ph][c]) {
                    h.unit0 = static_cast<uint32_t>(u);
                    u += static_cast<uint64_t>(h.ntiles) * h.ngroups;
                }
                units[ph][c] = static_cast<uint32_t>(u);
                if (pos + lists[ph][c].size() > item_cap) return ST_EINVAL;
                std::copy(lists[ph][c].begin(), lists[ph][c].end(), sl.h_items + pos);
                pos += static_cast<uint32_t>(lists[ph][c].size());
            }
        // Stage the bit-sliced lists back to back, tiles numbered per matrix.
        struct BsLaunch {
            BsProgram *bp;
            uint32_t start, n, ntiles;
        };
        std::vector<BsLaunch> bs_launches[kPhases];
        uint32_t bpos = 0;
        for (int ph = 0; ph < kPhases; ++ph)
            for (auto &kv : bs_lists[ph]) {
                std::vector<BsItem> &v = kv.second.second;
                if (bpos + v.size() > item_cap) return ST_EINVAL;
                uint64_t tile = 0;
                for (BsItem &it : v) {
                    it.tile0 = static_cast<uint32_t>(tile);
                    tile += it.ntiles;
                }
                if (tile > 0xffffff00ull) return ST_EINVAL;
                std::copy(v.begin(), v.end(), sl.h_bs + bpos);
                bs_launches[ph].push_back(BsLaunch{kv.first, bpos, static_cast<uint32_t>(v.size()),
                                                   static_cast<uint32_t>(tile)});
                bpos += static_cast<uint32_t>(v.size());
            }
        // from here on work is enqueued: a failure drains the stream first
        auto drain = [&](int st) {
            (void)hipStreamSynchronize(sl.stream);
            return st;
        };
        hipError_t e;
        if (pos && (e = hipMemcpyAsync(sl.d_items, sl.h_items, pos * sizeof(HostItem), hipMemcpyHostToDevice,
                                       sl.stream)) != hipSuccess)
            return drain(hip_fail(e));
        if (bpos && (e = hipMemcpyAsync(sl.d_bs, sl.h_bs, bpos * sizeof(BsItem), hipMemcpyHostToDevice,
                                        sl.stream)) != hipSuccess)
            return drain(hip_fail(e));
        for (int ph = 0; ph < kPhases; ++ph) {
            for (const BsLaunch &l : bs_launches[ph]) {
                int rc = bs_launch_items(*l.bp, sl.d_bs + l.start, l.n, l.ntiles, sl.stream);
                if (rc != ST_OK) return drain(rc);
            }
            for (const MfItem &m : mf_lists[ph]) {
                int rc = m.pe->launch_mfma(m.in, m.in_ld, m.out, m.out_ld, m.s, sl.stream);
                if (rc != ST_OK) return drain(rc);
            }
            for (int c = 0; c < kClasses; ++c) {
                if (!units[ph][c]) continue;
                PmkBatch h{static_cast<HostItem *>(sl.d_items) + start[ph][c],
                           static_cast<uint32_t>(lists[ph][c].size()), units[ph][c],
                           sl.d_counters + (ph * kClasses + c) * 8 * 16};
                if ((e = pmk_batch(rg_of(c), vec, &h, sl.stream)) != hipSuccess) return drain(hip_fail(e));
            }
        }
        if ((e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) return drain(hip_fail(e));
        const uint64_t tb = device_table_bytes();
        std::lock_guard<std::mutex> lk(mu);
        table_high = std::max(table_high, tb);
        return ST_OK;
    }

    // Hand a slot's requests to the client as completed with status st (or,
    // for st == PM_OK, with the status of the slot's event).
    void complete(Slot &sl, int st) {
        const uint64_t t = now_ns();
        std::lock_guard<std::mutex> lk(mu);
        for (Req *q : sl.reqs) {
            pm_completion c{};
            c.ticket = q->ticket;
            c.tag = q->r.tag;
            c.status = st;
            c.out = arena_base + q->out_off;
            c.out_ld = q->out_ld;
            c.out_blocks = q->out_blocks;
            c.t_submit_ns = q->t_submit;
            c.t_admit_ns = q->t_admit;
            c.t_done_ns = t;
            live[q->ticket] = {q->out_off, q->bytes};
            done.push_back(c);
            ++completed;
            if (st != PM_OK) ++failed;
            delete q;
        }
        sl.reqs.clear();
        sl.busy = false;
    }

    void run() {
        (void)hipSetDevice(device);
        int idle_spins = 0;
        while (!stop) {
            bool progressed = false;
            // 1. reap finished micro-batches
            for (Slot &sl : slots) {
                if (!sl.busy) continue;
                hipError_t e = hipEventQuery(sl.done);
                if (e == hipErrorNotReady) continue;
                complete(sl, e == hipSuccess ? PM_OK : PM_EHIP);
                progressed = true;
            }
            // 2. releases and admission
            std::vector<Req *> admitted;
            Slot *free_slot = nullptr;
            for (Slot &sl : slots)
                if (!sl.busy) { free_slot = &sl; break; }
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto &rel : releases) arena.release(rel.first, rel.second);
                if (!releases.empty()) progressed = true;
                releases.clear();
                if (free_slot) {
                    uint32_t items = 0;
                    uint64_t batch_bytes = 0;
                    while (!pending.empty() && admitted.size() < cfg.max_batch) {
                        Req *q = pending.front();
                        const uint32_t need = q->r.op == PM_REQ_REPAIR ? static_cast<uint32_t>(q->helpers.size()) + 1 : 1;
                        if (items + need > item_cap) break;
                        if (cfg.max_batch_bytes && !admitted.empty() &&
                            batch_bytes + request_bytes(q) > cfg.max_batch_bytes)
                            break;
                        if (!admit(q)) break;   // arrival order: wait for memory
                        items += need;
                        batch_bytes += q->bytes;
                        pending.pop_front();
                        admitted.push_back(q);
                    }
                }
            }
            if (!admitted.empty()) {
                free_slot->reqs = std::move(admitted);
                const uint64_t t0 = now_ns();
                const int st = launch(*free_slot);
                const uint64_t dt = now_ns() - t0;
                if (st != ST_OK) {
                    // nothing of this micro-batch is on the GPU any more: its
                    // requests complete now, with the error
                    complete(*free_slot, st);
                    if (st == ST_EHIP) {   // the stream may be unusable
                        std::lock_guard<std::mutex> lk(mu);
                        error = st;
                    }
                } else {
                    free_slot->busy = true;
                }
                uint32_t now_busy = 0;
                for (const Slot &sl : slots) now_busy += sl.busy ? 1u : 0u;
                std::lock_guard<std::mutex> lk(mu);
                launch_ns += dt;
                ++batches;
                max_busy = std::max(max_busy, now_busy);
                progressed = true;
            }
            if (progressed) {
                idle_spins = 0;
            } else if (++idle_spins > 2000) {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait_for(lk, std::chrono::microseconds(200));
                idle_spins = 0;
            } else {
                std::this_thread::yield();
            }
        }
    }
};

extern "C" {

pm_status pm_server_create(const pm_server_cfg *cfg, pm_server **out) {
    if (!cfg || !out || cfg->hbm_budget_bytes < kAlign || cfg->streams == 0 || cfg->streams > 16 ||
        cfg->max_batch == 0 || cfg->queue_cap == 0)
        return PM_EINVAL;
    if (cfg->dwords_per_lane && cfg->dwords_per_lane != 2 && cfg->dwords_per_lane != 4) return PM_EINVAL;
    *out = nullptr;
    std::unique_ptr<pm_server> s(new pm_server());
    s->cfg = *cfg;
    hipError_t e;
    s->reserve = cfg->table_reserve_bytes ? cfg->table_reserve_bytes
                                          : std::max<uint64_t>(cfg->hbm_budget_bytes / 32, uint64_t(16) << 20);
    if (s->reserve + kAlign > cfg->hbm_budget_bytes) return PM_EINVAL;
    const uint64_t arena_bytes = (cfg->hbm_budget_bytes - s->reserve) / kAlign * kAlign;
    if ((e = hipGetDevice(&s->device)) != hipSuccess) return static_cast<pm_status>(hip_fail(e));
    if ((e = hipMalloc(reinterpret_cast<void **>(&s->arena_base), arena_bytes)) != hipSuccess) {
        s->arena_base = nullptr;
        return e == hipErrorOutOfMemory ? PM_ENOMEM : static_cast<pm_status>(hip_fail(e));
    }
    s->arena.init(arena_bytes);
    s->item_cap = cfg->max_batch * 32u + 64u;
    s->slots.resize(cfg->streams);
    for (Slot &sl : s->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_items), s->item_cap * sizeof(HostItem), 0)) !=
                hipSuccess ||
            (e = hipMalloc(&sl.d_items, s->item_cap * sizeof(HostItem))) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void **>(&sl.h_bs), s->item_cap * sizeof(BsItem), 0)) !=
                hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void **>(&sl.d_bs), s->item_cap * sizeof(BsItem))) != hipSuccess ||
            (e = hipMalloc(reinterpret_cast<void **>(&sl.d_counters),
                           kPhases * kClasses * 8 * 16 * sizeof(uint32_t))) != hipSuccess ||
            // the work-list kernels leave their counters at zero: only the first launch needs this
            (e = hipMemset(sl.d_counters, 0, kPhases * kClasses * 8 * 16 * sizeof(uint32_t))) != hipSuccess)
            return static_cast<pm_status>(hip_fail(e));
    }
    pm_server *raw = s.get();
    s->sched = std::thread([raw] { raw->run(); });
    *out = s.release();
    return PM_OK;
}

pm_status pm_server_submit(pm_server *s, const pm_request *req, uint64_t *ticket) {
    if (!s || !req || !req->code || req->block_bytes == 0) return PM_EINVAL;
    std::unique_ptr<Req> q(new Req());
    q->r = *req;
    int st;
    switch (req->op) {
        case PM_REQ_ENCODE:
            st = resolve_op(const_cast<pm_code *>(req->code), OPK_ENCODE, 0, nullptr, &q->main);
            break;
        case PM_REQ_DECODE:
            st = resolve_op(const_cast<pm_code *>(req->code), OPK_DECODE, 0, req->ids, &q->main);
            break;
        case PM_REQ_REPAIR:
            if (!req->helper_nodes) return PM_EINVAL;
            st = resolve_op(const_cast<pm_code *>(req->code), OPK_NEWCOMER, req->failed, req->ids, &q->main);
            if (st == ST_OK) st = resolve_op(const_cast<pm_code *>(req->code), OPK_HELPER, req->failed, nullptr,
                                             &q->helper);
            if (st == ST_OK) {
                q->helpers.assign(req->helper_nodes, req->helper_nodes + q->main.in_n);
                for (const uint8_t *h : q->helpers)
                    if ((st = check_regions(h, req->node_ld, q->helper.in_n, req->block_bytes)) != ST_OK) break;
            }
            break;
        default:
            return PM_EINVAL;
    }
    if (st != ST_OK) return static_cast<pm_status>(st);
    if (req->op != PM_REQ_REPAIR &&
        (st = check_regions(req->in, req->in_ld, q->main.in_n, req->block_bytes)) != ST_OK)
        return static_cast<pm_status>(st);
    q->r.ids = nullptr;
    q->r.helper_nodes = nullptr;
    q->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->error != PM_OK) return static_cast<pm_status>(s->error);
        if (s->pending.size() >= s->cfg.queue_cap) return PM_EBUSY;
        const uint64_t ld = (req->block_bytes + 15) / 16 * 16;
        const uint64_t need = (q->main.out_n + (req->op == PM_REQ_REPAIR ? q->main.in_n : 0)) * ld;
        if ((need + kAlign - 1) / kAlign * kAlign > s->arena.size) return PM_ENOMEM;
        q->ticket = s->next_ticket++;
        if (ticket) *ticket = q->ticket;
        s->pending.push_back(q.release());
    }
    s->cv.notify_one();
    return PM_OK;
}

pm_status pm_server_poll(pm_server *s, pm_completion *out, size_t cap, size_t *n_done) {
    if (!s || (!out && cap) || !n_done) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    size_t n = 0;
    while (n < cap && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_done = n;
    return static_cast<pm_status>(s->error);
}

pm_status pm_server_release(pm_server *s, uint64_t ticket) {
    if (!s) return PM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->live.find(ticket);
        if (it == s->live.end()) return PM_EINVAL;
        s->releases.push_back(it->second);
        s->live.erase(it);
    }
    s->cv.notify_one();
    return PM_OK;
}

pm_status pm_server_stats(pm_server *s, pm_server_stat *st) {
    if (!s || !st) return PM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    // releases not yet taken by the scheduler count as done (the arena is
    // only touched under this lock)
    for (auto &rel : s->releases) s->arena.release(rel.first, rel.second);
    s->releases.clear();
    st->completed = s->completed;
    st->batches = s->batches;
    st->pending = s->pending.size();
    st->arena_used = s->arena.used;
    st->arena_high_water = s->arena.high;
    st->max_concurrent_batches = s->max_busy;
    st->pad = 0;
    st->failed = s->failed;
    st->arena_bytes = s->arena.size;
    st->table_reserve_bytes = s->reserve;
    st->table_bytes_high = s->table_high;
    st->launch_host_ns = s->launch_ns;
    return static_cast<pm_status>(s->error);
}

pm_status pm_server_replay(pm_server *s, const pm_request *reqs, const uint64_t *arrival_ns, size_t n,
                           uint32_t flags, pm_completion *out) {
    if (!s || (!reqs && n) || (!arrival_ns && n) || (!out && n)) return PM_EINVAL;
    std::vector<uint64_t> ticket_of(n, 0);
    std::map<uint64_t, size_t> index_of;
    std::vector<pm_completion> buf(256);
    size_t next = 0, finished = 0;
    const uint64_t t0 = now_ns();
    auto drain = [&]() -> int {
        size_t got = 0;
        pm_status st = pm_server_poll(s, buf.data(), buf.size(), &got);
        if (st != PM_OK) return st;
        for (size_t i = 0; i < got; ++i) {
            auto it = index_of.find(buf[i].ticket);
            if (it == index_of.end()) continue;
            out[it->second] = buf[i];
            index_of.erase(it);
            ++finished;
            if (!(flags & PM_REPLAY_KEEP)) pm_server_release(s, buf[i].ticket);
        }
        return PM_OK;
    };
    while (finished < n) {
        const uint64_t t = now_ns() - t0;
        if (next < n && t >= arrival_ns[next]) {
            uint64_t ticket = 0;
            pm_status st = pm_server_submit(s, &reqs[next], &ticket);
            if (st == PM_OK) {
                ticket_of[next] = ticket;
                index_of[ticket] = next;
                ++next;
                continue;
            }
            if (st != PM_EBUSY) return st;
        }
        int st = drain();
        if (st != PM_OK) return static_cast<pm_status>(st);
        if (next < n && now_ns() - t0 < arrival_ns[next]) std::this_thread::yield();
    }
    return PM_OK;
}

void pm_server_destroy(pm_server *s) { delete s; }

}  // extern "C"
