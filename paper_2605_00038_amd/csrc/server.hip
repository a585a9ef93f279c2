// Serving loop of the C ABI (lbp_server_*): per-shot streaming decode of
// request queues for several codes on one device.
//
// Each code slot owns a ring of R items in pinned, coherent host memory
// (syndrome + lottery key in; correction, flags and iterations out, plus a
// completion queue of finished items) and a persistent BP grid that claims published items one shot per
// wave.  A shot's result is visible as soon as that shot has finished: there
// are no batch boundaries, so a converging shot never waits behind a slow one.
// Shots whose BP run fails leave their lambda in device memory and are marked
// OSD-pending; the worker gathers them and launches OSD on the CUs the BP
// grid leaves free.  The BP grid exits after a short idle period (and on
// destroy); the worker relaunches it when new items are published.
//
// One worker thread per server moves requests from the slot queues into the
// rings (first come first served, at most R items in flight), reads the
// completion queue, starts OSD launches and completes requests.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lbp.h"
#include "lbp_internal.h"
#include "serve_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kMaxRing = 65536;        // items in flight per slot (upper bound, power of two)
constexpr int64_t kMinRing = 1024;
constexpr int64_t kQueueFactor = 16;       // admission: queued shots per slot <= kQueueFactor * R
constexpr int64_t kOsdList = 4096;         // failed shots per OSD launch
constexpr uint64_t kIdleTicks = 200000;    // the BP grid exits after 2 ms without a claim (100 MHz clock)
// Batched claims: every claim is one CAS on the ring's head, a device-wide
// round trip that capped a slot at ~6e5 items/s.  A wave takes up to kClaimMax
// items at once, one more per two full rounds of the grid's claimers waiting
// beyond its claim (below that backlog every claim is one item).  LBP_SERVE_CLAIM_MAX / LBP_SERVE_CLAIM_BACKLOG
// (read at lbp_server_add_code) override the two, for tests.
constexpr uint32_t kClaimMax = 8;

uint32_t env_u32(const char *name, uint32_t dflt, uint32_t lo, uint32_t hi) {
    const char *e = std::getenv(name);
    if (!e) return dflt;
    const long v = std::atol(e);
    return v < (long)lo ? lo : (v > (long)hi ? hi : (uint32_t)v);
}
// With several code slots the grids share the GPU's few hardware queues: a grid
// that waits out 2 ms of idleness holds its queue, and every launch of another
// slot's stream behind it on that queue, so grids of a shared server exit after
// 20 us without a claim and the worker relaunches them when items arrive.
constexpr uint64_t kIdleTicksShared = 2000;
constexpr double kOsdFraction = 0.375;     // CUs left to OSD launches
constexpr int64_t kDefaultBudget = (int64_t)16 << 30;
constexpr auto kQueryGap = std::chrono::microseconds(20);

lbp_status sfail(lbp_status s, const std::string &m) {
    lbp::set_error(m.c_str());
    return s;
}

struct Request {
    uint64_t ticket = 0;
    int slot = 0;
    int64_t n = 0;
    uint64_t seed = 0, first_id = 0;
    std::vector<uint32_t> syn;
    std::vector<uint32_t> corr;
    std::vector<uint8_t> flags;
    std::vector<int32_t> iters;
    int64_t dispatched = 0;   // shots placed in the ring
    int64_t outstanding = 0;  // shots in the ring not yet complete
    bool cancelled = false;
    bool done = false;
    lbp_status status = LBP_OK;
    std::string err;
    Clock::time_point t_submit, t_done;
};
using ReqPtr = std::shared_ptr<Request>;

// Requests by ticket.  Tickets are handed out in submission order (under the
// inbox lock) and enter the table in that order, so the live tickets form a
// window [base, base + q.size()) over a deque: insert, find and erase are O(1)
// and the table never rehashes (a hash map's rehash of ~10^5 requests stalled
// the worker, which holds the server lock while it publishes and completes
// shots, for milliseconds).  Erased or never-entered tickets are null entries;
// the window's front advances past them.
struct TicketTable {
    uint64_t base = 0;
    std::deque<ReqPtr> q;
    void put(uint64_t t, ReqPtr r) {
        if (q.empty()) base = t;
        if (t < base) return;  // tickets enter in order: not reached
        while (base + q.size() <= t) q.emplace_back();
        q[(size_t)(t - base)] = std::move(r);
    }
    ReqPtr find(uint64_t t) const { return t >= base && t - base < q.size() ? q[(size_t)(t - base)] : nullptr; }
    void erase(uint64_t t) {
        if (t >= base && t - base < q.size()) q[(size_t)(t - base)].reset();
        while (!q.empty() && !q.front()) {
            q.pop_front();
            ++base;
        }
    }
};

enum : uint8_t { S_FREE = 0, S_BP = 1, S_OSD_WAIT = 2, S_OSD_RUN = 3, S_DONE = 4 };

// What submit needs of a slot without taking the server lock.
struct SlotInfo {
    int mw = 0, nw = 0;
    int64_t R = 0;
    std::atomic<int64_t> queued{0};  // shots submitted and not yet in the ring
};

struct Slot {
    lbp_code code = nullptr;
    lbp_decoder dec = nullptr;
    int mw = 0, nw = 0, n = 0;
    int64_t R = 0;
    lbp::ServeShape shape{};
    // host rings (pinned, coherent)
    uint32_t *h_syn = nullptr;
    uint64_t *h_keys = nullptr, *h_tail = nullptr, *h_cq = nullptr;
    uint32_t *h_stop = nullptr, *h_corr = nullptr, *h_ocount = nullptr;
    uint8_t *h_flags = nullptr;
    int32_t *h_iters = nullptr, *h_list = nullptr;
    // device
    lbp::ServeRing ring{};
    lbp::ServeRing *d_ring = nullptr;
    unsigned long long *d_ctl = nullptr;  // head, tail, token, last claim, completion-queue tail, exiting
    float *d_llr = nullptr;      // staged lambda of OSD-pending items: llr_bytes per ring item
    int64_t llr_bytes = 0;
    int32_t *d_list = nullptr;
    uint32_t *d_ocount = nullptr;
    hipStream_t s_bp = nullptr, s_osd = nullptr;
    hipEvent_t e_bp = nullptr, e_osd = nullptr;
    bool bp_running = false, osd_running = false;
    Clock::time_point next_query{};  // event queries are runtime calls: at most one round per kQueryGap
    // item bookkeeping
    uint64_t published = 0, done_upto = 0;
    std::vector<ReqPtr> ref_req;  // request of each occupied ring slot (keeps it alive)
    std::vector<int64_t> ref_off;
    std::vector<uint8_t> state;
    std::vector<uint64_t> osd_wait, osd_run;
    uint64_t cq_head = 0;  // next completion-queue position to read
    uint64_t bp_done = 0;  // items through BP (published - bp_done are still in BP)
    std::deque<ReqPtr> queue;
    SlotInfo *info = nullptr;
    int64_t dev_bytes = 0;
    // statistics
    int64_t bp_launches = 0, shots = 0, max_inflight = 0, osd_launches = 0;
};

}  // namespace

struct lbp_server_s {
    int device = 0;
    int64_t budget = 0, used = 0;
    int max_slots = 0;
    // mu: slots, tickets and request progress (worker, poll, wait, cancel)
    std::mutex mu;
    std::vector<std::unique_ptr<Slot>> slots;
    TicketTable tickets;
    std::condition_variable cv_done;
    std::string dead_msg;
    // in_mu: the inbox of submitted requests and the worker's sleep (lock order: mu, then in_mu)
    std::mutex in_mu;
    std::vector<ReqPtr> inbox;
    std::atomic<int64_t> inbox_n{0};  // inbox.size(), readable without in_mu
    std::condition_variable cv_work;
    bool idle = false, stop = false;
    std::atomic<bool> stop_seen{false};  // stop, readable without in_mu
    // lock-free
    SlotInfo info[64];
    std::atomic<int> n_slots{0};
    std::atomic<uint64_t> next_ticket{1};
    std::atomic<int> dead{LBP_OK};  // a device error stops the server
    std::thread worker;
};

namespace {

void free_slot(Slot &sl) {
    if (sl.h_stop) __atomic_store_n(sl.h_stop, 1u, __ATOMIC_RELEASE);
    if (sl.s_bp) (void)hipStreamSynchronize(sl.s_bp);
    if (sl.s_osd) (void)hipStreamSynchronize(sl.s_osd);
    if (sl.dec) lbp_decoder_destroy(sl.dec);
    for (void *p : {(void *)sl.h_syn, (void *)sl.h_keys, (void *)sl.h_tail, (void *)sl.h_cq, (void *)sl.h_stop,
                    (void *)sl.h_corr, (void *)sl.h_ocount, (void *)sl.h_flags, (void *)sl.h_iters, (void *)sl.h_list})
        if (p) (void)hipHostFree(p);
    for (void *p : {(void *)sl.d_ring, (void *)sl.d_ctl, (void *)sl.d_llr, (void *)sl.d_list, (void *)sl.d_ocount})
        if (p) (void)hipFree(p);
    if (sl.e_bp) (void)hipEventDestroy(sl.e_bp);
    if (sl.e_osd) (void)hipEventDestroy(sl.e_osd);
    if (sl.s_bp) (void)hipStreamDestroy(sl.s_bp);
    if (sl.s_osd) (void)hipStreamDestroy(sl.s_osd);
}

// CU masks of a slot's streams: OSD launches get 12 of every 32 CUs (the OSD
// fraction), BP grids the other 20, so a long OSD launch (large codes) never
// holds the CUs a BP grid needs.  The pattern is taken modulo 32, so every XCD
// keeps CUs of both kinds whether the mask bits run along or across XCDs.
void cu_masks(int ncu, std::vector<uint32_t> &bp, std::vector<uint32_t> &osd) {
    const int words = (ncu + 31) / 32;
    bp.assign((size_t)words, 0u);
    osd.assign((size_t)words, 0u);
    const int osd_per32 = (int)(32 * kOsdFraction + 0.5);
    for (int i = 0; i < ncu; ++i) {
        if (i % 32 < osd_per32) osd[(size_t)(i / 32)] |= 1u << (i % 32);
        else bp[(size_t)(i / 32)] |= 1u << (i % 32);
    }
}

// Allocate the rings and device state of a slot with R items.
lbp_status setup_slot(Slot &sl, int64_t R) {
    sl.R = R;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    const unsigned hf = hipHostMallocCoherent | hipHostMallocMapped;
    chk(hipHostMalloc((void **)&sl.h_syn, (size_t)R * sl.mw * 4, hf));
    chk(hipHostMalloc((void **)&sl.h_keys, (size_t)R * 16, hf));
    chk(hipHostMalloc((void **)&sl.h_tail, 64, hf));
    chk(hipHostMalloc((void **)&sl.h_stop, 64, hf));
    chk(hipHostMalloc((void **)&sl.h_corr, (size_t)R * sl.nw * 4, hf));
    chk(hipHostMalloc((void **)&sl.h_flags, (size_t)R, hf));
    chk(hipHostMalloc((void **)&sl.h_iters, (size_t)R * 4, hf));
    chk(hipHostMalloc((void **)&sl.h_cq, (size_t)R * 8, hf));
    chk(hipHostMalloc((void **)&sl.h_list, (size_t)kOsdList * 4, hipHostMallocDefault));
    chk(hipHostMalloc((void **)&sl.h_ocount, 64, hipHostMallocDefault));
    chk(hipMalloc((void **)&sl.d_ring, sizeof(lbp::ServeRing)));
    chk(hipMalloc((void **)&sl.d_ctl, 64));
    chk(hipMalloc((void **)&sl.d_llr, (size_t)R * sl.llr_bytes));
    chk(hipMalloc((void **)&sl.d_list, (size_t)kOsdList * 4));
    chk(hipMalloc((void **)&sl.d_ocount, 64));
    int ncu = 0, dev = 0;
    chk(hipGetDevice(&dev));
    chk(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (e == hipSuccess && ncu >= 32) {
        std::vector<uint32_t> mbp, mosd;
        cu_masks(ncu, mbp, mosd);
        chk(hipExtStreamCreateWithCUMask(&sl.s_bp, (uint32_t)mbp.size(), mbp.data()));
        chk(hipExtStreamCreateWithCUMask(&sl.s_osd, (uint32_t)mosd.size(), mosd.data()));
    } else {
        chk(hipStreamCreateWithFlags(&sl.s_bp, hipStreamNonBlocking));
        chk(hipStreamCreateWithFlags(&sl.s_osd, hipStreamNonBlocking));
    }
    chk(hipEventCreateWithFlags(&sl.e_bp, hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&sl.e_osd, hipEventDisableTiming));
    if (e != hipSuccess)
        return sfail(e == hipErrorOutOfMemory ? LBP_ENOMEM : LBP_EDEVICE,
                     std::string("lbp_server_add_code: ") + hipGetErrorString(e));
    std::memset(sl.h_cq, 0, (size_t)R * 8);  // lap field 0: no entry yet
    *sl.h_tail = 0;
    *sl.h_stop = 0;
    std::memset(sl.h_ocount, 0, 64);
    unsigned long long zero[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    chk(hipMemcpy(sl.d_ctl, zero, 64, hipMemcpyHostToDevice));
    chk(hipMemcpy(sl.d_ocount, zero, 64, hipMemcpyHostToDevice));
    lbp::ServeRing &r = sl.ring;
    r.syn = sl.h_syn;
    r.keys = sl.h_keys;
    r.host_tail = sl.h_tail;
    r.host_stop = sl.h_stop;
    r.corr = sl.h_corr;
    r.flags = sl.h_flags;
    r.iters = sl.h_iters;
    r.cq = sl.h_cq;
    r.cq_tail = sl.d_ctl + 4;
    r.head = sl.d_ctl;
    r.tail = sl.d_ctl + 1;
    r.token = (uint32_t *)(sl.d_ctl + 2);
    r.last_claim = sl.d_ctl + 3;
    r.exiting = (uint32_t *)(sl.d_ctl + 5);
    r.llr = sl.d_llr;
    r.llr16 = (int16_t *)sl.d_llr;
    r.mask = R - 1;
    r.idle_ticks = kIdleTicks;
    // one more item per claim for every two full rounds of the grid's claimers
    // waiting beyond it: a wave (or a workgroup that decodes one shot) takes
    // several items only when every claimer has work anyway (the host publishes
    // in bursts, so one round would split bursts that idle claimers could take)
    int32_t wpb = 1, blocks = 1, group = 1;
    (void)lbp_decoder_shape(sl.dec, &wpb, &blocks, &group, nullptr, nullptr, nullptr);
    const uint32_t claimers = (uint32_t)std::max(1, 2 * sl.shape.bp_blocks * (group > 1 ? 1 : wpb));
    r.claim_max = env_u32("LBP_SERVE_CLAIM_MAX", kClaimMax, 1, 64);
    r.claim_backlog = env_u32("LBP_SERVE_CLAIM_BACKLOG", claimers, 1, 1u << 20);
    chk(hipMemcpy(sl.d_ring, &r, sizeof(r), hipMemcpyHostToDevice));
    if (e != hipSuccess) return sfail(LBP_EDEVICE, std::string("lbp_server_add_code: ") + hipGetErrorString(e));
    sl.ref_req.assign((size_t)R, ReqPtr());
    sl.ref_off.assign((size_t)R, 0);
    sl.state.assign((size_t)R, S_FREE);
    sl.dev_bytes = (int64_t)R * sl.llr_bytes + lbp_decoder_device_bytes(sl.dec) + 4096;
    return LBP_OK;
}

void finish_request(lbp_server srv, Request &r, Clock::time_point now) {
    r.done = true;
    r.t_done = now;
    if (r.cancelled) srv->tickets.erase(r.ticket);
}

// One shot finished (lock held): copy its outputs and release its ring slot.
void complete_item(lbp_server srv, Slot &sl, uint64_t item, Clock::time_point now) {
    const int64_t k = (int64_t)(item & (uint64_t)(sl.R - 1));
    Request *r = sl.ref_req[k].get();
    const int64_t off = sl.ref_off[k];
    if (!r->cancelled) {
        std::memcpy(r->corr.data() + off * sl.nw, sl.h_corr + k * sl.nw, (size_t)sl.nw * 4);
        r->flags[off] = sl.h_flags[k];
        r->iters[off] = sl.h_iters[k];
    }
    sl.state[k] = S_DONE;
    sl.shots += 1;
    if (--r->outstanding == 0 && (r->dispatched == r->n || r->cancelled)) finish_request(srv, *r, now);
    sl.ref_req[k].reset();
}

// Move queued shots into the ring (lock held).  Returns true if any moved.
bool publish(Slot &sl) {
    const uint64_t start = sl.published;
    while (!sl.queue.empty() && (int64_t)(sl.published - sl.done_upto) < sl.R) {
        ReqPtr r = sl.queue.front();
        if (r->cancelled) {
            sl.queue.pop_front();  // its undispatched shots left the count when it was cancelled
            continue;
        }
        while (r->dispatched < r->n && (int64_t)(sl.published - sl.done_upto) < sl.R) {
            const uint64_t item = sl.published++;
            const int64_t k = (int64_t)(item & (uint64_t)(sl.R - 1));
            const int64_t off = r->dispatched++;
            std::memcpy(sl.h_syn + k * sl.mw, r->syn.data() + off * sl.mw, (size_t)sl.mw * 4);
            sl.h_keys[2 * k] = r->seed;
            sl.h_keys[2 * k + 1] = r->first_id + (uint64_t)off;
            sl.ref_req[k] = r;
            sl.ref_off[k] = off;
            sl.state[k] = S_BP;
            r->outstanding += 1;
            sl.info->queued.fetch_sub(1, std::memory_order_relaxed);
        }
        if (r->dispatched == r->n) sl.queue.pop_front();
    }
    if (sl.published == start) return false;
    __atomic_store_n(sl.h_tail, sl.published, __ATOMIC_RELEASE);
    sl.max_inflight = std::max<int64_t>(sl.max_inflight, (int64_t)(sl.published - sl.done_upto));
    return true;
}

// Advance the reuse bound past finished items.
void retire(Slot &sl) {
    while (sl.done_upto < sl.published && sl.state[sl.done_upto & (uint64_t)(sl.R - 1)] == S_DONE) {
        sl.state[sl.done_upto & (uint64_t)(sl.R - 1)] = S_FREE;
        ++sl.done_upto;
    }
}

// One pass over a slot (lock held).  Returns true if anything progressed.
bool service(lbp_server srv, Slot &sl, bool &busy) {
    bool progressed = publish(sl);
    const auto now = Clock::now();
    // BP results, in completion-queue order
    const uint64_t item_mask = (1ull << lbp::CQ_ITEM_BITS) - 1;
    for (;;) {
        const int64_t q = (int64_t)(sl.cq_head & (uint64_t)(sl.R - 1));
        const uint64_t e = __atomic_load_n(sl.h_cq + q, __ATOMIC_ACQUIRE);
        if ((e >> lbp::CQ_ITEM_BITS) != (lbp::cq_entry(sl.cq_head, 0, sl.R - 1) >> lbp::CQ_ITEM_BITS)) break;
        // the item in flight whose low bits the entry carries
        const uint64_t item = sl.done_upto + (((e & item_mask) - sl.done_upto) & item_mask);
        const int64_t k = (int64_t)(item & (uint64_t)(sl.R - 1));
        if (item >= sl.published || sl.state[k] != S_BP || !sl.ref_req[k]) {
            srv->dead_msg = "server: completion queue names item " + std::to_string(item) + " (in flight: " +
                            std::to_string(sl.done_upto) + ".." + std::to_string(sl.published) + ")";
            srv->dead = LBP_EDEVICE;
            return true;
        }
        ++sl.cq_head;
        ++sl.bp_done;
        progressed = true;
        if (sl.h_flags[k] & lbp::FLAG_OSD_PENDING) {
            sl.state[k] = S_OSD_WAIT;
            sl.osd_wait.push_back(item);
        } else {
            complete_item(srv, sl, item, now);
        }
    }
    const bool query = now >= sl.next_query;
    if (query) sl.next_query = now + kQueryGap;
    // OSD launches
    if (query && sl.osd_running && hipEventQuery(sl.e_osd) == hipSuccess) {
        sl.osd_running = false;
        for (uint64_t item : sl.osd_run) complete_item(srv, sl, item, now);
        sl.osd_run.clear();
        progressed = true;
    }
    if (!sl.osd_running && !sl.osd_wait.empty()) {
        const size_t cnt = std::min<size_t>(sl.osd_wait.size(), (size_t)kOsdList);
        for (size_t q = 0; q < cnt; ++q) {
            const uint64_t item = sl.osd_wait[q];
            sl.h_list[q] = (int32_t)(item & (uint64_t)(sl.R - 1));
            sl.state[sl.h_list[q]] = S_OSD_RUN;
            sl.osd_run.push_back(item);
        }
        sl.osd_wait.erase(sl.osd_wait.begin(), sl.osd_wait.begin() + (long)cnt);
        sl.h_ocount[1] = (uint32_t)cnt;
        hipError_t e = hipMemcpyAsync(sl.d_list, sl.h_list, cnt * 4, hipMemcpyHostToDevice, sl.s_osd);
        if (e == hipSuccess) e = hipMemcpyAsync(sl.d_ocount, sl.h_ocount, 8, hipMemcpyHostToDevice, sl.s_osd);
        lbp_status st = e == hipSuccess ? lbp::serve_launch_osd(sl.dec, sl.ring, sl.d_list, sl.d_ocount,
                                                                sl.shape.osd_blocks, sl.s_osd)
                                        : LBP_EDEVICE;
        if (st == LBP_OK && hipEventRecord(sl.e_osd, sl.s_osd) == hipSuccess) {
            sl.osd_running = true;
            sl.osd_launches += 1;
        } else {
            srv->dead_msg = std::string("server: OSD launch failed: ") + lbp_last_error();
            srv->dead = LBP_EDEVICE;
        }
        progressed = true;
    }
    // keep a BP grid running while items wait for it
    if (query && sl.bp_running && hipEventQuery(sl.e_bp) == hipSuccess) sl.bp_running = false;
    const bool bp_waiting = sl.bp_done < sl.published;
    if (!sl.bp_running && bp_waiting && srv->dead.load() == LBP_OK) {
        // Persistent grids of several code slots share the BP CUs: a grid sized for
        // all of them would keep the other slots' grids from becoming resident
        // while its ring stays busy, and their requests would wait for it to idle out.
        const int nslots = (int)srv->slots.size();
        const int blocks = std::max(1, sl.shape.bp_blocks / std::max(1, nslots));
        lbp_status st = lbp::serve_launch_bp(sl.dec, sl.d_ring, sl.ring.exiting, blocks, sl.s_bp);
        if (st == LBP_OK && hipEventRecord(sl.e_bp, sl.s_bp) == hipSuccess) {
            sl.bp_running = true;
            sl.bp_launches += 1;
        } else {
            srv->dead_msg = std::string("server: BP launch failed: ") + lbp_last_error();
            srv->dead = LBP_EDEVICE;
        }
        progressed = true;
    }
    retire(sl);
    busy = busy || bp_waiting || sl.osd_running || !sl.osd_wait.empty() || !sl.queue.empty();
    return progressed;
}

// A device error ends every pending request with that error (mu held).
void fail_all(lbp_server srv) {
    const auto now = Clock::now();
    std::vector<ReqPtr> in;
    {
        std::lock_guard<std::mutex> il(srv->in_mu);
        in.swap(srv->inbox);
        srv->inbox_n.store(0);
    }
    for (auto &r : in) srv->tickets.put(r->ticket, r);
    for (auto &p : srv->tickets.q) {
        if (!p || p->done) continue;
        Request &r = *p;
        r.status = (lbp_status)srv->dead.load();
        r.err = srv->dead_msg;
        r.done = true;
        r.t_done = now;
    }
    for (auto &sp : srv->slots) {
        sp->queue.clear();
        sp->info->queued.store(0);
    }
}

// Move submitted requests into the ticket table and slot queues (mu held).
// Returns false when the server is stopping.
bool drain_inbox(lbp_server srv) {
    std::vector<ReqPtr> in;
    if (srv->inbox_n.load(std::memory_order_acquire) > 0 || srv->stop_seen.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> il(srv->in_mu);
        if (srv->stop) return false;
        in.swap(srv->inbox);
        srv->inbox_n.store(0, std::memory_order_relaxed);
    }
    for (auto &r : in) {
        srv->tickets.put(r->ticket, r);
        srv->slots[r->slot]->queue.push_back(r);
    }
    return true;
}

void worker_main(lbp_server srv) {
    (void)hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    while (drain_inbox(srv)) {
        bool busy = false, progressed = false;
        for (auto &sp : srv->slots) progressed |= service(srv, *sp, busy);
        if (srv->dead.load() != LBP_OK) {
            fail_all(srv);
            srv->cv_done.notify_all();
            lk.unlock();
            std::unique_lock<std::mutex> il(srv->in_mu);
            srv->cv_work.wait(il, [&] { return srv->stop; });
            return;
        }
        if (progressed) srv->cv_done.notify_all();
        lk.unlock();
        if (progressed || busy) {  // let pollers in between passes
            if (!progressed)
                for (int k = 0; k < 64; ++k) __builtin_ia32_pause();
        } else {
            std::unique_lock<std::mutex> il(srv->in_mu);
            srv->idle = true;
            srv->cv_work.wait(il, [&] { return srv->stop || !srv->inbox.empty(); });
            srv->idle = false;
        }
        lk.lock();
    }
}

lbp_status copy_out(const Request &r, uint32_t *corrections, uint8_t *flags, int32_t *iters) {
    if (r.status != LBP_OK) return sfail(r.status, r.err);
    if (corrections) std::memcpy(corrections, r.corr.data(), r.corr.size() * 4);
    if (flags) std::memcpy(flags, r.flags.data(), r.flags.size());
    if (iters) std::memcpy(iters, r.iters.data(), r.iters.size() * 4);
    return LBP_OK;
}

}  // namespace

extern "C" {

lbp_status lbp_server_create(int64_t device_mem_budget_bytes, int32_t max_slots, lbp_server *out) {
    lbp::set_error("");
    if (!out) return sfail(LBP_EINVAL, "lbp_server_create: NULL out");
    *out = nullptr;
    if (max_slots < 1 || max_slots > 64) return sfail(LBP_EINVAL, "lbp_server_create: 1 <= max_slots <= 64");
    if (device_mem_budget_bytes < 0) return sfail(LBP_EINVAL, "lbp_server_create: negative budget");
    auto *srv = new lbp_server_s();
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        return sfail(LBP_EDEVICE, "lbp_server_create: hipGetDevice failed");
    }
    srv->budget = device_mem_budget_bytes ? device_mem_budget_bytes : kDefaultBudget;
    srv->max_slots = max_slots;
    try {
        srv->worker = std::thread(worker_main, srv);
    } catch (...) {
        delete srv;
        return sfail(LBP_ENOMEM, "lbp_server_create: cannot start the worker thread");
    }
    *out = srv;
    return LBP_OK;
}

lbp_status lbp_server_add_code(lbp_server srv, lbp_code code, const lbp_params *prm, int32_t *code_slot) {
    lbp::set_error("");
    if (!srv || !code || !prm || !code_slot) return sfail(LBP_EINVAL, "lbp_server_add_code: NULL argument");
    int64_t left;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if ((int)srv->slots.size() >= srv->max_slots) return sfail(LBP_EBUSY, "lbp_server_add_code: all slots in use");
        left = srv->budget - srv->used;
    }
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    auto sl = std::make_unique<Slot>();
    sl->code = code;
    const int m = lbp_code_rows(code);
    sl->n = lbp_code_cols(code);
    sl->mw = (m + 31) / 32;
    sl->nw = (sl->n + 31) / 32;
    lbp_status st = lbp_decoder_create(code, prm, kOsdList, &sl->dec);
    if (st == LBP_OK) st = lbp::serve_shape(sl->dec, kOsdFraction, &sl->shape);
    if (st != LBP_OK) {
        std::string msg = lbp_last_error();
        free_slot(*sl);
        (void)hipSetDevice(prev);
        return sfail(st, msg);
    }
    // the largest ring whose lambda staging (R items of llr_bytes: 2n for Int x.y
    // codes of at most 1024 checks, else 8n) fits the budget left
    sl->llr_bytes = lbp::serve_llr_bytes(sl->dec);
    const int64_t fixed = lbp_decoder_device_bytes(sl->dec) + 4096;
    int64_t R = kMaxRing;
    while (R > kMinRing && fixed + R * sl->llr_bytes > left) R /= 2;
    if (fixed + R * sl->llr_bytes > left) {
        free_slot(*sl);
        (void)hipSetDevice(prev);
        return sfail(LBP_ENOMEM, "lbp_server_add_code: the code's buffers do not fit the device memory budget");
    }
    st = setup_slot(*sl, R);
    (void)hipSetDevice(prev);
    if (st != LBP_OK) {
        std::string msg = lbp_last_error();
        free_slot(*sl);
        return sfail(st, msg);
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if ((int)srv->slots.size() >= srv->max_slots || srv->used + sl->dev_bytes > srv->budget) {
        free_slot(*sl);
        return sfail(LBP_EBUSY, "lbp_server_add_code: slots or budget taken concurrently");
    }
    srv->used += sl->dev_bytes;
    const int idx = (int)srv->slots.size();
    SlotInfo &inf = srv->info[idx];
    inf.mw = sl->mw;
    inf.nw = sl->nw;
    inf.R = sl->R;
    inf.queued.store(0);
    sl->info = &inf;
    srv->slots.push_back(std::move(sl));
    if (srv->slots.size() > 1) {
        // the next grid of each slot reads the new idle time: the copy is ordered
        // on the slot's BP stream (a running grid keeps the one it started with)
        int prev_dev = -1;
        (void)hipGetDevice(&prev_dev);
        (void)hipSetDevice(srv->device);
        for (auto &sp : srv->slots) {
            if (sp->ring.idle_ticks == kIdleTicksShared) continue;
            sp->ring.idle_ticks = kIdleTicksShared;
            if (hipMemcpyAsync(sp->d_ring, &sp->ring, sizeof(sp->ring), hipMemcpyHostToDevice, sp->s_bp) != hipSuccess) {
                srv->dead_msg = "server: ring update failed";
                srv->dead = LBP_EDEVICE;
            }
        }
        if (prev_dev >= 0) (void)hipSetDevice(prev_dev);
    }
    srv->n_slots.store(idx + 1, std::memory_order_release);  // submit may use the slot from here on
    *code_slot = (int32_t)idx;
    return LBP_OK;
}

static lbp_status submit_impl(lbp_server srv, int32_t code_slot, int64_t n_shots, uint64_t seed, uint64_t first_shot_id,
                       const uint32_t *host_syndromes, uint64_t *ticket, ReqPtr *out_req);

lbp_status lbp_server_submit(lbp_server srv, int32_t code_slot, int64_t n_shots, uint64_t seed,
                             uint64_t first_shot_id, const uint32_t *host_syndromes, uint64_t *ticket) {
    return submit_impl(srv, code_slot, n_shots, seed, first_shot_id, host_syndromes, ticket, nullptr);
}

static lbp_status submit_impl(lbp_server srv, int32_t code_slot, int64_t n_shots, uint64_t seed, uint64_t first_shot_id,
                       const uint32_t *host_syndromes, uint64_t *ticket, ReqPtr *out_req) {
    lbp::set_error("");
    if (!srv || !ticket) return sfail(LBP_EINVAL, "lbp_server_submit: NULL argument");
    if (n_shots < 1) return sfail(LBP_EINVAL, "lbp_server_submit: n_shots must be >= 1");
    if (!host_syndromes) return sfail(LBP_EINVAL, "lbp_server_submit: NULL syndromes");
    if (code_slot < 0 || code_slot >= srv->n_slots.load(std::memory_order_acquire))
        return sfail(LBP_EINVAL, "lbp_server_submit: unknown code slot");
    if (srv->dead.load() != LBP_OK) return sfail((lbp_status)srv->dead.load(), "lbp_server_submit: server stopped after a device error");
    SlotInfo &inf = srv->info[code_slot];
    // admission: reserve the shots in the slot's queue count
    if (inf.queued.fetch_add(n_shots) + n_shots > kQueueFactor * inf.R) {
        inf.queued.fetch_sub(n_shots);
        return sfail(LBP_EBUSY, "lbp_server_submit: queue full (admission refused)");
    }
    auto r = std::make_shared<Request>();
    r->slot = code_slot;
    r->n = n_shots;
    r->seed = seed;
    r->first_id = first_shot_id;
    try {
        r->syn.assign(host_syndromes, host_syndromes + (size_t)n_shots * inf.mw);
        r->corr.resize((size_t)n_shots * inf.nw);
        r->flags.resize((size_t)n_shots);
        r->iters.resize((size_t)n_shots);
    } catch (...) {
        inf.queued.fetch_sub(n_shots);
        return sfail(LBP_ENOMEM, "lbp_server_submit: host allocation failed");
    }
    r->t_submit = Clock::now();
    bool wake;
    {
        // tickets are numbered in inbox order, the order the ticket table takes them in
        std::lock_guard<std::mutex> il(srv->in_mu);
        r->ticket = srv->next_ticket.fetch_add(1);
        *ticket = r->ticket;
        if (out_req) *out_req = r;
        srv->inbox.push_back(std::move(r));
        srv->inbox_n.fetch_add(1, std::memory_order_release);
        wake = srv->idle;
    }
    if (wake) srv->cv_work.notify_one();
    return LBP_OK;
}

// The request of a ticket, from the ticket table or the inbox (mu held).
static ReqPtr find_ticket(lbp_server srv, uint64_t ticket, bool *in_inbox) {
    *in_inbox = false;
    if (ReqPtr r = srv->tickets.find(ticket)) return r;
    std::lock_guard<std::mutex> il(srv->in_mu);
    for (auto &r : srv->inbox)
        if (r->ticket == ticket) {
            *in_inbox = true;
            return r;
        }
    return nullptr;
}

lbp_status lbp_server_poll(lbp_server srv, uint64_t ticket, uint32_t *corrections, uint8_t *flags, int32_t *iters) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_poll: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    bool in_inbox;
    ReqPtr r = find_ticket(srv, ticket, &in_inbox);
    if (!r) return sfail(LBP_EINVAL, "lbp_server_poll: unknown ticket");
    if (in_inbox || !r->done) return LBP_ENOTREADY;
    srv->tickets.erase(ticket);
    return copy_out(*r, corrections, flags, iters);
}

lbp_status lbp_server_wait(lbp_server srv, uint64_t ticket, int64_t timeout_us, uint32_t *corrections, uint8_t *flags,
                           int32_t *iters) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    bool in_inbox;
    ReqPtr r = find_ticket(srv, ticket, &in_inbox);
    if (!r) return sfail(LBP_EINVAL, "lbp_server_wait: unknown ticket");
    auto ready = [&] { return r->done; };
    if (timeout_us < 0) srv->cv_done.wait(lk, ready);
    else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return LBP_ENOTREADY;
    srv->tickets.erase(ticket);
    return copy_out(*r, corrections, flags, iters);
}

lbp_status lbp_server_cancel(lbp_server srv, uint64_t ticket) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_cancel: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    bool in_inbox;
    ReqPtr r = find_ticket(srv, ticket, &in_inbox);
    if (!r) return sfail(LBP_EINVAL, "lbp_server_cancel: unknown ticket");
    if (in_inbox) {
        std::lock_guard<std::mutex> il(srv->in_mu);
        for (auto q = srv->inbox.begin(); q != srv->inbox.end(); ++q)
            if (q->get() == r.get()) {
                srv->inbox.erase(q);
                srv->inbox_n.fetch_sub(1);
                break;
            }
        srv->info[r->slot].queued.fetch_sub(r->n);
        return LBP_OK;
    }
    if (!r->done) {
        r->cancelled = true;
        Slot &sl = *srv->slots[r->slot];
        // shots not yet in the ring are never published
        for (auto q = sl.queue.begin(); q != sl.queue.end(); ++q)
            if (q->get() == r.get()) {
                sl.queue.erase(q);
                break;
            }
        sl.info->queued.fetch_sub(r->n - r->dispatched);
        if (r->outstanding > 0) r->dispatched = r->n;  // shots in the ring complete (and are discarded) later
    }
    srv->tickets.erase(ticket);
    return LBP_OK;
}

lbp_status lbp_server_slot_info(lbp_server srv, int32_t code_slot, int64_t *ring_items, int64_t *bp_launches,
                                int64_t *shots, int64_t *max_inflight, int64_t *queued_shots) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_slot_info: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (code_slot < 0 || code_slot >= (int)srv->slots.size()) return sfail(LBP_EINVAL, "lbp_server_slot_info: unknown code slot");
    const Slot &sl = *srv->slots[code_slot];
    if (ring_items) *ring_items = sl.R;
    if (bp_launches) *bp_launches = sl.bp_launches;
    if (shots) *shots = sl.shots;
    if (max_inflight) *max_inflight = sl.max_inflight;
    if (queued_shots) *queued_shots = sl.info->queued.load();
    return LBP_OK;
}

lbp_status lbp_server_run_load(lbp_server srv, int32_t n_codes, const int32_t *code_slots,
                               const uint32_t *const *host_syndromes, const int64_t *pool, int64_t n_requests,
                               int64_t shots_per_request, double requests_per_s, uint64_t seed,
                               int32_t *request_code, double *latency_us, double *elapsed_s) {
    lbp::set_error("");
    if (!srv || !code_slots || !host_syndromes || !pool || !latency_us)
        return sfail(LBP_EINVAL, "lbp_server_run_load: NULL argument");
    if (n_codes < 1 || n_requests < 1 || shots_per_request < 1 || !(requests_per_s >= 0.0))
        return sfail(LBP_EINVAL, "lbp_server_run_load: bad sizes or rate");
    std::vector<int> mw(n_codes);
    for (int k = 0; k < n_codes; ++k) {
        if (code_slots[k] < 0 || code_slots[k] >= srv->n_slots.load(std::memory_order_acquire))
            return sfail(LBP_EINVAL, "lbp_server_run_load: unknown code slot");
        if (pool[k] < shots_per_request || !host_syndromes[k])
            return sfail(LBP_EINVAL, "lbp_server_run_load: syndrome pool smaller than one request");
        mw[k] = srv->info[code_slots[k]].mw;
    }
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(requests_per_s > 0 ? requests_per_s : 1.0);
    std::uniform_int_distribution<int> pick(0, n_codes - 1);
    std::vector<int64_t> cursor(n_codes, 0);
    std::vector<ReqPtr> reqs((size_t)n_requests);
    std::vector<Clock::time_point> arrival((size_t)n_requests);
    const auto t0 = Clock::now();
    double t_next = 0.0;
    for (int64_t q = 0; q < n_requests; ++q) {
        const int k = n_codes > 1 ? pick(rng) : 0;
        if (request_code) request_code[q] = k;
        if (cursor[k] + shots_per_request > pool[k]) cursor[k] = 0;
        const uint32_t *syn = host_syndromes[k] + cursor[k] * mw[k];
        cursor[k] += shots_per_request;
        if (requests_per_s > 0) {
            t_next += gap(rng);
            arrival[q] = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(t_next));
            while (Clock::now() < arrival[q]) {
            }
        } else {
            arrival[q] = Clock::now();
        }
        uint64_t ticket = 0;
        lbp_status st;
        while ((st = submit_impl(srv, code_slots[k], shots_per_request, seed, (uint64_t)q * shots_per_request, syn,
                                 &ticket, &reqs[q])) == LBP_EBUSY)
            std::this_thread::yield();
        if (st != LBP_OK) return st;
    }
    Clock::time_point t_last = t0;
    for (int64_t q = 0; q < n_requests; ++q) {
        lbp_status st = lbp_server_wait(srv, reqs[q]->ticket, -1, nullptr, nullptr, nullptr);
        if (st != LBP_OK) return st;
        latency_us[q] = std::chrono::duration<double, std::micro>(reqs[q]->t_done - arrival[q]).count();
        t_last = std::max(t_last, reqs[q]->t_done);
    }
    if (elapsed_s) *elapsed_s = std::chrono::duration<double>(t_last - t0).count();
    return LBP_OK;
}

void lbp_server_destroy(lbp_server srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> il(srv->in_mu);
        srv->stop = true;
        srv->stop_seen.store(true, std::memory_order_release);
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srv->device);
    for (auto &sp : srv->slots) free_slot(*sp);
    (void)hipSetDevice(prev);
    delete srv;
}

}  // extern "C"
