// Serving loop of the C ABI (lbp_server_*): continuous batching of decode
// requests for several codes on one device.
//
// One worker thread per server.  Each code slot owns `kInflight` batch
// buffers; each buffer has its own stream, decoder workspace, device arrays
// and pinned host staging.  Whenever a buffer is free and requests of that
// slot are queued, the worker packs queued shots (FIFO, splitting large
// requests) into it, copies them in, decodes with per-shot lottery keys
// (seed, shot_id) and copies the results out.  A batch in flight is polled
// with hipEventQuery; its results are scattered back into the requests, and a
// request becomes visible to lbp_server_poll once all of its shots are back.
// Per-shot keys make every result independent of how requests were packed.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lbp.h"
#include "lbp_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kInflight = 3;             // batch buffers per code slot
constexpr int64_t kDefaultBudget = (int64_t)4 << 30;
constexpr int64_t kMaxTick = 8192;       // shots per batch (upper bound)
constexpr int64_t kQueueFactor = 64;     // admission: queued shots per slot <= kQueueFactor * tick

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
    int64_t dispatched = 0;   // shots handed to batches
    int64_t outstanding = 0;  // shots in batches not yet completed
    bool cancelled = false;
    bool done = false;
    lbp_status status = LBP_OK;
    std::string err;
    Clock::time_point t_submit, t_done;
};
using ReqPtr = std::shared_ptr<Request>;

struct Segment {
    ReqPtr req;
    int64_t req_off, batch_off, count;
};

struct Batch {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    lbp_decoder dec = nullptr;
    uint32_t *d_syn = nullptr, *d_corr = nullptr;
    uint8_t *d_flags = nullptr;
    int32_t *d_iters = nullptr;
    uint64_t *d_keys = nullptr;
    uint32_t *h_syn = nullptr, *h_corr = nullptr;
    uint8_t *h_flags = nullptr;
    int32_t *h_iters = nullptr;
    uint64_t *h_keys = nullptr;
    bool busy = false;
    int64_t shots = 0;
    lbp_status status = LBP_OK;
    std::string err;
    std::vector<Segment> segs;
};

struct Slot {
    lbp_code code = nullptr;
    int mw = 0, nw = 0;
    int64_t tick = 0;
    Batch b[kInflight];
    std::deque<ReqPtr> queue;
    int64_t queued_shots = 0;
    // statistics
    int64_t batches = 0, shots = 0, max_fill = 0;
};

}  // namespace

struct lbp_server_s {
    int device = 0;
    int64_t budget = 0, used = 0;
    int max_slots = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::unordered_map<uint64_t, ReqPtr> tickets;
    uint64_t next_ticket = 1;
};

namespace {

void free_batch(Batch &b) {
    if (b.stream) hipStreamSynchronize(b.stream);
    if (b.dec) lbp_decoder_destroy(b.dec);
    hipFree(b.d_syn);
    hipFree(b.d_corr);
    hipFree(b.d_flags);
    hipFree(b.d_iters);
    hipFree(b.d_keys);
    if (b.h_syn) hipHostFree(b.h_syn);
    if (b.h_corr) hipHostFree(b.h_corr);
    if (b.h_flags) hipHostFree(b.h_flags);
    if (b.h_iters) hipHostFree(b.h_iters);
    if (b.h_keys) hipHostFree(b.h_keys);
    if (b.done) hipEventDestroy(b.done);
    if (b.stream) hipStreamDestroy(b.stream);
    b = Batch{};
}

// Launch one batch (worker thread, server lock NOT held: the batch's segments
// reference requests that only the worker mutates while they are dispatched).
void launch_batch(Slot &sl, Batch &b) {
    const int64_t S = b.shots;
    for (const Segment &g : b.segs) {
        const Request &r = *g.req;
        std::memcpy(b.h_syn + g.batch_off * sl.mw, r.syn.data() + g.req_off * sl.mw, (size_t)g.count * sl.mw * 4);
        for (int64_t j = 0; j < g.count; ++j) {
            b.h_keys[2 * (g.batch_off + j)] = r.seed;
            b.h_keys[2 * (g.batch_off + j) + 1] = r.first_id + (uint64_t)(g.req_off + j);
        }
    }
    b.status = LBP_OK;
    hipError_t e = hipMemcpyAsync(b.d_syn, b.h_syn, (size_t)S * sl.mw * 4, hipMemcpyHostToDevice, b.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.d_keys, b.h_keys, (size_t)S * 16, hipMemcpyHostToDevice, b.stream);
    if (e != hipSuccess) {
        b.status = LBP_EDEVICE;
        b.err = std::string("server: hipMemcpyAsync: ") + hipGetErrorString(e);
        return;
    }
    lbp_status st = lbp_decode_keyed(b.dec, S, b.d_keys, b.d_syn, b.d_corr, b.d_flags, b.d_iters, nullptr, b.stream);
    if (st != LBP_OK) {
        b.status = st;
        b.err = lbp_last_error();
        return;
    }
    e = hipMemcpyAsync(b.h_corr, b.d_corr, (size_t)S * sl.nw * 4, hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.h_flags, b.d_flags, (size_t)S, hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.h_iters, b.d_iters, (size_t)S * 4, hipMemcpyDeviceToHost, b.stream);
    if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
    if (e != hipSuccess) {
        b.status = LBP_EDEVICE;
        b.err = std::string("server: ") + hipGetErrorString(e);
    }
}

// Fill a free batch from the slot's queue (lock held).  Returns false if empty.
bool pack_batch(Slot &sl, Batch &b) {
    b.segs.clear();
    b.shots = 0;
    while (!sl.queue.empty() && b.shots < sl.tick) {
        ReqPtr r = sl.queue.front();
        if (r->cancelled || r->status != LBP_OK) {  // never dispatched further
            sl.queued_shots -= r->n - r->dispatched;
            sl.queue.pop_front();
            continue;
        }
        const int64_t take = std::min(r->n - r->dispatched, sl.tick - b.shots);
        b.segs.push_back({r, r->dispatched, b.shots, take});
        r->dispatched += take;
        r->outstanding += take;
        b.shots += take;
        sl.queued_shots -= take;
        if (r->dispatched == r->n) sl.queue.pop_front();
    }
    return b.shots > 0;
}

// Scatter the results of a finished batch into its requests (lock held).
void complete_batch(lbp_server srv, Slot &sl, Batch &b) {
    const auto now = Clock::now();
    for (const Segment &g : b.segs) {
        Request &r = *g.req;
        if (b.status != LBP_OK && r.status == LBP_OK) {
            r.status = b.status;
            r.err = b.err;
        }
        if (!r.cancelled && b.status == LBP_OK) {
            std::memcpy(r.corr.data() + g.req_off * sl.nw, b.h_corr + g.batch_off * sl.nw, (size_t)g.count * sl.nw * 4);
            std::memcpy(r.flags.data() + g.req_off, b.h_flags + g.batch_off, (size_t)g.count);
            std::memcpy(r.iters.data() + g.req_off, b.h_iters + g.batch_off, (size_t)g.count * 4);
        }
        r.outstanding -= g.count;
        if (r.outstanding == 0 && (r.dispatched == r.n || r.cancelled || r.status != LBP_OK)) {
            r.done = true;
            r.t_done = now;
            if (r.cancelled) srv->tickets.erase(r.ticket);
        }
    }
    sl.batches += 1;
    sl.shots += b.shots;
    sl.max_fill = std::max(sl.max_fill, b.shots);
    b.segs.clear();
    b.busy = false;
}

void worker_main(lbp_server srv) {
    hipSetDevice(srv->device);
    std::unique_lock<std::mutex> lk(srv->mu);
    size_t rr = 0;
    while (!srv->stop) {
        bool progressed = false, any_busy = false;
        // 1. completions
        for (auto &sp : srv->slots) {
            for (Batch &b : sp->b) {
                if (!b.busy) continue;
                if (b.status != LBP_OK || hipEventQuery(b.done) == hipSuccess) {
                    complete_batch(srv, *sp, b);
                    progressed = true;
                } else {
                    any_busy = true;
                }
            }
        }
        if (progressed) srv->cv_done.notify_all();
        // 2. dispatch, round robin over slots
        const size_t ns = srv->slots.size();
        for (size_t k = 0; k < ns; ++k) {
            Slot &sl = *srv->slots[(rr + k) % ns];
            for (Batch &b : sl.b) {
                if (b.busy || sl.queue.empty()) continue;
                if (!pack_batch(sl, b)) continue;
                b.busy = true;
                any_busy = true;
                progressed = true;
                lk.unlock();
                launch_batch(sl, b);
                lk.lock();
            }
        }
        rr = ns ? (rr + 1) % ns : 0;
        if (progressed) continue;
        if (any_busy) {
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else {
            srv->cv_work.wait(lk, [&] {
                if (srv->stop) return true;
                for (auto &sp : srv->slots)
                    if (!sp->queue.empty()) return true;
                return false;
            });
        }
    }
}

lbp_status copy_out(const Slot &sl, const Request &r, uint32_t *corrections, uint8_t *flags, int32_t *iters) {
    if (r.status != LBP_OK) return sfail(r.status, r.err);
    if (corrections) std::memcpy(corrections, r.corr.data(), r.corr.size() * 4);
    if (flags) std::memcpy(flags, r.flags.data(), r.flags.size());
    if (iters) std::memcpy(iters, r.iters.data(), r.iters.size() * 4);
    (void)sl;
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
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if ((int)srv->slots.size() >= srv->max_slots) return sfail(LBP_EBUSY, "lbp_server_add_code: all slots in use");
    }
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(srv->device);
    auto sl = std::make_unique<Slot>();
    sl->code = code;
    const int m = lbp_code_rows(code), n = lbp_code_cols(code);
    sl->mw = (m + 31) / 32;
    sl->nw = (n + 31) / 32;
    lbp_status st = LBP_OK;
    int64_t bytes = 0;
    // largest tick (power of two <= kMaxTick) whose buffers fit what is left of the budget
    int64_t left;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        left = srv->budget - srv->used;
    }
    for (int64_t tick = kMaxTick; tick >= 1; tick /= 2) {
        for (Batch &b : sl->b) free_batch(b);
        bytes = 0;
        st = LBP_OK;
        for (Batch &b : sl->b) {
            st = lbp_decoder_create(code, prm, tick, &b.dec);
            if (st != LBP_OK) break;
            bytes += lbp_decoder_device_bytes(b.dec);
            const size_t io = (size_t)tick * (sl->mw * 4 + sl->nw * 4 + 1 + 4 + 16);
            bytes += (int64_t)io;
            hipError_t e = hipSuccess;
            auto chk = [&](hipError_t x) {
                if (e == hipSuccess) e = x;
            };
            chk(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
            chk(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
            chk(hipMalloc((void **)&b.d_syn, (size_t)tick * sl->mw * 4));
            chk(hipMalloc((void **)&b.d_corr, (size_t)tick * sl->nw * 4));
            chk(hipMalloc((void **)&b.d_flags, (size_t)tick));
            chk(hipMalloc((void **)&b.d_iters, (size_t)tick * 4));
            chk(hipMalloc((void **)&b.d_keys, (size_t)tick * 16));
            chk(hipHostMalloc((void **)&b.h_syn, (size_t)tick * sl->mw * 4, hipHostMallocDefault));
            chk(hipHostMalloc((void **)&b.h_corr, (size_t)tick * sl->nw * 4, hipHostMallocDefault));
            chk(hipHostMalloc((void **)&b.h_flags, (size_t)tick, hipHostMallocDefault));
            chk(hipHostMalloc((void **)&b.h_iters, (size_t)tick * 4, hipHostMallocDefault));
            chk(hipHostMalloc((void **)&b.h_keys, (size_t)tick * 16, hipHostMallocDefault));
            if (e != hipSuccess) {
                st = e == hipErrorOutOfMemory ? LBP_ENOMEM : LBP_EDEVICE;
                lbp::set_error((std::string("lbp_server_add_code: ") + hipGetErrorString(e)).c_str());
                break;
            }
        }
        if (st == LBP_OK && bytes <= left) {
            sl->tick = tick;
            break;
        }
        if (st != LBP_OK && st != LBP_ENOMEM) break;  // parameters or device error: no smaller tick helps
    }
    if (st != LBP_OK || sl->tick == 0) {
        std::string msg = lbp_last_error();
        for (Batch &b : sl->b) free_batch(b);
        hipSetDevice(prev);
        if (st != LBP_OK && st != LBP_ENOMEM) return sfail(st, msg);
        return sfail(LBP_ENOMEM, "lbp_server_add_code: the code's buffers do not fit the device memory budget");
    }
    hipSetDevice(prev);
    std::lock_guard<std::mutex> lk(srv->mu);
    if ((int)srv->slots.size() >= srv->max_slots || srv->used + bytes > srv->budget) {
        for (Batch &b : sl->b) free_batch(b);
        return sfail(LBP_EBUSY, "lbp_server_add_code: slots or budget taken concurrently");
    }
    srv->used += bytes;
    *code_slot = (int32_t)srv->slots.size();
    srv->slots.push_back(std::move(sl));
    return LBP_OK;
}

lbp_status lbp_server_submit(lbp_server srv, int32_t code_slot, int64_t n_shots, uint64_t seed,
                             uint64_t first_shot_id, const uint32_t *host_syndromes, uint64_t *ticket) {
    lbp::set_error("");
    if (!srv || !ticket) return sfail(LBP_EINVAL, "lbp_server_submit: NULL argument");
    if (n_shots < 1) return sfail(LBP_EINVAL, "lbp_server_submit: n_shots must be >= 1");
    if (!host_syndromes) return sfail(LBP_EINVAL, "lbp_server_submit: NULL syndromes");
    auto r = std::make_shared<Request>();
    int mw, nw;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (code_slot < 0 || code_slot >= (int)srv->slots.size()) return sfail(LBP_EINVAL, "lbp_server_submit: unknown code slot");
        Slot &sl = *srv->slots[code_slot];
        if (sl.queued_shots + n_shots > kQueueFactor * sl.tick)
            return sfail(LBP_EBUSY, "lbp_server_submit: queue full (admission refused)");
        mw = sl.mw;
        nw = sl.nw;
    }
    r->slot = code_slot;
    r->n = n_shots;
    r->seed = seed;
    r->first_id = first_shot_id;
    try {
        r->syn.assign(host_syndromes, host_syndromes + (size_t)n_shots * mw);
        r->corr.resize((size_t)n_shots * nw);
        r->flags.resize((size_t)n_shots);
        r->iters.resize((size_t)n_shots);
    } catch (...) {
        return sfail(LBP_ENOMEM, "lbp_server_submit: host allocation failed");
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        Slot &sl = *srv->slots[code_slot];
        if (sl.queued_shots + n_shots > kQueueFactor * sl.tick)
            return sfail(LBP_EBUSY, "lbp_server_submit: queue full (admission refused)");
        r->ticket = srv->next_ticket++;
        r->t_submit = Clock::now();
        srv->tickets[r->ticket] = r;
        sl.queue.push_back(r);
        sl.queued_shots += n_shots;
        *ticket = r->ticket;
    }
    srv->cv_work.notify_one();
    return LBP_OK;
}

lbp_status lbp_server_poll(lbp_server srv, uint64_t ticket, uint32_t *corrections, uint8_t *flags, int32_t *iters) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_poll: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return sfail(LBP_EINVAL, "lbp_server_poll: unknown ticket");
    ReqPtr r = it->second;
    if (!r->done) return LBP_ENOTREADY;
    srv->tickets.erase(it);
    return copy_out(*srv->slots[r->slot], *r, corrections, flags, iters);
}

lbp_status lbp_server_wait(lbp_server srv, uint64_t ticket, int64_t timeout_us, uint32_t *corrections, uint8_t *flags,
                           int32_t *iters) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return sfail(LBP_EINVAL, "lbp_server_wait: unknown ticket");
    ReqPtr r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_us < 0) srv->cv_done.wait(lk, ready);
    else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) return LBP_ENOTREADY;
    srv->tickets.erase(r->ticket);
    return copy_out(*srv->slots[r->slot], *r, corrections, flags, iters);
}

lbp_status lbp_server_cancel(lbp_server srv, uint64_t ticket) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_cancel: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return sfail(LBP_EINVAL, "lbp_server_cancel: unknown ticket");
    ReqPtr r = it->second;
    if (!r->done) {
        r->cancelled = true;
        if (r->outstanding > 0) return LBP_OK;  // dropped when its batches complete
        // still queued in full or in part: drop the undispatched rest now
        Slot &sl = *srv->slots[r->slot];
        for (auto q = sl.queue.begin(); q != sl.queue.end(); ++q)
            if (q->get() == r.get()) {
                sl.queued_shots -= r->n - r->dispatched;
                sl.queue.erase(q);
                break;
            }
    }
    srv->tickets.erase(it);
    return LBP_OK;
}

lbp_status lbp_server_slot_info(lbp_server srv, int32_t code_slot, int64_t *tick_shots, int64_t *batches,
                                int64_t *shots, int64_t *max_fill, int64_t *queued_shots) {
    lbp::set_error("");
    if (!srv) return sfail(LBP_EINVAL, "lbp_server_slot_info: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (code_slot < 0 || code_slot >= (int)srv->slots.size()) return sfail(LBP_EINVAL, "lbp_server_slot_info: unknown code slot");
    const Slot &sl = *srv->slots[code_slot];
    if (tick_shots) *tick_shots = sl.tick;
    if (batches) *batches = sl.batches;
    if (shots) *shots = sl.shots;
    if (max_fill) *max_fill = sl.max_fill;
    if (queued_shots) *queued_shots = sl.queued_shots;
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
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (int k = 0; k < n_codes; ++k) {
            if (code_slots[k] < 0 || code_slots[k] >= (int)srv->slots.size())
                return sfail(LBP_EINVAL, "lbp_server_run_load: unknown code slot");
            if (pool[k] < shots_per_request || !host_syndromes[k])
                return sfail(LBP_EINVAL, "lbp_server_run_load: syndrome pool smaller than one request");
            mw[k] = srv->slots[code_slots[k]]->mw;
        }
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
        while ((st = lbp_server_submit(srv, code_slots[k], shots_per_request, seed, (uint64_t)q * shots_per_request,
                                       syn, &ticket)) == LBP_EBUSY)
            std::this_thread::yield();
        if (st != LBP_OK) return st;
        std::lock_guard<std::mutex> lk(srv->mu);
        reqs[q] = srv->tickets[ticket];
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
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(srv->device);
    for (auto &sp : srv->slots)
        for (Batch &b : sp->b) free_batch(b);
    hipSetDevice(prev);
    delete srv;
}

}  // extern "C"
