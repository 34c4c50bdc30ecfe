// Serving engine: continuous batching of retrieval / join requests under an
// HBM budget.
//
//   * Arena: the caller hands the server one device region (the budget); a
//     best-fit allocator with coalescing carves request outputs and batch
//     workspaces out of it, so admission accounts for every byte the server
//     uses.
//   * Admission: requests are admitted in arrival order (head-of-line order,
//     no overtaking) while their output -- and, for requests that run on
//     their own, their workspace -- fits the arena; a request larger than the
//     whole arena fails at once.  Batches of direct work use a descriptor
//     workspace each slot owns, so launching never allocates.
//   * Batching: whenever one of the `max_inflight` stream slots is free, the
//     small requests of the admitted queue (in admission order, up to
//     max_batch_requests, outputs up to batch_max_kib each; requests that run
//     alone keep their place between them) are launched there as one
//     persistent batch -- a replay of the slot's captured graph, or
//     the same two kernels launched directly -- after waiting up to
//     batch_window_us for a partial batch to fill.  A batch carries direct
//     work and DPG work alike (a DPG request's steps use scratch reserved for
//     it at admission); dimension-order joins and large requests run alone
//     through their single-request entry point, whose dedicated kernels are
//     faster for large outputs and need no batching to hide launch cost.  A
//     batch that would hold a single request also takes that path, so
//     batching costs nothing at low load.  With max_batch_requests = 1 every
//     request takes it (the per-request baseline).
//     Requests arriving while batches run are admitted and launched on the
//     next free slot, so their work overlaps on the device.
//   * Completion: a request of a persistent batch is done as soon as the
//     kernel sets its completion word (host memory), while the rest of the
//     batch may still run; a request launched alone, when its stream event
//     fires.  Latency is completion time minus submit time (host steady
//     clock).  Outputs stay valid until released.
// One scheduler thread owns the context and all HIP calls.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "dpg_internal.h"

namespace dpg {

using Clock = std::chrono::steady_clock;

}  // namespace dpg

struct dpg_arena {
    dpg::Arena arena;
    uintptr_t base;
    dpg_arena(uintptr_t b, size_t size, size_t align) : arena(size, align), base(b) {}
};

namespace dpg {

enum TicketState { T_QUEUED = 0, T_ADMITTED = 1, T_RUNNING = 2, T_DONE = 3, T_FAILED = 4 };

struct Ticket {
    dpg_request req{};
    int state = T_QUEUED;
    dpg_status status = DPG_OK;
    bool batched = false;          // runs inside a slot's persistent batch launch
    size_t own_ws = 0;             // workspace of its single-request entry point
    bool finished = false;         // completed (DONE or FAILED) while its batch may still run
    size_t out_off = 0, out_bytes = 0, ws_off = 0, ws_bytes = 0;
    bool has_out = false, has_ws = false;
    Clock::time_point submit, admit, done;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    bool busy = false;
    bool batch_launch = false;      // tickets run as one persistent batch (per-request completion words)
    std::vector<uint64_t> tickets;  // in the order of the launched request array
    std::vector<uint8_t> seen_done; // (batch) completion word already seen, per ticket
    std::vector<size_t> newly_done; // (batch) tickets whose completion word the last poll found set
    hipError_t polled = hipErrorNotReady;  // the last poll's event query
    Clock::time_point poll_time;           // and when it was taken
    dpg_batch_graph *graph = nullptr;
    size_t batch_ws_off = 0, batch_ws_bytes = 0;  // descriptors of a batch of direct work
};

// Batches of fewer requests launch the batch kernel directly even with
// use_graph.
constexpr int32_t kGraphMinRequests = 16;
// With this many slots busy and requests still waiting for admission (the
// server is saturated), a partial batch waits for a slot to finish (the
// device is fed meanwhile), so that requests gather into larger batches.
// Below saturation nothing waits for admission, and a request starts at once.
constexpr int kHoldBusySlots = 2;

static size_t output_bytes(const dpg_request &q) {
    const int64_t row = q.kind == DPG_REQ_RETRIEVE ? q.rec_bytes : (int64_t)q.fact_bytes + q.rec_bytes;
    return (size_t)(q.n > 0 ? q.n : 0) * (size_t)(row > 0 ? row : 0);
}

}  // namespace dpg

struct dpg_server {
    dpg_ctx *ctx = nullptr;
    dpg_server_config cfg{};
    dpg::Arena *arena = nullptr;
    size_t capacity = 0;  // arena bytes requests can ever hold (the slots keep the rest)
    char *base = nullptr;
    std::vector<dpg::Slot> slots;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::unordered_map<uint64_t, dpg::Ticket> tickets;
    std::deque<uint64_t> pending;   // submitted, not admitted
    std::deque<uint64_t> admitted;  // output reserved, waiting for a slot
    std::deque<uint64_t> completed; // finished, not yet reported by next_completed
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread thread;
    dpg_status fatal = DPG_OK;
    // statistics
    std::vector<double> latencies_ms;
    int64_t submitted = 0, n_completed = 0, n_failed = 0, batches = 0;
    double launch_s = 0;  // host time spent enqueueing work
    double bytes_delivered = 0;
    dpg::Clock::time_point first_submit, last_done;
    bool any_submit = false;
};

namespace dpg {

// One ticket is finished: its workspace goes back to the arena, its output
// stays until released.
static void finish_ticket(dpg_server *s, uint64_t t, dpg_status st, Clock::time_point now) {
    auto it = s->tickets.find(t);
    if (it == s->tickets.end()) return;
    Ticket &tk = it->second;
    if (tk.finished) return;
    tk.finished = true;
    tk.done = now;
    if (tk.has_ws) s->arena->release(tk.ws_off);
    tk.has_ws = false;
    if (st == DPG_OK) {
        tk.state = T_DONE;
        s->n_completed++;
        s->bytes_delivered += (double)tk.out_bytes;
        s->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - tk.submit).count());
    } else {
        tk.state = T_FAILED;
        tk.status = st;
        s->n_failed++;
    }
    s->completed.push_back(t);
    s->last_done = now;
}

// The slot's launch has ended (its stream event): every ticket not yet
// finished is, and the slot is free.
static void finish_batch(dpg_server *s, Slot &sl, dpg_status st, Clock::time_point now) {
    for (uint64_t t : sl.tickets) finish_ticket(s, t, st, now);
    sl.tickets.clear();
    sl.busy = false;
    sl.batch_launch = false;
}

// Polls a busy slot (without the server lock: only the scheduler thread
// touches the slots): the requests of a running persistent batch whose
// completion word is newly set, which finish before the rest of the batch,
// then the slot's event.
static void poll_slot(Slot &sl) {
    sl.newly_done.clear();
    if (sl.batch_launch)
        for (size_t i = 0; i < sl.tickets.size(); ++i)
            if (!sl.seen_done[i] && dpg_batch_graph_request_done(sl.graph, (int32_t)i)) {
                sl.seen_done[i] = 1;
                sl.newly_done.push_back(i);
            }
    sl.polled = hipEventQuery(sl.event);
    sl.poll_time = Clock::now();
}

// What a slot's launch needs, copied out of the tickets under the server lock
// so that the HIP calls can run without it.
struct LaunchWork {
    bool single = false;        // one ticket through its single-request entry point
    dpg_request q{};            // (single) the request
    char *w = nullptr;          // (single) its workspace
    size_t wb = 0;
    std::vector<dpg_request> reqs;  // (batch) the requests, in ticket order
};

// Take `batch` onto the slot (under the lock): batched tickets together in
// one persistent launch (graph replay when available), or one unbatched
// ticket through its single-request entry point with the workspace reserved
// at admission.
static LaunchWork prepare_launch(dpg_server *s, Slot &sl, const std::vector<uint64_t> &batch) {
    LaunchWork w;
    const Ticket &first = s->tickets[batch[0]];
    // A batch of one runs through the single-request entry point (no
    // descriptor upload), borrowing the idle slot's descriptor workspace.
    const bool alone = first.batched && batch.size() == 1 && (first.has_ws || first.own_ws <= sl.batch_ws_bytes);
    if (!first.batched || alone) {
        w.single = true;
        w.q = first.req;
        const bool slot_ws = alone && !first.has_ws;
        w.w = slot_ws ? s->base + sl.batch_ws_off : (first.has_ws ? s->base + first.ws_off : nullptr);
        w.wb = slot_ws ? sl.batch_ws_bytes : first.ws_bytes;
    } else {
        w.reqs.reserve(batch.size());
        for (uint64_t t : batch) {
            const Ticket &tk = s->tickets[t];
            dpg_request q = tk.req;
            // the scratch of a DPG request's steps, reserved at admission
            q.workspace = tk.has_ws ? s->base + tk.ws_off : nullptr;
            q.workspace_bytes = tk.has_ws ? tk.ws_bytes : 0;
            w.reqs.push_back(q);
        }
    }
    sl.tickets = batch;
    sl.seen_done.assign(batch.size(), 0);
    sl.batch_launch = first.batched && !alone;
    sl.busy = true;
    s->batches++;
    for (uint64_t t : batch) s->tickets[t].state = T_RUNNING;
    return w;
}

// The slot's HIP work (without the server lock: only the scheduler thread
// touches the context, the slots and their streams).
static dpg_status launch_work(dpg_server *s, Slot &sl, const LaunchWork &w) {
    dpg_ctx *ctx = s->ctx;
    dpg_status st;
    if (w.single) {
        const dpg_request &q = w.q;
        st = q.kind == DPG_REQ_RETRIEVE
                 ? dpg_retrieve(ctx, q.src, q.n_src, q.rec_bytes, q.rids, q.n, q.dst, w.w, w.wb, (dpg_algo)q.algo, 0,
                                sl.stream)
                 : dpg_fk_join(ctx, q.fact, q.n, q.fact_bytes, q.fk_offset, q.src, q.n_src, q.rec_bytes, q.dst,
                               (dpg_join_order)q.order, w.w, w.wb, (dpg_algo)q.algo, 0, sl.stream);
    } else {
        const int32_t n = (int32_t)w.reqs.size();
        // a graph replay costs more host time than launching the kernel
        // (30-45 against about 10 us per batch here): it is used for
        // batches that amortize it
        st = batch_graph_launch(sl.graph, w.reqs.data(), n, sl.stream,
                                s->cfg.use_graph != 0 && n >= kGraphMinRequests);
    }
    if (st != DPG_OK) return st;
    if (hipEventRecord(sl.event, sl.stream) != hipSuccess) return DPG_ERR_HIP;
    return DPG_OK;
}

static void scheduler(dpg_server *s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        bool changed = false;
        // 1. completions: the device is polled without the lock, so that
        //    submitters and clients are not held up by the polling
        lk.unlock();
        for (Slot &sl : s->slots)
            if (sl.busy) poll_slot(sl);
        lk.lock();
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            for (size_t i : sl.newly_done) {
                finish_ticket(s, sl.tickets[i], DPG_OK, sl.poll_time);
                changed = true;
            }
            if (sl.polled == hipSuccess) {
                finish_batch(s, sl, DPG_OK, sl.poll_time);
                changed = true;
            } else if (sl.polled != hipErrorNotReady) {
                finish_batch(s, sl, DPG_ERR_HIP, sl.poll_time);
                changed = true;
            }
        }
        // 2. admission, in arrival order: reserve the output and, for work
        //    that runs on its own, its workspace
        bool any_busy = false;
        for (Slot &sl : s->slots) any_busy |= sl.busy;
        // Nothing will free memory when the server is stopping with no work
        // in flight or waiting: a head request that does not fit then fails.
        const bool nothing_will_free = s->stop && !any_busy && s->admitted.empty();
        while (!s->pending.empty()) {
            const uint64_t t = s->pending.front();
            Ticket &tk = s->tickets[t];
            const AdmitResult r = admit_head(*s->arena, s->capacity, tk.out_bytes, tk.ws_bytes, nothing_will_free);
            if (r.kind == ADMIT_WAIT) break;
            s->pending.pop_front();
            changed = true;
            if (r.kind == ADMIT_FAIL) {
                tk.state = T_FAILED;
                tk.status = DPG_ERR_BUSY;
                s->n_failed++;
                s->completed.push_back(t);
                continue;
            }
            tk.out_off = r.out_off;
            tk.ws_off = r.ws_off;
            tk.has_out = r.has_out;
            tk.has_ws = r.has_ws;
            tk.req.dst = tk.has_out ? s->base + tk.out_off : nullptr;
            tk.state = T_ADMITTED;
            tk.admit = Clock::now();
            s->admitted.push_back(t);
        }
        // 3. launches on free slots: an unbatched ticket at the head runs
        //    alone; otherwise the batched tickets of the admitted queue, in
        //    admission order (up to max_batch_requests), run as one batch --
        //    unbatched tickets between them keep their place and take the
        //    next free slot once they reach the head
        bool window_wait = false;
        int busy = 0;
        for (Slot &sl : s->slots) busy += sl.busy ? 1 : 0;
        const bool saturated = !s->pending.empty();
        for (Slot &sl : s->slots) {
            if (sl.busy || s->admitted.empty()) continue;
            std::vector<uint64_t> batch;
            const bool batched = s->tickets[s->admitted.front()].batched;
            if (batched && s->cfg.max_batch_requests > 1 && busy >= kHoldBusySlots && saturated && !s->stop) {
                size_t avail = 0;
                for (size_t k = 0; k < s->admitted.size() && (int32_t)avail < s->cfg.max_batch_requests &&
                                   k < (size_t)4 * (size_t)s->cfg.max_batch_requests;
                     ++k)
                    avail += s->tickets[s->admitted[k]].batched ? 1 : 0;
                if ((int32_t)avail < s->cfg.max_batch_requests) break;  // the batch fills while the device works
            }
            if (batched && s->cfg.batch_window_us > 0 && !s->stop) {
                size_t avail = 0;
                for (size_t k = 0; k < s->admitted.size() && (int32_t)avail < s->cfg.max_batch_requests &&
                                   k < (size_t)4 * (size_t)s->cfg.max_batch_requests;
                     ++k)
                    avail += s->tickets[s->admitted[k]].batched ? 1 : 0;
                if ((int32_t)avail < s->cfg.max_batch_requests) {
                    // a partial batch waits (up to the window) for more requests
                    const double waited = std::chrono::duration<double, std::micro>(
                                              Clock::now() - s->tickets[s->admitted.front()].admit)
                                              .count();
                    if (waited < s->cfg.batch_window_us) {
                        window_wait = true;
                        break;
                    }
                }
            }
            // the head of the queue decides (a bounded look-ahead keeps a
            // launch's host cost independent of the queue's length)
            const size_t look = std::min(s->admitted.size(), (size_t)4 * (size_t)s->cfg.max_batch_requests);
            std::vector<bool> flags(look);
            for (size_t k = 0; k < look; ++k) flags[k] = s->tickets[s->admitted[k]].batched;
            const std::vector<size_t> take = select_launch(flags, s->cfg.max_batch_requests);
            for (size_t k : take) batch.push_back(s->admitted[k]);
            for (size_t k = take.size(); k-- > 0;) s->admitted.erase(s->admitted.begin() + (std::ptrdiff_t)take[k]);
            ++busy;
            const LaunchWork work = prepare_launch(s, sl, batch);
            // Submitters are not held up by the launch's host work, so the
            // next launch finds the requests that arrived meanwhile (with the
            // lock held they came one per launch, and saturated servers
            // launched batches of one).
            lk.unlock();
            const auto t_launch = Clock::now();
            const dpg_status st = launch_work(s, sl, work);
            const double dt = std::chrono::duration<double>(Clock::now() - t_launch).count();
            lk.lock();
            s->launch_s += dt;
            if (st != DPG_OK) finish_batch(s, sl, st, Clock::now());
            changed = true;
        }
        if (changed) s->done_cv.notify_all();
        bool inflight = false;
        for (Slot &sl : s->slots) inflight |= sl.busy;
        if (s->stop && !inflight && s->pending.empty() && s->admitted.empty()) break;
        if (inflight || window_wait) {
            // work on the device, or a batch window open: check again shortly
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        } else if (!changed) {
            s->cv.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

static double percentile(std::vector<double> v, double p) {
    if (v.empty()) return 0;
    std::sort(v.begin(), v.end());
    const double pos = p * (double)(v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

}  // namespace dpg

using namespace dpg;

extern "C" {

dpg_status dpg_arena_create(uintptr_t base, size_t bytes, size_t align, dpg_arena **out) {
    if (!out || align == 0 || (align & (align - 1)) || base % align) return DPG_ERR_INVALID_ARG;
    *out = new dpg_arena(base, bytes, align);
    return DPG_OK;
}

dpg_status dpg_arena_alloc(dpg_arena *a, size_t bytes, uintptr_t *addr) {
    if (!a || !addr) return DPG_ERR_INVALID_ARG;
    size_t off = 0;
    if (!a->arena.alloc(bytes, &off)) return DPG_ERR_BUSY;
    *addr = a->base + off;
    return DPG_OK;
}

dpg_status dpg_arena_free(dpg_arena *a, uintptr_t addr) {
    if (!a || addr < a->base) return DPG_ERR_INVALID_ARG;
    return a->arena.release(addr - a->base) ? DPG_OK : DPG_ERR_INVALID_ARG;
}

dpg_status dpg_arena_stats(const dpg_arena *a, size_t *in_use, size_t *high_water, size_t *largest_free,
                           size_t *free_blocks) {
    if (!a) return DPG_ERR_INVALID_ARG;
    if (in_use) *in_use = a->arena.in_use();
    if (high_water) *high_water = a->arena.high_water();
    if (largest_free) *largest_free = a->arena.largest_free();
    if (free_blocks) *free_blocks = a->arena.free_blocks();
    return DPG_OK;
}

void dpg_arena_destroy(dpg_arena *a) { delete a; }

dpg_status dpg_server_create(dpg_ctx *ctx, const dpg_server_config *cfg, dpg_server **out) {
    if (!ctx || !cfg || !out) return DPG_ERR_INVALID_ARG;
    *out = nullptr;
    if (!cfg->arena || cfg->arena_bytes < kAlign || ((uintptr_t)cfg->arena) % kAlign) return DPG_ERR_INVALID_ARG;
    if (cfg->max_inflight < 1 || cfg->max_inflight > 16 || cfg->max_batch_requests < 1) return DPG_ERR_INVALID_ARG;
    dpg_server *s = new dpg_server();
    s->ctx = ctx;
    s->cfg = *cfg;
    s->base = (char *)cfg->arena;
    s->arena = new Arena(cfg->arena_bytes, kAlign);
    s->slots.resize(cfg->max_inflight);
    dpg_status st = DPG_OK;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(ctx->device) != hipSuccess) st = DPG_ERR_HIP;
    for (Slot &sl : s->slots) {
        if (st != DPG_OK) break;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.event, hipEventDisableTiming) != hipSuccess) {
            st = DPG_ERR_HIP;
            break;
        }
        if (cfg->max_batch_requests > 1) {
            sl.batch_ws_bytes = dpg_batch_graph_workspace_bytes(ctx, cfg->max_batch_requests);
            if (!s->arena->alloc(sl.batch_ws_bytes, &sl.batch_ws_off)) {
                st = DPG_ERR_WORKSPACE_TOO_SMALL;
                break;
            }
            // the bound batch object (pinned descriptor staging; its graph is
            // replayed only with use_graph)
            st = dpg_batch_graph_create(ctx, cfg->max_batch_requests, s->base + sl.batch_ws_off, sl.batch_ws_bytes,
                                        sl.stream, &sl.graph);
        }
    }
    (void)hipSetDevice(prev);
    s->capacity = s->arena->size() - s->arena->in_use();
    if (st != DPG_OK) {
        for (Slot &sl : s->slots) {
            if (sl.graph) dpg_batch_graph_destroy(sl.graph);
            if (sl.event) (void)hipEventDestroy(sl.event);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete s->arena;
        delete s;
        return st;
    }
    s->thread = std::thread(scheduler, s);
    *out = s;
    return DPG_OK;
}

}  // extern "C"

namespace dpg {

// A request's ticket, planned without the server lock.
static Ticket make_ticket(dpg_server *s, const dpg_request &req) {
    Ticket tk;
    tk.req = req;
    tk.req.dst = nullptr;
    tk.out_bytes = output_bytes(req);
    tk.submit = Clock::now();
    size_t own_ws = 0, batch_ws = 0;
    // the output will live somewhere in the arena: inputs must lie outside it
    tk.status = plan_batch_request(s->ctx, tk.req, s->base, s->cfg.arena_bytes, &own_ws, &batch_ws);
    if (tk.status == DPG_OK) {
        const size_t max_batched = (size_t)(s->cfg.batch_max_kib > 0 ? s->cfg.batch_max_kib : 4096) << 10;
        tk.batched = s->cfg.max_batch_requests > 1 && tk.out_bytes <= max_batched;
        // direct work in a batch needs no workspace of its own; DPG steps
        // need scratch (enough for the single-request entry point too, which
        // runs a batch of one)
        tk.ws_bytes = !tk.batched ? own_ws : batch_ws ? std::max(own_ws, batch_ws) : 0;
        tk.own_ws = own_ws;
    } else {
        tk.state = T_FAILED;
    }
    return tk;
}

// Queue a planned ticket (under the server lock).
static uint64_t enqueue_ticket(dpg_server *s, Ticket &tk) {
    const uint64_t id = s->next_ticket++;
    if (!s->any_submit) {
        s->first_submit = tk.submit;
        s->any_submit = true;
    }
    s->submitted++;
    const bool failed = tk.state == T_FAILED;
    if (failed) {
        tk.done = tk.submit;
        s->n_failed++;
    }
    s->tickets.emplace(id, tk);
    if (failed) s->completed.push_back(id);
    else s->pending.push_back(id);
    return id;
}

}  // namespace dpg

extern "C" {

dpg_status dpg_server_submit(dpg_server *s, const dpg_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket) return DPG_ERR_INVALID_ARG;
    Ticket tk = make_ticket(s, *req);
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return DPG_ERR_INVALID_ARG;
        *ticket = enqueue_ticket(s, tk);
    }
    s->cv.notify_one();
    return DPG_OK;
}

dpg_status dpg_server_submit_many(dpg_server *s, const dpg_request *reqs, int32_t n, uint64_t *tickets) {
    if (!s || n < 0 || (n > 0 && (!reqs || !tickets))) return DPG_ERR_INVALID_ARG;
    std::vector<Ticket> tks;
    tks.reserve((size_t)n);
    for (int32_t i = 0; i < n; ++i) tks.push_back(make_ticket(s, reqs[i]));
    {
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return DPG_ERR_INVALID_ARG;
        for (int32_t i = 0; i < n; ++i) tickets[i] = enqueue_ticket(s, tks[(size_t)i]);
    }
    s->cv.notify_one();
    return DPG_OK;
}

dpg_status dpg_server_poll(dpg_server *s, uint64_t ticket, int32_t *state, dpg_status *status, void **dst,
                           double *latency_ms) {
    if (!s) return DPG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return DPG_ERR_INVALID_ARG;
    const Ticket &tk = it->second;
    if (state) *state = tk.state;
    if (status) *status = tk.status;
    if (dst) *dst = tk.state == T_DONE ? tk.req.dst : nullptr;
    if (latency_ms)
        *latency_ms = tk.state >= T_DONE ? std::chrono::duration<double, std::milli>(tk.done - tk.submit).count() : 0;
    return DPG_OK;
}

dpg_status dpg_server_next_completed(dpg_server *s, int32_t timeout_ms, uint64_t *ticket) {
    if (!s || !ticket) return DPG_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = Clock::now() + std::chrono::milliseconds(timeout_ms > 0 ? timeout_ms : 0);
    while (s->completed.empty()) {
        if (timeout_ms <= 0 || s->done_cv.wait_until(lk, deadline) == std::cv_status::timeout) {
            if (s->completed.empty()) return DPG_ERR_BUSY;
        }
    }
    *ticket = s->completed.front();
    s->completed.pop_front();
    return DPG_OK;
}

dpg_status dpg_server_release(dpg_server *s, uint64_t ticket) {
    if (!s) return DPG_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->tickets.find(ticket);
        if (it == s->tickets.end()) return DPG_ERR_INVALID_ARG;
        if (it->second.state < T_DONE) return DPG_ERR_BUSY;
        if (it->second.has_out) s->arena->release(it->second.out_off);
        s->tickets.erase(it);
    }
    s->cv.notify_one();
    return DPG_OK;
}

dpg_status dpg_server_stats_get(dpg_server *s, dpg_server_stats *out) {
    if (!s || !out) return DPG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    *out = dpg_server_stats{};
    out->submitted = s->submitted;
    out->completed = s->n_completed;
    out->failed = s->n_failed;
    out->batches = s->batches;
    out->p50_ms = percentile(s->latencies_ms, 0.50);
    out->p99_ms = percentile(s->latencies_ms, 0.99);
    out->max_ms = s->latencies_ms.empty() ? 0 : *std::max_element(s->latencies_ms.begin(), s->latencies_ms.end());
    double sum = 0;
    for (double v : s->latencies_ms) sum += v;
    out->mean_ms = s->latencies_ms.empty() ? 0 : sum / (double)s->latencies_ms.size();
    out->bytes_delivered = s->bytes_delivered;
    out->span_s = s->any_submit && s->n_completed
                      ? std::chrono::duration<double>(s->last_done - s->first_submit).count()
                      : 0;
    out->arena_in_use = s->arena->in_use();
    out->arena_high_water = s->arena->high_water();
    out->launch_s = s->launch_s;
    return DPG_OK;
}

dpg_status dpg_server_reset_stats(dpg_server *s) {
    if (!s) return DPG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(s->mu);
    s->latencies_ms.clear();
    s->submitted = s->n_completed = s->n_failed = s->batches = 0;
    s->bytes_delivered = 0;
    s->launch_s = 0;
    s->any_submit = false;
    return DPG_OK;
}

void dpg_server_destroy(dpg_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->thread.joinable()) s->thread.join();
    for (Slot &sl : s->slots) {
        if (sl.graph) dpg_batch_graph_destroy(sl.graph);
        if (sl.event) (void)hipEventDestroy(sl.event);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s->arena;
    delete s;
}

}  // extern "C"
