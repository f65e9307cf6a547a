// Serving runtime: continuous batching of bridge queries on one device.
//
// Requests enter a bounded FIFO.  A scheduler admits the head request as soon
// as the device-memory budget has room for it, onto one of two paths:
//  * slots: each slot runs the full plain path for one request on its own
//    stream and context, so the kernels of different requests overlap;
//  * the batch lane, for requests within the batched kernels' limits (V
//    within a workgroup's LDS, E under a cap): a lane worker takes every lane
//    request queued when it becomes free, packs their edge lists into one
//    device buffer and certifies them all in one batched call (the persistent
//    kernels, without graph capture).  Two workers alternate, so one packs
//    and finishes a tick on the host while the other's kernels run.
// A lane-eligible request takes a free slot while the lane has nothing
// queued (a lone request finishes sooner on the plain path), and waits for
// one while fewer requests wait than there are slots and the lane is idle;
// beyond that backlog, and while the lane works, such requests collect in the
// lane, where the per-request launch and synchronisation costs are paid once
// per tick.  Latency is
// stamped from submission to the moment the result is available.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace br {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    void* pin = nullptr;               // owned copy in pinned staging memory (host submissions) ...
    size_t pin_cap = 0;
    std::vector<int32_t> h_edges;      // ... or in pageable memory when the pinned pool is full
    const int32_t* d_edges = nullptr;  // caller's device buffer (device submissions)
    int64_t E = 0;
    int32_t V = 0;
    int32_t M = 1;
    int mode = 1;                      // final step, fixed when the request is admitted
    int64_t ws_bytes = 0;              // device workspace it needs (for its final step)
    int64_t buf_bytes = 0;             // device copy of its edges (host submissions)
    bool lane = false;                 // served by the batch lane (fixed at submission)
    int64_t lane_bytes = 0;            // its charge while queued for or in a lane tick
    Clock::time_point t_submit;
    // result
    int status = BR_OK;
    std::string msg;
    std::vector<int32_t> bridges;
    double latency_ms = 0;
    bool done = false;
};

struct Slot {
    br_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    void* d_buf = nullptr;             // device copy of host-submitted edges
    size_t d_cap = 0;
    int64_t held = 0;                  // device bytes charged to this slot (kept after a request)
    bool trimming = false;             // its buffers are being released by the scheduler
    std::shared_ptr<Request> job;
    std::thread th;
};

// one worker of the batch lane: its context (plans and arenas), stream and
// packed edge buffer, kept between ticks and charged to the budget
struct LaneWorker {
    br_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    void* buf = nullptr;               // packed edges, then the gather table
    size_t cap = 0;
    GatherItem* h_items = nullptr;     // pinned staging of the gather table
    int32_t h_items_cap = 0;
    int64_t held = 0;                  // device bytes charged between ticks
    bool busy = false;                 // a tick is running
    bool trimming = false;             // its buffers are being released by the scheduler
    std::thread th;
};

constexpr size_t kQueueMax = 65536;
constexpr int kLaneWorkers = 2;
constexpr int64_t kLaneMaxEdges = int64_t(1) << 21;   // default edge cap of lane requests

}  // namespace
}  // namespace br

struct br_server {
    int device = 0;
    int final_step = 1;                // of the requests admitted from now on
    // in_use: device bytes the slots hold -- a slot keeps its workspace and
    // edge buffer after a request (sized exactly to what it was charged), so
    // idle slots count too until the scheduler releases them
    int64_t budget = 0, in_use = 0, peak_in_use = 0;
    std::vector<std::unique_ptr<br::Slot>> slots;
    std::deque<std::shared_ptr<br::Request>> queue;
    std::map<uint64_t, std::shared_ptr<br::Request>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::mutex mu;
    std::condition_variable cv_sched, cv_slot, cv_done;
    std::thread sched;
    // statistics
    std::vector<double> lat;
    int64_t edges_done = 0;
    int64_t inflight = 0, peak_inflight = 0;
    br::Clock::time_point busy_start;
    double busy_ms = 0;
    // pinned staging for host submissions: free buffers, bytes held, cap
    std::vector<std::pair<void*, size_t>> pin_free;
    int64_t pin_total = 0, pin_limit = 0;
    std::unique_ptr<br::Pool> copier;    // parallel copy of submitted edge lists
    std::mutex copy_mu;
    // batch lane: requests with V <= lane_max_v and E <= lane_max_e
    int32_t lane_max_v = 0;              // 0: lane off
    int64_t lane_max_e = 0;
    std::deque<std::shared_ptr<br::Request>> lane_q;
    std::condition_variable cv_lane;
    std::vector<std::unique_ptr<br::LaneWorker>> lanes;
    int64_t ticks = 0, lane_requests = 0;
};

namespace br {
namespace {

// device bytes a request needs while it runs: the plain path's workspace for
// its final step, and the copy of its edges when they came from the host
void charge(Request& r, bool host_edges, int mode, int device) {
    const Plan P = plan_for(device, r.E, r.V, r.M);
    r.ws_bytes = (int64_t)plan_workspace_bytes(P, mode == 1);
    r.buf_bytes = host_edges ? 8 * r.E : 0;
}

// Device bytes one request adds to a batch-lane tick (an upper bound): its
// packed edges, its certificate regions (per merge level at most its edges,
// per node at most 2(V-1) pairs), per-node counters and metadata, root flags
// and bridge keys, and for graphs above the small kernel's limit its part of
// the union certificate and of the bridge step's scratch.  Chunks of at least
// 4,096 edges (the smallest chunk size the batched path uses).
int64_t lane_need(const Request& r) {
    const int64_t C = 4096, M = std::max<int64_t>(1, (r.E + C - 1) / C);
    int R = 0;
    while ((int64_t(1) << R) < M) R++;
    const int64_t V = r.V;
    const int64_t regions = std::min<int64_t>(r.E * (R + 1), 2 * V * M);
    int64_t b = 8 * r.E + 8 * regions + (96 + 4 * (int64_t)R) * M + 8 * V + 8192;
    if (r.V > batched_max_v_dev()) b += 16 * V + 4 * device_bridges_words(r.V) + 8192;
    return b;
}

bool lane_fits(const br_server* S, const Request& r) {
    return S->lane_max_v > 0 && r.V <= S->lane_max_v && r.E <= S->lane_max_e;
}

// what slot sl holds after running r (buffers only ever grow to what is needed)
int64_t held_after(const Slot& sl, const Request& r) {
    return std::max<int64_t>((int64_t)sl.ctx->ws.size, r.ws_bytes) + std::max<int64_t>((int64_t)sl.d_cap, r.buf_bytes);
}

// release an idle slot's device buffers (scheduler thread, slot not running)
void release_slot(Slot& sl) {
    (void)hipSetDevice(sl.ctx->device);
    (void)hipStreamSynchronize(sl.stream);
    if (sl.ctx->ws.base) (void)hipFree(sl.ctx->ws.base);
    sl.ctx->ws.base = nullptr;
    sl.ctx->ws.size = 0;
    sl.ctx->solo_key_base = nullptr;
    if (sl.d_buf) (void)hipFree(sl.d_buf);
    sl.d_buf = nullptr;
    sl.d_cap = 0;
    (void)hipGetLastError();
}

// a pinned buffer of at least `bytes` (best fit among the free ones, else a new
// one while the pool stays under its cap); {nullptr, 0} when none
std::pair<void*, size_t> acquire_pinned(br_server* S, size_t bytes) {
    {
        std::lock_guard<std::mutex> g(S->mu);
        size_t best = SIZE_MAX;
        int at = -1;
        for (size_t i = 0; i < S->pin_free.size(); i++)
            if (S->pin_free[i].second >= bytes && S->pin_free[i].second < best) {
                best = S->pin_free[i].second;
                at = (int)i;
            }
        if (at >= 0) {
            auto b = S->pin_free[at];
            S->pin_free.erase(S->pin_free.begin() + at);
            return b;
        }
        size_t cap = (size_t)1 << 20;
        while (cap < bytes) cap <<= 1;
        if (S->pin_total + (int64_t)cap > S->pin_limit) return {nullptr, 0};
        S->pin_total += (int64_t)cap;
        bytes = cap;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocPortable) != hipSuccess) {
        (void)hipGetLastError();
        std::lock_guard<std::mutex> g(S->mu);
        S->pin_total -= (int64_t)bytes;
        return {nullptr, 0};
    }
    return {p, bytes};
}

// copy with every worker of the server's copy pool (one copy at a time)
void parallel_copy(br_server* S, void* dst, const void* src, size_t bytes) {
    if (bytes < ((size_t)4 << 20)) {
        std::memcpy(dst, src, bytes);
        return;
    }
    std::lock_guard<std::mutex> g(S->copy_mu);
    const int n = S->copier->size();
    S->copier->run([&](int w) {
        const size_t lo = bytes * (size_t)w / n, hi = bytes * (size_t)(w + 1) / n;
        std::memcpy(static_cast<char*>(dst) + lo, static_cast<const char*>(src) + lo, hi - lo);
    });
}

// chunk count per request: keep chunks several times larger than V (so phase 0
// compresses) and at most 64 of them
int32_t choose_m(int64_t E, int32_t V) {
    int64_t m = E / (8 * (int64_t)std::max(V, 1));
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(m, 64));
}

void run_request(br_server* S, Slot& sl, Request& r) {
    br_set_final_step(sl.ctx, r.mode);
    const int32_t* d = r.d_edges;
    if (!d && r.E > 0) {
        const size_t bytes = 8 * (size_t)r.E;
        if (sl.d_cap < bytes) {
            if (sl.d_buf) (void)hipFree(sl.d_buf);
            sl.d_buf = nullptr;
            sl.d_cap = 0;
            if (hipMalloc(&sl.d_buf, bytes) != hipSuccess) {
                (void)hipGetLastError();
                r.status = BR_ENOMEM;
                r.msg = "server: device allocation failed";
                return;
            }
            sl.d_cap = bytes;
        }
        // one asynchronous upload from the request's own copy (a DMA from the
        // pinned staging buffer; pageable copies go through the runtime's staging)
        const void* src = r.pin ? r.pin : static_cast<const void*>(r.h_edges.data());
        if (hipMemcpyAsync(sl.d_buf, src, bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess) {
            (void)hipGetLastError();
            r.status = BR_EHIP;
            r.msg = "server: upload failed";
            return;
        }
        d = static_cast<const int32_t*>(sl.d_buf);
    }
    r.bridges.resize(2 * (size_t)std::max(r.V - 1, 1));
    int64_t n = 0;
    r.status = br_bridges_find(sl.ctx, d, r.E, r.V, r.M, r.bridges.data(), std::max(r.V - 1, 1), &n, sl.stream);
    if (r.status != BR_OK) {
        r.msg = br_last_error();
        r.bridges.clear();
        return;
    }
    r.bridges.resize(2 * (size_t)n);
}

void slot_loop(br_server* S, Slot* sl) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> g(S->mu);
            S->cv_slot.wait(g, [&] { return S->stop || sl->job; });
            if (!sl->job) return;   // stopping and idle
            r = sl->job;
        }
        run_request(S, *sl, *r);
        {
            std::lock_guard<std::mutex> g(S->mu);
            r->latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
            r->done = true;
            r->h_edges.clear();
            r->h_edges.shrink_to_fit();
            if (r->pin) {                      // the stream was synchronised by the bridge search
                S->pin_free.emplace_back(r->pin, r->pin_cap);
                r->pin = nullptr;
            }
            // the slot keeps what it allocated; charge what it really holds
            const int64_t now = (int64_t)sl->ctx->ws.size + (int64_t)sl->d_cap;
            S->in_use += now - sl->held;
            sl->held = now;
            S->peak_in_use = std::max(S->peak_in_use, S->in_use);
            S->inflight--;
            if (S->inflight == 0) S->busy_ms += std::chrono::duration<double, std::milli>(Clock::now() - S->busy_start).count();
            if (r->status == BR_OK) {
                S->lat.push_back(r->latency_ms);
                S->edges_done += r->E;
            }
            sl->job.reset();
        }
        S->cv_sched.notify_one();
        S->cv_done.notify_all();
    }
}

// One tick of a lane worker: the edge lists of `batch` packed into one device
// buffer (uploads and device-to-device copies on the worker's stream, in
// request order), one batched query over all of them with plans built for
// this tick only, and the bridges split per request.
int lane_run(LaneWorker& L, const std::vector<std::shared_ptr<Request>>& batch, int mode) {
    const int32_t G = (int32_t)batch.size();
    std::vector<int64_t> eoff(G + 1, 0), boff(G + 1, 0);
    std::vector<int32_t> V(G);
    int64_t room = 0;
    for (int32_t g = 0; g < G; g++) {
        eoff[g + 1] = eoff[g] + batch[g]->E;
        V[g] = batch[g]->V;
        room += std::max(V[g] - 1, 0);
    }
    int32_t ndev = 0;
    for (int32_t g = 0; g < G; g++) ndev += (batch[g]->d_edges && batch[g]->E > 0) ? 1 : 0;
    const size_t ebytes = (8 * (size_t)eoff[G] + 255) & ~size_t(255);
    const size_t bytes = std::max<size_t>(ebytes + sizeof(GatherItem) * (size_t)ndev, 256);
    if (ndev > L.h_items_cap) {
        if (L.h_items) (void)hipHostFree(L.h_items);
        L.h_items = nullptr;
        L.h_items_cap = 0;
        int32_t c = 64;
        while (c < ndev) c *= 2;
        if (hipHostMalloc(reinterpret_cast<void**>(&L.h_items), sizeof(GatherItem) * (size_t)c, hipHostMallocDefault) !=
            hipSuccess) {
            (void)hipGetLastError();
            return fail(BR_ENOMEM, "server: pinned allocation failed");
        }
        L.h_items_cap = c;
    }
    if (L.cap < bytes) {
        if (L.buf) (void)hipFree(L.buf);
        L.buf = nullptr;
        L.cap = 0;
        if (hipMalloc(&L.buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(BR_ENOMEM, "server: device allocation failed");
        }
        L.cap = bytes;
    }
    int32_t* d = static_cast<int32_t*>(L.buf);
    // host sources: one upload each; device sources: one gather launch
    int32_t k = 0;
    int64_t longest = 0;
    for (int32_t g = 0; g < G; g++) {
        const Request& r = *batch[g];
        if (r.E == 0) continue;
        if (r.d_edges) {
            L.h_items[k++] = GatherItem{r.d_edges, eoff[g], r.E};
            longest = std::max(longest, r.E);
            continue;
        }
        const void* src = r.pin ? r.pin : static_cast<const void*>(r.h_edges.data());
        if (hipMemcpyAsync(d + 2 * eoff[g], src, 8 * (size_t)r.E, hipMemcpyHostToDevice, L.stream) != hipSuccess) {
            (void)hipGetLastError();
            return fail(BR_EHIP, "server: edge upload failed");
        }
    }
    if (k > 0) {
        GatherItem* d_items = reinterpret_cast<GatherItem*>(static_cast<char*>(L.buf) + ebytes);
        if (hipMemcpyAsync(d_items, L.h_items, sizeof(GatherItem) * (size_t)k, hipMemcpyHostToDevice, L.stream) !=
            hipSuccess) {
            (void)hipGetLastError();
            return fail(BR_EHIP, "server: gather table upload failed");
        }
        launch_gather_edges(d_items, k, longest, d, L.stream);
        if (hipGetLastError() != hipSuccess) return fail(BR_EHIP, "server: gather launch failed");
    }
    br_set_final_step(L.ctx, mode);
    std::vector<int32_t> out(2 * (size_t)std::max<int64_t>(room, 1));
    // the query's launches wait for the worker's stream, so the copies above
    // come first
    const int rc = batched_query(L.ctx, d, eoff.data(), V.data(), G, 0, out.data(), room, boff.data(), L.stream, true);
    if (rc != BR_OK) return rc;
    for (int32_t g = 0; g < G; g++)
        batch[g]->bridges.assign(out.begin() + 2 * boff[g], out.begin() + 2 * boff[g + 1]);
    return BR_OK;
}

// what a worker holds between ticks: its packed edge buffer and its context's
// plan arenas
int64_t lane_held_now(const LaneWorker& L) { return (int64_t)L.cap + (int64_t)batched_device_bytes(L.ctx); }

void lane_loop(br_server* S, LaneWorker* L) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        int mode = 1;
        {
            std::unique_lock<std::mutex> g(S->mu);
            S->cv_lane.wait(g, [&] { return S->stop || (!S->lane_q.empty() && !L->trimming); });
            if (S->lane_q.empty()) return;   // stopping and idle
            // everything queued, up to the first request that was admitted
            // with the other final step
            mode = S->lane_q.front()->mode;
            while (!S->lane_q.empty() && S->lane_q.front()->mode == mode) {
                batch.push_back(S->lane_q.front());
                S->lane_q.pop_front();
            }
            L->busy = true;
        }
        int rc = lane_run(*L, batch, mode);
        (void)hipStreamSynchronize(L->stream);   // its copies are done whatever the outcome
        if (rc != BR_OK) {
            // an error of one request (an id out of range, say) must not fail
            // the others: each runs again on its own
            if (batch.size() == 1) {
                batch[0]->status = rc;
                batch[0]->msg = br_last_error();
            } else {
                for (auto& r : batch) {
                    const int rc1 = lane_run(*L, {r}, mode);
                    if (rc1 != BR_OK) {
                        r->status = rc1;
                        r->msg = br_last_error();
                    }
                }
            }
        }
        {
            std::lock_guard<std::mutex> g(S->mu);
            const auto now = Clock::now();
            int64_t charged = 0;
            for (auto& r : batch) {
                r->latency_ms = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
                r->done = true;
                if (r->status != BR_OK) r->bridges.clear();
                r->h_edges.clear();
                r->h_edges.shrink_to_fit();
                if (r->pin) {
                    S->pin_free.emplace_back(r->pin, r->pin_cap);
                    r->pin = nullptr;
                }
                charged += r->lane_bytes;
                if (r->status == BR_OK) {
                    S->lat.push_back(r->latency_ms);
                    S->edges_done += r->E;
                }
            }
            // the tick's charges go; what the worker keeps is charged instead
            const int64_t held = lane_held_now(*L);
            S->in_use += held - L->held - charged;
            L->held = held;
            S->peak_in_use = std::max(S->peak_in_use, S->in_use);
            S->inflight -= (int64_t)batch.size();
            if (S->inflight == 0) S->busy_ms += std::chrono::duration<double, std::milli>(now - S->busy_start).count();
            S->ticks++;
            S->lane_requests += (int64_t)batch.size();
            L->busy = false;
        }
        S->cv_sched.notify_one();
        S->cv_done.notify_all();
        S->cv_lane.notify_all();
    }
}

// release what an idle lane worker holds (scheduler thread, no tick running)
void release_lane(br_server* S, LaneWorker& L) {
    (void)hipSetDevice(S->device);
    (void)hipStreamSynchronize(L.stream);
    batched_release(L.ctx);
    if (L.buf) (void)hipFree(L.buf);
    L.buf = nullptr;
    L.cap = 0;
    (void)hipGetLastError();
}

// The free slot for r that needs the fewest new bytes, and that number.
Slot* pick_slot(br_server* S, const Request& r, int64_t* extra) {
    Slot* best = nullptr;
    for (auto& s : S->slots) {
        if (s->job || s->trimming) continue;
        const int64_t x = held_after(*s, r) - s->held;
        if (!best || x < *extra) {
            best = s.get();
            *extra = x;
        }
    }
    return best;
}

// Release idle holders of device memory -- slots not running a request and
// lane workers not running a tick -- largest first, until `extra` more bytes
// fit the budget.  `keep` (the slot about to be used) goes last, and only when
// nothing runs.  Returns whether anything was released (the lock is dropped
// meanwhile: the caller decides again).
bool trim(br_server* S, std::unique_lock<std::mutex>& g, int64_t extra, Slot* keep) {
    struct Holder { Slot* slot; LaneWorker* lane; int64_t held; };
    std::vector<Holder> idle;
    for (auto& s : S->slots)
        if (!s->job && !s->trimming && s.get() != keep && s->held > 0) idle.push_back({s.get(), nullptr, s->held});
    for (auto& l : S->lanes)
        if (!l->busy && !l->trimming && l->held > 0) idle.push_back({nullptr, l.get(), l->held});
    std::sort(idle.begin(), idle.end(), [](const Holder& a, const Holder& b) { return a.held > b.held; });
    std::vector<Holder> rel;
    int64_t freed = 0;
    for (const Holder& h : idle) {
        if (S->in_use - freed + extra <= S->budget) break;
        rel.push_back(h);
        freed += h.held;
    }
    if (S->in_use - freed + extra > S->budget && S->inflight == 0 && keep && keep->held > 0)
        rel.push_back({keep, nullptr, keep->held});   // nothing runs: the chosen slot starts over from nothing too
    if (rel.empty()) return false;
    for (const Holder& h : rel) (h.slot ? h.slot->trimming : h.lane->trimming) = true;
    g.unlock();
    for (const Holder& h : rel) {
        if (h.slot) release_slot(*h.slot);
        else release_lane(S, *h.lane);
    }
    g.lock();
    for (const Holder& h : rel) {
        if (h.slot) {
            S->in_use -= h.slot->held;
            h.slot->held = 0;
            h.slot->trimming = false;
        } else {
            S->in_use -= h.lane->held;
            h.lane->held = 0;
            h.lane->trimming = false;
        }
    }
    S->cv_lane.notify_all();
    return true;
}

// put r on slot sl (scheduler thread, lock held, budget checked)
void admit_slot(br_server* S, Slot* sl, std::shared_ptr<Request> r) {
    const int64_t after = held_after(*sl, *r);
    S->in_use += after - sl->held;
    sl->held = after;
    S->peak_in_use = std::max(S->peak_in_use, S->in_use);
    sl->job = std::move(r);
    if (S->inflight == 0) S->busy_start = Clock::now();
    S->inflight++;
    S->peak_inflight = std::max(S->peak_inflight, S->inflight);
    S->cv_slot.notify_all();
}

void sched_loop(br_server* S) {
    std::unique_lock<std::mutex> g(S->mu);
    for (;;) {
        S->cv_sched.wait(g, [&] {
            if (S->stop) return true;
            if (S->queue.empty()) return false;
            if (S->queue.front()->lane) return true;
            for (auto& s : S->slots)
                if (!s->job && !s->trimming) return true;
            return false;
        });
        if (S->stop) return;
        auto r = S->queue.front();
        r->mode = S->final_step;
        if (r->lane) {
            // a free slot that has room takes it while the lane has nothing queued
            bool free_slot = false;
            if (S->lane_q.empty()) {
                charge(*r, r->d_edges == nullptr, r->mode, S->device);
                int64_t extra = 0;
                Slot* sl = pick_slot(S, *r, &extra);
                if (sl && S->in_use + extra <= S->budget) {
                    S->queue.pop_front();
                    admit_slot(S, sl, std::move(r));
                    continue;
                }
                free_slot = sl != nullptr;
            }
            // no slot: the lane takes it once requests back up (as many
            // waiting as there are slots) and for as long as it is working;
            // otherwise waiting for a slot is quicker than a tick (small
            // requests at 20k QPS: p50 0.49 ms on slots against 1.36 ms when
            // every overflow went to the lane)
            bool lane_busy = !S->lane_q.empty();
            for (auto& l : S->lanes) lane_busy = lane_busy || l->busy;
            if (!free_slot && !lane_busy && S->queue.size() < S->slots.size() && S->inflight > 0) {
                S->cv_sched.wait(g);
                continue;
            }
            // the batch lane: charged its estimate until its tick completes
            const int64_t need = lane_need(*r);
            if (S->in_use + need > S->budget) {
                if (trim(S, g, need, nullptr)) continue;
                if (S->inflight > 0) {
                    S->cv_sched.wait(g);
                    continue;
                }
                // nothing runs: one that exceeds the budget on its own runs alone
            }
            S->queue.pop_front();
            r->lane_bytes = need;
            S->in_use += need;
            S->peak_in_use = std::max(S->peak_in_use, S->in_use);
            S->lane_q.push_back(r);
            if (S->inflight == 0) S->busy_start = Clock::now();
            S->inflight++;
            S->peak_inflight = std::max(S->peak_inflight, S->inflight);
            S->cv_lane.notify_one();
            continue;
        }
        charge(*r, r->d_edges == nullptr, r->mode, S->device);
        int64_t extra = 0;
        Slot* sl = pick_slot(S, *r, &extra);
        if (S->in_use + extra > S->budget) {
            if (trim(S, g, extra, sl)) continue;   // decide again with the memory released
            // one that exceeds the budget on its own runs alone
            if (S->inflight > 0) {
                S->cv_sched.wait(g);
                continue;
            }
        }
        // admit the head (FIFO)
        S->queue.pop_front();
        admit_slot(S, sl, std::move(r));
    }
}

int enqueue(br_server* S, std::shared_ptr<Request> r, uint64_t* ticket) {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->queue.size() >= kQueueMax) return fail(BR_EBUSY, "server: queue full (%zu requests)", S->queue.size());
    r->ticket = S->next_ticket++;
    r->t_submit = Clock::now();
    S->queue.push_back(r);
    S->all[r->ticket] = r;
    *ticket = r->ticket;
    S->cv_sched.notify_one();
    return BR_OK;
}

int take(br_server* S, uint64_t ticket, int32_t* h_out, int64_t cap, int64_t* n, bool wait, int* done) {
    std::unique_lock<std::mutex> g(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(BR_EINVAL, "server: unknown ticket %llu", (unsigned long long)ticket);
    auto r = it->second;
    if (wait) S->cv_done.wait(g, [&] { return r->done; });
    if (done) *done = r->done ? 1 : 0;
    if (!r->done) return BR_OK;
    if (r->status != BR_OK) {
        const int st = r->status;
        const std::string msg = r->msg;
        S->all.erase(it);
        return fail(st, "%s", msg.c_str());
    }
    const int64_t nb = (int64_t)r->bridges.size() / 2;
    *n = nb;
    if (nb > cap) return fail(BR_ECAP, "server: %lld bridges, capacity %lld", (long long)nb, (long long)cap);
    std::copy(r->bridges.begin(), r->bridges.end(), h_out);
    S->all.erase(it);
    return BR_OK;
}

}  // namespace
}  // namespace br

using namespace br;

extern "C" {

int br_server_create(br_server** out, int device, int64_t mem_budget, int32_t max_slots) {
    if (!out || mem_budget <= 0 || max_slots < 1 || max_slots > 64) return fail(BR_EINVAL, "br_server_create: bad argument");
    *out = nullptr;
    auto S = std::make_unique<br_server>();
    S->device = device;
    S->budget = mem_budget;
    S->pin_limit = std::min<int64_t>(mem_budget / 4, (int64_t)8 << 30);
    S->copier = std::make_unique<Pool>(8);
    for (int32_t i = 0; i < max_slots; i++) {
        auto sl = std::make_unique<Slot>();
        int rc = br_create(&sl->ctx, device);
        if (rc) {
            for (auto& s : S->slots) br_destroy(s->ctx);
            return rc;
        }
        sl->ctx->exact_ws = true;
        if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) {
            br_destroy(sl->ctx);
            for (auto& s : S->slots) br_destroy(s->ctx);
            return hip_fail(hipGetLastError(), "hipStreamCreate");
        }
        S->slots.push_back(std::move(sl));
    }
    for (int i = 0; i < kLaneWorkers; i++) {
        auto L = std::make_unique<LaneWorker>();
        int rc = br_create(&L->ctx, device);
        if (rc == BR_OK && hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess)
            rc = hip_fail(hipGetLastError(), "hipStreamCreate");
        if (rc) {
            if (L->ctx) br_destroy(L->ctx);
            for (auto& l : S->lanes) {
                (void)hipStreamDestroy(l->stream);
                br_destroy(l->ctx);
            }
            for (auto& s : S->slots) {
                (void)hipStreamDestroy(s->stream);
                br_destroy(s->ctx);
            }
            return rc;
        }
        S->lanes.push_back(std::move(L));
    }
    S->lane_max_v = batched_max_v_big();
    S->lane_max_e = kLaneMaxEdges;
    br_server* raw = S.release();
    for (auto& sl : raw->slots) sl->th = std::thread(slot_loop, raw, sl.get());
    for (auto& l : raw->lanes) l->th = std::thread(lane_loop, raw, l.get());
    raw->sched = std::thread(sched_loop, raw);
    *out = raw;
    return BR_OK;
}

static int submit_common(br_server* S, std::shared_ptr<Request> r, uint64_t* ticket, bool host) {
    r->M = choose_m(r->E, r->V);
    {
        std::lock_guard<std::mutex> g(S->mu);
        r->lane = lane_fits(S, *r);
    }
    int64_t need = 0;
    if (r->lane) {
        need = lane_need(*r);
    } else {
        charge(*r, host, 1, S->device);   // the larger of the two final steps' needs
        need = r->ws_bytes + r->buf_bytes;
    }
    if (need > S->budget)
        return fail(BR_ENOMEM, "server: request needs %lld bytes, budget is %lld", (long long)need, (long long)S->budget);
    return enqueue(S, std::move(r), ticket);
}

int br_submit(br_server* S, const int32_t* h_edges, int64_t E, int32_t V, uint64_t* ticket) {
    if (!S || !ticket || E < 0 || V < 1 || (E > 0 && !h_edges)) return fail(BR_EINVAL, "br_submit: bad argument");
    auto r = std::make_shared<Request>();
    r->E = E;
    r->V = V;
    const size_t bytes = 8 * (size_t)E;
    auto pb = E > 0 ? acquire_pinned(S, bytes) : std::pair<void*, size_t>{nullptr, 0};
    if (pb.first) {
        parallel_copy(S, pb.first, h_edges, bytes);
        r->pin = pb.first;
        r->pin_cap = pb.second;
    } else {
        r->h_edges.assign(h_edges, h_edges + 2 * E);
    }
    const int rc = submit_common(S, r, ticket, true);
    if (rc != BR_OK && r->pin) {                // not queued: the buffer goes back to the pool
        std::lock_guard<std::mutex> g(S->mu);
        S->pin_free.emplace_back(r->pin, r->pin_cap);
        r->pin = nullptr;
    }
    return rc;
}

int br_submit_device(br_server* S, const int32_t* d_edges, int64_t E, int32_t V, uint64_t* ticket) {
    if (!S || !ticket || E < 0 || V < 1 || (E > 0 && !d_edges)) return fail(BR_EINVAL, "br_submit_device: bad argument");
    auto r = std::make_shared<Request>();
    r->E = E;
    r->V = V;
    r->d_edges = d_edges;
    return submit_common(S, std::move(r), ticket, false);
}

int br_poll(br_server* S, uint64_t ticket, int32_t* h_out, int64_t cap, int64_t* n, int* done) {
    if (!S || !n || !done || cap < 0 || (cap > 0 && !h_out)) return fail(BR_EINVAL, "br_poll: bad argument");
    return take(S, ticket, h_out, cap, n, false, done);
}

int br_wait(br_server* S, uint64_t ticket, int32_t* h_out, int64_t cap, int64_t* n) {
    if (!S || !n || cap < 0 || (cap > 0 && !h_out)) return fail(BR_EINVAL, "br_wait: bad argument");
    return take(S, ticket, h_out, cap, n, true, nullptr);
}

int br_server_stats(br_server* S, br_server_stats_t* out, int reset) {
    if (!S || !out) return fail(BR_EINVAL, "br_server_stats: bad argument");
    std::lock_guard<std::mutex> g(S->mu);
    std::vector<double> l = S->lat;
    std::sort(l.begin(), l.end());
    std::memset(out, 0, sizeof *out);
    out->completed = (int64_t)l.size();
    if (!l.empty()) {
        auto pct = [&](double p) { return l[std::min(l.size() - 1, (size_t)(p * (l.size() - 1) + 0.5))]; };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double s = 0;
        for (double x : l) s += x;
        out->mean_ms = s / l.size();
        out->max_ms = l.back();
    }
    double busy = S->busy_ms;
    if (S->inflight > 0) busy += std::chrono::duration<double, std::milli>(Clock::now() - S->busy_start).count();
    out->edges_per_s = busy > 0 ? S->edges_done / (busy / 1000.0) : 0.0;
    out->peak_inflight = S->peak_inflight;
    out->device_bytes = S->in_use;
    out->peak_device_bytes = S->peak_in_use;
    out->batched_ticks = S->ticks;
    out->batched_requests = S->lane_requests;
    if (reset) {
        S->lat.clear();
        S->edges_done = 0;
        S->busy_ms = 0;
        S->peak_inflight = S->inflight;
        S->peak_in_use = S->in_use;
        S->ticks = 0;
        S->lane_requests = 0;
        if (S->inflight > 0) S->busy_start = Clock::now();
    }
    return BR_OK;
}

int br_server_set_batching(br_server* S, int32_t max_v, int64_t max_e) {
    if (!S || max_v < 0 || max_v > batched_max_v_big() || max_e < 0)
        return fail(BR_EINVAL, "br_server_set_batching: need 0 <= max_v <= %d and max_e >= 0", (int)batched_max_v_big());
    std::lock_guard<std::mutex> g(S->mu);
    S->lane_max_v = max_v;    // taken by each request when it is submitted
    S->lane_max_e = max_e;
    return BR_OK;
}

int br_server_set_final_step(br_server* S, int mode) {
    if (!S || mode < 0 || mode > 1) return fail(BR_EINVAL, "br_server_set_final_step: bad argument");
    std::lock_guard<std::mutex> g(S->mu);
    S->final_step = mode;     // taken by each request when it is admitted
    return BR_OK;
}

int br_server_destroy(br_server* S) {
    if (!S) return BR_OK;
    {
        std::unique_lock<std::mutex> g(S->mu);
        // finish what is queued or running
        S->cv_done.wait(g, [&] { return S->queue.empty() && S->inflight == 0; });
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->cv_slot.notify_all();
    S->cv_lane.notify_all();
    if (S->sched.joinable()) S->sched.join();
    for (auto& l : S->lanes) {
        if (l->th.joinable()) l->th.join();
        (void)hipStreamSynchronize(l->stream);
        (void)hipStreamDestroy(l->stream);
        if (l->buf) (void)hipFree(l->buf);
        if (l->h_items) (void)hipHostFree(l->h_items);
        br_destroy(l->ctx);
    }
    for (auto& sl : S->slots) {
        if (sl->th.joinable()) sl->th.join();
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
        if (sl->d_buf) (void)hipFree(sl->d_buf);
        br_destroy(sl->ctx);
    }
    for (auto& b : S->pin_free) (void)hipHostFree(b.first);
    delete S;
    return BR_OK;
}

}  // extern "C"
