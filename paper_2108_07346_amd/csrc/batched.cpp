// Batched bridge queries: G independent graphs, one persistent launch.
//
// Host side of the batched path: plans the per-graph phase trees (chunks of
// chunk_edges edges, node regions, merge counters), orders the work items
// largest-first, captures "clear counters -> persistent kernel -> copy
// certificates to the host" in a HIP graph that is replayed while the batch
// shape and input buffer stay the same, then runs the final depth-first
// search of every graph on a pool of host threads.  chunk_edges = 0 asks the
// library's tuner, which times candidate chunk sizes and workgroups per CU on
// the batch itself and remembers the winner per device and batch shape
// (tuner.cpp).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "internal.hpp"

namespace br {



namespace {

// simple fixed pool of host threads for the final search


struct BatchPlan {
    // key
    int32_t G = 0, C = 0, bpc = 0;
    bool big = false;                // the class of graphs above the small kernel's V (160 KB kernel)
    std::vector<int64_t> eoff;
    std::vector<int32_t> V;
    // small graphs are the ones certified in LDS; the others go through br_bridges_find
    std::vector<int32_t> small, large;
    std::vector<int32_t> Mg;
    std::vector<int64_t> rbase, cbase, noff, ncap, items;
    int64_t nodes = 0, counters = 0, area0 = 0, cert_pairs = 0;
    // device memory: [clear block: ncnt | arrive | queue | err][meta][cert]
    void* dmem = nullptr;
    size_t clear_words = 0;
    BatchDev dev{};
    // pinned host: node-0 regions + node-0 counters + err
    void* hmem = nullptr;
    int2* h_area0 = nullptr;
    uint32_t* h_cnt0 = nullptr;
    uint32_t* h_err = nullptr;
    // final step on the device: the certificates of all small graphs as one
    // certificate of their disjoint union (vertex ids shifted by vbase)
    std::vector<int64_t> vbase;      // [S+1]
    int64_t vtot = 0;
    // final step on the device: per graph bridge keys (u << 16 | v, sorted) in
    // one array; header word 0 = number of keys, words 16 + 2s, 17 + 2s = base
    // and count of small graph s; the keys follow the header directly
    uint32_t* d_sb = nullptr;
    uint32_t* h_sb = nullptr;
    int32_t* d_lists = nullptr;      // small graphs by size class: [na] then [nb]
    int32_t na = 0, nb = 0;
    int cus = 1;
    int64_t sb_hdr = 0;              // header words (16 + 2S)
    int64_t sb_keys = 0;             // room for keys: sum of (V_s - 1)
    size_t keys_hint = 0;            // keys of the previous call (size of the first copy)
    // captured launches: the persistent kernel, then (final step on the device)
    // the combined certificate and its bridge step, with an event in between
    hipGraph_t graph = nullptr, graph2 = nullptr;
    hipGraphExec_t exec = nullptr, exec2 = nullptr;
    const void* graph_edges = nullptr;
    int graph_mode = -1;
    int blocks = 0;
    // big class, final step on the device: the node-0 certificates as one
    // certificate of their disjoint union and one bridge step over it
    int2 *d_f1u = nullptr, *d_f2u = nullptr;
    uint32_t* d_cntu = nullptr;
    int64_t* d_uoff = nullptr;
    int32_t* d_bws = nullptr;
    uint64_t* d_ukeys = nullptr;     // set when the step is enqueued
    uint32_t* d_un = nullptr;        // key count (status word 1; the status block precedes the keys)
    uint32_t* h_ustat = nullptr;     // pinned: status block + keys
    int32_t max_v = 0;
    bool owns = true;                // dmem / hmem allocated for this plan (else borrowed arenas)
    size_t dbytes = 0;
    ~BatchPlan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (exec2) (void)hipGraphExecDestroy(exec2);
        if (graph2) (void)hipGraphDestroy(graph2);
        if (owns && dmem) (void)hipFree(dmem);
        if (owns && hmem) (void)hipHostFree(hmem);
    }
};

struct BatchState {
    std::unique_ptr<Pool> pool;
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;           // second branch of the captured final step (default priority)
    hipEvent_t fork = nullptr, join = nullptr;
    hipEvent_t ready = nullptr;              // the caller's stream has produced the input
    std::vector<std::unique_ptr<BatchPlan>> plans;      // small LRU
    std::vector<DfsScratch> scratch;
    std::vector<std::vector<uint64_t>> keys;
    std::unique_ptr<uint64_t[]> outk;           // per-graph bridge slots (reused, never zero-filled)
    size_t outk_n = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEvent_t k0 = nullptr, k1 = nullptr;   // around the persistent kernel's graph (counter clear + kernel)
    hipEvent_t k2 = nullptr;                 // after the bridge step's graph
    // arenas of the plans built for one call only (serving), one per size
    // class: grown, never shrunk
    struct Arena {
        void* arena_d = nullptr;
        size_t arena_d_cap = 0;
        void* arena_h = nullptr;
        size_t arena_h_cap = 0;
    } arenas[2];
    std::unique_ptr<BatchPlan> transient[2];
};

BatchState* state_of(br_ctx* c) {
    if (!c->batched) c->batched = new BatchState();
    return static_cast<BatchState*>(c->batched);
}

int64_t part_lo(int64_t E, int64_t M, int64_t i) { return i * (E / M) + (i * (E % M)) / M; }

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Plan of one class of the batch: the small class takes the graphs with
// V <= batched_max_v_dev() (and lists those above batched_max_v_big() as
// `large`, for the plain path); the big class the graphs in between.
int build_plan(BatchPlan& P, const int64_t* eoff, const int32_t* V, int32_t G, int32_t C, int32_t bpc, int cus,
               bool big, BatchState::Arena* arena, hipStream_t upload) {
    P.G = G;
    P.C = C;
    P.bpc = bpc;
    P.big = big;
    P.eoff.assign(eoff, eoff + G + 1);
    P.V.assign(V, V + G);
    const int32_t lo = big ? batched_max_v_dev() : 0, hi = big ? batched_max_v_big() : batched_max_v_dev();
    for (int32_t g = 0; g < G; g++) {
        if (V[g] > lo && V[g] <= hi) P.small.push_back(g);
        else if (!big && V[g] > batched_max_v_big()) P.large.push_back(g);
    }
    for (int32_t g : P.small) P.max_v = std::max(P.max_v, V[g]);
    const int32_t S = (int32_t)P.small.size();
    // per small graph (indexed by position s in P.small): chunks, nodes, counters
    P.Mg.resize(S);
    P.rbase.resize(S);
    P.cbase.resize(S);
    int64_t rest = S, ctr = 0;
    for (int32_t s = 0; s < S; s++) {
        const int64_t E = eoff[P.small[s] + 1] - eoff[P.small[s]];
        const int64_t M = std::max<int64_t>(1, (E + C - 1) / C);
        if (M >= (1 << 20)) return fail(BR_EINVAL, "batched: graph %d needs %lld chunks", P.small[s], (long long)M);
        P.Mg[s] = (int32_t)M;
        P.rbase[s] = rest;
        rest += M - 1;
        int R = 0;
        while ((int64_t(1) << R) < M) R++;
        P.cbase[s] = ctr;
        ctr += (int64_t)R * ((M + 1) / 2);
    }
    P.nodes = rest;
    P.counters = ctr;
    P.noff.assign(P.nodes, 0);
    P.ncap.assign(P.nodes, 0);
    // node-0 regions first (one contiguous copy to the host), then the others
    int64_t acc = 0;
    for (int pass = 0; pass < 2; pass++) {
        for (int32_t s = 0; s < S; s++) {
            const int32_t g = P.small[s];
            const int64_t E = eoff[g + 1] - eoff[g], M = P.Mg[s], bound = 2 * (int64_t(V[g]) - 1);
            for (int64_t i = (pass == 0 ? 0 : 1); i < (pass == 0 ? 1 : M); i++) {
                int64_t span = M;
                if (i) span = std::min<int64_t>(int64_t(1) << __builtin_ctzll((unsigned long long)i), M - i);
                const int64_t cap = std::min(part_lo(E, M, std::min<int64_t>(M, i + span)) - part_lo(E, M, i), bound);
                const int64_t idx = i ? P.rbase[s] + i - 1 : s;
                P.noff[idx] = acc;
                P.ncap[idx] = cap;
                acc += cap;
            }
        }
        if (pass == 0) P.area0 = acc;
    }
    P.cert_pairs = acc;
    // items, largest chunk first (ties: graph order)
    struct It { int64_t len, code; };
    std::vector<It> its;
    for (int32_t s = 0; s < S; s++) {
        const int32_t g = P.small[s];
        const int64_t E = eoff[g + 1] - eoff[g], M = P.Mg[s];
        for (int64_t k = 0; k < M; k++) its.push_back({part_lo(E, M, k + 1) - part_lo(E, M, k), ((int64_t)s << 20) | k});
    }
    std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) { return a.len > b.len; });
    P.items.resize(its.size());
    for (size_t i = 0; i < its.size(); i++) P.items[i] = its[i].code;
    // device memory: [clear block | metadata uploaded in one copy | the rest]
    P.clear_words = 2 * (size_t)P.nodes + (size_t)P.counters + 2;
    P.vbase.assign((size_t)S + 1, 0);
    for (int32_t s = 0; s < S; s++) P.vbase[s + 1] = P.vbase[s] + V[P.small[s]];
    P.vtot = P.vbase[S];
    if (P.vtot >= (int64_t(1) << 30)) return fail(BR_EINVAL, "batched: %lld vertices in one batch", (long long)P.vtot);
    P.sb_hdr = 16 + 2 * (int64_t)S;
    P.sb_keys = std::max<int64_t>(1, P.vtot - S);   // sum of (V_s - 1): every bridge of every graph
    const size_t o_clear = 0;
    size_t o = a256(o_clear + 4 * P.clear_words);
    const size_t o_meta = o;
    const size_t o_eoff = o; o = a256(o + 8 * 2 * (size_t)std::max(S, 1));
    const size_t o_V = o; o = a256(o + 4 * (size_t)S);
    const size_t o_M = o; o = a256(o + 4 * (size_t)S);
    const size_t o_rb = o; o = a256(o + 8 * (size_t)S);
    const size_t o_cb = o; o = a256(o + 8 * (size_t)S);
    const size_t o_noff = o; o = a256(o + 8 * (size_t)P.nodes);
    const size_t o_ncap = o; o = a256(o + 8 * (size_t)P.nodes);
    const size_t o_items = o; o = a256(o + 8 * std::max<size_t>(P.items.size(), 1));
    const size_t o_vb = o; o = a256(o + 8 * (size_t)(S + 1));
    const size_t o_lists = o; if (!big) o = a256(o + 4 * (size_t)std::max(S, 1));
    const size_t meta_bytes = o - o_meta;
    const size_t o_cert = o; o = a256(o + 8 * (size_t)std::max<int64_t>(P.cert_pairs, 1));
    const size_t o_root = o; o = a256(o + 4 * (size_t)std::max<int64_t>(P.vtot, 1));
    const size_t o_sb = o; if (!big) o = a256(o + 4 * (size_t)(P.sb_hdr + P.sb_keys));
    size_t o_f1u = o, o_f2u = o, o_cntu = o, o_uoff = o, o_bws = o;
    if (big && S) {
        o_f1u = o; o = a256(o + 8 * (size_t)P.vtot);
        o_f2u = o; o = a256(o + 8 * (size_t)P.vtot);
        o_cntu = o; o = a256(o + 8);
        o_uoff = o; o = a256(o + 8 * 2 * (size_t)S);
        o_bws = o; o = a256(o + 4 * (size_t)device_bridges_words((int32_t)P.vtot));
    }
    // pinned host staging: node-0 regions, node-0 counters, error word, keys;
    // then room for the metadata's one upload
    const size_t h_keys = a256(8 * (size_t)std::max<int64_t>(P.area0, 1)) + a256(8 * (size_t)std::max(S, 1)) + 256;
    const size_t h_meta = h_keys + (big ? a256(256 + 8 * (size_t)std::max<int64_t>(P.vtot, 1))
                                        : a256(4 * (size_t)(P.sb_hdr + P.sb_keys)));
    const size_t hbytes = h_meta + a256(meta_bytes);
    if (arena) {
        // a plan for one call: the batch state's arenas (grown when too small)
        if (arena->arena_d_cap < o) {
            if (arena->arena_d) BR_HIP(hipFree(arena->arena_d));
            arena->arena_d = nullptr;
            arena->arena_d_cap = 0;
            BR_HIP(hipMalloc(&arena->arena_d, o));
            arena->arena_d_cap = o;
        }
        if (arena->arena_h_cap < hbytes) {
            if (arena->arena_h) BR_HIP(hipHostFree(arena->arena_h));
            arena->arena_h = nullptr;
            arena->arena_h_cap = 0;
            BR_HIP(hipHostMalloc(&arena->arena_h, hbytes, hipHostMallocDefault));
            arena->arena_h_cap = hbytes;
        }
        P.dmem = arena->arena_d;
        P.hmem = arena->arena_h;
        P.owns = false;
    } else {
        BR_HIP(hipMalloc(&P.dmem, o));
        BR_HIP(hipHostMalloc(&P.hmem, hbytes, hipHostMallocDefault));
        P.owns = true;
    }
    P.dbytes = o;
    char* d = static_cast<char*>(P.dmem);
    char* h = static_cast<char*>(P.hmem);
    {
        // metadata assembled in pinned memory with the device layout, one copy
        char* m = h + h_meta;
        auto put = [&](size_t off, const void* src, size_t n) { if (n) std::memcpy(m + (off - o_meta), src, n); };
        std::vector<int32_t> sV(S);
        std::vector<int64_t> se2(2 * (size_t)S);     // graph s: edges [se2[2s], se2[2s+1])
        for (int32_t s = 0; s < S; s++) {
            sV[s] = V[P.small[s]];
            se2[2 * s] = eoff[P.small[s]];
            se2[2 * s + 1] = eoff[P.small[s] + 1];
        }
        put(o_eoff, se2.data(), 8 * 2 * (size_t)S);
        put(o_V, sV.data(), 4 * (size_t)S);
        put(o_M, P.Mg.data(), 4 * (size_t)S);
        put(o_rb, P.rbase.data(), 8 * (size_t)S);
        put(o_cb, P.cbase.data(), 8 * (size_t)S);
        put(o_noff, P.noff.data(), 8 * (size_t)P.nodes);
        put(o_ncap, P.ncap.data(), 8 * (size_t)P.nodes);
        put(o_items, P.items.data(), 8 * P.items.size());
        put(o_vb, P.vbase.data(), 8 * (size_t)S);
        if (!big) {
            std::vector<int32_t> la, lb;
            for (int32_t s = 0; s < S; s++) (V[P.small[s]] <= small_bridges_split_v() ? la : lb).push_back(s);
            P.na = (int32_t)la.size();
            P.nb = (int32_t)lb.size();
            la.insert(la.end(), lb.begin(), lb.end());
            put(o_lists, la.data(), 4 * (size_t)S);
        }
        // ordered before the plan's launches (the same stream); the pinned
        // source is rewritten only by a later call, after that call's wait
        BR_HIP(hipMemcpyAsync(d + o_meta, m, meta_bytes, hipMemcpyHostToDevice, upload));
    }
    P.d_sb = reinterpret_cast<uint32_t*>(d + o_sb);
    P.d_lists = reinterpret_cast<int32_t*>(d + o_lists);
    if (big && S) {
        P.d_f1u = reinterpret_cast<int2*>(d + o_f1u);
        P.d_f2u = reinterpret_cast<int2*>(d + o_f2u);
        P.d_cntu = reinterpret_cast<uint32_t*>(d + o_cntu);
        P.d_uoff = reinterpret_cast<int64_t*>(d + o_uoff);
        P.d_bws = reinterpret_cast<int32_t*>(d + o_bws);
    }
    P.cus = std::max(1, cus);
    uint32_t* clr = reinterpret_cast<uint32_t*>(d + o_clear);
    P.dev.eoff = reinterpret_cast<const int64_t*>(d + o_eoff);
    P.dev.V = reinterpret_cast<const int32_t*>(d + o_V);
    P.dev.Mg = reinterpret_cast<const int32_t*>(d + o_M);
    P.dev.rbase = reinterpret_cast<const int64_t*>(d + o_rb);
    P.dev.cbase = reinterpret_cast<const int64_t*>(d + o_cb);
    P.dev.noff = reinterpret_cast<const int64_t*>(d + o_noff);
    P.dev.ncap = reinterpret_cast<const int64_t*>(d + o_ncap);
    P.dev.items = reinterpret_cast<const int64_t*>(d + o_items);
    P.dev.n_items = (int64_t)P.items.size();
    P.dev.cert = reinterpret_cast<int2*>(d + o_cert);
    P.dev.ncnt = clr;
    P.dev.arrive = clr + 2 * P.nodes;
    P.dev.queue = clr + 2 * P.nodes + P.counters;
    P.dev.err = P.dev.queue + 1;
    P.dev.vbase = reinterpret_cast<const int64_t*>(d + o_vb);
    P.dev.rootw = reinterpret_cast<uint32_t*>(d + o_root);
    P.h_area0 = reinterpret_cast<int2*>(h);
    P.h_cnt0 = reinterpret_cast<uint32_t*>(h + a256(8 * (size_t)std::max<int64_t>(P.area0, 1)));
    P.h_err = P.h_cnt0 + 2 * (size_t)std::max(S, 1);
    P.h_sb = reinterpret_cast<uint32_t*>(h + a256(8 * (size_t)std::max<int64_t>(P.area0, 1)) +
                                         a256(8 * (size_t)std::max(S, 1)) + 256);
    P.h_ustat = P.h_sb;                  // big class: the same room holds the status block and the keys
    // the big class fills one workgroup per CU (its LDS)
    P.blocks = std::max(1, big ? cus : cus * bpc);
    return BR_OK;
}

// enqueue clear -> kernel -> copies on s (captured into P.graph on first use)
// the captured part: clear the counters, the persistent kernel, and with the
// final step on the device the combined certificate and its bridge step
int enqueue(BatchPlan& P, const int32_t* d_edges, hipStream_t s, int mode, int part, BatchState* st) {
    P.dev.edges = reinterpret_cast<const int2*>(d_edges);
    if (part == 0) {
        launch_fill_u32(P.dev.ncnt, (int64_t)P.clear_words, 0u, s);
        BR_HIP(hipGetLastError());
        if (P.dev.n_items) launch_batched(P.dev, P.blocks, s, P.big);
        BR_HIP(hipGetLastError());
        return BR_OK;
    }
    if (mode == 1 && P.big && !P.small.empty()) {
        const int32_t S = (int32_t)P.small.size();
        launch_union_certificate(P.dev, S, P.d_uoff, P.d_f1u, P.d_f2u, P.d_cntu, s);
        BR_HIP(hipGetLastError());
        int rc = device_bridges_cert(P.d_f1u, P.d_f2u, 1, P.d_cntu, P.dev.rootw, 1, (int32_t)P.vtot, P.dev.err, P.d_bws,
                                     &P.d_ukeys, &P.d_un, s);
        if (rc) return rc;
        BR_HIP(hipGetLastError());
        return BR_OK;
    }
    if (mode == 1 && !P.small.empty()) {
        launch_fill_u32(P.d_sb, 16, 0u, s);
        // fork: the two size classes run side by side, then join back on s
        BR_HIP(hipEventRecord(st->fork, s));
        BR_HIP(hipStreamWaitEvent(st->stream2, st->fork, 0));
        launch_small_bridges(P.dev, P.d_lists, P.na, P.d_lists + P.na, P.nb, P.d_sb, P.d_sb + P.sb_hdr, P.cus, s,
                             st->stream2);
        BR_HIP(hipGetLastError());
        BR_HIP(hipEventRecord(st->join, st->stream2));
        BR_HIP(hipStreamWaitEvent(s, st->join, 0));
    }
    return BR_OK;
}

// node-0 certificates (or, with the final step on the device, the number of
// bridges), their counters and the error word to the host
int copy_back(BatchPlan& P, hipStream_t s, int mode) {
    const int32_t S = (int32_t)P.small.size();
    if (mode == 1 && P.big) {
        if (S) {
            const size_t guess = std::min<size_t>(std::max<size_t>(P.keys_hint, 1024), (size_t)std::max<int64_t>(P.vtot, 1));
            BR_HIP(hipMemcpyAsync(P.h_ustat, P.d_un - 1, 256 + 8 * guess, hipMemcpyDeviceToHost, s));
        }
        BR_HIP(hipMemcpyAsync(P.h_err, P.dev.err, 4, hipMemcpyDeviceToHost, s));
        return BR_OK;
    }
    if (mode == 1) {
        if (S) {
            // header, per-graph table and the first keys in one copy
            const size_t guess = std::min<size_t>(std::max<size_t>(P.keys_hint, 4096), (size_t)P.sb_keys);
            BR_HIP(hipMemcpyAsync(P.h_sb, P.d_sb, 4 * ((size_t)P.sb_hdr + guess), hipMemcpyDeviceToHost, s));
        }
        BR_HIP(hipMemcpyAsync(P.h_err, P.dev.err, 4, hipMemcpyDeviceToHost, s));
        return BR_OK;
    }
    if (P.area0) BR_HIP(hipMemcpyAsync(P.h_area0, P.dev.cert, 8 * (size_t)P.area0, hipMemcpyDeviceToHost, s));
    if (S) BR_HIP(hipMemcpyAsync(P.h_cnt0, P.dev.ncnt, 8 * (size_t)S, hipMemcpyDeviceToHost, s));
    BR_HIP(hipMemcpyAsync(P.h_err, P.dev.err, 4, hipMemcpyDeviceToHost, s));
    return BR_OK;
}

static int capture(BatchPlan& P, const int32_t* d_edges, hipStream_t s, int mode, int part, hipGraph_t* graph,
                   hipGraphExec_t* exec, BatchState* st) {
    BR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = enqueue(P, d_edges, s, mode, part, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    *graph = g;
    BR_HIP(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return BR_OK;
}

int run_device(BatchState& st, BatchPlan& P, const int32_t* d_edges, int mode, bool captured = true) {
    hipStream_t s = st.stream;
    const bool two = mode == 1 && !P.small.empty();
    if (!captured) {
        // a plan used once: the launches go straight to the stream
        BR_HIP(hipEventRecord(st.k0, s));
        int rc = enqueue(P, d_edges, s, mode, 0, &st);
        if (rc) return rc;
        BR_HIP(hipEventRecord(st.k1, s));
        if (two) {
            rc = enqueue(P, d_edges, s, mode, 1, &st);
            if (rc) return rc;
        }
        BR_HIP(hipEventRecord(st.k2, s));
        return copy_back(P, s, mode);
    }
    if (!(P.exec && P.graph_edges == d_edges && P.graph_mode == mode)) {
        for (hipGraphExec_t* x : {&P.exec, &P.exec2})
            if (*x) { (void)hipGraphExecDestroy(*x); *x = nullptr; }
        for (hipGraph_t* g : {&P.graph, &P.graph2})
            if (*g) { (void)hipGraphDestroy(*g); *g = nullptr; }
        P.graph_edges = nullptr;
        int rc = capture(P, d_edges, s, mode, 0, &P.graph, &P.exec, &st);
        if (rc) return rc;
        if (two) {
            rc = capture(P, d_edges, s, mode, 1, &P.graph2, &P.exec2, &st);
            if (rc) return rc;
        }
        P.graph_edges = d_edges;
        P.graph_mode = mode;
    }
    BR_HIP(hipEventRecord(st.k0, s));
    BR_HIP(hipGraphLaunch(P.exec, s));
    BR_HIP(hipEventRecord(st.k1, s));
    if (two) BR_HIP(hipGraphLaunch(P.exec2, s));
    BR_HIP(hipEventRecord(st.k2, s));
    return copy_back(P, s, mode);
}

std::string shape_key(int device, const int64_t* eoff, const int32_t* V, int32_t G) {
    // batch shape bucket for the tuner: device arch, G, total edges and
    // largest V (log2 buckets)
    int64_t E = eoff[G] - eoff[0];
    int32_t mv = 0;
    for (int32_t g = 0; g < G; g++) mv = std::max(mv, V[g]);
    return arch_name(device) + "|batched|g" + std::to_string(log2_bucket(G)) + "|e" + std::to_string(log2_bucket(E)) +
           "|v" + std::to_string(log2_bucket(mv));
}

bool same_shape(const BatchPlan& P, const int64_t* eoff, const int32_t* V, int32_t G, int32_t C, int32_t bpc, bool big) {
    return P.G == G && P.C == C && P.bpc == bpc && P.big == big && std::equal(P.eoff.begin(), P.eoff.end(), eoff) &&
           std::equal(P.V.begin(), P.V.end(), V);
}

}  // namespace

size_t batched_device_bytes(br_ctx* c) {
    if (!c->batched) return 0;
    auto* st = static_cast<BatchState*>(c->batched);
    size_t n = 0;
    for (auto& a : st->arenas) n += a.arena_d_cap;
    for (auto& P : st->plans)
        if (P->owns) n += P->dbytes;
    return n;
}

void batched_release(br_ctx* c) {
    if (!c->batched) return;
    auto* st = static_cast<BatchState*>(c->batched);
    if (st->stream) (void)hipStreamSynchronize(st->stream);
    st->plans.clear();
    for (auto& t : st->transient) t.reset();
    for (auto& a : st->arenas) {
        if (a.arena_d) (void)hipFree(a.arena_d);
        if (a.arena_h) (void)hipHostFree(a.arena_h);
    }
    if (st->e0) (void)hipEventDestroy(st->e0);
    if (st->e1) (void)hipEventDestroy(st->e1);
    if (st->k0) (void)hipEventDestroy(st->k0);
    if (st->k1) (void)hipEventDestroy(st->k1);
    if (st->k2) (void)hipEventDestroy(st->k2);
    if (st->fork) (void)hipEventDestroy(st->fork);
    if (st->join) (void)hipEventDestroy(st->join);
    if (st->ready) (void)hipEventDestroy(st->ready);
    if (st->stream2) (void)hipStreamDestroy(st->stream2);
    if (st->stream) (void)hipStreamDestroy(st->stream);
    delete st;
    c->batched = nullptr;
}

// Bridges of every graph of a big-class plan after its launches completed:
// from the bridge step over the union of their certificates (mode 1) or from
// Algorithm 1 per graph on the host (mode 0); out[k] = pairs of graph small[k].
static int gather_big(BatchState& st, BatchPlan& P, int mode, std::vector<std::vector<int32_t>>& out) {
    const int32_t S = (int32_t)P.small.size();
    out.assign(S, {});
    if (mode == 1) {
        if (!S) return BR_OK;
        const uint32_t* hs = P.h_ustat;
        const size_t guess = std::min<size_t>(std::max<size_t>(P.keys_hint, 1024), (size_t)std::max<int64_t>(P.vtot, 1));
        const uint32_t nk = hs[1];
        if (hs[4] != 0 || (int64_t)nk > P.vtot)
            return fail(BR_EINTERNAL, "batched: union bridge step status %u, %u keys", hs[4], nk);
        uint64_t* hk = reinterpret_cast<uint64_t*>(P.h_ustat + 64);
        if (nk > guess) {
            BR_HIP(hipMemcpyAsync(hk + guess, P.d_ukeys + guess, 8 * (size_t)(nk - guess), hipMemcpyDeviceToHost, st.stream));
            BR_HIP(hipStreamSynchronize(st.stream));
        }
        P.keys_hint = nk;
        std::vector<uint64_t> keys(hk, hk + nk);
        canonical_sort(keys);
        // keys in ascending global order: each graph's keys are one run
        int32_t s = 0;
        for (uint64_t k : keys) {
            const int64_t u = (int64_t)(k >> 32), v = (int64_t)(k & 0xffffffffu);
            while (s + 1 < S && P.vbase[s + 1] <= u) s++;
            if (u < P.vbase[s] || v >= P.vbase[s + 1]) return fail(BR_EINTERNAL, "batched: a bridge joins two graphs");
            out[s].push_back((int32_t)(u - P.vbase[s]));
            out[s].push_back((int32_t)(v - P.vbase[s]));
        }
        return BR_OK;
    }
    std::atomic<int32_t> next{0};
    std::atomic<int> bad{0};
    st.pool->run([&](int w) {
        DfsScratch& sc = st.scratch[w];
        std::vector<uint64_t>& keys = st.keys[w];
        for (;;) {
            const int32_t s = next.fetch_add(1);
            if (s >= S) break;
            const uint32_t n1 = P.h_cnt0[2 * s], n2 = P.h_cnt0[2 * s + 1];
            const int64_t off = P.noff[s], capg = P.ncap[s];
            if ((int64_t)n1 + n2 > capg) {
                bad = 1;
                continue;
            }
            keys.clear();
            certificate_bridges(P.h_area0 + off, n1, P.h_area0 + off + capg - n2, n2, P.V[P.small[s]], sc, keys);
            canonical_sort(keys);
            for (uint64_t k : keys) {
                out[s].push_back((int32_t)(k >> 32));
                out[s].push_back((int32_t)(k & 0xffffffffu));
            }
        }
    });
    if (bad) return fail(BR_EINTERNAL, "batched: certificate counts exceed their region");
    return BR_OK;
}

static int get_plan(br_ctx* c, BatchState& st, const int64_t* eoff, const int32_t* V, int32_t G, int32_t C,
                    int32_t bpc, BatchPlan** out, bool big = false) {
    for (size_t i = 0; i < st.plans.size(); i++) {
        if (same_shape(*st.plans[i], eoff, V, G, C, bpc, big)) {
            std::rotate(st.plans.begin(), st.plans.begin() + i, st.plans.begin() + i + 1);
            *out = st.plans[0].get();
            return BR_OK;
        }
    }
    hipDeviceProp_t prop;
    BR_HIP(hipGetDeviceProperties(&prop, c->device));
    auto P = std::make_unique<BatchPlan>();
    int rc = build_plan(*P, eoff, V, G, C, bpc, prop.multiProcessorCount, big, nullptr, st.stream);
    if (rc) return rc;
    st.plans.insert(st.plans.begin(), std::move(P));
    if (st.plans.size() > 4) st.plans.pop_back();
    *out = st.plans[0].get();
    return BR_OK;
}

// a plan for one call of a batch shape not worth keeping (serving): built in
// the class's arena, never captured
static int get_transient(br_ctx* c, BatchState& st, const int64_t* eoff, const int32_t* V, int32_t G, int32_t C,
                         int32_t bpc, BatchPlan** out, bool big) {
    const int k = big ? 1 : 0;
    st.transient[k].reset(new BatchPlan());
    const int cus = g_cus > 0 ? g_cus : 256;
    int rc = build_plan(*st.transient[k], eoff, V, G, C, bpc, cus, big, &st.arenas[k], st.stream);
    if (rc) return rc;
    *out = st.transient[k].get();
    return BR_OK;
}

int batched_query(br_ctx* c, const int32_t* d_edges, const int64_t* h_edge_off, const int32_t* h_V, int32_t G,
                  int32_t chunk_edges, int32_t* h_bridges, int64_t cap, int64_t* h_bridge_off, void* stream,
                  bool transient) {
    auto t0 = std::chrono::steady_clock::now();
    BR_HIP(hipSetDevice(c->device));
    BatchState& st = *state_of(c);
    if (!st.stream) {
        BR_HIP(hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking));
        BR_HIP(hipEventCreate(&st.e0));
        BR_HIP(hipEventCreate(&st.e1));
        BR_HIP(hipEventCreate(&st.k0));
        BR_HIP(hipEventCreate(&st.k1));
        BR_HIP(hipEventCreate(&st.k2));
        BR_HIP(hipStreamCreateWithFlags(&st.stream2, hipStreamNonBlocking));
        BR_HIP(hipEventCreateWithFlags(&st.fork, hipEventDisableTiming));
        BR_HIP(hipEventCreateWithFlags(&st.join, hipEventDisableTiming));
        BR_HIP(hipEventCreateWithFlags(&st.ready, hipEventDisableTiming));
        if (prepare_small_bridges() != 0) return fail(BR_EHIP, "batched: cannot raise the LDS limit of the bridge kernel");
        if (small_bridges_max_v() < batched_max_v_dev()) return fail(BR_EINTERNAL, "batched: bridge kernel limit below the LDS path's");
    }
    if (!st.pool) {
        int n = (int)std::thread::hardware_concurrency();
        n = std::max(1, std::min(n, 16));
        st.pool = std::make_unique<Pool>(n);
        st.scratch.resize(n);
        st.keys.resize(n);
    }
    // the caller's stream must have produced the input
    BR_HIP(hipEventRecord(st.ready, static_cast<hipStream_t>(stream)));
    BR_HIP(hipStreamWaitEvent(st.stream, st.ready, 0));

    // chunk size and workgroups per CU: given, or the tuner's (measured on
    // this batch the first time its shape bucket is seen on this device,
    // and kept in BR_AUTOTUNE_CACHE when that names a file)
    int32_t C = chunk_edges, bpc = batched_blocks_per_cu();
    if (C == 0) {
        const std::string key = shape_key(c->device, h_edge_off, h_V, G);
        TuneEntry t;
        if (tune_get(key, t) && t.count("chunk_edges") && t.count("blocks_per_cu")) {
            C = (int32_t)t["chunk_edges"];
            bpc = (int32_t)t["blocks_per_cu"];
        } else if (transient) {
            C = 32768;            // nothing measured for this shape yet: no time to measure now
        } else {
            // time every candidate on this batch (device part only)
            float best = 1e30f;
            int32_t bestC = 16384, bestB = bpc;
            for (int32_t b = 1; b <= batched_max_blocks_per_cu(); b++)
                for (int32_t cand : {4096, 8192, 16384, 32768, 65536, 131072}) {
                    BatchPlan* P = nullptr;
                    int rc = get_plan(c, st, h_edge_off, h_V, G, cand, b, &P);
                    if (rc) return rc;
                    float ms = 1e30f;
                    for (int rep = 0; rep < 3; rep++) {
                        BR_HIP(hipEventRecord(st.e0, st.stream));
                        rc = run_device(st, *P, d_edges, 0);
                        if (rc) return rc;
                        BR_HIP(hipEventRecord(st.e1, st.stream));
                        BR_HIP(hipEventSynchronize(st.e1));
                        float f = 0.f;
                        BR_HIP(hipEventElapsedTime(&f, st.e0, st.e1));
                        if (rep > 0) ms = std::min(ms, f);
                    }
                    if (ms < best) {
                        best = ms;
                        bestC = cand;
                        bestB = b;
                    }
                }
            tune_put(key, {{"chunk_edges", bestC}, {"blocks_per_cu", bestB}, {"ms", best}});
            C = bestC;
            bpc = bestB;
        }
    }
    BatchPlan* P = nullptr;
    int rc = transient ? get_transient(c, st, h_edge_off, h_V, G, C, bpc, &P, false)
                       : get_plan(c, st, h_edge_off, h_V, G, C, bpc, &P);
    if (rc) return rc;
    // graphs above the small kernel's V and within a CU's LDS: the 160 KB
    // kernel, one workgroup per CU, in the same call
    BatchPlan* PM = nullptr;
    for (int32_t g = 0; g < G; g++)
        if (h_V[g] > batched_max_v_dev() && h_V[g] <= batched_max_v_big()) {
            rc = transient ? get_transient(c, st, h_edge_off, h_V, G, C, 1, &PM, true)
                           : get_plan(c, st, h_edge_off, h_V, G, C, 1, &PM, true);
            if (rc) return rc;
            break;
        }
    const int mode = c->final_step;
    if (c->profiling) BR_HIP(hipEventRecord(st.e0, st.stream));
    rc = run_device(st, *P, d_edges, mode, !transient);
    if (rc) return rc;
    if (PM) {
        rc = run_device(st, *PM, d_edges, mode, !transient);
        if (rc) return rc;
    }
    if (c->profiling) BR_HIP(hipEventRecord(st.e1, st.stream));
    BR_HIP(hipStreamSynchronize(st.stream));
    auto t1 = std::chrono::steady_clock::now();
    for (BatchPlan* Q : {P, PM}) {
        if (!Q) continue;
        if (*Q->h_err & 1u) return fail(BR_ERANGE, "batched: an edge has a vertex id outside its graph's [0, V)");
        if (*Q->h_err) return fail(BR_EINTERNAL, "batched: certificate region overflow");
    }
    std::vector<std::vector<int32_t>> mid_out;
    if (PM) {
        rc = gather_big(st, *PM, mode, mid_out);
        if (rc) return rc;
    }

    // final search per small graph; bridges of graph g go to a slot of V_g - 1
    // pairs, compacted afterwards
    const int32_t S = (int32_t)P->small.size();
    std::vector<int64_t> slot(S + 1, 0), nb(G, 0);
    if (PM)
        for (size_t k = 0; k < PM->small.size(); k++) nb[PM->small[k]] = (int64_t)mid_out[k].size() / 2;
    for (int32_t s = 0; s < S; s++) slot[s + 1] = slot[s] + std::max(P->V[P->small[s]] - 1, 0);
    uint64_t* outk = nullptr;
    const uint32_t* keys = nullptr;     // mode 1: the device's sorted keys, (u | v << 16)
    if (mode != 1) {
        if (st.outk_n < (size_t)std::max<int64_t>(slot[S], 1)) {
            st.outk_n = (size_t)std::max<int64_t>(slot[S], 1);
            st.outk.reset(new uint64_t[st.outk_n]);
        }
        outk = st.outk.get();
    }
    if (mode == 1) {
        // per graph: base and count in the key array, keys already sorted
        const size_t guess = std::min<size_t>(std::max<size_t>(P->keys_hint, 4096), (size_t)P->sb_keys);
        const uint32_t* hdr = P->h_sb;
        keys = P->h_sb + P->sb_hdr;
        const uint32_t nk = S ? hdr[0] : 0;
        if (nk > (uint32_t)P->sb_keys) return fail(BR_EINTERNAL, "batched: %u bridge keys for room %lld", nk, (long long)P->sb_keys);
        if (nk > guess) {
            BR_HIP(hipMemcpyAsync(P->h_sb + P->sb_hdr + guess, P->d_sb + P->sb_hdr + guess, 4 * (size_t)(nk - guess),
                                  hipMemcpyDeviceToHost, st.stream));
            BR_HIP(hipStreamSynchronize(st.stream));
        }
        P->keys_hint = nk;
        // counts only here; the keys go straight to the caller's array below
        for (int32_t s = 0; s < S; s++) {
            const uint32_t base = hdr[16 + 2 * s], cnt = hdr[17 + 2 * s];
            if ((uint64_t)base + cnt > nk || (int64_t)cnt > slot[s + 1] - slot[s])
                return fail(BR_EINTERNAL, "batched: graph %d reports %u bridges at %u", (int)P->small[s], cnt, base);
            nb[P->small[s]] = cnt;
        }
    } else {
        std::atomic<int32_t> next{0};
        std::atomic<int> bad{0};
        st.pool->run([&](int w) {
            DfsScratch& sc = st.scratch[w];
            std::vector<uint64_t>& keys = st.keys[w];
            for (;;) {
                const int32_t s = next.fetch_add(1);
                if (s >= S) break;
                const int32_t g = P->small[s];
                const uint32_t n1 = P->h_cnt0[2 * s], n2 = P->h_cnt0[2 * s + 1];
                const int64_t off = P->noff[s], capg = P->ncap[s];
                if ((int64_t)n1 + n2 > capg) {
                    bad = 1;
                    continue;
                }
                keys.clear();
                certificate_bridges(P->h_area0 + off, n1, P->h_area0 + off + capg - n2, n2, P->V[g], sc, keys);
                canonical_sort(keys);
                std::copy(keys.begin(), keys.end(), outk + slot[s]);
                nb[g] = (int64_t)keys.size();
            }
        });
        if (bad) return fail(BR_EINTERNAL, "batched: certificate counts exceed their region");
    }
    auto t2 = std::chrono::steady_clock::now();
    // graphs above the LDS limit: the plain path, with the same chunk size
    std::vector<std::vector<int32_t>> large_out(P->large.size());
    for (size_t k = 0; k < P->large.size(); k++) {
        const int32_t g = P->large[k];
        const int64_t E = h_edge_off[g + 1] - h_edge_off[g];
        const int32_t M = (int32_t)std::max<int64_t>(1, std::min<int64_t>((E + C - 1) / C, 1 << 20));
        large_out[k].resize(2 * (size_t)std::max(h_V[g] - 1, 1));
        int64_t n = 0;
        rc = br_bridges_find(c, d_edges + 2 * h_edge_off[g], E, h_V[g], M, large_out[k].data(),
                             std::max(h_V[g] - 1, 1), &n, st.stream);
        if (rc) return rc;
        nb[g] = n;
        large_out[k].resize(2 * (size_t)n);
    }
    // assemble in graph order
    h_bridge_off[0] = 0;
    for (int32_t g = 0; g < G; g++) h_bridge_off[g + 1] = h_bridge_off[g] + nb[g];
    const int64_t total = h_bridge_off[G];
    if (total <= cap) {
        for (int32_t s = 0; s < S; s++) {
            const int32_t g = P->small[s];
            int32_t* o = h_bridges + 2 * h_bridge_off[g];
            if (mode == 1) {
                const uint32_t* k = keys + P->h_sb[16 + 2 * s];
                for (int64_t i = 0; i < nb[g]; i++) {
                    o[2 * i] = (int32_t)(k[i] >> 16);
                    o[2 * i + 1] = (int32_t)(k[i] & 0xffffu);
                }
            } else {
                for (int64_t i = 0; i < nb[g]; i++) {
                    o[2 * i] = (int32_t)(outk[slot[s] + i] >> 32);
                    o[2 * i + 1] = (int32_t)(outk[slot[s] + i] & 0xffffffffu);
                }
            }
        }
        for (size_t k = 0; k < P->large.size(); k++)
            std::copy(large_out[k].begin(), large_out[k].end(), h_bridges + 2 * h_bridge_off[P->large[k]]);
        if (PM)
            for (size_t k = 0; k < PM->small.size(); k++)
                std::copy(mid_out[k].begin(), mid_out[k].end(), h_bridges + 2 * h_bridge_off[PM->small[k]]);
    }
    auto t3 = std::chrono::steady_clock::now();
    if (c->profiling) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, st.e0, st.e1) != hipSuccess) ms = 0.f;
        c->prof.ms_cert = ms;
        if (hipEventElapsedTime(&ms, st.k0, st.k1) != hipSuccess) ms = 0.f;   // clear + persistent kernel
        c->prof.ms_phase0 = ms;
        if (hipEventElapsedTime(&ms, st.k1, st.k2) != hipSuccess) ms = 0.f;   // combined bridge step (if any)
        c->prof.ms_bridge_dev = mode == 1 ? ms : 0.0;
        (void)hipGetLastError();
        c->prof.ms_merge = 0;
        c->prof.ms_d2h = 0;
    }
    c->prof.ms_dfs = std::chrono::duration<double, std::milli>(t2 - t1).count();
    c->prof.ms_canon = std::chrono::duration<double, std::milli>(t3 - t2).count();
    c->prof.ms_total = std::chrono::duration<double, std::milli>(t3 - t0).count();
    c->prof.rounds = C;
    c->prof.launches = 1;
    if (total > cap) return fail(BR_ECAP, "batched: %lld bridges, capacity %lld", (long long)total, (long long)cap);
    return BR_OK;
}

}  // namespace br

using namespace br;

extern "C" {

int32_t br_batched_max_v(void) { return batched_max_v_dev(); }
int32_t br_lds_max_v(void) { return batched_max_v_big(); }

int br_bridges_find_batched(br_ctx* c, const int32_t* d_edges, const int64_t* h_edge_off, const int32_t* h_V,
                            int32_t G, int32_t chunk_edges, int32_t* h_bridges, int64_t cap, int64_t* h_bridge_off,
                            void* stream) {
    if (!c || !h_edge_off || !h_V || !h_bridge_off || G < 0 || chunk_edges < 0 || cap < 0 || (cap > 0 && !h_bridges))
        return fail(BR_EINVAL, "br_bridges_find_batched: bad argument");
    if (h_edge_off[0] != 0) return fail(BR_EINVAL, "batched: offsets must start at 0");
    for (int32_t g = 0; g < G; g++) {
        if (h_edge_off[g + 1] < h_edge_off[g]) return fail(BR_EINVAL, "batched: offsets decrease at graph %d", g);
        if (h_V[g] < 1) return fail(BR_EINVAL, "batched: V[%d] = %d < 1", g, h_V[g]);
    }
    if (h_edge_off[G] > 0 && !d_edges) return fail(BR_EINVAL, "batched: null edge list");
    return batched_query(c, d_edges, h_edge_off, h_V, G, chunk_edges, h_bridges, cap, h_bridge_off, stream, false);
}

}  // extern "C"
