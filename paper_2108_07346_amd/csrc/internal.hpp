// Internal declarations of libbridges (host side).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstdint>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bridges.h"

namespace br {

// ---- errors -----------------------------------------------------------------
int fail(int code, const char* fmt, ...);          // sets the thread-local message, returns code
int hip_fail(hipError_t e, const char* what);      // BR_EHIP (or BR_ENOMEM) with the HIP message
#define BR_HIP(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return br::hip_fail(e_, #call); \
    } while (0)

// ---- host worker pool: run(fn) calls fn(i) on every worker i and waits ----------
class Pool {
  public:
    explicit Pool(int n) {
        for (int i = 0; i < n; i++) th_.emplace_back([this, i] { loop(i); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    int size() const { return (int)th_.size(); }
    // run fn(worker) on every worker and wait
    void run(const std::function<void(int)>& fn) {
        std::unique_lock<std::mutex> g(mu_);
        fn_ = &fn;
        pending_ = (int)th_.size();
        gen_++;
        cv_.notify_all();
        done_.wait(g, [this] { return pending_ == 0; });
        fn_ = nullptr;
    }

  private:
    void loop(int i) {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int)>* f;
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                f = fn_;
            }
            (*f)(i);
            std::lock_guard<std::mutex> g(mu_);
            if (--pending_ == 0) done_.notify_one();
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_;
    const std::function<void(int)>* fn_ = nullptr;
    int pending_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// ---- tuner (tuner.cpp) ----------------------------------------------------------
// A tuned choice: named numbers ("solo", "variant", "chunk_edges", ...).
using TuneEntry = std::map<std::string, double>;
std::string arch_name(int device);      // e.g. "gfx950"
int log2_bucket(int64_t x);             // smallest b with 2^b >= x
bool tune_get(const std::string& key, TuneEntry& out);
void tune_put(const std::string& key, const TuneEntry& e);   // also saved to BR_AUTOTUNE_CACHE if set

// ---- device geometry shared with the kernels ---------------------------------
// Chunk i of the phase tree is edges [lo(i), lo(i+1)) with lo(i) = floor(iE/M).
struct Plan {
    int64_t E = 0;
    int32_t V = 0, M = 1;
    int32_t rounds = 0;            // ceil(log2 M)
    int32_t tile = 0;              // edges per workgroup tile in phase 0
    int32_t tpc = 0;               // tiles per chunk (same for every chunk)
    int32_t xcd_map = 0;           // keep each chunk's workgroups on one XCD
    int64_t blocks0 = 0;           // phase-0 grid (single stage)
    std::vector<int64_t> stages;   // chunk-relative stage boundaries, last = chunk size bound
    std::vector<int64_t> off, cap; // per node: certificate region (pairs)
    int64_t cert_pairs = 0;        // sum of caps
    std::vector<int64_t> round_cap;// per round: largest sibling cap
    int32_t qs = 2;                // union-find state words per vertex (F at +0, F' at +1)
    // one workgroup per node (solo_kernels.hip) for phase 0 and merge levels
    // 1..solo_top; the rounds above run as team launches on the dense states
    bool solo = false;
    int32_t solo_top = 0;
    int32_t solo_variant = 0;      // worker shape (solo_kernels.hip)
    bool prem = false;             // team merges: each thread's edges of a tile requested at once
    int32_t solo_cmp = 16;         // phase 0 compresses its slot every cmp * V / 8 edges up to 2 V, then at 8 V
    int32_t solo_nbk = 0;          // phase 0 reads its chunk bucketed: buckets by the smaller endpoint (0: input order)
    int32_t solo_nbk2 = 1;         // ... times buckets by the larger endpoint (at most 1,024 in all)
    bool solo_mbk = false;         // ... and the merges inside the kernel read their siblings so too
    bool solo_wm = false;          // written-bits maps in LDS: loads of words never stored are skipped
    int32_t workers = 0;           // persistent workgroups
    int32_t nslots = 0;            // union-find slots (workers' own + free pool)
    int32_t tile0_max = 0;         // team path: largest first-stage tile (0 = the kernel's)
    // the whole phase tree in LDS (batched_kernels.hip: one graph, a
    // workgroup per chunk and last-arriver merges) when V fits a workgroup's LDS
    bool lds = false;
    bool lds_big = false;          // the 160 KB kernel (V above the small kernel's limit)
    int32_t lds_blocks = 0;
    int64_t lds_counters = 0;      // merge arrival counters
};

// Certificate regions: node i owns pairs [off[i], off[i]+cap[i]); its F1 grows
// from the front, its F2 from the back; cnt[2i], cnt[2i+1] count them.
struct DevBufs {
    const int2* edges = nullptr;   // edge i < split is edges[i]
    const int2* edges2 = nullptr;  // edge i >= split is edges2[i - split]
    int64_t split = 0;
    uint32_t* state = nullptr;     // [M][V][qs] offset-encoded parents (0 = root), F at +0, F' at +1
    int64_t qs = 2;                // words per vertex of the state (2, or 8: one vertex per 32 bytes)
    uint32_t* packed = nullptr;    // [M][V][2]: where a qs = 8 state is compressed to after the first stage
    int2* cert = nullptr;
    const int64_t* off = nullptr;  // [M]
    const int64_t* cap = nullptr;  // [M]
    uint32_t* cnt = nullptr;       // [M][2]
    uint32_t* err = nullptr;       // bit 0: id out of range; bit 1: region overflow
    int32_t shift = 0;             // node i's state is state + (i >> shift) * qs * V
};

// Buffers of the one-workgroup-per-node path (solo_kernels.hip).
struct SoloBufs {
    uint32_t* slots = nullptr;     // [nslots][2][V] tagged union-find words
    uint32_t* slot_tag = nullptr;  // [nslots] (kept across calls; zero = slot cleared)
    uint32_t* pool = nullptr;      // [ceil(nslots / 32)] free-slot bits
    uint32_t* park = nullptr;      // [2M]: parked slot per left node, then arrival counters
    uint32_t* queue = nullptr;     // [1]
    uint32_t* dense = nullptr;     // [ceil(M / 2^top)][V][2] node states at level top
    int2* sbuf = nullptr;          // [workers][sbuf_stride] reordered chunk copies (solo_nbk > 0)
    int64_t sbuf_stride = 0;
    int32_t nslots = 0, workers = 0;
};
size_t solo_lds_bytes(int32_t V, bool wm);
bool solo_wm_fits(int32_t V);              // the written-bits maps fit beside the claim tables
int solo_prepare(int32_t V);       // once per process: the kernel's LDS limit
int32_t solo_max_v();
int solo_blocks_per_cu(int variant, int32_t V, bool wm);
int solo_block(int variant);       // threads per worker of a worker shape
int solo_variants();
void launch_solo(const Plan& P, const DevBufs& B, const SoloBufs& S, hipStream_t s);
// compute units and the LDS a workgroup may use on the device the library
// runs on (set by br_create; 256 and 64 KB until then)
extern int g_cus;
extern int g_max_lds;

// Batched path (one persistent launch over many small graphs).  Graph s of
// the launch has edges [eoff[2s], eoff[2s+1]), V[s] vertices, Mg[s] chunks;
// its node k lives at index k == 0 ? s : rbase[s] + k - 1 (all node-0 regions
// come first); its merge counters start at cbase[s].
struct BatchDev {
    const int2* edges;
    const int64_t* eoff;      // [2S] start, end
    const int32_t* V;         // [S]
    const int32_t* Mg;        // [S]
    const int64_t* rbase;     // [S]
    const int64_t* cbase;     // [S]
    const int64_t* noff;      // [nodes] region offset (pairs)
    const int64_t* ncap;      // [nodes] region capacity
    const int64_t* items;     // [n_items] (s << 20) | chunk
    int64_t n_items;
    int2* cert;               // node regions
    uint32_t* ncnt;           // [nodes][2]
    uint32_t* arrive;         // merge arrival counters
    uint32_t* queue;          // [1] next item
    uint32_t* err;            // bit 0: id out of range; bit 1: region overflow
    const int64_t* vbase;     // [S] first vertex of graph s in the combined numbering
    uint32_t* rootw;          // [sum V] 0 at each root of F of the graph's final certificate, else 1
};
// big: the kernel for graphs of up to batched_max_v_big() vertices (one
// workgroup per CU); else up to batched_max_v_dev()
void launch_batched(const BatchDev& B, int blocks, hipStream_t s, bool big = false);
int32_t batched_max_v_big();
// node-0 certificates of the batch's graphs 0..S-1 as one certificate of their
// disjoint union (ids shifted by vbase): F edges at f1u, F' edges at f2u,
// their numbers at cntu[0], cntu[1]; uoff [2S] scratch
// one device edge list to gather: n edges from src to edge offset `at`
struct GatherItem {
    const int32_t* src;
    int64_t at, n;
};
// copies every item's edges into dst in one launch (items in device memory;
// max_edges = the largest n)
void launch_gather_edges(const GatherItem* d_items, int32_t n, int64_t max_edges, int32_t* dst, hipStream_t s);
void launch_union_certificate(const BatchDev& B, int32_t S, int64_t* uoff, int2* f1u, int2* f2u, uint32_t* cntu,
                              hipStream_t s);
// Final step on the device for the batched path: one workgroup per small graph
// finds the bridges of node 0's certificate in LDS; keys (u << 16 | v, sorted)
// go to out_keys at a base taken from out_hdr[0]; out_hdr[16 + 2s] / [17 + 2s]
// receive graph s's base and count.  out_hdr[0] must be zero at launch.
// list_a holds the graphs with V <= small_bridges_split_v(), list_b the rest.
// The two size classes go to streams s (small) and s_b (large) so that they
// can overlap; the caller orders s_b after earlier work on s and joins it back.
void launch_small_bridges(const BatchDev& B, const int32_t* list_a, int32_t na, const int32_t* list_b, int32_t nb,
                          uint32_t* out_hdr, uint32_t* out_keys, int cus, hipStream_t s, hipStream_t s_b);
// Allows the kernels above their LDS sizes (once per process, before any launch or capture).
int prepare_small_bridges();
int32_t small_bridges_split_v();
int32_t small_bridges_max_v();   // largest V the kernel above takes
int32_t batched_max_v_dev();
int32_t batched_blocks_per_cu();
int32_t batched_max_blocks_per_cu();

// Largest V the final steps take: they count the 2(V-1) arcs of the
// certificate's forest tours in 30-bit fields (and the host search in int32).
constexpr int32_t kFinalStepMaxV = 1 << 29;

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
void launch_phase0(const Plan& P, DevBufs& B, hipStream_t s);
int phase0_launches(const Plan& P);   // kernels launch_phase0 enqueues for this plan
// enqueues one merge round; returns the number of kernels launched
int launch_merge_round(const Plan& P, const DevBufs& B, int32_t step, hipStream_t s);
void launch_copy_out(const Plan& P, const DevBufs& B, int32_t* d_out, int64_t out_cap, int64_t* d_counts,
                     hipStream_t s);

// The plan of one query.  tuned: a tuner entry for this shape (knobs it
// names replace the size rules); environment variables BR_SOLO, BR_SOLO_TOP,
// BR_SOLO_WPC and BR_SOLO_VARIANT replace both (measurements).
Plan make_plan(int64_t E, int32_t V, int32_t M, bool allow_solo = true, const TuneEntry* tuned = nullptr);
// make_plan with the tuner's entry for this device and shape, if any
Plan plan_for(int device, int64_t E, int32_t V, int32_t M);
std::string plain_tune_key(int device, int64_t E, int32_t V, int32_t M);
// device workspace of one plain-path query with this plan (state, certificate
// regions, node tables and, with the device final step, the bridge step's scratch)
size_t plan_workspace_bytes(const Plan& P, bool device_final);

// Final step on the device (bridge_kernels.hip): scratch words it needs, and
// the launch sequence over node 0's certificate; the bridges' keys land at
// *d_keys (count at *d_n) on the device.
int64_t device_bridges_words(int32_t V);
// In-place exclusive scan of a[0..n) in one launch; status[ceil(n / 1024)] and
// *ticket must be zero at launch.
void device_scan1(int32_t* a, int64_t n, uint64_t* status, uint32_t* ticket, hipStream_t s);
// Scan-first certificate (two breadth-first forests, the second avoiding the
// first's vertex pairs) of an edge list on the device; workspace in 4-byte
// words, and the call that fills h_f1 / h_f2 (V pairs each) and the counts.
int64_t scan_first_words(int64_t E, int32_t V);
int scan_first_certificate(const int2* edges, int64_t E, int32_t V, char* ws, hipStream_t s, uint32_t* h_small,
                           int2* h_f1, int2* h_f2, uint32_t* n1, uint32_t* n2, int* levels1, int* levels2);
int scan_first_device(const int2* edges, int64_t E, int32_t V, char* ws, hipStream_t s, uint32_t* h_small, int* levels1,
                      int* levels2, int2** d_f1, int2** d_f2, uint32_t** d_cnt, uint32_t** d_err, uint32_t** d_roots);
// Articulation points of a certificate on the device (F spanning forest, roots
// flagged 0 in q[qs * v]); ids as 64-bit keys at *d_keys, their number at *d_n
// (the bridge step's status-block layout).
int device_articulation_cert(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q,
                             int32_t qs, int32_t V, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s);
// copies |F|, |F'| (cnt[0..1]) and *err into the 256-byte status block whose
// word 1 is the key count d_n of a bridge step (the keys follow the block)
void launch_bridge_status(const uint32_t* cnt, const uint32_t* err, uint32_t* d_n, hipStream_t s);
int device_bridges(const Plan& P, const DevBufs& B, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s);

// 2-edge-connected classes of node 0's certificate on the device: int32 labels
// (smallest id of each class) where the keys would go, their count at *d_n.
int device_classes(const Plan& P, const DevBufs& B, int32_t* ws, int32_t** d_label, uint32_t** d_n, hipStream_t s);
// ... and the bridge tree's edges (class-label keys min << 32 | max, unordered;
// their number in status word 5, (*d_n)[4]) at *d_tkeys
int device_bridge_tree(const Plan& P, const DevBufs& B, int32_t* ws, int32_t** d_label, uint32_t** d_n,
                       uint64_t** d_tkeys, hipStream_t s);
// also fills the status block before the keys (|F|, |F'|, *err or 0)
int device_bridges_cert(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q, int32_t qs,
                        int32_t V, const uint32_t* err, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s);

// device address of the fixed scratch array on `device` (current on the
// calling thread), looked up once; br_create calls it
int static_scratch_init(int device);

// ---- host side of the path --------------------------------------------------
// Algorithm 1 (iterative) on the certificate; appends canonical keys (min<<32|max).
struct DfsScratch {
    std::vector<int32_t> head, fill, st_v, st_pe, st_it;
    std::vector<int2> arc;       // (target, edge id) per arc, grouped by source
    std::vector<int2> dl;        // (disc, low) per vertex
};
void certificate_bridges(const int2* f1, int64_t n1, const int2* f2, int64_t n2, int32_t V, DfsScratch& S,
                         std::vector<uint64_t>& keys);

void canonical_sort(std::vector<uint64_t>& keys);
// Articulation points of the graph (V, F u F') by a low-link depth-first
// search on the host: vertex ids ascending in out.
void certificate_articulation(const int2* f1, int64_t n1, const int2* f2, int64_t n2, int32_t V, DfsScratch& S,
                              std::vector<int32_t>& out);

// ---- context ------------------------------------------------------------------
struct Arena {
    void* base = nullptr;
    size_t size = 0;
};

}  // namespace br

struct br_ctx {
    int device = 0;
    br::Arena ws;                  // device workspace
    void* pinned = nullptr;        // pinned host staging
    size_t pinned_size = 0;
    int64_t* h_meta = nullptr;     // pinned: off/cap upload staging
    size_t h_meta_n = 0;
    br::DfsScratch dfs;
    std::vector<uint64_t> keys;
    int profiling = 0;
    size_t keys_hint = 0;          // bridges found by the previous call (first copy size)
    int final_step = 1;            // 0: host search (Algorithm 1), 1: device bridge step
    int32_t* bws = nullptr;        // device bridge-step scratch inside the workspace
    br_profile prof{};
    hipEvent_t ev[8] = {};
    // recorded at the end of the work every entry point enqueues; the next call
    // orders its stream after it before touching the shared workspace
    hipEvent_t ev_done = nullptr;
    bool done_recorded = false;
    bool exact_ws = false;         // workspace sized exactly to the request (server slots)
    // the solo path's slots keep their tags across calls: cleared again when
    // the workspace, V or the slot count change
    const void* solo_key_base = nullptr;
    int32_t solo_key_v = 0, solo_key_slots = 0;
    // batched path state
    void* batched = nullptr;
};

namespace br {
int ensure_workspace(br_ctx* c, size_t bytes, hipStream_t s);
// br_bridges_find_batched after argument checks; transient: the batch shape
// is used once (serving ticks): plans built in reused arenas, launched
// without graph capture, chunk size from the tuner's cache or a default
int batched_query(br_ctx* c, const int32_t* d_edges, const int64_t* h_edge_off, const int32_t* h_V, int32_t G,
                  int32_t chunk_edges, int32_t* h_bridges, int64_t cap, int64_t* h_bridge_off, void* stream,
                  bool transient);
void batched_release(br_ctx* c);
// device bytes the context's batched plans and arenas hold
size_t batched_device_bytes(br_ctx* c);
int ensure_pinned(br_ctx* c, size_t bytes);
// Run phases a1..a5 on d_edges; on return (asynchronously) node 0 holds the final certificate.
// The input is the concatenation of d_a [Ea] and d_b [Eb] (d_b may be null with Eb = 0).
// device_final: reserve the device bridge step's scratch in the workspace.
// plan_knobs: plan with these tuner knobs instead of the tuner's entry.
int run_certificate(br_ctx* c, const int32_t* d_a, int64_t Ea, const int32_t* d_b, int64_t Eb, int32_t V, int32_t M,
                    hipStream_t s, Plan& P, DevBufs& B, bool device_final, const TuneEntry* plan_knobs = nullptr);
int run_certificate_with(br_ctx* c, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, hipStream_t s, Plan& P,
                         DevBufs& B, bool device_final, const TuneEntry* plan_knobs);
// Order stream s after everything earlier calls on this context enqueued
// (they may have used another stream), and mark the end of this call's work.
int ctx_begin(br_ctx* c, hipStream_t s);
int ctx_end(br_ctx* c, hipStream_t s);
}  // namespace br
