// Scan-first certificate for vertex connectivity on the GPU: the input for the
// articulation points ("failure points" of the paper's abstract).
//
// Algorithm 2 builds its forests with a search ("pick a vertex and start a
// DFS") and union-find; for bridges any maximal forests will do, but cut
// vertices survive only in a certificate whose forests come from a scan-first
// search: F is a breadth-first forest of G, F' a breadth-first forest of G
// without the vertex pairs F uses (every parallel copy of an F pair is left
// out as well, since vertex connectivity ignores multiplicity).  Breadth-first
// search level by level is a scan-first search when each newly reached vertex
// takes as parent its smallest-id neighbour one level up (scanning each level
// in id order), which is the rule applied here; each tree starts at the
// smallest vertex of its component.
//
// Pieces: a union-find pass for the components (in stages with full path
// compression between them, as in phase 0; roots are the smallest ids), an
// adjacency array of the edge list, and one launch per breadth-first level.
// A vertex's candidate word holds (level of the parent) << 32 | parent, so an
// atomic minimum keeps the shallowest, then smallest-id parent; the wavefront
// that handles a vertex of level d emits its tree edge (its candidate is final:
// only level d - 1 could set it) and offers (d << 32 | itself) to its
// neighbours, and the first touch of a neighbour appends it to level d + 1.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace br {

namespace {

constexpr int kT = 256;
constexpr uint64_t kNoCand = ~uint64_t(0);

#define GRID_LOOP(i, n) for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

int grid_for(int64_t n) {
    int64_t g = (n + kT - 1) / kT;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 16384));
}

__device__ __forceinline__ bool excluded(const int32_t* par1, int32_t u, int32_t w) {
    return par1 && (par1[w] == u || par1[u] == w);
}

// component union-find over the edges (skipping loops and, with par1, the
// pairs of the first forest); q[x] = x - parent(x), 0 at a root; the larger
// root is hooked under the smaller, so each component's root is its smallest id
__device__ __forceinline__ uint32_t cc_find(uint32_t* q, uint32_t x) {
    uint32_t d = __hip_atomic_load(q + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    while (d != 0) {
        const uint32_t p = x - d;
        const uint32_t dp = __hip_atomic_load(q + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (dp == 0) return p;
        __hip_atomic_store(q + x, d + dp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        x = p - dp;
        d = __hip_atomic_load(q + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    return x;
}

__device__ __forceinline__ void cc_unite(uint32_t* q, uint32_t u, uint32_t v) {
    for (;;) {
        u = cc_find(q, u);
        v = cc_find(q, v);
        if (u == v) return;
        if (u < v) { const uint32_t t = u; u = v; v = t; }
        uint32_t expect = 0;
        if (__hip_atomic_compare_exchange_strong(q + u, &expect, u - v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        u = u - expect;
    }
}

// edges [lo, hi), kCcU per thread with their loads issued together; an edge
// whose endpoints already have the same parent is done after two loads (after
// a full compression that parent is the root)
constexpr int kCcU = 4;

__global__ void k_cc(const int2* edges, int64_t lo, int64_t hi, int32_t V, const int32_t* par1, uint32_t* q,
                     uint32_t* err) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < hi; i0 += kCcU * stride) {
        int2 e[kCcU];
        bool ok[kCcU];
#pragma unroll
        for (int j = 0; j < kCcU; j++) {
            const int64_t i = i0 + j * stride;
            e[j] = i < hi ? edges[i] : make_int2(0, 0);
            ok[j] = i < hi;
            if (ok[j] && ((uint32_t)e[j].x >= (uint32_t)V || (uint32_t)e[j].y >= (uint32_t)V)) {
                atomicOr(err, 1u);
                ok[j] = false;
            }
            if (ok[j] && (e[j].x == e[j].y || excluded(par1, e[j].x, e[j].y))) ok[j] = false;
        }
        uint32_t pu[kCcU], pv[kCcU];
#pragma unroll
        for (int j = 0; j < kCcU; j++) {
            pu[j] = ok[j] ? (uint32_t)e[j].x - __hip_atomic_load(q + e[j].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0u;
            pv[j] = ok[j] ? (uint32_t)e[j].y - __hip_atomic_load(q + e[j].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kCcU; j++)
            if (ok[j] && pu[j] != pv[j]) cc_unite(q, pu[j], pv[j]);
    }
}

// every vertex straight under its root (no hook runs concurrently)
__global__ void k_cc_compress(uint32_t* q, int32_t V) {
    GRID_LOOP(x, (int64_t)V) {
        const uint32_t d = q[x];
        if (d == 0) continue;
        uint32_t r = (uint32_t)x - d;
        for (uint32_t e = q[r]; e != 0; e = q[r]) r -= e;
        if (r != (uint32_t)x - d) q[x] = (uint32_t)x - r;
    }
}

// ---- adjacency (neighbour ids, grouped by vertex) ------------------------------
//
// By a counting sort in two levels.  Buckets of 2^sh consecutive vertices
// (nb <= kMaxBuckets of them): every block counts the arcs of its tile of the
// edge list per bucket in LDS and adds the counts to the bucket totals; after a
// scan of the totals each block reserves one run per bucket and writes its arcs
// (source, target) there; then one block per bucket counts its arcs per source
// in LDS, scans the counts into the vertex heads and places every target.  Only
// nb global atomics per block are left of the 4E a direct build would make
// (a degree count and a slot reservation per arc end).  Graphs with more
// vertices than the bucket limit allows use the direct build.
constexpr int kMaxBuckets = 4096;
constexpr int kMaxBucketShift = 13;     // 2^13 counters = 32 KB of LDS per block
constexpr int kBktBlocks = 512;

__device__ __forceinline__ bool arc_edge(int2 e, int32_t V) {
    return (uint32_t)e.x < (uint32_t)V && (uint32_t)e.y < (uint32_t)V && e.x != e.y;
}

// in-place exclusive scan of v[0..n) (n <= 256 * per) by one block; returns the total
__device__ uint32_t block_scan_lds(uint32_t* v, int n, uint32_t* part) {
    const int per = (n + kT - 1) / kT;
    const int l0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int j = 0; j < per; j++)
        if (l0 + j < n) s += v[l0 + j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kT; off <<= 1) {
        const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t ex = part[threadIdx.x] - s;
    for (int j = 0; j < per; j++)
        if (l0 + j < n) { const uint32_t c = v[l0 + j]; v[l0 + j] = ex; ex += c; }
    const uint32_t total = part[kT - 1];
    __syncthreads();
    return total;
}

__device__ __forceinline__ void tile_of(int64_t E, int64_t& lo, int64_t& hi) {
    lo = E * blockIdx.x / gridDim.x;
    hi = E * (blockIdx.x + 1) / gridDim.x;
}

__device__ void count_tile(const int2* edges, int64_t lo, int64_t hi, int32_t V, int sh, uint32_t* h) {
    for (int64_t i = lo + threadIdx.x; i < hi; i += kT) {
        const int2 e = edges[i];
        if (!arc_edge(e, V)) continue;
        atomicAdd(&h[(uint32_t)e.x >> sh], 1u);
        atomicAdd(&h[(uint32_t)e.y >> sh], 1u);
    }
}

__global__ void __launch_bounds__(kT) k_bkt_count(const int2* edges, int64_t E, int32_t V, int sh, int nb,
                                                  uint32_t* total) {
    __shared__ uint32_t h[kMaxBuckets];
    for (int b = threadIdx.x; b < nb; b += kT) h[b] = 0;
    __syncthreads();
    int64_t lo, hi;
    tile_of(E, lo, hi);
    count_tile(edges, lo, hi, V, sh, h);
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kT)
        if (h[b]) atomicAdd(&total[b], h[b]);
}

// total[0..nb) -> base[0..nb] (exclusive, base[nb] = all arcs) and cur = base
__global__ void __launch_bounds__(kT) k_bkt_scan(const uint32_t* total, int nb, uint32_t* base, uint32_t* cur) {
    __shared__ uint32_t v[kMaxBuckets];
    __shared__ uint32_t part[kT];
    for (int b = threadIdx.x; b < nb; b += kT) v[b] = total[b];
    __syncthreads();
    const uint32_t all = block_scan_lds(v, nb, part);
    for (int b = threadIdx.x; b < nb; b += kT) { base[b] = v[b]; cur[b] = v[b]; }
    if (threadIdx.x == 0) base[nb] = all;
}

__global__ void __launch_bounds__(kT) k_bkt_scatter(const int2* edges, int64_t E, int32_t V, int sh, int nb,
                                                    uint32_t* cur, int2* arcs) {
    __shared__ uint32_t h[kMaxBuckets];
    for (int b = threadIdx.x; b < nb; b += kT) h[b] = 0;
    __syncthreads();
    int64_t lo, hi;
    tile_of(E, lo, hi);
    count_tile(edges, lo, hi, V, sh, h);
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kT)
        if (h[b]) h[b] = atomicAdd(&cur[b], h[b]);     // this block's run in bucket b
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += kT) {
        const int2 e = edges[i];
        if (!arc_edge(e, V)) continue;
        arcs[atomicAdd(&h[(uint32_t)e.x >> sh], 1u)] = e;
        arcs[atomicAdd(&h[(uint32_t)e.y >> sh], 1u)] = make_int2(e.y, e.x);
    }
}

// block b: the arcs of bucket b -> head[] of its vertices and adj[] (targets)
__global__ void __launch_bounds__(kT) k_bkt_csr(const int2* arcs, const uint32_t* base, int32_t V, int sh,
                                                uint32_t* head, int32_t* adj) {
    __shared__ uint32_t c[1 << kMaxBucketShift];
    __shared__ uint32_t part[kT];
    const int n = 1 << sh;
    const uint32_t mask = (uint32_t)n - 1;
    const int64_t lo = base[blockIdx.x], hi = base[blockIdx.x + 1];
    for (int l = threadIdx.x; l < n; l += kT) c[l] = 0;
    __syncthreads();
    for (int64_t k = lo + threadIdx.x; k < hi; k += kT) atomicAdd(&c[(uint32_t)arcs[k].x & mask], 1u);
    __syncthreads();
    block_scan_lds(c, n, part);
    const int64_t v0 = (int64_t)blockIdx.x << sh;
    for (int l = threadIdx.x; l < n; l += kT) {
        c[l] += (uint32_t)lo;
        if (v0 + l < V) head[v0 + l] = c[l];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) head[V] = (uint32_t)hi;
    __syncthreads();
    for (int64_t k = lo + threadIdx.x; k < hi; k += kT) {
        const int2 a = arcs[k];
        adj[atomicAdd(&c[(uint32_t)a.x & mask], 1u)] = a.y;
    }
}

// direct build (graphs past the bucket limit): degrees, then (after a scan of
// head) each arc at its place
__global__ void k_adj_degree(const int2* edges, int64_t E, int32_t V, uint32_t* head) {
    GRID_LOOP(i, E) {
        const int2 e = edges[i];
        if (!arc_edge(e, V)) continue;
        atomicAdd(&head[e.x], 1u);
        atomicAdd(&head[e.y], 1u);
    }
}

__global__ void k_adj_fill(const int2* edges, int64_t E, int32_t V, const uint32_t* head, uint32_t* cur, int32_t* adj) {
    GRID_LOOP(i, E) {
        const int2 e = edges[i];
        if (!arc_edge(e, V)) continue;
        adj[head[e.x] + atomicAdd(&cur[e.x], 1u)] = e.y;
        adj[head[e.y] + atomicAdd(&cur[e.y], 1u)] = e.x;
    }
}

// A level list holds one int4 per vertex: (vertex, first arc, end of its arcs, 0),
// so that a level's wavefront goes from its list entry straight to the arcs.

// search start: the root of every component is level 0 and the first frontier
__global__ void k_bfs_start(const uint32_t* q, int32_t V, const uint32_t* head, int32_t* par, uint64_t* cand,
                            int4* frontier, uint32_t* fcount) {
    GRID_LOOP(v, (int64_t)V) {
        const bool root = q[v] == 0;
        par[v] = -1;
        cand[v] = root ? 0 : kNoCand;
        if (root) frontier[atomicAdd(fcount, 1u)] = make_int4((int32_t)v, (int32_t)head[v], (int32_t)head[v + 1], 0);
    }
}

// level d: one wavefront per vertex w of the level -- its tree edge (parent
// from the candidate word) goes to slot base_d + (w's place in the level),
// base_d being the number of tree edges of the earlier levels (kept in
// base[d & 1]; block 0 writes base[(d + 1) & 1]); then its offers to the
// neighbours, newly reached ones appended with one reservation per wavefront.
// A wavefront's first list entry is loaded together with the level size (the
// list has room for V entries; entries past the level are stale and unused),
// and a neighbour's arc range is loaded together with the offer, so a level
// costs one dependent load fewer per step.
__global__ void k_bfs_level(const int4* level_list, const uint32_t* count, uint32_t* count_after_next, int32_t d,
                            int32_t V, uint32_t* base, const uint32_t* head, const int32_t* adj, const int32_t* par1,
                            uint64_t* cand, int32_t* par, int4* next_list, uint32_t* next_count, int2* out,
                            int64_t cap, uint32_t* err) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int4 first = wave < V ? level_list[wave] : make_int4(0, 0, 0, 0);
    const uint32_t n = *count;
    const uint32_t b0 = base[d & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *count_after_next = 0;                       // the count level d + 2 will use
        base[(d + 1) & 1] = b0 + (d > 0 ? n : 0u);
    }
    for (int64_t f = wave; f < n; f += waves) {
        const int4 it = f == wave ? first : level_list[f];
        const int32_t w = it.x;
        if (d > 0 && lane == 0) {
            const int32_t p = (int32_t)(cand[w] & 0xffffffffu);
            par[w] = p;
            const int64_t pos = (int64_t)b0 + f;
            if (pos < cap) out[pos] = make_int2(p, w);
            else atomicOr(err, 2u);
        }
        const uint64_t mine = ((uint64_t)(uint32_t)d << 32) | (uint32_t)w;
        const int64_t h0 = (uint32_t)it.y, h1 = (uint32_t)it.z;
        for (int64_t kb = h0; kb < h1; kb += 64) {
            const int64_t k = kb + lane;
            bool got = false;
            int32_t x = 0;
            uint32_t x0 = 0, x1 = 0;
            if (k < h1) {
                x = adj[k];
                if (!excluded(par1, w, x) && cand[x] > mine) {
                    x0 = head[x];
                    x1 = head[x + 1];
                    got = atomicMin(reinterpret_cast<unsigned long long*>(cand + x), (unsigned long long)mine) ==
                          (unsigned long long)kNoCand;
                }
            }
            const uint64_t m = __ballot(got);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                uint32_t at = 0;
                if (lane == leader) at = atomicAdd(next_count, (uint32_t)__popcll(m));
                at = __shfl(at, leader);
                if (got)
                    next_list[at + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                        make_int4(x, (int32_t)x0, (int32_t)x1, 0);
            }
        }
    }
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) { GRID_LOOP(i, n) p[i] = 0; }
// roots of F (no BFS parent) flagged 0, every other vertex 1
__global__ void k_root_flags(const int32_t* par1, int32_t V, uint32_t* flag) { GRID_LOOP(v, (int64_t)V) flag[v] = par1[v] < 0 ? 0u : 1u; }
__global__ void k_copy_u32(const uint32_t* a, uint32_t* b) { if (threadIdx.x == 0) *b = *a; }

}  // namespace

// bucket size 2^sh: about 1,000 to 2,000 buckets (at least 64 vertices each)
struct BktPlan {
    int sh, nb;
    bool on;
};

static BktPlan bucket_plan(int32_t V) {
    int sh = 6;
    while (sh < kMaxBucketShift && ((int64_t)V >> sh) >= 2048) sh++;
    const int64_t nb = ((int64_t)V + (int64_t(1) << sh) - 1) >> sh;
    return {sh, (int)std::min<int64_t>(nb, kMaxBuckets + 1), nb <= kMaxBuckets};
}

// Workspace words (4-byte) for the scan-first certificate of E edges on V vertices.
struct ApWs {
    uint32_t *q, *fcount, *err, *nout, *head, *cur, *btot, *bbase, *bcur;
    int32_t *par1, *par2, *adj;
    int4 *fa, *fb;
    uint64_t *cand, *scan_status;
    int2 *arcs, *f1, *f2;
    int64_t zero_words, words;
};

static ApWs ap_carve(char* base, int64_t E, int32_t V) {
    ApWs w{};
    const BktPlan P = bucket_plan(V);
    int64_t o = 0;
    auto take = [&](int64_t bytes) { char* p = base ? base + o : nullptr; o += (bytes + 255) & ~int64_t(255); return p; };
    // cleared together at the start
    w.q = reinterpret_cast<uint32_t*>(take(4 * (int64_t)V));
    w.head = reinterpret_cast<uint32_t*>(take(4 * ((int64_t)V + 1)));
    w.cur = reinterpret_cast<uint32_t*>(take(P.on ? 4 : 4 * (int64_t)V));
    w.btot = reinterpret_cast<uint32_t*>(take(4 * (int64_t)kMaxBuckets));
    w.fcount = reinterpret_cast<uint32_t*>(take(4 * 256));   // per-level frontier counts, then scan ticket
    w.err = reinterpret_cast<uint32_t*>(take(256));           // [0] error, [1..2] |F|, |F'|
    w.scan_status = reinterpret_cast<uint64_t*>(take(8 * (((int64_t)V + 1 + 1023) / 1024)));
    w.zero_words = o / 4;
    w.nout = w.err + 1;
    w.bbase = reinterpret_cast<uint32_t*>(take(4 * ((int64_t)kMaxBuckets + 1)));
    w.bcur = reinterpret_cast<uint32_t*>(take(4 * (int64_t)kMaxBuckets));
    w.par1 = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.par2 = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.fa = reinterpret_cast<int4*>(take(16 * (int64_t)V));
    w.fb = reinterpret_cast<int4*>(take(16 * (int64_t)V));
    w.cand = reinterpret_cast<uint64_t*>(take(8 * (int64_t)V));
    w.f1 = reinterpret_cast<int2*>(take(8 * (int64_t)std::max(V, 1)));
    w.f2 = reinterpret_cast<int2*>(take(8 * (int64_t)std::max(V, 1)));
    w.adj = reinterpret_cast<int32_t*>(take(8 * std::max<int64_t>(E, 1)));
    w.arcs = reinterpret_cast<int2*>(take(P.on ? 16 * std::max<int64_t>(E, 1) : 8));
    w.words = o / 4;
    return w;
}

int64_t scan_first_words(int64_t E, int32_t V) { return ap_carve(nullptr, E, V).words; }

// One breadth-first forest: levels are run in groups; a group ends early on
// the device (an empty level makes every later launch return at once), and
// the host only checks the level size between groups.
static int bfs_forest(const ApWs& W, int32_t V, const int32_t* par1, int32_t* par, int2* out, uint32_t* nout,
                      hipStream_t s, uint32_t* h_count, int* levels) {
    // fcount[0..127]: level sizes (ring), fcount[128..129]: tree edges before the level (ping-pong)
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kT), 0, s, W.fcount, (int64_t)130);
    hipLaunchKernelGGL(k_bfs_start, dim3(grid_for(V)), dim3(kT), 0, s, W.q, V, (const uint32_t*)W.head, par, W.cand, W.fa,
                       W.fcount);
    int4 *cur_l = W.fa, *nxt_l = W.fb;
    int d = 0;
    constexpr int kGroup = 16;
    for (;;) {
        for (int k = 0; k < kGroup && d < V; k++, d++) {
            hipLaunchKernelGGL(k_bfs_level, dim3(2048), dim3(kT), 0, s, (const int4*)cur_l,
                               (const uint32_t*)(W.fcount + d % 128), W.fcount + (d + 2) % 128, d, V, W.fcount + 128,
                               (const uint32_t*)W.head, (const int32_t*)W.adj, par1, W.cand, par, nxt_l,
                               W.fcount + (d + 1) % 128, out, (int64_t)V, W.err);
            std::swap(cur_l, nxt_l);
        }
        BR_HIP(hipGetLastError());
        BR_HIP(hipMemcpyAsync(h_count, W.fcount + d % 128, 4, hipMemcpyDeviceToHost, s));
        BR_HIP(hipStreamSynchronize(s));
        if (*h_count == 0 || d >= V) break;
    }
    // tree edges emitted = base after the last level that had vertices
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, s, W.fcount + 128 + (d & 1), nout);
    *levels = d;
    return BR_OK;
}

// components of the edges (minus the pairs of par1 when given): union-find in
// stages with full compression between them; afterwards q[v] == 0 exactly at
// the smallest vertex of each component
static void components(const ApWs& W, const int2* edges, int64_t E, int32_t V, const int32_t* par1, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(V)), dim3(kT), 0, s, W.q, (int64_t)V);
    const int64_t cuts[4] = {0, std::min<int64_t>(E, 2 * (int64_t)V), std::min<int64_t>(E, 8 * (int64_t)V), E};
    for (int k = 0; k < 3; k++) {
        if (cuts[k + 1] <= cuts[k]) continue;
        if (k > 0) hipLaunchKernelGGL(k_cc_compress, dim3(grid_for(V)), dim3(kT), 0, s, W.q, V);
        hipLaunchKernelGGL(k_cc, dim3(grid_for((cuts[k + 1] - cuts[k] + kCcU - 1) / kCcU)), dim3(kT), 0, s, edges, cuts[k],
                           cuts[k + 1], V, par1, W.q, W.err);
    }
    hipLaunchKernelGGL(k_cc_compress, dim3(grid_for(V)), dim3(kT), 0, s, W.q, V);
}

// The scan-first certificate (F, F') of d_edges, left on the device: F at
// *d_f1, F' at *d_f2, |F| and |F'| at (*d_cnt)[0..1], the error word at
// *d_err, and per vertex 0 at the roots of F, 1 elsewhere, at *d_roots.
int scan_first_device(const int2* edges, int64_t E, int32_t V, char* ws, hipStream_t s, uint32_t* h_small, int* levels1,
                      int* levels2, int2** d_f1, int2** d_f2, uint32_t** d_cnt, uint32_t** d_err, uint32_t** d_roots) {
    const ApWs W = ap_carve(ws, E, V);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(W.zero_words)), dim3(kT), 0, s, reinterpret_cast<uint32_t*>(ws),
                       W.zero_words);
    // components and adjacency
    components(W, edges, E, V, nullptr, s);
    const BktPlan P = bucket_plan(V);
    if (P.on) {
        const int g = (int)std::max<int64_t>(1, std::min<int64_t>(kBktBlocks, (E + 1023) / 1024));
        hipLaunchKernelGGL(k_bkt_count, dim3(g), dim3(kT), 0, s, edges, E, V, P.sh, P.nb, W.btot);
        hipLaunchKernelGGL(k_bkt_scan, dim3(1), dim3(kT), 0, s, (const uint32_t*)W.btot, P.nb, W.bbase, W.bcur);
        hipLaunchKernelGGL(k_bkt_scatter, dim3(g), dim3(kT), 0, s, edges, E, V, P.sh, P.nb, W.bcur, W.arcs);
        hipLaunchKernelGGL(k_bkt_csr, dim3(P.nb), dim3(kT), 0, s, (const int2*)W.arcs, (const uint32_t*)W.bbase, V, P.sh,
                           W.head, W.adj);
    } else {
        hipLaunchKernelGGL(k_adj_degree, dim3(grid_for(E)), dim3(kT), 0, s, edges, E, V, W.head);
        device_scan1(reinterpret_cast<int32_t*>(W.head), (int64_t)V + 1, W.scan_status, W.fcount + 255, s);
        hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(E)), dim3(kT), 0, s, edges, E, V, (const uint32_t*)W.head, W.cur,
                           W.adj);
    }
    BR_HIP(hipGetLastError());
    // F: breadth-first forest of G
    int rc = bfs_forest(W, V, nullptr, W.par1, W.f1, W.nout, s, h_small, levels1);
    if (rc) return rc;
    // F': breadth-first forest of G without F's vertex pairs (own components)
    components(W, edges, E, V, W.par1, s);
    rc = bfs_forest(W, V, W.par1, W.par2, W.f2, W.nout + 1, s, h_small, levels2);
    if (rc) return rc;
    hipLaunchKernelGGL(k_root_flags, dim3(grid_for(V)), dim3(kT), 0, s, (const int32_t*)W.par1, V, W.q);
    BR_HIP(hipGetLastError());
    *d_f1 = W.f1;
    *d_f2 = W.f2;
    *d_cnt = W.nout;
    *d_err = W.err;
    *d_roots = W.q;
    return BR_OK;
}

// The same certificate copied to the host (pinned h_f1 / h_f2, V pairs each).
int scan_first_certificate(const int2* edges, int64_t E, int32_t V, char* ws, hipStream_t s, uint32_t* h_small,
                           int2* h_f1, int2* h_f2, uint32_t* n1, uint32_t* n2, int* levels1, int* levels2) {
    int2 *f1 = nullptr, *f2 = nullptr;
    uint32_t *cnt = nullptr, *err = nullptr, *roots = nullptr;
    int rc = scan_first_device(edges, E, V, ws, s, h_small, levels1, levels2, &f1, &f2, &cnt, &err, &roots);
    if (rc) return rc;
    BR_HIP(hipMemcpyAsync(h_small, err, 16, hipMemcpyDeviceToHost, s));
    BR_HIP(hipStreamSynchronize(s));
    const uint32_t e = h_small[0];
    *n1 = std::min<uint32_t>(h_small[1], (uint32_t)V);
    *n2 = std::min<uint32_t>(h_small[2], (uint32_t)V);
    if (e & 1u) return fail(BR_ERANGE, "scan-first certificate: an edge has a vertex id outside [0, %d)", V);
    if (e) return fail(BR_EINTERNAL, "scan-first certificate: forest larger than V - 1");
    if (*n1) BR_HIP(hipMemcpyAsync(h_f1, f1, 8 * (size_t)*n1, hipMemcpyDeviceToHost, s));
    if (*n2) BR_HIP(hipMemcpyAsync(h_f2, f2, 8 * (size_t)*n2, hipMemcpyDeviceToHost, s));
    BR_HIP(hipStreamSynchronize(s));
    return BR_OK;
}

}  // namespace br
