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

#include <cstring>

#include "device_util.hpp"
#include "internal.hpp"

namespace br {

namespace {

constexpr int kT = 256;
constexpr uint64_t kNoCand = ~uint64_t(0);


__device__ __forceinline__ bool excluded(const int32_t* par1, int32_t u, int32_t w) {
    return par1 && (par1[w] == u || par1[u] == w);
}

// component union-find over the edges (skipping loops and, with par1, the
// pairs of the first forest); q[cs x] = x - parent(x), 0 at a root (cs words
// per vertex: 8 while the state stays within 64 MB, so that a hook, performed
// at the memory side, disturbs the words of fewer other vertices); the larger
// root is hooked under the smaller, so each component's root is its smallest id
__device__ __forceinline__ uint32_t cc_find(uint32_t* q, int64_t cs, uint32_t x) {
    uint32_t d = __hip_atomic_load(q + cs * (int64_t)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    while (d != 0) {
        const uint32_t p = x - d;
        const uint32_t dp = __hip_atomic_load(q + cs * (int64_t)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (dp == 0) return p;
        __hip_atomic_store(q + cs * (int64_t)x, d + dp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        x = p - dp;
        d = __hip_atomic_load(q + cs * (int64_t)x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    return x;
}

__device__ __forceinline__ void cc_unite(uint32_t* q, int64_t cs, uint32_t u, uint32_t v) {
    for (;;) {
        u = cc_find(q, cs, u);
        v = cc_find(q, cs, v);
        if (u == v) return;
        if (u < v) { const uint32_t t = u; u = v; v = t; }
        uint32_t expect = 0;
        if (__hip_atomic_compare_exchange_strong(q + cs * (int64_t)u, &expect, u - v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        u = u - expect;
    }
}

// edges [lo, hi), kCcU per thread with their loads issued together; an edge
// whose endpoints already have the same parent is done after two loads (after
// a full compression that parent is the root)
constexpr int kCcU = 4;

__global__ void k_cc(const int2* edges, int64_t lo, int64_t hi, int32_t V, const int32_t* par1, uint32_t* q, int64_t cs,
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
            pu[j] = ok[j] ? (uint32_t)e[j].x - __hip_atomic_load(q + cs * (int64_t)e[j].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0u;
            pv[j] = ok[j] ? (uint32_t)e[j].y - __hip_atomic_load(q + cs * (int64_t)e[j].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0u;
        }
#pragma unroll
        for (int j = 0; j < kCcU; j++)
            if (ok[j] && pu[j] != pv[j]) cc_unite(q, cs, pu[j], pv[j]);
    }
}

// every vertex straight under its root (no hook runs concurrently)
__global__ void k_cc_compress(uint32_t* q, int64_t cs, int32_t V) {
    GRID_LOOP(x, (int64_t)V) {
        const uint32_t d = q[cs * x];
        if (d == 0) continue;
        uint32_t r = (uint32_t)x - d;
        for (uint32_t e = q[cs * (int64_t)r]; e != 0; e = q[cs * (int64_t)r]) r -= e;
        if (r != (uint32_t)x - d) q[cs * x] = (uint32_t)x - r;
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
constexpr int kBktBlocks = 256;

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

// totals -> base[0..nb] (exclusive, base[nb] = all arcs) and the cursors = base
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
// Level counters are 64-bit words (arcs << 30 | vertices): the vertices of a
// level and the sum of their degrees, the latter choosing how the next level
// is found.  V <= 2^29 keeps the vertex count below bit 30 and 2E < 2^32 keeps
// the arc sum below bit 62.
constexpr int kCountBits = 30;
constexpr uint64_t kCountMask = (uint64_t(1) << kCountBits) - 1;
constexpr int kUpG = 16;    // lanes per vertex in a bottom-up level
constexpr int kUpU = 8;     // arcs per lane loaded together in a bottom-up level

// Returning atomics to one address are serialised at the memory side (about
// 12 ns each on MI355X, measured), so a level appends its newly reached
// vertices with one reservation per block, not per wavefront: a block of
// kLvT threads stages them in LDS and reserves its run once at its end; only
// a block whose LDS run is full reserves per wavefront for the rest.
constexpr int kLvT = 1024;
constexpr int kLvBlocks = 256;
constexpr int kLvBuf = 2048;

struct LevelLds {
    int4 buf[kLvBuf];
    uint32_t n, fail, arcs;
    uint32_t base;
};

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void lds_begin(LevelLds& L) {
    if (threadIdx.x == 0) {
        L.n = 0;
        L.fail = kLvBuf;
        L.arcs = 0;
    }
    __syncthreads();
}

// one wavefront step (whole wavefront active, m = ballot(add) != 0): the lanes
// with `add` stage (item, degree deg)
__device__ __forceinline__ void lds_stage(LevelLds& L, bool add, int4 item, uint32_t deg, uint64_t m,
                                          unsigned long long* ring, int4* list) {
    const uint32_t sum = wave_sum(add ? deg : 0u);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)m) - 1;
    const uint32_t cnt = (uint32_t)__popcll(m);
    uint32_t at = 0;
    if (lane == leader) at = atomicAdd(&L.n, cnt);
    at = __shfl(at, leader);
    if (at + cnt <= (uint32_t)kLvBuf) {
        if (lane == leader) atomicAdd(&L.arcs, sum);
        if (add) L.buf[at + lane_rank(m)] = item;
    } else {
        // LDS run full: this and every later step of the block reserve on their own
        uint32_t g = 0;
        if (lane == leader) {
            atomicMin(&L.fail, at);
            g = (uint32_t)(atomicAdd(ring, ((unsigned long long)sum << kCountBits) | (unsigned long long)cnt) & kCountMask);
        }
        g = __shfl(g, leader);
        if (add) list[g + lane_rank(m)] = item;
    }
}

// every thread of the block: LDS entries [0, min(n, fail)) are all written
// (steps succeed in order until the first that does not fit); one reservation
__device__ __forceinline__ void lds_flush(LevelLds& L, unsigned long long* ring, int4* list) {
    __syncthreads();
    const uint32_t stored = min(L.n, L.fail);
    if (threadIdx.x == 0 && stored)
        L.base = (uint32_t)(atomicAdd(ring, ((unsigned long long)L.arcs << kCountBits) | (unsigned long long)stored) &
                            kCountMask);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < stored; i += blockDim.x) list[L.base + i] = L.buf[i];
}

// search start: the root of every component is level 0 and the first frontier;
// block b takes the vertices [V b / G, V (b + 1) / G)
__global__ void __launch_bounds__(kLvT) k_bfs_start(const uint32_t* q, int64_t cs, int32_t V, const uint32_t* head, int32_t* par,
                                                    uint64_t* cand, int32_t* lvl, int4* frontier,
                                                    unsigned long long* ring) {
    __shared__ LevelLds L;
    lds_begin(L);
    const int64_t lo = (int64_t)V * blockIdx.x / gridDim.x, hi = (int64_t)V * (blockIdx.x + 1) / gridDim.x;
    // every thread of the block runs every turn (staging is a wavefront
    // operation, and the turns end with a barrier)
    for (int64_t turn = lo; turn < hi; turn += kLvT) {
        const int64_t v = turn + threadIdx.x;
        const bool in = v < hi;
        const bool root = in && q[cs * v] == 0;
        uint32_t h0 = 0, h1 = 0;
        if (in) {
            par[v] = -1;
            cand[v] = root ? 0 : kNoCand;
            lvl[v] = root ? 0 : -1;
        }
        if (root) {
            h0 = head[v];
            h1 = head[v + 1];
        }
        const uint64_t m = __ballot(root);
        if (m) lds_stage(L, root, make_int4((int32_t)v, (int32_t)h0, (int32_t)h1, 0), h1 - h0, m, ring, frontier);
        // empty the LDS run before the next turn could overflow it (graphs
        // with many components)
        __syncthreads();
        if (L.n > (uint32_t)(kLvBuf - kLvT)) {
            lds_flush(L, ring, frontier);
            __syncthreads();
            if (threadIdx.x == 0) {
                L.n = 0;
                L.fail = kLvBuf;
                L.arcs = 0;
            }
            __syncthreads();
        }
    }
    lds_flush(L, ring, frontier);
}

// Level d finds level d + 1 top-down or bottom-up, whichever costs less: the
// top-down pass scans the level's arcs (mf), often with a 64-bit atomic each,
// the bottom-up pass the arcs of the unvisited vertices (mu) with two loads
// each, after one look at every vertex; bottom-up is taken when
// mu + V/4 < 4 mf.  acc[0..1] (ping-pong by d) hold the tree edges emitted
// before level d, acc[2..3] the arcs of the levels before d; block 0 writes
// the values for d + 1 and clears the counter level d + 2 will use.
//
// Top-down: one wavefront per vertex w of the level -- its tree edge (parent
// from the candidate word) goes to slot base_d + (w's place in the level);
// then its offers to the neighbours by 64-bit atomic minimum of
// (d << 32 | w), the first touch of a neighbour reaching it.  A wavefront's
// first list entry is loaded together with the level counter (the list has
// room for V entries; entries past the level are stale and unused), and a
// neighbour's arc range together with the offer.
//
// Bottom-up: the level's tree edges are emitted one per thread; then kUpG
// lanes per unvisited vertex x scan its arcs for neighbours of level d (F's
// vertex pairs excluded in F'), kUpU arcs per lane loaded together, and the
// smallest one becomes x's parent -- the same choice the atomic minimum makes.
// Only x's own lanes write x's words.
__global__ void __launch_bounds__(kLvT) k_bfs_level(const int4* level_list, unsigned long long* ring, int32_t d,
                                                    int32_t V, uint64_t* acc, const uint32_t* head, const int32_t* adj,
                                                    const int32_t* par1, uint64_t* cand, int32_t* lvl, int32_t* par,
                                                    int4* next_list, int2* out, int64_t cap, uint32_t* err) {
    __shared__ LevelLds L;
    const int lane = threadIdx.x & 63;
    const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t threads = (int64_t)gridDim.x * blockDim.x;
    const int64_t wave = gtid >> 6;
    const int64_t waves = threads >> 6;
    const int4 first = wave < V ? level_list[wave] : make_int4(0, 0, 0, 0);
    const uint64_t cw = ring[d % 128];
    const uint32_t n = (uint32_t)(cw & kCountMask);
    const uint64_t mf = cw >> kCountBits;
    const uint64_t b0 = acc[d & 1], seen = acc[2 + (d & 1)];
    const uint64_t mu = (uint64_t)head[V] - seen - mf;      // arcs of the vertices in no level up to d
    unsigned long long* next = ring + (d + 1) % 128;
    if (gtid == 0) {
        ring[(d + 2) % 128] = 0;
        acc[(d + 1) & 1] = b0 + (d > 0 ? n : 0u);
        acc[2 + ((d + 1) & 1)] = seen + mf;
    }
    if (n == 0) return;         // the same for every thread
    lds_begin(L);
    if (mu + ((uint64_t)V >> 2) >= 4 * mf) {
        // ---- top-down
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
                    if (got) lvl[x] = d + 1;
                    lds_stage(L, got, make_int4(x, (int32_t)x0, (int32_t)x1, 0), x1 - x0, m, next, next_list);
                }
            }
        }
    } else {
        // ---- bottom-up
        if (d > 0) {
            for (int64_t f = gtid; f < n; f += threads) {
                const int32_t w = level_list[f].x;
                const int32_t p = (int32_t)(cand[w] & 0xffffffffu);
                par[w] = p;
                const int64_t pos = (int64_t)b0 + f;
                if (pos < cap) out[pos] = make_int2(p, w);
                else atomicOr(err, 2u);
            }
        }
        const int sub = lane & (kUpG - 1);
        // whole wavefronts run the loop: groups past V idle through the last turn
        const int64_t groups = threads / kUpG;
        const int64_t end = ((int64_t)V + 64 / kUpG - 1) / (64 / kUpG) * (64 / kUpG);
        for (int64_t x = gtid / kUpG; x < end; x += groups) {
            uint32_t best = 0xffffffffu, h0 = 0, h1 = 0;
            if (x < V && lvl[x] < 0) {
                h0 = head[x];
                h1 = head[x + 1];
                const int32_t px = par1 ? par1[x] : -1;
                // kUpU arcs per lane at a time: their loads, then their neighbours' words, issued together
                for (int64_t kb = (int64_t)h0 + sub; kb < h1; kb += kUpG * kUpU) {
                    int32_t y[kUpU], l[kUpU], py[kUpU];
#pragma unroll
                    for (int j = 0; j < kUpU; j++) y[j] = kb + j * kUpG < h1 ? adj[kb + j * kUpG] : -1;
#pragma unroll
                    for (int j = 0; j < kUpU; j++) {
                        l[j] = y[j] >= 0 ? lvl[y[j]] : -1;
                        py[j] = par1 && y[j] >= 0 ? par1[y[j]] : -1;
                    }
#pragma unroll
                    for (int j = 0; j < kUpU; j++)
                        if (l[j] == d && px != y[j] && py[j] != (int32_t)x && (uint32_t)y[j] < best) best = (uint32_t)y[j];
                }
            }
            for (int o = 1; o < kUpG; o <<= 1) best = min(best, (uint32_t)__shfl_xor(best, o));
            const bool found = sub == 0 && best != 0xffffffffu;
            if (found) {
                cand[x] = ((uint64_t)(uint32_t)d << 32) | best;
                lvl[x] = d + 1;
            }
            const uint64_t m = __ballot(found);
            if (m) lds_stage(L, found, make_int4((int32_t)x, (int32_t)h0, (int32_t)h1, 0), h1 - h0, m, next, next_list);
        }
    }
    lds_flush(L, next, next_list);
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) { GRID_LOOP(i, n) p[i] = 0; }
// roots of F (no BFS parent) flagged 0, every other vertex 1
__global__ void k_root_flags(const int32_t* par1, int32_t V, uint32_t* flag) { GRID_LOOP(v, (int64_t)V) flag[v] = par1[v] < 0 ? 0u : 1u; }
__global__ void k_copy_lo(const uint64_t* a, uint32_t* b) { if (threadIdx.x == 0) *b = (uint32_t)*a; }

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
    uint32_t *q, *ticket, *err, *nout, *head, *cur, *btot, *bbase, *bcur;
    uint64_t* ring;
    int32_t *par1, *par2, *adj, *lvl;
    int4 *fa, *fb;
    uint64_t *cand, *scan_status;
    int2 *arcs, *f1, *f2;
    int64_t cs;                 // words per vertex of the component state
    int64_t zero_words, words;
};

static ApWs ap_carve(char* base, int64_t E, int32_t V) {
    ApWs w{};
    const BktPlan P = bucket_plan(V);
    int64_t o = 0;
    auto take = [&](int64_t bytes) { char* p = base ? base + o : nullptr; o += (bytes + 255) & ~int64_t(255); return p; };
    // cleared together at the start
    w.cs = (int64_t)V * 32 <= (int64_t(64) << 20) ? 8 : 1;
    w.q = reinterpret_cast<uint32_t*>(take(4 * (int64_t)V * w.cs));
    w.head = reinterpret_cast<uint32_t*>(take(4 * ((int64_t)V + 1)));
    w.cur = reinterpret_cast<uint32_t*>(take(P.on ? 4 : 4 * (int64_t)V));
    w.btot = reinterpret_cast<uint32_t*>(take(4 * (int64_t)kMaxBuckets));
    w.ring = reinterpret_cast<uint64_t*>(take(8 * 256));     // level counters (ring of 128), acc[4]
    w.ticket = reinterpret_cast<uint32_t*>(take(4));          // ticket of the direct build's scan
    w.err = reinterpret_cast<uint32_t*>(take(256));           // [0] error, [1..2] |F|, |F'|
    w.scan_status = reinterpret_cast<uint64_t*>(take(8 * (((int64_t)V + 1 + 1023) / 1024)));
    w.zero_words = o / 4;
    w.nout = w.err + 1;
    w.bbase = reinterpret_cast<uint32_t*>(take(4 * ((int64_t)kMaxBuckets + 1)));
    w.bcur = reinterpret_cast<uint32_t*>(take(4 * (int64_t)kMaxBuckets));
    w.par1 = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.par2 = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.lvl = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
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
    // ring[0..127]: level counters, ring[128..131]: acc (tree edges and arcs before the level, ping-pong)
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kT), 0, s, reinterpret_cast<uint32_t*>(W.ring), (int64_t)2 * 132);
    const int gs = (int)std::max<int64_t>(1, std::min<int64_t>(kLvBlocks, ((int64_t)V + kLvT - 1) / kLvT));
    hipLaunchKernelGGL(k_bfs_start, dim3(gs), dim3(kLvT), 0, s, W.q, W.cs, V, (const uint32_t*)W.head, par, W.cand, W.lvl, W.fa,
                       reinterpret_cast<unsigned long long*>(W.ring));
    int4 *cur_l = W.fa, *nxt_l = W.fb;
    int d = 0;
    constexpr int kGroup = 16;
    for (;;) {
        for (int k = 0; k < kGroup && d < V; k++, d++) {
            hipLaunchKernelGGL(k_bfs_level, dim3(kLvBlocks), dim3(kLvT), 0, s, (const int4*)cur_l,
                               reinterpret_cast<unsigned long long*>(W.ring), d, V, W.ring + 128, (const uint32_t*)W.head,
                               (const int32_t*)W.adj, par1, W.cand, W.lvl, par, nxt_l, out, (int64_t)V, W.err);
            std::swap(cur_l, nxt_l);
        }
        BR_HIP(hipGetLastError());
        BR_HIP(hipMemcpyAsync(h_count, W.ring + d % 128, 8, hipMemcpyDeviceToHost, s));
        BR_HIP(hipStreamSynchronize(s));
        uint64_t c = 0;
        std::memcpy(&c, h_count, 8);
        if ((c & kCountMask) == 0 || d >= V) break;
    }
    // tree edges emitted = acc after the last level that had vertices
    hipLaunchKernelGGL(k_copy_lo, dim3(1), dim3(64), 0, s, (const uint64_t*)(W.ring + 128 + (d & 1)), nout);
    *levels = d;
    return BR_OK;
}

// components of the edges (minus the pairs of par1 when given): union-find in
// stages with full compression between them; afterwards q[cs v] == 0 exactly at
// the smallest vertex of each component
static void components(const ApWs& W, const int2* edges, int64_t E, int32_t V, const int32_t* par1, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(V * W.cs)), dim3(kT), 0, s, W.q, (int64_t)V * W.cs);
    const int64_t cuts[4] = {0, std::min<int64_t>(E, 2 * (int64_t)V), std::min<int64_t>(E, 8 * (int64_t)V), E};
    for (int k = 0; k < 3; k++) {
        if (cuts[k + 1] <= cuts[k]) continue;
        if (k > 0) hipLaunchKernelGGL(k_cc_compress, dim3(grid_for(V)), dim3(kT), 0, s, W.q, W.cs, V);
        hipLaunchKernelGGL(k_cc, dim3(grid_for((cuts[k + 1] - cuts[k] + kCcU - 1) / kCcU)), dim3(kT), 0, s, edges, cuts[k],
                           cuts[k + 1], V, par1, W.q, W.cs, W.err);
    }
    hipLaunchKernelGGL(k_cc_compress, dim3(grid_for(V)), dim3(kT), 0, s, W.q, W.cs, V);
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
        device_scan1(reinterpret_cast<int32_t*>(W.head), (int64_t)V + 1, W.scan_status, W.ticket, s);
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
