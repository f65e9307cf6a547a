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
// Pieces: a union-find pass for the components (roots are the smallest ids,
// as in cert_kernels.hip), an adjacency array of the edge list, and per BFS
// level an expand kernel (one wavefront per frontier vertex, candidate parents
// by 64-bit atomic min of (parent, edge id)) and a settle kernel (new levels,
// the next frontier, the chosen tree edges).
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

__global__ void k_cc(const int2* edges, int64_t E, int32_t V, const int32_t* par1, uint32_t* q, uint32_t* err) {
    GRID_LOOP(i, E) {
        const int2 e = edges[i];
        if ((uint32_t)e.x >= (uint32_t)V || (uint32_t)e.y >= (uint32_t)V) { atomicOr(err, 1u); continue; }
        if (e.x == e.y || excluded(par1, e.x, e.y)) continue;
        uint32_t u = (uint32_t)e.x, v = (uint32_t)e.y;
        for (;;) {
            u = cc_find(q, u);
            v = cc_find(q, v);
            if (u == v) break;
            if (u < v) { const uint32_t t = u; u = v; v = t; }
            uint32_t expect = 0;
            if (__hip_atomic_compare_exchange_strong(q + u, &expect, u - v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                break;
            u = u - expect;
        }
    }
}

// adjacency: degrees, then (after a scan of head) each arc at its place
__global__ void k_adj_degree(const int2* edges, int64_t E, int32_t V, int32_t* head) {
    GRID_LOOP(i, E) {
        const int2 e = edges[i];
        if ((uint32_t)e.x >= (uint32_t)V || (uint32_t)e.y >= (uint32_t)V || e.x == e.y) continue;
        atomicAdd(&head[e.x], 1);
        atomicAdd(&head[e.y], 1);
    }
}

__global__ void k_adj_fill(const int2* edges, int64_t E, int32_t V, const int32_t* head, int32_t* cur, int2* adj) {
    GRID_LOOP(i, E) {
        const int2 e = edges[i];
        if ((uint32_t)e.x >= (uint32_t)V || (uint32_t)e.y >= (uint32_t)V || e.x == e.y) continue;
        adj[head[e.x] + atomicAdd(&cur[e.x], 1)] = make_int2(e.y, (int32_t)i);
        adj[head[e.y] + atomicAdd(&cur[e.y], 1)] = make_int2(e.x, (int32_t)i);
    }
}

// search start: the root of every component is level 0 and the first frontier
__global__ void k_bfs_start(const uint32_t* q, int32_t V, int32_t* level, int32_t* par, uint64_t* cand,
                            int32_t* frontier, uint32_t* fcount) {
    GRID_LOOP(v, (int64_t)V) {
        const bool root = q[v] == 0;
        level[v] = root ? 0 : -1;
        par[v] = -1;
        cand[v] = kNoCand;
        if (root) frontier[atomicAdd(fcount, 1u)] = (int32_t)v;
    }
}

// one wavefront per frontier vertex u: every unreached neighbour w gets u as a
// candidate parent (smallest (u, edge id) wins)
__global__ void k_bfs_expand(const int32_t* frontier, const uint32_t* fcount, const int32_t* head, const int2* adj,
                             const int32_t* level, const int32_t* par1, uint64_t* cand) {
    const uint32_t n = *fcount;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t f = wave; f < n; f += waves) {
        const int32_t u = frontier[f];
        for (int32_t k = head[u] + lane; k < head[u + 1]; k += 64) {
            const int2 a = adj[k];
            const int32_t w = a.x;
            if (level[w] != -1 || excluded(par1, u, w)) continue;
            const uint64_t key = ((uint64_t)(uint32_t)u << 32) | (uint32_t)a.y;
            if (key < cand[w]) atomicMin(reinterpret_cast<unsigned long long*>(cand + w), (unsigned long long)key);
        }
    }
}

// vertices reached in this level: level, parent, next frontier, tree edge out
__global__ void k_bfs_settle(int32_t V, int32_t d, const int2* edges, int32_t* level, int32_t* par, uint64_t* cand,
                             int32_t* next, uint32_t* ncount, int2* out, uint32_t* nout, int64_t cap, uint32_t* err) {
    GRID_LOOP(v, (int64_t)V) {
        bool got = false;
        int2 e = make_int2(0, 0);
        if (level[v] == -1) {
            const uint64_t c = cand[v];
            if (c != kNoCand) {
                got = true;
                level[v] = d + 1;
                par[v] = (int32_t)(c >> 32);
                e = edges[c & 0xffffffffu];
                next[atomicAdd(ncount, 1u)] = (int32_t)v;
            }
        }
        const uint64_t m = __ballot(got);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            uint32_t base = 0;
            if (__lane_id() == leader) base = atomicAdd(nout, (uint32_t)__popcll(m));
            base = __shfl(base, leader);
            if (got) {
                const uint32_t pos = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (pos < cap) out[pos] = e;
                else atomicOr(err, 2u);
            }
        }
    }
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) { GRID_LOOP(i, n) p[i] = 0; }

}  // namespace

// Workspace words (4-byte) for the scan-first certificate of E edges on V vertices.
struct ApWs {
    uint32_t *q, *fcount, *err, *nout;
    int32_t *head, *cur, *level, *par1, *par2, *fa, *fb;
    uint64_t *cand, *scan_status;
    int2 *adj, *f1, *f2;
    int64_t zero_words, words;
};

static ApWs ap_carve(char* base, int64_t E, int32_t V) {
    ApWs w{};
    int64_t o = 0;
    auto take = [&](int64_t bytes) { char* p = base ? base + o : nullptr; o += (bytes + 255) & ~int64_t(255); return p; };
    // cleared together at the start
    w.q = reinterpret_cast<uint32_t*>(take(4 * (int64_t)V));
    w.head = reinterpret_cast<int32_t*>(take(4 * ((int64_t)V + 1)));
    w.cur = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.fcount = reinterpret_cast<uint32_t*>(take(4 * 256));   // per-level frontier counts, then scan ticket
    w.err = reinterpret_cast<uint32_t*>(take(256));           // [0] error, [1..2] |F|, |F'|
    w.scan_status = reinterpret_cast<uint64_t*>(take(8 * (((int64_t)V + 1 + 1023) / 1024)));
    w.zero_words = o / 4;
    w.nout = w.err + 1;
    w.level = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.par1 = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.par2 = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.fa = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.fb = reinterpret_cast<int32_t*>(take(4 * (int64_t)V));
    w.cand = reinterpret_cast<uint64_t*>(take(8 * (int64_t)V));
    w.f1 = reinterpret_cast<int2*>(take(8 * (int64_t)std::max(V, 1)));
    w.f2 = reinterpret_cast<int2*>(take(8 * (int64_t)std::max(V, 1)));
    w.adj = reinterpret_cast<int2*>(take(16 * std::max<int64_t>(E, 1)));
    w.words = o / 4;
    return w;
}

int64_t scan_first_words(int64_t E, int32_t V) { return ap_carve(nullptr, E, V).words; }

// One breadth-first forest: levels are run in groups; a group ends early on
// the device (an empty frontier makes every later launch return at once), and
// the host only checks the frontier count between groups.
static int bfs_forest(const ApWs& W, const int2* edges, int32_t V, const int32_t* par1, int32_t* par, int2* out,
                      uint32_t* nout, hipStream_t s, uint32_t* h_count, int* levels) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kT), 0, s, W.fcount, (int64_t)128);
    hipLaunchKernelGGL(k_bfs_start, dim3(grid_for(V)), dim3(kT), 0, s, W.q, V, W.level, par, W.cand, W.fa, W.fcount);
    int32_t *cur_f = W.fa, *nxt_f = W.fb;
    int d = 0;
    constexpr int kGroup = 16;
    for (;;) {
        for (int k = 0; k < kGroup && d < V; k++, d++) {
            uint32_t* fc = W.fcount + (d % 128);
            uint32_t* nc = W.fcount + ((d + 1) % 128);
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, nc, (int64_t)1);
            hipLaunchKernelGGL(k_bfs_expand, dim3(2048), dim3(kT), 0, s, (const int32_t*)cur_f, (const uint32_t*)fc,
                               (const int32_t*)W.head, (const int2*)W.adj, (const int32_t*)W.level, par1, W.cand);
            hipLaunchKernelGGL(k_bfs_settle, dim3(grid_for(V)), dim3(kT), 0, s, V, d, edges, W.level, par, W.cand, nxt_f,
                               nc, out, nout, (int64_t)V, W.err);
            std::swap(cur_f, nxt_f);
        }
        BR_HIP(hipGetLastError());
        BR_HIP(hipMemcpyAsync(h_count, W.fcount + (d % 128), 4, hipMemcpyDeviceToHost, s));
        BR_HIP(hipStreamSynchronize(s));
        if (*h_count == 0 || d >= V) break;
    }
    *levels = d;
    return BR_OK;
}

// The scan-first certificate (F, F') of d_edges on the device; on return the
// host holds |F|, |F'| and both edge lists (pinned buffers of the context).
int scan_first_certificate(const int2* edges, int64_t E, int32_t V, char* ws, hipStream_t s, uint32_t* h_small,
                           int2* h_f1, int2* h_f2, uint32_t* n1, uint32_t* n2, int* levels1, int* levels2) {
    const ApWs W = ap_carve(ws, E, V);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(W.zero_words)), dim3(kT), 0, s, reinterpret_cast<uint32_t*>(ws),
                       W.zero_words);
    // components and adjacency
    hipLaunchKernelGGL(k_cc, dim3(grid_for(E)), dim3(kT), 0, s, edges, E, V, (const int32_t*)nullptr, W.q, W.err);
    hipLaunchKernelGGL(k_adj_degree, dim3(grid_for(E)), dim3(kT), 0, s, edges, E, V, W.head);
    device_scan1(W.head, (int64_t)V + 1, W.scan_status, W.fcount + 255, s);
    hipLaunchKernelGGL(k_adj_fill, dim3(grid_for(E)), dim3(kT), 0, s, edges, E, V, (const int32_t*)W.head, W.cur, W.adj);
    BR_HIP(hipGetLastError());
    // F: breadth-first forest of G
    int rc = bfs_forest(W, edges, V, nullptr, W.par1, W.f1, W.nout, s, h_small, levels1);
    if (rc) return rc;
    // F': breadth-first forest of G without F's vertex pairs (own components)
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(V)), dim3(kT), 0, s, W.q, (int64_t)V);
    hipLaunchKernelGGL(k_cc, dim3(grid_for(E)), dim3(kT), 0, s, edges, E, V, (const int32_t*)W.par1, W.q, W.err);
    rc = bfs_forest(W, edges, V, W.par1, W.par2, W.f2, W.nout + 1, s, h_small, levels2);
    if (rc) return rc;
    BR_HIP(hipMemcpyAsync(h_small, W.err, 16, hipMemcpyDeviceToHost, s));
    BR_HIP(hipStreamSynchronize(s));
    const uint32_t err = h_small[0];
    *n1 = std::min<uint32_t>(h_small[1], (uint32_t)V);
    *n2 = std::min<uint32_t>(h_small[2], (uint32_t)V);
    if (err & 1u) return fail(BR_ERANGE, "scan-first certificate: an edge has a vertex id outside [0, %d)", V);
    if (err) return fail(BR_EINTERNAL, "scan-first certificate: forest larger than V - 1");
    if (*n1) BR_HIP(hipMemcpyAsync(h_f1, W.f1, 8 * (size_t)*n1, hipMemcpyDeviceToHost, s));
    if (*n2) BR_HIP(hipMemcpyAsync(h_f2, W.f2, 8 * (size_t)*n2, hipMemcpyDeviceToHost, s));
    BR_HIP(hipStreamSynchronize(s));
    return BR_OK;
}

}  // namespace br
