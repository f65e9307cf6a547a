// Bridges of the merged certificate on the GPU (an alternative to the host
// search of Algorithm 1 for the final step).
//
// The certificate is S = F u F' with F a spanning forest of the graph
// (Algorithm 2).  Every bridge lies in F.  Root each tree of F, number its
// vertices in preorder and record subtree sizes; then the tree edge
// (parent(c), c) is a bridge exactly when no edge of S joins the subtree of c
// to the rest: the smallest and largest preorder number adjacent (through F'
// edges, or the vertex itself) to any vertex of the subtree both stay inside
// the subtree's preorder interval.  This is the test the low-link of
// Algorithm 1 performs, applied to an arbitrary rooted spanning tree instead
// of a depth-first one (a parallel copy of a tree edge sits in F' and keeps
// it from being a bridge).
//
// Rooting uses the Euler tour of each tree: arcs 2k (u->v) and 2k+1 (v->u)
// of tree edge k, the successor of arc (x->y) being the arc after (y->x) in
// y's adjacency list, each tour cut open at its union-find root; list ranking
// by pointer jumping gives every arc its position in its tour.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace br {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int32_t arc_src(const int2* f1, int32_t a) { const int2 e = f1[a >> 1]; return (a & 1) ? e.y : e.x; }
__device__ __forceinline__ int32_t arc_dst(const int2* f1, int32_t a) { const int2 e = f1[a >> 1]; return (a & 1) ? e.x : e.y; }

#define GRID_LOOP(i, n) for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_zero_i32(int32_t* p, int64_t n) { GRID_LOOP(i, n) p[i] = 0; }

__global__ void k_degree(const int2* f1, const uint32_t* cnt, int32_t* deg) {
    const int64_t n1 = cnt[0];
    GRID_LOOP(k, n1) {
        const int2 e = f1[k];
        atomicAdd(&deg[e.x], 1);
        atomicAdd(&deg[e.y], 1);
    }
}

// ---- exclusive scan (int32), reduce-then-scan in blocks of kT*4 -------------
constexpr int kSB = kT * 4;

__device__ __forceinline__ int32_t block_exclusive(int32_t v, int32_t* sh, int32_t& total) {
    // inclusive scan of one value per thread across the block
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t s = 0;
        for (int i = 0; i < kT / 64; i++) { const int32_t t = sh[i]; sh[i] = s; s += t; }
        sh[kT / 64] = s;
    }
    __syncthreads();
    total = sh[kT / 64];
    const int32_t r = x - v + sh[w];
    __syncthreads();
    return r;
}

__global__ void k_scan_block(int32_t* a, int64_t n, int32_t* sums) {
    __shared__ int32_t sh[kT / 64 + 1];
    const int64_t base = blockIdx.x * (int64_t)kSB + threadIdx.x * 4;
    int32_t v[4], s = 0;
    for (int j = 0; j < 4; j++) { v[j] = base + j < n ? a[base + j] : 0; s += v[j]; }
    int32_t total;
    int32_t ex = block_exclusive(s, sh, total);
    for (int j = 0; j < 4; j++) { if (base + j < n) a[base + j] = ex; ex += v[j]; }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ void k_scan_add(int32_t* a, int64_t n, const int32_t* sums) {
    const int32_t add = sums[blockIdx.x];
    const int64_t base = blockIdx.x * (int64_t)kSB + threadIdx.x * 4;
    for (int j = 0; j < 4; j++) if (base + j < n) a[base + j] += add;
}

// ---- adjacency of F -----------------------------------------------------------
__global__ void k_fill_adj(const int2* f1, const uint32_t* cnt, const int32_t* head, int32_t* cur, int32_t* adj,
                           int32_t* posof) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) {
        const int32_t x = arc_src(f1, (int32_t)a);
        const int32_t p = head[x] + atomicAdd(&cur[x], 1);
        adj[p] = (int32_t)a;
        posof[a] = p;
    }
}

// successor in the Euler tour; tours cut open at union-find roots of F
__global__ void k_succ(const int2* f1, const uint32_t* cnt, const int32_t* head, const int32_t* adj,
                       const int32_t* posof, const uint32_t* q, int32_t qs, int32_t* nxt, int32_t* rank, int32_t* tail) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) {
        const int32_t y = arc_dst(f1, (int32_t)a);
        const int32_t p = posof[a ^ 1];
        const int32_t nx = (p + 1 < head[y + 1]) ? p + 1 : head[y];
        int32_t s = adj[nx];
        // arc (c -> r) closing the tour of root r: r's last listed arc is (r -> c)
        if (q[qs * (size_t)y] == 0 && p == head[y + 1] - 1) s = -1;
        nxt[a] = s;
        rank[a] = s < 0 ? 0 : 1;
        tail[a] = s < 0 ? (int32_t)a : s;
    }
}

__global__ void k_jump(const uint32_t* cnt, const int32_t* nxt, const int32_t* rank, const int32_t* tail, int32_t* nxt2,
                       int32_t* rank2, int32_t* tail2, int32_t* changed) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) {
        const int32_t s = nxt[a];
        if (s >= 0) {
            rank2[a] = rank[a] + rank[s];
            tail2[a] = tail[s];
            nxt2[a] = nxt[s];
            if (nxt[s] >= 0) *changed = 1;
        } else {
            rank2[a] = rank[a];
            tail2[a] = tail[a];
            nxt2[a] = -1;
        }
    }
}

// per root: tour length (arcs) and vertex count; written at the root's slot
__global__ void k_root_sizes(const int32_t* head, const int32_t* adj, const int32_t* rank, const uint32_t* q, int32_t qs,
                             int32_t V, int32_t* tour_len, int32_t* tree_n) {
    GRID_LOOP(r, (int64_t)V) {
        int32_t L = 0, nv = 0;
        if (q[qs * (size_t)r] == 0 && head[r + 1] > head[r]) {
            L = rank[adj[head[r]]] + 1;
            nv = L / 2 + 1;
        }
        tour_len[r] = L;
        tree_n[r] = nv;
    }
}

// tour position of every arc; downward arcs give parent, subtree size and a flag in tour order
__global__ void k_positions(const int2* f1, const uint32_t* cnt, const int32_t* rank, const int32_t* tail,
                            const int32_t* tour_len, const int32_t* tour_base, int32_t* pos, int32_t* flag) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) {
        const int32_t r = arc_dst(f1, tail[a]);
        const int32_t p = tour_len[r] - 1 - rank[a];
        pos[a] = p;
    }
}

__global__ void k_down(const int2* f1, const uint32_t* cnt, const int32_t* tail, const int32_t* pos,
                       const int32_t* tour_base, int32_t* flag, int32_t* in_arc, int32_t* sub) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) {
        const int32_t p = pos[a], pr = pos[a ^ 1];
        if (p < pr) {   // a = (x -> y) enters y for the first time
            const int32_t y = arc_dst(f1, (int32_t)a);
            const int32_t r = arc_dst(f1, tail[a]);
            flag[tour_base[r] + p] = 1;
            in_arc[y] = (int32_t)a;
            sub[y] = (pr - p + 1) / 2;
        }
    }
}

// preorder numbers; lo = hi = own preorder to start
__global__ void k_preorder(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* head, const int32_t* in_arc,
                           const int32_t* tail, const int32_t* pos, const int32_t* tour_base, const int32_t* down_ex,
                           const int32_t* vbase, const int32_t* tree_n, int32_t V, int32_t* pre, int32_t* sub, int32_t* lo,
                           int32_t* hi) {
    GRID_LOOP(v, (int64_t)V) {
        int32_t pv = -1;
        if (head[v + 1] > head[v]) {
            if (q[qs * (size_t)v] == 0) {        // root of its tree
                pv = vbase[v];
                sub[v] = tree_n[v];
            } else {
                const int32_t a = in_arc[v];
                const int32_t r = arc_dst(f1, tail[a]);
                pv = vbase[r] + 1 + (down_ex[tour_base[r] + pos[a]] - down_ex[tour_base[r]]);
            }
        }
        pre[v] = pv;
        lo[v] = pv;
        hi[v] = pv;
    }
}

// F' edges pull each endpoint's lo/hi toward the other endpoint's preorder
__global__ void k_nontree(const int2* f2, int32_t dir, const uint32_t* cnt, const int32_t* pre, int32_t* lo, int32_t* hi) {
    const int64_t n2 = cnt[1];
    GRID_LOOP(k, n2) {
        const int2 e = f2[dir * k];
        const int32_t px = pre[e.x], py = pre[e.y];
        atomicMin(&lo[e.x], py);
        atomicMax(&hi[e.x], py);
        atomicMin(&lo[e.y], px);
        atomicMax(&hi[e.y], px);
    }
}

__global__ void k_to_preorder(const int32_t* pre, const int32_t* lo, const int32_t* hi, int32_t V, int32_t* tmin,
                              int32_t* tmax) {
    GRID_LOOP(v, (int64_t)V) {
        const int32_t p = pre[v];
        if (p >= 0) { tmin[p] = lo[v]; tmax[p] = hi[v]; }
    }
}

__global__ void k_sparse_level(const int32_t* pmin, const int32_t* pmax, int32_t* cmin, int32_t* cmax, int64_t n,
                               int64_t half) {
    GRID_LOOP(i, n) {
        const int64_t j = i + half < n ? i + half : n - 1;
        cmin[i] = min(pmin[i], pmin[j]);
        cmax[i] = max(pmax[i], pmax[j]);
    }
}

__device__ __forceinline__ int floor_log2(uint32_t x) { return 31 - __clz(x); }

__global__ void k_bridges(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* head, const int32_t* in_arc,
                          const int32_t* pre, const int32_t* sub, const int32_t* tmin, const int32_t* tmax, int64_t nt,
                          int32_t V, uint64_t* out, uint32_t* nout) {
    GRID_LOOP(v, (int64_t)V) {
        bool br = false;
        uint64_t key = 0;
        if (head[v + 1] > head[v] && q[qs * (size_t)v] != 0) {
            const int32_t l = pre[v], r = pre[v] + sub[v] - 1;
            const int j = floor_log2((uint32_t)(r - l + 1));
            const int64_t lev = (int64_t)j * nt;
            const int32_t mn = min(tmin[lev + l], tmin[lev + r - (1 << j) + 1]);
            const int32_t mx = max(tmax[lev + l], tmax[lev + r - (1 << j) + 1]);
            if (mn >= l && mx <= r) {
                br = true;
                const int2 e = f1[in_arc[v] >> 1];
                const uint32_t a = (uint32_t)min(e.x, e.y), b = (uint32_t)max(e.x, e.y);
                key = (uint64_t)a << 32 | b;
            }
        }
        const uint64_t m = __ballot(br);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            uint32_t base = 0;
            if (__lane_id() == leader) base = atomicAdd(nout, (uint32_t)__popcll(m));
            base = __shfl(base, leader);
            if (br) out[base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] = key;
        }
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + kT - 1) / kT;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 16384));
}

}  // namespace

// scratch words needed by device_scan for n elements
int64_t scan_scratch_words(int64_t n);
static int64_t scan_scratch(int64_t n) { return scan_scratch_words(n); }
int64_t scan_scratch_words(int64_t n) {
    int64_t s = 0;
    while (n > kSB) {
        n = (n + kSB - 1) / kSB;
        s += n + 64;
    }
    return s + 64;
}

void device_scan(int32_t* a, int64_t n, int32_t* scratch, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = (n + kSB - 1) / kSB;
    if (blocks == 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(kT), 0, s, a, n, (int32_t*)nullptr);
        return;
    }
    int32_t* sums = scratch;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)blocks), dim3(kT), 0, s, a, n, sums);
    device_scan(sums, blocks, scratch + blocks + 64, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)blocks), dim3(kT), 0, s, a, n, (const int32_t*)sums);
}

// Scratch layout of the bridge step, shared by the size query and the launch
// sequence so that the two cannot disagree.
struct BridgeWs {
    int32_t *head, *cur, *adj, *posof, *nxt, *rank, *tail, *nxt2, *rank2, *tail2, *tour_len, *tree_n, *tour_base,
        *vbase, *pos, *flag, *in_arc, *sub, *pre, *lo, *hi, *tmin, *tmax, *misc, *scr;
    uint64_t* keys;
    int64_t words;
};

static BridgeWs carve(int32_t* base, int32_t V) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    int J = 1;
    while ((int64_t(1) << J) < V) J++;
    BridgeWs w{};
    int64_t o = 0;
    auto take = [&](int64_t n) { int32_t* p = base ? base + o : nullptr; o += (n + 63) & ~int64_t(63); return p; };
    w.head = take(V + 2);
    w.cur = take(V + 1);
    w.adj = take(A);
    w.posof = take(A);
    w.nxt = take(A);
    w.rank = take(A);
    w.tail = take(A);
    w.nxt2 = take(A);
    w.rank2 = take(A);
    w.tail2 = take(A);
    w.tour_len = take(V);
    w.tree_n = take(V);
    w.tour_base = take(V + 1);
    w.vbase = take(V + 1);
    w.pos = take(A);
    w.flag = take(A + 1);
    w.in_arc = take(V);
    w.sub = take(V);
    w.pre = take(V);
    w.lo = take(V);
    w.hi = take(V);
    w.tmin = take((int64_t)(J + 1) * V);
    w.tmax = take((int64_t)(J + 1) * V);
    w.keys = reinterpret_cast<uint64_t*>(take(2 * (int64_t)V + 2));
    w.misc = take(64);   // [0] changed flag, [1] key count
    w.scr = take(scan_scratch(std::max<int64_t>(A, V) + 1));
    w.words = o;
    return w;
}

int64_t device_bridges_words(int32_t V) { return carve(nullptr, V).words; }

// Bridges of a certificate held on the device: F = f1[0..cnt[0]), F' =
// f2[dir*k] for k < cnt[1] (counts read on the device), vertex v is the root of
// its tree of F iff q[qs*v] == 0.  Writes up to V keys at *d_keys and their
// number at *d_n.
int device_bridges_cert(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q, int32_t qs,
                        int32_t V, int32_t max_tree, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    // list ranking and the subtree range tables only need the largest tree:
    // tours have at most 2(max_tree - 1) arcs, subtrees at most max_tree vertices
    max_tree = std::max(2, std::min(max_tree, V));
    int J = 1;
    while ((int64_t(1) << J) < max_tree) J++;
    const BridgeWs W = carve(ws, V);
    int32_t *head = W.head, *cur = W.cur, *adj = W.adj, *posof = W.posof, *nxt = W.nxt, *rank = W.rank,
            *tail = W.tail, *nxt2 = W.nxt2, *rank2 = W.rank2, *tail2 = W.tail2, *tour_len = W.tour_len,
            *tree_n = W.tree_n, *tour_base = W.tour_base, *vbase = W.vbase, *pos = W.pos, *flag = W.flag,
            *in_arc = W.in_arc, *sub = W.sub, *pre = W.pre, *lo = W.lo, *hi = W.hi, *tmin = W.tmin, *tmax = W.tmax,
            *misc = W.misc, *scr = W.scr;
    uint64_t* keys = W.keys;
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(V + 2)), dim3(kT), 0, s, head, (int64_t)V + 2);
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(V + 1)), dim3(kT), 0, s, cur, (int64_t)V + 1);
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(A + 1)), dim3(kT), 0, s, flag, A + 1);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(kT), 0, s, misc, (int64_t)64);
    hipLaunchKernelGGL(k_degree, dim3(grid_for(V)), dim3(kT), 0, s, f1, cnt, head);
    device_scan(head, V + 1, scr, s);
    hipLaunchKernelGGL(k_fill_adj, dim3(grid_for(A)), dim3(kT), 0, s, f1, cnt, head, cur, adj, posof);
    hipLaunchKernelGGL(k_succ, dim3(grid_for(A)), dim3(kT), 0, s, f1, cnt, head, adj, posof, q, qs, nxt, rank, tail);
    int rounds = 0;
    while ((int64_t(1) << rounds) < 2 * (int64_t)max_tree) rounds++;
    for (int i = 0; i < rounds; i++) {
        hipLaunchKernelGGL(k_jump, dim3(grid_for(A)), dim3(kT), 0, s, cnt, nxt, rank, tail, nxt2, rank2, tail2, misc);
        std::swap(nxt, nxt2);
        std::swap(rank, rank2);
        std::swap(tail, tail2);
    }
    hipLaunchKernelGGL(k_root_sizes, dim3(grid_for(V)), dim3(kT), 0, s, head, adj, rank, q, qs, V, tour_len, tree_n);
    BR_HIP(hipMemcpyAsync(tour_base, tour_len, sizeof(int32_t) * V, hipMemcpyDeviceToDevice, s));
    BR_HIP(hipMemcpyAsync(vbase, tree_n, sizeof(int32_t) * V, hipMemcpyDeviceToDevice, s));
    device_scan(tour_base, V, scr, s);
    device_scan(vbase, V, scr, s);
    hipLaunchKernelGGL(k_positions, dim3(grid_for(A)), dim3(kT), 0, s, f1, cnt, rank, tail, tour_len, tour_base, pos, flag);
    hipLaunchKernelGGL(k_down, dim3(grid_for(A)), dim3(kT), 0, s, f1, cnt, tail, pos, tour_base, flag, in_arc, sub);
    device_scan(flag, A + 1, scr, s);
    hipLaunchKernelGGL(k_preorder, dim3(grid_for(V)), dim3(kT), 0, s, f1, q, qs, head, in_arc, tail, pos, tour_base, flag,
                       vbase, tree_n, V, pre, sub, lo, hi);
    hipLaunchKernelGGL(k_nontree, dim3(grid_for(V)), dim3(kT), 0, s, f2, dir, cnt, pre, lo, hi);
    hipLaunchKernelGGL(k_to_preorder, dim3(grid_for(V)), dim3(kT), 0, s, pre, lo, hi, V, tmin, tmax);
    for (int j = 1; j <= J; j++)
        hipLaunchKernelGGL(k_sparse_level, dim3(grid_for(V)), dim3(kT), 0, s, tmin + (int64_t)(j - 1) * V,
                           tmax + (int64_t)(j - 1) * V, tmin + (int64_t)j * V, tmax + (int64_t)j * V, (int64_t)V,
                           (int64_t)1 << (j - 1));
    hipLaunchKernelGGL(k_bridges, dim3(grid_for(V)), dim3(kT), 0, s, f1, q, qs, head, in_arc, pre, sub, tmin, tmax, (int64_t)V,
                       V, keys, reinterpret_cast<uint32_t*>(misc + 1));
    *d_keys = keys;
    *d_n = reinterpret_cast<uint32_t*>(misc + 1);
    return BR_OK;
}

// Bridges of node 0's certificate of the plain path (F' stored backwards from
// the end of the region; roots read from node 0's carried union-find state).
int device_bridges(const Plan& P, const DevBufs& B, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s) {
    const int2* f1 = B.cert + P.off[0];
    const int2* f2 = B.cert + P.off[0] + P.cap[0] - 1;
    return device_bridges_cert(f1, f2, -1, B.cnt, B.state, 2, P.V, P.V, ws, d_keys, d_n, s);
}

}  // namespace br
