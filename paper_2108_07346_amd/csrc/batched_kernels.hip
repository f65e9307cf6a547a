// Batched certificates for many small graphs in one persistent launch.
//
// Work items are (graph, chunk) pairs: graph g's edge list is split into M_g
// chunks exactly as in the paper's phase tree (Section III), and the items are
// handed out largest-first from a device queue.  A workgroup certifies one
// chunk (Algorithm 2) with the whole union-find state in LDS, then takes part
// in the graph's merge tree: the merge of nodes i and i + 2^(q-1) in round q
// is done by whichever workgroup finishes the second of the two (an arrival
// counter per merge), re-running the certificate on the union of the two
// certificates, again in LDS.  Node 0's region of each graph ends up holding
// the graph's certificate: F from the front, F' from the back.
//
// LDS union-find: one 32-bit word per vertex, low half = x - parent in F,
// high half = x - parent in F' (0 = root; V <= kMaxV keeps both in 16 bits).
// Hooking is a 32-bit LDS compare-and-swap that changes one half; a swap that
// fails because the other half moved is simply retried.  The larger root is
// hooked under the smaller representative, so chains decrease and the loop
// ends (see cert_kernels.hip for the argument).

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace br {

namespace {

constexpr int kBB = 512;          // threads per workgroup
constexpr int kMaxV = 4096;       // vertices per graph in LDS
constexpr int kStage = 2 * (kMaxV - 1);

struct LdsState {
    uint32_t q[kMaxV];            // packed F / F' offsets
    uint32_t stage[kStage];       // merged certificate: (u | v << 16), F from front, F' from back
    uint32_t n1, n2;              // counters of the current certificate
    int32_t item, last, errv;
};

template <int F>
__device__ __forceinline__ uint32_t half(uint32_t w) { return F ? (w >> 16) : (w & 0xffffu); }

template <int F>
__device__ __forceinline__ uint32_t with_half(uint32_t w, uint32_t h) {
    return F ? ((w & 0xffffu) | (h << 16)) : ((w & 0xffff0000u) | h);
}

template <int F>
__device__ __forceinline__ uint32_t lfind(uint32_t* q, uint32_t x) {
    uint32_t w = q[x];
    uint32_t d = half<F>(w);
    while (d != 0) {
        const uint32_t p = x - d;
        const uint32_t dp = half<F>(q[p]);
        if (dp == 0) return p;
        // path halving by compare-and-swap: the other half of the word may be
        // changing under a concurrent hook, so never overwrite it blindly; a
        // failed swap just skips this shortcut
        atomicCAS(&q[x], w, with_half<F>(w, d + dp));
        x = p - dp;
        w = q[x];
        d = half<F>(w);
    }
    return x;
}

template <int F>
__device__ __forceinline__ bool lunite(uint32_t* q, uint32_t u, uint32_t v) {
    for (;;) {
        u = lfind<F>(q, u);
        v = lfind<F>(q, v);
        if (u == v) return false;
        if (u < v) { const uint32_t t = u; u = v; v = t; }
        uint32_t w = q[u];
        for (;;) {
            if (half<F>(w) != 0) break;                       // u was hooked meanwhile
            const uint32_t nw = with_half<F>(w, u - v);
            const uint32_t old = atomicCAS(&q[u], w, nw);
            if (old == w) return true;
            w = old;                                          // other half changed, or u hooked
        }
        u = u - half<F>(w);
    }
}

// Offer (u,v) to F, then to F'.  Both parents come from one 32-bit word per
// endpoint: when the endpoints already share a parent in a forest (the usual
// case once the state is compressed) that forest rejects without a search.
__device__ __forceinline__ void loffer(uint32_t* q, uint32_t u, uint32_t v, bool& a1, bool& a2) {
    const uint32_t wu = q[u], wv = q[v];
    const uint32_t p1u = u - (wu & 0xffffu), p1v = v - (wv & 0xffffu);
    a1 = (p1u != p1v) && lunite<0>(q, p1u, p1v);
    a2 = false;
    if (!a1) {
        const uint32_t p2u = u - (wu >> 16), p2v = v - (wv >> 16);
        a2 = (p2u != p2v) && lunite<1>(q, p2u, p2v);
    }
}

// Full path compression of the LDS state (no concurrent hooks: called between
// barriers), so that later edges inside a component hit the shared-parent test.
__device__ void lcompress(uint32_t* q, uint32_t V) {
    for (uint32_t x = threadIdx.x; x < V; x += blockDim.x) {
        const uint32_t w = q[x];
        uint32_t r1 = x - (w & 0xffffu), r2 = x - (w >> 16);
        for (uint32_t d = q[r1] & 0xffffu; d; d = q[r1] & 0xffffu) r1 -= d;
        for (uint32_t d = q[r2] >> 16; d; d = q[r2] >> 16) r2 -= d;
        const uint32_t nw = (x - r1) | ((x - r2) << 16);
        if (nw != w) atomicCAS(&q[x], w, nw);
    }
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// wavefront-aggregated reservation of slots on an LDS counter
__device__ __forceinline__ uint32_t reserve(uint32_t* ctr, bool want, uint64_t& mask) {
    mask = __ballot(want);
    if (mask == 0) return 0;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(mask));
    return __shfl(base, leader) + lane_rank(mask);
}

__device__ __forceinline__ int64_t part_lo(int64_t E, int64_t M, int64_t i) { return i * (E / M) + (i * (E % M)) / M; }

}  // namespace



namespace {

// Certify edges [t0, t1) of graph g (ids < V) into an empty LDS state and write
// the accepted edges to node region (off, cap).  Counts go to S.n1, S.n2.
// Each thread takes kU edges per step and the next step's edges are loaded
// before the current ones are offered, so that enough loads are in flight to
// cover HBM latency while the LDS work proceeds.
constexpr int kU = 4;

__device__ __forceinline__ void load_step(const BatchDev& B, int64_t base, int64_t t1, int2 (&e)[kU]) {
    for (int j = 0; j < kU; j++) {
        const int64_t i = base + j * kBB + threadIdx.x;
        e[j] = i < t1 ? B.edges[i] : make_int2(-1, -1);
    }
}

__device__ void certify_chunk(LdsState& S, const BatchDev& B, int64_t t0, int64_t t1, uint32_t V, int64_t off,
                              int64_t cap) {
    for (uint32_t x = threadIdx.x; x < V; x += kBB) S.q[x] = 0;
    if (threadIdx.x == 0) { S.n1 = 0; S.n2 = 0; }
    __syncthreads();
    // compress after the first 2V and 8V edges (dense chunks are then mostly
    // rejected by the shared-parent test)
    int64_t next_cmp = t0 + 2 * (int64_t)V;
    constexpr int64_t kStep = (int64_t)kBB * kU;
    int2 cur[kU], nxt[kU];
    if (t0 < t1) load_step(B, t0, t1, cur);
    for (int64_t base = t0; base < t1; base += kStep) {
        if (base >= next_cmp) {
            __syncthreads();
            lcompress(S.q, V);
            __syncthreads();
            next_cmp = next_cmp == t0 + 2 * (int64_t)V ? t0 + 8 * (int64_t)V : INT64_MAX;
        }
        if (base + kStep < t1) load_step(B, base + kStep, t1, nxt);
        for (int j = 0; j < kU; j++) {
            const int2 e = cur[j];
            const bool live = base + j * kBB + threadIdx.x < t1;
            bool a1 = false, a2 = false;
            if (live) {
                if ((uint32_t)e.x < V && (uint32_t)e.y < V) loffer(S.q, (uint32_t)e.x, (uint32_t)e.y, a1, a2);
                else atomicOr(B.err, 1u);
            }
            uint64_t m;
            const uint32_t p1 = reserve(&S.n1, a1, m);
            if (a1) { if (p1 < cap) B.cert[off + p1] = e; else atomicOr(B.err, 2u); }
            const uint32_t p2 = reserve(&S.n2, a2, m);
            if (a2) { if (p2 < cap) B.cert[off + cap - 1 - p2] = e; else atomicOr(B.err, 2u); }
        }
        for (int j = 0; j < kU; j++) cur[j] = nxt[j];
    }
    __syncthreads();
}

// Offer the certificate stored in node region (off, cap) with counts (n1, n2)
// to the LDS state, staging accepted edges in S.stage.
__device__ void offer_region(LdsState& S, const BatchDev& B, int64_t off, int64_t cap, uint32_t n1, uint32_t n2) {
    const int64_t total = (int64_t)n1 + n2;
    for (int64_t base = 0; base < total; base += kBB) {
        const int64_t k = base + threadIdx.x;
        bool a1 = false, a2 = false;
        int2 e = make_int2(0, 0);
        if (k < total) {
            const uint64_t r = __hip_atomic_load(reinterpret_cast<const uint64_t*>(B.cert + (k < n1 ? off + k : off + cap - n2 + (k - n1))),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            e = make_int2((int32_t)(uint32_t)r, (int32_t)(uint32_t)(r >> 32));
            if ((uint32_t)e.x < kMaxV && (uint32_t)e.y < kMaxV) loffer(S.q, (uint32_t)e.x, (uint32_t)e.y, a1, a2);
            else atomicOr(B.err, 2u);
        }
        const uint32_t w = (uint32_t)e.x | ((uint32_t)e.y << 16);
        uint64_t m;
        const uint32_t p1 = reserve(&S.n1, a1, m);
        if (a1) { if (p1 < kStage) S.stage[p1] = w; else atomicOr(B.err, 2u); }
        const uint32_t p2 = reserve(&S.n2, a2, m);
        if (a2) { if (p2 < kStage) S.stage[kStage - 1 - p2] = w; else atomicOr(B.err, 2u); }
    }
}

}  // namespace

__global__ void __launch_bounds__(kBB) k_batched(BatchDev B) {
    __shared__ LdsState S;
    for (;;) {
        if (threadIdx.x == 0) S.item = (int32_t)atomicAdd(B.queue, 1u);
        __syncthreads();
        const int64_t it = S.item;
        if (it >= B.n_items) break;
        const int64_t code = B.items[it];
        const int32_t g = (int32_t)(code >> 20);
        int64_t node = code & ((1 << 20) - 1);
        const int64_t Mg = B.Mg[g];
        const uint32_t V = (uint32_t)B.V[g];
        const int64_t e0 = B.eoff[2 * g], Eg = B.eoff[2 * g + 1] - e0;
        const int64_t rb = B.rbase[g];
        auto nidx = [&](int64_t k) { return k ? rb + k - 1 : (int64_t)g; };
        // phase 0: chunk `node` of graph g
        certify_chunk(S, B, e0 + part_lo(Eg, Mg, node), e0 + part_lo(Eg, Mg, node + 1), V, B.noff[nidx(node)],
                      B.ncap[nidx(node)]);
        uint32_t n1 = S.n1, n2 = S.n2;
        // merge rounds: climb while this workgroup is the second of a pair to finish
        int64_t step = 1, level = 0, cb = B.cbase[g];
        for (;;) {
            if (threadIdx.x == 0) {
                B.ncnt[2 * nidx(node)] = n1;
                B.ncnt[2 * nidx(node) + 1] = n2;
            }
            if (step >= Mg) {                               // node 0 holds the graph's certificate
                // the LDS state encodes its F: publish the roots of F's trees
                const int64_t vb = B.vbase[g];
                for (uint32_t x = threadIdx.x; x < V; x += kBB) B.rootw[vb + x] = (S.q[x] & 0xffffu) ? 1u : 0u;
                break;
            }
            const int64_t i = node & ~(2 * step - 1);       // left node of this round's pair
            const int64_t j = i + step;
            if (j >= Mg) {                                  // no partner: pass through
                node = i;
                step *= 2;
                level++;
                continue;
            }
            // publish this node's certificate: the barrier orders every
            // thread's stores before thread 0's device-scope release (which
            // writes the XCD's L2 back), then one arrival per workgroup
            __syncthreads();
            if (threadIdx.x == 0) {
                __threadfence();
                const uint32_t prev = atomicAdd(&B.arrive[cb + level * ((Mg + 1) / 2) + (i >> (level + 1))], 1u);
                S.last = prev == 1u;
                if (S.last) __threadfence();                // acquire the partner's certificate
            }
            __syncthreads();
            if (!S.last) break;                             // the partner will merge
            // merge: Certificate(X_i u X_j), staged in LDS, written back to node i
            for (uint32_t x = threadIdx.x; x < V; x += kBB) S.q[x] = 0;
            if (threadIdx.x == 0) { S.n1 = 0; S.n2 = 0; }
            __syncthreads();
            const uint32_t ai1 = __hip_atomic_load(&B.ncnt[2 * nidx(i)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ai2 = __hip_atomic_load(&B.ncnt[2 * nidx(i) + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t aj1 = __hip_atomic_load(&B.ncnt[2 * nidx(j)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t aj2 = __hip_atomic_load(&B.ncnt[2 * nidx(j) + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t offi = B.noff[nidx(i)], capi = B.ncap[nidx(i)];
            const int64_t offj = B.noff[nidx(j)], capj = B.ncap[nidx(j)];
            offer_region(S, B, offi, capi, min(ai1, (uint32_t)capi), min(ai2, (uint32_t)capi - min(ai1, (uint32_t)capi)));
            offer_region(S, B, offj, capj, min(aj1, (uint32_t)capj), min(aj2, (uint32_t)capj - min(aj1, (uint32_t)capj)));
            __syncthreads();
            n1 = min(S.n1, (uint32_t)kStage);
            n2 = min(S.n2, (uint32_t)kStage - n1);
            if ((int64_t)n1 + n2 > capi) {
                if (threadIdx.x == 0) atomicOr(B.err, 2u);
                n1 = 0;
                n2 = 0;
            }
            for (uint32_t k = threadIdx.x; k < n1 + n2; k += kBB) {
                const uint32_t w = k < n1 ? S.stage[k] : S.stage[kStage - n2 + (k - n1)];
                const int64_t pos = k < n1 ? offi + k : offi + capi - n2 + (k - n1);
                B.cert[pos] = make_int2((int32_t)(w & 0xffffu), (int32_t)(w >> 16));
            }
            __syncthreads();
            node = i;
            step *= 2;
            level++;
        }
        __syncthreads();
    }
}

namespace {

// ---- bridge step of one small graph, entirely in LDS --------------------------
//
// The same computation as the bridge step on the device for one large
// certificate (bridge_kernels.hip), for the certificate that k_batched left in
// node 0's region of a graph with V <= kMaxV: F rooted by its Euler tours
// (list ranking by pointer jumping), preorder numbers and subtree sizes, each
// vertex's smallest and largest preorder number reachable through F' or
// itself, and a tree edge (parent(c), c) kept as a bridge iff the subtree of c
// reaches nothing outside its own preorder interval (the low-link test of
// Algorithm 1 applied to an arbitrary rooted spanning tree).  One workgroup
// per graph; buffers are reused from phase to phase.
constexpr int kST = 1024;                     // threads of the small-graph bridge step
constexpr int kMaxA = 2 * (kMaxV - 1);        // arcs of a spanning forest of kMaxV vertices
constexpr uint32_t kEnd = 0xffffu;
constexpr int kPerT = (kMaxA + kST - 1) / kST;   // arcs per thread

struct SmallLds {
    uint32_t e1[kMaxV];           // F edges, u | v << 16
    uint32_t head[kMaxV + 4];     // degrees, then adjacency starts
    uint32_t cur[kMaxV];          // fill cursors; tour base | tree base << 16 per root; then the keys
    uint16_t adj[kMaxA + 6];      // arcs by source; then down flags and their scan; then the min tree
    uint16_t posof[kMaxA + 6];    // place of each arc in its source's list; then tour length per root; then the max tree
    uint32_t link[kMaxA + 2];     // next arc | distance << 16; then lo / hi per preorder number
    uint16_t tail[kMaxA + 6];     // farthest arc reached; then each arc's place in its tour
    uint16_t in_arc[kMaxV];
    uint16_t sub[kMaxV];
    uint16_t pre[kMaxV];          // root of the vertex's tree, then its preorder number
    uint32_t wsum[kST / 64 + 2];
    uint32_t nkeys, total, base, bad;
};

// exclusive scan of one value per thread over the workgroup; total to *tot
__device__ __forceinline__ uint32_t wg_exclusive(uint32_t v, uint32_t* wsum, uint32_t* tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < kST / 64; i++) { const uint32_t c = wsum[i]; wsum[i] = t; t += c; }
        *tot = t;
    }
    __syncthreads();
    const uint32_t r = x - v + wsum[w];
    __syncthreads();
    return r;
}

// in-place exclusive scan of n <= 8 * kST 16-bit values
__device__ void scan_u16(uint16_t* a, int n, uint32_t* wsum, uint32_t* tot) {
    const int b = threadIdx.x * 8;
    uint32_t v[8], s = 0;
    for (int j = 0; j < 8; j++) { v[j] = b + j < n ? a[b + j] : 0u; s += v[j]; }
    uint32_t ex = wg_exclusive(s, wsum, tot);
    for (int j = 0; j < 8; j++) { if (b + j < n) a[b + j] = (uint16_t)ex; ex += v[j]; }
    __syncthreads();
}

__device__ __forceinline__ uint32_t e_src(const uint32_t* e1, uint32_t a) {
    const uint32_t e = e1[a >> 1];
    return (a & 1) ? (e >> 16) : (e & 0xffffu);
}
__device__ __forceinline__ uint32_t e_dst(const uint32_t* e1, uint32_t a) {
    const uint32_t e = e1[a >> 1];
    return (a & 1) ? (e & 0xffffu) : (e >> 16);
}

__global__ void __launch_bounds__(kST) k_small_bridges(const BatchDev B, int32_t S, uint32_t* out_hdr, uint32_t* out_keys) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    SmallLds& L = *reinterpret_cast<SmallLds*>(lds_raw);
    const int tid = threadIdx.x;
    for (int64_t g = blockIdx.x; g < S; g += gridDim.x) {
        const uint32_t V = (uint32_t)B.V[g];
        const int64_t off = B.noff[g], cap = B.ncap[g], vb = B.vbase[g];
        const uint32_t c1 = min((int64_t)B.ncnt[2 * g], cap);
        const uint32_t n1 = c1, n2 = (uint32_t)min((int64_t)B.ncnt[2 * g + 1], cap - (int64_t)c1);
        const uint32_t A = 2 * n1;
        if (tid == 0) { L.nkeys = 0; L.bad = 0; }
        __syncthreads();
        const bool ok = V >= 1 && V <= (uint32_t)kMaxV && n1 <= V - 1;
        if (!ok) {
            if (tid == 0) { atomicOr(B.err, 4u); out_hdr[16 + 2 * g] = 0; out_hdr[16 + 2 * g + 1] = 0; }
            __syncthreads();
            continue;
        }
        // ---- adjacency of F
        for (uint32_t k = tid; k < n1; k += kST) {
            const int2 e = B.cert[off + k];
            if ((uint32_t)e.x >= V || (uint32_t)e.y >= V || e.x == e.y) L.bad = 1;
            L.e1[k] = ((uint32_t)e.x & 0xffffu) | ((uint32_t)e.y << 16);
        }
        for (uint32_t x = tid; x <= V; x += kST) { L.head[x] = 0; if (x < V) { L.cur[x] = 0; L.pre[x] = kEnd; L.in_arc[x] = kEnd; L.sub[x] = 0; } }
        __syncthreads();
        if (L.bad) {
            if (tid == 0) { atomicOr(B.err, 4u); out_hdr[16 + 2 * g] = 0; out_hdr[16 + 2 * g + 1] = 0; }
            __syncthreads();
            continue;
        }
        for (uint32_t k = tid; k < n1; k += kST) {
            atomicAdd(&L.head[L.e1[k] & 0xffffu], 1u);
            atomicAdd(&L.head[L.e1[k] >> 16], 1u);
        }
        __syncthreads();
        {   // exclusive scan of head[0..V] (V + 1 <= 4097 entries, 8 per thread)
            const int b = tid * 8;
            uint32_t v[8], sm = 0;
            for (int j = 0; j < 8; j++) { v[j] = b + j <= (int)V ? L.head[b + j] : 0u; sm += v[j]; }
            uint32_t ex = wg_exclusive(sm, L.wsum, &L.total);
            for (int j = 0; j < 8; j++) { if (b + j <= (int)V) L.head[b + j] = ex; ex += v[j]; }
            __syncthreads();
        }
        for (uint32_t a = tid; a < A; a += kST) {
            const uint32_t x = e_src(L.e1, a);
            const uint32_t p = L.head[x] + atomicAdd(&L.cur[x], 1u);
            L.adj[p] = (uint16_t)a;
            L.posof[a] = (uint16_t)p;
        }
        __syncthreads();
        // ---- Euler tour successors, cut open at the roots of F
        for (uint32_t a = tid; a < A; a += kST) {
            const uint32_t y = e_dst(L.e1, a);
            const uint32_t p = L.posof[a ^ 1];
            const uint32_t nx = (p + 1 < L.head[y + 1]) ? p + 1 : L.head[y];
            uint32_t sx = L.adj[nx];
            if (B.rootw[vb + y] == 0 && p == L.head[y + 1] - 1) sx = kEnd;
            L.link[a] = sx == kEnd ? kEnd : (sx | (1u << 16));
            L.tail[a] = (uint16_t)(sx == kEnd ? a : sx);
        }
        __syncthreads();
        // ---- list ranking by pointer jumping
        for (uint32_t span = 1; span < A; span *= 2) {
            uint32_t nl[kPerT], nt[kPerT];
#pragma unroll
            for (int j = 0; j < kPerT; j++) {
                const uint32_t a = tid + j * kST;
                if (a >= A) continue;
                const uint32_t l = L.link[a];
                const uint32_t nx = l & 0xffffu;
                if (nx != kEnd) {
                    const uint32_t l2 = L.link[nx];
                    nl[j] = (l2 & 0xffffu) | (((l >> 16) + (l2 >> 16)) << 16);
                    nt[j] = L.tail[nx];
                } else {
                    nl[j] = l;
                    nt[j] = L.tail[a];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kPerT; j++) {
                const uint32_t a = tid + j * kST;
                if (a < A) { L.link[a] = nl[j]; L.tail[a] = (uint16_t)nt[j]; }
            }
            __syncthreads();
        }
        // ---- tours: arcs and vertices per root, and their prefix sums
        {
            const int b = tid * 4;
            uint32_t v[4], sm = 0;
            for (int j = 0; j < 4; j++) {
                const uint32_t r = b + j;
                uint32_t Lr = 0;
                if (r < V && B.rootw[vb + r] == 0 && L.head[r + 1] > L.head[r]) Lr = (L.link[L.adj[L.head[r]]] >> 16) + 1;
                v[j] = Lr | ((Lr ? Lr / 2 + 1 : 0u) << 16);
                sm += v[j];
            }
            uint32_t ex = wg_exclusive(sm, L.wsum, &L.total);
            for (int j = 0; j < 4; j++) {
                const uint32_t r = b + j;
                if (r < V) { L.cur[r] = ex; L.posof[r] = (uint16_t)(v[j] & 0xffffu); }
                ex += v[j];
            }
            __syncthreads();
        }
        const uint32_t nslots = L.total >> 16;   // vertices in trees of F
        for (uint32_t k = tid; k <= A; k += kST) L.adj[k] = 0;
        __syncthreads();
        // ---- place of every arc in its tour; downward arcs give parent arc, subtree size, tree root
        {
            uint32_t np[kPerT];
#pragma unroll
            for (int j = 0; j < kPerT; j++) {
                const uint32_t a = tid + j * kST;
                if (a >= A) continue;
                const uint32_t r = e_dst(L.e1, L.tail[a]);
                const uint32_t Lr = L.posof[r];
                const uint32_t p = Lr - 1 - (L.link[a] >> 16);
                const uint32_t ra = e_dst(L.e1, L.tail[a ^ 1]);
                const uint32_t pr = L.posof[ra] - 1 - (L.link[a ^ 1] >> 16);
                np[j] = p;
                if (p < pr && p < Lr && pr < Lr) {
                    const uint32_t y = e_dst(L.e1, a);
                    L.in_arc[y] = (uint16_t)a;
                    L.sub[y] = (uint16_t)((pr - p + 1) / 2);
                    L.pre[y] = (uint16_t)r;
                    L.adj[(L.cur[r] & 0xffffu) + p] = 1;
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kPerT; j++) {
                const uint32_t a = tid + j * kST;
                if (a < A) L.tail[a] = (uint16_t)np[j];
            }
            __syncthreads();
        }
        scan_u16(L.adj, (int)A + 1, L.wsum, &L.total);
        // ---- preorder numbers; lo = hi = own number
        uint32_t* lo = L.link;
        uint32_t* hi = L.link + kMaxV;
        for (uint32_t v = tid; v < V; v += kST) {
            uint32_t pv = kEnd;
            if (L.head[v + 1] > L.head[v]) {
                if (B.rootw[vb + v] == 0) {
                    pv = L.cur[v] >> 16;
                    L.sub[v] = (uint16_t)(L.posof[v] / 2 + 1);
                } else {
                    const uint32_t r = L.pre[v], ia = L.in_arc[v];
                    if (r < V && ia < A) {   // else only an inconsistent certificate
                        const uint32_t tb = L.cur[r] & 0xffffu, p = L.tail[ia];
                        if (tb + p <= A) pv = (L.cur[r] >> 16) + 1 + (L.adj[tb + p] - L.adj[tb]);
                    }
                }
                if (pv < nslots) { lo[pv] = pv; hi[pv] = pv; } else pv = kEnd;
            }
            L.pre[v] = (uint16_t)pv;
        }
        __syncthreads();
        for (uint32_t k = tid; k < n2; k += kST) {
            const int2 e = B.cert[off + cap - n2 + k];
            if ((uint32_t)e.x >= V || (uint32_t)e.y >= V) continue;
            const uint32_t px = L.pre[e.x], py = L.pre[e.y];
            if (px >= nslots || py >= nslots) continue;
            atomicMin(&lo[px], py);
            atomicMax(&hi[px], py);
            atomicMin(&lo[py], px);
            atomicMax(&hi[py], px);
        }
        __syncthreads();
        // ---- min / max trees over preorder numbers (leaves at [n, 2n))
        uint16_t* tmn = L.adj;
        uint16_t* tmx = L.posof;
        const uint32_t n = nslots;
        for (uint32_t i = tid; i < n; i += kST) { tmn[n + i] = (uint16_t)lo[i]; tmx[n + i] = (uint16_t)hi[i]; }
        __syncthreads();
        if (n > 1) {
            for (int lev = 31 - __clz(n - 1); lev >= 0; lev--) {
                const uint32_t i0 = 1u << lev, i1 = min(2u << lev, n);
                for (uint32_t i = i0 + tid; i < i1; i += kST) {
                    tmn[i] = min(tmn[2 * i], tmn[2 * i + 1]);
                    tmx[i] = max(tmx[2 * i], tmx[2 * i + 1]);
                }
                __syncthreads();
            }
        }
        // ---- the subtree test for every tree edge
        for (uint32_t v = tid; v < V; v += kST) {
            const uint32_t pv = L.pre[v];
            if (pv >= n || B.rootw[vb + v] == 0) continue;
            const uint32_t l = pv, r = pv + L.sub[v] - 1;
            if (r >= n || L.sub[v] == 0) continue;
            uint32_t mn = 0xffffu, mx = 0, x = l + n, y = r + n + 1;
            while (x < y) {
                if (x & 1) { mn = min(mn, (uint32_t)tmn[x]); mx = max(mx, (uint32_t)tmx[x]); x++; }
                if (y & 1) { y--; mn = min(mn, (uint32_t)tmn[y]); mx = max(mx, (uint32_t)tmx[y]); }
                x >>= 1;
                y >>= 1;
            }
            if (mn >= l && mx <= r) {
                const uint32_t e = L.e1[L.in_arc[v] >> 1];
                const uint32_t a = e & 0xffffu, b = e >> 16;
                L.cur[atomicAdd(&L.nkeys, 1u)] = (min(a, b) << 16) | max(a, b);
            }
        }
        __syncthreads();
        // ---- canonical order (bitonic sort) and output
        const uint32_t nk = min(L.nkeys, (uint32_t)kMaxV);
        uint32_t P = 1;
        while (P < nk) P <<= 1;
        for (uint32_t k = nk + tid; k < P; k += kST) L.cur[k] = 0xffffffffu;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = tid; i < P; i += kST) {
                    const uint32_t q = i ^ j;
                    if (q > i) {
                        const uint32_t x = L.cur[i], y = L.cur[q];
                        if (((i & k) == 0) == (x > y)) { L.cur[i] = y; L.cur[q] = x; }
                    }
                }
                __syncthreads();
            }
        }
        if (tid == 0) {
            L.base = nk ? atomicAdd(out_hdr, nk) : 0u;
            out_hdr[16 + 2 * g] = L.base;
            out_hdr[16 + 2 * g + 1] = nk;
        }
        __syncthreads();
        for (uint32_t k = tid; k < nk; k += kST) out_keys[L.base + k] = L.cur[k];
        __syncthreads();
    }
}

}  // namespace

size_t small_bridges_lds() { return sizeof(SmallLds); }

void launch_small_bridges(const BatchDev& B, int32_t S, uint32_t* out_hdr, uint32_t* out_keys, int blocks,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_small_bridges, dim3(blocks), dim3(kST), sizeof(SmallLds), s, B, S, out_hdr, out_keys);
}

int prepare_small_bridges() {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_bridges),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SmallLds));
    return e == hipSuccess ? 0 : -1;
}

void launch_batched(const BatchDev& B, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_batched, dim3(blocks), dim3(kBB), 0, s, B);
}

int32_t batched_max_v_dev() { return kMaxV; }
int32_t batched_blocks_per_cu() { return 3; }

}  // namespace br
