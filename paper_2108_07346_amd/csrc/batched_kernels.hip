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
// high half = x - parent in F' (0 = root; V <= 65,536 keeps both in 16 bits).
// Two instances: graphs up to 4,096 vertices (three workgroups per CU) and
// graphs up to 40,944 vertices (the whole LDS of a CU, one workgroup).
// Hooking is a 32-bit LDS compare-and-swap that changes one half; a swap that
// fails because the other half moved is simply retried.  The larger root is
// hooked under the smaller representative, so chains decrease and the loop
// ends (see cert_kernels.hip for the argument).

#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace br {

namespace {

constexpr int kBB = 512;          // threads per workgroup
constexpr int kMaxV = 4096;       // vertices per graph of the small kernel
// the large kernel: the whole 160 KB of a CU's LDS for one graph's state, less
// the counters (the offsets stay 16-bit: V <= 65,536)
constexpr int kMaxVBig = (160 * 1024 - 64) / 4;

// Staged = true: a merge re-runs the certificate on X_i u X_j into a fresh
// state, staging the result in LDS before writing node i's region back (the
// small kernel).  Staged = false: a merge rebuilds node i's state from its
// own certificate (F's edges into F, F''s into F' -- all accepted, nothing
// written) and streams X_j in, appending what is accepted to node i's region
// after its edges (the same certificate as the state-carrying merge; no
// stage, so the state can take all of LDS).
template <int MaxV, bool Staged>
struct LdsState {
    static constexpr int kStage = Staged ? 2 * (MaxV - 1) : 1;
    uint32_t q[MaxV];             // packed F / F' offsets
    uint32_t stage[kStage];       // merged certificate: (u | v << 16), F from front, F' from back
    uint32_t n12;                 // edges of the current certificate: F in the low half, F' in the high
                                  // (each a forest count, at most V - 1 < 2^16, so no carry)
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


// wavefront-aggregated reservation of slots for F's and F''s accepted edges
// on the packed LDS counter: one atomic and one broadcast per wavefront step
// for both forests (the two were each an LDS atomic plus a permute)
__device__ __forceinline__ void reserve2(uint32_t* ctr, bool a1, bool a2, uint32_t& p1, uint32_t& p2) {
    const uint64_t m1 = __ballot(a1), m2 = __ballot(a2);
    p1 = p2 = 0;
    if ((m1 | m2) == 0) return;
    const int leader = __ffsll((unsigned long long)(m1 | m2)) - 1;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m1) | ((uint32_t)__popcll(m2) << 16));
    base = __shfl(base, leader);
    p1 = (base & 0xffffu) + lane_rank(m1);
    p2 = (base >> 16) + lane_rank(m2);
}

__device__ __forceinline__ int64_t part_lo(int64_t E, int64_t M, int64_t i) { return i * (E / M) + (i * (E % M)) / M; }

}  // namespace



namespace {

// Certify edges [t0, t1) of graph g (ids < V) into an empty LDS state and write
// the accepted edges to node region (off, cap).  Counts go to S.n12.
// Each thread takes kU edges per step and the next step's edges are loaded
// before the current ones are offered, so that enough loads are in flight to
// cover HBM latency while the LDS work proceeds.
constexpr int kU = 4;

__device__ __forceinline__ void load_step(const BatchDev& B, int64_t base, int64_t t1, int2 (&e)[kU]) {
#pragma unroll
    for (int j = 0; j < kU; j++) {
        const int64_t i = base + j * kBB + threadIdx.x;
        e[j] = i < t1 ? B.edges[i] : make_int2(-1, -1);
    }
}

template <class LS>
__device__ void certify_chunk(LS& S, const BatchDev& B, int64_t t0, int64_t t1, uint32_t V, int64_t off,
                              int64_t cap) {
    for (uint32_t x = threadIdx.x; x < V; x += kBB) S.q[x] = 0;
    if (threadIdx.x == 0) S.n12 = 0;
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
        if constexpr (LS::kStage >= kBB * kU) {
            // Where the stage area is free (it only serves merges), each
            // wavefront first applies the shared-parent test to all of its
            // kU x 64 edges and packs the ones the test cannot reject into a
            // list of its own there; those are then offered 64 at a time, so
            // that the searches of a few lanes no longer hold a whole
            // wavefront (in a dense chunk most edges are rejected by the test).
            uint32_t* wl = S.stage + (threadIdx.x / 64) * (64 * kU);
            uint32_t nh = 0;
#pragma unroll
            for (int j = 0; j < kU; j++) {
                const uint32_t x = (uint32_t)cur[j].x, y = (uint32_t)cur[j].y;
                bool hard = false;
                if (base + j * kBB + threadIdx.x < t1) {
                    if (x < V && y < V) {
                        const uint32_t wu = S.q[x], wv = S.q[y];
                        hard = x - (wu & 0xffffu) != y - (wv & 0xffffu) || x - (wu >> 16) != y - (wv >> 16);
                    } else {
                        atomicOr(B.err, 1u);
                    }
                }
                const uint64_t m = __ballot(hard);
                if (hard) wl[nh + lane_rank(m)] = x | (y << 16);
                nh += (uint32_t)__popcll(m);
            }
            __builtin_amdgcn_wave_barrier();     // the list, written by the wavefront's lanes, is read back by them
            for (uint32_t k0 = 0; k0 < nh; k0 += 64) {
                const uint32_t k = k0 + __lane_id();
                bool a1 = false, a2 = false;
                int2 e = make_int2(0, 0);
                if (k < nh) {
                    const uint32_t w = wl[k];
                    e = make_int2((int32_t)(w & 0xffffu), (int32_t)(w >> 16));
                    loffer(S.q, (uint32_t)e.x, (uint32_t)e.y, a1, a2);
                }
                uint32_t p1, p2;
                reserve2(&S.n12, a1, a2, p1, p2);
                if (a1) { if (p1 < cap) B.cert[off + p1] = e; else atomicOr(B.err, 2u); }
                if (a2) { if (p2 < cap) B.cert[off + cap - 1 - p2] = e; else atomicOr(B.err, 2u); }
            }
            __builtin_amdgcn_wave_barrier();     // every lane's reads of the list before the next step's writes
        } else {
#pragma unroll
            for (int j = 0; j < kU; j++) {
                const int2 e = cur[j];
                const bool live = base + j * kBB + threadIdx.x < t1;
                bool a1 = false, a2 = false;
                if (live) {
                    if ((uint32_t)e.x < V && (uint32_t)e.y < V) loffer(S.q, (uint32_t)e.x, (uint32_t)e.y, a1, a2);
                    else atomicOr(B.err, 1u);
                }
                uint32_t p1, p2;
                reserve2(&S.n12, a1, a2, p1, p2);
                if (a1) { if (p1 < cap) B.cert[off + p1] = e; else atomicOr(B.err, 2u); }
                if (a2) { if (p2 < cap) B.cert[off + cap - 1 - p2] = e; else atomicOr(B.err, 2u); }
            }
        }
#pragma unroll
        for (int j = 0; j < kU; j++) cur[j] = nxt[j];
    }
    __syncthreads();
}

// Offer the certificate stored in node region (off, cap) with counts (n1, n2)
// to the LDS state, staging accepted edges in S.stage.
template <class LS>
__device__ void offer_region(LS& S, const BatchDev& B, int64_t off, int64_t cap, uint32_t n1, uint32_t n2,
                             uint32_t maxv) {
    constexpr int kStage = LS::kStage;
    const int64_t total = (int64_t)n1 + n2;
    for (int64_t base = 0; base < total; base += kBB) {
        const int64_t k = base + threadIdx.x;
        bool a1 = false, a2 = false;
        int2 e = make_int2(0, 0);
        if (k < total) {
            const uint64_t r = __hip_atomic_load(reinterpret_cast<const uint64_t*>(B.cert + (k < n1 ? off + k : off + cap - n2 + (k - n1))),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            e = make_int2((int32_t)(uint32_t)r, (int32_t)(uint32_t)(r >> 32));
            if ((uint32_t)e.x < maxv && (uint32_t)e.y < maxv) loffer(S.q, (uint32_t)e.x, (uint32_t)e.y, a1, a2);
            else atomicOr(B.err, 2u);
        }
        const uint32_t w = (uint32_t)e.x | ((uint32_t)e.y << 16);
        uint32_t p1, p2;
        reserve2(&S.n12, a1, a2, p1, p2);
        if (a1) { if (p1 < kStage) S.stage[p1] = w; else atomicOr(B.err, 2u); }
        if (a2) { if (p2 < kStage) S.stage[kStage - 1 - p2] = w; else atomicOr(B.err, 2u); }
    }
}

__device__ __forceinline__ int2 region_edge(const BatchDev& B, int64_t off, int64_t cap, uint32_t n1, uint32_t n2,
                                            int64_t k) {
    const uint64_t r = __hip_atomic_load(reinterpret_cast<const uint64_t*>(B.cert + (k < n1 ? off + k : off + cap - n2 + (k - n1))),
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int2((int32_t)(uint32_t)r, (int32_t)(uint32_t)(r >> 32));
}

// Node i's state from its certificate in (off, cap): F's edges hooked in F,
// then (after a barrier) F''s in F'.  Each set is a forest, so every edge is
// accepted whatever the order; nothing is written.
template <class LS>
__device__ void rebuild_state(LS& S, const BatchDev& B, int64_t off, int64_t cap, uint32_t n1, uint32_t n2,
                              uint32_t V) {
    for (int64_t k = threadIdx.x; k < n1; k += kBB) {
        const int2 e = region_edge(B, off, cap, n1, n2, k);
        if ((uint32_t)e.x < V && (uint32_t)e.y < V) (void)lunite<0>(S.q, (uint32_t)e.x, (uint32_t)e.y);
        else atomicOr(B.err, 2u);
    }
    __syncthreads();
    for (int64_t k = (int64_t)n1 + threadIdx.x; k < (int64_t)n1 + n2; k += kBB) {
        const int2 e = region_edge(B, off, cap, n1, n2, k);
        if ((uint32_t)e.x < V && (uint32_t)e.y < V) (void)lunite<1>(S.q, (uint32_t)e.x, (uint32_t)e.y);
        else atomicOr(B.err, 2u);
    }
}

// The certificate in (offj, capj) offered to the state; accepted edges are
// appended to region (offi, capi) after the edges S.n12 already counts.
template <class LS>
__device__ void offer_region_append(LS& S, const BatchDev& B, int64_t offj, int64_t capj, uint32_t n1, uint32_t n2,
                                    uint32_t V, int64_t offi, int64_t capi) {
    const int64_t total = (int64_t)n1 + n2;
    for (int64_t base = 0; base < total; base += kBB) {
        const int64_t k = base + threadIdx.x;
        bool a1 = false, a2 = false;
        int2 e = make_int2(0, 0);
        if (k < total) {
            e = region_edge(B, offj, capj, n1, n2, k);
            if ((uint32_t)e.x < V && (uint32_t)e.y < V) loffer(S.q, (uint32_t)e.x, (uint32_t)e.y, a1, a2);
            else atomicOr(B.err, 2u);
        }
        uint32_t p1, p2;
        reserve2(&S.n12, a1, a2, p1, p2);
        if (a1) { if (p1 < capi) B.cert[offi + p1] = e; else atomicOr(B.err, 2u); }
        if (a2) { if (p2 < capi) B.cert[offi + capi - 1 - p2] = e; else atomicOr(B.err, 2u); }
    }
}

}  // namespace

template <int MaxV, bool Staged>
__global__ void __launch_bounds__(kBB) k_batched(BatchDev B) {
    using LS = LdsState<MaxV, Staged>;
    constexpr int kStage = LS::kStage;
    __shared__ LS S;
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
        uint32_t n1 = S.n12 & 0xffffu, n2 = S.n12 >> 16;
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
            if (threadIdx.x == 0) S.n12 = 0;
            __syncthreads();
            const uint32_t ai1 = __hip_atomic_load(&B.ncnt[2 * nidx(i)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ai2 = __hip_atomic_load(&B.ncnt[2 * nidx(i) + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t aj1 = __hip_atomic_load(&B.ncnt[2 * nidx(j)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t aj2 = __hip_atomic_load(&B.ncnt[2 * nidx(j) + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int64_t offi = B.noff[nidx(i)], capi = B.ncap[nidx(i)];
            const int64_t offj = B.noff[nidx(j)], capj = B.ncap[nidx(j)];
            const uint32_t ci1 = min(ai1, (uint32_t)capi), ci2 = min(ai2, (uint32_t)capi - ci1);
            const uint32_t cj1 = min(aj1, (uint32_t)capj), cj2 = min(aj2, (uint32_t)capj - cj1);
            if constexpr (Staged) {
                offer_region(S, B, offi, capi, ci1, ci2, (uint32_t)MaxV);
                offer_region(S, B, offj, capj, cj1, cj2, (uint32_t)MaxV);
                __syncthreads();
                n1 = min(S.n12 & 0xffffu, (uint32_t)kStage);
                n2 = min(S.n12 >> 16, (uint32_t)kStage - n1);
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
            } else {
                rebuild_state(S, B, offi, capi, ci1, ci2, V);
                if (threadIdx.x == 0) S.n12 = ci1 | (ci2 << 16);
                __syncthreads();
                offer_region_append(S, B, offj, capj, cj1, cj2, V, offi, capi);
                __syncthreads();
                n1 = S.n12 & 0xffffu;
                n2 = S.n12 >> 16;
                if ((int64_t)n1 + n2 > capi && threadIdx.x == 0) atomicOr(B.err, 2u);
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
// The node-0 certificates of S graphs as one certificate of their disjoint
// union: offsets of each graph's F and F' edges in the union (one block), then
// the copies with the graph's first vertex added to both endpoints.
constexpr int kUT = 1024;
__global__ void __launch_bounds__(kUT) k_union_offsets(BatchDev B, int32_t S, int64_t* uoff, uint32_t* cntu) {
    __shared__ int64_t p1[kUT], p2[kUT];
    const int64_t per = ((int64_t)S + kUT - 1) / kUT;
    const int64_t s0 = min((int64_t)S, (int64_t)threadIdx.x * per), s1 = min((int64_t)S, s0 + per);
    int64_t a = 0, b = 0;
    for (int64_t s = s0; s < s1; s++) {
        const uint32_t cap = (uint32_t)B.ncap[s];
        const uint32_t n1 = min(B.ncnt[2 * s], cap), n2 = min(B.ncnt[2 * s + 1], cap - n1);
        a += n1;
        b += n2;
    }
    p1[threadIdx.x] = a;
    p2[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t x = 0, y = 0;
        for (int t = 0; t < kUT; t++) {
            const int64_t u = p1[t], v = p2[t];
            p1[t] = x;
            p2[t] = y;
            x += u;
            y += v;
        }
        cntu[0] = (uint32_t)x;
        cntu[1] = (uint32_t)y;
    }
    __syncthreads();
    a = p1[threadIdx.x];
    b = p2[threadIdx.x];
    for (int64_t s = s0; s < s1; s++) {
        uoff[s] = a;
        uoff[S + s] = b;
        const uint32_t cap = (uint32_t)B.ncap[s];
        const uint32_t n1 = min(B.ncnt[2 * s], cap), n2 = min(B.ncnt[2 * s + 1], cap - n1);
        a += n1;
        b += n2;
    }
}

__global__ void k_union_copy(BatchDev B, int32_t S, const int64_t* uoff, int2* f1u, int2* f2u) {
    for (int64_t s = blockIdx.x; s < S; s += gridDim.x) {
        const int64_t off = B.noff[s], cap = B.ncap[s];
        const uint32_t n1 = min(B.ncnt[2 * s], (uint32_t)cap), n2 = min(B.ncnt[2 * s + 1], (uint32_t)cap - n1);
        const int32_t vb = (int32_t)B.vbase[s];
        for (uint32_t k = threadIdx.x; k < n1 + n2; k += blockDim.x) {
            const int2 e = k < n1 ? B.cert[off + k] : B.cert[off + cap - n2 + (k - n1)];
            const int2 g = make_int2(e.x + vb, e.y + vb);
            if (k < n1) f1u[uoff[s] + k] = g;
            else f2u[uoff[S + s] + (k - n1)] = g;
        }
    }
}
}  // namespace

void launch_union_certificate(const BatchDev& B, int32_t S, int64_t* uoff, int2* f1u, int2* f2u, uint32_t* cntu,
                              hipStream_t s) {
    if (S <= 0) return;
    hipLaunchKernelGGL(k_union_offsets, dim3(1), dim3(kUT), 0, s, B, S, uoff, cntu);
    hipLaunchKernelGGL(k_union_copy, dim3((unsigned)std::min<int32_t>(S, 65535)), dim3(256), 0, s, B, S,
                       (const int64_t*)uoff, f1u, f2u);
}

void launch_batched(const BatchDev& B, int blocks, hipStream_t s, bool big) {
    if (big) hipLaunchKernelGGL((k_batched<kMaxVBig, false>), dim3(blocks), dim3(kBB), 0, s, B);
    else hipLaunchKernelGGL((k_batched<kMaxV, true>), dim3(blocks), dim3(kBB), 0, s, B);
}

int32_t batched_max_v_dev() { return kMaxV; }
int32_t batched_max_v_big() { return kMaxVBig; }

namespace {
// Gather of several device edge lists into one packed buffer: item x copies
// items[x].n edges from items[x].src to dst + items[x].at, the blocks of
// column y taking runs y, y + gridDim.y, ... of kGatherRun edges.
constexpr int64_t kGatherRun = 16384;
__global__ void __launch_bounds__(256) k_gather_edges(const GatherItem* items, int2* dst) {
    const GatherItem it = items[blockIdx.x];
    const int2* src = reinterpret_cast<const int2*>(it.src);
    for (int64_t lo = blockIdx.y * kGatherRun; lo < it.n; lo += (int64_t)gridDim.y * kGatherRun) {
        const int64_t hi = min(lo + kGatherRun, it.n);
        for (int64_t k = lo + threadIdx.x; k < hi; k += 256) dst[it.at + k] = src[k];
    }
}
}  // namespace

void launch_gather_edges(const GatherItem* d_items, int32_t n, int64_t max_edges, int32_t* dst, hipStream_t s) {
    if (n <= 0 || max_edges <= 0) return;
    const int64_t runs = std::min<int64_t>((max_edges + kGatherRun - 1) / kGatherRun, 1024);
    hipLaunchKernelGGL(k_gather_edges, dim3((unsigned)n, (unsigned)runs), dim3(256), 0, s, d_items,
                       reinterpret_cast<int2*>(dst));
}
int32_t batched_blocks_per_cu() { return 3; }
// workgroups of the small kernel that fit one CU's LDS together
int32_t batched_max_blocks_per_cu() {
    return std::max<int32_t>(1, (int32_t)((160 * 1024) / sizeof(LdsState<kMaxV, true>)));
}

}  // namespace br
