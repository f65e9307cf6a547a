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
// y's cyclic arc list, each tour cut open at its union-find root; list ranking
// by pointer jumping gives every arc its position in its tour.
//
// Launches: one clear, the arc lists, the ranking (one launch whose threads
// jump asynchronously), tour sizes, downward arcs, one scan, preorder numbers,
// the F' ranges, the range tables (two launches while the block table fits a
// workgroup's LDS), the test -- eleven in all.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_util.hpp"
#include "internal.hpp"

namespace br {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int32_t arc_src(const int2* f1, int32_t a) { const int2 e = f1[a >> 1]; return (a & 1) ? e.y : e.x; }
__device__ __forceinline__ int32_t arc_dst(const int2* f1, int32_t a) { const int2 e = f1[a >> 1]; return (a & 1) ? e.x : e.y; }


constexpr int kSB = kT * 4;   // elements per block of the one-pass scans

// ---- one-pass exclusive scans (decoupled look-back) ----------------------------
//
// Each block takes a ticket (its order of arrival), scans its kSB elements,
// publishes its aggregate, then adds the prefixes published by the blocks
// before it.  A block only waits on blocks with smaller tickets, which are
// already running, so the waits end.  Two 30-bit sums travel in one 64-bit
// status word together with a 2-bit state (0 none, 1 aggregate, 2 inclusive).
constexpr uint64_t kLoMask = (uint64_t(1) << 30) - 1;

__device__ __forceinline__ uint64_t st_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// exclusive scan of one packed value per thread across the block; the block's
// total goes to `total`.  Packed sums never carry between the two halves.
__device__ __forceinline__ uint64_t block_exclusive64(uint64_t v, uint64_t* sh, uint64_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int i = 0; i < kT / 64; i++) { const uint64_t t = sh[i]; sh[i] = s; s += t; }
        sh[kT / 64] = s;
    }
    __syncthreads();
    total = sh[kT / 64];
    const uint64_t r = x - v + sh[w];
    __syncthreads();
    return r;
}

// prefix of everything before this block: thread 0 publishes the aggregate,
// then wavefront 0 inspects 64 predecessors per round trip, summing back to the
// nearest one that already holds its inclusive prefix
__device__ __forceinline__ uint64_t look_back(uint64_t* status, uint32_t ticket, uint64_t total, uint64_t* sh) {
    constexpr uint64_t kVal = ~(uint64_t(3) << 62);
    if (threadIdx.x == 0) st_store(status + ticket, (uint64_t(ticket == 0 ? 2 : 1) << 62) | total);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint64_t prefix = 0;
        for (int64_t j = (int64_t)ticket - 1; j >= 0; j -= 64) {
            const int64_t idx = j - lane;
            uint64_t w = uint64_t(2) << 62;                   // before block 0: inclusive, zero
            if (idx >= 0)
                do { w = st_load(status + idx); } while ((w >> 62) == 0);
            const uint64_t incl = __ballot((w >> 62) == 2);
            const int stop = incl ? __ffsll((unsigned long long)incl) - 1 : 63;
            uint64_t v = lane <= stop ? (w & kVal) : 0;
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
            prefix += v;
            if (incl) break;
        }
        if (lane == 0) {
            if (ticket != 0) st_store(status + ticket, (uint64_t(2) << 62) | (prefix + total));
            sh[kT / 64 + 1] = prefix;
        }
    }
    __syncthreads();
    return sh[kT / 64 + 1];
}

// in-place exclusive scan of a[0..n); status[] and *ticket zeroed beforehand
__global__ void __launch_bounds__(kT) k_scan1(int32_t* a, int64_t n, uint64_t* status, uint32_t* ticket) {
    __shared__ uint64_t sh[kT / 64 + 2];
    __shared__ uint32_t tk;
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t t = tk;
    const int64_t base = (int64_t)t * kSB + threadIdx.x * 4;
    int32_t v[4];
    uint64_t sum = 0;
    for (int j = 0; j < 4; j++) { v[j] = base + j < n ? a[base + j] : 0; sum += (uint32_t)v[j]; }
    uint64_t total;
    uint64_t ex = block_exclusive64(sum, sh, total);
    ex += look_back(status, t, total, sh);
    for (int j = 0; j < 4; j++) { if (base + j < n) a[base + j] = (int32_t)ex; ex += (uint32_t)v[j]; }
}

// ---- arc lists of F -------------------------------------------------------------
//
// first[x] = 1 + an arc leaving x (0: none), nxt[a] = 1 + the arc after a in
// its source's list (0: a is the last).  The order inside a list is whatever
// order the insertions took; the tours only need some cyclic order per vertex,
// and every result derived from them (bridges, cut vertices, class labels) is
// the same for any order.
__global__ void k_zero_i32(int32_t* p, int64_t n) { GRID_LOOP(i, n) p[i] = 0; }

__global__ void k_link(const int2* f1, const uint32_t* cnt, int32_t* first, int32_t* nxt) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) nxt[a] = atomicExch(&first[arc_src(f1, (int32_t)a)], (int32_t)a + 1);
}

// ---- list ranking of the Euler tours -------------------------------------------
//
// One 64-bit word per arc a: (dist << 32) | lo.  lo >= 0: arc lo lies dist
// steps after a.  lo < 0: the tour ends dist steps after a, at arc ~lo.  Zero:
// not written yet (no word written is ever zero).  A word only ever moves
// further along the tour, so a word read while its owner updates it is still
// a true statement, and threads can jump without waiting for each other:
// each replaces its word (a -> n) by (a -> the target of n's word) until its
// tour's end is reached.  Loads and stores are device-scope so that progress
// made on one XCD is seen by the others.
__device__ __forceinline__ uint64_t lk_pack(int32_t lo, uint32_t dist) { return (uint64_t)dist << 32 | (uint32_t)lo; }
__device__ __forceinline__ int32_t lk_lo(uint64_t w) { return (int32_t)(uint32_t)w; }
__device__ __forceinline__ uint32_t lk_dist(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ __forceinline__ uint64_t lk_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lk_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// successor of arc a = (x -> y) in its tour: the arc after (y -> x) in y's
// list, wrapping to y's first; the tour of a root y ends at the arc entering y
// whose reverse is y's last arc
__device__ __forceinline__ uint64_t tour_step(const int2* f1, const int32_t* first, const int32_t* nxt,
                                              const uint32_t* q, int32_t qs, int32_t a) {
    const int32_t b = a ^ 1;
    const int32_t y = arc_src(f1, b);
    const int32_t n = nxt[b];
    if (n == 0 && q[qs * (size_t)y] == 0) return lk_pack(~a, 0);
    return lk_pack((n != 0 ? n : first[y]) - 1, 1);
}

// one jump of word w of arc a; dist >= A only on an inconsistent forest
// (a cycle without a root): the word is then closed at a, A steps on, a
// position no tour has (the later steps skip such arcs)
__device__ __forceinline__ uint64_t tour_jump(const int2* f1, const int32_t* first, const int32_t* nxt,
                                              const uint32_t* q, int32_t qs, const uint64_t* link, int64_t A,
                                              int32_t a, uint64_t w) {
    const int32_t n = lk_lo(w);
    if ((int64_t)n >= A) return lk_pack(~a, (uint32_t)A);
    uint64_t u = lk_load(link + n);
    if (u == 0) u = tour_step(f1, first, nxt, q, qs, n);
    const uint32_t d = lk_dist(w) + lk_dist(u);
    return d >= (uint64_t)A ? lk_pack(~a, (uint32_t)A) : lk_pack(lk_lo(u), d);
}

// K arcs per thread held in registers (arcs t, t + stride, ...).  (Ranking
// inside one XCD, with plain loads through its L2, measured slower: dense
// 0.156 against 0.119 ms for the whole bridge step.)
template <int K>
__global__ void __launch_bounds__(kT) k_rank(const int2* f1, const uint32_t* cnt, const int32_t* first,
                                             const int32_t* nxt, const uint32_t* q, int32_t qs, uint64_t* link) {
    const int64_t A = 2 * (int64_t)cnt[0];
    const int64_t t = blockIdx.x * (int64_t)kT + threadIdx.x, stride = (int64_t)gridDim.x * kT;
    uint64_t w[K];
    uint32_t live = 0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int64_t a = t + k * stride;
        w[k] = 0;
        if (a < A) {
            w[k] = tour_step(f1, first, nxt, q, qs, (int32_t)a);
            lk_store(link + a, w[k]);
            if (lk_lo(w[k]) >= 0) live |= 1u << k;
        }
    }
    while (live) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (!((live >> k) & 1u)) continue;
            w[k] = tour_jump(f1, first, nxt, q, qs, link, A, (int32_t)(t + k * stride), w[k]);
            lk_store(link + t + k * stride, w[k]);
            if (lk_lo(w[k]) < 0) live &= ~(1u << k);
        }
    }
}

// any number of arcs per thread, their words kept in memory (lists longer
// than the resident threads can hold in registers)
__global__ void __launch_bounds__(kT) k_rank_mem(const int2* f1, const uint32_t* cnt, const int32_t* first,
                                                 const int32_t* nxt, const uint32_t* q, int32_t qs, uint64_t* link) {
    const int64_t A = 2 * (int64_t)cnt[0];
    const int64_t t = blockIdx.x * (int64_t)kT + threadIdx.x, stride = (int64_t)gridDim.x * kT;
    for (int64_t a = t; a < A; a += stride) lk_store(link + a, tour_step(f1, first, nxt, q, qs, (int32_t)a));
    for (bool live = true; live;) {
        live = false;
        for (int64_t a = t; a < A; a += stride) {
            uint64_t w = lk_load(link + a);
            if (lk_lo(w) < 0) continue;
            w = tour_jump(f1, first, nxt, q, qs, link, A, (int32_t)a, w);
            lk_store(link + a, w);
            live |= lk_lo(w) >= 0;
        }
    }
}

// per vertex r: the arcs and vertices of its tree if r is a root (else 0),
// and their exclusive prefix sums over r -- one pass, two sums per status word
__global__ void __launch_bounds__(kT) k_tours(const int32_t* first, const uint64_t* link,
                                              const uint32_t* q, int32_t qs, int32_t V, int32_t* tour_len,
                                              int32_t* tree_n, int32_t* tour_base, int32_t* vbase, uint64_t* status,
                                              uint32_t* ticket) {
    __shared__ uint64_t sh[kT / 64 + 2];
    __shared__ uint32_t tk;
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t t = tk;
    const int64_t base = (int64_t)t * kSB + threadIdx.x * 4;
    int32_t L[4], N[4];
    uint64_t sum = 0;
    for (int j = 0; j < 4; j++) {
        const int64_t r = base + j;
        L[j] = 0;
        N[j] = 0;
        if (r < V && q[qs * (size_t)r] == 0 && first[r] != 0) {
            L[j] = (int32_t)lk_dist(link[first[r] - 1]) + 1;
            N[j] = L[j] / 2 + 1;
        }
        sum += (uint64_t)(uint32_t)L[j] | ((uint64_t)(uint32_t)N[j] << 30);
    }
    uint64_t total;
    uint64_t ex = block_exclusive64(sum, sh, total);
    ex += look_back(status, t, total, sh);
    for (int j = 0; j < 4; j++) {
        const int64_t r = base + j;
        if (r < V) {
            tour_len[r] = L[j];
            tree_n[r] = N[j];
            tour_base[r] = (int32_t)(ex & kLoMask);
            vbase[r] = (int32_t)(ex >> 30);
        }
        ex += (uint64_t)(uint32_t)L[j] | ((uint64_t)(uint32_t)N[j] << 30);
    }
}

__device__ __forceinline__ int32_t tour_pos(const int2* f1, const uint64_t* link, const int32_t* tour_len, int32_t a,
                                            int32_t* root) {
    const uint64_t l = link[a];
    const int32_t r = arc_dst(f1, ~lk_lo(l));
    *root = r;
    return tour_len[r] - 1 - (int32_t)lk_dist(l);
}

// downward arcs (first entry into a vertex): parent arc, subtree size and a
// flag at the arc's place in the concatenated tours
__global__ void k_down(const int2* f1, const uint32_t* cnt, const uint64_t* link, const int32_t* tour_len,
                       const int32_t* tour_base, int32_t* flag, int32_t* in_arc, int32_t* sub) {
    const int64_t A = 2 * (int64_t)cnt[0];
    GRID_LOOP(a, A) {
        int32_t r;
        const int32_t p = tour_pos(f1, link, tour_len, (int32_t)a, &r);
        const int32_t L = tour_len[r], pr = L - 1 - (int32_t)lk_dist(link[a ^ 1]);
        if (p < 0 || pr >= L) continue;   // only an inconsistent forest gets here
        if (p < pr) {   // a = (x -> y) enters y for the first time
            const int32_t y = arc_dst(f1, (int32_t)a);
            flag[tour_base[r] + p] = 1;
            in_arc[y] = (int32_t)a;
            sub[y] = (pr - p + 1) / 2;
        }
    }
}

// preorder numbers; the range tables start with every vertex's own number
__global__ void k_preorder(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* first, const int32_t* in_arc,
                           const uint64_t* link, const int32_t* tour_len, const int32_t* tour_base, const int32_t* down_ex,
                           const int32_t* vbase, const int32_t* tree_n, int32_t V, int32_t* pre, int32_t* sub,
                           int32_t* tmin, int32_t* tmax) {
    GRID_LOOP(v, (int64_t)V) {
        int32_t pv = -1;
        if (first[v] != 0) {
            if (q[qs * (size_t)v] == 0) {        // root of its tree
                pv = vbase[v];
                sub[v] = tree_n[v];
            } else {
                int32_t r;
                const int32_t p = tour_pos(f1, link, tour_len, in_arc[v], &r);
                if (p >= 0 && p < tour_len[r]) pv = vbase[r] + 1 + (down_ex[tour_base[r] + p] - down_ex[tour_base[r]]);
            }
            if (pv >= 0 && pv < V) {
                tmin[pv] = pv;
                tmax[pv] = pv;
            }
        }
        pre[v] = pv;
    }
}

// F' edges pull each endpoint's range toward the other endpoint's number
// (both endpoints of an F' edge lie in one tree of F, so both are numbered)
__global__ void k_nontree(const int2* f2, int32_t dir, const uint32_t* cnt, const int32_t* pre, int32_t* tmin,
                          int32_t* tmax) {
    const int64_t n2 = cnt[1];
    GRID_LOOP(k, n2) {
        const int2 e = f2[dir * k];
        const int32_t px = pre[e.x], py = pre[e.y];
        if (px < 0 || py < 0) continue;   // only an inconsistent certificate gets here
        atomicMin(&tmin[px], py);
        atomicMax(&tmax[px], py);
        atomicMin(&tmin[py], px);
        atomicMax(&tmax[py], px);
    }
}

// ---- range minimum / maximum over preorder intervals ---------------------------
//
// Blocks of 64 numbers (one wavefront each).  Inside a block, level j (1..5)
// holds the min/max of the 2^j numbers starting at each position (clipped at
// the block's end), so any range inside one block takes two lookups; a sparse
// table over the blocks' own min/max answers a run of whole blocks; one
// workgroup builds that table in LDS when it is small.
constexpr int kRB = 64;
constexpr int kInLev = 5;              // in-block levels 1..5 (level 6 = the block value)
constexpr int kLdsBlocks = 4096;       // block tables up to this size are built in LDS

__device__ __forceinline__ int floor_log2(uint32_t x) { return 31 - __clz(x); }

__device__ void build_block_table(int32_t* tmn, int32_t* tmx, int64_t nb, int32_t levels, int32_t* smn, int32_t* smx) {
    for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) { smn[i] = tmn[i]; smx[i] = tmx[i]; }
    __syncthreads();
    constexpr int kPer = kLdsBlocks / kT;
    for (int32_t j = 1; j < levels; j++) {
        const int64_t half = int64_t(1) << (j - 1);
        int32_t a[kPer], b[kPer];
        for (int k = 0; k < kPer; k++) {
            const int64_t i = threadIdx.x + (int64_t)k * kT;
            if (i < nb) {
                const int64_t q = i + half < nb ? i + half : nb - 1;
                a[k] = min(smn[i], smn[q]);
                b[k] = max(smx[i], smx[q]);
            }
        }
        __syncthreads();
        for (int k = 0; k < kPer; k++) {
            const int64_t i = threadIdx.x + (int64_t)k * kT;
            if (i < nb) {
                smn[i] = a[k];
                smx[i] = b[k];
                tmn[j * nb + i] = a[k];
                tmx[j * nb + i] = b[k];
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void rmq_block_levels(const int32_t* tmin, const int32_t* tmax, int64_t n, int32_t* lmin,
                                                 int32_t* lmax, int32_t* tmn, int32_t* tmx, int64_t nb) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int32_t a = i < n ? tmin[i] : INT32_MAX, b = i < n ? tmax[i] : INT32_MIN;
    for (int j = 1; j <= kInLev + 1; j++) {
        const int o = 1 << (j - 1);
        const int32_t da = __shfl_down(a, o), db = __shfl_down(b, o);
        if (lane + o < 64) { a = min(a, da); b = max(b, db); }
        if (j <= kInLev) {
            if (i < n) { lmin[(int64_t)(j - 1) * n + i] = a; lmax[(int64_t)(j - 1) * n + i] = b; }
        } else if (lane == 0 && (i >> 6) < nb) {
            tmn[i >> 6] = a;
            tmx[i >> 6] = b;
        }
    }
}

// per block: in-block levels and the block's min/max (level 0 of the block table)
__global__ void __launch_bounds__(kT) k_rmq_blocks(const int32_t* tmin, const int32_t* tmax, int64_t n, int32_t* lmin,
                                                   int32_t* lmax, int32_t* tmn, int32_t* tmx, int64_t nb) {
    rmq_block_levels(tmin, tmax, n, lmin, lmax, tmn, tmx, nb);
}

// the block table in one workgroup, in LDS (nb <= kLdsBlocks).  A separate
// launch: folded into k_rmq_blocks as "the last workgroup builds it", every
// workgroup's device-scope release (an L2 write-back) cost more than the
// launch (dense: 30 us against 5 + 10 us)
__global__ void __launch_bounds__(kT) k_rmq_table(int32_t* tmn, int32_t* tmx, int64_t nb, int32_t levels) {
    __shared__ int32_t smn[kLdsBlocks], smx[kLdsBlocks];
    build_block_table(tmn, tmx, nb, levels, smn, smx);
}

// sparse table level j (j >= 1) over nb block values, levels stored nb apart
__global__ void k_rmq_level(int32_t* tmn, int32_t* tmx, int64_t nb, int32_t j) {
    const int64_t half = int64_t(1) << (j - 1);
    int32_t *pmn = tmn + (j - 1) * nb, *pmx = tmx + (j - 1) * nb, *cmn = tmn + j * nb, *cmx = tmx + j * nb;
    GRID_LOOP(i, nb) {
        const int64_t k = i + half < nb ? i + half : nb - 1;
        cmn[i] = min(pmn[i], pmn[k]);
        cmx[i] = max(pmx[i], pmx[k]);
    }
}

struct Rmq {
    const int32_t *t, *u, *lmin, *lmax, *tmn, *tmx;
    int64_t n, nb;
};

// min/max over [a, b] inside one block
__device__ __forceinline__ void in_block(const Rmq& R, int32_t a, int32_t b, int32_t& mn, int32_t& mx) {
    const int j = floor_log2((uint32_t)(b - a + 1));
    if (j == 0) {
        mn = R.t[a];
        mx = R.u[a];
    } else if (j <= kInLev) {
        const int64_t o = (int64_t)(j - 1) * R.n;
        const int32_t c = b - (1 << j) + 1;
        mn = min(R.lmin[o + a], R.lmin[o + c]);
        mx = max(R.lmax[o + a], R.lmax[o + c]);
    } else {   // the whole block
        mn = R.tmn[a >> 6];
        mx = R.tmx[a >> 6];
    }
}

__device__ __forceinline__ void range_minmax(const Rmq& R, int32_t l, int32_t r, int32_t& mn, int32_t& mx) {
    const int32_t bl = l >> 6, br = r >> 6;
    if (bl == br) {
        in_block(R, l, r, mn, mx);
        return;
    }
    int32_t m2, x2;
    in_block(R, l, bl * 64 + 63, mn, mx);
    in_block(R, br * 64, r, m2, x2);
    mn = min(mn, m2);
    mx = max(mx, x2);
    if (br - bl > 1) {
        const int32_t a = bl + 1, b = br - 1;
        const int j = floor_log2((uint32_t)(b - a + 1));
        const int64_t lev = (int64_t)j * R.nb;
        mn = min(mn, min(R.tmn[lev + a], R.tmn[lev + b - (1 << j) + 1]));
        mx = max(mx, max(R.tmx[lev + a], R.tmx[lev + b - (1 << j) + 1]));
    }
}

// Result keys leave a block through LDS with one reservation on *nout per
// block: returning atomics to one address are serialised at the memory side
// (about 12 ns each on MI355X, measured), so one per wavefront would cost more
// than the test itself.  A block whose LDS run is full reserves per wavefront
// for the rest.  Launched with at most kOutBlocks blocks.
constexpr int kOutBuf = 2048;
constexpr int kOutBlocks = 1024;

struct OutLds {
    uint64_t buf[kOutBuf];
    uint32_t n, fail, base;
};

__device__ __forceinline__ void out_begin(OutLds& L) {
    if (threadIdx.x == 0) {
        L.n = 0;
        L.fail = kOutBuf;
    }
    __syncthreads();
}

// the active lanes of a wavefront; m = ballot(add) != 0
__device__ __forceinline__ void out_put(OutLds& L, bool add, uint64_t key, uint64_t m, uint64_t* out, uint32_t* nout) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const uint32_t cnt = (uint32_t)__popcll(m);
    const uint32_t rank = lane_rank(m);
    uint32_t at = 0;
    if (__lane_id() == leader) at = atomicAdd(&L.n, cnt);
    at = __shfl(at, leader);
    if (at + cnt <= (uint32_t)kOutBuf) {
        if (add) L.buf[at + rank] = key;
    } else {
        uint32_t g = 0;
        if (__lane_id() == leader) {
            atomicMin(&L.fail, at);
            g = atomicAdd(nout, cnt);
        }
        g = __shfl(g, leader);
        if (add) out[g + rank] = key;
    }
}

// every thread of the block: entries [0, min(n, fail)) are all written
__device__ __forceinline__ void out_end(OutLds& L, uint64_t* out, uint32_t* nout) {
    __syncthreads();
    const uint32_t stored = min(L.n, L.fail);
    if (threadIdx.x == 0 && stored) L.base = atomicAdd(nout, stored);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < stored; i += blockDim.x) out[L.base + i] = L.buf[i];
}

// st (if not null): the status block, whose |F|, |F'| and error words are
// filled here (the key count, st[1] = *nout, by the keys' reservations)
__global__ void k_bridges(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* first, const int32_t* in_arc,
                          const int32_t* pre, const int32_t* sub, Rmq R, int32_t V, int64_t A, uint64_t* out,
                          uint32_t* nout, const uint32_t* cnt, const uint32_t* err, uint32_t* st) {
    __shared__ OutLds L;
    if (st && blockIdx.x == 0 && threadIdx.x == 0) {
        st[2] = cnt[0];
        st[3] = cnt[1];
        st[4] = err ? *err : 0u;
    }
    out_begin(L);
    GRID_LOOP(v, (int64_t)V) {
        bool br = false;
        uint64_t key = 0;
        if (first[v] != 0 && q[qs * (size_t)v] != 0) {
            const int32_t l = pre[v], r = pre[v] + sub[v] - 1, a = in_arc[v];
            int32_t mn = -1, mx = V;
            if (l >= 0 && r >= l && r < V && a >= 0 && a < A) range_minmax(R, l, r, mn, mx);
            if (mn >= l && mx <= r) {
                br = true;
                const int2 e = f1[a >> 1];
                const uint32_t a = (uint32_t)min(e.x, e.y), b = (uint32_t)max(e.x, e.y);
                key = (uint64_t)a << 32 | b;
            }
        }
        const uint64_t m = __ballot(br);
        if (m) out_put(L, br, key, m, out, nout);
    }
    out_end(L, out, nout);
}

// ---- articulation points of the certificate ------------------------------------
//
// The test of Tarjan and Vishkin on the rooted spanning tree F (any spanning
// tree will do, breadth-first included).  Tree edges are named by their child
// c and grouped by a union-find: an edge of F' between two unrelated vertices
// (neither in the other's subtree) joins their parent edges, and the parent
// edge of c joins that of its parent p (p not a root) when c's subtree reaches
// a vertex outside p's subtree.  The groups are the blocks; a vertex is an
// articulation point iff the edges to its children do not all lie in the block
// of its own parent edge -- for a root, iff they lie in at least two blocks.
__device__ __forceinline__ uint32_t tv_find(uint32_t* g, uint32_t x) {
    uint32_t d = g[x];
    while (d != 0) {
        const uint32_t p = x - d, dp = g[p];
        if (dp == 0) return p;
        g[x] = d + dp;
        x = p - dp;
        d = g[x];
    }
    return x;
}

__device__ __forceinline__ void tv_unite(uint32_t* g, uint32_t a, uint32_t b) {
    for (;;) {
        a = tv_find(g, a);
        b = tv_find(g, b);
        if (a == b) return;
        if (a < b) { const uint32_t t = a; a = b; b = t; }
        uint32_t expect = 0;
        if (__hip_atomic_compare_exchange_strong(g + a, &expect, a - b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a -= expect;
    }
}

__global__ void k_tv_init(int32_t V, uint32_t* g, int32_t* rmin, int32_t* rmax, int32_t* apf) {
    GRID_LOOP(v, (int64_t)V) {
        g[v] = 0;
        rmin[v] = INT32_MAX;
        rmax[v] = -1;
        apf[v] = 0;
    }
}

// tree edge (w, v), w not a root: joins (parent(w), w) when v's subtree escapes w's
__global__ void k_tv_tree(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* first, const int32_t* in_arc,
                          const int32_t* pre, const int32_t* sub, Rmq R, int32_t V, int64_t A, uint32_t* g) {
    GRID_LOOP(v, (int64_t)V) {
        if (first[v] == 0 || q[qs * (size_t)v] == 0) continue;
        const int32_t a = in_arc[v];
        if (a < 0 || a >= A) continue;
        const int32_t w = arc_src(f1, a);
        if (q[qs * (size_t)w] == 0) continue;
        const int32_t l = pre[v], r = pre[v] + sub[v] - 1, pw = pre[w];
        if (l < 0 || r < l || r >= V || pw < 0) continue;
        int32_t mn, mx;
        range_minmax(R, l, r, mn, mx);
        if (mn < pw || mx >= pw + sub[w]) tv_unite(g, (uint32_t)v, (uint32_t)w);
    }
}

// edge of F' between unrelated vertices: joins their parent edges
__global__ void k_tv_cross(const int2* f2, int32_t dir, const uint32_t* cnt, const int32_t* pre, const int32_t* sub,
                           uint32_t* g) {
    const int64_t n2 = cnt[1];
    GRID_LOOP(k, n2) {
        const int2 e = f2[dir * k];
        const int32_t px = pre[e.x], py = pre[e.y];
        if (px < 0 || py < 0 || e.x == e.y) continue;
        const bool related = (px <= py && py < px + sub[e.x]) || (py <= px && px < py + sub[e.y]);
        if (!related) tv_unite(g, (uint32_t)e.x, (uint32_t)e.y);
    }
}

__global__ void k_tv_compress(uint32_t* g, int32_t V) {
    GRID_LOOP(x, (int64_t)V) {
        const uint32_t d = g[x];
        if (d == 0) continue;
        uint32_t r = (uint32_t)x - d;
        for (uint32_t e = g[r]; e != 0; e = g[r]) r -= e;
        g[x] = (uint32_t)x - r;
    }
}

// per tree edge (w, v): compare v's block with the block of w's own parent edge
__global__ void k_tv_mark(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* first, const int32_t* in_arc,
                          int32_t V, int64_t A, const uint32_t* g, int32_t* rmin, int32_t* rmax, int32_t* apf) {
    GRID_LOOP(v, (int64_t)V) {
        if (first[v] == 0 || q[qs * (size_t)v] == 0) continue;
        const int32_t a = in_arc[v];
        if (a < 0 || a >= A) continue;
        const int32_t w = arc_src(f1, a);
        const int32_t cv = (int32_t)((uint32_t)v - g[v]);
        if (q[qs * (size_t)w] == 0) {
            atomicMin(&rmin[w], cv);
            atomicMax(&rmax[w], cv);
        } else if (cv != (int32_t)((uint32_t)w - g[w])) {
            apf[w] = 1;
        }
    }
}

__global__ void k_tv_list(const uint32_t* q, int32_t qs, const int32_t* first, int32_t V, const int32_t* rmin,
                          const int32_t* rmax, const int32_t* apf, uint64_t* out, uint32_t* nout) {
    __shared__ OutLds L;
    out_begin(L);
    GRID_LOOP(v, (int64_t)V) {
        bool cut = false;
        if (first[v] != 0)
            cut = q[qs * (size_t)v] == 0 ? (rmax[v] >= 0 && rmin[v] != rmax[v]) : apf[v] != 0;
        const uint64_t m = __ballot(cut);
        if (m) out_put(L, cut, (uint64_t)v, m, out, nout);
    }
    out_end(L, out, nout);
}

// ---- 2-edge-connected classes of the certificate ----------------------------
//
// The classes are the components left once the bridges are removed.  Every
// edge of F' is a non-tree edge, so never a bridge; a tree edge (parent(v), v)
// is a bridge iff no edge of F' leaves v's subtree (the test of k_bridges).
// The non-bridges are united with the larger root hooked under the smaller, so
// after full compression each vertex's root is the smallest id of its class.
__global__ void k_class_tree(const int2* f1, const uint32_t* q, int32_t qs, const int32_t* first, const int32_t* in_arc,
                             const int32_t* pre, const int32_t* sub, Rmq R, int32_t V, int64_t A, uint32_t* g) {
    GRID_LOOP(v, (int64_t)V) {
        if (first[v] == 0 || q[qs * (size_t)v] == 0) continue;      // no tree edge above v
        const int32_t a = in_arc[v];
        if (a < 0 || a >= A) continue;
        const int32_t l = pre[v], r = pre[v] + sub[v] - 1;
        if (l < 0 || r < l || r >= V) continue;
        int32_t mn, mx;
        range_minmax(R, l, r, mn, mx);
        if (mn >= l && mx <= r) continue;                                  // a bridge
        tv_unite(g, (uint32_t)v, (uint32_t)arc_src(f1, a));
    }
}

__global__ void k_class_cross(const int2* f2, int32_t dir, const uint32_t* cnt, uint32_t* g) {
    const int64_t n2 = cnt[1];
    GRID_LOOP(k, n2) {
        const int2 e = f2[dir * k];
        if (e.x != e.y) tv_unite(g, (uint32_t)e.x, (uint32_t)e.y);
    }
}

// labels (after full compression) and the number of classes (roots), one
// reservation per block
__global__ void k_class_out(const uint32_t* g, int32_t V, int32_t* label, uint32_t* nclass) {
    __shared__ uint32_t roots;
    if (threadIdx.x == 0) roots = 0;
    __syncthreads();
    GRID_LOOP(v, (int64_t)V) {
        const uint32_t r = (uint32_t)v - g[v];
        label[v] = (int32_t)r;
        if (r == (uint32_t)v) atomicAdd(&roots, 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0 && roots) atomicAdd(nclass, roots);
}

// Edges of the bridge tree: a tree edge (u, v) of F joins two classes iff it
// is a bridge (an edge of F inside a class lies on a cycle; every bridge lies
// in every spanning forest), and then it becomes the tree edge between the
// two classes' labels, as the key min << 32 | max.  Keys staged in LDS, one
// reservation per block on *ntree.
__global__ void k_tree_keys(const int2* f1, const uint32_t* cnt, const int32_t* label, uint64_t* keys, uint32_t* ntree) {
    __shared__ uint64_t stage[kT];
    __shared__ uint32_t n, base;
    const int64_t m = cnt[0];
    for (int64_t b0 = blockIdx.x * (int64_t)kT; b0 < m; b0 += (int64_t)gridDim.x * kT) {
        if (threadIdx.x == 0) n = 0;
        __syncthreads();
        const int64_t k = b0 + threadIdx.x;
        if (k < m) {
            const int2 e = f1[k];
            const uint32_t a = (uint32_t)label[e.x], c = (uint32_t)label[e.y];
            if (a != c) stage[atomicAdd(&n, 1u)] = (uint64_t)min(a, c) << 32 | max(a, c);
        }
        __syncthreads();
        if (threadIdx.x == 0) base = n ? atomicAdd(ntree, n) : 0u;
        __syncthreads();
        if (threadIdx.x < n) keys[base + threadIdx.x] = stage[threadIdx.x];
        __syncthreads();
    }
}

// counters of the certificate and the result next to the keys, for one copy
__global__ void k_status(const uint32_t* cnt, const uint32_t* err, uint32_t* misc) {
    if (threadIdx.x == 0) {
        misc[2] = cnt[0];
        misc[3] = cnt[1];
        misc[4] = err ? *err : 0u;
    }
}


}  // namespace

// Scratch layout of the bridge step, shared by the size query and the launch
// sequence so that the two cannot disagree.  Everything from `first` up to the
// end of `misc` is cleared by one kernel at the start (the ranking words
// included: zero marks a word not written yet); the keys follow `misc`
// directly, so that the counters and the keys leave in one copy.
struct BridgeWs {
    int32_t *first, *cur, *flag, *tickets, *misc, *nxt, *posof, *tour_len, *tree_n, *tour_base, *vbase, *in_arc, *sub,
        *pre, *tmin, *tmax, *lmin, *lmax, *tmn, *tmx;
    uint64_t *st_tours, *st_flag, *keys, *link;
    int64_t zero_words, nb;
    int32_t levels;
    int64_t words;
};

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static BridgeWs carve(int32_t* base, int32_t V) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    BridgeWs w{};
    int64_t o = 0;
    auto take = [&](int64_t n) { int32_t* p = base ? base + o : nullptr; o += (n + 63) & ~int64_t(63); return p; };
    w.first = take(V + 2);
    w.flag = take(A + 1);
    w.tickets = take(64);   // [1] tour scan ticket, [2] flag scan ticket
    w.st_tours = reinterpret_cast<uint64_t*>(take(2 * cdiv(V, kSB)));
    w.st_flag = reinterpret_cast<uint64_t*>(take(2 * cdiv(A + 1, kSB)));
    w.in_arc = take(V);
    w.sub = take(V);
    w.link = reinterpret_cast<uint64_t*>(take(2 * A));
    w.misc = take(64);   // [1] key count, [2..4] |F|, |F'|, error word
    w.zero_words = o;
    w.keys = reinterpret_cast<uint64_t*>(take(2 * (int64_t)V + 2));
    w.cur = take(V + 1);
    w.nxt = take(A);
    w.posof = take(A);
    w.tour_len = take(V);
    w.tree_n = take(V);
    w.tour_base = take(V);
    w.vbase = take(V);
    w.pre = take(V);
    w.tmin = take(V);
    w.tmax = take(V);
    w.lmin = take((int64_t)kInLev * V);
    w.lmax = take((int64_t)kInLev * V);
    w.nb = cdiv(V, kRB);
    w.levels = 1;
    while ((int64_t(1) << w.levels) <= w.nb) w.levels++;
    w.tmn = take(w.levels * w.nb);
    w.tmx = take(w.levels * w.nb);
    w.words = o;
    return w;
}

int64_t device_bridges_words(int32_t V) { return carve(nullptr, V).words; }

void device_scan1(int32_t* a, int64_t n, uint64_t* status, uint32_t* ticket, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scan1, dim3((unsigned)cdiv(n, kSB)), dim3(kT), 0, s, a, n, status, ticket);
}

// Bridges of a certificate held on the device: F = f1[0..cnt[0]), F' =
// f2[dir*k] for k < cnt[1] (counts read on the device), vertex v is the root of
// its tree of F iff q[qs*v] == 0.  Writes up to V keys at *d_keys and their
// number at *d_n; *d_n sits 4 bytes into a 256-byte status block that the keys
// follow directly.
// The part shared by the bridge and articulation-point tests: adjacency of F,
// Euler tours ranked, preorder numbers, subtree sizes, min/max preorder numbers
// reached through F' and their range tables.
// The ranking launch: K arcs per thread in registers while the grid stays
// within what the device holds resident at once, else the words in memory.
static void launch_rank(const int2* f1, const uint32_t* cnt, const int32_t* first, const int32_t* nxt,
                        const uint32_t* q, int32_t qs, uint64_t* link, int64_t A, hipStream_t s) {
    static int resident = 0;      // workgroups of k_rank resident on the device
    static std::once_flag once;
    std::call_once(once, [] {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rank<1>, kT, 0) != hipSuccess || per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        resident = std::max(1, per_cu) * std::max(1, g_cus);
    });
    const int64_t cap = (int64_t)resident * kT;   // threads
    if (A <= cap)
        hipLaunchKernelGGL(k_rank<1>, dim3((unsigned)cdiv(A, kT)), dim3(kT), 0, s, f1, cnt, first, nxt, q, qs, link);
    else if (A <= 2 * cap)
        hipLaunchKernelGGL(k_rank<2>, dim3((unsigned)cdiv(A, 2 * kT)), dim3(kT), 0, s, f1, cnt, first, nxt, q, qs, link);
    else if (A <= 4 * cap)
        hipLaunchKernelGGL(k_rank<4>, dim3((unsigned)cdiv(A, 4 * kT)), dim3(kT), 0, s, f1, cnt, first, nxt, q, qs, link);
    else
        hipLaunchKernelGGL(k_rank_mem, dim3((unsigned)resident), dim3(kT), 0, s, f1, cnt, first, nxt, q, qs, link);
}

static BridgeWs number_tree(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q,
                            int32_t qs, int32_t V, int32_t* ws, hipStream_t s, Rmq* R) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    const BridgeWs W = carve(ws, V);
    hipLaunchKernelGGL(k_zero_i32, dim3(grid_for(W.zero_words)), dim3(kT), 0, s, W.first, W.zero_words);
    hipLaunchKernelGGL(k_link, dim3(grid_for(A)), dim3(kT), 0, s, f1, cnt, W.first, W.nxt);
    launch_rank(f1, cnt, W.first, W.nxt, q, qs, W.link, A, s);
    hipLaunchKernelGGL(k_tours, dim3((unsigned)cdiv(V, kSB)), dim3(kT), 0, s, W.first, (const uint64_t*)W.link, q, qs, V,
                       W.tour_len, W.tree_n, W.tour_base, W.vbase, W.st_tours, reinterpret_cast<uint32_t*>(W.tickets) + 1);
    hipLaunchKernelGGL(k_down, dim3(grid_for(A)), dim3(kT), 0, s, f1, cnt, (const uint64_t*)W.link, W.tour_len,
                       W.tour_base, W.flag, W.in_arc, W.sub);
    hipLaunchKernelGGL(k_scan1, dim3((unsigned)cdiv(A + 1, kSB)), dim3(kT), 0, s, W.flag, A + 1, W.st_flag,
                       reinterpret_cast<uint32_t*>(W.tickets) + 2);
    hipLaunchKernelGGL(k_preorder, dim3(grid_for(V)), dim3(kT), 0, s, f1, q, qs, W.first, W.in_arc,
                       (const uint64_t*)W.link, W.tour_len, W.tour_base, W.flag, W.vbase, W.tree_n, V, W.pre, W.sub,
                       W.tmin, W.tmax);
    hipLaunchKernelGGL(k_nontree, dim3(grid_for(V)), dim3(kT), 0, s, f2, dir, cnt, W.pre, W.tmin, W.tmax);
    const int64_t rblocks = cdiv(W.nb * kRB, kT);
    hipLaunchKernelGGL(k_rmq_blocks, dim3((unsigned)rblocks), dim3(kT), 0, s, W.tmin, W.tmax, (int64_t)V, W.lmin,
                       W.lmax, W.tmn, W.tmx, W.nb);
    if (W.nb <= kLdsBlocks) {
        hipLaunchKernelGGL(k_rmq_table, dim3(1), dim3(kT), 0, s, W.tmn, W.tmx, W.nb, W.levels);
    } else {
        for (int32_t j = 1; j < W.levels; j++)
            hipLaunchKernelGGL(k_rmq_level, dim3(grid_for(W.nb)), dim3(kT), 0, s, W.tmn, W.tmx, W.nb, j);
    }
    *R = Rmq{W.tmin, W.tmax, W.lmin, W.lmax, W.tmn, W.tmx, (int64_t)V, W.nb};
    return W;
}

int device_bridges_cert(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q, int32_t qs,
                        int32_t V, const uint32_t* err, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    Rmq R;
    const BridgeWs W = number_tree(f1, f2, dir, cnt, q, qs, V, ws, s, &R);
    hipLaunchKernelGGL(k_bridges, dim3(std::min(grid_for(V), kOutBlocks)), dim3(kT), 0, s, f1, q, qs, W.first,
                       W.in_arc, W.pre, W.sub, R, V, A, W.keys, reinterpret_cast<uint32_t*>(W.misc + 1), cnt, err,
                       reinterpret_cast<uint32_t*>(W.misc));
    *d_keys = W.keys;
    *d_n = reinterpret_cast<uint32_t*>(W.misc + 1);
    return BR_OK;
}

// Articulation points of a certificate held on the device (same arguments as
// device_bridges_cert); F must be the spanning forest of the certificate.
// Writes the vertex ids (as 64-bit keys, unordered) at *d_keys and their number
// at *d_n, in the same status-block layout.  Scratch reused from the numbering:
// cur (blocks), tour_len / tree_n (roots' min / max child block), posof (flags).
int device_articulation_cert(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q,
                             int32_t qs, int32_t V, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    Rmq R;
    const BridgeWs W = number_tree(f1, f2, dir, cnt, q, qs, V, ws, s, &R);
    uint32_t* g = reinterpret_cast<uint32_t*>(W.cur);
    hipLaunchKernelGGL(k_tv_init, dim3(grid_for(V)), dim3(kT), 0, s, V, g, W.tour_len, W.tree_n, W.posof);
    hipLaunchKernelGGL(k_tv_tree, dim3(grid_for(V)), dim3(kT), 0, s, f1, q, qs, W.first, W.in_arc, W.pre, W.sub, R, V, A, g);
    hipLaunchKernelGGL(k_tv_cross, dim3(grid_for(V)), dim3(kT), 0, s, f2, dir, cnt, W.pre, W.sub, g);
    hipLaunchKernelGGL(k_tv_compress, dim3(grid_for(V)), dim3(kT), 0, s, g, V);
    hipLaunchKernelGGL(k_tv_mark, dim3(grid_for(V)), dim3(kT), 0, s, f1, q, qs, W.first, W.in_arc, V, A, (const uint32_t*)g,
                       W.tour_len, W.tree_n, W.posof);
    hipLaunchKernelGGL(k_tv_list, dim3(std::min(grid_for(V), kOutBlocks)), dim3(kT), 0, s, q, qs, W.first, V, W.tour_len, W.tree_n, W.posof,
                       W.keys, reinterpret_cast<uint32_t*>(W.misc + 1));
    *d_keys = W.keys;
    *d_n = reinterpret_cast<uint32_t*>(W.misc + 1);
    return BR_OK;
}

// 2-edge-connected classes of a certificate held on the device (same
// arguments as device_bridges_cert): int32 labels (smallest id of each class)
// at *d_label, the number of classes at *d_n, in the same status-block layout
// (the labels take the place of the keys).
int device_classes_cert(const int2* f1, const int2* f2, int32_t dir, const uint32_t* cnt, const uint32_t* q,
                        int32_t qs, int32_t V, int32_t* ws, int32_t** d_label, uint32_t** d_n, hipStream_t s) {
    const int64_t A = 2 * (int64_t)std::max(V - 1, 1);
    Rmq R;
    const BridgeWs W = number_tree(f1, f2, dir, cnt, q, qs, V, ws, s, &R);
    uint32_t* g = reinterpret_cast<uint32_t*>(W.cur);
    int32_t* label = reinterpret_cast<int32_t*>(W.keys);
    hipLaunchKernelGGL(k_tv_init, dim3(grid_for(V)), dim3(kT), 0, s, V, g, W.tour_len, W.tree_n, W.posof);
    hipLaunchKernelGGL(k_class_tree, dim3(grid_for(V)), dim3(kT), 0, s, f1, q, qs, W.first, W.in_arc, W.pre, W.sub, R, V, A,
                       g);
    hipLaunchKernelGGL(k_class_cross, dim3(grid_for(V)), dim3(kT), 0, s, f2, dir, cnt, g);
    hipLaunchKernelGGL(k_tv_compress, dim3(grid_for(V)), dim3(kT), 0, s, g, V);
    hipLaunchKernelGGL(k_class_out, dim3(std::min(grid_for(V), kOutBlocks)), dim3(kT), 0, s, (const uint32_t*)g, V, label,
                       reinterpret_cast<uint32_t*>(W.misc + 1));
    *d_label = label;
    *d_n = reinterpret_cast<uint32_t*>(W.misc + 1);
    return BR_OK;
}

// The bridge tree of node 0's certificate: labels and class count as
// device_classes; the tree's edges (keys min << 32 | max of the two classes,
// unordered) at *d_tkeys, their number at (*d_n)[4] (status word 5).
int device_bridge_tree(const Plan& P, const DevBufs& B, int32_t* ws, int32_t** d_label, uint32_t** d_n,
                       uint64_t** d_tkeys, hipStream_t s) {
    const int2* f1 = B.cert + P.off[0];
    const int2* f2 = B.cert + P.off[0] + P.cap[0] - 1;
    int rc = device_classes_cert(f1, f2, -1, B.cnt, B.state, (int32_t)B.qs, P.V, ws, d_label, d_n, s);
    if (rc) return rc;
    // the list-ranking links are free once the tree is numbered: room for V - 1 keys
    const BridgeWs W = carve(ws, P.V);
    uint64_t* tkeys = reinterpret_cast<uint64_t*>(W.link);
    const int64_t m = std::max<int64_t>(P.cap[0], 1);
    hipLaunchKernelGGL(k_tree_keys, dim3((unsigned)std::min<int64_t>((m + kT - 1) / kT, kOutBlocks)), dim3(kT), 0, s, f1,
                       B.cnt, (const int32_t*)*d_label, tkeys, *d_n + 4);
    launch_bridge_status(B.cnt, B.err, *d_n, s);
    *d_tkeys = tkeys;
    return BR_OK;
}

// Classes of node 0's certificate of the plain path, with the status words.
int device_classes(const Plan& P, const DevBufs& B, int32_t* ws, int32_t** d_label, uint32_t** d_n, hipStream_t s) {
    const int2* f1 = B.cert + P.off[0];
    const int2* f2 = B.cert + P.off[0] + P.cap[0] - 1;
    const int rc = device_classes_cert(f1, f2, -1, B.cnt, B.state, (int32_t)B.qs, P.V, ws, d_label, d_n, s);
    if (rc) return rc;
    launch_bridge_status(B.cnt, B.err, *d_n, s);
    return BR_OK;
}

// Bridges of node 0's certificate of the plain path (F' stored backwards from
// the end of the region; roots read from node 0's carried union-find state).
int device_bridges(const Plan& P, const DevBufs& B, int32_t* ws, uint64_t** d_keys, uint32_t** d_n, hipStream_t s) {
    const int2* f1 = B.cert + P.off[0];
    const int2* f2 = B.cert + P.off[0] + P.cap[0] - 1;
    return device_bridges_cert(f1, f2, -1, B.cnt, B.state, (int32_t)B.qs, P.V, B.err, ws, d_keys, d_n, s);
}

// |F|, |F'| and the error word into the status block that holds the key count
void launch_bridge_status(const uint32_t* cnt, const uint32_t* err, uint32_t* d_n, hipStream_t s) {
    hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, s, cnt, err, d_n - 1);
}

}  // namespace br
