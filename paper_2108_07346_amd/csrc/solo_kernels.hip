// The phase tree with one workgroup per node (paper, Section III; Algorithm 2
// per chunk and per merge), for plans with at least as many chunks as
// workgroups in flight.
//
// A persistent kernel: every workgroup ("worker") takes chunks in order from a
// queue, builds the chunk's certificate alone (phase 0), then climbs the merge
// tree while it is the second of a pair to finish (an arrival counter per
// merge): it streams the sibling's certificate into the left node's
// union-find state (the state-carrying merge), up to level `top`; there it
// writes the node's fully compressed state into a dense array for the merge
// rounds above, which run as team launches (cert_kernels.hip).
//
// Union-find state in resident slots.  A slot holds, for each vertex, one
// 32-bit word per forest (F in the first V words, F' in the next V):
// tag << ob | (x - parent), with ob = bit width of V - 1.  A word whose tag is
// not the slot's current tag reads as a root, so a slot is reset for a new
// chunk by taking the next tag (the slot is cleared only when its tags run
// out).  Parents always have smaller ids than their children.
//
// Hooks without global atomics.  Only the owning workgroup touches a slot
// while it works on it, so two lanes can race only within the workgroup, and
// only within one round: the lanes offer their edges, then meet at a barrier
// after which every parent word the workgroup stored is visible to all of
// them.  A hook first claims the root in a claim table in LDS (one table per
// forest, a bit per root hashed by its low bits, emptied at every barrier by
// the lanes that set its bits),
// and only the lane whose claim sets the bit writes the root's parent word,
// with a plain store.  A root hooked in an earlier round is no root to any
// finds of this round (its word is visible); two lanes that reach the same
// root in this round meet at its bit; a lane whose claim finds the bit set
// (that root, or another that shares its bit) retries the edge after the
// barrier.  Lanes read parent words with plain loads: a value, however stale,
// names a vertex of the same component with a smaller id, so finds that meet
// prove the endpoints connected; and the root a winning lane hooks is a root
// of a component other than the one of the vertex it hooks it under (that
// vertex has the smaller id, and chains only decrease).  So F is a maximal
// forest of the edges offered to it and F' of the edges F rejected, as
// Algorithm 2 requires.  The tables are a few KB, so several workers share a
// CU whatever V is.
//
// Slots change hands between workers only through the free pool and the
// parking table; whoever gives a slot away first makes its writes visible
// device-wide (release fence), whoever takes one first invalidates what its
// caches may hold (acquire fence).

#include <hip/hip_runtime.h>

#include <mutex>

#include "device_util.hpp"
#include "internal.hpp"

namespace br {

namespace {

// a worker is SB threads; each thread offers SU edges of a tile together

struct SoloLds {
    uint32_t flag[2];               // block_any
    uint32_t n1, n2;                // counts of the node being written
    int32_t item, slot, act, adopted;   // adopted: the merge continues in another worker's slot
    uint32_t tag, nj1, nj2, groot;      // groot: the F root most sampled vertices reach (before a merge)
    uint32_t nr, nr_snap;           // phase 0: edges waiting for a retry at the front of the worker's copy
};

// kernel parameters
struct SoloArgs {
    const int2* edges;
    const int2* edges2;
    int64_t split;
    int64_t E;
    int32_t V, M;
    int32_t ob;                     // bits of the offset field of a state word
    int32_t top;                    // merges of levels 1..top run here
    int32_t nslots;
    int32_t bm_words;               // words of one LDS claim table (a power of two)
    int64_t cmp_first;              // phase 0: first full compression after this many edges
    int2* sbuf;                     // reordering: [workers][sbuf_stride] edges (nbk > 0)
    int64_t sbuf_stride;
    int32_t nbk, bshift;            // buckets by the smaller endpoint (id >> bshift), 0: edges in input order
    int32_t nbk2, bshift2;          // ... times buckets by the larger one (id >> bshift2; 1: none)
    int32_t mbk;                    // merges inside the kernel read the sibling's certificate bucketed too
    int32_t wm_words;               // words of one written-bits map in LDS (0: no maps)
    uint32_t* slots;                // [nslots][2][V]
    uint32_t* slot_tag;             // [nslots] current tag of each slot (kept across calls)
    uint32_t* pool;                 // [ceil(nslots / 32)] bit set = slot free
    uint32_t* park;                 // [M] slot + 1 parked by left node i, 0 = none
    uint32_t* arrive;               // [M] arrivals at the merge whose right node is j
    uint32_t* queue;                // [1] next chunk
    uint32_t* dense;                // [ceil(M / 2^top)][V][2] node states at level top, compressed, untagged
    int2* cert;
    const int64_t* off;
    const int64_t* cap;
    uint32_t* cnt;                  // [M][2]
    uint32_t* err;                  // bit 0: id out of range; bit 1: region overflow
};

struct St {
    uint32_t* q;                    // slot base: F at q[x], F' at q[V + x]
    uint32_t V, tag, ob, mask;
    uint32_t cmask;                 // claim-table bits - 1
    uint32_t* wm;                   // LDS: bit x of F's map (first wmw words) / F''s map set once x's
    uint32_t wmw;                   //   word of the current tag may have been stored; null: no maps
    uint32_t* gm;                   // LDS (in place of F's map): bit x set if x was in one component of F
                                    //   (the largest, as sampled) when the slot was last compressed; null: none
    // the written-bits map of forest F (F's is taken by gm while gm is set)
    template <int F>
    __device__ __forceinline__ uint32_t* mapf() const { return (F == 0 && gm) ? nullptr : wm; }
    // x - parent(x) from x's word; a word of another tag, or one that could
    // not belong to x, reads as a root
    __device__ __forceinline__ uint32_t off(uint32_t w, uint32_t x) const {
        const uint32_t d = w & mask;
        return ((w >> ob) == tag && d <= x) ? d : 0u;
    }
    __device__ __forceinline__ uint32_t word(uint32_t d) const { return (tag << ob) | d; }
};

__device__ __forceinline__ uint32_t sld(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void sst(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// x's word in forest F (q: that forest's words), or 0 -- which reads as a
// root -- when x's bit in F's written-bits map (wm, the F map first, then
// F''s, wmw words each) is clear.  A map bit is set by the lane that stores
// the word turning x from a root into a child (the claim winner; every other
// store rewrites a child's word), so a clear bit proves no such store
// happened in an earlier round: the word in memory is of an older tag and
// reads as a root anyway.  A bit set in this round may be missed, like a word
// stored in this round; the claim tables settle that case as they do for
// words.  In a fresh chunk most words read were never written (endpoints seen
// for the first time, roots): the map saves their global loads.
template <int F>
__device__ __forceinline__ uint32_t wld(const uint32_t* wm, uint32_t wmw, const uint32_t* q, uint32_t x) {
    const bool stored = !wm || ((wm[(F ? wmw : 0u) + (x >> 5)] >> (x & 31)) & 1u);
    uint32_t w = 0u;
    if (stored) w = sld(q + x);
    return w;
}
template <int F>
__device__ __forceinline__ void wmark(uint32_t* wm, uint32_t wmw, uint32_t x) {
    if (wm) atomicOr(&wm[(F ? wmw : 0u) + (x >> 5)], 1u << (x & 31));
}

// representative of x in forest F (path halving on the way), d = x - its
// parent as read from x's word already (0: x reads as a root)
template <int F>
__device__ __forceinline__ uint32_t sfind_at(const St& S, uint32_t x, uint32_t d) {
    uint32_t* q = S.q + (F ? S.V : 0u);
    const uint32_t* wm = S.mapf<F>();
    while (d != 0) {
        const uint32_t p = x - d;
        const uint32_t dp = S.off(wld<F>(wm, S.wmw, q, p), p);
        if (dp == 0) return p;
        sst(q + x, S.word(d + dp));
        x = p - dp;
        d = S.off(wld<F>(wm, S.wmw, q, x), x);
    }
    return x;
}
template <int F>
__device__ __forceinline__ uint32_t sfind(const St& S, uint32_t x) {
    return sfind_at<F>(S, x, S.off(wld<F>(S.mapf<F>(), S.wmw, S.q + (F ? S.V : 0u), x), x));
}

// wavefront-aggregated reservation of slots on an LDS counter
__device__ __forceinline__ uint32_t lreserve(uint32_t* ctr, bool want) {
    const uint64_t m = __ballot(want);
    if (m == 0) return 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
    return __shfl(base, leader) + lane_rank(m);
}

// accepted edges go to the node's region: F from the front, F' from the back
// (every lane calls this: ballots)
__device__ __forceinline__ void emit(SoloLds& L, const SoloArgs& A, int64_t off, int64_t cap, int acc, int2 e) {
    const uint32_t p1 = lreserve(&L.n1, acc == 0);
    const uint32_t p2 = lreserve(&L.n2, acc == 1);
    if (acc == 0) { if (p1 < cap) A.cert[off + p1] = e; else atomicOr(A.err, 2u); }
    if (acc == 1) { if (p2 < cap) A.cert[off + cap - 1 - p2] = e; else atomicOr(A.err, 2u); }
}

// Barrier for the whole workgroup (global and LDS stores before it are
// visible after it) that also tells every lane whether any lane had p set,
// and empties the claim tables for the next round: every set bit has exactly
// one winner, which clears it (bits c1[j] of table t1 for j in mask w1, and
// c2/t2/w2 likewise).  It also copies the count of waiting edges for the
// lanes to read until the next such barrier.
template <int kSU>
__device__ __forceinline__ bool block_any(SoloLds& L, bool p, int& ph, uint32_t* t1, const uint32_t (&c1)[kSU],
                                          uint32_t w1, uint32_t* t2, const uint32_t (&c2)[kSU], uint32_t w2) {
    __syncthreads();
    if (p) L.flag[ph] = 1u;
    if (threadIdx.x == 0) L.nr_snap = L.nr;
#pragma unroll
    for (int j = 0; j < kSU; j++) {
        if (w1 >> j & 1) atomicAnd(&t1[c1[j] >> 5], ~(1u << (c1[j] & 31)));
        if (w2 >> j & 1) atomicAnd(&t2[c2[j] >> 5], ~(1u << (c2[j] & 31)));
    }
    __syncthreads();
    const bool any = L.flag[ph] != 0;
    if (threadIdx.x == 0) L.flag[ph ^ 1] = 0u;
    ph ^= 1;
    return any;
}

// Offer the edges of mask m (bit j: edge (u[j], v[j])) to forest F, all of
// them together: the endpoints' words, then their parents' words, are loaded
// for every edge before any is decided, so that the loads of the thread's
// edges are in flight at once; longer chains are then followed one by one
// (path halving, and the endpoint pointed straight at its root).  Out:
// masks of edges whose endpoints were already connected (same), that hooked
// a root (won), that lost a root to another lane (lost: retry later).
template <int F, int kSU>
__device__ __forceinline__ void bunite(const St& S, uint32_t* bm, const uint32_t (&u)[kSU], const uint32_t (&v)[kSU],
                                       uint32_t m, uint32_t& same, uint32_t& won, uint32_t& lost, uint32_t (&cl)[kSU]) {
    uint32_t* q = S.q + (F ? S.V : 0u);
    uint32_t* wm = S.mapf<F>();
    const uint32_t mm = m;
    uint32_t a[kSU], b[kSU], wa[kSU], wb[kSU];
#pragma unroll
    for (int j = 0; j < kSU; j++) {
        if (mm >> j & 1) {
            wa[j] = wld<F>(wm, S.wmw, q, u[j]);
            wb[j] = wld<F>(wm, S.wmw, q, v[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < kSU; j++) {
        if (mm >> j & 1) {
            a[j] = u[j] - S.off(wa[j], u[j]);
            b[j] = v[j] - S.off(wb[j], v[j]);
            wa[j] = (a[j] != b[j] && a[j] != u[j]) ? wld<F>(wm, S.wmw, q, a[j]) : 0u;
            wb[j] = (a[j] != b[j] && b[j] != v[j]) ? wld<F>(wm, S.wmw, q, b[j]) : 0u;
        }
    }
    same = won = lost = 0;
#pragma unroll
    for (int j = 0; j < kSU; j++) {
        // outcome r: 0 connected already, 1 hooked, 2 lost a race (the three
        // masks are updated without branches: no selected-by-address stores)
        uint32_t r = 0;
        if (mm >> j & 1) {
            uint32_t x = a[j], y = b[j];
            if (x != y) {
                // the parents' words loaded above start the finds
                if (S.off(wa[j], x) != 0) {
                    x = sfind_at<F>(S, x, S.off(wa[j], x));
                    sst(q + u[j], S.word(u[j] - x));
                }
                if (S.off(wb[j], y) != 0) {
                    y = sfind_at<F>(S, y, S.off(wb[j], y));
                    sst(q + v[j], S.word(v[j] - y));
                }
            }
            if (x != y) {
                const uint32_t hi = max(x, y), lo = min(x, y);
                const uint32_t c = hi & S.cmask;       // the root's claim bit
                const uint32_t bit = 1u << (c & 31);
                r = (atomicOr(&bm[c >> 5], bit) & bit) ? 2u : 1u;
                cl[j] = c;
                if (r == 1) {
                    sst(q + hi, S.word(hi - lo));
                    wmark<F>(wm, S.wmw, hi);
                }
            }
        }
        const uint32_t jb = (m >> j & 1) << j;
        same |= (r == 0 ? jb : 0u);
        won |= (r == 1 ? jb : 0u);
        lost |= (r == 2 ? jb : 0u);
    }
}

// Full path compression of a slot (no hook runs concurrently).  With gm,
// also the component map of F: bit x set iff x's root is groot (gm has
// ceil(V / 32) words; each wavefront writes the bits of its 64 vertices).
template <int kSB>
__device__ __forceinline__ void compress_slot(const St& S, uint32_t* gm = nullptr, uint32_t groot = 0) {
    const uint32_t gwords = (S.V + 31) / 32;
    for (int f = 0; f < 2; f++) {
        uint32_t* q = S.q + (f ? S.V : 0u);
        for (uint32_t x0 = 0; x0 < S.V; x0 += kSB) {      // the same trip count for every lane
            const uint32_t x = x0 + threadIdx.x;
            uint32_t r = x;
            if (x < S.V) {
                const uint32_t d = S.off(sld(q + x), x);
                if (d != 0) {
                    r = x - d;
                    for (uint32_t e = S.off(sld(q + r), r); e != 0; e = S.off(sld(q + r), r)) r -= e;
                    if (r != x - d) sst(q + x, S.word(x - r));
                }
            }
            if (f == 0 && gm) {
                const uint64_t m = __ballot(x < S.V && r == groot);
                const uint32_t w0 = (x0 + (threadIdx.x & ~63u)) >> 5;
                if ((threadIdx.x & 63u) == 0 && w0 < gwords) gm[w0] = (uint32_t)m;
                if ((threadIdx.x & 63u) == 0 && w0 + 1 < gwords) gm[w0 + 1] = (uint32_t)(m >> 32);
            }
        }
    }
}

// Offer a run of edges to the slot.  src 0: the input edge list, ids checked;
// src 1: a node region's certificate (F part [0, rn1), F' part after it);
// src 2: the worker's reordered copy of its chunk (sb).  With a wait buffer
// wb, the edges of a tile that lose a race do not hold the workgroup for a
// round of their own: they wait in wb, with their stage in bit 31 of the
// first id, and are offered again as tiles of their own after the last one
// (any order of the edges gives maximal forests).  wcap: wb's capacity in
// edges, or -1 when wb is sb itself (its front, over edges already offered);
// a tile defers only while the room left is certain to hold all its edges.
// stage0: where every edge starts (0: F, then F' if F rejects it; 1: F'
// only).  out: write accepted edges to (off, cap).  stages: compress the slot
// every cmp_first edges up to 2V, then at 8V (phase 0).  Each thread takes kSU
// edges of a tile and offers them together; edges that lost a race are
// retried, after a barrier, until none is left.
template <int kSB, int kSU>
__device__ __forceinline__ void stream(SoloLds& L, const SoloArgs& A, const St& S, uint32_t* bm1, uint32_t* bm2, int src, int64_t t0,
                       int64_t t1, int64_t roff, int64_t rcap, uint32_t rn1, uint32_t rn2, uint32_t stage0, bool out,
                       bool stages, int64_t off, int64_t cap, int& ph, int2* sb = nullptr,
                       int2* wb = nullptr, int64_t wcap = -1) {
    constexpr int64_t kST = (int64_t)kSB * kSU;      // edges per tile
    // phase 0: compress after cmp_first edges, then every cmp_first edges
    // up to 2 V, then at 8 V
    int64_t next_cmp = stages ? t0 + A.cmp_first : INT64_MAX;
    auto load = [&](int64_t i) -> int2 {
        if (i >= t1) return wb[i - t1];                       // the waiting edges
        if (src == 0) return i < A.split ? A.edges[i] : A.edges2[i - A.split];
        if (src == 2) return sb[i];
        return A.cert[i < rn1 ? roff + i : roff + rcap - rn2 + (i - rn1)];
    };
    const bool defer = wb != nullptr;
    bool late = false;                                   // tiles of waiting edges (indices t1 + k: wb[k])
    int64_t tend = t1;
    // the next tile's edges loaded a round ahead, where the registers allow
    // (with three edges per thread at 1,024 threads even one edge ahead
    // spills)
    constexpr bool kAhead = kSU <= 2;
    int2 nx[kSU];
#pragma unroll
    for (int j = 0; j < kSU; j++) {
        const int64_t i = t0 + j * kSB + threadIdx.x;
        nx[j] = (kAhead && i < t1) ? load(i) : make_int2(0, 0);
    }
    for (int64_t base = t0;; base += kST) {
        if (base >= tend) {
            if (!defer || late) break;
            late = true;
            base = t1;
            tend = t1 + (int64_t)L.nr_snap;
            if (base >= tend) break;
        }
        // losses of this tile wait in wb if [nr, nr + kST) fits (in sb: below the tile)
        const bool dtile = defer && !late && (int64_t)L.nr_snap + kST <= (wcap < 0 ? base : wcap);
        if (base >= next_cmp) {
            __syncthreads();
            compress_slot<kSB>(S);
            __syncthreads();
            const int64_t done = next_cmp - t0;
            next_cmp = done < 2 * (int64_t)S.V ? next_cmp + A.cmp_first
                                                 : (done < 8 * (int64_t)S.V ? t0 + 8 * (int64_t)S.V : INT64_MAX);
        }
        uint32_t u[kSU], v[kSU];
        uint32_t pend = 0, st1 = stage0 ? 0xffffffffu : 0u;   // st1 bit j: edge j is past F
#pragma unroll
        for (int j = 0; j < kSU; j++) {
            const int64_t i = base + j * kSB + threadIdx.x;
            const int2 e = (late || !kAhead) ? (i < tend ? load(i) : make_int2(0, 0)) : nx[j];
            u[j] = (uint32_t)e.x;
            v[j] = (uint32_t)e.y;
            if (late) {
                st1 |= (u[j] >> 31) << j;
                u[j] &= 0x7fffffffu;
            }
            // the next fresh tile's edge (the waiting edges are not read ahead:
            // this round may still add to them)
            const int64_t in = i + kST;
            if (kAhead) nx[j] = (!late && in < t1) ? load(in) : make_int2(0, 0);
        }
#pragma unroll
        for (int j = 0; j < kSU; j++) {
            if (base + j * kSB + threadIdx.x < tend) {
                if (u[j] < S.V && v[j] < S.V) pend |= 1u << j;
                else atomicOr(A.err, src == 0 ? 1u : 2u);
            }
        }
        // an edge with both endpoints in the component map's component is
        // rejected by F without a search (components only grow, so they are
        // still joined): it starts at F'
        if (S.gm) {
#pragma unroll
            for (int j = 0; j < kSU; j++)
                if ((pend >> j & 1) && ((S.gm[u[j] >> 5] >> (u[j] & 31)) & (S.gm[v[j] >> 5] >> (v[j] & 31)) & 1u))
                    st1 |= 1u << j;
        }
        uint32_t c1[kSU], c2[kSU];                         // claim bits this lane set
        for (;;) {
            uint32_t same = 0, won1 = 0, won2 = 0, lost = 0;
            const uint32_t m1 = pend & ~st1;
            if (m1) {
                uint32_t l1 = 0;
                bunite<0, kSU>(S, bm1, u, v, m1, same, won1, l1, c1);
                lost |= l1;
                st1 |= same;                    // F rejected them: on to F'
            }
            const uint32_t m2 = pend & st1;
            if (m2) {
                uint32_t s2 = 0, l2 = 0;
                bunite<1, kSU>(S, bm2, u, v, m2, s2, won2, l2, c2);
                lost |= l2;
            }
            if (out) {
#pragma unroll
                for (int j = 0; j < kSU; j++)
                    emit(L, A, off, cap, (won1 >> j & 1) ? 0 : ((won2 >> j & 1) ? 1 : -1),
                         make_int2((int32_t)u[j], (int32_t)v[j]));
            }
            pend = lost;
            if (dtile) {
#pragma unroll
                for (int j = 0; j < kSU; j++) {
                    const bool w = pend >> j & 1;
                    const uint32_t p = lreserve(&L.nr, w);
                    if (w) wb[p] = make_int2((int32_t)(u[j] | (st1 >> j & 1) << 31), (int32_t)v[j]);
                }
                pend = 0;
            }
            if (!block_any<kSU>(L, pend != 0, ph, bm1, c1, won1, bm2, c2, won2)) break;
        }
    }
}

__device__ __forceinline__ int64_t part_lo(int64_t E, int64_t M, int64_t i) { return i * (E / M) + (i * (E % M)) / M; }

// Copy the n edges load(0 .. n-1) with both ids below V to sb grouped by
// bucket -- the smaller endpoint's id >> bshift, then the larger's id >>
// bshift2 (a counting sort over nbk * nbk2 <= kMaxBuckets buckets: one pass
// to count, one to place) -- so that the stream then reads the endpoints'
// words from narrow id ranges.  Any order of the edges offered to a slot
// gives a pair of maximal forests; an id out of range sets `bad` in err and
// its edge is left out, as in input order.  cnt: kMaxBuckets + 1 words of
// LDS.  Returns the number of edges copied (every lane).
constexpr int kMaxBuckets = 1024;
template <int kSB, class Load>
__device__ __forceinline__ int64_t bucket_into(const SoloArgs& A, int64_t n, Load load, uint32_t bad, int2* sb, uint32_t V,
                               uint32_t* cnt) {
    uint32_t& total = cnt[kMaxBuckets];
    const int nb = A.nbk * A.nbk2;
    const uint32_t nbk2 = (uint32_t)A.nbk2, s1 = (uint32_t)A.bshift, s2 = (uint32_t)A.bshift2;
    uint32_t* err = A.err;
    auto key = [=](int2 e) -> uint32_t {
        const uint32_t a = min((uint32_t)e.x, (uint32_t)e.y), b = max((uint32_t)e.x, (uint32_t)e.y);
        return (a >> s1) * nbk2 + (b >> s2);
    };
    // kBK edges per thread per step, their loads issued together
    constexpr int kBK = 4;
    for (int b = threadIdx.x; b < nb; b += kSB) cnt[b] = 0u;
    __syncthreads();
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)kBK * kSB) {
        int2 e[kBK];
#pragma unroll
        for (int k = 0; k < kBK; k++) {
            const int64_t i = i0 + (int64_t)k * kSB;
            e[k] = i < n ? load(i) : make_int2(0, 0);
        }
#pragma unroll
        for (int k = 0; k < kBK; k++) {
            if (i0 + (int64_t)k * kSB >= n) continue;
            if ((uint32_t)e[k].x < V && (uint32_t)e[k].y < V) atomicAdd(&cnt[key(e[k])], 1u);
            else atomicOr(err, bad);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < nb; b++) {
            const uint32_t c = cnt[b];
            cnt[b] = acc;
            acc += c;
        }
        total = acc;
    }
    __syncthreads();
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += (int64_t)kBK * kSB) {
        int2 e[kBK];
#pragma unroll
        for (int k = 0; k < kBK; k++) {
            const int64_t i = i0 + (int64_t)k * kSB;
            e[k] = i < n ? load(i) : make_int2(0, 0);
        }
#pragma unroll
        for (int k = 0; k < kBK; k++)
            if (i0 + (int64_t)k * kSB < n && (uint32_t)e[k].x < V && (uint32_t)e[k].y < V)
                sb[atomicAdd(&cnt[key(e[k])], 1u)] = e[k];
    }
    __syncthreads();        // sb written by the workgroup, read back by it
    return (int64_t)total;
}

// the edges of input chunk [lo, ...) and of a node region's certificate (F
// part [0, n1), F' part after it), as loaders by index (captured by value:
// a reference to the kernel's argument block would move it to private memory)
struct InputLoad {
    const int2 *e1, *e2;
    int64_t split, lo;
    __device__ int2 operator()(int64_t k) const { return lo + k < split ? e1[lo + k] : e2[lo + k - split]; }
};
struct RegionLoad {
    const int2* c;
    int64_t off, cap, n1, n2;
    __device__ int2 operator()(int64_t k) const { return c[k < n1 ? off + k : off + cap - n2 + (k - n1)]; }
};

// a free slot from the pool (thread 0), -1 if none; acquire on success
__device__ __forceinline__ int pool_pop(const SoloArgs& A) {
    const int words = (A.nslots + 31) / 32;
    for (int w = 0; w < words; w++) {
        uint32_t v = __hip_atomic_load(&A.pool[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (v) {
            const uint32_t bit = v & (~v + 1u);
            const uint32_t old = atomicAnd(&A.pool[w], ~bit);
            if (old & bit) {
                __threadfence();
                return w * 32 + __ffs((int)bit) - 1;
            }
            v = old & ~bit;
        }
    }
    return -1;
}

// give a slot back (thread 0; the caller has released what it wrote)
__device__ __forceinline__ void pool_push(const SoloArgs& A, int s) { atomicOr(&A.pool[s >> 5], 1u << (s & 31)); }

}  // namespace

template <int kSB, int kSU>
__global__ void __launch_bounds__(kSB) k_solo(SoloArgs A) {
    extern __shared__ uint4 lds_raw[];
    SoloLds& L = *reinterpret_cast<SoloLds*>(lds_raw);
    uint32_t* bm1 = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(lds_raw) + sizeof(SoloLds));
    uint32_t* bm2 = bm1 + A.bm_words;
    // after the claim tables and the bucket counters: the written-bits maps
    uint32_t* wmap = A.wm_words ? bm2 + A.bm_words + (kMaxBuckets + 1) : nullptr;
    const uint32_t V = (uint32_t)A.V;
    const uint32_t mask = A.ob >= 32 ? 0xffffffffu : ((1u << A.ob) - 1u);
    const uint32_t tag_max = A.ob >= 31 ? 1u : ((1u << (32 - A.ob)) - 1u);
    const int64_t top_step = int64_t(1) << A.top;
    if (threadIdx.x == 0) {
        L.slot = blockIdx.x;        // every worker starts with its own slot
        L.flag[0] = L.flag[1] = 0u;
    }
    int ph = 0;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) L.item = (int32_t)atomicAdd(A.queue, 1u);
        __syncthreads();
        const int64_t c = L.item;
        if (c >= A.M) break;
        // ---- phase 0: the certificate of chunk c in a fresh tag of my slot
        if (threadIdx.x == 0) {
            uint32_t t = A.slot_tag[L.slot] + 1;
            L.act = 0;
            if (t > tag_max) { t = 1; L.act = 1; }
            A.slot_tag[L.slot] = t;
            L.tag = t;
            L.n1 = L.n2 = 0;
            L.nr = L.nr_snap = 0;
        }
        __syncthreads();
        St S{A.slots + (size_t)L.slot * 2 * V, V, L.tag, (uint32_t)A.ob, mask, 32u * (uint32_t)A.bm_words - 1u,
             wmap, (uint32_t)A.wm_words, nullptr};
        if (L.act == 1)         // tags ran out: every word back to "root"
            for (uint32_t x = threadIdx.x; x < 2 * V; x += kSB) S.q[x] = 0u;
        for (int x = threadIdx.x; x < 2 * A.bm_words; x += kSB) bm1[x] = 0u;
        if (wmap)               // a fresh tag: no word of it stored yet
            for (int x = threadIdx.x; x < 2 * A.wm_words; x += kSB) wmap[x] = 0u;
        __syncthreads();
        {
            // the chunk in input order, or bucketed into the worker's buffer
            // (one call site of the stream: each one costs registers)
            int64_t t0 = part_lo(A.E, A.M, c), t1 = part_lo(A.E, A.M, c + 1);
            int src = 0;
            int2* sb = nullptr;
            if (A.nbk > 0) {
                sb = A.sbuf + (size_t)blockIdx.x * (size_t)A.sbuf_stride;
                t1 = bucket_into<kSB>(A, t1 - t0, InputLoad{A.edges, A.edges2, A.split, t0}, 1u, sb, V, bm2 + A.bm_words);
                t0 = 0;
                src = 2;
            }
            stream<kSB, kSU>(L, A, S, bm1, bm2, src, t0, t1, 0, 0, 0, 0, 0, true, true, A.off[c], A.cap[c], ph, sb, sb);
        }
        // ---- climb the merge tree while this worker finishes a pair second
        int64_t node = c, step = 1;
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) {
                A.cnt[2 * node] = L.n1;
                A.cnt[2 * node + 1] = L.n2;
                if ((int64_t)L.n1 + L.n2 > A.cap[node]) atomicOr(A.err, 2u);
            }
            if (step >= A.M || step >= top_step) {
                // the node's state, fully compressed and untagged, for the
                // merge rounds above (and, at the top, the final step)
                // kU vertices per thread at a time, the chains of both forests
                // followed together (chain c: vertex c / 2, forest c % 2), so
                // that each step's loads are in flight at once
                constexpr int kU = 2;
                uint2* dn = reinterpret_cast<uint2*>(A.dense) + (size_t)(node >> A.top) * V;
                for (uint32_t x0 = 0; x0 < V; x0 += kU * kSB) {
                    uint32_t y[2 * kU];
                    uint32_t live = 0;
#pragma unroll
                    for (int c = 0; c < 2 * kU; c++) {
                        y[c] = x0 + (uint32_t)(c / 2) * kSB + threadIdx.x;
                        if (y[c] < V) live |= 1u << c;
                    }
                    while (live) {
                        uint32_t e[2 * kU];
#pragma unroll
                        for (int c = 0; c < 2 * kU; c++)
                            e[c] = (live >> c & 1) ? S.off(sld(S.q + (c & 1 ? V : 0u) + y[c]), y[c]) : 0u;
#pragma unroll
                        for (int c = 0; c < 2 * kU; c++) {
                            y[c] -= e[c];
                            if (e[c] == 0) live &= ~(1u << c);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < kU; k++) {
                        const uint32_t x = x0 + (uint32_t)k * kSB + threadIdx.x;
                        if (x < V) dn[x] = make_uint2(x - y[2 * k], x - y[2 * k + 1]);
                    }
                }
                break;
            }
            const int64_t i = node & ~(2 * step - 1), j = i + step;
            if (j >= A.M) {                                   // no partner: passes through
                node = i;
                step *= 2;
                continue;
            }
            __syncthreads();   // every lane's writes (region, state) done before thread 0 publishes
            if (threadIdx.x == 0) {
                int spare = -1;
                L.adopted = 0;
                if (node == i) {       // park my state for the right node's worker, in case it comes last
                    spare = pool_pop(A);
                    A.park[i] = spare >= 0 ? (uint32_t)L.slot + 1 : 0u;
                }
                __threadfence();       // release: region, counts, state, parking
                const uint32_t prev = atomicAdd(&A.arrive[j], 1u);
                int act;
                if (prev == 0) {       // first of the pair: the partner merges
                    if (spare >= 0) L.slot = spare;     // the parked slot is no longer mine
                    act = 0;
                } else {
                    __threadfence();   // acquire the partner's region, counts and parking
                    if (node == i) {   // my own state is still here
                        if (spare >= 0) pool_push(A, spare);
                        A.park[i] = 0;
                        act = 1;
                    } else {
                        const uint32_t p = __hip_atomic_load(&A.park[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (p) {       // adopt the left node's state, give mine back
                            pool_push(A, L.slot);
                            L.slot = (int32_t)p - 1;
                            A.park[i] = 0;
                            L.adopted = 1;
                            act = 1;
                        } else {
                            act = 2;   // the left state is gone: rebuild it in my slot
                        }
                    }
                }
                L.act = act;
                if (act == 2) {
                    uint32_t t = A.slot_tag[L.slot] + 1;
                    if (t > tag_max) { t = 1; L.act = 3; }
                    A.slot_tag[L.slot] = t;
                }
                L.tag = A.slot_tag[L.slot];
                L.n1 = A.cnt[2 * i];
                L.n2 = A.cnt[2 * i + 1];
                L.nj1 = A.cnt[2 * j];
                L.nj2 = A.cnt[2 * j + 1];
                L.nr = L.nr_snap = 0;
            }
            __syncthreads();
            const int act = L.act;
            if (act == 0) break;
            S.q = A.slots + (size_t)L.slot * 2 * V;
            S.tag = L.tag;
            if (L.adopted) S.wm = nullptr;     // my maps describe my old slot, not the adopted one
            if (L.adopted || act >= 2) S.gm = nullptr;   // and so does the component map
            for (int x = threadIdx.x; x < 2 * A.bm_words; x += kSB) bm1[x] = 0u;
            if (act >= 2 && S.wm)              // rebuilt under a fresh tag
                for (int x = threadIdx.x; x < 2 * A.wm_words; x += kSB) S.wm[x] = 0u;
            if (act == 3)
                for (uint32_t x = threadIdx.x; x < 2 * V; x += kSB) S.q[x] = 0u;
            const int64_t offi = A.off[i], capi = A.cap[i];
            const uint32_t ni1 = min(L.n1, (uint32_t)capi), ni2 = min(L.n2, (uint32_t)capi - ni1);
            __syncthreads();
            if (act >= 2) {
                // node i's state from its certificate: F's edges into F (a
                // forest: all accepted), then F''s into F' (all accepted)
                stream<kSB, kSU>(L, A, S, bm1, bm2, 1, 0, ni1, offi, capi, ni1, ni2, 0, false, false, 0, 0, ph);
                stream<kSB, kSU>(L, A, S, bm1, bm2, 1, ni1, (int64_t)ni1 + ni2, offi, capi, ni1, ni2, 1, false, false, 0, 0, ph);
            }
            // X_j into node i's state; accepted edges extend node i's region
            const int64_t offj = A.off[j], capj = A.cap[j];
            const uint32_t nj1 = min(L.nj1, (uint32_t)capj), nj2 = min(L.nj2, (uint32_t)capj - nj1);
            if ((int64_t)nj1 + nj2 >= (int64_t)V / 2) {
                if (wmap) {
                    // the root most of 64 evenly spread vertices reach in F
                    // (the largest component, as a rule): its members get
                    // marked while the slot is compressed
                    if (threadIdx.x < 64) {
                        const uint32_t r = sfind<0>(S, (uint32_t)(((uint64_t)threadIdx.x * V) >> 6));
                        uint32_t c = 0;
                        for (int k = 0; k < 64; k++) c += __shfl(r, k) == r ? 1u : 0u;
                        uint32_t key = (c << 6) | threadIdx.x;
                        for (int o = 32; o > 0; o >>= 1) key = max(key, (uint32_t)__shfl_xor((int)key, o));
                        if (threadIdx.x == (key & 63u)) L.groot = r;
                    }
                    __syncthreads();
                    compress_slot<kSB>(S, wmap, L.groot);
                    S.gm = wmap;                   // F's written-bits map gives way to the component map
                } else {
                    compress_slot<kSB>(S);
                }
                __syncthreads();
            }
            int64_t nj = (int64_t)nj1 + nj2;
            int src = 1;
            int2* sb = nullptr;
            // the worker's copy buffer is idle in merges: edges that lose a race wait there
            int2* wb = A.nbk > 0 ? A.sbuf + (size_t)blockIdx.x * (size_t)A.sbuf_stride : nullptr;
            int64_t wcap = A.sbuf_stride;
            if (A.mbk && A.nbk > 0 && nj <= A.sbuf_stride) {
                // X_j bucketed like a phase-0 chunk (sb's last reads came before a barrier)
                sb = A.sbuf + (size_t)blockIdx.x * (size_t)A.sbuf_stride;
                nj = bucket_into<kSB>(A, nj, RegionLoad{A.cert, offj, capj, (int64_t)nj1, (int64_t)nj2}, 2u, sb, V,
                                      bm2 + A.bm_words);
                src = 2;
                wcap = -1;
            }
            stream<kSB, kSU>(L, A, S, bm1, bm2, src, 0, nj, offj, capj, nj1, nj2, 0, true, false, offi, capi, ph, sb,
                             wb, wcap);
            node = i;
            step *= 2;
        }
    }
}

namespace {
// per call: the free pool (slots past the workers'), no parking, no arrivals, queue at 0
__global__ void k_solo_init(uint32_t* pool, int32_t nslots, int32_t first_free, uint32_t* park_arrive, int64_t n,
                            uint32_t* queue) {
    const int words = (nslots + 31) / 32;
    GRID_LOOP(k, n) park_arrive[k] = 0u;
    GRID_LOOP(w, words) {
        uint32_t v = 0;
        for (int b = 0; b < 32; b++) {
            const int s = (int)w * 32 + b;
            if (s >= first_free && s < nslots) v |= 1u << b;
        }
        pool[w] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0u;
}
}  // namespace

// Claim-table words per forest: V bits rounded up to a power of two, at most
// 2^18 bits (32 KB); a larger V shares bits between roots.
static int32_t claim_words(int32_t V) {
    int64_t bits = 32;
    while (bits < (int64_t)V && bits < (int64_t(1) << 18)) bits <<= 1;
    return (int32_t)(bits / 32);
}

// the control block, the two claim tables, the bucket counters of phase 0,
// and (wm) the two written-bits maps of V bits each
static int32_t written_words(int32_t V) { return (int32_t)(((int64_t)V + 31) / 32); }
size_t solo_lds_bytes(int32_t V, bool wm) {
    return sizeof(SoloLds) + 2 * 4 * (size_t)claim_words(V) + 4 * (size_t)(kMaxBuckets + 1) +
           (wm ? 2 * 4 * (size_t)written_words(V) : 0);
}
bool solo_wm_fits(int32_t V) { return solo_lds_bytes(V, true) <= (size_t)g_max_lds; }

// Worker shapes: (threads, edges per thread offered together), chosen per
// plan (the tuner measures them).  Three edges per thread at 1,024 threads
// still fits the 128 registers such a workgroup allows; four does not.
struct SoloVariant {
    const void* fn;
    int sb;
};
static const SoloVariant kVariants[] = {
    {reinterpret_cast<const void*>(&k_solo<512, 2>), 512},
    {reinterpret_cast<const void*>(&k_solo<1024, 1>), 1024},
    {reinterpret_cast<const void*>(&k_solo<1024, 2>), 1024},
    {reinterpret_cast<const void*>(&k_solo<512, 1>), 512},
    {reinterpret_cast<const void*>(&k_solo<1024, 3>), 1024},
};
int solo_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
int solo_block(int variant) { return kVariants[std::max(0, std::min(variant, solo_variants() - 1))].sb; }

int solo_prepare(int32_t V) {
    const size_t b = solo_lds_bytes(V, false);
    if (b > (size_t)g_max_lds) return fail(BR_EINTERNAL, "solo: V = %d needs %zu bytes of LDS", V, b);
    static std::once_flag once;
    static hipError_t e = hipSuccess;
    std::call_once(once, [] {
        for (const SoloVariant& k : kVariants) {
            if (e != hipSuccess) break;
            e = hipFuncSetAttribute(k.fn, hipFuncAttributeMaxDynamicSharedMemorySize, g_max_lds);
        }
    });
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(k_solo)");
    return BR_OK;
}

void launch_solo(const Plan& P, const DevBufs& B, const SoloBufs& Sb, hipStream_t s) {
    const int64_t n = 2 * (int64_t)P.M;
    hipLaunchKernelGGL(k_solo_init, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024))),
                       dim3(256), 0, s, Sb.pool, Sb.nslots, Sb.workers, Sb.park, n, Sb.queue);
    SoloArgs A;
    A.edges = B.edges;
    A.edges2 = B.edges2;
    A.split = B.split;
    A.E = P.E;
    A.V = P.V;
    A.M = P.M;
    int ob = 1;
    while (ob < 31 && (int64_t(1) << ob) <= (int64_t)P.V - 1) ob++;
    A.ob = ob;
    A.top = P.solo_top;
    A.nslots = Sb.nslots;
    A.bm_words = claim_words(P.V);
    A.cmp_first = std::max<int64_t>(1024, (int64_t)P.solo_cmp * P.V / 8);
    A.sbuf = Sb.sbuf;
    A.sbuf_stride = Sb.sbuf_stride;
    A.nbk = Sb.sbuf ? P.solo_nbk : 0;
    A.nbk2 = std::max(1, std::min(P.solo_nbk2, kMaxBuckets / std::max(1, A.nbk)));
    auto shift_for = [&](int n) {
        int b = 0;
        while (n > 0 && ((int64_t)(P.V - 1) >> b) >= n) b++;
        return b;
    };
    A.bshift = shift_for(A.nbk);
    A.bshift2 = shift_for(A.nbk2);
    A.mbk = P.solo_mbk ? 1 : 0;
    A.wm_words = P.solo_wm ? written_words(P.V) : 0;
    A.slots = Sb.slots;
    A.slot_tag = Sb.slot_tag;
    A.pool = Sb.pool;
    A.park = Sb.park;
    A.arrive = Sb.park + P.M;
    A.queue = Sb.queue;
    A.dense = Sb.dense;
    A.cert = B.cert;
    A.off = B.off;
    A.cap = B.cap;
    A.cnt = B.cnt;
    A.err = B.err;
    const SoloVariant& k = kVariants[std::max(0, std::min(P.solo_variant, solo_variants() - 1))];
    void* args[] = {&A};
    (void)hipLaunchKernel(k.fn, dim3((unsigned)Sb.workers), dim3(k.sb), args, solo_lds_bytes(P.V, P.solo_wm), s);
}

// largest V of the plan (the slots hold 8 V bytes each, all of them within
// 8 GiB: at least 8 slots)
int32_t solo_max_v() { return 1 << 27; }

// workgroups of the variant that fit on one CU with the LDS V needs
int solo_blocks_per_cu(int variant, int32_t V, bool wm) {
    const SoloVariant& k = kVariants[std::max(0, std::min(variant, solo_variants() - 1))];
    int n = 0;
    if (solo_prepare(V) != BR_OK ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k.fn, k.sb, solo_lds_bytes(V, wm)) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return std::max(1, n);
}

}  // namespace br
