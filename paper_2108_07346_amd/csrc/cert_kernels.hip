// Certificate kernels for gfx950: per-chunk certificates (phase 0) and the
// pairwise merge rounds of the phase tree (paper, Section III; Algorithm 2).
//
// Union-find state.  For every vertex x and forest f (0 = F, 1 = F') one
// 32-bit word q[qs*x+f] holds x - parent(x); 0 marks a root, so a zero-filled
// buffer is the all-singletons state.  qs = 2 packs 16 vertices into a
// 128-byte line; qs = 8 gives each vertex 32 bytes, so that a hook (a swap
// performed at the memory side, which takes the line out of L2) disturbs the
// words of fewer other vertices -- faster where the whole state stays small.  Parents always have smaller ids than
// their children (a root is hooked under the smaller root), which makes
// every pointer chain strictly decreasing and the structure acyclic.
//
// Concurrency.  Many lanes update one chunk's state at once.  Lanes read
// parent words with plain cached loads; any value they see, however stale,
// names a vertex of the same component with a smaller id (components only
// merge, and a word only ever moves to a smaller parent).  So two finds that
// meet prove the endpoints connected: a rejected edge is never wrongly
// rejected.  An edge is accepted only by a compare-and-swap that turns a
// current root into a child of the other endpoint's representative, which
// merges two distinct components (the representative cannot lie below the
// root: chains only decrease).  A failed swap returns the root's new parent
// and the search continues from there, so the larger of the two ids strictly
// decreases each retry and the loop ends.  Per edge this is one fused pass:
// offered to F, and if F rejects it, offered to F' (F' is then a maximal
// forest of the edges F rejected, as Algorithm 2 requires).
//
// Certificate regions.  Node i owns pairs [off[i], off[i] + cap[i]); accepted
// F edges are appended from the front, F' edges from the back, each through
// one atomic add per wavefront (ballot + popcount + lane rank).

#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "internal.hpp"

namespace br {

namespace {

constexpr int kBlock = 512;
constexpr int kTile = 4096;   // edges per workgroup tile (a multiple of kBlock)

__device__ __forceinline__ uint32_t ld(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void st(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ uint64_t ld2(const uint32_t* p) {
    return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// representative of x in forest F (path halving on the way)
template <int F>
__device__ __forceinline__ uint32_t uf_find(uint32_t* q, int64_t qs, uint32_t x) {
    uint32_t d = ld(q + qs * (int64_t)x + F);
    while (d != 0) {
        const uint32_t p = x - d;
        const uint32_t dp = ld(q + qs * (int64_t)p + F);
        if (dp == 0) return p;
        st(q + qs * (int64_t)x + F, d + dp);   // x now points at its grandparent
        x = p - dp;
        d = ld(q + qs * (int64_t)x + F);
    }
    return x;
}

// true iff this call merged the components of u and v in forest F
template <int F>
__device__ __forceinline__ bool uf_unite(uint32_t* q, int64_t qs, uint32_t u, uint32_t v) {
    for (;;) {
        u = uf_find<F>(q, qs, u);
        v = uf_find<F>(q, qs, v);
        if (u == v) return false;
        if (u < v) { const uint32_t t = u; u = v; v = t; }
        uint32_t expect = 0;
        if (__hip_atomic_compare_exchange_strong(q + qs * (int64_t)u + F, &expect, u - v, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return true;
        u = u - expect;   // u was hooked meanwhile: continue from its parent
    }
}

// Offer edge (u,v) to F, then (if rejected) to F'.  su, sv are the
// endpoints' parent words (F low, F' high), loaded earlier with one 8-byte
// load each: however stale, each names an ancestor (or the vertex itself), a
// valid place to start the finds from.
__device__ __forceinline__ void offer_from(uint32_t* q, int64_t qs, uint32_t u, uint32_t v, uint64_t su, uint64_t sv,
                                           bool& a1, bool& a2) {
    const uint32_t p1u = u - (uint32_t)su, p1v = v - (uint32_t)sv;
    a1 = (p1u != p1v) && uf_unite<0>(q, qs, p1u, p1v);
    a2 = false;
    if (!a1) {
        const uint32_t p2u = u - (uint32_t)(su >> 32), p2v = v - (uint32_t)(sv >> 32);
        a2 = (p2u != p2v) && uf_unite<1>(q, qs, p2u, p2v);
    }
}


// Accepted edges of one workgroup tile are staged in LDS (F from the front,
// F' from the back of the stage), then the tile reserves its ranges in the
// node's region with one global atomic per forest and copies them out.  Every
// lane of the workgroup must call these (ballots and barriers).
struct Stage {
    int2 e[kTile];
    uint32_t n1, n2;
    uint32_t base1, base2;
};

__device__ __forceinline__ void stage_reset(Stage& S) {
    if (threadIdx.x == 0) { S.n1 = 0; S.n2 = 0; }
    __syncthreads();
}

__device__ __forceinline__ void stage_put(Stage& S, bool a1, bool a2, int2 e) {
    const uint64_t m1 = __ballot(a1), m2 = __ballot(a2);
    const int lane = __lane_id();
    if (m1) {
        const int leader = __ffsll((unsigned long long)m1) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&S.n1, (uint32_t)__popcll(m1));
        base = __shfl(base, leader);
        if (a1) S.e[base + lane_rank(m1)] = e;
    }
    if (m2) {
        const int leader = __ffsll((unsigned long long)m2) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&S.n2, (uint32_t)__popcll(m2));
        base = __shfl(base, leader);
        if (a2) S.e[kTile - 1 - (base + lane_rank(m2))] = e;
    }
}

__device__ __forceinline__ void stage_flush(Stage& S, const DevBufs& B, int64_t node) {
    __syncthreads();
    const uint32_t n1 = S.n1, n2 = S.n2;
    if (threadIdx.x == 0) {
        S.base1 = n1 ? atomicAdd(B.cnt + 2 * node, n1) : 0;
        S.base2 = n2 ? atomicAdd(B.cnt + 2 * node + 1, n2) : 0;
    }
    __syncthreads();
    const int64_t off = B.off[node], cap = B.cap[node];
    const int64_t b1 = S.base1, b2 = S.base2;
    for (uint32_t k = threadIdx.x; k < n1 + n2; k += kBlock) {
        int64_t pos;
        int2 e;
        if (k < n1) { pos = b1 + k; e = S.e[k]; }
        else { pos = b2 + (k - n1); e = S.e[kTile - 1 - (k - n1)]; }
        if (pos >= cap) { atomicOr(B.err, 2u); continue; }
        B.cert[k < n1 ? off + pos : off + cap - 1 - pos] = e;
    }
}

// Offer edges [t0, t1) (t1 - t0 <= kTile) of a tile to the state q, staging
// the accepted ones; load(i, e) fetches edge i and says whether it is valid.
// Pre: all of the thread's edges are requested at once, and each edge's parent
// words while the previous edge is decided; else one edge at a time.
template <bool Pre, class Load>
__device__ __forceinline__ void offer_tile(Stage& S, uint32_t* q, int64_t qs, int64_t t0, int64_t t1, Load load) {
    if (!Pre) {
        for (int64_t base = t0; base < t1; base += kBlock) {
            const int64_t i = base + threadIdx.x;
            bool a1 = false, a2 = false;
            int2 e = make_int2(0, 0);
            if (i < t1 && load(i, e))
                offer_from(q, qs, (uint32_t)e.x, (uint32_t)e.y, ld2(q + qs * (int64_t)e.x), ld2(q + qs * (int64_t)e.y),
                           a1, a2);
            stage_put(S, a1, a2, e);
        }
        return;
    }
    constexpr int kPer = kTile / kBlock;
    const int n = (int)((t1 - t0 + kBlock - 1) / kBlock);    // the same for every lane
    int2 e[kPer];
    uint32_t ok = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        const int64_t i = t0 + (int64_t)j * kBlock + threadIdx.x;
        e[j] = make_int2(0, 0);
        if (j < n && i < t1 && load(i, e[j])) ok |= 1u << j;
    }
    uint64_t su = 0, sv = 0;
    if (ok & 1u) {
        su = ld2(q + qs * (int64_t)e[0].x);
        sv = ld2(q + qs * (int64_t)e[0].y);
    }
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        if (j >= n) break;
        uint64_t nu = 0, nv = 0;
        if (j + 1 < kPer && (ok >> (j + 1) & 1u)) {
            nu = ld2(q + qs * (int64_t)e[j + 1].x);
            nv = ld2(q + qs * (int64_t)e[j + 1].y);
        }
        bool a1 = false, a2 = false;
        if (ok >> j & 1u) offer_from(q, qs, (uint32_t)e[j].x, (uint32_t)e[j].y, su, sv, a1, a2);
        stage_put(S, a1, a2, e[j]);
        su = nu;
        sv = nv;
    }
}

__device__ __forceinline__ int64_t chunk_lo(int64_t E, int32_t M, int64_t i) {
    // floor(i*E/M) without overflow: i*(E/M) + floor(i*(E%M)/M)
    return i * (E / M) + (i * (E % M)) / M;
}

// Phase 0: workgroup b certifies one tile of one chunk into that chunk's state.
// Stage [rel_lo, rel_hi) of every chunk (offsets relative to the chunk start).
__global__ void __launch_bounds__(kBlock) k_phase0(DevBufs B, int64_t E, int32_t V, int32_t M, int32_t tile,
                                                   int32_t tpc, int32_t xcd_map, int64_t rel_lo, int64_t rel_hi) {
    int64_t c, s;
    const int64_t b = blockIdx.x;
    if (xcd_map) {       // chunk c lives on XCD c % 8: blocks b with b % 8 == c % 8
        const int64_t j = b >> 3;
        c = (b & 7) + 8 * (j / tpc);
        s = j % tpc;
    } else {
        c = b / tpc;
        s = b % tpc;
    }
    if (c >= M) return;
    const int64_t lo = chunk_lo(E, M, c), hi = min(chunk_lo(E, M, c + 1), lo + rel_hi);
    const int64_t t0 = lo + rel_lo + s * (int64_t)tile;
    const int64_t t1 = min(t0 + (int64_t)tile, hi);
    if (t0 >= t1) return;
    __shared__ Stage S;
    stage_reset(S);
    uint32_t* q = B.state + (size_t)c * (size_t)B.qs * (size_t)V;
    // one edge at a time: prefetching a thread's tile measured slower here
    // (dense M = 16 phase 0: 0.334 -> 0.344 ms in the first stage, no gain
    // in the rejecting stage)
    offer_tile<false>(S, q, B.qs, t0, t1, [&](int64_t i, int2& e) {
        e = i < B.split ? B.edges[i] : B.edges2[i - B.split];
        if ((uint32_t)e.x < (uint32_t)V && (uint32_t)e.y < (uint32_t)V) return true;
        atomicOr(B.err, 1u);
        return false;
    });
    stage_flush(S, B, c);
}

// One merge round with partner distance `step`: node i (i % 2step == 0) keeps
// its union-find state (which encodes exactly its F and F') and streams the
// certificate of node i+step through it; the accepted edges extend node i's F
// and F'.  This equals recomputing the certificate of the union with node i's
// edges offered first.
template <bool Pre>
__global__ void __launch_bounds__(kBlock) k_merge(DevBufs B, int32_t V, int32_t M, int32_t step, int32_t tile,
                                                  int32_t tpm) {
    const int64_t m = blockIdx.x / tpm, s = blockIdx.x % tpm;
    const int64_t i = m * 2 * (int64_t)step, j = i + step;
    if (j >= M) return;
    const int64_t offj = B.off[j], capj = B.cap[j];
    // counters past the region mean an overflow already flagged in B.err; clamp
    // so that no read leaves node j's region
    const int64_t n1 = min((int64_t)B.cnt[2 * j], capj), n2 = min((int64_t)B.cnt[2 * j + 1], capj - n1);
    const int64_t total = n1 + n2;
    const int64_t t0 = s * (int64_t)tile, t1 = min(t0 + (int64_t)tile, total);
    if (t0 >= t1) return;
    __shared__ Stage S;
    stage_reset(S);
    uint32_t* q = B.state + (size_t)(i >> B.shift) * (size_t)B.qs * (size_t)V;
    offer_tile<Pre>(S, q, B.qs, t0, t1, [&](int64_t k, int2& e) {
        e = B.cert[k < n1 ? offj + k : offj + capj - n2 + (k - n1)];
        return true;
    });
    stage_flush(S, B, i);
}

// Node 0's certificate -> caller's buffer (F then F'), plus counts and status.
__global__ void k_copy_out(DevBufs B, int2* out, int64_t out_cap, int64_t* counts) {
    const int64_t n1 = B.cnt[0], n2 = B.cnt[1], cap = B.cap[0], off = B.off[0];
    const uint32_t err = *B.err;
    const bool ok = err == 0 && n1 + n2 <= cap && n1 + n2 <= out_cap;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; ok && k < n1 + n2;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = B.cert[k < n1 ? off + k : off + cap - n2 + (k - n1)];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[0] = n1;
        counts[1] = n2;
        counts[2] = (err & 1u) ? BR_ERANGE : ((err != 0 || n1 + n2 > cap) ? BR_EINTERNAL : (n1 + n2 > out_cap ? BR_ECAP : BR_OK));
    }
}

// Full path compression of the first `slots` chunk states between stages: every
// vertex points straight at its representative, so that later edges inside a
// component are rejected by the two-load test in offer_from() without any search.
// No hook runs concurrently, so plain stores are safe.
__global__ void k_compress(uint32_t* state, int64_t qs, int32_t V, int64_t slots) {
    const int64_t n = (int64_t)V * slots;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t* q = state + (size_t)(k / V) * (size_t)qs * (size_t)V;
        const uint32_t x = (uint32_t)(k % V);
        for (int f = 0; f < 2; f++) {
            const uint32_t d = q[qs * (int64_t)x + f];
            if (d == 0) continue;
            uint32_t r = x - d;
            for (uint32_t e = q[qs * (int64_t)r + f]; e != 0; e = q[qs * (int64_t)r + f]) r -= e;
            if (r != x - d) q[qs * (int64_t)x + f] = x - r;
        }
    }
}

// The same full compression, written into a packed copy (two words per
// vertex) of a state laid out with qs words per vertex; the source is only
// read, so the copy is exact whatever order the threads run in.
__global__ void k_compress_pack(const uint32_t* state, int64_t qs, uint32_t* packed, int32_t V, int64_t slots) {
    const int64_t n = (int64_t)V * slots;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t* q = state + (size_t)(k / V) * (size_t)qs * (size_t)V;
        const uint32_t x = (uint32_t)(k % V);
        uint32_t out[2];
        for (int f = 0; f < 2; f++) {
            uint32_t r = x;
            for (uint32_t e = q[qs * (int64_t)r + f]; e != 0; e = q[qs * (int64_t)r + f]) r -= e;
            out[f] = x - r;
        }
        reinterpret_cast<uint2*>(packed)[k] = make_uint2(out[0], out[1]);
    }
}

// Full path compression of the packed states of the nodes that receive in a
// merge round (node n * stride for n < count), between rounds (no hook runs
// concurrently).
__global__ void k_compress_nodes(uint32_t* state, int32_t V, int64_t stride, int64_t count) {
    const int64_t n = (int64_t)V * count;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        uint32_t* q = state + (size_t)(k / V) * (size_t)stride * 2 * (size_t)V;
        const uint32_t x = (uint32_t)(k % V);
        for (int f = 0; f < 2; f++) {
            const uint32_t d = q[2 * (size_t)x + f];
            if (d == 0) continue;
            uint32_t r = x - d;
            for (uint32_t e = q[2 * (size_t)r + f]; e != 0; e = q[2 * (size_t)r + f]) r -= e;
            if (r != x - d) q[2 * (size_t)x + f] = x - r;
        }
    }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

}  // namespace

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
}

// Stages of phase 0 with a full compression between them.  A state spread
// over qs > 2 words per vertex (for the stages where hooks happen) is
// compressed into the packed copy at B.packed before the last stage (mostly
// rejections), or after the only stage, and B is switched to it for the rest
// and the merges; with a single chunk (no merges) B.packed is null and the
// state keeps its layout.  Before merges the state is fully compressed again.
void launch_phase0(const Plan& P, DevBufs& B, hipStream_t s) {
    if (P.E == 0) return;
    const int64_t per = (P.E + P.M - 1) / P.M;
    const int64_t chunk_slots = P.xcd_map ? 8 * (((int64_t)P.M + 7) / 8) : P.M;
    for (size_t k = 0; k + 1 < P.stages.size(); k++) {
        const int64_t rlo = P.stages[k], rhi = std::min(P.stages[k + 1], per);
        if (rlo >= rhi) break;
        if (k > 0) {
            const int64_t n = (int64_t)P.V * P.M;
            const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)));
            if (B.qs != 2 && B.packed && k + 2 == P.stages.size()) {     // before the last stage, merges to come
                hipLaunchKernelGGL(k_compress_pack, grid, dim3(256), 0, s, (const uint32_t*)B.state, B.qs, B.packed, P.V,
                                   (int64_t)P.M);
                B.state = B.packed;
                B.qs = 2;
            } else {
                hipLaunchKernelGGL(k_compress, grid, dim3(256), 0, s, B.state, B.qs, P.V, (int64_t)P.M);
            }
        }
        // the first stage (nearly all hooks) in tiles small enough for about
        // 512 workgroups in all (few chunks: more, shorter hook chains in
        // flight); later stages (mostly rejections) in full tiles, one
        // reservation each on the chunk's counters
        int64_t tile = P.tile;
        if (k == 0) {
            if (P.tile0_max >= kBlock) tile = std::min<int64_t>(tile, P.tile0_max / kBlock * kBlock);
            while (tile > kBlock && (int64_t)P.M * ((rhi - rlo + tile - 1) / tile) < 512) tile /= 2;
        }
        const int64_t tpc = std::max<int64_t>(1, (rhi - rlo + tile - 1) / tile);
        hipLaunchKernelGGL(k_phase0, dim3((unsigned)(chunk_slots * tpc)), dim3(kBlock), 0, s, B, P.E, P.V, P.M,
                           (int32_t)tile, (int32_t)tpc, P.xcd_map, rlo, rhi);
    }
    // merges to come: a state still spread is compressed into the packed copy;
    // a packed one that only saw a single stage of hooks over chunks of at
    // least 3V/4 edges (deep trees) is compressed in place, so that the merges'
    // finds take one step (measured: dense M = 64 merges 0.54 -> 0.42 ms; with
    // smaller chunks the trees are shallow and the pass costs more than it saves)
    if (P.M > 1) {
        const int64_t n = (int64_t)P.V * P.M;
        const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)));
        if (B.qs != 2 && B.packed) {
            hipLaunchKernelGGL(k_compress_pack, grid, dim3(256), 0, s, (const uint32_t*)B.state, B.qs, B.packed, P.V,
                               (int64_t)P.M);
            B.state = B.packed;
            B.qs = 2;
        } else if (P.stages.size() == 2 && 4 * per >= 3 * (int64_t)P.V) {
            hipLaunchKernelGGL(k_compress, grid, dim3(256), 0, s, B.state, B.qs, P.V, (int64_t)P.M);
        }
    }
}

int phase0_launches(const Plan& P) {
    // mirrors launch_phase0's choices
    if (P.solo) return 2;
    if (P.lds) return 1;
    if (P.E == 0) return 0;
    const int64_t per = (P.E + P.M - 1) / P.M;
    const bool has_packed = P.qs != 2 && P.M > 1;
    bool packed_now = P.qs == 2;
    int n = 0;
    for (size_t k = 0; k + 1 < P.stages.size(); k++) {
        if (P.stages[k] >= std::min(P.stages[k + 1], per)) break;
        if (k > 0) {
            n++;   // compression between stages
            if (!packed_now && has_packed && k + 2 == P.stages.size()) packed_now = true;
        }
        n++;
    }
    if (P.M > 1) {
        if (!packed_now && has_packed) n++;
        else if (P.stages.size() == 2 && 4 * per >= 3 * (int64_t)P.V) n++;
    }
    return n;
}

int launch_merge_round(const Plan& P, const DevBufs& B, int32_t step, hipStream_t s) {
    int launches = 1;
    const int64_t merges = (P.M - step - 1) / (2 * (int64_t)step) + 1;
    int64_t maxcap = 0, total = 0;
    for (int64_t i = 0; i + step < P.M; i += 2 * (int64_t)step) {
        maxcap = std::max(maxcap, P.cap[i + step]);
        total += P.cap[i + step];
    }
    // tile sized so that the round spreads over about a thousand workgroups:
    // small tiles for the few large merges at the top of the tree, larger ones
    // (fewer reservations on each node's counters) when many merges run at once
    int64_t tile = (total + 1023) / 1024;
    tile = (tile + kBlock - 1) / kBlock * kBlock;
    tile = std::max<int64_t>(kBlock, std::min<int64_t>(tile, kTile));
    const int64_t tpm = std::max<int64_t>(1, (maxcap + tile - 1) / tile);
    // chunks of at most 2V edges (phase 0 in one stage: nearly every edge a
    // hook, and so are the first merges): after a round whose sibling
    // certificates held at least 3V/4 edges each, the receiving states carry
    // deep trees of fresh hooks; compress them so that this round's finds take
    // one step (measured: dense M = 64 / 256 / 1024 merges -12 / -13 / -9%,
    // large M = 4096 -13%; with larger chunks the merges mostly reject and the
    // pass costs more than it saves)
    if (step >= 2 && B.qs == 2 && P.stages.size() == 2) {
        int64_t prev = 0;
        for (int64_t i = 0; i + step / 2 < P.M; i += step) prev = std::max(prev, P.cap[i + step / 2]);
        if (4 * prev >= 3 * (int64_t)P.V) {
            const int64_t n = (int64_t)P.V * merges;
            hipLaunchKernelGGL(k_compress_nodes, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536))),
                               dim3(256), 0, s, B.state, P.V, (2 * (int64_t)step) >> B.shift, merges);
            launches++;
        }
    }
    hipLaunchKernelGGL(P.prem ? k_merge<true> : k_merge<false>, dim3((unsigned)(merges * tpm)), dim3(kBlock), 0, s, B,
                       P.V, P.M, step, (int32_t)tile, (int32_t)tpm);
    return launches;
}

void launch_copy_out(const Plan& P, const DevBufs& B, int32_t* d_out, int64_t out_cap, int64_t* d_counts,
                     hipStream_t s) {
    int64_t blocks = (P.cap[0] + 255) / 256;
    blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 4096));
    hipLaunchKernelGGL(k_copy_out, dim3((unsigned)blocks), dim3(256), 0, s, B, reinterpret_cast<int2*>(d_out),
                       out_cap, d_counts);
}

int32_t block_size() { return kBlock; }
int32_t tile_size() { return kTile; }

}  // namespace br
