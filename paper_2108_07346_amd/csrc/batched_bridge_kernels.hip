// Final step of the batched path on the device: the bridges of each small
// graph's certificate, one workgroup per graph, entirely in LDS.
//
// The certificate is the one the persistent batched kernel leaves in node 0's
// region of each graph (F from the front, F' from the back, graph-local ids),
// with the roots of F's trees flagged in rootw.

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace br {

namespace {

constexpr int kLimitV = 4096;                 // vertices per small graph (the batched kernel's LDS limit)
constexpr int kSplitV = 1024;                 // graphs up to this size run in smaller workgroups, several per CU

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
// per graph; buffers are reused from phase to phase.  Two instances: graphs of
// up to kSplitV vertices in 256-thread workgroups with ~39 KB of LDS (several
// per CU), larger ones in 1024-thread workgroups with ~155 KB.
constexpr uint32_t kEnd = 0xffffu;

template <int kMaxV, int kST>
struct SmallLds {
    static constexpr int kMaxA = 2 * (kMaxV - 1);   // arcs of a spanning forest of kMaxV vertices
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
template <int kST>
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
template <int kST>
__device__ void scan_u16(uint16_t* a, int n, uint32_t* wsum, uint32_t* tot) {
    const int b = threadIdx.x * 8;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) { v[j] = b + j < n ? a[b + j] : 0u; s += v[j]; }
    uint32_t ex = wg_exclusive<kST>(s, wsum, tot);
#pragma unroll
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

template <int kMaxV, int kST>
__global__ void __launch_bounds__(kST) k_small_bridges(const BatchDev B, const int32_t* list, int32_t nlist,
                                                       uint32_t* out_hdr, uint32_t* out_keys) {
    static_assert(4 * kST >= kMaxV && 8 * kST >= 2 * kMaxV, "per-thread scan widths must cover the arrays");
    constexpr int kMaxA = 2 * (kMaxV - 1);
    constexpr int kPerT = (kMaxA + kST - 1) / kST;   // arcs per thread
    extern __shared__ __align__(16) unsigned char lds_raw[];
    SmallLds<kMaxV, kST>& L = *reinterpret_cast<SmallLds<kMaxV, kST>*>(lds_raw);
    const int tid = threadIdx.x;
    for (int64_t it = blockIdx.x; it < nlist; it += gridDim.x) {
        const int64_t g = list[it];
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
#pragma unroll
            for (int j = 0; j < 8; j++) { v[j] = b + j <= (int)V ? L.head[b + j] : 0u; sm += v[j]; }
            uint32_t ex = wg_exclusive<kST>(sm, L.wsum, &L.total);
#pragma unroll
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
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t r = b + j;
                uint32_t Lr = 0;
                if (r < V && B.rootw[vb + r] == 0 && L.head[r + 1] > L.head[r]) Lr = (L.link[L.adj[L.head[r]]] >> 16) + 1;
                v[j] = Lr | ((Lr ? Lr / 2 + 1 : 0u) << 16);
                sm += v[j];
            }
            uint32_t ex = wg_exclusive<kST>(sm, L.wsum, &L.total);
#pragma unroll
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
        scan_u16<kST>(L.adj, (int)A + 1, L.wsum, &L.total);
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

int32_t small_bridges_max_v() { return kLimitV; }
int32_t small_bridges_split_v() { return kSplitV; }

void launch_small_bridges(const BatchDev& B, const int32_t* list_a, int32_t na, const int32_t* list_b, int32_t nb,
                          uint32_t* out_hdr, uint32_t* out_keys, int cus, hipStream_t s, hipStream_t s_b) {
    if (nb > 0)
        hipLaunchKernelGGL((k_small_bridges<kLimitV, 1024>), dim3((unsigned)std::min(nb, 4 * cus)), dim3(1024),
                           sizeof(SmallLds<kLimitV, 1024>), s_b, B, list_b, nb, out_hdr, out_keys);
    if (na > 0)
        hipLaunchKernelGGL((k_small_bridges<kSplitV, 256>), dim3((unsigned)std::min(na, 16 * cus)), dim3(256),
                           sizeof(SmallLds<kSplitV, 256>), s, B, list_a, na, out_hdr, out_keys);
}

int prepare_small_bridges() {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_bridges<kLimitV, 1024>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SmallLds<kLimitV, 1024>));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small_bridges<kSplitV, 256>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(SmallLds<kSplitV, 256>));
    return e == hipSuccess ? 0 : -1;
}

}  // namespace br
