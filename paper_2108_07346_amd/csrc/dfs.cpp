// Final step of the path: the bridges of the merged certificate by the
// low-link depth-first search of Algorithm 1 (paper, Section IV-A), then the
// canonical order.  The certificate has at most 2(V-1) edges (Lemma 1), so
// this sequential step is O(V) (Section V).
//
// Readings of Algorithm 1 used here: one global discovery clock; descend
// into unvisited neighbours; skip only the edge the search arrived by (by
// edge id, so a parallel copy of it acts as a back edge); adjacency lists
// instead of a scan over all vertices; an explicit stack instead of
// recursion; a new search from every vertex not yet reached.  A tree edge
// (p, c) is a bridge iff low[c] > disc[p].
//
// Layout for a latency-bound walk: arcs are (target, edge id) pairs grouped by
// source, and each vertex's discovery time and low-link share one 8-byte
// slot, so visiting an arc touches one arc slot and one vertex slot.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace br {

void walk(const int32_t* head, const int2* arc, int32_t V, DfsScratch& S, std::vector<uint64_t>& keys);

void certificate_bridges(const int2* f1, int64_t n1, const int2* f2, int64_t n2, int32_t V, DfsScratch& S,
                         std::vector<uint64_t>& keys) {
    const int64_t m = n1 + n2;
    auto edge = [&](int64_t k) -> const int2& { return k < n1 ? f1[k] : f2[k - n1]; };
    // adjacency grouped by source (counting sort), edge ids kept for the parent test
    S.head.assign((size_t)V + 1, 0);
    for (int64_t k = 0; k < m; k++) {
        const int2 e = edge(k);
        if (e.x == e.y) continue;
        S.head[e.x + 1]++;
        S.head[e.y + 1]++;
    }
    for (int32_t v = 0; v < V; v++) S.head[v + 1] += S.head[v];
    const int64_t arcs = S.head[V];
    S.arc.resize((size_t)std::max<int64_t>(arcs, 1));
    S.fill.assign(S.head.begin(), S.head.end() - 1);
    for (int64_t k = 0; k < m; k++) {
        const int2 e = edge(k);
        if (e.x == e.y) continue;
        S.arc[S.fill[e.x]++] = make_int2(e.y, (int32_t)k);
        S.arc[S.fill[e.y]++] = make_int2(e.x, (int32_t)k);
    }
    walk(S.head.data(), S.arc.data(), V, S, keys);
}

// The search proper over an adjacency grouped by source.  Roots are taken in
// id order (vertices without arcs carry no bridge).
void walk(const int32_t* head, const int2* arc, int32_t V, DfsScratch& S, std::vector<uint64_t>& keys) {
    S.dl.assign((size_t)V, make_int2(0, 0));    // disc 0 = not reached; times start at 1
    S.st_v.resize((size_t)V);
    S.st_pe.resize((size_t)V);
    S.st_it.resize((size_t)V);
    int2* dl = S.dl.data();
    int32_t clock = 0;
    for (int32_t r = 0; r < V; r++) {
        if (dl[r].x || head[r + 1] == head[r]) continue;
        int32_t top = 0;
        S.st_v[0] = r;
        S.st_pe[0] = -1;
        S.st_it[0] = head[r];
        ++clock;
        dl[r] = make_int2(clock, clock);
        while (top >= 0) {
            const int32_t x = S.st_v[top];
            int32_t it = S.st_it[top];
            const int32_t end = head[x + 1];
            const int32_t pe = S.st_pe[top];
            int32_t lowx = dl[x].y;
            bool descended = false;
            while (it < end) {
                const int2 a = arc[it++];
                if (it < end) __builtin_prefetch(&dl[arc[it].x]);
                if (a.y == pe) continue;
                const int32_t y = a.x;
                const int32_t dy = dl[y].x;
                if (!dy) {
                    dl[x].y = lowx;
                    S.st_it[top] = it;
                    ++clock;
                    dl[y] = make_int2(clock, clock);
                    ++top;
                    S.st_v[top] = y;
                    S.st_pe[top] = a.y;
                    S.st_it[top] = head[y];
                    __builtin_prefetch(&arc[head[y]]);
                    descended = true;
                    break;
                }
                lowx = dy < lowx ? dy : lowx;
            }
            if (descended) continue;
            dl[x].y = lowx;
            // x is finished: fold its low-link into its parent and test the tree edge
            --top;
            if (top >= 0) {
                const int32_t p = S.st_v[top];
                if (lowx < dl[p].y) dl[p].y = lowx;
                if (lowx > dl[p].x) {
                    const uint32_t a = (uint32_t)std::min(p, x), b = (uint32_t)std::max(p, x);
                    keys.push_back((uint64_t)a << 32 | b);
                }
            }
        }
    }
}

// Keys are (a << 32 | b) with a < b < 2^31.  Packed into 2w bits (w = bits of
// the largest field) and sorted least-significant digit first, digits of about
// log2(n) bits; a handful of keys go through std::sort.
void canonical_sort(std::vector<uint64_t>& keys) {
    const size_t n = keys.size();
    if (n < 64) {
        std::sort(keys.begin(), keys.end());
        return;
    }
    uint32_t all = 0;
    for (const uint64_t k : keys) all |= (uint32_t)(k >> 32) | (uint32_t)k;
    const int w = all ? 32 - __builtin_clz(all) : 1;
    const uint64_t lo_mask = (uint64_t(1) << w) - 1;
    int dbits = 6;
    while (dbits < 11 && (size_t(1) << (dbits + 1)) <= n) dbits++;
    const uint32_t dmask = (1u << dbits) - 1;
    thread_local std::vector<uint64_t> tmp;
    thread_local std::vector<uint32_t> cnt;
    tmp.resize(n);
    cnt.resize(size_t(1) << dbits);
    for (size_t i = 0; i < n; i++) keys[i] = (keys[i] >> 32) << w | (keys[i] & 0xffffffffu);
    uint64_t *src = keys.data(), *dst = tmp.data();
    for (int sh = 0; sh < 2 * w; sh += dbits) {
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (size_t i = 0; i < n; i++) cnt[(src[i] >> sh) & dmask]++;
        uint32_t run = 0;
        for (uint32_t& c : cnt) {
            const uint32_t t = c;
            c = run;
            run += t;
        }
        for (size_t i = 0; i < n; i++) dst[cnt[(src[i] >> sh) & dmask]++] = src[i];
        std::swap(src, dst);
    }
    for (size_t i = 0; i < n; i++) keys[i] = (src[i] >> w) << 32 | (src[i] & lo_mask);
}


}  // namespace br

namespace br {

// Articulation points of the certificate (V, F u F'): the same low-link
// search, with the vertex test -- a non-root p separates iff some child c has
// low[c] >= disc[p], a root iff it has two or more children.  Parallel copies
// and the arriving edge need no special case here (a back edge into p only
// lowers low[c] to disc[p]).
void certificate_articulation(const int2* f1, int64_t n1, const int2* f2, int64_t n2, int32_t V, DfsScratch& S,
                              std::vector<int32_t>& out) {
    const int64_t m = n1 + n2;
    auto edge = [&](int64_t k) -> const int2& { return k < n1 ? f1[k] : f2[k - n1]; };
    S.head.assign((size_t)V + 1, 0);
    for (int64_t k = 0; k < m; k++) {
        const int2 e = edge(k);
        if (e.x == e.y) continue;
        S.head[e.x + 1]++;
        S.head[e.y + 1]++;
    }
    for (int32_t v = 0; v < V; v++) S.head[v + 1] += S.head[v];
    S.arc.resize((size_t)std::max<int32_t>(S.head[V], 1));
    S.fill.assign(S.head.begin(), S.head.end() - 1);
    for (int64_t k = 0; k < m; k++) {
        const int2 e = edge(k);
        if (e.x == e.y) continue;
        S.arc[S.fill[e.x]++] = make_int2(e.y, (int32_t)k);
        S.arc[S.fill[e.y]++] = make_int2(e.x, (int32_t)k);
    }
    S.dl.assign((size_t)V, make_int2(0, 0));    // (disc, low); disc 0 = not reached
    S.st_v.resize((size_t)V);
    S.st_it.resize((size_t)V);
    std::vector<uint8_t> cut((size_t)V, 0);
    int2* dl = S.dl.data();
    const int32_t* head = S.head.data();
    const int2* arc = S.arc.data();
    int32_t clock = 0;
    for (int32_t r = 0; r < V; r++) {
        if (dl[r].x || head[r + 1] == head[r]) continue;
        int32_t sp = 0, children = 0;
        S.st_v[0] = r;
        S.st_it[0] = head[r];
        ++clock;
        dl[r] = make_int2(clock, clock);
        while (sp >= 0) {
            const int32_t x = S.st_v[sp];
            if (S.st_it[sp] < head[x + 1]) {
                const int32_t y = arc[S.st_it[sp]++].x;
                if (!dl[y].x) {
                    ++clock;
                    dl[y] = make_int2(clock, clock);
                    if (sp == 0) children++;
                    ++sp;
                    S.st_v[sp] = y;
                    S.st_it[sp] = head[y];
                } else if (dl[y].x < dl[x].y) {
                    dl[x].y = dl[y].x;
                }
            } else {
                --sp;
                if (sp >= 0) {
                    const int32_t p = S.st_v[sp];
                    if (dl[x].y < dl[p].y) dl[p].y = dl[x].y;
                    if (sp > 0 && dl[x].y >= dl[p].x) cut[p] = 1;
                }
            }
        }
        if (children >= 2) cut[r] = 1;
    }
    out.clear();
    for (int32_t v = 0; v < V; v++)
        if (cut[v]) out.push_back(v);
}

}  // namespace br
