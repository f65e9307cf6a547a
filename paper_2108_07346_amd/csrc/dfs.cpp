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
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace br {

void certificate_bridges(const int2* f1, int64_t n1, const int2* f2, int64_t n2, int32_t V, DfsScratch& S,
                         std::vector<uint64_t>& keys) {
    const int64_t m = n1 + n2;
    auto edge = [&](int64_t k) -> const int2& { return k < n1 ? f1[k] : f2[k - n1]; };
    // adjacency (CSR) with edge ids; heads are int32: m <= 2(V-1) < 2^32
    S.head.assign((size_t)V + 1, 0);
    for (int64_t k = 0; k < m; k++) {
        const int2 e = edge(k);
        if (e.x == e.y) continue;
        S.head[e.x + 1]++;
        S.head[e.y + 1]++;
    }
    for (int32_t v = 0; v < V; v++) S.head[v + 1] += S.head[v];
    const int64_t arcs = S.head[V];
    S.adj_to.resize((size_t)std::max<int64_t>(arcs, 1));
    S.adj_id.resize((size_t)std::max<int64_t>(arcs, 1));
    S.st_it.assign(S.head.begin(), S.head.end() - 1);   // fill cursors, reused as DFS cursors below
    for (int64_t k = 0; k < m; k++) {
        const int2 e = edge(k);
        if (e.x == e.y) continue;
        int32_t a = S.st_it[e.x]++;
        S.adj_to[a] = e.y;
        S.adj_id[a] = (int32_t)k;
        a = S.st_it[e.y]++;
        S.adj_to[a] = e.x;
        S.adj_id[a] = (int32_t)k;
    }
    S.disc.assign((size_t)V, 0);    // 0 = not reached; times start at 1
    S.low.resize((size_t)V);
    S.st_v.resize((size_t)V);
    S.st_pe.resize((size_t)V);
    S.st_it.resize((size_t)V);
    int32_t clock = 0;
    // roots: endpoints in certificate order (vertices without certificate
    // edges are isolated in the certificate and carry no bridge)
    for (int64_t k = 0; k < m; k++) {
        const int32_t r = edge(k).x;
        if (S.disc[r]) continue;
        int32_t top = 0;
        S.st_v[0] = r;
        S.st_pe[0] = -1;
        S.st_it[0] = S.head[r];
        S.disc[r] = S.low[r] = ++clock;
        while (top >= 0) {
            const int32_t x = S.st_v[top];
            int32_t& it = S.st_it[top];
            const int32_t end = S.head[x + 1];
            bool descended = false;
            while (it < end) {
                const int32_t a = it++;
                if (S.adj_id[a] == S.st_pe[top]) continue;
                const int32_t y = S.adj_to[a];
                if (!S.disc[y]) {
                    S.disc[y] = S.low[y] = ++clock;
                    ++top;
                    S.st_v[top] = y;
                    S.st_pe[top] = S.adj_id[a];
                    S.st_it[top] = S.head[y];
                    descended = true;
                    break;
                }
                if (S.disc[y] < S.low[x]) S.low[x] = S.disc[y];
            }
            if (descended) continue;
            // x is finished: fold its low-link into its parent and test the tree edge
            --top;
            if (top >= 0) {
                const int32_t p = S.st_v[top];
                if (S.low[x] < S.low[p]) S.low[p] = S.low[x];
                if (S.low[x] > S.disc[p]) {
                    const uint32_t a = (uint32_t)std::min(p, x), b = (uint32_t)std::max(p, x);
                    keys.push_back((uint64_t)a << 32 | b);
                }
            }
        }
    }
}

void canonical_sort(std::vector<uint64_t>& keys) { std::sort(keys.begin(), keys.end()); }

}  // namespace br
