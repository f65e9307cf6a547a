/*
 * oracle/tarjan.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain CPU oracle for the bridge set of a graph.  Only tests, the smoke
 * check and the benchmark's CPU-baseline leg load this file's library; the
 * product library never links or calls it, and it shares no code with it.
 *
 * What it computes (paper, Section I): a bridge is an edge whose removal
 * increases the number of connected components.  How: the sequential low-link
 * depth-first search the paper gives as Algorithm 1 (Section IV-A), run on the
 * whole input graph, with these readings of that listing:
 *   - the time counter is global, starts at 0 once and advances at every
 *     discovery;
 *   - the tree-edge branch is taken when the neighbour has NOT been visited;
 *   - the parent is skipped by edge id, not by vertex, so that a doubled edge
 *     counts as a back edge (multigraph input);
 *   - neighbours come from adjacency lists, not a scan of all vertices
 *     (the O(V+E) bound of Section V);
 *   - every unvisited vertex starts a new search (disconnected input);
 *   - recursion is replaced by an explicit stack.
 * A tree edge (p, c) is a bridge iff low[c] > disc[p].  Self-loops are
 * dropped (they never disconnect anything).  Output: (min, max) pairs sorted
 * ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/*
 * edges: int32 [E][2], ids in [0, V).  out: room for cap pairs.
 * Returns 0 on success with *n_out = number of bridges (pairs written only if
 * *n_out <= cap), -1 on bad arguments, -2 if an id is out of range,
 * -3 if out of memory.
 */
int oracle_bridges(const int32_t* edges, int64_t E, int64_t V, int32_t* out, int64_t cap, int64_t* n_out) {
    if (E < 0 || V < 0 || (E > 0 && !edges) || !n_out || E > 4294967294LL || V > 2147483647LL) return -1;
    for (int64_t e = 0; e < E; e++)
        if (edges[2 * e] < 0 || edges[2 * e] >= V || edges[2 * e + 1] < 0 || edges[2 * e + 1] >= V) return -2;
    int64_t* off = (int64_t*)calloc((size_t)V + 1, sizeof(int64_t));
    if (!off) return -3;
    for (int64_t e = 0; e < E; e++) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a == b) continue;
        off[a + 1]++; off[b + 1]++;
    }
    for (int64_t v = 0; v < V; v++) off[v + 1] += off[v];
    int64_t A = off[V];
    int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(A > 0 ? A : 1));
    uint32_t* eid = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(A > 0 ? A : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V > 0 ? V : 1));
    int32_t* disc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    int32_t* low = (int32_t*)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    int32_t* st_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
    int64_t* st_pe = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V > 0 ? V : 1));
    int64_t* st_it = (int64_t*)malloc(sizeof(int64_t) * (size_t)(V > 0 ? V : 1));
    uint64_t* br = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(V > 0 ? V : 1));
    if (!nbr || !eid || !fill || !disc || !low || !st_v || !st_pe || !st_it || !br) {
        free(off); free(nbr); free(eid); free(fill); free(disc); free(low); free(st_v); free(st_pe); free(st_it); free(br);
        return -3;
    }
    memcpy(fill, off, sizeof(int64_t) * (size_t)V);
    for (int64_t e = 0; e < E; e++) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a == b) continue;
        nbr[fill[a]] = b; eid[fill[a]++] = (uint32_t)e;
        nbr[fill[b]] = a; eid[fill[b]++] = (uint32_t)e;
    }
    for (int64_t v = 0; v < V; v++) disc[v] = -1;

    int32_t t = 0;
    int64_t nb = 0;
    for (int64_t s = 0; s < V; s++) {
        if (disc[s] != -1) continue;
        int64_t sp = 0;
        st_v[0] = (int32_t)s; st_pe[0] = -1; st_it[0] = off[s];
        disc[s] = low[s] = t++;
        while (sp >= 0) {
            int32_t x = st_v[sp];
            if (st_it[sp] < off[x + 1]) {
                int64_t a = st_it[sp]++;
                int32_t y = nbr[a];
                if ((int64_t)eid[a] == st_pe[sp]) continue;        /* the edge we came in by */
                if (disc[y] == -1) {                                /* tree edge: descend */
                    disc[y] = low[y] = t++;
                    sp++;
                    st_v[sp] = y; st_pe[sp] = (int64_t)eid[a]; st_it[sp] = off[y];
                } else if (disc[y] < low[x]) {                      /* back edge */
                    low[x] = disc[y];
                }
            } else {                                                /* x finished: return to parent */
                sp--;
                if (sp >= 0) {
                    int32_t p = st_v[sp];
                    if (low[x] < low[p]) low[p] = low[x];
                    if (low[x] > disc[p]) {
                        uint64_t a = (uint64_t)(p < x ? p : x), b = (uint64_t)(p < x ? x : p);
                        br[nb++] = (a << 32) | b;
                    }
                }
            }
        }
    }
    qsort(br, (size_t)nb, sizeof(uint64_t), cmp_u64);
    *n_out = nb;
    if (out && nb <= cap)
        for (int64_t i = 0; i < nb; i++) { out[2 * i] = (int32_t)(br[i] >> 32); out[2 * i + 1] = (int32_t)(br[i] & 0xffffffffu); }
    free(off); free(nbr); free(eid); free(fill); free(disc); free(low); free(st_v); free(st_pe); free(st_it); free(br);
    return 0;
}
