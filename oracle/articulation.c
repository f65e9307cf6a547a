/*
 * oracle/articulation.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain CPU oracle for the "failure points" the paper's abstract promises:
 * the articulation points of a graph, i.e. the vertices whose removal (with
 * their edges) increases the number of connected components -- the vertex
 * counterpart of the bridge definition of Section I.  Only tests, the smoke
 * check and the benchmark's CPU-baseline leg load this file's library; the
 * product library never links or calls it, and it shares no code with it.
 *
 * How: the sequential low-link depth-first search (the one Algorithm 1 of
 * Section IV-A runs for bridges, with the same readings: a global discovery
 * clock, "not visited" opening the tree branch, adjacency lists, every
 * unvisited vertex starting a new search, an explicit stack) on the whole
 * input graph.  The vertex test differs from the edge test in two places:
 *   - a non-root vertex p is a cut vertex iff some child c in the search
 *     tree has low[c] >= disc[p] (no back edge from c's subtree climbs above
 *     p), where Algorithm 1's bridge test is the strict low[c] > disc[p];
 *   - a search root is a cut vertex iff it has at least two children.
 * Parallel edges change nothing for vertices (a back edge into p still gives
 * low[c] = disc[p]), so the parent edge need not be skipped; self-loops are
 * dropped.  Output: vertex ids ascending.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * edges: int32 [E][2], ids in [0, V).  out: room for cap vertex ids.
 * Returns 0 with *n_out = number of articulation points (ids written only if
 * *n_out <= cap), -1 on bad arguments, -2 if an id is out of range, -3 if out
 * of memory.
 */
int oracle_articulation_points(const int32_t* edges, int64_t E, int64_t V, int32_t* out, int64_t cap,
                               int64_t* n_out) {
    if (E < 0 || V < 0 || (E > 0 && !edges) || !n_out || V > 2147483647LL) return -1;
    for (int64_t e = 0; e < E; e++)
        if (edges[2 * e] < 0 || edges[2 * e] >= V || edges[2 * e + 1] < 0 || edges[2 * e + 1] >= V) return -2;
    const size_t nv = (size_t)(V > 0 ? V : 1);
    int64_t* off = (int64_t*)calloc((size_t)V + 1, sizeof(int64_t));
    if (!off) return -3;
    for (int64_t e = 0; e < E; e++) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a == b) continue;
        off[a + 1]++;
        off[b + 1]++;
    }
    for (int64_t v = 0; v < V; v++) off[v + 1] += off[v];
    const int64_t A = off[V];
    int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(A > 0 ? A : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * nv);
    int32_t* disc = (int32_t*)malloc(sizeof(int32_t) * nv);
    int32_t* low = (int32_t*)malloc(sizeof(int32_t) * nv);
    int32_t* st_v = (int32_t*)malloc(sizeof(int32_t) * nv);
    int64_t* st_it = (int64_t*)malloc(sizeof(int64_t) * nv);
    uint8_t* cut = (uint8_t*)calloc(nv, 1);
    if (!nbr || !fill || !disc || !low || !st_v || !st_it || !cut) {
        free(off); free(nbr); free(fill); free(disc); free(low); free(st_v); free(st_it); free(cut);
        return -3;
    }
    memcpy(fill, off, sizeof(int64_t) * (size_t)V);
    for (int64_t e = 0; e < E; e++) {
        int32_t a = edges[2 * e], b = edges[2 * e + 1];
        if (a == b) continue;
        nbr[fill[a]++] = b;
        nbr[fill[b]++] = a;
    }
    for (int64_t v = 0; v < V; v++) disc[v] = -1;

    int32_t t = 0;
    for (int64_t s = 0; s < V; s++) {
        if (disc[s] != -1) continue;
        int64_t sp = 0, root_children = 0;
        st_v[0] = (int32_t)s;
        st_it[0] = off[s];
        disc[s] = low[s] = t++;
        while (sp >= 0) {
            const int32_t x = st_v[sp];
            if (st_it[sp] < off[x + 1]) {
                const int32_t y = nbr[st_it[sp]++];
                if (disc[y] == -1) {                       /* tree edge: descend */
                    disc[y] = low[y] = t++;
                    if (sp == 0) root_children++;
                    sp++;
                    st_v[sp] = y;
                    st_it[sp] = off[y];
                } else if (disc[y] < low[x]) {             /* back edge (or the parent) */
                    low[x] = disc[y];
                }
            } else {                                       /* x finished: return to parent */
                sp--;
                if (sp >= 0) {
                    const int32_t p = st_v[sp];
                    if (low[x] < low[p]) low[p] = low[x];
                    if (sp > 0 && low[x] >= disc[p]) cut[p] = 1;
                }
            }
        }
        if (root_children >= 2) cut[s] = 1;
    }
    int64_t n = 0;
    for (int64_t v = 0; v < V; v++) n += cut[v];
    *n_out = n;
    if (out && n <= cap) {
        int64_t k = 0;
        for (int64_t v = 0; v < V; v++)
            if (cut[v]) out[k++] = (int32_t)v;
    }
    free(off); free(nbr); free(fill); free(disc); free(low); free(st_v); free(st_it); free(cut);
    return 0;
}
