/*
 * oracle/certificate.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Sequential reference of the paper's sparse-certificate construction, used by
 * the tests to check certificate properties on the CPU.  Only tests and the
 * benchmark's CPU-baseline leg use it; it shares no code with the GPU library.
 *
 * Certificate (Algorithm 2, Section IV-B): F is a spanning forest of (V, U)
 * found with a union-find over the edge list (an edge joining two different
 * trees is kept); F' is a spanning forest of (V, U - F) found the same way;
 * the certificate is S = F u F'.  Lemma 1 (Section III) bounds |S| by
 * 2(n-1).  The listing starts a DFS to visit the edges; any visiting order
 * gives a maximal spanning forest, so this reference takes the edges in list
 * order, in two passes exactly as the listing orders them (F first, then F').
 *
 * Phase tree (Section III): E is split into M sets U_0..U_{M-1} (contiguous
 * ranges [floor(iE/M), floor((i+1)E/M)) of the given list); phase 0 computes
 * X_i = Certificate(U_i); in round q = 1..ceil(log2 M), every i divisible by
 * 2^q with a partner i + 2^(q-1) < M replaces X_i by
 * Certificate(X_i u X_{i+2^(q-1)}); a missing partner leaves X_i unchanged
 * (U_{i+l} is empty for i + l >= M).  X_0 is the final certificate.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t uf_find(int64_t* par, int64_t x) {
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

/* Spanning forest of the listed edges, skipping those with skip[e] != 0.
 * Kept edges are marked in keep[] and copied to out.  Returns the count. */
static int64_t forest_pass(const int32_t* edges, int64_t E, int64_t V, const uint8_t* skip, uint8_t* keep,
                           int64_t* par, int32_t* out) {
    for (int64_t v = 0; v < V; v++) par[v] = v;
    int64_t n = 0;
    for (int64_t e = 0; e < E; e++) {
        if (skip && skip[e]) continue;
        int64_t a = uf_find(par, edges[2 * e]), b = uf_find(par, edges[2 * e + 1]);
        if (a == b) continue;
        par[a] = b;
        if (keep) keep[e] = 1;
        out[2 * n] = edges[2 * e]; out[2 * n + 1] = edges[2 * e + 1];
        n++;
    }
    return n;
}

/*
 * Certificate of edges[E][2] on V vertices.  f1 and f2 must each have room
 * for min(E, V-1) pairs.  Returns 0, -1 on bad arguments, -2 on an
 * out-of-range id, -3 if out of memory.
 */
int oracle_certificate(const int32_t* edges, int64_t E, int64_t V, int32_t* f1, int64_t* n1, int32_t* f2, int64_t* n2) {
    if (E < 0 || V < 1 || (E > 0 && (!edges || !f1 || !f2)) || !n1 || !n2) return -1;
    for (int64_t e = 0; e < E; e++)
        if (edges[2 * e] < 0 || edges[2 * e] >= V || edges[2 * e + 1] < 0 || edges[2 * e + 1] >= V) return -2;
    int64_t* par = (int64_t*)malloc(sizeof(int64_t) * (size_t)V);
    uint8_t* inF = (uint8_t*)calloc((size_t)(E > 0 ? E : 1), 1);
    if (!par || !inF) { free(par); free(inF); return -3; }
    *n1 = forest_pass(edges, E, V, NULL, inF, par, f1);      /* F  of G  = (V, U)     */
    *n2 = forest_pass(edges, E, V, inF, NULL, par, f2);      /* F' of G' = (V, U - F) */
    free(par); free(inF);
    return 0;
}

/*
 * The phase tree over M contiguous chunks.  x0 must have room for
 * min(E, 2(V-1)) pairs; the final certificate is written F first, then F'
 * (*n1 and *n2 pairs).  rounds_max[q] (q = 0..ceil(log2 M), may be NULL)
 * receives the largest certificate size after phase q.
 */
int oracle_phase_tree(const int32_t* edges, int64_t E, int64_t V, int64_t M, int32_t* x0, int64_t* n1, int64_t* n2,
                      int64_t* rounds_max) {
    if (E < 0 || V < 1 || M < 1 || (E > 0 && !edges) || !x0 || !n1 || !n2) return -1;
    int64_t cap = 2 * (V - 1);
    int32_t** X = (int32_t**)calloc((size_t)M, sizeof(int32_t*));
    int64_t* xn = (int64_t*)calloc((size_t)M, sizeof(int64_t));
    int64_t* xf = (int64_t*)calloc((size_t)M, sizeof(int64_t));     /* |F| part of X_i */
    int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(2 * cap > 0 ? 2 * cap : 1));
    int32_t* t1 = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(cap > 0 ? cap : 1));
    int32_t* t2 = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(cap > 0 ? cap : 1));
    if (!X || !xn || !xf || !buf || !t1 || !t2) { free(X); free(xn); free(xf); free(buf); free(t1); free(t2); return -3; }
    int rc = 0;
    int64_t mx = 0;
    /* phase 0 */
    for (int64_t i = 0; i < M && rc == 0; i++) {
        int64_t lo = (int64_t)(((__int128)i * E) / M), hi = (int64_t)(((__int128)(i + 1) * E) / M);
        int64_t a, b;
        rc = oracle_certificate(edges + 2 * lo, hi - lo, V, t1, &a, t2, &b);
        if (rc) break;
        X[i] = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(a + b > 0 ? a + b : 1));
        memcpy(X[i], t1, sizeof(int32_t) * 2 * (size_t)a);
        memcpy(X[i] + 2 * a, t2, sizeof(int32_t) * 2 * (size_t)b);
        xn[i] = a + b; xf[i] = a;
        if (xn[i] > mx) mx = xn[i];
    }
    if (rounds_max) rounds_max[0] = mx;
    /* merge rounds */
    int q = 0;
    for (int64_t step = 1; step < M && rc == 0; step *= 2) {
        q++;
        mx = 0;
        for (int64_t i = 0; i < M; i += 2 * step) {
            if (i + step < M) {
                int64_t j = i + step, a, b;
                memcpy(buf, X[i], sizeof(int32_t) * 2 * (size_t)xn[i]);
                memcpy(buf + 2 * xn[i], X[j], sizeof(int32_t) * 2 * (size_t)xn[j]);
                rc = oracle_certificate(buf, xn[i] + xn[j], V, t1, &a, t2, &b);
                if (rc) break;
                free(X[i]); free(X[j]); X[j] = NULL;
                X[i] = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(a + b > 0 ? a + b : 1));
                memcpy(X[i], t1, sizeof(int32_t) * 2 * (size_t)a);
                memcpy(X[i] + 2 * a, t2, sizeof(int32_t) * 2 * (size_t)b);
                xn[i] = a + b; xf[i] = a;
            }
            if (xn[i] > mx) mx = xn[i];
        }
        if (rounds_max) rounds_max[q] = mx;
    }
    if (rc == 0) {
        memcpy(x0, X[0], sizeof(int32_t) * 2 * (size_t)xn[0]);
        *n1 = xf[0]; *n2 = xn[0] - xf[0];
    }
    for (int64_t i = 0; i < M; i++) free(X[i]);
    free(X); free(xn); free(xf); free(buf); free(t1); free(t2);
    return rc;
}
