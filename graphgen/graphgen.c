/*
 * graphgen.c -- seeded synthetic planted-cluster multigraphs.
 *
 * This module only produces inputs.  It holds none of the bridge method's
 * arithmetic (no union-find, no DFS, no certificate) and is the one piece of
 * code that both the CPU oracle and the GPU library are fed from.
 *
 * Model (one graph):
 *   - k clusters with near-equal sizes summing to vc vertices; each cluster is
 *     an Erdos-Renyi G(s, p) over its unordered vertex pairs;
 *   - a uniformly random labelled tree on the clusters (Pruefer sequence); each
 *     tree edge joins a uniformly random vertex of each of its two clusters;
 *   - n_extra extra edges between random vertices of two distinct random
 *     clusters, resampled so that they repeat no tree edge and no other extra
 *     edge (the graph stays simple);
 *   - n_cross i.i.d. uniform edges between vertices of distinct clusters,
 *     drawn with replacement (parallel copies are kept: multigraph); with
 *     cross_block = b > 0 the clusters form blocks of b consecutive clusters,
 *     the cluster tree is a random tree inside every block plus a random tree
 *     over the blocks (each of its edges joining random clusters of the two
 *     blocks), and each cross edge joins two distinct clusters of one block;
 *     the tree edges between blocks then stay uncovered by cross edges;
 *   - n_pend pendant vertices with ids vc..vc+n_pend-1, each joined by one
 *     edge to a uniformly random cluster vertex.
 * Then (optionally) the vertex ids are relabelled by a keyed bijection of
 * [0,V), the edge list is permuted by a keyed bijection of [0,E) and every
 * pair's orientation is flipped with probability 1/2.
 *
 * Randomness: every draw is SplitMix64's output at a fixed counter of a keyed
 * stream (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014), so the bytes do not depend on the thread count
 * or the host.  Bijections are 4-round Feistel networks on the next even
 * power of two with cycle walking.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* i-th output (0-based) of SplitMix64 started from state `key`. */
static inline uint64_t rng_at(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GG_GAMMA); }
static inline uint64_t subkey(uint64_t key, uint64_t tag) { return mix64(key ^ mix64(tag * GG_GAMMA + 0x632BE59BD9B4E019ULL)); }
/* uniform integer in [0,n) by the multiply-high method */
static inline uint64_t below(uint64_t r, uint64_t n) { return (uint64_t)(((unsigned __int128)r * n) >> 64); }

/* stream tags */
enum { T_INTRA = 1, T_TREE = 2, T_TREE_END = 3, T_EXTRA = 4, T_PEND = 5, T_CROSS = 6,
       T_RELABEL = 7, T_SHUFFLE = 8, T_ORIENT = 9, T_BLOCK_TREE = 10 };

/* ---- keyed bijection of [0,n) ------------------------------------------- */
typedef struct { uint64_t n, key; int half; uint64_t mask; } perm_t;

static void perm_init(perm_t* P, uint64_t n, uint64_t key) {
    int b = 2;
    while (b < 64 && ((uint64_t)1 << b) < n) b += 2;
    P->n = n; P->key = key; P->half = b / 2; P->mask = ((uint64_t)1 << P->half) - 1;
}
static inline uint64_t feistel(const perm_t* P, uint64_t x) {
    uint64_t L = x >> P->half, R = x & P->mask;
    for (int r = 0; r < 4; r++) {
        uint64_t F = mix64(P->key + (uint64_t)r * GG_GAMMA + R) & P->mask;
        uint64_t t = R; R = L ^ F; L = t;
    }
    return (L << P->half) | R;
}
static inline uint64_t perm_apply(const perm_t* P, uint64_t x) {
    if (P->n <= 1) return 0;
    do { x = feistel(P, x); } while (x >= P->n);
    return x;
}

/* ---- graph description ---------------------------------------------------- */
typedef struct gg_graph {
    uint64_t key;
    int32_t k, cross_block;
    int64_t vc, n_pend, n_extra, n_cross;
    double p;
    int relabel, shuffle;
    /* derived */
    int64_t V, E, n_intra;
    int64_t* cl_off;      /* [k+1] first vertex of each cluster */
    int64_t* cnt_off;     /* [k+1] prefix of intra edge counts */
    int32_t* tree;        /* [(k-1)*2] pre-relabel endpoints */
    int32_t* extra;       /* [n_extra*2] */
    uint64_t thr;         /* Bernoulli threshold on 53-bit draws */
    perm_t relab;
} gg_graph;

static int gg_threads(void) {
    const char* s = getenv("GG_THREADS");
    long n = s ? atol(s) : sysconf(_SC_NPROCESSORS_ONLN);
    if (n < 1) n = 1;
    if (n > 16) n = 16;
    return (int)n;
}

typedef struct { void (*fn)(void*, int64_t); void* arg; int64_t ntask; int64_t next; pthread_mutex_t mu; } pool_t;
static void* pool_worker(void* a) {
    pool_t* P = (pool_t*)a;
    for (;;) {
        pthread_mutex_lock(&P->mu);
        int64_t t = P->next++;
        pthread_mutex_unlock(&P->mu);
        if (t >= P->ntask) break;
        P->fn(P->arg, t);
    }
    return NULL;
}
/* run fn(arg, t) for t in [0,ntask) on up to nthr threads; results must not depend on the schedule */
static void run_tasks(void (*fn)(void*, int64_t), void* arg, int64_t ntask, int nthr) {
    if (nthr > ntask) nthr = (int)ntask;
    if (nthr <= 1) { for (int64_t t = 0; t < ntask; t++) fn(arg, t); return; }
    pool_t P; P.fn = fn; P.arg = arg; P.ntask = ntask; P.next = 0;
    pthread_mutex_init(&P.mu, NULL);
    pthread_t th[16];
    for (int i = 0; i < nthr; i++) pthread_create(&th[i], NULL, pool_worker, &P);
    for (int i = 0; i < nthr; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&P.mu);
}

static inline int64_t cl_size(const gg_graph* G, int32_t j) { return G->cl_off[j + 1] - G->cl_off[j]; }
static inline int32_t cl_of(const gg_graph* G, int64_t v) {
    int32_t lo = 0, hi = G->k - 1;
    while (lo < hi) { int32_t mid = (lo + hi + 1) / 2; if (G->cl_off[mid] <= v) lo = mid; else hi = mid - 1; }
    return lo;
}

/* intra-cluster pairs of cluster j, in (a<b) lexicographic order; write==NULL counts */
static int64_t intra_pass(const gg_graph* G, int32_t j, int32_t* out) {
    uint64_t key = subkey(subkey(G->key, T_INTRA), (uint64_t)j);
    int64_t s = cl_size(G, j), base = G->cl_off[j], c = 0;
    uint64_t t = 0;
    for (int64_t a = 0; a < s; a++)
        for (int64_t b = a + 1; b < s; b++, t++)
            if ((rng_at(key, t) >> 11) < G->thr) {
                if (out) { out[2 * c] = (int32_t)(base + a); out[2 * c + 1] = (int32_t)(base + b); }
                c++;
            }
    return c;
}
static void task_count(void* a, int64_t j) { gg_graph* G = (gg_graph*)a; G->cnt_off[j + 1] = intra_pass(G, (int32_t)j, NULL); }

static int has_pair(const int32_t* e, int64_t n, int32_t a, int32_t b) {
    for (int64_t i = 0; i < n; i++)
        if ((e[2 * i] == a && e[2 * i + 1] == b) || (e[2 * i] == b && e[2 * i + 1] == a)) return 1;
    return 0;
}

void gg_free(gg_graph* G) {
    if (!G) return;
    free(G->cl_off); free(G->cnt_off); free(G->tree); free(G->extra); free(G);
}

/* A uniformly random labelled tree on n nodes (Pruefer sequence of length
 * n-2 drawn from stream tk at counters base.., decoded in linear time): its
 * n-1 edges as node pairs into ce[2(n-1)]. */
static void pruefer_tree(uint64_t tk, uint64_t base, int32_t n, int32_t* ce) {
    if (n < 2) return;
    int32_t* seq = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 2 ? n - 2 : 1));
    int32_t* deg = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t i = 0; i < n; i++) deg[i] = 1;
    for (int32_t i = 0; i < n - 2; i++) { seq[i] = (int32_t)below(rng_at(tk, base + (uint64_t)i), (uint64_t)n); deg[seq[i]]++; }
    int32_t ptr = 0; while (deg[ptr] != 1) ptr++;
    int32_t leaf = ptr, ne = 0;
    for (int32_t i = 0; i < n - 2; i++) {
        int32_t x = seq[i];
        ce[2 * ne] = leaf; ce[2 * ne + 1] = x; ne++;
        deg[x]--;
        if (deg[x] == 1 && x < ptr) leaf = x;
        else { ptr++; while (deg[ptr] != 1) ptr++; leaf = ptr; }
    }
    ce[2 * ne] = leaf; ce[2 * ne + 1] = n - 1;
    free(seq); free(deg);
}

/*
 * Plan a graph: draws the cluster tree and extra edges, counts the intra
 * edges.  Returns NULL on bad parameters.  gg_V / gg_E then give the sizes.
 */
gg_graph* gg_plan(uint64_t seed, int32_t k, int64_t vc, double p, int64_t n_extra, int64_t n_cross,
                  int64_t n_pend, int relabel, int shuffle, int32_t cross_block) {
    if (k < 1 || vc < k || p < 0.0 || p > 1.0 || n_extra < 0 || n_cross < 0 || n_pend < 0) return NULL;
    if (cross_block < 0 || cross_block == 1 || (cross_block > 0 && k % cross_block != 0)) return NULL;
    if (vc + n_pend > 2147483647LL) return NULL;
    if (k < 2 && (n_extra > 0 || n_cross > 0)) return NULL;
    gg_graph* G = (gg_graph*)calloc(1, sizeof(gg_graph));
    G->key = mix64(seed ^ 0x5EEDBA5E5EEDBA5EULL);
    G->k = k; G->vc = vc; G->p = p; G->n_extra = n_extra; G->n_cross = n_cross; G->n_pend = n_pend;
    G->relabel = relabel; G->shuffle = shuffle; G->cross_block = cross_block;
    G->V = vc + n_pend;
    G->thr = (p >= 1.0) ? ((uint64_t)1 << 53) : (uint64_t)(p * 9007199254740992.0);
    G->cl_off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k + 1));
    G->cnt_off = (int64_t*)calloc((size_t)(k + 1), sizeof(int64_t));
    G->cl_off[0] = 0;
    for (int32_t j = 0; j < k; j++) G->cl_off[j + 1] = G->cl_off[j] + vc / k + (j < vc % k ? 1 : 0);
    /* a simple graph cannot hold more extra edges than there are inter-cluster pairs */
    {
        double inter = 0.0;
        for (int32_t j = 0; j < k; j++) inter += (double)cl_size(G, j) * (double)(vc - cl_size(G, j));
        inter *= 0.5;
        if ((double)(k - 1 + n_extra) > inter) { gg_free(G); return NULL; }
    }
    run_tasks(task_count, G, k, vc > 4096 ? gg_threads() : 1);
    for (int32_t j = 0; j < k; j++) G->cnt_off[j + 1] += G->cnt_off[j];
    G->n_intra = G->cnt_off[k];

    /* cluster tree: Pruefer sequence of length k-2, decoded in linear time;
       with blocks, a tree inside each block (counters after the block's
       first) and a tree over the blocks (a separate stream) */
    G->tree = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(k > 1 ? k - 1 : 1));
    if (k >= 2) {
        uint64_t tk = subkey(G->key, T_TREE);
        int32_t* ce = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(k - 1));
        int32_t ne = 0;
        if (cross_block == 0) {
            pruefer_tree(tk, 0, k, ce);
            ne = k - 1;
        } else {
            const int32_t b = cross_block, nb = k / b;
            int32_t* be = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(b > nb ? b : nb));
            for (int32_t t = 0; t < nb; t++) {
                pruefer_tree(tk, (uint64_t)t * (uint64_t)b, b, be);
                for (int32_t i = 0; i < b - 1; i++, ne++) { ce[2 * ne] = t * b + be[2 * i]; ce[2 * ne + 1] = t * b + be[2 * i + 1]; }
            }
            uint64_t bk = subkey(G->key, T_BLOCK_TREE);
            pruefer_tree(bk, 0, nb, be);
            for (int32_t i = 0; i + 1 < nb; i++, ne++) {
                ce[2 * ne] = be[2 * i] * b + (int32_t)below(rng_at(bk, (uint64_t)k + 2 * (uint64_t)i), (uint64_t)b);
                ce[2 * ne + 1] = be[2 * i + 1] * b + (int32_t)below(rng_at(bk, (uint64_t)k + 2 * (uint64_t)i + 1), (uint64_t)b);
            }
            free(be);
        }
        uint64_t ek = subkey(G->key, T_TREE_END);
        for (int32_t i = 0; i < ne; i++) {
            int32_t ca = ce[2 * i], cb = ce[2 * i + 1];
            G->tree[2 * i] = (int32_t)(G->cl_off[ca] + (int64_t)below(rng_at(ek, 2 * (uint64_t)i), (uint64_t)cl_size(G, ca)));
            G->tree[2 * i + 1] = (int32_t)(G->cl_off[cb] + (int64_t)below(rng_at(ek, 2 * (uint64_t)i + 1), (uint64_t)cl_size(G, cb)));
        }
        free(ce);
    }
    /* extra inter-cluster edges, resampled on repeats (simple graph) */
    G->extra = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(n_extra > 0 ? n_extra : 1));
    {
        uint64_t xk = subkey(G->key, T_EXTRA), ctr = 0;
        for (int64_t i = 0; i < n_extra; i++) {
            for (;;) {
                int32_t ca = (int32_t)below(rng_at(xk, ctr++), (uint64_t)k);
                int32_t cb = (int32_t)below(rng_at(xk, ctr++), (uint64_t)(k - 1));
                if (cb >= ca) cb++;
                int32_t a = (int32_t)(G->cl_off[ca] + (int64_t)below(rng_at(xk, ctr++), (uint64_t)cl_size(G, ca)));
                int32_t b = (int32_t)(G->cl_off[cb] + (int64_t)below(rng_at(xk, ctr++), (uint64_t)cl_size(G, cb)));
                if (has_pair(G->tree, k - 1, a, b) || has_pair(G->extra, i, a, b)) continue;
                G->extra[2 * i] = a; G->extra[2 * i + 1] = b;
                break;
            }
        }
    }
    G->E = G->n_intra + (k - 1) + n_extra + n_pend + n_cross;
    perm_init(&G->relab, (uint64_t)G->V, subkey(G->key, T_RELABEL));
    return G;
}

int64_t gg_V(const gg_graph* G) { return G->V; }
int64_t gg_E(const gg_graph* G) { return G->E; }
int64_t gg_n_intra(const gg_graph* G) { return G->n_intra; }

static inline int32_t relabel_v(const gg_graph* G, int32_t v) {
    return G->relabel ? (int32_t)perm_apply(&G->relab, (uint64_t)v) : v;
}

/* planted pieces after relabelling: tree edges [k-1][2], extra [n_extra][2], pendant edges [n_pend][2] */
void gg_planted(const gg_graph* G, int32_t* tree, int32_t* extra, int32_t* pend) {
    for (int32_t i = 0; i + 1 < G->k; i++) { tree[2 * i] = relabel_v(G, G->tree[2 * i]); tree[2 * i + 1] = relabel_v(G, G->tree[2 * i + 1]); }
    for (int64_t i = 0; i < G->n_extra; i++) { extra[2 * i] = relabel_v(G, G->extra[2 * i]); extra[2 * i + 1] = relabel_v(G, G->extra[2 * i + 1]); }
    uint64_t pk = subkey(G->key, T_PEND);
    for (int64_t i = 0; i < G->n_pend; i++) {
        pend[2 * i] = relabel_v(G, (int32_t)(G->vc + i));
        pend[2 * i + 1] = relabel_v(G, (int32_t)below(rng_at(pk, (uint64_t)i), (uint64_t)G->vc));
    }
}

/* ---- fill ------------------------------------------------------------------ */
typedef struct { gg_graph* G; int32_t* items; int32_t* out; perm_t sh; uint64_t okey; int64_t blk; int32_t* rl; } fill_t;

static void task_intra(void* a, int64_t j) {
    fill_t* F = (fill_t*)a;
    intra_pass(F->G, (int32_t)j, F->items + 2 * F->G->cnt_off[j]);
}
static void task_cross(void* a, int64_t t) {
    fill_t* F = (fill_t*)a; const gg_graph* G = F->G;
    uint64_t ck = subkey(G->key, T_CROSS);
    int64_t lo = t * F->blk, hi = lo + F->blk; if (hi > G->n_cross) hi = G->n_cross;
    int32_t* dst = F->items + 2 * (G->n_intra + (G->k - 1) + G->n_extra + G->n_pend);
    for (int64_t i = lo; i < hi; i++) {
        int64_t u = (int64_t)below(rng_at(ck, 2 * (uint64_t)i), (uint64_t)G->vc);
        int32_t cu = cl_of(G, u);
        int64_t v;
        if (G->cross_block == 0) {
            v = (int64_t)below(rng_at(ck, 2 * (uint64_t)i + 1), (uint64_t)(G->vc - cl_size(G, cu)));
            if (v >= G->cl_off[cu]) v += cl_size(G, cu);
        } else {       /* a vertex of another cluster of u's block */
            const int32_t b0 = cu / G->cross_block * G->cross_block;
            const int64_t lo_v = G->cl_off[b0], hi_v = G->cl_off[b0 + G->cross_block];
            v = lo_v + (int64_t)below(rng_at(ck, 2 * (uint64_t)i + 1), (uint64_t)(hi_v - lo_v - cl_size(G, cu)));
            if (v >= G->cl_off[cu]) v += cl_size(G, cu);
        }
        dst[2 * i] = (int32_t)u; dst[2 * i + 1] = (int32_t)v;
    }
}
static void task_place(void* a, int64_t t) {
    fill_t* F = (fill_t*)a; const gg_graph* G = F->G;
    int64_t lo = t * F->blk, hi = lo + F->blk; if (hi > G->E) hi = G->E;
    for (int64_t i = lo; i < hi; i++) {
        uint64_t src = G->shuffle ? perm_apply(&F->sh, (uint64_t)i) : (uint64_t)i;
        int32_t u = F->items[2 * src], v = F->items[2 * src + 1];
        if (F->rl) { u = F->rl[u]; v = F->rl[v]; }
        if (G->shuffle && (rng_at(F->okey, (uint64_t)i) & 1)) { int32_t x = u; u = v; v = x; }
        F->out[2 * i] = u; F->out[2 * i + 1] = v;
    }
}

/* Write the E edges as int32 pairs into out[E][2].  Returns 0, or -1 if out of memory. */
int gg_fill(gg_graph* G, int32_t* out) {
    int32_t* items = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(G->E > 0 ? G->E : 1));
    if (!items) return -1;
    int nthr = G->E > (1 << 20) ? gg_threads() : 1;
    fill_t F; F.G = G; F.items = items; F.out = out; F.blk = 1 << 20;
    perm_init(&F.sh, (uint64_t)G->E, subkey(G->key, T_SHUFFLE));
    F.okey = subkey(G->key, T_ORIENT);
    run_tasks(task_intra, &F, G->k, nthr);
    int64_t o = G->n_intra;
    for (int32_t i = 0; i + 1 < G->k; i++, o++) { items[2 * o] = G->tree[2 * i]; items[2 * o + 1] = G->tree[2 * i + 1]; }
    for (int64_t i = 0; i < G->n_extra; i++, o++) { items[2 * o] = G->extra[2 * i]; items[2 * o + 1] = G->extra[2 * i + 1]; }
    uint64_t pk = subkey(G->key, T_PEND);
    for (int64_t i = 0; i < G->n_pend; i++, o++) {
        items[2 * o] = (int32_t)(G->vc + i);
        items[2 * o + 1] = (int32_t)below(rng_at(pk, (uint64_t)i), (uint64_t)G->vc);
    }
    if (G->n_cross > 0) run_tasks(task_cross, &F, (G->n_cross + F.blk - 1) / F.blk, nthr);
    F.rl = NULL;
    if (G->relabel) {
        F.rl = (int32_t*)malloc(sizeof(int32_t) * (size_t)G->V);
        if (!F.rl) { free(items); return -1; }
        for (int64_t v = 0; v < G->V; v++) F.rl[v] = (int32_t)perm_apply(&G->relab, (uint64_t)v);
    }
    run_tasks(task_place, &F, (G->E + F.blk - 1) / F.blk, nthr);
    free(F.rl);
    free(items);
    return 0;
}

/* uniform double in [0,1) from a 53-bit draw: shared by the Python parameter samplers */
double gg_unit(uint64_t seed, uint64_t tag, uint64_t i) {
    return (double)(rng_at(subkey(mix64(seed ^ 0x5EEDBA5E5EEDBA5EULL), tag), i) >> 11) * (1.0 / 9007199254740992.0);
}

/* cluster index of every (relabelled) vertex; -1 for pendant vertices */
void gg_cluster_of(const gg_graph* G, int32_t* out) {
    for (int32_t j = 0; j < G->k; j++)
        for (int64_t v = G->cl_off[j]; v < G->cl_off[j + 1]; v++) out[relabel_v(G, (int32_t)v)] = j;
    for (int64_t i = 0; i < G->n_pend; i++) out[relabel_v(G, (int32_t)(G->vc + i))] = -1;
}
