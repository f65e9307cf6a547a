/*
 * bridges.h -- C ABI of libbridges: bridges of a multigraph through sparse
 * 2-edge-connectivity certificates, on one AMD Instinct MI355X (gfx950).
 *
 * Method (Kumar & Singh, "An Efficient Parallel Algorithm for finding Bridges
 * in a Dense Graph"):
 *   - a bridge is an edge whose removal increases the number of connected
 *     components (Section I);
 *   - the edge list is split into M sets; each set's certificate is a spanning
 *     forest F plus a spanning forest F' of the remaining edges
 *     (Algorithm 2, Section IV-B), at most 2(V-1) edges (Lemma 1, Section III);
 *   - the M certificates are merged pairwise in ceil(log2 M) rounds, each merge
 *     being the certificate of the union of two certificates (Section III);
 *   - the bridges of the final certificate are the bridges of the input; they
 *     are found on the GPU by rooting the certificate's forest and testing
 *     every tree edge's subtree (the low-link test of Algorithm 1, Section
 *     IV-A, made parallel as Section VII suggests), or by Algorithm 1's
 *     depth-first search itself on the host (br_set_final_step).
 *
 * Conventions for every entry point
 *   - Vertex ids are int32 in [0, V) with 1 <= V <= 2^31 - 1 for the
 *     certificate calls (br_cert_build, br_cert_merge); the calls that run a
 *     final step on the certificate (br_bridges_find, br_two_edge_components,
 *     br_articulation_points, br_certificate_bridges) take 1 <= V <= 2^29:
 *     they count the 2(V-1) arcs of the certificate forest's tours in 30-bit
 *     fields.  A larger V is BR_EINVAL before any device work.
 *   - An edge list is int32 [E][2] (array of pairs, 8 bytes per edge), each
 *     undirected edge listed once in either orientation.  Self-loops are
 *     accepted and never bridges; parallel edges are accepted (multigraph:
 *     an edge with a parallel copy is never a bridge).
 *   - Edge counts, capacities and offsets are int64.
 *   - "d_" pointers are device memory on the context's device, "h_" pointers
 *     are host memory.  The caller owns every buffer it passes; the library
 *     never frees or retains them past the call (the server copies what it
 *     keeps).  The library owns its workspace.
 *   - A stream argument is a hipStream_t passed as void* (NULL = the null
 *     stream).  Calls marked "asynchronous" enqueue work on it and return;
 *     calls marked "synchronous" return after the result is on the host.
 *     Every call on a context is ordered after the device work of the
 *     previous call on that context, whatever streams the two use (they
 *     share the context's workspace); the caller orders its own buffers
 *     (inputs ready before the call, outputs read after the stream).  Device
 *     inputs are read on the stream passed in.
 *   - Return value: BR_OK or a negative BR_E* code; br_last_error() then
 *     gives a message (thread-local).  Nothing is thrown across the ABI.
 *   - A context is used by one host thread at a time.
 *   - Results are canonical: bridges as (min, max) pairs sorted ascending.
 */
#ifndef PAPER_2108_07346_BRIDGES_H
#define PAPER_2108_07346_BRIDGES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BR_OK 0
#define BR_EINVAL (-1)    /* null pointer, V < 1, E < 0, M < 1, bad sizes          */
#define BR_ERANGE (-2)    /* an edge has a vertex id outside [0, V)                 */
#define BR_ENOMEM (-3)    /* device or host allocation failed                       */
#define BR_EHIP (-4)      /* a HIP runtime call failed (message names it)           */
#define BR_EBUSY (-5)     /* server queue full / ticket not finished                */
#define BR_ECAP (-6)      /* output capacity too small; required size reported      */
#define BR_EINTERNAL (-7) /* an impossible state was detected (a bug)               */

typedef struct br_ctx br_ctx;

/* Message describing the last failure on this host thread ("" if none). */
const char* br_last_error(void);

/* Create a context on HIP device `device`.  Owns a growable device workspace,
 * pinned host staging and the host search buffers. */
int br_create(br_ctx** ctx, int device);
int br_destroy(br_ctx* ctx);

/*
 * br_cert_build -- certificate of a whole edge list through the M-chunk phase
 * tree (Section III; Algorithm 2 per chunk and per merge).
 *   d_edges   device int32 [E][2]; chunk i is edges [floor(iE/M), floor((i+1)E/M)),
 *             M may exceed E (then some chunks are empty).
 *   d_cert    device int32 [cert_cap][2]; receives F (spanning forest of the
 *             input) first, then F' (a spanning forest of the edges the merges
 *             left outside F).  cert_cap >= min(E, 2(V-1)) always suffices.
 *   d_counts  device int64 [3]: |F|, |F'|, status (BR_OK, or BR_ERANGE if an
 *             id was out of range; the other values are then meaningless).
 * Asynchronous.  Returns BR_EINVAL / BR_ECAP (cert_cap too small) / BR_ENOMEM /
 * BR_EHIP before enqueueing anything.
 */
int br_cert_build(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* d_cert,
                  int64_t cert_cap, int64_t* d_counts, void* stream);

/*
 * br_cert_build_static -- br_cert_build for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It computes the same certificate through
 * the same kernels, in a fixed device array of BR_STATIC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends, instead
 * of the context's workspace; it allocates no device memory and clears that
 * array with kernels (no memset).  The array holds, 256-byte aligned: the
 * error word, 8M bytes of counters, 8VM bytes of union-find state, 8 bytes
 * per pair of the node regions (sum over the M nodes of min(edges under the
 * node, 2(V-1))) and 16M bytes of node tables; a request that does not fit
 * returns BR_ENOMEM naming the size it needs, before any device work.  Every
 * call on one GPU uses that GPU's one array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other contexts)
 * race, and the caller serialises them.  Arguments, the layout of d_cert and
 * d_counts, asynchrony and the other errors are those of br_cert_build.
 */
#define BR_STATIC_SCRATCH_BYTES ((int64_t)64 << 20)
int br_cert_build_static(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* d_cert,
                         int64_t cert_cap, int64_t* d_counts, void* stream);

/*
 * br_cert_merge -- certificate of the union of two edge lists, the merge step
 * of Section III (usually both lists are certificates; any lists work).
 *   d_a [Ea][2], d_b [Eb][2], d_out [cap][2], d_counts [3] as for br_cert_build.
 *   cap >= min(Ea + Eb, 2(V-1)) always suffices.
 * Asynchronous; errors as for br_cert_build.
 */
int br_cert_merge(br_ctx* ctx, const int32_t* d_a, int64_t Ea, const int32_t* d_b, int64_t Eb, int32_t V,
                  int32_t* d_out, int64_t cap, int64_t* d_counts, void* stream);

/*
 * br_bridges_find -- the whole path: certificate over M chunks (as
 * br_cert_build), then the bridges of the final certificate (by default on the
 * GPU; Algorithm 1's depth-first search on the host with br_set_final_step
 * mode 0), then canonical order.
 *   h_bridges host int32 [cap][2]; cap >= V-1 always suffices.
 *   *n_bridges number of bridges; if it exceeds cap the call returns BR_ECAP
 *              and writes no pairs.
 * Synchronous with respect to `stream`.  BR_ERANGE if an id is out of range.
 */
int br_bridges_find(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_bridges,
                    int64_t cap, int64_t* n_bridges, void* stream);

/*
 * br_two_edge_components -- the 2-edge-connected classes of the graph (its
 * vertices grouped by "still connected after removing any one edge", i.e.
 * the components left once the bridges of Section I are removed), through the
 * same certificate path: the certificate keeps every single-edge-removal
 * connectivity of the input (Section III), so the classes are those of the
 * certificate without its bridges.  With the default final step (see
 * br_set_final_step) the bridges and the union of the remaining certificate
 * edges run on the GPU; with final step 0 the bridges come from Algorithm 1
 * on the host and the union runs there too.
 *   h_label  host int32 [V]: the smallest vertex id of each vertex's class.
 *   *n_classes number of classes (= number of bridges + number of components).
 * Synchronous; errors as for br_bridges_find.
 */
int br_two_edge_components(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_label,
                           int64_t* n_classes, void* stream);

/*
 * br_bridge_tree -- the bridge tree: the graph obtained by contracting every
 * 2-edge-connected class to one node (Section I's bridges are exactly the
 * edges left between classes), a forest with one tree per connected
 * component.  Computed as br_two_edge_components does; a tree edge of the
 * certificate's forest F whose endpoints lie in different classes is a bridge
 * and becomes the tree edge between the two classes.
 *   h_label  host int32 [V]: class of each vertex (its smallest vertex id), as
 *            br_two_edge_components.
 *   h_tree   host int32 [cap][2]: the tree's edges as (min, max) class labels,
 *            ascending; one per bridge, so cap >= V-1 always suffices.
 *   *n_classes number of classes (the tree's nodes); *n_tree number of edges
 *            (the bridges).  BR_ECAP (labels and counts written, no edges) if
 *            *n_tree exceeds cap.
 * Synchronous; errors as for br_bridges_find.
 */
int br_bridge_tree(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, int32_t* h_label,
                   int32_t* h_tree, int64_t cap, int64_t* n_classes, int64_t* n_tree, void* stream);

/*
 * br_certificate_bridges -- the final step alone, on the host: Algorithm 1's
 * depth-first search (Section IV-A) on a certificate S = F u F' given as two
 * host edge lists, then canonical order.  Any edge lists are accepted (the
 * search does not rely on F being a forest); used on certificates, whose
 * bridges are those of the graph they certify (Section III).
 *   h_f1 [n1][2], h_f2 [n2][2] host int32 (either may be null when its count is 0).
 *   h_bridges [cap][2] host; *n_bridges as for br_bridges_find (BR_ECAP if cap is
 *   too small).  BR_ERANGE if an id is outside [0, V).  Needs no device.
 */
int br_certificate_bridges(const int32_t* h_f1, int64_t n1, const int32_t* h_f2, int64_t n2, int32_t V,
                           int32_t* h_bridges, int64_t cap, int64_t* n_bridges);

/*
 * br_bridges_find_batched -- br_bridges_find over G independent graphs in one
 * launch of a persistent kernel (replayed from a captured HIP graph when the
 * same batch shape repeats).
 *   d_edges     device int32 [h_edge_off[G]][2], graph g's edges at
 *               [h_edge_off[g], h_edge_off[g+1]) with graph-local ids in [0, h_V[g]).
 *   h_edge_off  host int64 [G+1], non-decreasing, h_edge_off[0] = 0.
 *   h_V         host int32 [G], each >= 1.
 *   chunk_edges edges per work item (0 = chosen by the built-in tuner).
 *   h_bridges   host int32 [cap][2]; graph g's bridges at
 *               [h_bridge_off[g], h_bridge_off[g+1]), canonical per graph.
 *   h_bridge_off host int64 [G+1].
 * Synchronous.  BR_ECAP if cap < total bridges (h_bridge_off is still filled).
 * Graphs with V above the library's in-LDS limit (br_batched_max_v()) are
 * processed through br_bridges_find inside the call.
 */
int br_bridges_find_batched(br_ctx* ctx, const int32_t* d_edges, const int64_t* h_edge_off, const int32_t* h_V,
                            int32_t G, int32_t chunk_edges, int32_t* h_bridges, int64_t cap, int64_t* h_bridge_off,
                            void* stream);
int32_t br_batched_max_v(void);
/* Largest V for which a plain-path call can run the whole phase tree of
 * Section III inside one workgroup's LDS per chunk (the union-find of
 * Algorithm 2 as two 16-bit parent offsets per vertex in 160 KB); such calls
 * do when their chunks are short enough for one CU each. */
int32_t br_lds_max_v(void);

/*
 * br_autotune -- measure the launch shapes of the certificate path for this
 * device and input shape and keep the fastest for later calls on inputs of
 * the same shape bucket (V and E in powers of two, the same M): the team
 * path (many workgroups per chunk) with three first-stage tiles, the
 * whole-tree LDS kernel where V fits, and the one-workgroup-per-node path in
 * each worker shape with the depths of the merges it does itself around its
 * default; then the winner again with its team merges requesting each
 * thread's edges at once, and (one-workgroup-per-node) with the siblings'
 * certificates of its own merges bucketed by endpoint ranges, then with its
 * chunks in input order instead of bucketed.  Each candidate computes
 * the certificate of d_edges (one settling run, best of two timed runs, HIP
 * events on `stream`).  The choice is kept in memory and, when the
 * environment variable BR_AUTOTUNE_CACHE names a file, in that file (JSON,
 * keyed by GPU architecture and shape bucket), where later processes find it
 * without measuring; a shape already in the cache is not measured again.
 * br_bridges_find_batched with chunk_edges = 0 tunes its chunk size and
 * workgroups per CU the same way.
 *   out  host char [out_cap]: the choice as a JSON object ("source":
 *        "measured" or "cache"), truncated to fit; may be null with out_cap 0.
 * Synchronous.  Errors as for br_cert_build.
 */
int br_autotune(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t M, char* out, int64_t out_cap,
                void* stream);

/*
 * Phase timings of the last br_bridges_find / br_bridges_find_batched on this
 * context, in milliseconds, measured with HIP events on the call's stream
 * (device phases) and a steady clock (host phases).  Filled only when
 * profiling is enabled with br_set_profiling(ctx, 1) (it adds event records);
 * br_set_profiling(ctx, 2) also fills alg_bytes (one more copy of the
 * per-node counters after each call).
 */
typedef struct br_profile {
    double ms_phase0;      /* per-chunk certificate kernel (Section III, phase 0) */
    double ms_merge;       /* all merge rounds                                     */
    double ms_cert;        /* whole device part incl. workspace clears            */
    double ms_d2h;         /* certificate copy to the host                        */
    double ms_dfs;         /* Algorithm 1 on the certificate, host                */
    double ms_canon;       /* canonical order                                     */
    double ms_total;       /* wall clock of the whole call                        */
    int64_t cert_f1, cert_f2;  /* |F|, |F'| of the final certificate              */
    int64_t rounds;        /* merge rounds run                                    */
    int64_t launches;      /* kernel launches                                     */
    double ms_bridge_dev;  /* device bridge step (final step 1 only)              */
    int64_t plan_kind;     /* certificate plan of the last plain-path call: 0 many
                              workgroups per chunk, 1 one workgroup per node
                              (resident slots), 2 the whole tree in LDS        */
    int64_t alg_bytes;     /* br_bridges_find at profiling level 2, plans 0 and 1:
                              the bytes the method itself moves at this M
                              (Section III): 8 per input edge read by phase 0,
                              8 per certificate edge written to a node's region,
                              8 per edge of a right sibling's certificate read
                              by its merge (the merges carry state, so a
                              region's final size counts every edge written
                              to it once); 0 otherwise                         */
} br_profile;
int br_set_profiling(br_ctx* ctx, int on);

/*
 * Final step used by br_bridges_find on this context:
 *   0           -- Algorithm 1's depth-first search (Section IV-A) on the
 *                  certificate, in the library's host code, after copying the
 *                  certificate (at most 2(V-1) edges) to the host;
 *   1 (default) -- the same bridge set computed on the GPU: F of the
 *                  certificate rooted by Euler tours, preorder numbers and
 *                  subtree sizes by list ranking, and a tree edge kept as a
 *                  bridge iff no certificate edge leaves the child's subtree
 *                  (the low-link test of Algorithm 1 on an arbitrary rooted
 *                  spanning tree; the parallelisation the paper's Section VII
 *                  asks for).  Only the bridges are copied to the host.
 * BR_EINVAL for another mode.
 */
int br_set_final_step(br_ctx* ctx, int mode);
int br_get_profile(br_ctx* ctx, br_profile* out);

/*
 * br_articulation_points -- the "failure points" of the abstract: vertices
 * whose removal (with their edges) increases the number of connected
 * components (Section I's bridge definition carried over to vertices).
 * Path: a scan-first certificate of the whole edge list on the GPU -- F a
 * breadth-first forest of G (each tree from the smallest vertex of its
 * component; a newly reached vertex takes its smallest-id neighbour one level
 * up as parent), F' a breadth-first forest of G without the vertex pairs of F
 * (all parallel copies of them left out) -- then the cut-vertex test on
 * F u F' (at most 2(V-1) edges).  With the default final step (see
 * br_set_final_step) the test runs on the GPU: F rooted by its Euler tours,
 * tree edges grouped into blocks (an edge of F' between unrelated vertices
 * joins their parent edges; a child's parent edge joins its parent's when the
 * child's subtree reaches outside the parent's), a vertex cut iff its child
 * edges are not all in its own parent edge's block (a root: in two or more
 * blocks).  Final step 0 runs the low-link search on the host instead: a
 * non-root p cuts iff a child c has low[c] >= disc[p], a root iff it has two
 * or more children.  The
 * union-find forests of Algorithm 2 (Section IV-B) would not do: they keep
 * edge connectivity but not vertex connectivity; search-ordered forests keep
 * both (the certificate definition of Section III, for 2-vertex connectivity).
 *   d_edges  device int32 [E][2], E <= 2^31 - 1; self-loops and parallel edges accepted.
 *   h_out    host int32 [cap]: vertex ids ascending; cap >= V always suffices.
 *   *n_out   number of articulation points; BR_ECAP (no ids written) if it exceeds cap.
 * Synchronous with respect to `stream`.  BR_ERANGE if an id is out of range.
 */
int br_articulation_points(br_ctx* ctx, const int32_t* d_edges, int64_t E, int32_t V, int32_t* h_out, int64_t cap,
                           int64_t* n_out, void* stream);

/*
 * Serving: continuous batching of bridge queries on one device.
 *   br_server_create  device, device-memory budget in bytes for resident
 *                     requests (edge lists, union-find state, certificates;
 *                     slots and lane workers keep their buffers between
 *                     requests and they stay charged until the scheduler
 *                     releases them to admit a request that would not fit
 *                     otherwise), max_slots (1..64) requests on the plain
 *                     path in flight on the device at once, each on its own
 *                     stream.  Requests are admitted in arrival order as
 *                     soon as the budget has room for them.  A slot runs the
 *                     whole path of br_bridges_find with a chunk count chosen
 *                     from the request's size (M = clamp(E / 8V, 1, 64)).
 *                     Requests within the batching limits (br_server_set_
 *                     batching; by default V <= br_lds_max_v() and E <= 2^21)
 *                     take a free slot while the batch lane has nothing
 *                     queued, and otherwise join the lane: a lane worker
 *                     certifies every lane request queued when it becomes
 *                     free in one call of the batched path (two workers
 *                     alternate).  Both paths give the bridges
 *                     br_bridges_find gives.
 * Submit/poll/wait may be called from several host threads.
 */
typedef struct br_server br_server;
typedef struct br_server_stats_t {
    int64_t completed;
    double p50_ms, p99_ms, mean_ms, max_ms;
    double edges_per_s;    /* edges of completed requests / busy wall time */
    int64_t peak_inflight; /* most requests resident on the device at once */
    int64_t device_bytes;  /* device memory the slots hold now (charged to the budget) */
    int64_t peak_device_bytes; /* the most they held at once (never above the budget
                                  unless a single request larger than the others' room ran alone) */
    int64_t batched_ticks;     /* batch-lane ticks (batched calls) since the last reset */
    int64_t batched_requests;  /* requests those ticks served */
} br_server_stats_t;
int br_server_create(br_server** srv, int device, int64_t mem_budget, int32_t max_slots);
int br_submit(br_server* srv, const int32_t* h_edges, int64_t E, int32_t V, uint64_t* ticket);
/* As br_submit for an edge list already resident on the server's device
 * (d_edges [E][2]); the caller keeps it alive and unchanged until the ticket
 * is done.  Nothing is copied.  The edges must be complete when the call is
 * made (the server reads them on its own streams, unordered with the
 * caller's: synchronise the stream that wrote them first). */
int br_submit_device(br_server* srv, const int32_t* d_edges, int64_t E, int32_t V, uint64_t* ticket);
int br_poll(br_server* srv, uint64_t ticket, int32_t* h_out, int64_t cap, int64_t* n, int* done);
int br_wait(br_server* srv, uint64_t ticket, int32_t* h_out, int64_t cap, int64_t* n);
int br_server_stats(br_server* srv, br_server_stats_t* out, int reset);
/* Final step of the requests admitted from now on (see br_set_final_step);
 * each request keeps the mode it was admitted with, requests already queued
 * or running are not affected. */
int br_server_set_final_step(br_server* srv, int mode);
/* Batching limits of the requests submitted from now on: those with
 * V <= max_v and E <= max_e may join the batch lane; max_v = 0 or max_e = 0
 * sends every request to a slot.  max_v in [0, br_lds_max_v()], max_e >= 0,
 * else BR_EINVAL.  Requests already submitted keep their limits. */
int br_server_set_batching(br_server* srv, int32_t max_v, int64_t max_e);
int br_server_destroy(br_server* srv);

/*
 * br_probe_read -- measurement utility, not a step of the method: reads
 * d_buf [bytes] once with 16-byte loads (d_buf 16-byte aligned) and adds a
 * fold of what it read to *d_sink (device uint64), asynchronously on
 * `stream`.  Timed around its launch it gives the read bandwidth the device
 * reaches, which benchmarks report beside the HBM peak.  BR_EINVAL for a null
 * or misaligned pointer or bytes < 0.
 */
int br_probe_read(const void* d_buf, int64_t bytes, uint64_t* d_sink, void* stream);

#ifdef __cplusplus
}
#endif
#endif
