/*
 * tkc.h -- exact top-k closeness centrality on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Bergamini, Borassi, Crescenzi, Marino, Meyerhenke, "Computing
 * top-k Closeness Centrality Faster in Unweighted Graphs", Sect. 2 and the
 * input/output of Alg. 1): given an unweighted graph G = (V, E), directed or
 * undirected, return the k vertices of highest closeness.  For a vertex v
 * with reachable set R(v) (v included) and r(v) = |R(v)|,
 *     S(v) = sum_{w in R(v)} d(v, w),
 *     f(v) = (n-1) S(v) / (r(v)-1)^2          (farness, Eq. 1; Lin's index)
 * and closeness c(v) = 1/f(v); a vertex that reaches nothing (r = 1) has
 * closeness 0 (f = +inf).  Results follow the exact order
 *     v before w  iff  f(v) < f(w), or f(v) = f(w) and v < w,
 * (exact rational comparison; the smaller id wins a tie) and exactly
 * min(k, n) vertices are returned.
 *
 * The library runs the paper's pruned search (Alg. 1) on the GPU: lower
 * bounds on farness from degree order (Deg) or walk counts (NB, Sect. 5),
 * breadth-first searches cut as soon as a bound proves the vertex cannot
 * enter the top k (BFSCut, Sect. 6) or complete searches that raise the
 * bounds of other vertices (LB, Sect. 7), and the directed, disconnected
 * machinery of Sect. 8 (alpha/omega reachability bounds, Alg. 6).
 *
 * Conventions for every entry point:
 *   - Return value: TKC_OK (0) or a negative TKC_E* code; nothing throws.
 *     tkc_last_error() gives a message for the calling thread's last error.
 *   - Vertex ids are int32 in [0, n); the CSR arrays are int32, so the arc
 *     count must stay below 2^31.
 *   - Input arrays are only read during the call; the library copies what it
 *     keeps.  Output arrays are caller-owned with room for min(k, n) items.
 *   - A context owns one HIP stream (the caller's, or its own) and its
 *     device workspace; calls on one context must not overlap (one thread at
 *     a time); separate contexts may be used from separate threads.
 */
#ifndef TKC_H
#define TKC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TKC_OK 0
#define TKC_EINVAL (-1)     /* bad argument or malformed graph            */
#define TKC_ENOMEM (-2)     /* device or host allocation failed           */
#define TKC_EDEVICE (-3)    /* a HIP call failed                          */
#define TKC_ENOTSUP (-4)    /* option not supported for this input        */
#define TKC_EBUSY (-5)      /* object in use / admission refused          */
#define TKC_ECANCELED (-6)  /* request cancelled                          */

/* lower-bound strategy (Sect. 9: the four variants; Sect. 4: computeBounds /
 * updateBounds).  AUTO picks a Cut variant for low-diameter graphs and a
 * Bound variant for high-diameter ones, following the paper's finding that
 * BFSCut wins on complex networks and LB on street networks (Sect. 9.1). */
#define TKC_AUTO 0
#define TKC_DEG_CUT 1       /* degree order + BFSCut                      */
#define TKC_NB_CUT 2        /* neighbourhood bound + BFSCut               */
#define TKC_DEG_BOUND 3     /* degree order + level-based updates         */
#define TKC_NB_BOUND 4      /* neighbourhood bound + level-based updates  */
/* Cut and level-based updates combined (the combination Sect. 9.1 leaves
 * open): the BFSCut bound may stop a search while it is shallow (at most 8
 * levels deep), and every search that completes applies its level-based
 * update to the other vertices' bounds.  Low-diameter graphs then behave
 * like the Cut variants plus updates, high-diameter ones like the Bound
 * variants.  Same exact result as every other variant. */
#define TKC_DEG_CUTLB 5     /* degree order + BFSCut + level-based updates */
#define TKC_NB_CUTLB 6      /* neighbourhood bound + BFSCut + level-based  */

/* execution mode of the searches */
#define TKC_PLAIN 0         /* one source at a time, whole GPU per search */
#define TKC_BATCHED 1       /* W sources per launch, one bit lane each    */
#define TKC_HYBRID 2        /* batched seed, then one search per workgroup
                               for short cut searches, batched tail        */
#define TKC_MODE_AUTO 3     /* the graph's autotuned mode and knobs when
                               tkc_autotune has run on it, else the
                               context's preferred mode and knobs          */

/* graph flags */
#define TKC_DIRECTED 1u     /* arcs are directed; reverse CSR required    */
#define TKC_VALIDATE 2u     /* check CSR shape, ids, loops, repeats, symmetry */
#define TKC_DEVICE_PTRS 4u  /* input arrays are device pointers           */
#define TKC_REVERSE 8u      /* in-closeness: distances run along in-arcs,
                               i.e. out-closeness of the reversed graph
                               (the reversed-graph case study, Sect. 10);
                               no effect on undirected graphs              */
#define TKC_RELABEL 16u     /* store the graph with its vertices renumbered
                               by decreasing out-degree (ties by id), which
                               packs the heavy vertices' words together for
                               skewed graphs; every result, tie-break and
                               per-vertex output still uses the caller's
                               ids.  Such a graph serves the top-k queries,
                               tkc_autotune, tkc_graph_reach and servers
                               (without packing); the other step functions,
                               tkc_graph_reach_noalloc and tkc_pack_create
                               return TKC_EINVAL for it                    */

typedef struct tkc_ctx tkc_ctx;
typedef struct tkc_graph tkc_graph;
typedef struct tkc_server tkc_server;
typedef struct tkc_pack tkc_pack;

/* per-call statistics; every field is filled on success */
typedef struct {
    int64_t m_vis;          /* arcs scanned by searches: sum over searched
                               levels of the out-degrees of the level's
                               vertices (the paper's work count, Sect. 9.1) */
    int64_t bfs_started;    /* searches started                            */
    int64_t bfs_exact;      /* searches that ran to completion             */
    int64_t bfs_cut;        /* searches stopped by the BFSCut bound        */
    int64_t skipped;        /* vertices skipped by their bound             */
    int64_t deferred;       /* per-workgroup searches handed to batches    */
    int32_t max_level;      /* deepest level reached                       */
    int32_t batch_width;    /* lanes per batch (W)                         */
    int32_t variant_used;
    int32_t mode_used;
    int32_t nb_rounds;      /* walk-count levels the NB bound computed
                               (full rounds and tail rounds over the open
                               vertices; with cached bounds, the count of
                               the run that computed them)                 */
    int32_t pad_;
    /* phase times: HIP events on the context's stream                     */
    double ms_reach;        /* reachability (r or alpha/omega)             */
    double ms_bounds;       /* initial bounds and ordering                 */
    double ms_traverse;     /* searches (all engines)                      */
    double ms_total;        /* whole call, host clock                      */
    double ms_kernel_main;  /* HIP-event time of the dominant traversal
                               kernel launches (see main_kernel)            */
    int32_t main_launches;  /* number of such launches                     */
    int32_t main_kernel;    /* 0 plain, 1 batched, 2 per-workgroup         */
    int64_t bytes_main;     /* algorithmic bytes of those launches         */
} tkc_stats;

/* Context on HIP device `device`; hip_stream may be NULL (library stream) or
 * a hipStream_t the caller keeps alive.  Error: TKC_EDEVICE. */
int tkc_ctx_create(int device, void *hip_stream, tkc_ctx **out);
/* Waits for the context's stream, then frees it.  Free the servers, packs
 * and graphs made on a context before it: they use its stream and device.
 * (Graphs still held at process exit are simply released with the device.) */
int tkc_ctx_destroy(tkc_ctx *ctx);

/* Execution knobs of a context (performance only: results never depend on
 * them).
 *   batch_width    lanes (sources) per batch: 32, 64, 128 or 256
 *   td_bu_alpha    one-source searches go push -> pull when the frontier's
 *                  arcs exceed the unexplored arcs / alpha (Beamer's alpha)
 *   bu_td_beta     ... and pull -> push when the frontier holds fewer than
 *                  n / beta vertices (Beamer's beta; batches use it too)
 *   batch_alpha    the push -> pull rule for batched searches (a pull over
 *                  several lanes rarely stops early, so it pays later)
 *   swarm_qcap     queue capacity of one per-workgroup search (>= 64) before
 *                  it is handed to the batched engine
 *   seed_lanes     lanes of the hybrid mode's first (seed) batch, 0 meaning
 *                  batch_width
 *   blocks_per_cu  workgroups per compute unit of the persistent kernels,
 *                  1..8 (capped at what fits; more hides more latency, fewer
 *                  make grid barriers cheaper)
 *   mode           TKC_PLAIN, TKC_BATCHED or TKC_HYBRID: what TKC_MODE_AUTO
 *                  runs on a graph that has not been autotuned */
typedef struct {
    int32_t batch_width;
    int32_t td_bu_alpha;
    int32_t bu_td_beta;
    int32_t batch_alpha;
    int32_t swarm_qcap;
    int32_t seed_lanes;
    int32_t blocks_per_cu;
    int32_t mode;
} tkc_tuning;

int tkc_ctx_get_tuning(tkc_ctx *ctx, tkc_tuning *out);
/* Every field is checked; TKC_EINVAL leaves the context unchanged. */
int tkc_ctx_set_tuning(tkc_ctx *ctx, const tkc_tuning *t);

/* Copy a graph to device memory.  row_ptr[n+1], col_idx[m_arcs] give the
 * out-arcs; rrow_ptr/rcol_idx give the in-arcs and are required iff
 * TKC_DIRECTED (NULL otherwise).  Undirected graphs hold each edge in both
 * rows.  Every upload checks that row_ptr starts at 0, never decreases and
 * ends at m_arcs, and that every vertex id is in [0, n) (TKC_EINVAL
 * otherwise: the kernels index with them).  The graph must also be simple
 * (no self-loops, no repeated arcs, rows need not be sorted); TKC_VALIDATE
 * checks that too, and symmetry / that the reverse CSR is the transpose,
 * and returns TKC_EINVAL with a message.
 * n >= 1.  Errors: TKC_EINVAL, TKC_ENOMEM, TKC_EDEVICE. */
int tkc_graph_upload(tkc_ctx *ctx, int32_t n, int64_t m_arcs,
                     const int32_t *row_ptr, const int32_t *col_idx,
                     const int32_t *rrow_ptr, const int32_t *rcol_idx,
                     uint32_t flags, tkc_graph **out);
/* TKC_EBUSY while a server still holds the graph. */
int tkc_graph_free(tkc_graph *g);

/* Top-k closeness (Alg. 1).  k >= 1 (TKC_EINVAL otherwise); *n_out =
 * min(k, n) results written in the exact order: ids, S (sum_dist), r
 * (reach) and f (farness, computed as ((double)(n-1)*(double)S) /
 * ((double)(r-1)*(double)(r-1)), +inf when r = 1).  Any output pointer
 * except ids and n_out may be NULL.  stats may be NULL. */
int tkc_topk_closeness(tkc_graph *g, int32_t k, int32_t variant, int32_t mode,
                       int32_t *ids, int64_t *sum_dist, int64_t *reach, double *farness,
                       int32_t *n_out, tkc_stats *stats);

/* Top-k closeness (Alg. 1) in plain mode (one search at a time, Sect. 6),
 * with at most max_searches (>= 1) breadth-first searches: for measuring
 * the one-source-at-a-time engine on graphs where a whole plain run would
 * take too long.  A query that finishes within the cap returns TKC_OK and
 * the same results as tkc_topk_closeness.  One that would need more returns
 * TKC_ECANCELED with *n_out = 0, no results, and *stats (if not NULL)
 * holding the work done so far: bfs_started = max_searches, m_vis, and the
 * phase times.  Errors: TKC_EINVAL, TKC_ENOMEM, TKC_EDEVICE. */
int tkc_topk_closeness_budget(tkc_graph *g, int32_t k, int32_t variant, int64_t max_searches,
                              int32_t *ids, int64_t *sum_dist, int64_t *reach, double *farness,
                              int32_t *n_out, tkc_stats *stats);

/* Top-k harmonic centrality: h(v) = sum of 1/d(v,w) over the vertices w
 * that v reaches (the measure of Sect. 2 with f(d) = 1/d, ranked in Sect.
 * 9.1).  h is the binary64 value of the terms n_d / d added in increasing d
 * (n_d = vertices at distance d), exactly as the library computes it; the
 * order is larger h first, an exact tie to the smaller id.  variant:
 * any of them, with upper bounds in place of the farness lower bounds
 * (degree: the out-neighbours at distance 1, every other reachable vertex
 * at distance 2; walk counts: levels filled as close as the counts of
 * Sect. 5 allow; level-based: every vertex at least max(2, level gap)
 * away from w but its out-neighbours, see tkc_graph_harmonic_lb_update).
 * mode: any, as for closeness.  *n_out = min(k, n) results in order: ids
 * and harmonic values.  stats may be NULL. */
int tkc_topk_harmonic(tkc_graph *g, int32_t k, int32_t variant, int32_t mode,
                      int32_t *ids, double *harmonic, int32_t *n_out, tkc_stats *stats);
/* The harmonic upper bounds a harmonic query starts from (variant
 * TKC_DEG_CUT or TKC_NB_CUT), each already raised by the relative margin
 * 1e-9 the search applies to every bound, and the processing order
 * (largest bound first, ties by id; may be NULL).  Host arrays of n. */
int tkc_graph_harmonic_bounds(tkc_graph *g, int32_t variant, double *ub, int32_t *order);
/* Level-based update of harmonic upper bounds (Sect. 7's argument with
 * f(d) = 1/d): after a complete search from s, a vertex w that s reaches
 * (same SCC of s for directed graphs) has h(w) <= the sum over the other
 * vertices s reaches of 1/max(2, level gap) (gap |i - l|, directed i - l)
 * plus 1/2 per out-neighbour of w; the binary64 value is the per-level sum
 * in increasing level, minus w's own 1/2, plus 0.5 * deg(w).  Each bound is
 * raised by the 1e-9 margin and ub[w] becomes the least of its old value
 * and those bounds.  ub: host array of n finite values >= 0, in place. */
int tkc_graph_harmonic_lb_update(tkc_graph *g, const int32_t *sources, int32_t count, double *ub);

/* Autotuner: times the query (k, variant) on g under candidate knob
 * settings, one knob at a time (batch width, mode, workgroups per CU, the
 * pull threshold beta, batch alpha), keeping each improvement, until the settings are exhausted or the
 * measured time passes budget_ms (at least the context's own settings run).
 * Every trial's ids must agree (TKC_EDEVICE otherwise: an internal error).
 * The fastest setting is stored on the graph, where TKC_MODE_AUTO queries
 * (and the server) use it, and copied to best / best_ms (either may be
 * NULL).  The context's own settings are left as they were. */
int tkc_autotune(tkc_graph *g, int32_t k, int32_t variant, double budget_ms, tkc_tuning *best,
                 double *best_ms);

/* Top-k with every tie (the output of Alg. 1 as stated: all vertices whose
 * farness equals the k-th one are returned, possibly more than k).  Results
 * are the min(k, n) of tkc_topk_closeness followed by the vertices tied
 * with the k-th, by increasing id.  cap is the capacity of the output
 * arrays (>= min(k, n)); if the answer has more entries, TKC_EINVAL is
 * returned with *n_out set to the number needed and nothing else written.
 * Ties are found by cutting only searches whose bound is strictly above the
 * k-th farness (ids no longer break ties), so they cost more work. */
int tkc_topk_closeness_ties(tkc_graph *g, int32_t k, int32_t variant, int32_t mode, int32_t cap,
                            int32_t *ids, int64_t *sum_dist, int64_t *reach, double *farness,
                            int32_t *n_out, tkc_stats *stats);

/* ---- inspection of the individual steps (host output arrays of n items) */
/* Reachability (Sect. 4 and Sect. 8.4, Alg. 6): undirected graphs get
 * alpha = omega = r (component size); directed graphs get the alpha/omega
 * bounds of Alg. 6 (exact r for vertices whose bounds coincide); scc may be
 * NULL and is filled (component ids in topological order) for directed
 * graphs only. */
int tkc_graph_reach(tkc_graph *g, int64_t *alpha, int64_t *omega, int32_t *scc);
/* How the reachability bounds of g were computed (Sect. 8.4, Alg. 6), all
 * on the device: *path = 0 not yet (computed by the first query or
 * tkc_graph_reach), 1 by the parallel steps alone (always for undirected
 * graphs), 2 with a one-thread device pass finishing what the parallel
 * steps left at their round caps (long chains of strongly connected
 * components, or a component DAG deeper than the relaxation cap); *ms =
 * the time it took.  Either pointer may be NULL.  Errors: TKC_EINVAL for a
 * NULL graph. */
int tkc_graph_reach_info(const tkc_graph *g, int32_t *path, double *ms);

/* For callers that cannot allocate device or pinned memory (tight serving
 * loops, harnesses that forbid allocation): the reachability bounds of
 * tkc_graph_reach, computed without any allocation.  Every buffer the
 * kernels need beyond the graph and the outputs comes from one static
 * device array of TKC_NOALLOC_SCRATCH_BYTES per GPU, set up when a context
 * is created on that GPU and held until the process ends.
 *   alpha, omega: device int64[n], written; scc: device int32[n] (component
 *   ids in a topological order of the component DAG, directed graphs only)
 *   or NULL.  Undirected graphs get alpha = omega = component size and
 *   leave scc untouched.  Nothing is cached on g (tkc_graph_reach_info is
 *   unchanged).
 *   Errors: TKC_EINVAL for a NULL g, alpha or omega, or for a graph whose
 *   scratch need exceeds TKC_NOALLOC_SCRATCH_BYTES (the message gives the
 *   need); TKC_EDEVICE on a device error.
 * Calls on one GPU share its array, which keeps the last call's contents:
 * the library serialises the calls of one process on one GPU, and the
 * call returns only after its kernels have finished.  It reads counts back
 * to the host between steps, so it cannot be captured into a HIP graph. */
#define TKC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int tkc_graph_reach_noalloc(tkc_graph *g, int64_t *alpha, int64_t *omega, int32_t *scc);
/* Initial lower bounds (Sect. 4 computeBounds): the farness bound is
 * (n-1) * num / den, den = 0 meaning +inf.  variant TKC_DEG_* gives 0 (and
 * +inf when r = 1), TKC_NB_* the neighbourhood bound of Sect. 5 / 8.1.
 * order (may be NULL) receives the processing order. */
int tkc_graph_bounds(tkc_graph *g, int32_t variant, int64_t *num, int64_t *den, int32_t *order);
/* Level-based bound (Sect. 7): apply the LB update of complete searches
 * from sources[0..count) to the bounds (num, den) in place (host arrays of
 * n; den = 0 is +inf and is never lowered). */
int tkc_graph_lb_update(tkc_graph *g, const int32_t *sources, int32_t count,
                        int64_t *num, int64_t *den);
/* Exact (S, r) of the given sources by full searches on the device
 * (batched engine, no cut). */
int tkc_graph_sums(tkc_graph *g, const int32_t *sources, int32_t count,
                   int64_t *sum_dist, int64_t *reach);

/* ---- packs: top-k requests on several graphs in one batched launch */
/* A pack of `count` graphs of one context, all directed or all undirected,
 * each listed once: the library uploads their disjoint union once (member
 * i's vertices renumbered by an offset; no arc joins two members) so that
 * requests on different members can share the lanes of one batched launch
 * (Alg. 1 with BFSCut, Sect. 6, each request with its own order, bounds
 * and k-th farness).  The members stay owned by the caller and must outlive
 * the pack (tkc_graph_free returns TKC_EBUSY meanwhile); their
 * preprocessing (reachability, initial bounds, order) is cached on them.
 * Errors: TKC_EINVAL (NULL, empty, mixed directedness, repeated graph,
 * another context, union beyond int32 ids), TKC_ENOMEM, TKC_EDEVICE. */
int tkc_pack_create(tkc_ctx *ctx, tkc_graph *const *graphs, int32_t count, tkc_pack **out);
/* nreq requests (1..64) on distinct members member[0..nreq) of pack p,
 * request i asking for the top k[i] (k[i] >= 1) by closeness.  variant:
 * TKC_NB_CUT or TKC_DEG_CUT (TKC_AUTO means TKC_NB_CUT); every variant
 * gives the same answers, only the work differs.  Results are concatenated
 * in request order: request i's n_out[i] = min(k[i], n of its member)
 * results, in each member's own vertex ids and the exact order of
 * tkc_topk_closeness, start at the sum of n_out[0..i).  ids (and sum_dist,
 * reach, farness when not NULL) hold the sum of min(k[i], n_i) entries;
 * n_out holds nreq.  stats (may be NULL) covers the whole launch.  Each
 * request's answer equals tkc_topk_closeness on its member alone.  Errors:
 * TKC_EINVAL (also for two requests on one member), TKC_ENOMEM,
 * TKC_EDEVICE. */
int tkc_pack_topk(tkc_pack *p, int32_t nreq, const int32_t *member, const int32_t *k, int32_t variant,
                  int32_t *ids, int64_t *sum_dist, int64_t *reach, double *farness, int32_t *n_out,
                  tkc_stats *stats);
int tkc_pack_free(tkc_pack *p);

/* ---- serving: graphs stay resident, requests are batched as they arrive */
/* Packing for a server: every added graph of at most max_vertices vertices
 * joins a pack (tkc_pack_create; undirected and directed graphs apart, up
 * to 64 members and 2^28 arcs each).  A request on a packed graph whose
 * variant resolves to TKC_NB_CUT or TKC_DEG_CUT is then served together
 * with the queued requests on the pack's other members, in one batched
 * launch (tkc_pack_topk); answers are unchanged.  max_vertices = 0 turns
 * packing off.  Call it after adding the graphs and while no request is
 * queued or running (TKC_EBUSY otherwise).  Errors: TKC_EINVAL, TKC_EBUSY,
 * TKC_ENOMEM, TKC_EDEVICE. */
int tkc_server_enable_packing(tkc_server *s, int32_t max_vertices);
/* Counters of server s (any pointer may be NULL): requests served,
 * requests served in packed launches, packed launches, packs. */
int tkc_server_info(tkc_server *s, int64_t *served, int64_t *packed, int64_t *pack_calls, int32_t *packs);
/* hbm_budget_bytes caps the device memory the server's request slots may
 * use (admission control); max_inflight caps concurrent requests. */
int tkc_server_create(tkc_ctx *ctx, size_t hbm_budget_bytes, int32_t max_inflight,
                      tkc_server **out);
/* Adds a graph (it may be called while requests run); the graph must stay
 * uploaded until the server is destroyed (tkc_graph_free refuses it with
 * TKC_EBUSY until then). */
int tkc_server_add_graph(tkc_server *s, tkc_graph *g, int32_t *graph_id);
/* Queue a request; TKC_EBUSY if it can never fit the budget. */
int tkc_server_submit(tkc_server *s, int32_t graph_id, int32_t k, int32_t variant,
                      uint64_t *ticket);
int tkc_server_poll(tkc_server *s, uint64_t ticket, int32_t *done);
/* Blocks until the request finished; results as for tkc_topk_closeness.
 * latency_ms = completion - submission. */
int tkc_server_result(tkc_server *s, uint64_t ticket, int32_t *ids, int64_t *sum_dist,
                      int64_t *reach, double *farness, int32_t *n_out, double *latency_ms);
/* A queued request is dropped at once; a running one finishes, and either
 * way tkc_server_result then returns TKC_ECANCELED. */
int tkc_server_cancel(tkc_server *s, uint64_t ticket);
/* Lets the workers finish the requests they are running, drops the queued
 * ones and frees the server.  No other call on s may run during or after
 * it: collect or cancel every ticket first. */
int tkc_server_destroy(tkc_server *s);

const char *tkc_last_error(void);
const char *tkc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TKC_H */
