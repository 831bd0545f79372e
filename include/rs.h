/*
 * rs.h -- C ABI of the MI355X robust-spanner (RS) scoring library.
 *
 * The library scores every vertex of an undirected graph by the Robust
 * Spanning Index of "A Parallel Algorithm for Finding Robust Spanners in
 * Large Social Networks" (arXiv 2508.01485) and returns the highest-scoring
 * vertices.  All compute runs in HIP kernels on one gfx950 device; this
 * header is the only interface (plain pointers and sizes, no C++ or torch
 * types).
 *
 * Conventions shared by every call
 *   - Every function returns rs_status.  The library never aborts, never
 *     throws across this boundary and never prints.  On any error the graph
 *     state is unchanged; rs_last_error() returns a detail string for the
 *     calling thread.
 *   - Vertex ids and community labels at this boundary are always the
 *     caller's ids.  The library may renumber internally.
 *   - The caller owns every buffer it passes in or receives into.  The
 *     library owns the device memory of a graph from rs_load_graph until
 *     rs_free_graph and never keeps caller pointers.
 *   - One rs_graph must not be used from two threads at once; distinct
 *     graphs may be used concurrently.
 */
#ifndef RS_H
#define RS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rs_graph rs_graph; /* one resident graph on one device + its HIP stream */

typedef enum {
    RS_OK = 0,
    RS_ERR_ARG = 1,   /* null pointer, negative size, bad flag or width */
    RS_ERR_GRAPH = 2, /* not a simple undirected graph, or a negative label */
    RS_ERR_RANGE = 3, /* an id >= n, or n / nnz too large for the offset width */
    RS_ERR_NOMEM = 4, /* device or host allocation failed */
    RS_ERR_HIP = 5,   /* a HIP runtime call failed (no device, launch error, ...) */
    RS_ERR_STATE = 6  /* call out of order (e.g. rs_topk before rs_score) */
} rs_status;

/*
 * Input graph: G = (V, E) undirected and simple, stored as CSR, plus one
 * non-overlapping community label per vertex (Section II; the CSR layout of
 * Section VI-A; community ids are user input, Section VI-A).
 *   n            number of vertices, 0 <= n < 2^31
 *   nnz          number of CSR entries = 2|E|
 *   offset_bytes 4 (int32) or 8 (int64): element width of row_offsets
 *   on_device    0: the three arrays are host pointers;
 *                1: they are HIP device pointers on the current device
 *   row_offsets  [n+1], row_offsets[0] = 0, non-decreasing, row_offsets[n] = nnz
 *   col          [nnz] int32 neighbour ids; each row strictly ascending, no
 *                self-loop, and (u,v) present iff (v,u) present
 *   labels       [n] int32 community ids, any non-negative values
 */
typedef struct {
    int64_t n;
    int64_t nnz;
    int32_t offset_bytes;
    int32_t on_device;
    const void *row_offsets;
    const int32_t *col;
    const int32_t *labels;
} rs_csr;

/*
 * rs_load_graph: validate the graph, renumber it internally (communities as
 * contiguous id ranges, rows re-sorted), copy it to device memory and return
 * a handle.  Returns only after the copies are complete.
 *   hip_stream  a hipStream_t to run all of this graph's work on, or NULL for
 *               a library-owned stream
 *   flags       0, or RS_LOAD_WIDE_OFFSETS: keep 64-bit edge offsets on the
 *               device even when nnz fits 32 bits (they are used anyway when
 *               nnz > INT32_MAX; the flag lets small graphs run that form)
 * Errors: RS_ERR_ARG, RS_ERR_GRAPH (asymmetric / unsorted / duplicate / self
 * loop / negative label), RS_ERR_RANGE, RS_ERR_NOMEM, RS_ERR_HIP.  *out is
 * set to NULL on error.
 */
#define RS_LOAD_WIDE_OFFSETS 1u

rs_status rs_load_graph(const rs_csr *csr, void *hip_stream, uint32_t flags, rs_graph **out);

/*
 * rs_score: one full scoring pass (Algorithm 1, Steps 1-3): border vertices
 * (Step 1), the per-(vertex, community) interaction matrix of neighbour
 * community counts and its entropy weights w_v(c) with Algorithm 2's shared
 * terms and the global w_max (Step 2), the inter-community subgraph G', and
 * the Robust Spanning Index of Eq. RSI for every vertex, normalized by w_max
 * (Step 3).  Enqueued on the graph's stream; returns without waiting.
 */
rs_status rs_score(rs_graph *g);

/*
 * rs_topk: the k highest-scoring live vertices (Algorithm 1, Step 4), ordered
 * by score descending, ties by the smaller caller id.  Writes
 * min(k, live vertices) entries to the host arrays ids[k] and scores[k] and
 * that count to *count; waits for the stream.  RS_ERR_STATE before the first
 * rs_score.
 */
rs_status rs_topk(rs_graph *g, int64_t k, int32_t *ids, double *scores, int64_t *count);

/*
 * Removal batch (the robustness disruptions of Section VII-B: random edge
 * and vertex removal).  Host arrays: n_edges pairs (src[i], dst[i]) and
 * n_vertices vertex ids.  Edges not in the graph are ignored and counted;
 * repeated entries are idempotent.  A removed vertex loses all its edges,
 * keeps its label, scores 0 and is excluded from rs_topk.
 */
typedef struct {
    int64_t n_edges;
    const int32_t *src;
    const int32_t *dst;
    int64_t n_vertices;
    const int32_t *vertices;
} rs_removals;

typedef struct {
    int64_t edges_removed;   /* distinct undirected edges deleted (including a removed vertex's edges) */
    int64_t edges_ignored;   /* batch edge entries that named no existing edge */
    int64_t vertices_removed;/* vertices newly removed */
    int64_t affected;        /* vertices whose score depends on the removed edges (re-scored) */
} rs_removal_result;

/*
 * rs_apply_removals: validate the whole batch (RS_ERR_RANGE for an id >= n,
 * RS_ERR_ARG for null arrays with non-zero counts) before mutating anything,
 * apply it, then re-score so that every reader and rs_topk reflect the
 * mutated graph exactly as a fresh full rs_score would (bit for bit).  The
 * re-score is incremental: rows are recomputed only for the endpoints of
 * removed edges, and scores only for the vertices that depend on them (the
 * endpoints, their neighbours in other communities, and the members of an
 * endpoint's community adjacent to those neighbours); if w_max moves, every
 * score is rescaled.  This follows the removal model of the experiments
 * (Section VII-B).  Waits for the stream once, after the removal itself
 * (res is then complete); the re-score stays queued on the graph's stream,
 * like rs_score's pass, and the library's readers wait for it.
 * RS_ERR_STATE before the first rs_score.
 */
rs_status rs_apply_removals(rs_graph *g, const rs_removals *batch, rs_removal_result *res);

/*
 * Target-community mode (Section VI-A: spanners are searched in large,
 * user-given communities and the interaction matrix has one column per
 * considered community, with T summed over those; Section VII-C: the k
 * largest communities by member count).  Keeps the k_c communities with the
 * most members at load (ties: the smaller caller label first) and removes
 * every vertex of the others as rs_apply_removals does, so the counts, T,
 * weights, w_max and triads involve the target communities only: the result
 * is the pass over the subgraph the targets induce (degrees included).
 * Vertices outside the targets score 0 and are excluded from rs_topk.  The
 * handle stays restricted; a later call keeps the intersection.  Runs the
 * first rs_score if none ran yet; res as for rs_apply_removals (all zero when
 * k_c covers every community).  Errors: RS_ERR_ARG for k_c < 1, RS_ERR_STATE
 * on a batch.  Waits for the stream.
 */
rs_status rs_restrict_to_targets(rs_graph *g, int32_t k_c, rs_removal_result *res);

/*
 * Reachable communities, for the absolute AWCC of the robustness experiments
 * (Section VII-B: the average of |zeta(v)| / d(v) over a vertex set, where
 * after a disruption only |zeta(v)| is recomputed, over the paths the
 * disrupted graph still has).  For each of the n_sources source vertices
 * (caller ids, at most 1,024), counts[i] = the number of distinct communities
 * among the vertices other than the source in the source's connected
 * component of the current graph (after every removal applied so far); a
 * removed or isolated source gets 0.  Host arrays; waits for the stream.
 * Errors: RS_ERR_ARG (NULL arrays, n_sources outside 0..1024), RS_ERR_RANGE
 * (a source id >= n).  Valid on a batch too (components never span graphs).
 */
rs_status rs_reachable_communities(rs_graph *g, int64_t n_sources, const int32_t *sources, int64_t *counts);

/*
 * rs_reachable_communities_static: rs_reachable_communities for callers that
 * cannot allocate (code under HIP stream capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and errors; it
 * calls no hipMalloc, hipFree or other allocating routine.  Its device
 * memory is one static array of 32 MiB per device, loaded with the library
 * and held until the process ends: the component labels (4 bytes per
 * vertex), one community bitmap per source (4 * ceil(k / 32) bytes, k the
 * number of communities) and the sources and counts.  A graph that needs
 * more is refused with RS_ERR_RANGE before anything runs.  Every call on one
 * device shares that device's array (it keeps the last call's contents; each
 * call clears what it reads), so calls that overlap on one device race: the
 * caller serialises them.  Host arrays; waits for the graph's stream.
 */
rs_status rs_reachable_communities_static(rs_graph *g, int64_t n_sources, const int32_t *sources, int64_t *counts);

/*
 * rs_read_scores: out[n] host array, indexed by caller vertex id.
 *   raw = 0: R(u) of Algorithm 1 (every triad term divided by w_max);
 *   raw = 1: the sum of Eq. RSI without the w_max division (= R * w_max).
 * Waits for the stream.
 */
rs_status rs_read_scores(rs_graph *g, double *out, int64_t n, int32_t raw);

typedef struct {
    int64_t n;              /* vertices */
    int64_t nnz;            /* live CSR entries (2 |E|) */
    int64_t n_alive;        /* vertices not removed */
    int64_t n_communities;  /* distinct labels */
    int64_t n_border;       /* |V_b| */
    int64_t m_inter;        /* inter-community edges = |E(G')| / 2 */
    int64_t sum_ell;        /* stored interaction-matrix entries = sum of distinct neighbour communities */
    int64_t sum_ell_x;      /* entries whose community is not the vertex's own */
    int64_t sum_tI;         /* ordered type-I triads over all vertices */
    int64_t sum_tII;        /* type-II triads over all vertices */
    int64_t sum_work_I;     /* list elements scanned by the type-I intersections */
    double omega_max;       /* w_max of the last pass */
} rs_counts;

/* rs_read_counts: totals of the last rs_score.  Waits for the stream. */
rs_status rs_read_counts(rs_graph *g, rs_counts *c);

/*
 * rs_read_vertex_counts: per-vertex integer results of the last pass, host
 * arrays of length n indexed by caller id; any pointer may be NULL.
 *   border  1 if the vertex has a neighbour in another community (Step 1)
 *   ell     distinct communities among its neighbours (the interaction-matrix row length)
 *   dprime  neighbours in other communities (its degree in G')
 *   tI, tII ordered type-I / type-II triads counted at the vertex
 *   w_own   w_v(C(v)), the vertex's weight toward its own community (Lemma 2)
 */
rs_status rs_read_vertex_counts(rs_graph *g, int32_t *border, int32_t *ell, int32_t *dprime,
                                int64_t *tI, int64_t *tII, double *w_own);

/*
 * rs_read_rows: the sparse interaction matrix of the last pass (Section
 * VI-A), one row per vertex in caller id order and entries sorted by caller
 * community label: row_off[n+1] (host), then comm / count / weight arrays of
 * row_off[n] entries each.  Call first with comm == NULL to get row_off only.
 */
rs_status rs_read_rows(rs_graph *g, int64_t *row_off, int32_t *comm, int32_t *count, double *weight);

/*
 * rs_read_gprime: the inter-community subgraph G' (Section VI-B: edges
 * (u,v) in E with C(u) != C(v)) as CSR in caller ids with ascending rows:
 * off[n+1], then col[off[n]].  Call with col == NULL to get off only.
 */
rs_status rs_read_gprime(rs_graph *g, int64_t *off, int32_t *col);

/*
 * Kernel timing.  rs_set_timing(g, 1) makes rs_score / rs_topk record HIP
 * events around every kernel on the graph's stream; rs_read_timings waits
 * for the stream, returns for each kernel id i < cap the summed
 * milliseconds ms[i] and launch count launches[i], and resets the sums.
 * rs_kernel_name(i) names kernel id i (NULL past the last one).
 */
rs_status rs_set_timing(rs_graph *g, int32_t on);
rs_status rs_read_timings(rs_graph *g, int32_t cap, double *ms, int64_t *launches, int32_t *n_kernels);
const char *rs_kernel_name(int32_t id);

/*
 * Batched scoring: many independent graphs scored together.  The batch is
 * one CSR over the disjoint union of the graphs: graph i owns the vertex
 * range [vertex_offsets[i], vertex_offsets[i+1]) (n_graphs + 1 offsets, from
 * 0 to csr->n; host arrays only), its edges stay inside that range (global
 * ids), and its labels are its own (graphs may reuse label values: no
 * community spans two graphs).  rs_score scores the whole batch in one pass
 * with each graph's own w_max (Algorithm 1, Step 2, per graph), so every
 * score equals that of the graph loaded alone, bit for bit.
 *   rs_load_batch   as rs_load_graph; RS_ERR_GRAPH also for an edge that
 *                   joins two graphs
 *   rs_topk_batch   the top-k of every graph (1 <= k <= 32): ids[i*k + j]
 *                   and scores[i*k + j] for graph i, ids relative to the
 *                   graph's first vertex, in the order of rs_topk; counts[i]
 *                   = min(k, live vertices of graph i).  Waits for the stream.
 * rs_apply_removals refuses a batch (RS_ERR_STATE).
 */
rs_status rs_load_batch(int32_t n_graphs, const int64_t *vertex_offsets, const rs_csr *csr, void *hip_stream,
                        uint32_t flags, rs_graph **out);
rs_status rs_topk_batch(rs_graph *g, int64_t k, int32_t *ids, double *scores, int64_t *counts);

/* rs_free_graph: release all device memory of g (NULL is ignored). */
/*
 * The static schedule's cut-offs (the degree bins of the pass): a row tile
 * covers consecutive vertices with at most row_entries row entries and
 * row_vertices vertices, and a longer row is a hub row with a workgroup of
 * its own; a score tile covers at most score_pairs foreign entries (pairs of
 * G') and score_vertices vertices, and a vertex with more foreign entries is
 * a score hub whose pairs are cut into chunks of 256 (one workgroup each),
 * with its foreign list staged in LDS when it has at most hub_list entries.
 * Every graph is loaded with the defaults (2048, 512, 256, 256, 1024), which
 * are also the largest values (row_entries at least 64).  This is the load
 * balance of the parallel algorithm's kernels (Section VI-B, grid-stride
 * kernels over vertices and edges; Section VI-C, the cost of skewed degrees).
 *
 * rs_get_tiling reads a graph's cut-offs.  rs_set_tiling re-cuts its schedule
 * (host work over n, and the schedule's device arrays are replaced); the
 * graph must then be scored again (RS_ERR_STATE from the readers until
 * rs_score).  Scores and counts do not depend on the cut-offs, except that
 * vertices that change between tile and hub sum their terms in another
 * order (the same values within rounding).  Errors: RS_ERR_ARG (a value out
 * of range).
 *
 * rs_autotune: the project's autotuner.  It cuts the schedule for each of the
 * n_cand candidates in turn, runs one untimed pass and then `reps` timed
 * passes (HIP events on the graph's stream), writes each candidate's mean
 * pass time in milliseconds to ms[i], and keeps the fastest (its index in
 * *best).  A graph scored before the call is scored again with the chosen
 * cut-offs.  Host arrays; waits for the stream.
 */
typedef struct {
    int32_t row_entries, row_vertices, score_pairs, score_vertices, hub_list;
} rs_tiling;
rs_status rs_get_tiling(rs_graph *g, rs_tiling *t);
rs_status rs_set_tiling(rs_graph *g, const rs_tiling *t);
rs_status rs_autotune(rs_graph *g, int32_t n_cand, const rs_tiling *cand, int32_t reps, int32_t *best, double *ms);

void rs_free_graph(rs_graph *g);

/*
 * Served scoring: a request loop over several resident graphs (the removal
 * model of Section VII-B applied as a stream of requests).  The server keeps a
 * host copy of each registered graph and loads it into device memory on its
 * first request, within an HBM budget: when a graph does not fit, idle graphs
 * are evicted least-recently-used first (an evicted graph is reloaded from
 * the validated, renumbered host form its first load built, with its removal
 * history applied).  n_slots worker threads
 * take requests in submission order; requests on one graph run one at a time
 * in that order, requests on different graphs overlap on the device (each
 * graph has its own stream).  A request applies a removal batch (incremental
 * re-score, as rs_apply_removals) and returns the top-k; its result equals
 * applying the graph's batches one by one to a lone rs_graph.
 *
 *   rs_server_create      n_slots >= 1 workers; hbm_budget bytes of device
 *                         memory for resident graphs (<= 0: unlimited)
 *   rs_server_add_graph   copies the CSR (host arrays only) and returns its
 *                         id (0, 1, ...); nothing is loaded yet
 *   rs_server_submit      copies the batch; returns a request id at once
 *   rs_server_wait        blocks until the request is done; ids[k] and
 *                         scores[k] receive its top-k (count of them), info
 *                         its timings (ns since the server started) and the
 *                         re-score's counts; the request is then forgotten
 *   rs_server_stats       loads, evictions, requests done, device bytes
 * Errors: RS_ERR_ARG, RS_ERR_RANGE (graph id or vertex id), RS_ERR_GRAPH,
 * RS_ERR_NOMEM (a graph larger than the whole budget), RS_ERR_HIP; a failed
 * request reports its status through rs_server_wait.
 */
typedef struct rs_server rs_server;
typedef struct {
    int64_t t_submit, t_start, t_done; /* ns since rs_server_create */
    int64_t affected;                  /* vertices re-scored by the removal */
    int64_t edges_removed;
    int32_t loaded;                    /* 1 if the graph was (re)loaded for this request */
    int32_t pad;
} rs_request_info;
typedef struct {
    int64_t requests_done, loads, evictions, device_bytes, peak_device_bytes;
} rs_server_stats_t;
rs_status rs_server_create(int32_t n_slots, int64_t hbm_budget, rs_server **out);
rs_status rs_server_add_graph(rs_server *s, const rs_csr *csr, int32_t *graph_id);
rs_status rs_server_submit(rs_server *s, int32_t graph_id, const rs_removals *batch, int64_t k, int64_t *request_id);
rs_status rs_server_wait(rs_server *s, int64_t request_id, int32_t *ids, double *scores, int64_t *count,
                         rs_request_info *info);
rs_status rs_server_stats(rs_server *s, rs_server_stats_t *st);
void rs_server_free(rs_server *s);


const char *rs_status_string(rs_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char *rs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RS_H */
