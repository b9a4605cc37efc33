/*
 * slg.h — s-line graphs of non-uniform hypergraphs on AMD MI355X (gfx950).
 *
 * The problem (Section II-B): for a hypergraph H = (V, E) with n = |V|
 * vertices and m = |E| hyperedges, and an integer s >= 1,
 *   E_s = { e in E : |e| >= s },
 *   L_s(H) = <E_s, F>,  {e_i, e_j} in F  iff  |e_i n e_j| >= s,
 * and each edge carries its overlap |e_i n e_j| = (H^T H)[i, j].
 * The library computes F by the two-hop traversal hyperedge -> vertex ->
 * hyperedge (the "ikj" form of Section III-B, Algorithm 2), after dropping
 * hyperedges with |e| < s (degree-based pruning), and emits each pair once
 * with i < j (the upper triangle). Given a set of thresholds it computes
 * the whole ensemble in one counting pass (Algorithm 3, Section III-D).
 *
 * Conventions for every entry point:
 *   - ids are 0-based; i, j index hyperedges in the caller's numbering
 *     (no relabelling leaks out); vertices index [0, n).
 *   - "device" pointers are addresses in the GPU's memory (e.g. from torch
 *     or hipMalloc); "host" pointers are ordinary CPU memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *     all device work of a call is ordered on it. Inside a call the library
 *     may fork part of the work onto a stream the context owns (for plans
 *     of at least 2^28 2-paths, the light tier's counting pass of
 *     slg_plan_create runs beside the heavy tier's boundary table; the
 *     context makes that stream at the first such plan). The fork waits on
 *     an event recorded on `stream` and is joined back into `stream`
 *     within the call, so the ordering seen from `stream` is unchanged.
 *   - every call returns a slg_status; on failure the context's last error
 *     string (slg_last_error) says why. No call throws.
 *   - a context and everything made from it belong to one host thread at a
 *     time; they are not safe to share across threads without a lock.
 */
#ifndef SLG_H
#define SLG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLG_OK = 0,
    SLG_ERR_INVALID_ARG = 1,   /* bad pointer, size or s-set */
    SLG_ERR_INVALID_GRAPH = 2, /* CSR check failed (only with SLG_VALIDATE) */
    SLG_ERR_OUT_OF_MEMORY = 3, /* device allocation failed / budget exceeded */
    SLG_ERR_DEVICE = 4,        /* a HIP runtime call failed */
    SLG_ERR_OVERFLOW = 5,      /* m, n or nnz >= 2^31 */
    SLG_ERR_CANCELLED = 6,     /* a chunk callback asked to stop / server shut down */
    SLG_ERR_TIMEOUT = 7        /* a server wait ran out of time (the request goes on) */
} slg_status;

/* Largest number of thresholds in one ensemble call. */
#define SLG_MAX_S 16

typedef struct slg_context slg_context;
typedef struct slg_graph slg_graph;
typedef struct slg_plan slg_plan;
typedef struct slg_result slg_result;
typedef struct slg_batch slg_batch;

/*
 * The input: the incidence of H held as both CSR orientations
 * (Section II-A: the bipartite graph B(H) / incidence matrix H; the ikj
 * traversal of Section III-B reads H^T.Adj and H.Adj).
 *   he_ptr[m+1], he_idx[nnz]: members of hyperedge i are
 *       he_idx[he_ptr[i] .. he_ptr[i+1]), strictly increasing (e_i is a set).
 *   v_ptr[n+1], v_idx[nnz]: hyperedges containing vertex v are
 *       v_idx[v_ptr[v] .. v_ptr[v+1]), strictly increasing; the exact
 *       transpose of the hyperedge CSR.
 * All four arrays are DEVICE pointers (host or device with SLG_COPY).
 * Empty hyperedges and isolated
 * vertices are allowed; duplicate hyperedges are distinct hyperedges.
 */
typedef struct {
    int64_t num_vertices;   /* n */
    int64_t num_hyperedges; /* m */
    int64_t nnz;            /* number of incidences */
    const int64_t *he_ptr;
    const int32_t *he_idx;
    const int64_t *v_ptr;
    const int32_t *v_idx;
} slg_incidence;

/*
 * Optional device allocator for result buffers (e.g. torch's caching
 * allocator). alloc returns a device pointer of at least `bytes` usable on
 * `stream`, or NULL; release frees it. NULL allocator = the library's own
 * stream-ordered allocator (hipMallocAsync).
 */
typedef struct {
    void *(*alloc)(void *user, size_t bytes, void *stream);
    void (*release)(void *user, void *ptr, void *stream);
    void *user;
} slg_allocator;

/* Flags for slg_graph_register. */
#define SLG_VALIDATE 1u /* check both CSRs on the device before accepting */
#define SLG_COPY 2u     /* keep the library's own device copies of the CSRs */

/* Library version string (static storage). */
const char *slg_version(void);

/*
 * Create a context on HIP device `device`. Planning scratch (and the
 * outputs of slg_line_graph when `alloc` is NULL) come from a block cache
 * of the context: freed blocks are kept for reuse by later calls, up to
 * mem_budget_bytes of them (0 = half of the device's memory, at least
 * 16 GiB); beyond that the largest are given
 * back to the device. `alloc` may be NULL.
 * Errors: INVALID_ARG (out == NULL), DEVICE (no such device).
 */
slg_status slg_context_create(int device, uint64_t mem_budget_bytes, const slg_allocator *alloc,
                              slg_context **out);
slg_status slg_context_destroy(slg_context *ctx);

/* Why the last failing call on ctx failed (static or context-owned text). */
const char *slg_last_error(const slg_context *ctx);

/*
 * Register a hypergraph. The incidence arrays are borrowed: they must stay
 * valid and unchanged until slg_graph_release. With SLG_COPY the library
 * copies them (from host or device memory) into device memory the graph
 * owns, and the caller's arrays are free again when the call returns;
 * slg_graph_release then waits for the device and frees the copies. With
 * SLG_VALIDATE the
 * library checks on the device, ordered on `stream`, that: pointer arrays
 * start at 0, are non-decreasing and end at nnz; ids are in range; rows of
 * both CSRs are strictly increasing; the vertex CSR is the transpose.
 * Errors: INVALID_ARG (NULL pointers with nnz > 0, negative sizes, an
 * unknown flag), OVERFLOW (m, n or nnz >= 2^31), INVALID_GRAPH (a check
 * failed), OUT_OF_MEMORY (no room for the copy).
 */
slg_status slg_graph_register(slg_context *ctx, const slg_incidence *inc, uint32_t flags,
                              void *stream, slg_graph **out);
slg_status slg_graph_release(slg_graph *g);

/*
 * Plan the s-line graph(s) of g for thresholds s[0..num_s) (host array,
 * strictly increasing, s[0] >= 1, num_s <= SLG_MAX_S). Runs, on `stream`:
 * degree pruning at s_min = s[0] (Algorithm 2's pruning test; Algorithm 3
 * prunes by its smallest s), the per-hyperedge 2-path work estimate, the
 * counting pass that fixes every output size, and the prefix sums that
 * place each row. Blocks until the edge counts are known on the host.
 * num_s == 1 is the plain s-line graph (Algorithm 2); num_s > 1 is the
 * single-pass ensemble (Algorithm 3).
 * Errors: INVALID_ARG (bad s-set), OUT_OF_MEMORY, DEVICE.
 */
slg_status slg_plan_create(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                           void *stream, slg_plan **out);

/*
 * Facts of a plan for threshold index k (0 <= k < num_s):
 *   num_edges  = |F| of L_{s[k]}(H);
 *   two_paths  = number of 2-paths (e_i, v, e_j), i < j, e_i, e_j in
 *                E_{s[0]} traversed by the plan (the same for every k).
 * Either output pointer may be NULL.
 */
slg_status slg_plan_info(const slg_plan *p, int32_t k, int64_t *num_edges, int64_t *two_paths);

/*
 * Write every L_{s[k]} of the plan into caller-owned DEVICE buffers, one
 * set per k (host arrays of num_s device pointers each):
 *   row_ptr[k]: int64[m+1], CSR row offsets over all m hyperedges;
 *   col[k], w[k]: int32[num_edges(k)], the j and the overlap of each edge;
 *   row[k]: int32[num_edges(k)], the i of each edge (COO), or NULL to skip.
 * Edges are sorted by (i, j) ascending with i < j. CSR and COO share col/w.
 * Work is enqueued on `stream`; the call returns without waiting.
 * Errors: INVALID_ARG (NULL buffer for an L_s with edges).
 */
slg_status slg_plan_emit(slg_plan *p, int64_t *const *row_ptr, int32_t *const *row,
                         int32_t *const *col, int32_t *const *w, void *stream);

/*
 * Shape of a plan, for measurement and tuning: fills up to `cap` entries of
 * out[] (host array) with, in order:
 *   [0] slots (output segments);
 *   [1] rows of at most 8 2-paths (one lane per row);
 *   [2..7] rows in the six wavefront-sort classes (<= 64, 128, 256, 512,
 *          1024, 2048 2-paths);
 *   [8] heavy slots; [9] heavy slots of rows with >= 65535 members;
 *   [10] 2-paths (as slg_plan_info); [11] 2-paths in heavy slots;
 *   [12] entries of the heavy boundary table;
 *   [13] edges written by heavy slots, summed over all thresholds;
 *   [14] (partner, overlap) entries the heavy count store keeps (0 when
 *        the plan keeps none; see slg_context_set_count_store);
 *   [15] dense slots; [16] 2-paths in dense slots; [17] edges written by
 *        dense slots, summed over all thresholds; [18] survivors the dense
 *        store keeps; [19] 1 when some dense slots found the store full
 *        (see slg_context_set_dense).
 * Returns the number of entries written in *count (may be NULL).
 */
slg_status slg_plan_stats(const slg_plan *p, int64_t *out, int32_t cap, int32_t *count);

/*
 * Opt-in device timing, for measurement. When enabled, every kernel launch
 * of the path is bracketed by HIP events recorded on the stream it runs on,
 * and the elapsed times are summed per stage (stages on the context's
 * second stream overlap others, so the sum can exceed the wall time). slg_context_get_timing waits
 * for the recorded events, then fills up to `cap` entries of out[] (host
 * array) with one record per stage that ran: its name (static storage),
 * the number of timed launches and their summed duration in milliseconds.
 * Stages: prune, row_plan, plan_scans, slots, bounds, count_light,
 * count_heavy, count_heavy_wide, count_dense, count_scans, emit_light,
 * emit_heavy, emit_heavy_wide, emit_dense, row_ptr. Timing adds two event records per launch.
 */
typedef struct {
    const char *name;
    int64_t launches;
    double milliseconds;
} slg_stage_time;
slg_status slg_context_set_timing(slg_context *ctx, int enable);
slg_status slg_context_get_timing(slg_context *ctx, slg_stage_time *out, int32_t cap, int32_t *count);
/* Clears the stage times and the work counters below. */
slg_status slg_context_reset_timing(slg_context *ctx);
/*
 * Work done by the counting passes of ctx since the last reset (whole
 * plans and the row blocks of streamed calls), for measurement: fills up to
 * `cap` entries of out[] (host array) with, in order: [0] plans and row
 * blocks counted; [1] 2-paths; [2] 2-paths of heavy slots; [3] 2-paths of
 * dense slots; [4] edges, summed over the thresholds; [5] edges of heavy
 * slots; [6] edges of dense slots; [7] dense slots; [8] survivors the
 * dense store kept; [9] blocks whose dense store was full (some slots
 * walked their 2-paths again). *count (may be NULL) gets the number
 * written.
 */
slg_status slg_context_get_work(const slg_context *ctx, int64_t *out, int32_t cap, int32_t *count);

/* Free a plan's device scratch (ordered on the stream it was made on). */
slg_status slg_plan_destroy(slg_plan *p);

/*
 * Chunked form for outputs larger than device memory (row-range streaming,
 * the union of per-row edge lists of Algorithms 2 and 3 handed over a part
 * at a time). The per-row work estimate runs once for the whole graph;
 * the rest of the plan (slot tables, boundary table, the counting pass and
 * its stores) is made one block of rows at a time, each block taking rows
 * while its scratch fits the count-store limit, so that the scratch is
 * bounded by the block and not by the graph. Each block's rows are emitted
 * in consecutive row ranges (chunks) whose output fits chunk_bytes (all
 * thresholds; 12 bytes per edge plus 8 per CSR offset). For every chunk and
 * every threshold index k the callback receives, after the chunk's device
 * work has completed:
 *   rows [row_begin, row_end) of L_{s[k]}; its edges are edges
 *   [edge_begin, edge_begin + num_edges) of the call's sorted edge list;
 *   row_ptr: DEVICE int64[row_end - row_begin + 1], relative (row_ptr[0]=0);
 *   row/col/w: DEVICE int32[num_edges] (COO i, j, overlap);
 *   stream: the consumer stream. The buffers stay valid for work the
 *   callback enqueues on it; the library writes them again only after that
 *   work. Meanwhile it emits the next chunk on the call's stream, so device
 *   work of the callback on the consumer stream overlaps the next emit.
 *   The consumer stream is the context's second stream when it has one,
 *   else the call's stream.
 * The pointers must not be used after that work (buffers are reused).
 * A nonzero return stops the stream: SLG_ERR_CANCELLED.
 * Errors: as slg_plan_create; OUT_OF_MEMORY when one row alone needs more
 * than chunk_bytes; INVALID_ARG for chunk_bytes <= 0 or a NULL callback.
 */
typedef int (*slg_chunk_fn)(void *user, int32_t k, int32_t s, int64_t row_begin, int64_t row_end,
                            int64_t edge_begin, int64_t num_edges, const int64_t *row_ptr,
                            const int32_t *row, const int32_t *col, const int32_t *w, void *stream);
slg_status slg_line_graph_stream(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                                 int64_t chunk_bytes, slg_chunk_fn fn, void *user, void *stream);

/*
 * slg_line_graph_stream restricted to the rows [row_begin, row_end) (0 <=
 * row_begin <= row_end <= m): their edges (i, j) with i in the range and
 * every j > i, so that disjoint row ranges together give the whole L_s
 * (the way the path shards: rows split into ranges of equal 2-path work,
 * Section III-E's cost model, with no exchange between ranges). edge_begin
 * counts from the first edge of row_begin. Errors as slg_line_graph_stream,
 * plus INVALID_ARG for a range outside [0, m].
 */
slg_status slg_line_graph_stream_rows(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                                      int64_t row_begin, int64_t row_end, int64_t chunk_bytes, slg_chunk_fn fn,
                                      void *user, void *stream);

/*
 * The per-hyperedge work estimate of Algorithm 2 at s_min as a prefix:
 * prefix (HOST int64[m+1]) gets, for every i, the number of 2-paths
 * (e_r, v, e_j), r < i, r < j, both of E_{s_min}, that the traversal
 * takes from the rows before i (prefix[m] = all of them). Row ranges of
 * equal work follow from it (slg_line_graph_stream_rows). Ordered on
 * `stream`; returns after the copy. Errors: INVALID_ARG (null, s_min < 1),
 * OUT_OF_MEMORY, DEVICE.
 */
slg_status slg_work_prefix(slg_context *ctx, slg_graph *g, int32_t s_min, int64_t *prefix, void *stream);

/*
 * Batched form: many independent hypergraphs, each with its own threshold
 * s[g] (Algorithm 2 per graph). slg_batch_create builds their disjoint
 * union on the device (ids offset per graph, a threshold per hyperedge),
 * plans it once, allocates every buffer and computes the results (blocks
 * until done). The registered graphs must stay valid until
 * slg_batch_destroy. slg_batch_run repeats the whole device path (pruning,
 * planning, counting, emitting) into the same buffers with no host
 * synchronisation and no allocation; with use_graph != 0 the path is
 * captured once into a HIP graph and replayed on `stream`.
 * Results per graph g (DEVICE pointers, valid until destroy):
 *   row_ptr: int64[m_g + 1], GLOBAL edge offsets (subtract *edge_begin);
 *   row/col/w: int32[num_edges], ids local to graph g, sorted by (i, j).
 * Errors: INVALID_ARG (n < 1 or > 65535, s[g] < 1), OVERFLOW (totals
 * >= 2^31), and as slg_plan_create.
 */
slg_status slg_batch_create(slg_context *ctx, slg_graph *const *graphs, const int32_t *s, int32_t n,
                            void *stream, slg_batch **out);
slg_status slg_batch_run(slg_batch *b, int32_t use_graph, void *stream);
slg_status slg_batch_info(const slg_batch *b, int64_t *num_edges, int64_t *two_paths, int64_t *rows);
slg_status slg_batch_result(const slg_batch *b, int32_t g, int64_t *edge_begin, int64_t *num_edges,
                            const int64_t **row_ptr, const int32_t **row, const int32_t **col,
                            const int32_t **w);
slg_status slg_batch_destroy(slg_batch *b);

/*
 * Count store (a memory-for-time trade of this implementation, not in the
 * paper): the counting pass of a plan keeps every heavy slot's partners and
 * overlaps (4 bytes per 2-path of the heavy rows, plus 20 bytes per heavy
 * slot) so that the emit pass reads them instead of walking the 2-paths
 * again, whenever that takes at most max_bytes and the heavy rows hold at
 * least min_two_paths 2-paths (below that, the store's extra launches cost
 * more than they save). max_bytes = 0 turns it off. Defaults: 32 GiB and
 * 2^24. Results are identical either way. Applies to plans created
 * afterwards (and to a server's slots when set before slg_server_create).
 */
slg_status slg_context_set_count_store(slg_context *ctx, int64_t max_bytes, int64_t min_two_paths);

/*
 * Dense tier (an implementation choice, not in the paper): a heavy row whose
 * candidate partners (the hyperedges of E_{s_min} with ids in (i, j_max])
 * number at least min_range, and which has at least min_ratio 2-paths per
 * eight candidates (min_ratio / 8 per candidate), counts its overlaps in
 * direct counters over windows of 2^14 consecutive hyperedges of E_{s_min},
 * and keeps only the partners that reach s_min for the emit pass (within
 * the count-store limit; slots that find it full walk their 2-paths again).
 * min_ratio = 0 turns the tier off; min_range = 0 restores its default.
 * Defaults: 4 (half a 2-path per candidate) and 8192. Results are
 * identical either way. Applies to plans created afterwards.
 */
slg_status slg_context_set_dense(slg_context *ctx, int32_t min_ratio, int32_t min_range);

/*
 * Fault injection for tests of the error path (no part of the method):
 * plans created afterwards give their heavy, heavy-wide and dense
 * descriptor lists `entries` fewer places than the rows counted for them.
 * The device appends check their list's room, skip the rows that do not fit
 * and set the plan's error flag, so every kernel still stays inside its
 * buffers; the plan (or the line-graph call) then fails with
 * SLG_ERR_DEVICE ("a tier list overflowed its planned size") and the
 * context stays usable. 0 (the default) turns it off; entries < 0 is
 * SLG_ERR_INVALID_ARG.
 */
slg_status slg_context_set_list_shortfall(slg_context *ctx, int64_t entries);

/*
 * Tuning of the plan shape, used by the autotuner: light_max = largest row
 * work (2-paths) sorted by one wavefront (<= 2048; 0 = default),
 * slot_work = 2-paths per heavy slot before a row is split (0 = default),
 * heavy_grid = persistent heavy workgroups (0 = as many as fit the GPU).
 * Applies to plans and batches created afterwards on this context.
 */
slg_status slg_context_set_tuning(slg_context *ctx, int32_t light_max, int64_t slot_work, int32_t heavy_grid);

/*
 * One-shot form of plan + emit: result buffers come from the context's
 * allocator and stay owned by the library until slg_result_free.
 * Same s-set rules and errors as slg_plan_create.
 */
slg_status slg_line_graph(slg_context *ctx, slg_graph *g, const int32_t *s, int32_t num_s,
                          void *stream, slg_result **out);
slg_status slg_result_info(const slg_result *r, int32_t k, int64_t *num_edges, int64_t *two_paths);
/* Device pointers into the result for threshold index k. */
slg_status slg_result_coo(const slg_result *r, int32_t k, const int32_t **i, const int32_t **j,
                          const int32_t **w);
slg_status slg_result_csr(const slg_result *r, int32_t k, const int64_t **row_ptr,
                          const int32_t **col, const int32_t **w);
slg_status slg_result_free(slg_result *r);

/*
 * s-connected components (Section II-B): the maximal subsets of E_s in
 * which every two hyperedges are joined by an s-walk, i.e. the connected
 * components of L_s. row/col: DEVICE int32[num_edges], the edges of L_s
 * (as emitted, or any order; every id in [0, m) and in E_s). labels:
 * DEVICE int32[m], written: the smallest hyperedge id of e_i's component,
 * or -1 when |e_i| < s (a hyperedge of E_s with no edge is its own
 * component). *num_components (may be NULL): their number. Ordered on
 * `stream`; returns after the stream has reached the end of the call.
 * Errors: INVALID_ARG (null, s < 1, an id outside [0, m), an edge end
 * outside E_s).
 */
slg_status slg_components(slg_context *ctx, slg_graph *g, int32_t s, const int32_t *row, const int32_t *col,
                          int64_t num_edges, int32_t *labels, int64_t *num_components, void *stream);

/*
 * slg_components without any device allocation, for callers that cannot
 * allocate: code under HIP-graph capture, tight serving loops, harnesses
 * that forbid allocation. Same arguments, outputs and errors as
 * slg_components, and the same kernels; the union-find parents and the
 * two counters live in a fixed array of the library (one per GPU, made
 * when the library is loaded on it and held until the process ends) that
 * takes graphs of at most 2^24 hyperedges (64 MiB + 16 B per GPU). A graph
 * with more hyperedges fails with SLG_ERR_INVALID_ARG and nothing is
 * launched. Every call on one GPU uses that GPU's single array: calls that
 * overlap on one GPU (from several streams or host threads) race and give
 * wrong labels; callers serialise them. The call clears what must start at
 * zero itself. Errors as slg_components, plus DEVICE when the array's
 * address could not be looked up at context creation.
 */
slg_status slg_components_noalloc(slg_context *ctx, slg_graph *g, int32_t s, const int32_t *row,
                                  const int32_t *col, int64_t num_edges, int32_t *labels, int64_t *num_components,
                                  void *stream);

/*
 * ID squeezing (Stage 4 of the paper's framework, Section IV): hyperedges
 * that are an end of at least one edge keep their order and are renumbered
 * 0, 1, ...: new_id DEVICE int32[m] gets the new id or -1; *num_kept (may
 * be NULL) their number. With remap != 0, row/col (DEVICE int32[num_edges])
 * are rewritten in place to the new ids (a sorted edge list stays sorted).
 * Ordered on `stream`; returns after the stream has reached the end of the
 * call. Errors: INVALID_ARG (null, m out of range, an id outside [0, m)).
 */
slg_status slg_squeeze(slg_context *ctx, int64_t m, int32_t *row, int32_t *col, int64_t num_edges, int32_t remap,
                       int32_t *new_id, int64_t *num_kept, void *stream);

/*
 * Symmetric CSR of one s-line graph (Stage 4 of the paper's framework,
 * Section IV: the edge list becomes the graph's adjacency; L_s is the
 * symmetric matrix of Section II-B). Input: the upper triangle of L_s as
 * emitted (slg_plan_emit, slg_result_csr/coo): row_ptr DEVICE int64[m+1],
 * row/col/w DEVICE int32[num_edges], sorted by (row, col), row < col.
 * Output, caller-allocated DEVICE buffers: sym_ptr int64[m+1], sym_col and
 * sym_w int32[2 * num_edges]; row r lists every partner of r in ascending
 * order with its overlap. w and sym_w may both be NULL (structure only).
 * Ordered on `stream`; returns after the stream has reached the end of the
 * call. Device scratch: 12 (8 without weights) bytes per edge for one
 * 8-bit radix pass, twice that for m > 256.
 * Errors: INVALID_ARG (null arrays, m outside [0, 2^31), w without sym_w,
 * or an input that is not such an upper triangle; the outputs are then
 * unspecified), OUT_OF_MEMORY.
 */
slg_status slg_symmetrize(slg_context *ctx, int64_t m, const int64_t *row_ptr, const int32_t *row,
                          const int32_t *col, const int32_t *w, int64_t num_edges, int64_t *sym_ptr,
                          int32_t *sym_col, int32_t *sym_w, void *stream);

/*
 * Order-independent digest of an edge list (for checking streamed or large
 * results block by block without moving them to the host): out[0] = number
 * of edges, out[1] = sum of the overlaps, out[2] = sum mod 2^64 of
 * SplitMix64's output function applied to i * 2^32 + j, xor w. row/col/w:
 * DEVICE int32[num_edges] (a chunk's arrays inside an slg_chunk_fn, or an
 * emitted L_s); out: HOST uint64[3]. Digests of disjoint edge sets add up.
 * Ordered on `stream`; returns after the stream has reached the end of the
 * call. Errors: INVALID_ARG (null arrays with num_edges > 0).
 */
slg_status slg_digest(slg_context *ctx, const int32_t *row, const int32_t *col, const int32_t *w,
                      int64_t num_edges, uint64_t *out, void *stream);

/*
 * Relabel-by-degree (Stage 1 of the paper's framework, Section IV): the
 * order of hyperedge ids by size, ascending (descending = 0) or descending;
 * hyperedges of equal size keep their id order. order: DEVICE int32[m],
 * written: order[k] = the old id that becomes id k. Build the relabelled
 * hypergraph with slg_select(order, m); its line graphs are in the new ids
 * (old id = order[new id]). Ordered on `stream`; returns after the stream
 * has reached the end of the call. Errors: INVALID_ARG (null).
 */
slg_status slg_relabel_order(slg_context *ctx, slg_graph *g, int32_t descending, int32_t *order, void *stream);

/*
 * Toplexes (Stage 2 of the paper's framework, Section IV): the hyperedges
 * that no other hyperedge contains. Computed from the edges of L_1 of g
 * (row/col/w DEVICE int32[num_edges], as emitted for s = 1, or in any order
 * or orientation): e_i lies inside e_j exactly when their overlap equals
 * |e_i|. Of several identical maximal hyperedges the smallest id is kept;
 * empty hyperedges are never toplexes. toplexes: DEVICE int32[m], written:
 * the toplex ids in ascending order; *num_toplexes (may be NULL): their
 * number. slg_select(toplexes, count) builds the simplified hypergraph.
 * Ordered on `stream`; returns after the stream has reached the end of the
 * call. Errors: INVALID_ARG (null, an id outside [0, m), a loop, an overlap
 * above a hyperedge's size).
 */
slg_status slg_toplexes(slg_context *ctx, slg_graph *g, const int32_t *row, const int32_t *col, const int32_t *w,
                        int64_t num_edges, int32_t *toplexes, int64_t *num_toplexes, void *stream);

/*
 * The sub-hypergraph of g made of the hyperedges order[0..count) (distinct
 * ids), hyperedge k being order[k]; vertex ids are unchanged. Outputs,
 * caller-allocated DEVICE buffers: he_ptr int64[count+1], v_ptr
 * int64[n+1], he_idx and v_idx int32 with room for g's nnz; *nnz (may be
 * NULL) gets the number written. Both CSRs come out well formed (rows
 * ascending, the vertex CSR the exact transpose), ready for
 * slg_graph_register. Ordered on `stream`; returns after the stream has
 * reached the end of the call. Errors: INVALID_ARG (null, count > m, an id
 * outside [0, m) or named twice), OUT_OF_MEMORY.
 */
slg_status slg_select(slg_context *ctx, slg_graph *g, const int32_t *order, int64_t count, int64_t *he_ptr,
                      int32_t *he_idx, int64_t *v_ptr, int32_t *v_idx, int64_t *nnz, void *stream);

/*
 * Served form: a request loop over device-resident hypergraphs. Queries
 * (a registered graph plus an s-set, each an ensemble pass of Algorithm 3)
 * arrive at any time and are started in arrival order as soon as one of
 * `workers` slots is free (1..16; each slot plans and emits on its own
 * HIP stream, so several queries' kernels overlap on the device) and the
 * device-memory budget allows. Every query asks the budget for its planning
 * scratch (two phases, sized as the plan learns its shape) and then for its
 * outputs; scratch is given back when the query ends, outputs when the
 * caller frees the result (slg_result_free). When a query cannot get memory
 * it waits, and no new query starts meanwhile; a second query that runs
 * short while one already waits gives back what it holds and goes back to
 * the head of the queue (it is planned again later; `attempts` counts
 * this). A query whose own need exceeds the whole budget fails with
 * SLG_ERR_OUT_OF_MEMORY. mem_budget_bytes = 0 means no limit.
 *
 * The server plans with its own contexts (one per slot, with ctx's device
 * and plan-shape tuning); ctx itself is only read at creation. Graphs
 * passed to submit must be registered on the same device and stay
 * registered until their queries are done. submit, wait, next and stats may
 * be called from any host threads. Results count against the budget until
 * freed: a caller that keeps results while waiting for a query that needs
 * their memory waits for ever (use a timeout, or `next`, which returns
 * queries in completion order). A served result is complete when handed
 * over; slg_result_free returns its buffers to the server's block cache
 * after the work already queued on the null stream, so finish work on
 * other streams that reads them first. Results may be freed after the
 * server is destroyed. The slots share one block cache that keeps at most
 * the budget (16 GiB without a budget) of freed blocks for reuse.
 */
typedef struct slg_server slg_server;
typedef struct {
    uint64_t ticket;
    slg_status status;   /* the query's own outcome */
    int32_t attempts;    /* times the query was planned */
    double queue_ms;     /* submit -> first start */
    double latency_ms;   /* submit -> outputs complete */
    int64_t two_paths;   /* 2-paths of the query's pass (at its smallest s) */
    char message[192];   /* why it failed ("" when status is SLG_OK) */
} slg_request_info;
slg_status slg_server_create(slg_context *ctx, int32_t workers, uint64_t mem_budget_bytes, slg_server **out);
/* Queue a query; *ticket names it. Errors: INVALID_ARG (null, bad s-set,
 * graph on another device), CANCELLED (server shutting down). */
slg_status slg_server_submit(slg_server *srv, slg_graph *g, const int32_t *s, int32_t num_s, uint64_t *ticket);
/*
 * Wait up to timeout_ms (< 0: no limit) for query `ticket`. Returns the
 * query's status once it has ended (then *out is its result, or NULL when
 * it failed, *info is filled, and the ticket is retired), TIMEOUT if it
 * has not, INVALID_ARG for an unknown or retired ticket.
 */
slg_status slg_server_wait(slg_server *srv, uint64_t ticket, int32_t timeout_ms, slg_result **out,
                           slg_request_info *info);
/* As wait, for whichever query ended first among those not yet retired. */
slg_status slg_server_next(slg_server *srv, int32_t timeout_ms, slg_result **out, slg_request_info *info);
/* out[0..8]: submitted, completed, failed, yields, queued, running,
 * bytes in use, peak bytes in use, bytes held by unfreed results. */
slg_status slg_server_stats(slg_server *srv, int64_t *out, int32_t cap, int32_t *count);
/* Cancels queued queries (CANCELLED), waits for running ones, frees the
 * results nobody took. */
slg_status slg_server_destroy(slg_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SLG_H */
