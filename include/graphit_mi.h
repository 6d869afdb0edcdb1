/*
 * graphit_mi.h -- C ABI of an MI355X (gfx950) graph-traversal library that
 * implements the data-parallel core of GraphIt (Zhang et al., "GraphIt: A
 * High-Performance Graph DSL", OOPSLA 2018): edgeset.apply over a frontier
 * vertexset in each of the paper's traversal schedules, driving PageRank,
 * BFS, connected components and single-source shortest paths.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Plain C types only.  "host" pointers are ordinary CPU memory; "device"
 *   pointers are HIP device memory on the current device (for instance the
 *   data pointer of a torch CUDA tensor).  Streams are hipStream_t passed as
 *   void*; NULL means the default stream.
 * - Every call returns a gi_status.  Arguments are checked on the host before
 *   any device work; on error nothing is enqueued and outputs are left
 *   unspecified.  gi_last_error() gives a message for the calling thread's
 *   last failing call.
 * - Stream order.  gi_pagerank and gi_batch_launch return once their
 *   kernels are enqueued on the given stream; their outputs are complete
 *   when that stream reaches them, and gi_sync_status (or reading the run's
 *   statistics) waits for them.  The other algorithm calls return when
 *   their outputs are complete: the frontier algorithms (gi_bfs, gi_cc,
 *   gi_sssp, gi_prdelta, gi_bc) enqueue steps in batches and read a
 *   completion flag back once per steps_per_sync steps, and
 *   gi_pagerank_eigenvector reads its norms back; the batched persistent
 *   kernel is the enqueue-only form of BFS, PageRank and SSSP
 *   (gi_batch_launch).
 * - Device memory.  Every device allocation of the library goes through one
 *   path: a graph's core arrays come from the caller's workspace when one is
 *   given to gi_graph_create_ex; everything else comes from the allocator
 *   registered with gi_set_allocator (a torch program registers torch's
 *   caching allocator, so torch owns that memory), or from hipMalloc when
 *   none is registered.  The one exception is the per-call scratch of
 *   gi_frontier_bitvec_to_sparse, taken stream-ordered with hipMallocAsync
 *   (gi_frontier_bitvec_to_sparse_noalloc takes none).
 * - A gi_graph owns device copies of its adjacency and a workspace sized at
 *   creation.  It is not thread-safe: one call at a time per graph, and the
 *   device work of one call must be ordered before the next call's (same
 *   stream, or the caller synchronizes).  Distinct graphs may be used from
 *   distinct threads and streams.
 * - Vertex ids are int32 in [0, n); edge counts are limited to 2^31-1 so that
 *   int32 offsets suffice (the evaluation notes the same 32-bit limit).
 */
#ifndef GRAPHIT_MI_H
#define GRAPHIT_MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GI_ABI_VERSION 1

typedef enum gi_status {
  GI_OK = 0,
  GI_ERR_INVALID_ARG = -1,   /* argument out of range, malformed adjacency   */
  GI_ERR_OUT_OF_MEMORY = -2, /* host or device allocation failed             */
  GI_ERR_DEVICE = -3,        /* a HIP call or kernel reported an error       */
  GI_ERR_UNSUPPORTED = -4,   /* schedule combination not offered             */
  GI_ERR_OVERFLOW = -5       /* count or distance exceeds its integer type   */
} gi_status;

typedef struct gi_graph gi_graph;

/* Traversal directions: configApplyDirection options of the scheduling
 * language (scheduling-language table; section 2, direction optimization). */
enum {
  GI_DIR_SPARSE_PUSH = 0,            /* frontier as sparse array, out-edges, atomics   */
  GI_DIR_DENSE_PUSH = 1,             /* all vertices, dense frontier test, out-edges    */
  GI_DIR_DENSE_PULL = 2,             /* all vertices, in-edges, no atomics              */
  GI_DIR_DENSE_PULL_SPARSE_PUSH = 3, /* per step: DensePull if frontier is large        */
  GI_DIR_DENSE_PUSH_SPARSE_PUSH = 4, /* per step: DensePush if frontier is large        */
  GI_DIR_LEARNED = 5                 /* per step: the attached selector's choice among
                                        SparsePush, DensePush and DensePull (BFS, CC;
                                        CC also the segmented DensePull);
                                        PageRank: unsegmented or segmented DensePull.
                                        The fallback (the hybrid rule with the
                                        schedule's divisor; unsegmented for PageRank)
                                        is kept unless the selector predicts it to be
                                        more than 15% slower (log-time margin 0.14).
                                        The choice is the direction only: the layout
                                        is the schedule's (segmented pulls use its
                                        segments, the automatic count when it has
                                        one; PageRank's unsegmented pull follows its
                                        vertex_order) */
};

/* Dense vertexset representation: configApplyDenseVertexSet options. */
enum { GI_FRONTIER_BITVECTOR = 0, GI_FRONTIER_BOOLMAP = 1 };

/* Segmented subgraphs: configApplyNumSSG options (section 2, cache
 * partitioning; section 6, SSG code generation). */
enum { GI_SEG_FIXED_VERTEX_COUNT = 0, GI_SEG_EDGE_AWARE_VERTEX_COUNT = 1 };

/* Schedule of a graph's edgeset.apply.  One field per scheduling function
 * (scheduling-language table), restated for a GPU:
 *   direction        configApplyDirection
 *   dense_frontier   configApplyDenseVertexSet (bitvector or bool array)
 *   num_segments     configApplyNumSSG: >1 splits the DensePull sources into
 *                    that many segmented subgraphs processed in order
 *   segment_strategy fixed-vertex-count or edge-aware-vertex-count
 *   hybrid_divisor   hybrid directions choose the dense side when
 *                    |F| + sum of out-degrees of F > m / hybrid_divisor
 *                    (section 2: sum of out-degrees against a threshold)
 *   steps_per_sync   frontier loops (BFS, CC, SSSP) enqueue this many
 *                    steps before reading the completion flag back; steps
 *                    after completion return at once (0 = library default:
 *                    first batch one step longer than the previous run of
 *                    the same algorithm on this graph, then 8 (64 for
 *                    SSSP) with two batches in flight).  Directions are
 *                    always decided on the device.
 *   pull_block_edges PageRank DensePull: in-edges staged in LDS per
 *                    destination block, 64..8192 (0 = library default: the
 *                    power of two in [256, 2048] nearest above m / 2048)
 *   block_threads    threads per workgroup of the PageRank DensePull
 *                    kernel: 64, 128, 256 or 512 (0 = library default 256)
 *   sssp_delta       bucket width of delta-stepping (0 = library default)
 *   segments_concurrent  PageRank with num_segments > 1: 0 processes the
 *                    segments one after another (the paper's order); 1 runs
 *                    them in one launch, workgroup b on segment b mod
 *                    num_segments, each segment adding into its own FP64
 *                    partial-sum buffer, then sums the partials (with 8
 *                    segments each of the 8 XCDs gathers from one segment,
 *                    which stays in its L2)
 *   cc_adjacency     how connected components reads edges both ways
 *                    (GI_CC_ADJ_*): AUTO (0) uses the symmetric copy when its
 *                    2m entries fit 32-bit offsets and the direct form
 *                    otherwise; SYMMETRIC (1) builds on first use a device
 *                    copy holding each vertex's out-row then its in-row
 *                    (2m entries; GI_ERR_OVERFLOW from gi_cc above 2^31-1);
 *                    DIRECT (2) builds no copy: push expands a frontier
 *                    vertex's out-row and in-row where they are, pull
 *                    reduces the CSR and CSC destination blocks separately
 *                    and merges the two minima of a vertex by atomic minimum
 *   vertex_order     PageRank DensePull (GI_ORDER_*): GIVEN (0) pulls over
 *                    the caller's numbering; OUT_DEGREE (1) pulls over a copy
 *                    of the in-adjacency renumbered by decreasing out-degree
 *                    (built on first use, 4(n + 1) + 4m + 8n bytes), so that
 *                    the sources gathered most often share cache lines and
 *                    the hottest sit in LDS; ranks come back under the
 *                    caller's numbering.  Unsegmented only (num_segments 1):
 *                    the ordering replaces the id-range segments
 *   pull_hot_sources with OUT_DEGREE: the highest-out-degree sources whose
 *                    contributions every workgroup copies into LDS per
 *                    iteration (-1 = library default, the most that fits
 *                    beside the waves' tile buffers in one workgroup's LDS;
 *                    0 = none; else rounded down to a multiple of 64 and
 *                    capped the same way)
 *   pull_items_per_thread with OUT_DEGREE: merge-path items (row ends plus
 *                    edges) per thread, 4, 8 or 16 (0 = library default 8;
 *                    16 only with block_threads <= 512)
 * block_threads may also be 1024 with vertex_order OUT_DEGREE.
 * Use gi_schedule_init for defaults; gi_set_schedule returns
 * GI_ERR_UNSUPPORTED for a combination it does not offer. */
enum { GI_CC_ADJ_AUTO = 0, GI_CC_ADJ_SYMMETRIC = 1, GI_CC_ADJ_DIRECT = 2 };
enum { GI_ORDER_GIVEN = 0, GI_ORDER_OUT_DEGREE = 1 };
typedef struct gi_schedule {
  int32_t direction;
  int32_t dense_frontier;
  int32_t num_segments;
  int32_t segment_strategy;
  int32_t hybrid_divisor;
  int32_t steps_per_sync;
  int32_t pull_block_edges;
  int32_t block_threads;
  uint32_t sssp_delta;
  int32_t segments_concurrent;
  int32_t cc_adjacency;
  int32_t vertex_order;
  int32_t pull_hot_sources;
  int32_t pull_items_per_thread;
  int32_t reserved[2];
} gi_schedule;

/* Per-run statistics of the last algorithm call on a graph. */
#define GI_MAX_TRACE 4096
typedef struct gi_run_stats {
  int32_t algorithm;      /* 0 PageRank, 1 BFS, 2 CC, 3 SSSP, 4 PageRankDelta,
                             5 betweenness, 6 PageRank + eigenvector           */
  int32_t steps;          /* edgeset.apply steps executed                        */
  int32_t dense_steps;    /* of which dense (pull or dense push)                 */
  int32_t trace_len;      /* entries valid in the arrays below (<= GI_MAX_TRACE) */
  int64_t edges_examined; /* sum over steps of sum of degrees of the frontier    */
  float kernel_ms;        /* GPU time between HIP events recorded on the call's
                             stream before the first and after the last launch of
                             the algorithm's main kernel(s)                      */
  int32_t launches;       /* main-kernel launches in that interval               */
  int8_t step_direction[GI_MAX_TRACE]; /* GI_DIR_* actually run per step          */
  int32_t step_frontier[GI_MAX_TRACE]; /* |F| entering each step                  */
  int64_t step_degree_sum[GI_MAX_TRACE]; /* sum of out-degrees of that frontier   */
  int64_t step_edges[GI_MAX_TRACE];      /* edges the step examined (pull: in-edges
                                            scanned up to the first frontier hit)  */
  int8_t step_segmented[GI_MAX_TRACE];   /* 1: the pull read the source segments
                                            (CC; schedule S3)                      */
} gi_run_stats;

/* ---- library ----------------------------------------------------------- */

/* Message for the calling thread's last failing call ("" if none). */
const char* gi_last_error(void);

/* GI_ABI_VERSION of the loaded library. */
int32_t gi_abi_version(void);

/* ---- graph ingest (host) ---------------------------------------------- */

/* Adjacency build from raw directed records (src[k] -> dst[k], k < nrec),
 * the edgeset load of the algorithm language (section 3).  Self-loops are
 * dropped, repeated pairs collapse to one edge keeping the smallest weight,
 * and each row is sorted by neighbour id.
 *   n                vertices; every id must lie in [0, n)
 *   src, dst         host, nrec entries each
 *   w                host, nrec weights, or NULL for an unweighted graph
 *   off              host out, n+1 entries (row offsets)
 *   idx              host out, capacity nrec (neighbour ids)
 *   w_out            host out, capacity nrec, or NULL
 *   m_out            host out, edges kept
 * Pass (dst, src) to build the in-adjacency (CSC).  Errors: INVALID_ARG for
 * a NULL array or an id out of range, OVERFLOW if more than 2^31-1 edges
 * remain, OUT_OF_MEMORY. */
gi_status gi_build_adjacency(int32_t n, int64_t nrec, const int32_t* src, const int32_t* dst,
                             const uint32_t* w, int32_t* off, int32_t* idx, uint32_t* w_out,
                             int64_t* m_out);

/* ---- device memory ----------------------------------------------------- */

/* Allocator the library takes device memory from (see the conventions above).
 *   alloc(bytes, device, ctx)   returns device memory of at least `bytes`
 *                               bytes on HIP device `device`, 256-byte
 *                               aligned, or NULL when it cannot
 *   release(ptr, device, ctx)   gives back memory alloc returned
 * Memory is released through the functions that allocated it, even if
 * another allocator is registered meanwhile.  Pass NULL, NULL to go back to
 * hipMalloc and hipFree.  Errors: INVALID_ARG when only one is NULL. */
typedef void* (*gi_alloc_fn)(size_t bytes, int32_t device, void* ctx);
typedef void (*gi_free_fn)(void* ptr, int32_t device, void* ctx);
gi_status gi_set_allocator(gi_alloc_fn alloc, gi_free_fn release, void* ctx);

/* Live device allocations of the library (workspace arrays not counted), and
 * how many of them came from a registered allocator (may be NULL). */
gi_status gi_live_allocations(int64_t* count, int64_t* from_registered);

/* ---- graph on the device ---------------------------------------------- */

/* Copy an adjacency to the device (section 3: edgeset with getOutNgh and
 * getInNgh; the out-degree vector of the PageRankDelta program is derived).
 *   out_off/out_idx  host CSR: n+1 offsets, m ids, rows sorted ascending
 *   out_w            host, m weights aligned with out_idx, or NULL
 *   in_off/in_idx    host CSC (the transpose), or both NULL to have the
 *                    library transpose the CSR
 *   in_w             host, weights aligned with in_idx, or NULL (derived
 *                    when out_w is given and in_off is NULL)
 * Validates monotone offsets, ids in range, strictly ascending rows, and that
 * the CSC holds exactly the CSR's edges (and weights).
 * Errors: INVALID_ARG, OVERFLOW (m > 2^31-1), OUT_OF_MEMORY, DEVICE. */
gi_status gi_graph_create(int32_t n, int64_t m, const int32_t* out_off, const int32_t* out_idx,
                          const uint32_t* out_w, const int32_t* in_off, const int32_t* in_idx,
                          const uint32_t* in_w, gi_graph** out);

/* Where the adjacency arrays given to gi_graph_create_ex live. */
enum { GI_PTR_HOST = 0, GI_PTR_DEVICE = 1 };

/* Bytes of device memory gi_graph_create_ex takes from a caller's workspace
 * for a graph of n vertices and m edges (weighted: nonzero when weights are
 * given): the adjacency in both directions, degrees, and the frontier-loop
 * buffers, each rounded up to 256 bytes.  An upper bound (it allows for the
 * most hub vertices m edges can make).  Errors: INVALID_ARG, OVERFLOW. */
gi_status gi_graph_workspace_size(int32_t n, int64_t m, int32_t weighted, size_t* bytes);

/* gi_graph_create with the arrays on the host or the device, the graph's
 * core arrays in a caller's workspace, and the copies on a caller's stream
 * (same adjacency model as gi_graph_create, section 3).
 *   ptr_kind         GI_PTR_HOST or GI_PTR_DEVICE: where out_off ... in_w
 *                    live (all in the same place); device arrays are read
 *                    on `stream` and staged to the host once, where they
 *                    are validated and the schedule tables are built
 *   workspace        device memory for the core arrays, 256-byte aligned,
 *                    of workspace_bytes >= gi_graph_workspace_size(...), or
 *                    NULL to take them from the allocator.  The caller keeps
 *                    it alive until gi_graph_destroy; structures built on
 *                    first use (segments, ordered copies, tables) still
 *                    come from the allocator
 *   stream           hipStream_t for the copies; the call returns when they
 *                    are complete (the caller may free its arrays then)
 * Errors: as gi_graph_create; INVALID_ARG for a bad ptr_kind, a misaligned
 * workspace, or one smaller than the graph needs; DEVICE for a failed copy. */
gi_status gi_graph_create_ex(int32_t n, int64_t m, const int32_t* out_off, const int32_t* out_idx,
                             const uint32_t* out_w, const int32_t* in_off, const int32_t* in_idx,
                             const uint32_t* in_w, int32_t ptr_kind, void* workspace,
                             size_t workspace_bytes, void* stream, gi_graph** out);

/* Release the graph and its device memory (NULL is a no-op). */
gi_status gi_graph_destroy(gi_graph* g);

/* Wait for the graph's last enqueued run (a call that returned after
 * enqueue) and report a device error it met.  Errors: INVALID_ARG (NULL),
 * DEVICE. */
gi_status gi_sync_status(gi_graph* g);

/* n, m, and the largest out- and in-degree. */
gi_status gi_graph_info(const gi_graph* g, int32_t* n, int64_t* m, int32_t* max_out_degree,
                        int32_t* max_in_degree);

/* Copy the device CSC back to host arrays (n+1, m, m-or-NULL entries). */
gi_status gi_graph_copy_in_adjacency(const gi_graph* g, int32_t* in_off, int32_t* in_idx,
                                     uint32_t* in_w);

/* ---- schedule ----------------------------------------------------------- */

gi_status gi_schedule_init(gi_schedule* s);
gi_status gi_set_schedule(gi_graph* g, const gi_schedule* s);
gi_status gi_get_schedule(const gi_graph* g, gi_schedule* s);

/* Hybrid direction rule (section 2): nonzero when the dense side should run,
 * i.e. frontier_size + frontier_degree_sum > edges / divisor.  Pure host
 * function, shared by the host-driven loop and mirrored on the device. */
int32_t gi_hybrid_choose_dense(int64_t frontier_size, int64_t frontier_degree_sum, int64_t edges,
                               int32_t divisor);

/* ---- algorithms (device outputs, stream ordered) --------------------- */

/* PageRank, pull form of the power iteration that PageRankDelta computes
 * with every vertex active (section 2, PageRankDelta; evaluation: 20
 * iterations, damping 0.85):
 *   x_0 = 1/n;  x_{k+1}[v] = (1-damping)/n + damping * sum_{u->v} x_k[u]/outdeg(u).
 * Runs DensePull (optionally segmented, num_segments > 1) regardless of the
 * direction field.  FP32 storage, FP64 accumulation.  Returns once the
 * iterations are enqueued on `stream` (ranks are complete when the stream
 * reaches them; gi_get_run_stats and gi_sync_status wait for them).  With
 * vertex_order = GI_ORDER_OUT_DEGREE, a call that repeats the previous
 * call's ranks, iters, damping and layout (step timing off) replays the run
 * as a HIP graph on the graph's own stream, which waits for `stream` and
 * which `stream` then waits for: same kernels, same stream order, fewer
 * launch gaps.
 *   ranks  device out, n floats: x_iters.
 * Errors: INVALID_ARG (iters < 0, damping outside [0,1], NULL), DEVICE. */
gi_status gi_pagerank(gi_graph* g, int32_t iters, float damping, float* ranks, void* stream);

/* Breadth-first search from src along out-edges (evaluation, algorithms
 * paragraph), one edgeset.apply per level in the scheduled direction(s).
 *   level   device out, n int32: hops from src, -1 when unreachable
 *   parent  device out, n int32, or NULL: a BFS tree (parent[src] = src,
 *           -1 when unreachable); which valid parent is reported depends
 *           on the schedule and on timing.
 * Errors: INVALID_ARG (src out of range, NULL level), DEVICE. */
gi_status gi_bfs(gi_graph* g, int32_t src, int32_t* level, int32_t* parent, void* stream);

/* Connected components by synchronous label propagation over edges taken
 * in both directions (evaluation, algorithms paragraph):
 *   label   device out, n int32: smallest vertex id of v's weakly
 *           connected component.
 * The first call builds the symmetric adjacency (2m entries, 32-bit
 * offsets) on the device.
 * Errors: INVALID_ARG, OVERFLOW (2m > 2^31 - 1, refused before any device
 * work), DEVICE. */
gi_status gi_cc(gi_graph* g, int32_t* label, void* stream);

/* Single-source shortest paths over uint32 weights by delta-stepping
 * (bucket width sssp_delta) with atomic-min relaxation (the paper's asyncMin
 * reduction, compiler section).
 *   dist    device out, n uint32: least path weight, UINT32_MAX when
 *           unreachable.
 * Errors: INVALID_ARG (unweighted graph, src out of range), OVERFLOW (a
 * finite distance reached UINT32_MAX), DEVICE. */
gi_status gi_sssp(gi_graph* g, int32_t src, uint32_t* dist, void* stream);

/* PageRankDelta, the paper's running example (section 2.1; its program in
 * the algorithm-language section, its schedule in the scheduling section):
 *   Rank = 0, Delta = 1/n, every vertex active; per round, active vertices
 *   add Delta/OutDegree into DeltaSum of their out-neighbours, then every
 *   vertex updates: in the first round Delta = a DeltaSum + (1-a)/n,
 *   Rank += Delta, Delta -= 1/n; later Delta = a DeltaSum, Rank += Delta;
 *   a vertex stays active when |Delta| > epsilon * Rank.
 * Stops after `rounds` rounds or when no vertex is active.  The schedule's
 * direction chooses SparsePush, DensePush, DensePull or the hybrid rule per
 * round (bitvector frontier; the learned direction is UNSUPPORTED).  All
 * arithmetic is FP64; with epsilon = 0 the ranks are the PageRank power
 * iteration's.  The trace records each round's active set.
 *   ranks   device out, n doubles.
 * Errors: INVALID_ARG (rounds < 0, damping outside [0,1], epsilon < 0 or not
 * finite), UNSUPPORTED, OUT_OF_MEMORY, DEVICE. */
gi_status gi_prdelta(gi_graph* g, int32_t rounds, double damping, double epsilon, double* ranks,
                     void* stream);

/* Betweenness centrality from one source (the paper's BC: a forward apply
 * counting shortest paths, then a backward apply of the dependencies, as
 * defined by Brandes, J. Math. Sociol. 2001):
 *   sigma[s] = 1, sigma[w] = sum of sigma[v] over edges v -> w with
 *   level[v] = level[w] - 1;
 *   dependency[v] = sum over v -> w with level[w] = level[v] + 1 of
 *   sigma[v] / sigma[w] * (1 + dependency[w]); dependency[s] = 0.
 * Forward levels choose their direction by the hybrid rule (section 2,
 * with the schedule's divisor): SparsePush with FP64 atomic adds for small
 * frontiers, DensePull (every unvisited vertex sums the path counts of its
 * in-neighbours in the frontier, atomic-free) for large ones.  The backward
 * sweep pulls: each vertex sums over its own out-row, atomic-free.  The
 * trace records each level's direction, size and out-degree sum.  Summing
 * the dependencies of every source gives the betweenness of every vertex.
 *   dependency  device out, n doubles (0 where unreachable).
 *   sigma       device out, n doubles, or NULL.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_bc(gi_graph* g, int32_t src, double* dependency, double* sigma, void* stream);

/* PageRank and eigenvector centrality together, fused or not (the paper's
 * loop fusion, apply-function fusion and vertex-data layout optimization,
 * section 4.3 and its evaluation of the PageRank + eigenvector fusion).
 * PageRank as gi_pagerank (DensePull, FP32 storage, FP64 sums); eigenvector
 * centrality by L2-normalised power iteration:
 *   x_0 = 1/n;  x_{k+1} = y / ||y||_2 with y[v] = sum_{u->v} x_k[u]
 *   (x_{k+1} = 0 when ||y|| = 0).
 * fused = 1: one pass over the in-edges per iteration gathers both values
 * of each source from one array of (contribution, x) pairs; fused = 0: two
 * passes over separate arrays.  Results agree either way.  With fused = 1
 * and the schedule's vertex_order = GI_ORDER_OUT_DEGREE the fused pass runs
 * over the degree-ordered in-adjacency (built on first use, shared with
 * gi_pagerank) and the results are written back under the caller's ids.
 *   ranks, eigen   device out, n floats each.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_pagerank_eigenvector(gi_graph* g, int32_t iters, float damping, float* ranks,
                                  float* eigen, int32_t fused, void* stream);

/* Statistics of the last algorithm call on g. */
gi_status gi_get_run_stats(const gi_graph* g, gi_run_stats* out);

/* Per-step timing, the cost record that schedule tuning needs (the paper's
 * autotuner, section 6.4, times whole runs; this times every edgeset.apply
 * step).  When enabled, each later call records HIP events on its stream
 * around every step it enqueues (one step = one PageRank iteration, or one
 * frontier step of BFS/CC/SSSP, counting the no-op steps enqueued after the
 * frontier emptied).  Errors: INVALID_ARG (enable not 0/1). */
gi_status gi_set_step_timing(gi_graph* g, int32_t enable);

/* Times of the steps of the last call (it has returned, so its work is
 * complete).  step_ms[k]: from the first kernel of step k (frontier count,
 * direction decision, compaction) to the end of its edge-traversal kernel;
 * main_ms[k]: that traversal kernel alone.  Writes min(cap, *count) entries;
 * *count = steps recorded (at most 4096).
 * Errors: INVALID_ARG (NULL count, cap < 0, NULL arrays with cap > 0), DEVICE. */
gi_status gi_get_step_times(const gi_graph* g, float* step_ms, float* main_ms, int32_t cap,
                            int32_t* count);

/* ---- learned schedule selector ------------------------------------------ */
/* A multilayer perceptron 12 -> 64 -> 64 -> 4 (ReLU) predicting the natural
 * log of the time in ms of the next step under each of four schedules:
 *   S0 SparsePush, S1 DensePush, S2 DensePull, S3 DensePull over segments.
 * It stands in for the hybrid rule's fixed threshold (section 2) and is
 * trained on the per-step timings the library records (the paper's
 * autotuner, section 6.4, searches whole-run timings instead).  Training
 * runs on the device in FP32 (mean squared error on log-time over the valid
 * schedules, Adam); inference inside a run uses BF16 weights with FP32
 * accumulation.  Parameters, row-major fp32:
 *   W1[12][64] b1[64] W2[64][64] b2[64] W3[64][4] b3[4]
 * Features are standardised as (x - mu) / sd before the first layer.
 *
 * Step features (one row of 12 floats per step):
 *   0 log2 n            1 log2 E (E = m; 2m for CC)   2 E / n
 *   3 log2(1 + max degree)   4 degree coefficient of variation (out-degree;
 *     out+in degree for CC)   5 |F| / n   6 sum deg(F) / E
 *   7 BFS: fraction of vertices not yet visited after this step's frontier;
 *     CC, PageRank: sum deg(F) / E
 *   8 log2(1 + |F|)     9 log2(1 + sum deg(F))
 *   10 |F_k| / max(1, |F_{k-1}|) clipped to [0, 64] (PageRank: 1)
 *   11 algorithm: BFS 0, CC 0.5, PageRank 1 */
#define GI_SEL_FEATURES 12
#define GI_SEL_SCHEDULES 4
#define GI_SEL_PARAMS 5252

enum { GI_ALG_PAGERANK = 0, GI_ALG_BFS = 1, GI_ALG_CC = 2, GI_ALG_SSSP = 3 };

typedef struct gi_selector gi_selector;

/* New selector with weights drawn He-uniform from a counter-based stream
 * (seed), zero biases, mu = 0, sd = 1.  Errors: INVALID_ARG, OUT_OF_MEMORY. */
gi_status gi_selector_create(uint64_t seed, gi_selector** out);
gi_status gi_selector_destroy(gi_selector* s);

/* Host copies of the parameters (GI_SEL_PARAMS floats) and of the feature
 * standardisation (GI_SEL_FEATURES floats each); any pointer may be NULL. */
gi_status gi_selector_get_params(const gi_selector* s, float* params, float* mu, float* sd);
/* Replace them (NULL leaves that part unchanged; sd entries must be > 0).
 * Resets the Adam moments.  Errors: INVALID_ARG. */
gi_status gi_selector_set_params(gi_selector* s, const float* params, const float* mu,
                                 const float* sd);

/* Inference range of the features (GI_SEL_FEATURES floats each; any
 * pointer may be NULL): every inference (gi_selector_predict, the learned
 * schedule) clamps feature f to [lo[f], hi[f]] before standardising it, so
 * a graph larger or more skewed than the training graphs is read as the
 * nearest edge of the training range rather than extrapolated.  A new
 * selector has lo = -FLT_MAX, hi = FLT_MAX (no clamp); training with
 * standardise sets the records' minimum and maximum; training itself does
 * not clamp.  set: NULL leaves that bound unchanged; lo[f] <= hi[f], no NaN.
 * Errors: INVALID_ARG, DEVICE. */
gi_status gi_selector_get_range(const gi_selector* s, float* lo, float* hi);
gi_status gi_selector_set_range(gi_selector* s, const float* lo, const float* hi);

/* Train on `count` host records: feats[count][12], log_ms[count][4],
 * valid[count][4] (nonzero where the schedule was timed; rows need at least
 * one).  Minibatches of 32 records in a seeded order (the same order every
 * epoch); one device launch runs all epochs.  If standardise is nonzero, mu
 * and sd are first set from the records (sd of a constant feature = 1), and
 * the inference range to the records' per-feature minimum and maximum.
 * loss (host, may be NULL) receives the mean loss of each epoch.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_selector_train(gi_selector* s, const float* feats, const float* log_ms,
                            const uint8_t* valid, int64_t count, int32_t epochs, float lr,
                            uint64_t seed, int32_t standardise, float* loss);

/* Gradient of the loss of one minibatch (1 <= count <= 32 host records)
 * with respect to the parameters, without updating them (host out,
 * GI_SEL_PARAMS floats), and the loss.  Errors: INVALID_ARG, DEVICE. */
gi_status gi_selector_gradient(gi_selector* s, const float* feats, const float* log_ms,
                               const uint8_t* valid, int32_t count, float* grad, float* loss);

/* Predicted log-times (host out, count x 4) for host feature rows, by the
 * device inference kernel with FP32 (bf16 = 0) or BF16 (bf16 = 1) weights.
 * Errors: INVALID_ARG, DEVICE. */
gi_status gi_selector_predict(const gi_selector* s, const float* feats, int64_t count,
                              int32_t bf16, float* out);

/* Attach a copy of the selector's current weights to g for
 * GI_DIR_LEARNED (NULL detaches).  Errors: INVALID_ARG, OUT_OF_MEMORY. */
gi_status gi_selector_attach(gi_graph* g, const gi_selector* s);

/* Features of the steps of the last BFS or CC call on g, as the device
 * computed them (host out, cap x 12); *count = steps recorded.
 * Errors: INVALID_ARG. */
gi_status gi_get_step_features(const gi_graph* g, float* feats, int32_t cap, int32_t* count);

/* Exhaustive per-step timing for selector training.  Runs `algorithm` on g
 * once per schedule S0..S3 that it offers, with per-step timing on (BFS and
 * CC: S0, S1, S2 with a bitvector frontier; CC's S3 and PageRank's S3: the
 * DensePull over the schedule's segments, or n*4/2 MiB segments when it has
 * one; PageRank, 20 iterations: S2 in the schedule's vertex_order, and S3),
 * the layout GI_DIR_LEARNED runs on.
 * The frontiers of BFS and of synchronous CC do not depend on the schedule,
 * so step k of every run meets the same frontier (checked: a mismatch is
 * GI_ERR_DEVICE).  Writes per step k < min(cap, *count): feats[k][12],
 * step_ms[k][4] (whole step: count, decide, compaction and traversal
 * kernels), valid[k][4].  The graph's schedule is restored afterwards.
 * src: BFS source (ignored otherwise).  Scratch outputs are allocated and
 * freed inside.  Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_trace_exhaustive(gi_graph* g, int32_t algorithm, int32_t src, float* feats,
                              float* step_ms, uint8_t* valid, int32_t cap, int32_t* count);

/* ---- batched persistent execution -------------------------------------- */
/* Many BFS, PageRank and SSSP instances over graphs of uneven size in one
 * persistent kernel launch (optionally replayed as a HIP graph).  Each task
 * runs on its own set of workgroups that meet at task-local barriers between
 * BFS levels and PageRank iterations, so no step costs a kernel launch and
 * small instances do not wait for the whole device.  BFS tasks choose
 * DensePull or push per level by the hybrid rule (section 2) with divisor
 * 20 and produce levels (and parents when asked); PageRank tasks use the DensePull
 * destination-block kernel with the graph's current block size.  Results
 * equal the plain entry points' (levels bit for bit; ranks within the
 * PageRank tolerance).  SSSP tasks run delta-stepping (near/far buckets,
 * as gi_sssp) with a task barrier per phase; distances equal gi_sssp's bit
 * for bit (they are unique).  A barrier that waits more than two seconds
 * fails the batch (GI_ERR_DEVICE) instead of hanging; a distance reaching
 * UINT32_MAX fails it with GI_ERR_OVERFLOW. */
typedef struct gi_task {
  int32_t graph;      /* index into the batch's graphs                          */
  int32_t algorithm;  /* GI_ALG_BFS, GI_ALG_PAGERANK or GI_ALG_SSSP             */
  int32_t src;        /* BFS / SSSP source                                      */
  int32_t iters;      /* PageRank iterations (>= 0)                             */
  float damping;      /* PageRank damping in [0, 1]                             */
  int32_t workgroups; /* workgroups of this task, 1..1024; 0 = the plan's choice
                         (a size rule at creation, then gi_batch_autotune)      */
  void* out;          /* device out, n entries: int32 levels (-1 unreachable)
                         for BFS, float ranks for PageRank, uint32 distances
                         (UINT32_MAX unreachable) for SSSP; kept by the caller  */
  void* parent;       /* BFS only, may be NULL: device out, n int32 parents
                         (parent[src] = src, -1 unreachable; any BFS tree)      */
  uint32_t sssp_delta; /* SSSP bucket width; 0 = the graph's schedule value
                         (sssp_delta, else 512).  SSSP needs a weighted graph  */
  int32_t hybrid_divisor; /* BFS: a level pulls when |F| + sum deg(F) > m / this
                         (section 2, direction optimization); 0 = the graph's
                         schedule value at creation (hybrid_divisor, 20 by
                         default).  Levels and parents do not depend on it   */
} gi_task;

typedef struct gi_batch gi_batch;

/* Plan a batch: validates the tasks, allocates each task's workspace and
 * deals the tasks' workgroups over a grid no larger than the kernel's
 * resident capacity.  The graphs must outlive the batch and keep the
 * schedule they had at creation (a changed PageRank block layout makes
 * gi_batch_run return INVALID_ARG).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_batch_create(gi_graph* const* graphs, int32_t ngraphs, const gi_task* tasks,
                          int32_t ntasks, gi_batch** out);

/* Autotuner, for each workgroup size of 256, 512 and 1024 threads (only the
 * pinned one after gi_batch_set_threads): first the PageRank block size of
 * each graph that has PageRank tasks (the batch's own destination blocks of
 * 256, 512, 1024, 2048 or 4096 edges; the graph's schedule is untouched),
 * timing the graph's first PageRank task alone with each and keeping the
 * fastest; then times each (graph, algorithm)
 * class alone on 256, 128, 64, ... workgroups (median of reps launches),
 * stopping at the first size more than twice as slow as the fastest so far;
 * keeps, among the sizes within twice the fastest, the one with the least
 * workgroup-time; gives tasks longer than the balanced share of the
 * grid their fastest size, caps those sizes at 64, 32 and 16, plans each
 * with XCD-local and with spread placement, and times each whole batch
 * (median of reps launches).  Keeps the workgroup size, task sizes,
 * placement and plan of the fastest whole batch, then refines it along
 * the critical path: tasks that end in the last tenth of a timed launch
 * and take at least a third of it get twice the workgroups (at most 256),
 * else half, the plan is rebuilt from the measured task durations, and a
 * resize is kept only if the whole batch gets at least 1% faster (up to
 * four rounds).
 * Tasks with fixed workgroups keep them.  The timing launches write the
 * tasks' outputs (with correct results).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_batch_autotune(gi_batch* b, int32_t reps);

/* PageRank destination-block size (edges per block) the batch uses for each
 * graph (host array of the batch's graph count): the graph's own block size
 * at creation, the autotuner's choice after gi_batch_autotune; 0 for graphs
 * without PageRank tasks.  Source segments are not used inside the batch:
 * a pool graph's contributions fit one XCD's L2.
 * Errors: INVALID_ARG. */
gi_status gi_batch_pr_block_edges(const gi_batch* b, int32_t* edges_per_block);

/* Threads per workgroup of the batch kernel: 256 (the default at creation),
 * 512 or 1024; pins that size for gi_batch_autotune and re-plans (task
 * workgroup counts are clamped to the resident grid of that size).
 * threads = 0 unpins it.  gi_batch_get_threads reports the current size.
 * Errors: INVALID_ARG (other sizes), OUT_OF_MEMORY, DEVICE. */
gi_status gi_batch_set_threads(gi_batch* b, int32_t threads);
gi_status gi_batch_get_threads(const gi_batch* b, int32_t* threads);

/* Placement of each task's workgroups: xcd_local = 1 (the default) keeps a
 * task that fits on one XCD's share of the grid on that XCD (workgroups are
 * dispatched to the 8 XCDs round-robin by index), so its workgroups share
 * one L2; 0 spreads them.  Setting it re-plans; gi_batch_autotune tries
 * both and keeps the faster.  Placement changes speed only.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_batch_set_placement(gi_batch* b, int32_t xcd_local);
gi_status gi_batch_get_placement(const gi_batch* b, int32_t* xcd_local);

/* Barrier of a task's workgroups between BFS levels, PageRank iterations and
 * SSSP phases.  GI_BARRIER_XCD (the default): a task whose workgroups all
 * run on one XCD (each workgroup reads its XCD from the hardware when the
 * task starts, so a placement the dispatcher did not keep is detected) skips
 * the L2 write-back before arriving: the XCD's L2 is shared by its
 * workgroups and the L1 writes through to it; the cache invalidation after
 * the wait is kept.  A task spread over several XCDs counts its arrivals
 * per XCD first (one counter line per XCD; each XCD's last arrival arrives
 * for it at the task's word), so at most 8 arrivals meet on one line.
 * Under GI_BARRIER_AGENT every task uses one counter at agent scope: the
 * L2 is written back before arriving and invalidated after.  Results do not
 * depend on the scope.  Errors: INVALID_ARG (another value, NULL, a launch in flight). */
enum { GI_BARRIER_AGENT = 0, GI_BARRIER_XCD = 1 };
gi_status gi_batch_set_barrier_scope(gi_batch* b, int32_t scope);
gi_status gi_batch_get_barrier_scope(const gi_batch* b, int32_t* scope);

/* Per-step trace of batch tasks (the batched counterpart of the per-step
 * trace in gi_get_run_stats).  gi_batch_set_trace keeps up to cap records
 * per task from the next run on (0 turns it off; it re-captures the HIP
 * graph).  gi_batch_get_trace reads task's records of the last run: for
 * each BFS level (PageRank iteration) its start on the device wall clock in
 * ns from the task's first step, whether it pulled, and the frontier size
 * (0 for PageRank); a final record marks the task's end (pull 0, frontier
 * 0).  At most cap records are written to each non-NULL array; *count gets
 * their number.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
gi_status gi_batch_set_trace(gi_batch* b, int32_t cap);
gi_status gi_batch_get_trace(const gi_batch* b, int32_t task, int64_t* start_ns, int32_t* pull,
                             int64_t* frontier, int32_t cap, int32_t* count);

/* Run every task once: one launch of the reset kernel and the persistent
 * kernel, captured once into a HIP graph and replayed when use_graph is
 * nonzero (on the batch's own stream, after the work enqueued on `stream`),
 * else launched on `stream`.  Returns after completion.
 * Errors: INVALID_ARG, DEVICE (including a barrier timeout). */
gi_status gi_batch_run(gi_batch* b, int32_t use_graph, void* stream);

/* gi_batch_run in two halves, so that other work can run on the device
 * while the batch does: gi_batch_launch enqueues the run (with use_graph,
 * on the batch's own stream, ordered after the work already enqueued on
 * `stream`; else on `stream`) and returns at once; gi_batch_wait waits for
 * it, records its time and checks the error flag.  One launch may be in
 * flight per batch; the outputs are not ready before gi_batch_wait returns.
 * While a launch is in flight the other gi_batch_* calls that change the
 * batch return INVALID_ARG.
 * Errors: INVALID_ARG, DEVICE (including a barrier timeout, from wait). */
gi_status gi_batch_launch(gi_batch* b, int32_t use_graph, void* stream);
gi_status gi_batch_wait(gi_batch* b);

/* GPU time of the last run (ms), grid size, and per task (arrays of the
 * batch's task count, may be NULL) its workgroups, its completed BFS
 * levels or PageRank iterations, and its duration in the last run (ms, from
 * the device wall clock, start to end of its first workgroup).
 * Errors: INVALID_ARG, DEVICE. */
gi_status gi_batch_info(const gi_batch* b, float* last_ms, int32_t* grid, int32_t* workgroups,
                        int32_t* levels, float* task_ms);

/* Per-task counters of the last run (host arrays of the batch's task count;
 * either may be NULL, not both):
 *   edges: edges relaxed.  For an SSSP task, every edge of every near-set
 *     member each time that member was relaxed, so edges / (edges out of
 *     the reached vertices) is the re-relaxation factor of delta-stepping
 *     (Meyer and Sanders): its work beyond a label-setting order, which
 *     relaxes each reached edge once.  0 for BFS and PageRank tasks.
 *   barrier_ms: time a workgroup of the task spent in task barriers, from
 *     its arrival to its release (device wall clock, mean over the task's
 *     workgroups; 0 for one-workgroup tasks, which need none).  Divided by
 *     the task's duration (gi_batch_info) it is the task's barrier-overhead
 *     fraction: the synchronisation that replaces the plain path's launches.
 * Errors: INVALID_ARG (also while a launch is in flight), DEVICE. */
gi_status gi_batch_task_counters(const gi_batch* b, int64_t* edges, float* barrier_ms);
gi_status gi_batch_destroy(gi_batch* b);

/* ---- frontier primitives (device, stream ordered) -------------------- */
/* Dense and sparse vertexset representations (section 2, direction
 * optimization and frontier data structure; scheduling-language table,
 * configApplyDenseVertexSet).  Bitvector: uint64 words, bit v%64 of word
 * v/64 set iff v is in the set; words beyond n must be provided
 * (ceil(n/64) words).  Bool map: one byte per vertex, nonzero iff member. */

/* Sparse array (count distinct ids) -> bitvector (cleared first). */
gi_status gi_frontier_sparse_to_bitvec(int32_t n, const int32_t* ids, int32_t count, uint64_t* bv,
                                       void* stream);
/* Bitvector -> sparse array in ascending id order; *count_dev receives the
 * number of members.  ids needs room for every member. */
gi_status gi_frontier_bitvec_to_sparse(int32_t n, const uint64_t* bv, int32_t* ids,
                                       int32_t* count_dev, void* stream);
/* Allocation-free variant of gi_frontier_bitvec_to_sparse, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, layout and result
 * as gi_frontier_bitvec_to_sparse; the caller still owns bv, ids and
 * *count_dev.  Its scratch (one int32 per bitvector word) is a fixed device
 * array of GI_NOALLOC_MAX_WORDS words (8 MiB) inside the library, one copy
 * per GPU, held until the process ends; no call allocates or frees memory.
 * n above 64 * GI_NOALLOC_MAX_WORDS (134,217,728 vertices) is refused with
 * GI_ERR_UNSUPPORTED before any device work, as is a device ordinal of
 * GI_NOALLOC_MAX_DEVICES or more.  All calls on one GPU share that GPU's
 * scratch: calls that overlap on one GPU (different streams, or host threads
 * without ordering between them) race and give undefined results; calls on
 * one stream are ordered and safe. */
#define GI_NOALLOC_MAX_WORDS (1 << 21)
#define GI_NOALLOC_MAX_DEVICES 64
gi_status gi_frontier_bitvec_to_sparse_noalloc(int32_t n, const uint64_t* bv, int32_t* ids,
                                               int32_t* count_dev, void* stream);
/* Bitvector <-> bool map. */
gi_status gi_frontier_bitvec_to_boolmap(int32_t n, const uint64_t* bv, uint8_t* bm, void* stream);
gi_status gi_frontier_boolmap_to_bitvec(int32_t n, const uint8_t* bm, uint64_t* bv, void* stream);
/* Frontier statistics for the hybrid rule: out[0] = count, out[1] = sum of
 * out-degrees of the members of a sparse array (device int64[2]). */
gi_status gi_frontier_degree_sum(const gi_graph* g, const int32_t* ids, int32_t count,
                                 int64_t* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GRAPHIT_MI_H */
