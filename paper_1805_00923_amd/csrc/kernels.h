// Kernel parameter blocks and host-side launchers (internal).
#pragma once

#include "common.h"
#include "selector.h"
#include "traverse.h"

namespace gi {

enum : int { ALG_PR = 0, ALG_BFS = 1, ALG_CC = 2, ALG_SSSP = 3, ALG_PRD = 4, ALG_BC = 5 };

// Rows of one adjacency split into destination blocks (PageRank and CC pull).
struct RowBlocks {
  const int4* table;    // per block: (first row, end row, first edge, end edge);
                        // a chunk of a long row: (row, -(chunk + 1), first edge, end edge)
  int ntab;
  const int32_t* off;
  const int32_t* idx;
};

// CC pull: destination blocks of the symmetric adjacency hold at most this
// many edges and rows.
constexpr int kCcCapE = 2048;
constexpr int kCcCapV = 1024;

// Scratch and launch shapes shared by the frontier loops of one graph.
struct Engine {
  int n;
  int tw;           // count/write: words per workgroup
  int cgrid;        // count/write workgroups (<= kMaxCount)
  Blk* blk;
  int32_t* ids;
  long long* excl;
  int32_t* chunk_item;
  long long chunk_cap;  // entries of chunk_item
  Control* ctl;
};

// PageRank destination blocks.  table[t] = (first row, end row, -1, 0) for
// a block of whole rows, or (row, row + 1, slot, chunk) for chunk `chunk` of
// a row longer than cap_e; `slot` indexes the long-row arrays.
struct PrRows {
  const int4* table;
  int ntab;
  const int32_t* off;   // row offsets into idx
  const int32_t* idx;   // source ids
  const int32_t* dst;   // row -> destination, or null when row == destination
  double* lr_acc;       // per long row: partial-sum accumulator (zero between uses)
  unsigned* lr_cnt;     // per long row: chunks finished (zero between uses)
  const int32_t* lr_chunks;  // per long row: number of chunks
};

struct PrVertex {
  const int32_t* outdeg;
  double base;   // (1-alpha)/n
  double alpha;
};

struct DecideArgs {
  Part* part;
  Control* ctl;
  int direction;   // GI_DIR_*
  int divisor;
  int forced_dir;  // >= 0: direction of every step
  long long edges; // m for BFS, 2m for CC (edges counted in both directions)
  int is_bfs;      // feature 7 is the unvisited fraction
  int max_steps;   // > 0: the run ends after this many steps
  FeatConst fc;    // graph-level features
  SelDev sel;      // attached selector (GI_DIR_LEARNED)
  int seg_pull;    // CC: 0 pulls unsegmented; 1 pulls over the source segments;
                   // 2 the learned choice may take the segmented pull (S3)
};

struct BfsArgs {
  DevGraph g;
  int32_t* level;
  int32_t* parent;  // may be null
  DenseSet cur;     // frontier of the step
  DenseSet next;    // frontier it produces
  uint64_t* vis;    // visited bitvector
  Part* part;
  Control* ctl;
};

// One source segment of the symmetric adjacency for the segmented CC pull:
// the rows (destinations dst[k]) with at least one neighbour in the segment,
// holding only those neighbours.
struct CcSeg {
  RowBlocks rows;
  const int32_t* dst;
};

struct CcArgs {
  DevGraph g;
  int32_t* cur;            // labels L_k
  int32_t* nxt;            // labels L_{k+1}
  DenseSet fr;             // vertices whose label changed in the previous round
  DenseSet next;           // vertices whose label changes in this round
  const int32_t* sym_off;  // symmetric adjacency (out-row then in-row); NULL
  const int32_t* sym_idx;  // when `direct`
  RowBlocks rows;          // destination blocks of the symmetric adjacency, or
                           // with `direct` of the out-rows (CSR)
  RowBlocks rows_in;       // with `direct`: destination blocks of the in-rows (CSC)
  int direct;              // 1: no symmetric copy; every round reads a vertex's
                           // out-row and in-row where they are (CSR and CSC)
  const CcSeg* segs;       // segmented pull: nseg source segments (nseg > 1), and
  int nseg;                // their partial minima, nseg x n (0xffffffff: none)
  uint32_t* seg_min;
  Part* part;
  Control* ctl;
};

struct SsspArgs {
  DevGraph g;
  uint32_t* dist;
  DenseSet cur;        // near set relaxed by this phase
  DenseSet next;       // near set of the next phase
  DenseSet far;        // far set
  unsigned long long delta;
  unsigned long long* fmin;  // per count-workgroup smallest far distance
  Part* part;
  Control* ctl;
};

// ---- launchers (return 0 on success) ----
int expand_chunk_size();
FrontierArgs frontier_args(const Engine& e, DenseSet cur, DenseSet next, const int32_t* deg,
                           const int32_t* fix_src, int32_t* fix_dst);
// Optional timing events around one step: `start` before the step's first
// kernel, `main` before its edge-traversal kernel, `end` after it.
struct StepEvents {
  hipEvent_t start, main, end;
};

int launch_ctl_init(Control* c, HostFlags* host, unsigned long long delta, hipStream_t s);
int launch_bfs_init(const BfsArgs& b, int src, DenseSet f0, DenseSet f1, hipStream_t s);
int enqueue_bfs_step(const Engine& e, const FrontierArgs& f, const DecideArgs& d,
                     const BfsArgs& b, const StepEvents* te, hipStream_t s);
int launch_cc_init(const CcArgs& c, DenseSet f0, DenseSet f1, int32_t* lab_other, hipStream_t s);
int launch_build_sym(const DevGraph& g, const int32_t* sym_off, int32_t* sym_idx, hipStream_t s);
int enqueue_cc_step(const Engine& e, const FrontierArgs& f, const DecideArgs& d, const CcArgs& c,
                    const StepEvents* te, hipStream_t s);
int launch_sssp_init(const SsspArgs& sa, int src, hipStream_t s);
int enqueue_sssp_step(const Engine& e, const FrontierArgs& f, const SsspArgs& sa,
                      const StepEvents* te, hipStream_t s);

// PageRankDelta (algos.hip).
struct PrdArgs {
  DevGraph g;
  double* delta;
  double* contrib;  // delta / outdeg of active vertices, 0 otherwise
  double* dsum;     // DeltaSum (zero between rounds)
  double* rank;
  DenseSet cur;
  DenseSet next;
  PrRows rows;      // in-row blocks for the pull
  int cap_e;
  double alpha;
  double base;      // (1 - alpha) / n
  double inv_n;
  double eps;
  Part* part;
  Control* ctl;
};
int launch_prd_init(const PrdArgs& a, hipStream_t s);

// Betweenness centrality, one source (algos.hip).
struct BcArgs {
  DevGraph g;
  int src;
  int32_t* level;
  double* sigma;   // shortest-path counts
  double* fs;      // sigma of the current frontier's vertices, 0 elsewhere (pull levels)
  double* bw;      // (1 + delta[w]) / sigma[w], set when w's dependency is final
  double* delta;   // dependencies (output)
  int32_t* order;  // vertices in discovery order, grouped by level
  unsigned long long* bounds;  // bounds[k] = first list index of level k (k <= levels)
  RowBlocks in_rows;  // in-row blocks (hub rows as chunks) for the pull levels
  int divisor;     // pull when |F| * divisor * (m / n) > m
  Control* ctl;
};
int launch_bc_init(const BcArgs& a, hipStream_t s);
int enqueue_bc_forward(const BcArgs& a, const StepEvents* te, hipStream_t s);
int enqueue_bc_backward_level(const BcArgs& a, long long begin, long long end, int level,
                              hipStream_t s);
int enqueue_prd_step(const Engine& e, const FrontierArgs& f, const DecideArgs& d,
                     const PrdArgs& a, const StepEvents* te, hipStream_t s);

// Selector training (selector.hip): parameters, Adam moments and the
// gradient buffer in device memory; records x[n][12], y[n][4] (log ms),
// valid[n][4]; minibatches follow `order`.
struct TrainArgs {
  float* p;
  float* m1;
  float* m2;
  float* grad;
  const float* x;
  const float* y;
  const uint8_t* valid;
  const int32_t* order;
  int n;
  const float* mu;
  const float* isd;
  int epochs;
  float lr, beta1, beta2, eps;
  int apply;       // 0: gradient only
  long long t0;    // Adam steps taken before this launch
  float* loss;     // per-epoch mean minibatch loss (may be null)
};
int launch_mlp_train(const TrainArgs& a, hipStream_t s);
int launch_mlp_predict(const SelDev& sd, const float* x, long long n, bool bf16, float* out,
                       hipStream_t s);

// Batched persistent execution (batch.hip).
struct BatchGraph {
  int n;
  long long m;
  const int32_t* out_off;
  const int32_t* out_idx;
  const int32_t* in_off;
  const int32_t* in_idx;
  const int32_t* outdeg;
  const uint32_t* out_w;  // edge weights (weighted graphs; SSSP tasks)
  const int32_t* in_probe;
  const int32_t* bfs_idx;  // in-rows starting with their probe (BFS pull), or null
  const int32_t* hubs;   // vertices with more than kHubDeg out-edges
  int nhubs;
  const int4* pr_table;  // PageRank destination blocks (the graph's current schedule)
  int pr_ntab;
  int pr_cap_e;
  const int32_t* lr_chunks;
  int n_long;            // rows split into chunks
};

struct TaskCtl {
  unsigned long long bar;    // barrier: (generation << 32) | arrivals
  unsigned long long qn[3];  // BFS frontier sizes, rotating
  unsigned long long ds[3];  // their degree sums
  int levels;                // BFS levels / PageRank iterations / SSSP phases completed
  int overflow;              // SSSP: a distance reached UINT32_MAX
  long long t_begin;         // wall clock at the task's start and end (rank 0)
  long long t_end;
  unsigned long long thresh; // SSSP: the current bucket ends below thresh
  unsigned long long fmin;   // SSSP: smallest far distance at or beyond thresh
  unsigned long long farc[3];  // SSSP: far-set sizes, rotating like qn
  unsigned long long ft[2];  // SSSP: lengths of the two far lists
  unsigned long long relaxed;  // SSSP: edges relaxed, summed over the workgroups
  unsigned long long bar_ticks;  // wall-clock ticks the workgroups spent in task barriers
  int qbad[3];               // SSSP: the near set's list is incomplete, rotating like qn
  int fbad;                  // SSSP: the far list is incomplete
  unsigned xcds;             // XCDs the task's workgroups run on (bit per XCC id)
  unsigned xcnt[8];          // the task's workgroups on each XCD
  // arrivals per XCD at a barrier of a task spread over several XCDs, one
  // 128-byte line each
  alignas(128) unsigned long long xarr[8][16];
};

struct BatchTask {
  int id;       // index in the batch
  int alg;      // ALG_BFS, ALG_PR or ALG_SSSP
  int graph;
  int src;
  int iters;
  unsigned delta;  // SSSP bucket width
  int div;         // BFS hybrid divisor: pull when |F| + deg(F) > m / div
  float damping;
  int k;        // workgroups
  void* out;    // int32 levels or float ranks
  int32_t* parent;  // BFS parents or null
  uint64_t* vis;
  uint64_t* bv0;
  uint64_t* bv1;
  uint64_t* bv2;
  float* c0;
  float* c1;
  double* lr_acc;
  unsigned* lr_cnt;
  int32_t* q;   // SSSP: member lists of bv0..bv2, then the two far lists (5 n)
  TaskCtl* ctl;
};

struct BatchArgs {
  const BatchGraph* graphs;
  const BatchTask* tasks;
  const int2* items;   // (task, rank) per workgroup list entry
  const int* wg_off;   // list of workgroup w: items[wg_off[w] .. wg_off[w+1])
  int* error;          // set when a barrier wait timed out
  long long spin_limit;  // wall-clock ticks a barrier may wait
  int lds_cap_e;
  int trace_cap;         // per-task step records kept (0: no trace)
  int xcd_barrier;       // 1: a task whose workgroups all run on one XCD uses the
                         // one-XCD barrier (L1 invalidate only); 0: agent scope
  long long* trace;      // [task][trace_cap][2]: wall clock at the step's start,
                         // (pull << 62) | frontier size (BFS) or 0 (PageRank)
  int algs;              // host side: the algorithms among the tasks (kBatchBfs |
                         // kBatchSssp | kBatchPr); a BFS-only batch launches a
                         // kernel built without the other task bodies
};

enum { kBatchBfs = 1, kBatchSssp = 2, kBatchPr = 4, kBatchAll = 7 };

bool batch_threads_ok(int bt);  // 256, 512 or 1024 threads per workgroup
size_t batch_lds_bytes(int cap_e, int cap_v);
int batch_occupancy(int bt, size_t lds, int algs);
int launch_batch(const BatchArgs& a, int bt, int grid, size_t lds, TaskCtl* ctl, int ntasks,
                 hipStream_t s);

int launch_pr_seg_concurrent(const PrRows* segs, int p, int cap_e, int cap_v, int bt,
                             const float* cin, const PrVertex& pv, double* acc, int n,
                             hipStream_t s);
int launch_pr_seg_final_multi(int n, int p, const PrVertex& pv, double* acc, float* cout,
                              float* rank, hipStream_t s);

// PageRank and eigenvector centrality, fused or not (pagerank.hip).
struct PrEcArgs {
  RowBlocks rb;               // in-row blocks of at most kPrEcCapE edges; a longer row
                              // as chunk entries (slot, -(chunk + 1), first edge, end edge)
  double* lacc;               // per long-row slot: (PageRank sum, eigenvector sum)
  const int32_t* lrow;        // row of each long-row slot
  int nlong;
  const float2* aos_in;       // fused: (PageRank contribution, eigenvector y) per vertex
  float2* aos_out;
  const float* y_in;          // eigenvector y alone (unfused)
  float* y_out;
  const double* norm2_prev;   // ||y_k||^2 (the next y is scaled by its inverse root)
  double* norm2_next;         // accumulates ||y_{k+1}||^2
  PrVertex pv;
  float* ranks;               // fused, last iteration: PageRank out
};
constexpr int kPrEcCapE = 2048;
constexpr int kPrEcCapV = 1024;
int launch_prec_rows(const PrEcArgs& a, bool fused, hipStream_t s);  // + long-row finish
int launch_prec_init(int n, const int32_t* outdeg, float2* aos, float* y, double* norm2,
                     int nnorm, hipStream_t s);
int launch_ec_final(int n, const float* y, const float2* aos, const double* norm2, float* out,
                    hipStream_t s);

int launch_pr_init(int n, const int32_t* outdeg, float* c0, float* rank, bool zero_iters,
                   hipStream_t s);
int launch_pr_rows(const PrRows& r, int cap_e, int cap_v, int bt, int grid, const float* cin,
                   int mode, const PrVertex& pv, float* cout, float* rank, double* acc,
                   hipStream_t s);
int launch_pr_seg_final(int n, const PrVertex& pv, double* acc, float* cout, float* rank,
                        hipStream_t s);

// PageRank over the degree-ordered in-adjacency, merge-path work split
// (pr_order.hip).
struct PrOrdArgs {
  const int32_t* off;     // degree-ordered in-row offsets (n + 1)
  const int32_t* idx;     // degree-ordered in-row source ids (m)
  const int2* tiles;      // per tile (first row, first edge); entry ntiles = (n, m)
  const int2* tslot;      // per tile: split slot of its first row (if that row
                          // began in an earlier tile) and of its last row (if
                          // it goes on in a later tile); -1 for none
  const int32_t* srow;    // per split slot: its row
  double* sacc;           // per split slot: parts summed so far (zero between passes)
  int nslots;
  const int32_t* outdeg;  // out-degree by new id
  const int32_t* old_id;  // new id -> caller's id
  int n;
  int m;
  int ntiles;
  int hot;                // sources [0, hot) are read from LDS (multiple of 4)
  double base;            // (1 - alpha) / n
  double alpha;
};

size_t pr_ord_lds_bytes(int hot, int bt, int u);
int pr_ord_occupancy(int hot, int bt, int u);  // workgroups per CU, -1 on error
int launch_pr_ord(const PrOrdArgs& a, int bt, int u, int grid, const float* cin, float* cout,
                  float* rank, hipStream_t s);
int launch_pr_ord_split(const PrOrdArgs& a, float* cout, float* rank, hipStream_t s);

int launch_sparse_to_bitvec(int n, const int32_t* ids, int count, uint64_t* bv, hipStream_t s);
int launch_bitvec_to_sparse(int n, const uint64_t* bv, int32_t* ids, int32_t* count,
                            int32_t* scratch, hipStream_t s);
int launch_bitvec_to_boolmap(int n, const uint64_t* bv, uint8_t* bm, hipStream_t s);
int launch_boolmap_to_bitvec(int n, const uint8_t* bm, uint64_t* bv, hipStream_t s);
int launch_degree_sum(const int32_t* outdeg, const int32_t* ids, int count, int64_t* out,
                      hipStream_t s);

}  // namespace gi
