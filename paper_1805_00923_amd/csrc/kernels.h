// Kernel parameter blocks and host-side launchers (internal).
#pragma once

#include "common.h"

namespace gi {

enum : int { ALG_PR = 0, ALG_BFS = 1, ALG_CC = 2, ALG_SSSP = 3 };

// State that survives across launches of the frontier loop.
struct LoopState {
  int step;       // steps done (BFS: current level)
  int rep;        // REP_SPARSE / REP_DENSE: where the current frontier lives
  int sa_cur;     // which sparse buffer holds the current frontier
  int vis_valid;  // BFS: visited bitvector matches the level array
  int cc_fix;     // CC: next push step must first copy cur->nxt on F
  int lab_cur;    // CC: which label buffer holds L_k (0: user array, 1: workspace)
  int pad[2];
};

struct LoopParams {
  DevGraph g;
  int alg;
  int direction;      // GI_DIR_*
  int divisor;
  int boolmap;        // dense frontier kind
  int max_steps;      // steps to run in this launch
  int forced_dir;     // >= 0: direction of the next step (trace/exhaustive)
  long long edges;    // edge count of the traversal view (m, or 2m for CC)
  int32_t* level;     // BFS
  int32_t* parent;    // BFS, may be null
  int32_t* lab[2];    // CC
  int32_t* sa[2];
  uint64_t* dbv[3];   // dense frontier rotation (bitvector)
  uint8_t* dbm[3];    // dense frontier rotation (bool map)
  uint64_t* vis;      // BFS visited bitvector
  Control* ctl;
  LoopState* st;
};

struct SsspState {
  int phase;       // relaxation steps done
  int near_cur;    // which near buffer holds the current pile
  int far_cur;     // which far buffer holds the current pile
  int pad;
  unsigned long long thresh;  // current bucket ends below thresh
};

struct SsspParams {
  DevGraph g;
  uint32_t* dist;
  int32_t* near[2];
  int32_t* far[2];
  int32_t* stamp;
  int32_t* in_far;
  unsigned long long delta;
  int max_phases;
  Control* ctl;
  SsspState* st;
};

struct PrRows {
  const int2* table;    // (first row, end row) per destination block
  int ntab;
  const int32_t* off;   // row offsets into idx
  const int32_t* idx;   // source ids
  const int32_t* dst;   // row -> destination, or null when row == destination
};

struct PrVertex {
  const int32_t* outdeg;
  double base;   // (1-alpha)/n
  double alpha;
};

// ---- launchers (return 0 on success) ----
int launch_loop_init(const LoopParams& p, int src, hipStream_t stream);
int loop_max_blocks(int block_threads);
int launch_loop(LoopParams p, int block_threads, int blocks, hipStream_t stream);

int launch_sssp_init(const SsspParams& p, int src, hipStream_t stream);
int sssp_max_blocks(int bt);
int launch_sssp(SsspParams p, int bt, int blocks, hipStream_t stream);

int launch_pr_init(int n, const int32_t* outdeg, float* c0, float* rank, bool zero_iters,
                   hipStream_t s);
int launch_pr_rows(const PrRows& r, int cap_e, int cap_v, int bt, int grid, const float* cin,
                   int mode, const PrVertex& pv, float* cout, float* rank, double* acc,
                   hipStream_t s);
int launch_pr_seg_final(int n, const PrVertex& pv, double* acc, float* cout, float* rank,
                        hipStream_t s);
int launch_pr_persistent(const PrRows& r, int cap_e, int cap_v, int bt, int n, int iters,
                         const PrVertex& pv, float* c0, float* c1, float* rank, Control* ctl,
                         int max_blocks_per_cu, hipStream_t s);

int launch_sparse_to_bitvec(int n, const int32_t* ids, int count, uint64_t* bv, hipStream_t s);
int launch_bitvec_to_sparse(int n, const uint64_t* bv, int32_t* ids, int32_t* count,
                            int32_t* scratch, hipStream_t s);
int launch_bitvec_to_boolmap(int n, const uint64_t* bv, uint8_t* bm, hipStream_t s);
int launch_boolmap_to_bitvec(int n, const uint8_t* bm, uint64_t* bv, hipStream_t s);
int launch_degree_sum(const int32_t* outdeg, const int32_t* ids, int count, int64_t* out,
                      hipStream_t s);

}  // namespace gi
