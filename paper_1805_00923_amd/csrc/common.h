// Internal definitions shared by the HIP kernels and the host driver.
// gfx950 (CDNA4): 64-lane wavefronts, 256 CUs in 8 XCDs, 160 KiB LDS per CU.
//
// Execution model of the frontier loops: one kernel launch per phase of a
// step, all on one stream.  A single-workgroup "decide" kernel reads the
// statistics the previous step left behind, picks the direction of the next
// step and writes it to device memory; every other kernel of the step reads
// that mode at entry and returns at once when it is not its turn.  The host
// enqueues a batch of steps and looks at the completion flag once per batch.
// Kernel boundaries order the phases, so no grid-wide barrier is needed.
//
// Statistics are reduced per workgroup and stored (plain stores, one slot
// per workgroup) rather than accumulated with atomics on a single address:
// device-scope atomics on one address serialize at the memory side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/graphit_mi.h"

namespace gi {

constexpr int kWave = 64;
constexpr int kLogSegmented = 16;  // StepLog flag: the pull read the source segments
constexpr int kHubDeg = 4096;   // rows longer than this are hubs (batched BFS push)
constexpr int kParts = 2048;     // step kernels run exactly this many workgroups,
                                 // one statistics slot each
constexpr int kMaxCount = 2048;  // at most this many count/write workgroups
constexpr int kMaxLog = 4096;    // per-step trace entries
constexpr int kMinChunk = 256;   // smallest expansion chunk (slots)
constexpr int kFeat = GI_SEL_FEATURES;  // selector features per step

// ---------------------------------------------------------------------------
// Device-side adjacency.  CSR rows (out-edges) and CSC rows (in-edges) are
// sorted by neighbour id; weights are aligned with the index arrays.
// ---------------------------------------------------------------------------
struct DevGraph {
  int32_t n;
  int64_t m;
  const int32_t* out_off;
  const int32_t* out_idx;
  const uint32_t* out_w;
  const int32_t* in_off;
  const int32_t* in_idx;
  const uint32_t* in_w;
  const int32_t* outdeg;  // out_off[v+1]-out_off[v]
  const int32_t* udeg;    // out-degree + in-degree
  const int32_t* in_probe;  // per vertex: its in-neighbour of largest out-degree, -1 if none
  const int32_t* bfs_idx = nullptr;  // in-rows by decreasing source out-degree (ties by
                                     // id), so each row starts with its probe; null: the
                                     // BFS pull scans in_idx
};

// Per-workgroup statistics of one phase.
struct Part {
  long long a;  // e.g. vertices added to the next frontier
  long long b;  // e.g. their degree sum
  long long c;  // e.g. edges examined
  long long d;
};

// Step modes written by the decide kernels.
enum : int {
  MODE_NEVER = -100,  // "no second mode" in a gate; never written as a mode
  MODE_NONE = -1,
  MODE_SPARSE_PUSH = GI_DIR_SPARSE_PUSH,
  MODE_DENSE_PUSH = GI_DIR_DENSE_PUSH,
  MODE_DENSE_PULL = GI_DIR_DENSE_PULL,
  MODE_SSSP_RELAX = 10,
  MODE_SSSP_SPLIT = 11,
};

// One entry of the per-step trace.
struct StepLog {
  int dir;          // GI_DIR_* run by the step, + kLogSegmented for a pull over
                    // the source segments
  int frontier;     // |F| entering the step
  long long degsum; // sum of degrees of F
  long long edges;  // edges the step examined
};

// Completion flags and the per-step trace, in pinned host memory written by
// the decide kernels: the host reads them after the batch event without a
// device-to-host copy.
struct HostFlags {
  int done;
  int error;
  int overflow;
  int steps;            // steps executed (valid once done)
  int dense_steps;      // valid once done
  int pad;
  long long edges_examined;  // valid once done
  StepLog log[kMaxLog];
  float feat[kMaxLog][kFeat];  // selector features of each step (BFS, CC)
};

// Control block of one algorithm run (device memory).
struct Control {
  int mode;           // mode of the step being executed
  int done;           // 1 once the frontier is empty
  int steps;          // steps decided so far
  int dense_steps;
  long long nf;       // |F| entering the current step
  long long dsum;     // sum of degrees of F
  long long sa_count; // sparse items (degree > 0) after compaction
  long long sa_slots; // their degree sum (edge slots of the expansion)
  long long nchunks;  // expansion chunks
  long long edges_examined;
  long long visited;  // sum of |F| over the steps decided so far (BFS)
  // betweenness: the current level is order[bc_start, bc_end); bc_count
  // vertices are listed so far
  unsigned long long bc_start;
  unsigned long long bc_end;
  unsigned long long bc_count;
  // SSSP
  unsigned long long thresh;   // current bucket ends below thresh
  unsigned long long told;     // previous threshold (split phase)
  long long far_count;
  int overflow;
  int buckets;
  int error;          // an internal size invariant failed (the run is abandoned)
  int chunk;          // slots per expansion chunk of the current sparse step
  int seg;            // the current pull step uses the source segments (CC)
  HostFlags* host;    // device address of the pinned host flags and trace
};

// Publish a flag to the pinned host copy.
__device__ __forceinline__ void host_flag(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Completion: the run's totals, then the flag the host polls.
__device__ __forceinline__ void publish_done(Control* c, int steps) {
  HostFlags* h = c->host;
  h->dense_steps = c->dense_steps;
  h->edges_examined = c->edges_examined;
  host_flag(&h->steps, steps);
  host_flag(&h->done, 1);
}

// ---------------------------------------------------------------------------
// Wave / workgroup helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long lanemask_lt() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T y = __shfl_xor(v, o, kWave);
    v = y < v ? y : v;
  }
  return v;
}

// Exclusive prefix sum across the wave.
template <typename T>
__device__ __forceinline__ T wave_excl_scan(T v, T* total) {
  const int l = __lane_id();
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  *total = __shfl(x, 63, kWave);
  return x - v;
}

// Sum of four counters over the workgroup; result valid in thread 0.
template <int BT>
__device__ __forceinline__ Part block_sum4(Part p) {
  __shared__ long long sh[4][BT / kWave];
  p.a = wave_sum(p.a);
  p.b = wave_sum(p.b);
  p.c = wave_sum(p.c);
  p.d = wave_sum(p.d);
  const int w = threadIdx.x / kWave;
  if (__lane_id() == 0) {
    sh[0][w] = p.a;
    sh[1][w] = p.b;
    sh[2][w] = p.c;
    sh[3][w] = p.d;
  }
  __syncthreads();
  Part r{0, 0, 0, 0};
  if (threadIdx.x == 0) {
    for (int i = 0; i < BT / kWave; ++i) {
      r.a += sh[0][i];
      r.b += sh[1][i];
      r.c += sh[2][i];
      r.d += sh[3][i];
    }
  }
  __syncthreads();
  return r;
}

// Workgroup exclusive scan of one value per thread (BT threads); returns
// the exclusive prefix and writes the workgroup total to *total.
template <int BT, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* total) {
  __shared__ T wsum[BT / kWave];
  T wt;
  const T ex = wave_excl_scan(v, &wt);
  const int w = threadIdx.x / kWave;
  if (__lane_id() == 0) wsum[w] = wt;
  __syncthreads();
  T base = 0, tot = 0;
  for (int i = 0; i < BT / kWave; ++i) {
    if (i < w) base += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return base + ex;
}

// Hybrid rule of the paper (section 2): dense when |F| + sum deg(F) exceeds
// edges / divisor, evaluated as (|F| + D_F) * divisor > edges.  Mirrors
// gi_hybrid_choose_dense on the device.
__host__ __device__ __forceinline__ bool hybrid_dense(long long nf, long long degsum,
                                                      long long edges, int divisor) {
  return (nf + degsum) * (long long)divisor > edges;
}

}  // namespace gi
