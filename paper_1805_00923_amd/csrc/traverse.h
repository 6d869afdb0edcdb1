// Edge-traversal building blocks shared by the BFS, CC and SSSP kernels.
//
// The paper's edgeset.apply comes in three directions (section 2, direction
// optimization): SparsePush walks the out-edges of a sparse-array frontier
// with atomic updates, DensePush walks the out-edges of every vertex whose
// dense-frontier bit is set, DensePull walks the in-edges of every vertex
// and needs no atomics.  The GPU versions below are device functions called
// by every workgroup of a grid with (block id, grid size), so the same code
// runs in a one-step launch and inside a persistent cooperative loop.
#pragma once

#include "common.h"

namespace gi {

// Frontier/dense-set kinds.
enum : int { REP_SPARSE = 0, REP_DENSE = 1 };

// Membership test of a dense vertexset: bitvector or bool map
// (configApplyDenseVertexSet).
struct DenseSet {
  uint64_t* bv;  // ceil(n/64) words, or null
  uint8_t* bm;   // n bytes, or null
  __device__ __forceinline__ bool test(int u) const {
    return bm ? bm[u] != 0 : ((bv[u >> 6] >> (u & 63)) & 1ull) != 0;
  }
};

// Item providers for the push expansion: item i -> (u, [beg, end)).
struct SparseItems {  // sparse array frontier
  const int32_t* ids;
  int count;
  const int32_t* off;
  __device__ __forceinline__ int nitems() const { return count; }
  __device__ __forceinline__ void get(int i, int& u, int& b, int& e) const {
    u = ids[i];
    b = off[u];
    e = off[u + 1];
  }
};

struct DenseItems {  // dense frontier: every vertex, filtered by membership
  DenseSet set;
  int n;
  const int32_t* off;
  __device__ __forceinline__ int nitems() const { return n; }
  __device__ __forceinline__ void get(int i, int& u, int& b, int& e) const {
    if (set.test(i)) {
      u = i;
      b = off[i];
      e = off[i + 1];
    } else {
      u = -1;
      b = e = 0;
    }
  }
};

// Wave-aggregated append of the lanes with p set: one atomic per wave.
// Must be called by all lanes of the wave together.
__device__ __forceinline__ void wave_append(bool p, int v, int32_t* out,
                                            unsigned long long* counter) {
  const unsigned long long mk = __ballot(p);
  if (mk == 0ull) return;
  const int leader = __ffsll((long long)mk) - 1;
  unsigned long long base = 0;
  if (__lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mk));
  base = __shfl(base, leader, kWave);
  if (p) out[base + __popcll(mk & lanemask_lt())] = v;
}

// Degree-binned push expansion over the items of a frontier.  Rows with at
// least BT edges are walked by the whole workgroup, rows with at least 64
// edges by one wave, and the remaining short rows of a wave are gathered
// with a wave prefix sum so that 64 consecutive lanes take 64 consecutive
// edge slots.  vis(u, e, valid) is called by full waves; `valid` is false
// for padding lanes.
template <int BT, class Items, class Visit>
__device__ void push_expand(int bid, int nbl, const Items& items, Visit& vis) {
  __shared__ int sh_owner, sh_u, sh_b, sh_e;
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int nitems = items.nitems();
  for (int base = bid * BT; base < nitems; base += nbl * BT) {
    const int i = base + tid;
    int u = -1, beg = 0, end = 0;
    if (i < nitems) items.get(i, u, beg, end);
    // workgroup-wide rows
    while (__syncthreads_or(end - beg >= BT)) {
      if (end - beg >= BT) sh_owner = tid;
      __syncthreads();
      if (tid == sh_owner) {
        sh_u = u;
        sh_b = beg;
        sh_e = end;
        beg = end;
      }
      __syncthreads();
      const int cu = sh_u, cb = sh_b, ce = sh_e;
      for (int k = cb; k < ce; k += BT) {
        const int e = k + tid;
        vis(cu, e, e < ce);
      }
      __syncthreads();
    }
    // wave-wide rows
    for (;;) {
      const unsigned long long mk = __ballot(end - beg >= kWave);
      if (mk == 0ull) break;
      const int leader = __ffsll((long long)mk) - 1;
      const int cu = __shfl(u, leader, kWave);
      const int cb = __shfl(beg, leader, kWave);
      const int ce = __shfl(end, leader, kWave);
      if (lane == leader) beg = end;
      for (int k = cb; k < ce; k += kWave) {
        const int e = k + lane;
        vis(cu, e, e < ce);
      }
    }
    // short rows: scan-based gather
    int total;
    const int deg = end - beg;
    const int excl = wave_excl_scan(deg, &total);
    for (int r = 0; r < total; r += kWave) {
      const int j = r + lane;
      int lo = 0;
#pragma unroll
      for (int s = 32; s > 0; s >>= 1) {
        const int cand = lo + s;
        const int ex = __shfl(excl, cand, kWave);
        if (ex <= j) lo = cand;
      }
      const int cu = __shfl(u, lo, kWave);
      const int cb = __shfl(beg, lo, kWave);
      const int ex = __shfl(excl, lo, kWave);
      vis(cu, cb + (j - ex), j < total);
    }
  }
}

// Per-lane step statistics, flushed once per wave at the end of a step.
struct StepAccum {
  long long cnt = 0;
  long long dsum = 0;
  long long work = 0;
  __device__ __forceinline__ void flush(StepCounters* sc, bool add_count) {
    const long long c = wave_sum(cnt), d = wave_sum(dsum), w = wave_sum(work);
    if (__lane_id() == 0) {
      if (add_count && c) atomicAdd(&sc->count, (unsigned long long)c);
      if (d) atomicAdd(&sc->degsum, (unsigned long long)d);
      if (w) atomicAdd(&sc->work, (unsigned long long)w);
    }
  }
};

// Output of a push step: sparse array (wave-aggregated append) or dense set
// (bitvector atomicOr / bool-map store into a cleared buffer).
struct PushOut {
  int kind;               // REP_SPARSE or REP_DENSE
  int32_t* ids;           // sparse output
  unsigned long long* count;
  DenseSet dense;         // dense output
  __device__ __forceinline__ void emit(bool won, int v, StepAccum& acc) const {
    if (kind == REP_SPARSE) {
      wave_append(won, v, ids, count);
    } else if (won) {
      if (dense.bm) dense.bm[v] = 1;
      else atomicOr((unsigned long long*)&dense.bv[v >> 6], 1ull << (v & 63));
      acc.cnt++;
    }
  }
};

// Grid-stride loop over 64-vertex words, one wave per word.
template <int BT>
__device__ __forceinline__ int first_wave(int bid) { return bid * (BT / kWave) + (int)(threadIdx.x / kWave); }
template <int BT>
__device__ __forceinline__ int num_waves(int nbl) { return nbl * (BT / kWave); }

// Sparse array -> dense set (set must be cleared beforehand).
template <int BT>
__device__ void scatter_to_dense(int bid, int nbl, const int32_t* ids, int count, DenseSet out) {
  for (int i = bid * BT + threadIdx.x; i < count; i += nbl * BT) {
    const int v = ids[i];
    if (out.bm) out.bm[v] = 1;
    else atomicOr((unsigned long long*)&out.bv[v >> 6], 1ull << (v & 63));
  }
}

// Dense set -> sparse array (ascending within a wave; waves in any order).
template <int BT>
__device__ void compact_dense(int bid, int nbl, int n, DenseSet in, int32_t* ids,
                              unsigned long long* count) {
  const int W = (n + 63) >> 6;
  const int lane = __lane_id();
  for (int w = first_wave<BT>(bid); w < W; w += num_waves<BT>(nbl)) {
    const int v = (w << 6) + lane;
    const bool p = v < n && in.test(v);
    wave_append(p, v, ids, count);
  }
}

// Clear a dense set (grid-stride).
template <int BT>
__device__ void clear_dense(int bid, int nbl, int n, DenseSet s) {
  if (s.bm) {
    for (int i = bid * BT + threadIdx.x; i < n; i += nbl * BT) s.bm[i] = 0;
  } else {
    const int W = (n + 63) >> 6;
    for (int i = bid * BT + threadIdx.x; i < W; i += nbl * BT) s.bv[i] = 0ull;
  }
}

}  // namespace gi
