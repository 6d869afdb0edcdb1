// Internal definitions shared by the HIP kernels and the host driver.
// gfx950 (CDNA4): 64-lane wavefronts, 256 CUs in 8 XCDs, 160 KiB LDS per CU.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/graphit_mi.h"

namespace gi {

constexpr int kWave = 64;
// Persistent (cooperative) grids use at most this many workgroups per CU.
constexpr int kMaxPersistentBlocksPerCU = 4;

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
};

// Control block for one algorithm run, in device memory.  Counters for step
// k live in slot k % 3 so that the slot for step k+2 can be cleared while
// step k runs and step k-1's counts are no longer read.
//
// Words that several workgroups update during a kernel sit in cache lines of
// their own and are only written with agent-scope atomics: the per-XCD L2
// caches are not coherent with each other, so a plain store that leaves a
// line dirty in one XCD must never share that line with words other XCDs
// update.  Fields written by workgroup 0 alone and read by the host after
// the kernel (the step log) live in separate lines.
struct alignas(128) StepCounters {
  unsigned long long count;   // |F'| produced by the step
  unsigned long long degsum;  // sum of degrees of F'
  unsigned long long work;    // edges examined by the step
  unsigned long long pad;     // spare counter (frontier compaction)
  unsigned long long fill[12];
};

struct Control {
  // grid barrier (line 0)
  alignas(128) unsigned int bar_count;  // arrivals
  unsigned int bar_gen;                 // generation
  int error;                            // nonzero: a persistent kernel gave up
  int err_block;                        // diagnostics of the first time-out
  unsigned int err_gen;
  unsigned int err_count;
  StepCounters slot[3];                 // lines 1-3
  // SSSP (line 4)
  alignas(128) unsigned long long far_count[2];  // far piles
  unsigned long long minreg[2];                  // smallest far distance
  int overflow;                                  // a distance reached UINT32_MAX
  // host-facing results, written by workgroup 0 only (line 5 on)
  alignas(128) int steps;                        // steps executed
  int dense_steps;
  int done;
  int buckets;                                   // SSSP bucket advances
  unsigned long long edges_examined;
  alignas(128) int dir_log[4096];  // per-step direction
  int f_log[4096];                 // per-step frontier size
  long long d_log[4096];           // per-step frontier degree sum
  long long w_log[4096];           // per-step edges examined
};

__device__ __forceinline__ void atomic_zero(unsigned long long* p) {
  __hip_atomic_store(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_read(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Wave helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

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

// Exclusive prefix sum across the wave (Hillis-Steele with shuffles).
__device__ __forceinline__ int wave_excl_scan(int v, int* total) {
  const int l = __lane_id();
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  *total = __shfl(x, 63, kWave);
  return x - v;
}

// Bounded-spin grid barrier for cooperative launches.  Every workgroup of
// the grid must call it the same number of times.  Every work-item makes its
// own global writes and atomics visible at agent scope before its workgroup
// arrives (a workgroup barrier alone does not wait for other waves' memory
// operations), and acquires after the release, so data written by any XCD
// before the barrier is seen by every XCD after it.  Returns false (and sets
// ctl->error) if the wait exceeds the spin limit, so that a kernel whose grid
// is not fully resident still drains instead of hanging.
__device__ __forceinline__ bool grid_barrier(Control* ctl, unsigned nblocks, unsigned* gen_lds) {
  __shared__ int ok_lds;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned g = *gen_lds;
    const unsigned arrived =
        __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->bar_gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > (1ll << 24)) {
          ok = 0;
          if (__hip_atomic_exchange(&ctl->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            __hip_atomic_store(&ctl->err_block, (int)blockIdx.x, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->err_gen, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->err_count,
                               __hip_atomic_load(&ctl->bar_count, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          break;
        }
        if ((spins & 255) == 0 &&
            __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
      }
    }
    *gen_lds = g + 1;
    ok_lds = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok_lds != 0;
}

// Hybrid rule of the paper (section 2): dense when |F| + sum deg(F) exceeds
// edges / divisor.  Mirrors gi_hybrid_choose_dense on the device.
__host__ __device__ __forceinline__ bool hybrid_dense(long long nf, long long degsum,
                                                      long long edges, int divisor) {
  return (nf + degsum) * (long long)divisor > edges;
}

}  // namespace gi
