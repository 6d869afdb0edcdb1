// Batched persistent execution: many BFS and PageRank instances over graphs
// of uneven size in one kernel launch.
//
// Every instance ("task") owns k workgroups; a task's workgroups meet at a
// task-local barrier between BFS levels and between PageRank iterations,
// so a small instance never waits for the grid and no step costs a kernel
// launch.  Each workgroup runs its (task, rank) list in one global order
// shared by all lists, and every workgroup of the grid is resident at once
// (the grid is sized from the occupancy); so the lowest unfinished task in
// that order always has all its workgroups either at its barriers or
// finished with earlier tasks, and every barrier is reached.  Barrier waits
// are bounded in wall-clock time: past the bound the batch sets an error
// flag, every later wait returns at once, and the kernel drains.
//
// BFS tasks: level-synchronous, direction chosen per level by the hybrid
// rule of the frontier engine (DensePull when |F| + sum deg(F) > m / 20,
// else push of the frontier members in the workgroup's word range, empty
// words skipped, with degree binning); bitvector frontiers in three
// rotating buffers, so the buffer cleared during a level is neither read
// nor written in it.
// PageRank tasks: the destination-block DensePull of pagerank.hip, blocks
// dealt round-robin over the task's workgroups.
// SSSP tasks: delta-stepping in the near/far form of the frontier engine
// (relax the near set; when it empties, move the far members of the next
// bucket into it), with task barriers in place of kernel launches.
//
// The kernel comes in three workgroup sizes (256, 512 and 1024 threads).
// Every workgroup that passes a barrier invalidates its L2 (agent-scope
// acquire), which also drops the lines of the other tasks sharing that L2;
// larger workgroups mean fewer barrier participants for the same threads,
// so the autotuner weighs that against the finer granularity of small ones.
#include "bfs_dev.h"
#include "kernels.h"
#include "pr_block.h"

namespace gi {

// Minimum waves per SIMD for each workgroup size: 5 workgroups of 256, 2 of
// 512 or 1 of 1024 threads per compute unit.
template <int BT>
constexpr int batch_min_waves() {
  return BT == 256 ? 5 : 4;
}

__device__ __forceinline__ long long wall_ticks() { return (long long)wall_clock64(); }

// XCD (XCC) of the calling wave, from the hardware register XCC_ID.
__device__ __forceinline__ unsigned xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu;  // XCC_ID[3:0]
}

// Record this workgroup's XCD in the task's mask; called by every workgroup
// of the task before the task's first barrier.
__device__ __forceinline__ void task_join(TaskCtl* c) {
  if (threadIdx.x == 0) atomicOr(&c->xcds, 1u << xcc_id());
}

// After the task's first barrier: true when every workgroup of the task runs
// on one XCD, so that they share one L2.  Read by all workgroups after the
// same barrier, so all take the same barrier form.
__device__ __forceinline__ bool task_on_one_xcd(const TaskCtl* c) {
  const unsigned m = __hip_atomic_load(&c->xcds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __popc(m) == 1;
}

// Barrier of the k workgroups of one task.  One 64-bit word holds
// (generation << 32) | arrivals, so an arrival learns its generation from
// the same atomic.  Every wave first waits for its own memory operations to
// complete; then one thread per workgroup releases, arrives, waits for the
// generation to move, and acquires for the whole workgroup: two cache
// maintenance operations per workgroup and barrier rather than two per
// wave.
//   Agent scope (the task's workgroups may sit on different XCDs, whose L2s
//   are not coherent with each other): release writes the L2 back, acquire
//   invalidates L1 and L2.
//   One XCD (`local`): the task's workgroups share one L2, and the vector L1
//   writes through to it, so a wave's completed stores are already in the
//   L2 every participant reads: the release's L2 write-back is skipped.
//   The acquire stays the device-scope invalidate: it is the one that drops
//   the CU's stale L1 lines (a group-scope invalidate leaves them outside
//   thread-group-split mode, as a probe of a pre-cached line showed), and
//   it leaves dirty L2 lines in place.  Lines written at several levels are
//   then written back to memory once, not at every barrier.
// Returns false once the batch has failed (timeout here or elsewhere).
__device__ bool task_barrier(TaskCtl* c, int k, int* gerr, long long limit, bool local = false) {
  __shared__ int s_ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = __hip_atomic_load(gerr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    if (ok && k > 1) {
      if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned long long old = atomicAdd(&c->bar, 1ull);
      const unsigned long long gen = old >> 32;
      if ((old & 0xffffffffull) == (unsigned long long)(k - 1)) {
        __hip_atomic_store(&c->bar, (gen + 1ull) << 32, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const long long t0 = wall_ticks();
        while ((__hip_atomic_load(&c->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) ==
               gen) {
          if (__hip_atomic_load(gerr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
            break;
          }
          if (wall_ticks() - t0 > limit) {
            __hip_atomic_store(gerr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __builtin_amdgcn_s_waitcnt(0);
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

template <int BT>
__device__ void bfs_task(const BatchGraph& G, const BatchTask& t, int r, const BatchArgs& a,
                         int* lds) {
  const int n = G.n, k = t.k, W = (n + 63) >> 6, tid = threadIdx.x;
  int32_t* level = static_cast<int32_t*>(t.out);
  TaskCtl* c = t.ctl;
  uint64_t* bv[3] = {t.bv0, t.bv1, t.bv2};
  // this workgroup's words and vertices
  const int w0 = (int)((long long)W * r / k), w1 = (int)((long long)W * (r + 1) / k);
  const int v0 = w0 * 64, v1 = min(n, w1 * 64);
  for (int v = v0 + tid; v < v1; v += BT) {
    level[v] = -1;
    if (t.parent) t.parent[v] = -1;
  }
  for (int w = w0 + tid; w < w1; w += BT) {
    t.vis[w] = 0ull;
    t.bv0[w] = 0ull;
    t.bv1[w] = 0ull;
    t.bv2[w] = 0ull;
  }
  task_join(c);
  if (!task_barrier(c, k, a.error, a.spin_limit)) return;
  const bool local = a.xcd_barrier && task_on_one_xcd(c);
  if (r == 0 && tid == 0) {
    const int s = t.src;
    level[s] = 0;
    if (t.parent) t.parent[s] = s;
    t.bv0[s >> 6] = 1ull << (s & 63);
    t.vis[s >> 6] = 1ull << (s & 63);
    c->qn[0] = 1;
    c->ds[0] = G.outdeg[s];
  }
  if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
  DevGraph dg{};
  dg.n = n;
  dg.m = G.m;
  dg.out_off = G.out_off;
  dg.out_idx = G.out_idx;
  dg.in_off = G.in_off;
  dg.in_idx = G.in_idx;
  dg.outdeg = G.outdeg;
  dg.in_probe = G.in_probe;
  int L = 0;
  for (;; ++L) {
    const long long nf = (long long)__hip_atomic_load(&c->qn[L % 3], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
    const long long df = (long long)__hip_atomic_load(&c->ds[L % 3], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
    if (nf == 0) break;  // task-uniform: read after the same barrier by all
    if (L > n) {         // more levels than vertices: a broken invariant
      if (tid == 0) __hip_atomic_store(a.error, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const bool pull = hybrid_dense(nf, df, G.m, 20);
    if (r == 0 && tid == 0) {
      // read by every workgroup at the previous level, accumulated at the next
      c->qn[(L + 2) % 3] = 0;
      c->ds[(L + 2) % 3] = 0;
      if (L < a.trace_cap) {
        long long* rec = a.trace + ((size_t)t.id * a.trace_cap + L) * 2;
        rec[0] = wall_ticks();
        rec[1] = ((long long)pull << 62) | nf;
      }
    }
    uint64_t* bclr = bv[(L + 2) % 3];
    for (int w = w0 + tid; w < w1; w += BT) bclr[w] = 0ull;
    BfsArgs b{};
    b.g = dg;
    b.level = level;
    b.parent = t.parent;
    b.cur = DenseSet{bv[L % 3], nullptr};
    b.next = DenseSet{bv[(L + 1) % 3], nullptr};
    b.vis = t.vis;
    long long found = 0, found_deg = 0;
    if (pull) {
      bfs_pull_range<BT, (BT == 256 ? 2 : 4)>(b, L + 1, w0, w1, (int)(threadIdx.x / kWave), BT / kWave, G.outdeg,
                          &found, &found_deg);
    } else {
      BfsVisit vis{G.out_idx, level, t.parent, L + 1, b.next, t.vis};
      vis.deg = G.outdeg;
      // a frontier whose degree sum is at most kHubDeg holds no hub
      if (df > kHubDeg) push_hubs<BT>(G.hubs, G.nhubs, b.cur, G.out_off, G.out_idx, r, k, vis);
      push_words<BT>(b.cur.bv, w0, w1, n, G.out_off, vis, kHubDeg, lds);
      found = vis.found;
      found_deg = vis.found_deg;
    }
    const Part p = block_sum4<BT>(Part{found, found_deg, 0, 0});
    if (tid == 0 && p.a > 0) {
      atomicAdd(&c->qn[(L + 1) % 3], (unsigned long long)p.a);
      atomicAdd(&c->ds[(L + 1) % 3], (unsigned long long)p.b);
    }
    if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
  }
  if (r == 0 && tid == 0) {
    c->levels = L;
    if (L < a.trace_cap) {
      long long* rec = a.trace + ((size_t)t.id * a.trace_cap + L) * 2;
      rec[0] = wall_ticks();
      rec[1] = 0;
    }
  }
}


// Relaxation of a batch SSSP phase: push with weights, the improved vertex
// goes to the next near set when its new distance is inside the bucket,
// else to the far set; insertions are counted for the phase totals.
struct BatchSsspVisit {
  const int32_t* idx;
  const uint32_t* w;
  uint32_t* dist;
  DenseSet near;
  DenseSet far;
  unsigned long long thresh;
  int* overflow;
  long long near_new = 0, far_new = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    if (!valid) return;
    const int v = idx[e];
    const unsigned long long nd = (unsigned long long)dist[u] + (unsigned long long)w[e];
    if (nd >= 0xFFFFFFFFull) {
      __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if ((uint32_t)nd >= dist[v]) return;
    const uint32_t old = atomicMin(&dist[v], (uint32_t)nd);
    if ((uint32_t)nd >= old) return;
    if (nd < thresh) {
      if (near.insert(v)) ++near_new;
    } else if (far.insert(v)) {
      ++far_new;
    }
  }
};

template <int BT>
__device__ void sssp_task(const BatchGraph& G, const BatchTask& t, int r, const BatchArgs& a,
                          int* lds) {
  const int n = G.n, k = t.k, W = (n + 63) >> 6, tid = threadIdx.x;
  uint32_t* dist = static_cast<uint32_t*>(t.out);
  TaskCtl* c = t.ctl;
  uint64_t* bv[3] = {t.bv0, t.bv1, t.bv2};
  uint64_t* far = t.vis;
  const unsigned long long delta = t.delta;
  const int w0 = (int)((long long)W * r / k), w1 = (int)((long long)W * (r + 1) / k);
  const int v0 = w0 * 64, v1 = min(n, w1 * 64);
  for (int v = v0 + tid; v < v1; v += BT) dist[v] = 0xFFFFFFFFu;
  for (int w = w0 + tid; w < w1; w += BT) {
    far[w] = 0ull;
    t.bv0[w] = 0ull;
    t.bv1[w] = 0ull;
    t.bv2[w] = 0ull;
  }
  task_join(c);
  if (!task_barrier(c, k, a.error, a.spin_limit)) return;
  const bool local = a.xcd_barrier && task_on_one_xcd(c);
  if (r == 0 && tid == 0) {
    dist[t.src] = 0u;
    t.bv0[t.src >> 6] = 1ull << (t.src & 63);
    c->qn[0] = 1;
    c->thresh = delta;
  }
  if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
  __shared__ unsigned long long s_red[BT / kWave];
  int P = 0;
  for (;; ++P) {
    const long long nf = (long long)__hip_atomic_load(&c->qn[P % 3], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long fc = __hip_atomic_load(&c->farc[P % 3], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long th = __hip_atomic_load(&c->thresh, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_load(&c->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      if (r == 0 && tid == 0) __hip_atomic_store(a.error, 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (nf == 0 && fc == 0) break;  // task-uniform: read after the same barrier by all
    if (P > 2 * n + 2) {            // more phases than possible: a broken invariant
      if (tid == 0) __hip_atomic_store(a.error, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if (r == 0 && tid == 0) {
      c->qn[(P + 2) % 3] = 0;
      c->farc[(P + 2) % 3] = 0;
      if (a.trace_cap > P) {
        long long* rec = a.trace + ((size_t)t.id * a.trace_cap + P) * 2;
        rec[0] = wall_ticks();
        rec[1] = nf;
      }
    }
    uint64_t* cur = bv[P % 3];
    uint64_t* nxt = bv[(P + 1) % 3];
    for (int w = w0 + tid; w < w1; w += BT) bv[(P + 2) % 3][w] = 0ull;
    if (nf > 0) {
      // relax the near set
      if (r == 0 && tid == 0) {
        c->fmin = ~0ull;
        if (fc) atomicAdd(&c->farc[(P + 1) % 3], fc);  // far members carry over
      }
      BatchSsspVisit vis{G.out_idx, G.out_w, dist, DenseSet{nxt, nullptr},
                         DenseSet{far, nullptr}, th, &c->overflow};
      push_words<BT>(cur, w0, w1, n, G.out_off, vis, 0x7fffffff, lds);
      const Part p = block_sum4<BT>(Part{vis.near_new, vis.far_new, 0, 0});
      if (tid == 0) {
        if (p.a) atomicAdd(&c->qn[(P + 1) % 3], (unsigned long long)p.a);
        if (p.b) atomicAdd(&c->farc[(P + 1) % 3], (unsigned long long)p.b);
      }
      if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
      continue;
    }
    // split: the next bucket starts at the smallest far distance at or
    // beyond the threshold
    unsigned long long mn = ~0ull;
    for (int w = w0 + tid; w < w1; w += BT) {
      uint64_t x = far[w];
      while (x) {
        const int v = (w << 6) + __ffsll((long long)x) - 1;
        x &= x - 1;
        const unsigned long long d = dist[v];
        if (d >= th && d < mn) mn = d;
      }
    }
    mn = wave_min(mn);
    if (__lane_id() == 0) s_red[tid / kWave] = mn;
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < BT / kWave; ++i) mn = s_red[i] < mn ? s_red[i] : mn;
      if (mn != ~0ull) atomicMin(&c->fmin, mn);
    }
    if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
    const unsigned long long fm = __hip_atomic_load(&c->fmin, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long tnew = fm == ~0ull ? th : (fm / delta + 1ull) * delta;
    long long moved = 0, kept = 0;
    for (int w = w0 + tid; w < w1; w += BT) {
      uint64_t x = far[w], keep = 0ull, mv = 0ull;
      while (x) {
        const int b = __ffsll((long long)x) - 1;
        x &= x - 1;
        const unsigned long long d = dist[(w << 6) + b];
        if (d < th) continue;  // stale: relaxed in an earlier bucket
        if (d < tnew) {
          mv |= 1ull << b;
          ++moved;
        } else {
          keep |= 1ull << b;
          ++kept;
        }
      }
      far[w] = keep;
      nxt[w] = mv;  // this workgroup's words; cleared two phases ago
    }
    const Part p = block_sum4<BT>(Part{moved, kept, 0, 0});
    if (tid == 0) {
      if (p.a) atomicAdd(&c->qn[(P + 1) % 3], (unsigned long long)p.a);
      if (p.b) atomicAdd(&c->farc[(P + 1) % 3], (unsigned long long)p.b);
    }
    // every workgroup has read the old threshold (it read fmin after the
    // barrier above); rank 0 publishes the new one for the next phase
    if (r == 0 && tid == 0) c->thresh = tnew;
    if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
  }
  if (r == 0 && tid == 0) {
    c->levels = P;
    if (P < a.trace_cap) {
      long long* rec = a.trace + ((size_t)t.id * a.trace_cap + P) * 2;
      rec[0] = wall_ticks();
      rec[1] = 0;
    }
  }
}

template <int BT>
__device__ void pr_task(const BatchGraph& G, const BatchTask& t, int r, const BatchArgs& a,
                        float* lds_val, int* lds_off) {
  const int n = G.n, k = t.k, tid = threadIdx.x;
  TaskCtl* c = t.ctl;
  float* ranks = static_cast<float*>(t.out);
  const int v0 = (int)((long long)n * r / k), v1 = (int)((long long)n * (r + 1) / k);
  const double x0 = 1.0 / (double)n;
  for (int v = v0 + tid; v < v1; v += BT) {
    if (t.iters == 0) {
      ranks[v] = (float)x0;
    } else {
      const int d = G.outdeg[v];
      t.c0[v] = d > 0 ? (float)(x0 / (double)d) : 0.0f;
    }
  }
  for (int i = r * BT + tid; i < G.n_long; i += k * BT) {
    t.lr_acc[i] = 0.0;
    t.lr_cnt[i] = 0u;
  }
  task_join(c);
  if (!task_barrier(c, k, a.error, a.spin_limit)) return;
  const bool local = a.xcd_barrier && task_on_one_xcd(c);
  PrVertex pv;
  pv.outdeg = G.outdeg;
  pv.alpha = (double)t.damping;
  pv.base = (1.0 - (double)t.damping) / (double)n;
  PrRows rows{G.pr_table, G.pr_ntab, G.in_off, G.in_idx, nullptr, t.lr_acc, t.lr_cnt,
              G.lr_chunks};
  for (int it = 0; it <= t.iters; ++it) {
    if (r == 0 && tid == 0 && it < a.trace_cap) {
      long long* rec = a.trace + ((size_t)t.id * a.trace_cap + it) * 2;
      rec[0] = wall_ticks();
      rec[1] = it < t.iters ? (1ll << 62) : 0;
    }
    if (it == t.iters) break;
    const float* cin = (it & 1) ? t.c1 : t.c0;
    float* cout = (it & 1) ? t.c0 : t.c1;
    float* rk = it == t.iters - 1 ? ranks : nullptr;
    for (int tb = r; tb < G.pr_ntab; tb += k)
      pr_rows_block<BT>(rows, tb, G.pr_cap_e, cin, 0, pv, cout, rk, nullptr, lds_val, lds_off);
    if (!task_barrier(c, k, a.error, a.spin_limit, local)) return;
  }
  if (r == 0 && tid == 0) c->levels = t.iters;
}

template <int BT>
__global__ __launch_bounds__(BT, batch_min_waves<BT>()) void k_batch(BatchArgs a) {
  extern __shared__ float smem[];
  float* lds_val = smem;
  int* lds_off = reinterpret_cast<int*>(smem + a.lds_cap_e);
  const int w = blockIdx.x;
  for (int i = a.wg_off[w]; i < a.wg_off[w + 1]; ++i) {
    const int2 it = a.items[i];
    const BatchTask& t = a.tasks[it.x];
    const BatchGraph& G = a.graphs[t.graph];
    if (it.y == 0 && threadIdx.x == 0) t.ctl->t_begin = wall_ticks();
    if (t.alg == ALG_BFS) bfs_task<BT>(G, t, it.y, a, reinterpret_cast<int*>(smem));
    else if (t.alg == ALG_SSSP) sssp_task<BT>(G, t, it.y, a, reinterpret_cast<int*>(smem));
    else pr_task<BT>(G, t, it.y, a, lds_val, lds_off);
    if (it.y == 0 && threadIdx.x == 0) t.ctl->t_end = wall_ticks();
  }
}

// Reset of the task control blocks and the error flag (part of the same
// stream order as the batch, and of its graph when captured).
__global__ void k_batch_init(TaskCtl* ctl, int ntasks, int* error) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ntasks; i += gridDim.x * blockDim.x) {
    TaskCtl z{};
    ctl[i] = z;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *error = 0;
}

// Dynamic LDS: the PageRank block staging or the BFS push member list,
// whichever is larger (a workgroup runs one task at a time).
size_t batch_lds_bytes(int cap_e, int cap_v) {
  return std::max(sizeof(float) * (size_t)cap_e + sizeof(int) * (size_t)(cap_v + 1),
                  sizeof(int) * (size_t)kPushList);
}

bool batch_threads_ok(int bt) { return bt == 256 || bt == 512 || bt == 1024; }

int batch_occupancy(int bt, size_t lds) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (bt) {
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<256>, 256, lds); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<512>, 512, lds); break;
    case 1024: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_batch<1024>, 1024, lds); break;
    default: return -1;
  }
  return e == hipSuccess ? blocks : -1;
}

int launch_batch(const BatchArgs& a, int bt, int grid, size_t lds, TaskCtl* ctl, int ntasks,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3(std::max(1, std::min(64, (ntasks + 255) / 256))),
                     dim3(256), 0, s, ctl, ntasks, a.error);
  switch (bt) {
    case 256: hipLaunchKernelGGL(k_batch<256>, dim3(grid), dim3(256), lds, s, a); break;
    case 512: hipLaunchKernelGGL(k_batch<512>, dim3(grid), dim3(512), lds, s, a); break;
    case 1024: hipLaunchKernelGGL(k_batch<1024>, dim3(grid), dim3(1024), lds, s, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gi
