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

// Record this workgroup's XCD in the task's mask and count; called by every
// workgroup of the task before the task's first barrier.
__device__ __forceinline__ void task_join(TaskCtl* c) {
  if (threadIdx.x == 0) {
    const unsigned x = xcc_id() & 7u;
    atomicOr(&c->xcds, 1u << x);
    atomicAdd(&c->xcnt[x], 1u);
  }
}

// Barrier forms after the task's first barrier (which is always the agent
// form: the XCD counts are final only after it).
enum { kBarAgent = 0, kBarLocal = 1, kBarTree = 2 };

// The form for the task's later barriers, from its XCDs: one XCD shares one
// L2 (kBarLocal); several count their arrivals per XCD first (kBarTree).
// Read by all workgroups after the same barrier, so all take the same form.
__device__ __forceinline__ int task_barrier_form(const TaskCtl* c, int xcd_barrier) {
  if (!xcd_barrier) return kBarAgent;
  const unsigned m = __hip_atomic_load(&c->xcds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __popc(m) == 1 ? kBarLocal : kBarTree;
}

// Wall-clock ticks the calling workgroup has spent in task barriers during
// its current task (thread 0 keeps it; k_batch resets and reports it).
__device__ __forceinline__ long long& barrier_ticks() {
  __shared__ long long s_ticks;
  return s_ticks;
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
//   Tree (several XCDs): as agent scope, but the arrivals meet first in a
//   counter of their XCD (a line of its own), and only each XCD's last
//   arrival goes on to the task's word: at most 8 arrivals meet there
//   instead of k, and the k atomics on one line no longer serialise.
//   One XCD (`local`): the task's workgroups share one L2, and the vector L1
//   writes through to it, so a wave's completed stores are already in the
//   L2 every participant reads: the release's L2 write-back is skipped.
//   The acquire stays the device-scope invalidate: it is the one that drops
//   the CU's stale L1 lines (a group-scope invalidate leaves them outside
//   thread-group-split mode, as a probe of a pre-cached line showed), and
//   it leaves dirty L2 lines in place.  Lines written at several levels are
//   then written back to memory once, not at every barrier.
// Returns false once the batch has failed (timeout here or elsewhere).
__device__ bool task_barrier(TaskCtl* c, int k, int* gerr, long long limit,
                             int form = kBarAgent) {
  __shared__ int s_ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = __hip_atomic_load(gerr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    if (ok && k > 1) {
      const long long t0 = wall_ticks();
      if (form != kBarLocal) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      unsigned long long gen;
      bool last = false;
      if (form == kBarTree) {
        // the generation cannot move before this workgroup arrives
        gen = __hip_atomic_load(&c->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32;
        const unsigned x = xcc_id() & 7u;
        const unsigned here = __hip_atomic_load(&c->xcnt[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (atomicAdd(&c->xarr[x][0], 1ull) == (unsigned long long)here - 1ull) {
          // this XCD's last arrival: clear its counter for the next barrier
          // (done before the task's word moves, so no later arrival misses
          // it) and arrive for the XCD
          __hip_atomic_store(&c->xarr[x][0], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_s_waitcnt(0);
          const unsigned nx = __popc(__hip_atomic_load(&c->xcds, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT));
          last = (atomicAdd(&c->bar, 1ull) & 0xffffffffull) == (unsigned long long)(nx - 1);
        }
      } else {
        const unsigned long long old = atomicAdd(&c->bar, 1ull);
        gen = old >> 32;
        last = (old & 0xffffffffull) == (unsigned long long)(k - 1);
      }
      if (last) {
        __hip_atomic_store(&c->bar, (gen + 1ull) << 32, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      } else {
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
      barrier_ticks() += wall_ticks() - t0;
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
  const int bform = task_barrier_form(c, a.xcd_barrier);
  if (r == 0 && tid == 0) {
    const int s = t.src;
    level[s] = 0;
    if (t.parent) t.parent[s] = s;
    t.bv0[s >> 6] = 1ull << (s & 63);
    t.vis[s >> 6] = 1ull << (s & 63);
    c->qn[0] = 1;
    c->ds[0] = G.outdeg[s];
  }
  if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
  DevGraph dg{};
  dg.n = n;
  dg.m = G.m;
  dg.out_off = G.out_off;
  dg.out_idx = G.out_idx;
  dg.in_off = G.in_off;
  dg.in_idx = G.in_idx;
  dg.outdeg = G.outdeg;
  dg.in_probe = G.in_probe;
  dg.bfs_idx = G.bfs_idx;
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
    const bool pull = hybrid_dense(nf, df, G.m, t.div);
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
    if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
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


// Appends v of each lane that holds one (v >= 0; -1: none) to q, at
// positions taken from *tail by one atomic per wave.
__device__ __forceinline__ void wave_append(int32_t* q, unsigned long long* tail, int v) {
  const unsigned long long mk = __ballot(v >= 0);
  if (mk == 0ull) return;
  const int lane = __lane_id();
  const int leader = __ffsll((long long)mk) - 1;
  int base = 0;
  if (lane == leader) base = (int)atomicAdd(tail, (unsigned long long)__popcll(mk));
  base = __shfl(base, leader, kWave);
  if (v >= 0) q[base + __popcll(mk & ((1ull << lane) - 1ull))] = v;
}

// Appends the members of word w held in bits (each lane its own word; 0:
// none) to q, at positions taken from *tail by one atomic per wave.
__device__ __forceinline__ void wave_append_bits(int32_t* q, unsigned long long* tail, int w,
                                                 uint64_t bits) {
  int tot;
  const int ex = wave_excl_scan((int)__popcll(bits), &tot);
  if (tot == 0) return;
  int base = 0;
  if (__lane_id() == 0) base = (int)atomicAdd(tail, (unsigned long long)tot);
  base = __shfl(base, 0, kWave) + ex;
  while (bits) {
    q[base++] = (w << 6) + __ffsll((long long)bits) - 1;
    bits &= bits - 1;
  }
}

// Relaxation of a scanned (word by word) batch SSSP phase: push with
// weights, the improved vertex goes to the next near set when its new
// distance is inside the bucket, else to the far set.  A vertex newly
// entered into a set is also written to that set's workgroup buffer in LDS
// (cap entries each; the counters keep counting past it), which the phase
// appends to the set's list at its end: the lists cost no round trip per
// edge.
struct BatchSsspVisit {
  const int32_t* idx;
  const uint32_t* w;
  uint32_t* dist;
  DenseSet near;
  DenseSet far;
  int* qbuf;  // LDS: new near members
  int* qcnt;
  int* fbuf;  // LDS: new far members
  int* fcnt;
  int cap;
  unsigned long long thresh;
  int* overflow;
  long long far_new = 0, edges = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    edges += valid;
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
      if (near.insert(v)) {
        const int p = atomicAdd(qcnt, 1);
        if (p < cap) qbuf[p] = v;
      }
    } else if (far.insert(v)) {
      ++far_new;
      const int p = atomicAdd(fcnt, 1);
      if (p < cap) fbuf[p] = v;
    }
  }
};

// A set of at most n / 64 members is cleared through its list: the list is
// no longer than the bitvector's words.
__device__ __forceinline__ bool sssp_list_clear(long long members, int n) {
  return members * 64 <= (long long)n;
}

// Local lists of a walked phase, in the kernel's dynamic LDS (int words):
// two lists of C entries (vertex, distance, row start, degree), the degree
// prefix of the list being expanded, and CF far candidates.
template <int BT>
struct WalkLds {
  static constexpr int C = BT < 384 ? BT : 384;
  static constexpr int CF = 512;
  static constexpr int kInts = 9 * C + 1 + CF;
  static_assert(kInts <= kPushList, "walk lists exceed the batch LDS");
};

// A near set that gives each of the task's k workgroups at most one local
// list (C members) is walked: such phases are few vertices deep and bound by
// memory latency, which the walk's local rounds pay without task barriers.
// Larger sets are scanned word by word in vertex order, all workgroups busy.
template <int BT>
__device__ __forceinline__ bool sssp_walk(long long members, int k) {
  return members <= (long long)k * WalkLds<BT>::C;
}

// One walked phase of a workgroup: its share ids[lo, hi) of the near set is
// relaxed, and so is every vertex those relaxations move into the current
// bucket, round after round from a workgroup-local list, until the list is
// empty (label-correcting inside the bucket, as the phases of the bucket
// are; every improvement is relaxed by the workgroup that made it, with the
// distance it wrote).  A round needs two dependent memory trips (the edge,
// then the atomic minimum together with the target's row bounds) and no
// task barrier.  Entries beyond the list's capacity go to the next phase's
// near set (nxt and its list); far improvements are gathered in LDS and
// entered into the far set once at the end.  Returns the far insertions;
// *edges (thread 0) counts the edges relaxed.
template <int BT>
__device__ long long sssp_walk_phase(const BatchGraph& G, uint32_t* dist, const int32_t* ids,
                                     long long lo, long long hi, unsigned long long th,
                                     DenseSet nxt, int32_t* near_q, unsigned long long* near_tail,
                                     DenseSet far, int32_t* far_q, unsigned long long* far_tail,
                                     int* overflow, int* lds, long long* edges) {
  using L = WalkLds<BT>;
  constexpr int C = L::C, CF = L::CF;
  int* Lv = lds;              // [2][C] vertex
  int* Ld = lds + 2 * C;      // [2][C] distance it was given
  int* Lb = lds + 4 * C;      // [2][C] row start
  int* Lg = lds + 6 * C;      // [2][C] degree
  int* pre = lds + 8 * C;     // [C + 1] degree prefix of the list in expansion
  int* fbuf = lds + 9 * C + 1;  // [CF] far candidates
  __shared__ int s_cnt[2], s_fcnt;
  const int tid = threadIdx.x, lane = __lane_id();
  const int32_t* off = G.out_off;
  const int32_t* idx = G.out_idx;
  const uint32_t* wt = G.out_w;
  long long far_new = 0;
  if (tid == 0) s_fcnt = 0;
  for (long long c0 = lo; c0 < hi; c0 += C) {  // block-uniform
    const int cnt0 = (int)min((long long)C, hi - c0);
    if (tid < cnt0) {
      const int v = ids[c0 + tid];
      const int b = off[v], e = off[v + 1];
      Lv[tid] = v;
      Ld[tid] = (int)dist[v];
      Lb[tid] = b;
      Lg[tid] = e - b;
    }
    if (tid == 0) s_cnt[0] = cnt0;
    int a = 0;
    __syncthreads();
    for (;;) {
      const int cnt = min(s_cnt[a], C);
      if (cnt == 0) break;  // block-uniform: read after a barrier, written before it
      int E;
      const int ex = block_excl_scan<BT>(tid < cnt ? Lg[a * C + tid] : 0, &E);
      if (tid < cnt) pre[tid] = ex;
      if (tid == 0) {
        s_cnt[a ^ 1] = 0;
        *edges += E;
      }
      __syncthreads();
      const int b = a ^ 1;
      for (int t0 = 0; t0 < E; t0 += BT) {  // block-uniform: the appends are wave-wide
        const int t = t0 + tid;
        int to_loc = -1, to_far = -1, nb = 0, ng = 0;
        unsigned ndv = 0;
        if (t < E) {
          int jl = 0, jh = cnt - 1;  // the last entry whose prefix is <= t
          while (jl < jh) {
            const int mid = (jl + jh + 1) >> 1;
            if (pre[mid] <= t) jl = mid;
            else jh = mid - 1;
          }
          const int e = Lb[a * C + jl] + (t - pre[jl]);
          const int v = idx[e];
          const unsigned long long nd =
              (unsigned long long)(unsigned)Ld[a * C + jl] + (unsigned long long)wt[e];
          if (nd >= 0xFFFFFFFFull) {
            __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            // the row bounds are loaded before the atomic: one round trip for both
            nb = off[v];
            const int ne = off[v + 1];
            const uint32_t old = atomicMin(&dist[v], (uint32_t)nd);
            if ((uint32_t)nd < old) {
              if (nd < th) {
                to_loc = v;
                ndv = (unsigned)nd;
                ng = ne - nb;
              } else {
                to_far = v;
              }
            }
          }
        }
        // into the next local list; past its capacity into the next phase
        int spill = -1;
        unsigned long long mk = __ballot(to_loc >= 0);
        if (mk) {
          const int leader = __ffsll((long long)mk) - 1;
          int base = 0;
          if (lane == leader) base = atomicAdd(&s_cnt[b], __popcll(mk));
          base = __shfl(base, leader, kWave);
          if (to_loc >= 0) {
            const int pos = base + __popcll(mk & ((1ull << lane) - 1ull));
            if (pos < C) {
              Lv[b * C + pos] = to_loc;
              Ld[b * C + pos] = (int)ndv;
              Lb[b * C + pos] = nb;
              Lg[b * C + pos] = ng;
            } else {
              spill = to_loc;
            }
          }
          if (__ballot(spill >= 0)) {
            const int ins = (spill >= 0 && nxt.insert(spill)) ? spill : -1;
            wave_append(near_q, near_tail, ins);
          }
        }
        // far candidates wait in LDS for one insertion pass at the end
        int fspill = -1;
        mk = __ballot(to_far >= 0);
        if (mk) {
          const int leader = __ffsll((long long)mk) - 1;
          int base = 0;
          if (lane == leader) base = atomicAdd(&s_fcnt, __popcll(mk));
          base = __shfl(base, leader, kWave);
          if (to_far >= 0) {
            const int pos = base + __popcll(mk & ((1ull << lane) - 1ull));
            if (pos < CF) fbuf[pos] = to_far;
            else fspill = to_far;
          }
          if (__ballot(fspill >= 0)) {
            const int ins = (fspill >= 0 && far.insert(fspill)) ? fspill : -1;
            wave_append(far_q, far_tail, ins);
            far_new += ins >= 0;
          }
        }
      }
      __syncthreads();
      a = b;
    }
    __syncthreads();  // every thread has seen the empty list before the next chunk
  }
  __syncthreads();  // s_fcnt is final (also when the share was empty)
  const int fc = min(s_fcnt, CF);
  for (int i0 = 0; i0 < fc; i0 += BT) {  // block-uniform: the appends are wave-wide
    const int i = i0 + tid;
    int ins = -1;
    if (i < fc) {
      const int v = fbuf[i];
      if (far.insert(v)) ins = v;
    }
    wave_append(far_q, far_tail, ins);
    far_new += ins >= 0;
  }
  return far_new;
}

// Rank r's share [lo, hi) of len list entries split over k workgroups.
__device__ __forceinline__ void list_share(long long len, int r, int k, long long* lo,
                                           long long* hi) {
  *lo = len * r / k;
  *hi = len * (r + 1) / k;
}

template <int BT>
__device__ void sssp_task(const BatchGraph& G, const BatchTask& t, int r, const BatchArgs& a,
                          int* lds) {
  const int n = G.n, k = t.k, W = (n + 63) >> 6, tid = threadIdx.x;
  uint32_t* dist = static_cast<uint32_t*>(t.out);
  TaskCtl* c = t.ctl;
  uint64_t* bv[3] = {t.bv0, t.bv1, t.bv2};
  int32_t* nq[3] = {t.q, t.q + (size_t)n, t.q + 2 * (size_t)n};  // member lists of bv[]
  int32_t* fl[2] = {t.q + 3 * (size_t)n, t.q + 4 * (size_t)n};    // far lists, alternating
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
  const int bform = task_barrier_form(c, a.xcd_barrier);
  if (r == 0 && tid == 0) {
    dist[t.src] = 0u;
    t.bv0[t.src >> 6] = 1ull << (t.src & 63);
    nq[0][0] = t.src;
    c->qn[0] = 1;
    c->thresh = delta;
  }
  if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
  __shared__ unsigned long long s_red[BT / kWave];
  // scanned phases: the new members of the next near set and of the far set
  constexpr int kBuf = 512;
  __shared__ int s_qbuf[kBuf], s_fbuf[kBuf];
  __shared__ int s_qcnt, s_fcnt;
  __shared__ long long s_base[2];
  long long relaxed = 0;  // edges this workgroup relaxed (thread 0)
  long long prev = 0;     // members of the previous phase's near set
  bool prev_listed = true;  // ... and whether its list was complete
  int fs = 0;             // far list in use
  int P = 0;
  for (;; ++P) {
    const long long nf = (long long)__hip_atomic_load(&c->qn[P % 3], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
    const bool listed = __hip_atomic_load(&c->qbad[P % 3], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT) == 0;
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
      // the counters of the phase after next (read by all in the previous phase)
      c->qn[(P + 2) % 3] = 0;
      c->qbad[(P + 2) % 3] = 0;
      c->farc[(P + 2) % 3] = 0;
      if (a.trace_cap > P) {
        long long* rec = a.trace + ((size_t)t.id * a.trace_cap + P) * 2;
        rec[0] = wall_ticks();
        rec[1] = nf;
      }
    }
    uint64_t* cur = bv[P % 3];
    uint64_t* nxt = bv[(P + 1) % 3];
    // the previous phase's near set is cleared for the next phase to fill:
    // through its list when short and complete, else word by word
    uint64_t* bclr = bv[(P + 2) % 3];
    long long lo, hi;
    if (prev_listed && sssp_list_clear(prev, n)) {
      const int32_t* q = nq[(P + 2) % 3];
      list_share(prev, r, k, &lo, &hi);
      for (long long i = lo + tid; i < hi; i += BT) bclr[q[i] >> 6] = 0ull;
    } else {
      for (int w = w0 + tid; w < w1; w += BT) bclr[w] = 0ull;
    }
    prev = nf;
    prev_listed = listed;
    if (nf > 0) {
      // relax the near set
      if (r == 0 && tid == 0) {
        c->fmin = ~0ull;
        if (fc) atomicAdd(&c->farc[(P + 1) % 3], fc);  // far members carry over
      }
      long long far_new, edges = 0;
      if (listed && sssp_walk<BT>(nf, k)) {
        list_share(nf, r, k, &lo, &hi);
        far_new = sssp_walk_phase<BT>(G, dist, nq[P % 3], lo, hi, th, DenseSet{nxt, nullptr},
                                      nq[(P + 1) % 3], &c->qn[(P + 1) % 3],
                                      DenseSet{far, nullptr}, fl[fs], &c->ft[fs], &c->overflow,
                                      lds, &edges);
      } else {
        if (tid == 0) s_qcnt = s_fcnt = 0;
        __syncthreads();
        BatchSsspVisit vis{G.out_idx, G.out_w, dist, DenseSet{nxt, nullptr},
                           DenseSet{far, nullptr}, s_qbuf, &s_qcnt, s_fbuf, &s_fcnt, kBuf, th,
                           &c->overflow};
        push_words<BT>(cur, w0, w1, n, G.out_off, vis, 0x7fffffff, lds);
        far_new = vis.far_new;
        edges = vis.edges;
        // the buffers go to the lists; a buffer that overflowed leaves its
        // list incomplete, which the flags record
        __syncthreads();
        const int qn_ = s_qcnt, fn_ = s_fcnt;
        if (tid == 0) {
          s_base[0] = qn_ ? (long long)atomicAdd(&c->qn[(P + 1) % 3], (unsigned long long)qn_) : 0;
          s_base[1] = fn_ ? (long long)atomicAdd(&c->ft[fs], (unsigned long long)min(fn_, kBuf)) : 0;
          if (qn_ > kBuf) __hip_atomic_store(&c->qbad[(P + 1) % 3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (fn_ > kBuf) __hip_atomic_store(&c->fbad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        for (int i = tid; i < min(qn_, kBuf); i += BT) nq[(P + 1) % 3][s_base[0] + i] = s_qbuf[i];
        for (int i = tid; i < min(fn_, kBuf); i += BT) fl[fs][s_base[1] + i] = s_fbuf[i];
      }
      const Part p = block_sum4<BT>(Part{far_new, edges, 0, 0});
      if (tid == 0 && p.a) atomicAdd(&c->farc[(P + 1) % 3], (unsigned long long)p.a);
      relaxed += p.b;  // thread 0's sum
      if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
      continue;
    }
    // split: the next bucket starts at the smallest far distance at or
    // beyond the threshold.  The far set is walked from its list when the
    // list is complete, else scanned word by word; a scan rebuilds the list
    // when the set is short enough to be walked next time.
    const bool fwalk = __hip_atomic_load(&c->fbad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    const bool rebuild = fwalk || sssp_list_clear((long long)fc, n);
    const long long flen = (long long)__hip_atomic_load(&c->ft[fs], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
    const int32_t* fcur = fl[fs];
    list_share(flen, r, k, &lo, &hi);
    unsigned long long mn = ~0ull;
    if (fwalk) {
      for (long long i = lo + tid; i < hi; i += BT) {
        const unsigned long long d = dist[fcur[i]];
        if (d >= th && d < mn) mn = d;
      }
    } else {
      for (int w = w0 + tid; w < w1; w += BT) {
        uint64_t x = far[w];
        while (x) {
          const unsigned long long d = dist[(w << 6) + __ffsll((long long)x) - 1];
          x &= x - 1;
          if (d >= th && d < mn) mn = d;
        }
      }
    }
    mn = wave_min(mn);
    if (__lane_id() == 0) s_red[tid / kWave] = mn;
    __syncthreads();
    if (tid == 0) {
      for (int i = 0; i < BT / kWave; ++i) mn = s_red[i] < mn ? s_red[i] : mn;
      if (mn != ~0ull) atomicMin(&c->fmin, mn);
    }
    if (r == 0 && tid == 0) c->ft[fs ^ 1] = 0;  // the list the kept members go to
    if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
    // every workgroup has read fbad above
    if (r == 0 && tid == 0) c->fbad = rebuild ? 0 : 1;
    const unsigned long long fm = __hip_atomic_load(&c->fmin, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long tnew = fm == ~0ull ? th : (fm / delta + 1ull) * delta;
    long long kept = 0;
    if (fwalk) {
      for (long long b0 = lo; b0 < hi; b0 += BT) {  // block-uniform: the appends are wave-wide
        const long long i = b0 + tid;
        int mv = -1, kp = -1;
        if (i < hi) {
          const int v = fcur[i];
          const unsigned long long d = dist[v];
          const unsigned long long bit = 1ull << (v & 63);
          if (d < tnew) {
            atomicAnd((unsigned long long*)&far[v >> 6], ~bit);
            if (d >= th) {  // below th: stale, relaxed in an earlier bucket
              atomicOr((unsigned long long*)&nxt[v >> 6], bit);
              mv = v;
            }
          } else {
            kp = v;
          }
        }
        wave_append(nq[(P + 1) % 3], &c->qn[(P + 1) % 3], mv);
        wave_append(fl[fs ^ 1], &c->ft[fs ^ 1], kp);
        kept += kp >= 0;
      }
    } else {
      for (int b0 = w0; b0 < w1; b0 += BT) {  // block-uniform: the appends are wave-wide
        const int w = b0 + tid;
        uint64_t keep = 0ull, mv = 0ull;
        if (w < w1) {
          uint64_t x = far[w];
          while (x) {
            const int b = __ffsll((long long)x) - 1;
            x &= x - 1;
            const unsigned long long d = dist[(w << 6) + b];
            if (d < th) continue;  // stale: relaxed in an earlier bucket
            if (d < tnew) mv |= 1ull << b;
            else keep |= 1ull << b;
          }
          far[w] = keep;
          nxt[w] = mv;  // this workgroup's words; cleared in the previous phase
        }
        wave_append_bits(nq[(P + 1) % 3], &c->qn[(P + 1) % 3], w, mv);
        if (rebuild) wave_append_bits(fl[fs ^ 1], &c->ft[fs ^ 1], w, keep);
        kept += __popcll(keep);
      }
    }
    const Part p = block_sum4<BT>(Part{kept, 0, 0, 0});
    if (tid == 0 && p.a) atomicAdd(&c->farc[(P + 1) % 3], (unsigned long long)p.a);
    // every workgroup has read the old threshold (it read fmin after the
    // barrier above); rank 0 publishes the new one for the next phase
    if (r == 0 && tid == 0) c->thresh = tnew;
    fs ^= 1;
    if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
  }
  if (tid == 0 && relaxed) atomicAdd(&c->relaxed, (unsigned long long)relaxed);
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
  const int bform = task_barrier_form(c, a.xcd_barrier);
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
    if (!task_barrier(c, k, a.error, a.spin_limit, bform)) return;
  }
  if (r == 0 && tid == 0) c->levels = t.iters;
}

// ALGS: the task bodies built in (kBatchBfs, or kBatchAll).  Without the
// SSSP and PageRank bodies the BFS path keeps more of its values in
// registers.
template <int BT, int ALGS>
__global__ __launch_bounds__(BT, batch_min_waves<BT>()) void k_batch(BatchArgs a) {
  extern __shared__ float smem[];
  float* lds_val = smem;
  int* lds_off = reinterpret_cast<int*>(smem + a.lds_cap_e);
  const int w = blockIdx.x;
  for (int i = a.wg_off[w]; i < a.wg_off[w + 1]; ++i) {
    const int2 it = a.items[i];
    const BatchTask& t = a.tasks[it.x];
    const BatchGraph& G = a.graphs[t.graph];
    if (threadIdx.x == 0) barrier_ticks() = 0;
    if (it.y == 0 && threadIdx.x == 0) t.ctl->t_begin = wall_ticks();
    if (t.alg == ALG_BFS) {
      if constexpr ((ALGS & kBatchBfs) != 0)
        bfs_task<BT>(G, t, it.y, a, reinterpret_cast<int*>(smem));
    } else if (t.alg == ALG_SSSP) {
      if constexpr ((ALGS & kBatchSssp) != 0)
        sssp_task<BT>(G, t, it.y, a, reinterpret_cast<int*>(smem));
    } else {
      if constexpr ((ALGS & kBatchPr) != 0) pr_task<BT>(G, t, it.y, a, lds_val, lds_off);
    }
    if (it.y == 0 && threadIdx.x == 0) t.ctl->t_end = wall_ticks();
    if (threadIdx.x == 0 && barrier_ticks() > 0)
      atomicAdd(&t.ctl->bar_ticks, (unsigned long long)barrier_ticks());
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

template <int BT, int ALGS>
static hipError_t batch_occ(int* blocks, size_t lds) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<BT, ALGS>, BT, lds);
}

int batch_occupancy(int bt, size_t lds, int algs) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
  const bool bfs = algs == kBatchBfs;
  switch (bt) {
    case 256: e = bfs ? batch_occ<256, kBatchBfs>(&blocks, lds) : batch_occ<256, kBatchAll>(&blocks, lds); break;
    case 512: e = bfs ? batch_occ<512, kBatchBfs>(&blocks, lds) : batch_occ<512, kBatchAll>(&blocks, lds); break;
    case 1024: e = bfs ? batch_occ<1024, kBatchBfs>(&blocks, lds) : batch_occ<1024, kBatchAll>(&blocks, lds); break;
    default: return -1;
  }
  return e == hipSuccess ? blocks : -1;
}

int launch_batch(const BatchArgs& a, int bt, int grid, size_t lds, TaskCtl* ctl, int ntasks,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_batch_init, dim3(std::max(1, std::min(64, (ntasks + 255) / 256))),
                     dim3(256), 0, s, ctl, ntasks, a.error);
#define GI_BATCH_LAUNCH(B)                                                         \
  if (bt == B) {                                                                   \
    if (a.algs == kBatchBfs)                                                       \
      hipLaunchKernelGGL((k_batch<B, kBatchBfs>), dim3(grid), dim3(B), lds, s, a); \
    else                                                                           \
      hipLaunchKernelGGL((k_batch<B, kBatchAll>), dim3(grid), dim3(B), lds, s, a); \
    return hipGetLastError() == hipSuccess ? 0 : -1;                               \
  }
  GI_BATCH_LAUNCH(256)
  GI_BATCH_LAUNCH(512)
  GI_BATCH_LAUNCH(1024)
#undef GI_BATCH_LAUNCH
  return -1;
}

}  // namespace gi
