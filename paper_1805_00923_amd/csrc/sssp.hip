// Single-source shortest paths by delta-stepping (Meyer and Sanders, J.
// Algorithms 2003) in its two-pile GPU form: the "near" pile holds vertices
// whose tentative distance lies below the current bucket threshold T and is
// relaxed repeatedly by SparsePush steps with atomic-min updates (the
// asyncMin reduction of the compiler section); improved vertices at or
// beyond T go to the "far" pile.  When the near pile empties, T moves to the
// end of the bucket that holds the smallest far distance and the far pile is
// split.  The paper's own SSSP is frontier Bellman-Ford; both reach the
// unique shortest-path distances.
#include "kernels.h"
#include "traverse.h"

namespace gi {

struct SsspVisit {
  const int32_t* idx;
  const uint32_t* w;
  uint32_t* dist;
  int32_t* stamp;      // phase a vertex was last queued for (near pile)
  int32_t* in_far;     // 1 while a vertex sits in the far pile
  int32_t* far_ids;
  unsigned long long* far_count;
  int next_phase;
  unsigned long long thresh;
  int* overflow;
  PushOut out;         // near pile of the next phase
  StepAccum acc;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    bool to_near = false, to_far = false;
    int v = -1;
    if (valid) {
      v = idx[e];
      acc.work++;
      const unsigned long long nd = (unsigned long long)dist[u] + (unsigned long long)w[e];
      if (nd >= 0xFFFFFFFFull) {
        __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else if ((uint32_t)nd < dist[v]) {
        const uint32_t old = atomicMin(&dist[v], (uint32_t)nd);
        if ((uint32_t)nd < old) {
          if (nd < thresh) to_near = atomicExch(&stamp[v], next_phase) != next_phase;
          else to_far = atomicExch(&in_far[v], 1) == 0;
        }
      }
    }
    out.emit(to_near, v, acc);
    wave_append(to_far, v, far_ids, far_count);
  }
};

template <int BT>
__device__ void sssp_body(const SsspParams& p, unsigned* gen) {
  const int bid = blockIdx.x, nbl = gridDim.x;
  Control* ctl = p.ctl;
  SsspState s = *p.st;
  for (int it = 0; it < p.max_phases; ++it) {
    StepCounters* in = &ctl->slot[s.phase % 3];
    const long long nn =
        (long long)__hip_atomic_load(&in->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bid == 0 && threadIdx.x == 0 && ctl->steps > 0 && ctl->steps <= 4096 &&
        ctl->w_log[ctl->steps - 1] == 0)
      ctl->w_log[ctl->steps - 1] = (long long)atomic_read(&ctl->slot[s.phase % 3].work);
    if (nn > 0) {
      // ---- relax the near pile (one SparsePush step)
      StepCounters* outc = &ctl->slot[(s.phase + 1) % 3];
      if (bid == 0 && threadIdx.x == 0) {
        const int k = ctl->steps;
        if (k < 4096) {
          ctl->dir_log[k] = GI_DIR_SPARSE_PUSH;
          ctl->f_log[k] = (int)nn;
          ctl->d_log[k] = (long long)atomic_read(&in->degsum);
        }
        ctl->steps = k + 1;
        if (k < 4096) ctl->w_log[k] = 0;
        StepCounters* z = &ctl->slot[(s.phase + 2) % 3];
        atomic_zero(&z->count);
        atomic_zero(&z->degsum);
        atomic_zero(&z->work);
        atomic_zero(&z->pad);
      }
      PushOut po;
      po.kind = REP_SPARSE;
      po.ids = p.near[s.near_cur ^ 1];
      po.count = &outc->count;
      po.dense = DenseSet{nullptr, nullptr};
      SsspVisit vis{p.g.out_idx, p.g.out_w, p.dist, p.stamp, p.in_far, p.far[s.far_cur],
                    &ctl->far_count[s.far_cur], s.phase + 1, s.thresh, &ctl->overflow, po,
                    StepAccum()};
      SparseItems items{p.near[s.near_cur], (int)nn, p.g.out_off};
      push_expand<BT>(bid, nbl, items, vis);
      vis.acc.flush(outc, false);
      s.near_cur ^= 1;
      s.phase += 1;
      if (!grid_barrier(ctl, nbl, gen)) return;
      continue;
    }
    // ---- near pile empty: move to the next non-empty bucket
    const long long nfar = (long long)__hip_atomic_load(&ctl->far_count[s.far_cur], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
    if (nfar == 0) {
      if (bid == 0 && threadIdx.x == 0) ctl->done = 1;
      break;
    }
    const int32_t* fids = p.far[s.far_cur];
    unsigned long long* mreg = &ctl->minreg[s.far_cur];
    for (int i = bid * BT + threadIdx.x; i < nfar; i += nbl * BT) {
      const uint32_t d = p.dist[fids[i]];
      if (d >= s.thresh) atomicMin(mreg, (unsigned long long)d);
    }
    if (bid == 0 && threadIdx.x == 0) {
      atomic_zero(&ctl->far_count[s.far_cur ^ 1]);
      __hip_atomic_store(&ctl->minreg[s.far_cur ^ 1], ~0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!grid_barrier(ctl, nbl, gen)) return;
    const unsigned long long mn =
        __hip_atomic_load(mreg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long told = s.thresh;
    const unsigned long long tnew = mn == ~0ull ? told : (mn / p.delta + 1ull) * p.delta;
    int32_t* near_out = p.near[s.near_cur];
    unsigned long long* ncount = &ctl->slot[s.phase % 3].count;  // 0 here
    for (int base = bid * BT; base < nfar; base += nbl * BT) {
      const int i = base + threadIdx.x;
      int v = -1;
      uint32_t d = 0;
      if (i < nfar) {
        v = fids[i];
        d = p.dist[v];
        p.in_far[v] = 0;
      }
      const bool keep_far = i < nfar && d >= tnew;
      const bool go_near = i < nfar && d >= told && d < tnew;
      if (keep_far) p.in_far[v] = 1;
      if (go_near) p.stamp[v] = s.phase;
      wave_append(go_near, v, near_out, ncount);
      wave_append(keep_far, v, p.far[s.far_cur ^ 1], &ctl->far_count[s.far_cur ^ 1]);
    }
    if (bid == 0 && threadIdx.x == 0) ctl->buckets++;
    s.far_cur ^= 1;
    s.thresh = tnew;
    if (!grid_barrier(ctl, nbl, gen)) return;
  }
  if (bid == 0 && threadIdx.x == 0) *p.st = s;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_sssp_loop(SsspParams p) {
  __shared__ unsigned gen;
  if (threadIdx.x == 0)
    gen = __hip_atomic_load(&p.ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  sssp_body<BT>(p, &gen);
}

__global__ void k_sssp_init(SsspParams p, int src) {
  const int n = p.g.n;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    p.dist[v] = v == src ? 0u : 0xFFFFFFFFu;
    p.stamp[v] = v == src ? 0 : -1;
    p.in_far[v] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Control* c = p.ctl;
    for (int k = 0; k < 3; ++k) {
      c->slot[k].count = 0;
      c->slot[k].degsum = 0;
      c->slot[k].work = 0;
      c->slot[k].pad = 0;
    }
    c->slot[0].count = 1;
    c->slot[0].degsum = (unsigned long long)p.g.outdeg[src];
    c->far_count[0] = c->far_count[1] = 0;
    c->minreg[0] = c->minreg[1] = ~0ull;
    c->overflow = 0;
    c->buckets = 0;
    c->bar_count = 0;
    c->bar_gen = 0;
    c->error = 0;
    c->steps = 0;
    c->dense_steps = 0;
    c->done = 0;
    c->edges_examined = 0;
    p.near[0][0] = src;
    SsspState s{};
    s.phase = 0;
    s.near_cur = 0;
    s.far_cur = 0;
    s.thresh = p.delta;
    *p.st = s;
  }
}

int launch_sssp_init(const SsspParams& p, int src, hipStream_t stream) {
  const int blocks = (int)std::min<long long>(2048, ((long long)p.g.n + 255) / 256 + 1);
  hipLaunchKernelGGL(k_sssp_init, dim3(blocks), dim3(256), 0, stream, p, src);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int sssp_max_blocks(int bt) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  hipError_t e = bt == 512
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sssp_loop<512>, 512, 0)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_sssp_loop<256>, 256, 0);
  if (e != hipSuccess || per < 1) return -1;
  return ncu * std::min(per, kMaxPersistentBlocksPerCU);
}

int launch_sssp(SsspParams p, int bt, int blocks, hipStream_t stream) {
  void* args[] = {&p};
  const void* fn = bt == 512 ? reinterpret_cast<const void*>(k_sssp_loop<512>)
                             : reinterpret_cast<const void*>(k_sssp_loop<256>);
  return hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(bt), args, 0, stream) == hipSuccess ? 0
                                                                                              : -1;
}

}  // namespace gi
