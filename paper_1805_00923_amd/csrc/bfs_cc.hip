// BFS and connected components: per-step edgeset.apply in every direction,
// driven by a device-side frontier loop (persistent cooperative kernel).
//
// BFS (evaluation, algorithms paragraph; the direction-optimized BFS that
// the paper adopts): SparsePush claims unvisited out-neighbours with a
// compare-and-swap on the level array (each vertex enters the next frontier
// once, so no de-duplication is needed); DensePull lets every unvisited
// vertex scan its in-edges and stop at the first one whose source is in the
// frontier (early exit); DensePush walks the out-edges of every member of a
// dense frontier.
//
// CC (synchronous label propagation): labels double-buffered; a push step
// lowers neighbours' next labels with atomic min (asyncMin, compiler
// section), a pull step takes the minimum over frontier neighbours without
// atomics.  Edges count in both directions.
#include "kernels.h"
#include "traverse.h"

namespace gi {

__device__ __forceinline__ DenseSet dense_at(const LoopParams& p, int k) {
  DenseSet s;
  const int r = ((k % 3) + 3) % 3;
  s.bv = p.boolmap ? nullptr : p.dbv[r];
  s.bm = p.boolmap ? p.dbm[r] : nullptr;
  return s;
}

// ----------------------------------------------------------------- BFS ----

struct BfsPushVisit {
  const int32_t* idx;
  int32_t* level;
  int32_t* parent;
  const int32_t* outdeg;
  int l1;
  PushOut out;
  StepAccum acc;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    bool won = false;
    int v = -1;
    if (valid) {
      v = idx[e];
      acc.work++;
      if (level[v] < 0) won = atomicCAS(&level[v], -1, l1) == -1;
      if (won) {
        if (parent) parent[v] = u;
        acc.dsum += outdeg[v];
      }
    }
    out.emit(won, v, acc);
  }
};

// Unvisited vertices scan in-edges for a frontier source; lanes first take
// up to kSeq edges alone, then the wave walks each remaining long row 64
// edges at a time.  Both stop at the first hit in in-edge order.
template <int BT>
__device__ void bfs_pull(int bid, int nbl, const LoopParams& p, int level_now, DenseSet cur,
                         DenseSet nxt, StepCounters* sc) {
  constexpr int kSeq = 8;
  const DevGraph& g = p.g;
  const int n = g.n, W = (n + 63) >> 6, lane = __lane_id(), l1 = level_now + 1;
  StepAccum acc;
  for (int w = first_wave<BT>(bid); w < W; w += num_waves<BT>(nbl)) {
    const int v = (w << 6) + lane;
    const uint64_t vw = p.vis[w];
    const bool cand = v < n && !((vw >> lane) & 1ull);
    bool found = false;
    int par = -1;
    if (__ballot(cand) != 0ull) {
      int b = 0, e = 0;
      if (cand) {
        b = g.in_off[v];
        e = g.in_off[v + 1];
      }
      const int lim = min(e, b + kSeq);
      for (int j = b; j < lim; ++j) {
        const int u = g.in_idx[j];
        acc.work++;
        if (cur.test(u)) {
          found = true;
          par = u;
          break;
        }
      }
      unsigned long long rm = __ballot(cand && !found && lim < e);
      while (rm) {
        const int leader = __ffsll((long long)rm) - 1;
        rm &= rm - 1;
        const int lb = __shfl(lim, leader, kWave);
        const int le = __shfl(e, leader, kWave);
        for (int j0 = lb; j0 < le; j0 += kWave) {
          const int j = j0 + lane;
          const int u = j < le ? g.in_idx[j] : 0;
          const bool hit = j < le && cur.test(u);
          const unsigned long long hm = __ballot(hit);
          // edges a sequential scan would examine: up to and including the first hit
          if (j < le && (hm == 0ull || lane <= __ffsll((long long)hm) - 1)) acc.work++;
          if (hm) {
            const int pu = __shfl(u, __ffsll((long long)hm) - 1, kWave);
            if (lane == leader) {
              found = true;
              par = pu;
            }
            break;
          }
        }
      }
    }
    const unsigned long long fm = __ballot(found);
    if (found) {
      p.level[v] = l1;
      if (p.parent) p.parent[v] = par;
      acc.dsum += g.outdeg[v];
    }
    if (nxt.bm) {
      if (v < n) nxt.bm[v] = found ? 1 : 0;
    } else if (lane == 0) {
      nxt.bv[w] = fm;
    }
    if (lane == 0) {
      p.vis[w] = vw | fm;
      acc.cnt += __popcll(fm);
    }
  }
  acc.flush(sc, true);
}

// level array -> (visited bitvector, dense frontier of level L).
template <int BT>
__device__ void bfs_level_to_dense(int bid, int nbl, const LoopParams& p, int level_now,
                                   DenseSet cur) {
  const int n = p.g.n, W = (n + 63) >> 6, lane = __lane_id();
  for (int w = first_wave<BT>(bid); w < W; w += num_waves<BT>(nbl)) {
    const int v = (w << 6) + lane;
    const int lv = v < n ? p.level[v] : -1;
    const unsigned long long cm = __ballot(lv == level_now);
    const unsigned long long vm = __ballot(lv >= 0);
    if (cur.bm) {
      if (v < n) cur.bm[v] = lv == level_now ? 1 : 0;
    } else if (lane == 0) {
      cur.bv[w] = cm;
    }
    if (lane == 0) p.vis[w] = vm;
  }
}

// ------------------------------------------------------------------ CC ----

struct CcPushVisit {
  const int32_t* idx;
  const int32_t* cur;
  int32_t* nxt;
  const DevGraph* g;
  PushOut out;
  StepAccum acc;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    bool chg = false;
    int v = -1;
    if (valid) {
      v = idx[e];
      acc.work++;
      const int lu = cur[u];
      if (lu < nxt[v]) {
        const int old = atomicMin(&nxt[v], lu);
        // the first lowering of this round sees the untouched value cur[v]
        if (lu < old && old == cur[v]) chg = true;
      }
      if (chg)
        acc.dsum += (g->out_off[v + 1] - g->out_off[v]) + (g->in_off[v + 1] - g->in_off[v]);
    }
    out.emit(chg, v, acc);
  }
};

// Pull: next[v] = min(cur[v], min over frontier neighbours (in and out) of cur[u]).
template <int BT>
__device__ void cc_pull(int bid, int nbl, const LoopParams& p, const int32_t* cur, int32_t* nxt,
                        DenseSet fr, DenseSet out, StepCounters* sc) {
  constexpr int kSeq = 16;
  const DevGraph& g = p.g;
  const int n = g.n, W = (n + 63) >> 6, lane = __lane_id();
  StepAccum acc;
  for (int w = first_wave<BT>(bid); w < W; w += num_waves<BT>(nbl)) {
    const int v = (w << 6) + lane;
    const bool inr = v < n;
    const int lv = inr ? cur[v] : 0;
    int mn = lv;
    for (int side = 0; side < 2; ++side) {
      const int32_t* off = side ? g.out_off : g.in_off;
      const int32_t* idx = side ? g.out_idx : g.in_idx;
      int b = 0, e = 0;
      if (inr) {
        b = off[v];
        e = off[v + 1];
      }
      const int lim = min(e, b + kSeq);
      for (int j = b; j < lim; ++j) {
        const int u = idx[j];
        if (fr.test(u)) mn = min(mn, cur[u]);
      }
      if (inr) acc.work += lim - b;
      unsigned long long rm = __ballot(lim < e);
      while (rm) {
        const int leader = __ffsll((long long)rm) - 1;
        rm &= rm - 1;
        const int lb = __shfl(lim, leader, kWave);
        const int le = __shfl(e, leader, kWave);
        int part = 0x7fffffff;
        for (int j0 = lb; j0 < le; j0 += kWave) {
          const int j = j0 + lane;
          if (j < le) {
            const int u = idx[j];
            if (fr.test(u)) part = min(part, cur[u]);
            acc.work++;
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part = min(part, __shfl_xor(part, o, kWave));
        if (lane == leader) mn = min(mn, part);
      }
    }
    const bool chg = inr && mn < lv;
    if (inr) nxt[v] = mn;
    const unsigned long long cm = __ballot(chg);
    if (out.bm) {
      if (inr) out.bm[v] = chg ? 1 : 0;
    } else if (lane == 0) {
      out.bv[w] = cm;
    }
    if (chg) acc.dsum += (g.out_off[v + 1] - g.out_off[v]) + (g.in_off[v + 1] - g.in_off[v]);
    if (lane == 0) acc.cnt += __popcll(cm);
  }
  acc.flush(sc, true);
}

// Copy cur -> nxt on the members of the current frontier.
template <int BT>
__device__ void cc_fixup_sparse(int bid, int nbl, const int32_t* ids, int count, const int32_t* cur,
                                int32_t* nxt) {
  for (int i = bid * BT + threadIdx.x; i < count; i += nbl * BT) {
    const int v = ids[i];
    nxt[v] = cur[v];
  }
}

template <int BT>
__device__ void cc_fixup_dense(int bid, int nbl, int n, DenseSet fr, const int32_t* cur,
                               int32_t* nxt) {
  for (int v = bid * BT + threadIdx.x; v < n; v += nbl * BT)
    if (fr.test(v)) nxt[v] = cur[v];
}

// ------------------------------------------------------- frontier loop ----

template <int BT>
__device__ void loop_body(const LoopParams& p, unsigned* gen) {
  const int bid = blockIdx.x, nbl = gridDim.x;
  Control* ctl = p.ctl;
  LoopState s = *p.st;  // uniform copy in every workgroup
  for (int it = 0; it < p.max_steps; ++it) {
    StepCounters* in = &ctl->slot[s.step % 3];
    StepCounters* outc = &ctl->slot[(s.step + 1) % 3];
    const long long nf =
        (long long)__hip_atomic_load(&in->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long dsum =
        (long long)__hip_atomic_load(&in->degsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (bid == 0 && threadIdx.x == 0 && ctl->steps > 0 && ctl->steps <= 4096)
      ctl->w_log[ctl->steps - 1] = (long long)atomic_read(&in->work);  // previous step's edges
    if (nf == 0) {
      if (bid == 0 && threadIdx.x == 0) ctl->done = 1;
      break;
    }
    // direction of this step
    int dir;
    if (p.forced_dir >= 0 && it == 0) dir = p.forced_dir;
    else if (p.direction == GI_DIR_DENSE_PULL_SPARSE_PUSH)
      dir = hybrid_dense(nf, dsum, p.edges, p.divisor) ? GI_DIR_DENSE_PULL : GI_DIR_SPARSE_PUSH;
    else if (p.direction == GI_DIR_DENSE_PUSH_SPARSE_PUSH)
      dir = hybrid_dense(nf, dsum, p.edges, p.divisor) ? GI_DIR_DENSE_PUSH : GI_DIR_SPARSE_PUSH;
    else dir = p.direction;
    if (bid == 0 && threadIdx.x == 0) {
      const int k = ctl->steps;
      if (k < 4096) {
        ctl->dir_log[k] = dir;
        ctl->f_log[k] = (int)nf;
        ctl->d_log[k] = dsum;
      }
      ctl->steps = k + 1;
      if (dir != GI_DIR_SPARSE_PUSH) ctl->dense_steps++;
      ctl->edges_examined += (unsigned long long)dsum;
      // clear the counters of step+2 (last read at step-1)
      StepCounters* z = &ctl->slot[(s.step + 2) % 3];
      atomic_zero(&z->count);
      atomic_zero(&z->degsum);
      atomic_zero(&z->work);
      atomic_zero(&z->pad);
    }
    const DenseSet dcur = dense_at(p, s.step), dnxt = dense_at(p, s.step + 1);
    // clear the dense buffer of step+2 (not touched by this step)
    clear_dense<BT>(bid, nbl, p.g.n, dense_at(p, s.step + 2));
    const int32_t* sa_in = p.sa[s.sa_cur];
    int32_t* sa_out = p.sa[s.sa_cur ^ 1];

    // 1. bring the frontier into the representation the direction reads
    bool need_bar = false;
    if (p.alg == ALG_BFS && dir == GI_DIR_DENSE_PULL && !(s.rep == REP_DENSE && s.vis_valid)) {
      bfs_level_to_dense<BT>(bid, nbl, p, s.step, dcur);
      s.vis_valid = 1;
      s.rep = REP_DENSE;
      need_bar = true;
    } else if (dir != GI_DIR_SPARSE_PUSH && s.rep == REP_SPARSE) {
      scatter_to_dense<BT>(bid, nbl, sa_in, (int)nf, dcur);  // dcur was cleared two steps ago
      s.rep = REP_DENSE;
      need_bar = true;
    } else if (dir == GI_DIR_SPARSE_PUSH && s.rep == REP_DENSE) {
      // slot step+1's spare counter was cleared during the previous step
      compact_dense<BT>(bid, nbl, p.g.n, dcur, sa_out, &ctl->slot[(s.step + 1) % 3].pad);
      need_bar = true;
    }
    // CC push needs nxt == cur on the frontier before any atomic min
    const int32_t* lcur = p.lab[s.lab_cur];
    int32_t* lnxt = p.lab[s.lab_cur ^ 1];
    if (p.alg == ALG_CC && dir != GI_DIR_DENSE_PULL && s.cc_fix) {
      if (dir == GI_DIR_SPARSE_PUSH && s.rep == REP_SPARSE)
        cc_fixup_sparse<BT>(bid, nbl, sa_in, (int)nf, lcur, lnxt);
      else
        cc_fixup_dense<BT>(bid, nbl, p.g.n, dcur, lcur, lnxt);
      need_bar = true;
    }
    if (need_bar) {
      if (!grid_barrier(ctl, nbl, gen)) return;
    }
    if (dir == GI_DIR_SPARSE_PUSH && s.rep == REP_DENSE) {
      // frontier was compacted into sa_out; use it as the input
      sa_in = sa_out;
      sa_out = p.sa[s.sa_cur];
      s.sa_cur ^= 1;
      s.rep = REP_SPARSE;
    }

    // 2. the edgeset.apply step
    PushOut po;
    po.kind = dir == GI_DIR_SPARSE_PUSH ? REP_SPARSE : REP_DENSE;
    po.ids = sa_out;
    po.count = &outc->count;
    po.dense = dnxt;
    if (p.alg == ALG_BFS) {
      if (dir == GI_DIR_DENSE_PULL) {
        bfs_pull<BT>(bid, nbl, p, s.step, dcur, dnxt, outc);
      } else {
        BfsPushVisit vis{p.g.out_idx, p.level, p.parent, p.g.outdeg, s.step + 1, po, StepAccum()};
        if (dir == GI_DIR_SPARSE_PUSH) {
          SparseItems items{sa_in, (int)nf, p.g.out_off};
          push_expand<BT>(bid, nbl, items, vis);
        } else {
          DenseItems items{dcur, p.g.n, p.g.out_off};
          push_expand<BT>(bid, nbl, items, vis);
        }
        vis.acc.flush(outc, po.kind == REP_DENSE);
        s.vis_valid = 0;
      }
    } else {
      if (dir == GI_DIR_DENSE_PULL) {
        cc_pull<BT>(bid, nbl, p, lcur, lnxt, dcur, dnxt, outc);
      } else {
        CcPushVisit vis{p.g.out_idx, lcur, lnxt, &p.g, po, StepAccum()};
        if (dir == GI_DIR_SPARSE_PUSH) {
          SparseItems items{sa_in, (int)nf, p.g.out_off};
          push_expand<BT>(bid, nbl, items, vis);
          vis.idx = p.g.in_idx;
          SparseItems items2{sa_in, (int)nf, p.g.in_off};
          push_expand<BT>(bid, nbl, items2, vis);
        } else {
          DenseItems items{dcur, p.g.n, p.g.out_off};
          push_expand<BT>(bid, nbl, items, vis);
          vis.idx = p.g.in_idx;
          DenseItems items2{dcur, p.g.n, p.g.in_off};
          push_expand<BT>(bid, nbl, items2, vis);
        }
        vis.acc.flush(outc, po.kind == REP_DENSE);
      }
      s.lab_cur ^= 1;
      s.cc_fix = 1;
    }
    if (dir == GI_DIR_SPARSE_PUSH) {
      s.sa_cur ^= 1;
      s.rep = REP_SPARSE;
    } else {
      s.rep = REP_DENSE;
    }
    s.step += 1;
    if (!grid_barrier(ctl, nbl, gen)) return;
  }
  if (bid == 0 && threadIdx.x == 0) *p.st = s;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_frontier_loop(LoopParams p) {
  __shared__ unsigned gen;
  if (threadIdx.x == 0)
    gen = __hip_atomic_load(&p.ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  loop_body<BT>(p, &gen);
}

// Initial state.  BFS: level = -1 (parent = -1) except the source; F = {src}.
// CC: both label buffers = id; F = V as a full dense set.
template <int BT>
__global__ __launch_bounds__(BT) void k_loop_init(LoopParams p, int src) {
  const int n = p.g.n;
  const int tid = blockIdx.x * BT + threadIdx.x, nt = gridDim.x * BT;
  for (int v = tid; v < n; v += nt) {
    if (p.alg == ALG_BFS) {
      p.level[v] = v == src ? 0 : -1;
      if (p.parent) p.parent[v] = v == src ? src : -1;
    } else {
      p.lab[0][v] = v;
      p.lab[1][v] = v;
    }
  }
  // dense rotation: slot 0 holds the initial CC frontier (all ones), slots 1
  // and 2 start cleared
  const int W = (n + 63) >> 6;
  for (int k = 0; k < 3; ++k) {
    DenseSet d = dense_at(p, k);
    if (d.bm) {
      for (int v = tid; v < n; v += nt) d.bm[v] = (p.alg == ALG_CC && k == 0) ? 1 : 0;
    } else {
      for (int w = tid; w < W; w += nt) {
        uint64_t word = 0;
        if (p.alg == ALG_CC && k == 0) {
          const int rem = n - (w << 6);
          word = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
        }
        d.bv[w] = word;
      }
    }
  }
  if (p.alg == ALG_BFS)
    for (int w = tid; w < W; w += nt) p.vis[w] = 0ull;
  if (tid == 0) {
    Control* c = p.ctl;
    for (int k = 0; k < 3; ++k) {
      c->slot[k].count = 0;
      c->slot[k].degsum = 0;
      c->slot[k].work = 0;
      c->slot[k].pad = 0;
    }
    c->bar_count = 0;
    c->bar_gen = 0;
    c->error = 0;
    c->steps = 0;
    c->dense_steps = 0;
    c->done = 0;
    c->edges_examined = 0;
    LoopState s{};
    if (p.alg == ALG_BFS) {
      c->slot[0].count = 1;
      c->slot[0].degsum = (unsigned long long)p.g.outdeg[src];
      p.sa[0][0] = src;
      s.rep = REP_SPARSE;
    } else {
      c->slot[0].count = (unsigned long long)n;
      c->slot[0].degsum = (unsigned long long)(2 * p.g.m);
      s.rep = REP_DENSE;
    }
    s.step = 0;
    s.sa_cur = 0;
    s.vis_valid = 0;
    s.cc_fix = 0;
    s.lab_cur = 0;
    *p.st = s;
  }
}

// ------------------------------------------------------- host launchers ----

int launch_loop_init(const LoopParams& p, int src, hipStream_t stream) {
  const int blocks = (int)std::min<long long>(1024, ((long long)p.g.n + 255) / 256 + 1);
  hipLaunchKernelGGL(k_loop_init<256>, dim3(blocks), dim3(256), 0, stream, p, src);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int loop_max_blocks(int block_threads) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  hipError_t e = hipSuccess;
  switch (block_threads) {
    case 256: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_frontier_loop<256>, 256, 0); break;
    case 512: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_frontier_loop<512>, 512, 0); break;
    default: return -1;
  }
  if (e != hipSuccess || per < 1) return -1;
  return ncu * std::min(per, kMaxPersistentBlocksPerCU);
}

int launch_loop(LoopParams p, int block_threads, int blocks, hipStream_t stream) {
  void* args[] = {&p};
  hipError_t e;
  if (block_threads == 512)
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_frontier_loop<512>), dim3(blocks),
                                   dim3(512), args, 0, stream);
  else
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_frontier_loop<256>), dim3(blocks),
                                   dim3(256), args, 0, stream);
  return e == hipSuccess ? 0 : -1;
}

}  // namespace gi
