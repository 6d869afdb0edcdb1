// BFS, connected components and delta-stepping SSSP on the multi-launch
// frontier engine (common.h, traverse.h).
//
// BFS (evaluation, algorithms paragraph; the paper adopts direction-optimized
// BFS): SparsePush claims unvisited out-neighbours with a compare-and-swap on
// the level array, so every vertex enters the next frontier once and no
// de-duplication is needed; DensePull lets every unvisited vertex scan its
// in-edges and stop at the first one whose source is in the frontier (early
// exit); DensePush walks the out-edges of every member of a dense frontier.
//
// CC (synchronous label propagation over edges taken both ways): labels are
// double-buffered.  Push steps lower neighbours' next labels with atomic min
// (the asyncMin reduction of the compiler section); pull steps take the
// minimum over the neighbours' labels without atomics.  Taking the minimum
// over all neighbours in a pull step gives the same labels as over frontier
// neighbours only: a neighbour outside the frontier kept the label it had
// one round earlier, which the vertex has already absorbed.
//
// SSSP: delta-stepping (Meyer and Sanders, J. Algorithms 2003) with a near
// set (tentative distance below the current bucket threshold) relaxed by
// SparsePush steps and a far set for everything improved at or beyond it;
// when the near set empties the threshold moves to the end of the bucket of
// the smallest far distance and the far set is split.
#include "kernels.h"
#include "traverse.h"

namespace gi {

// ---------------------------------------------------------------- decide --

// Sum the per-workgroup statistics of the step that just ran, log it, and
// choose the direction of the next step (BFS and CC).
__global__ __launch_bounds__(1024) void k_decide_frontier(DecideArgs a) {
  __shared__ long long s[3][1024];
  const int t = threadIdx.x;
  long long x = 0, y = 0, z = 0;
  for (int i = t; i < kMaxParts; i += 1024) {
    x += a.part[i].a;
    y += a.part[i].b;
    z += a.part[i].c;
  }
  s[0][t] = x;
  s[1][t] = y;
  s[2][t] = z;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      s[0][t] += s[0][t + o];
      s[1][t] += s[1][t + o];
      s[2][t] += s[2][t + o];
    }
    __syncthreads();
  }
  for (int i = t; i < kMaxParts; i += 1024) a.part[i] = Part{0, 0, 0, 0};
  if (t != 0) return;
  Control* c = a.ctl;
  if (c->done) {
    c->mode = MODE_NONE;
    return;
  }
  const long long nf = s[0][0], dsum = s[1][0], work = s[2][0];
  const int k = c->steps;
  if (k > 0 && k <= kMaxLog) c->w_log[k - 1] = work;
  c->edges_examined += work;
  if (nf == 0) {
    c->done = 1;
    c->mode = MODE_NONE;
    return;
  }
  int dir = a.direction;
  if (a.forced_dir >= 0) dir = a.forced_dir;
  else if (dir == GI_DIR_DENSE_PULL_SPARSE_PUSH)
    dir = hybrid_dense(nf, dsum, a.edges, a.divisor) ? GI_DIR_DENSE_PULL : GI_DIR_SPARSE_PUSH;
  else if (dir == GI_DIR_DENSE_PUSH_SPARSE_PUSH)
    dir = hybrid_dense(nf, dsum, a.edges, a.divisor) ? GI_DIR_DENSE_PUSH : GI_DIR_SPARSE_PUSH;
  if (k < kMaxLog) {
    c->dir_log[k] = dir;
    c->f_log[k] = (int)nf;
    c->d_log[k] = dsum;
    c->w_log[k] = 0;
  }
  c->steps = k + 1;
  if (dir != GI_DIR_SPARSE_PUSH) c->dense_steps++;
  c->nf = nf;
  c->dsum = dsum;
  c->mode = dir;
}

// ------------------------------------------------------------------- BFS --

struct BfsVisit {
  const int32_t* idx;
  int32_t* level;
  int32_t* parent;
  const int32_t* outdeg;
  int l1;
  DenseSet next;
  uint64_t* vis;
  long long cnt = 0, dsum = 0, work = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid, bool) {
    if (!valid) return;
    const int v = idx[e];
    ++work;
    if (level[v] >= 0) return;
    if (atomicCAS(&level[v], -1, l1) != -1) return;
    if (parent) parent[v] = u;
    next.insert(v);
    atomicOr((unsigned long long*)&vis[v >> 6], 1ull << (v & 63));
    ++cnt;
    dsum += outdeg[v];
  }
};

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_bfs_expand(BfsArgs b, ExpandArgs x) {
  if (x.ctl->mode != MODE_SPARSE_PUSH) return;
  BfsVisit vis{b.g.out_idx, b.level, b.parent, b.g.outdeg, x.ctl->steps, b.next, b.vis};
  expand_chunks<BT, CH>(x, vis);
  const Part p = block_sum4<BT>(Part{vis.cnt, vis.dsum, vis.work, 0});
  if (threadIdx.x == 0) b.part[blockIdx.x] = p;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_bfs_dense_push(BfsArgs b) {
  Control* ctl = b.ctl;
  if (ctl->mode != MODE_DENSE_PUSH) return;
  BfsVisit vis{b.g.out_idx, b.level, b.parent, b.g.outdeg, ctl->steps, b.next, b.vis};
  dense_push_expand<BT>(b.cur, b.g.n, b.g.out_off, vis, true);
  const Part p = block_sum4<BT>(Part{vis.cnt, vis.dsum, vis.work, 0});
  if (threadIdx.x == 0) b.part[blockIdx.x] = p;
}

// DensePull: one wave per 64-vertex word.  Unvisited lanes test their first
// in-edges in batches of four independent loads, then the wave walks each
// remaining long row 64 edges at a time; both stop at the first source in
// the frontier, in in-edge order.  The next frontier word and the visited
// word are written whole, without atomics.
template <int BT>
__global__ __launch_bounds__(BT) void k_bfs_pull(BfsArgs b) {
  Control* ctl = b.ctl;
  if (ctl->mode != MODE_DENSE_PULL) return;
  const DevGraph& g = b.g;
  const int n = g.n, W = (n + 63) >> 6, lane = __lane_id();
  const int l1 = ctl->steps;
  const DenseSet cur = b.cur, nxt = b.next;
  long long cnt = 0, dsum = 0, work = 0;
  const int wave0 = blockIdx.x * (BT / kWave) + (int)(threadIdx.x / kWave);
  const int nwaves = gridDim.x * (BT / kWave);
  for (int w = wave0; w < W; w += nwaves) {
    const int v = (w << 6) + lane;
    const uint64_t vw = b.vis[w];
    const bool cand = v < n && !((vw >> lane) & 1ull);
    bool found = false;
    int par = -1;
    if (__ballot(cand) != 0ull) {
      int j = 0, e = 0;
      if (cand) {
        j = g.in_off[v];
        e = g.in_off[v + 1];
      }
#pragma unroll
      for (int batch = 0; batch < 2; ++batch) {
        int u[4];
        bool h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] = (!found && j + q < e) ? g.in_idx[j + q] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) h[q] = u[q] >= 0 && cur.test(u[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!found && u[q] >= 0) {
            ++work;
            if (h[q]) {
              found = true;
              par = u[q];
            }
          }
        }
        if (!found) j = min(e, j + 4);
      }
      unsigned long long rm = __ballot(cand && !found && j < e);
      while (rm) {
        const int leader = __ffsll((long long)rm) - 1;
        rm &= rm - 1;
        const int lb = __shfl(j, leader, kWave);
        const int le = __shfl(e, leader, kWave);
        for (int j0 = lb; j0 < le; j0 += kWave) {
          const int jj = j0 + lane;
          const int uu = jj < le ? g.in_idx[jj] : 0;
          const bool hit = jj < le && cur.test(uu);
          const unsigned long long hm = __ballot(hit);
          // edges a sequential scan examines: up to and including the first hit
          if (jj < le && (hm == 0ull || lane <= __ffsll((long long)hm) - 1)) ++work;
          if (hm) {
            const int pu = __shfl(uu, __ffsll((long long)hm) - 1, kWave);
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
      b.level[v] = l1;
      if (b.parent) b.parent[v] = par;
      dsum += g.outdeg[v];
    }
    if (nxt.bm) {
      nxt.bm[v] = found ? 1 : 0;  // the bool map is padded to whole words
    } else if (lane == 0) {
      nxt.bv[w] = fm;
    }
    if (lane == 0) {
      b.vis[w] = vw | fm;
      cnt += __popcll(fm);
    }
  }
  const Part p = block_sum4<BT>(Part{cnt, dsum, work, 0});
  if (threadIdx.x == 0) b.part[blockIdx.x] = p;
}

// Initial state: level = -1 (parent = -1) except the source; F = {src}.
__global__ void k_bfs_init(BfsArgs b, int src, DenseSet f0, DenseSet f1) {
  const int n = b.g.n, W = (n + 63) >> 6;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += nt) {
    b.level[v] = v == src ? 0 : -1;
    if (b.parent) b.parent[v] = v == src ? src : -1;
  }
  for (int w = tid; w < W; w += nt) {
    const uint64_t word = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    b.vis[w] = word;
    if (f0.bv) f0.bv[w] = word;
    if (f1.bv) f1.bv[w] = 0ull;
  }
  for (long long i = tid; i < (long long)W * 64; i += nt) {
    if (f0.bm) f0.bm[i] = i == src ? 1 : 0;
    if (f1.bm) f1.bm[i] = 0;
  }
  for (int i = tid; i < kMaxParts; i += nt) b.part[i] = Part{0, 0, 0, 0};
  if (tid == 0) {
    b.part[0] = Part{1, b.g.outdeg[src], 0, 0};
    Control* c = b.ctl;
    c->mode = MODE_NONE;
    c->done = 0;
    c->steps = 0;
    c->dense_steps = 0;
    c->edges_examined = 0;
    c->error = 0;
  }
}

// -------------------------------------------------------------------- CC --

struct CcVisit {
  const int32_t* out_idx;
  const int32_t* in_idx;
  const int32_t* cur;
  int32_t* nxt;
  const int32_t* udeg;
  DenseSet next;
  long long cnt = 0, dsum = 0, work = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid, bool first) {
    if (!valid) return;
    const int v = first ? out_idx[e] : in_idx[e];
    ++work;
    const int lu = cur[u];
    if (lu >= nxt[v]) return;
    const int old = atomicMin(&nxt[v], lu);
    // the first lowering of this round sees the untouched value cur[v]
    if (lu < old && old == cur[v]) {
      next.insert(v);
      ++cnt;
      dsum += udeg[v];
    }
  }
};

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_cc_expand(CcArgs c, ExpandArgs x) {
  if (x.ctl->mode != MODE_SPARSE_PUSH) return;
  CcVisit vis{c.g.out_idx, c.g.in_idx, c.cur, c.nxt, c.g.udeg, c.next};
  expand_chunks<BT, CH>(x, vis);
  const Part p = block_sum4<BT>(Part{vis.cnt, vis.dsum, vis.work, 0});
  if (threadIdx.x == 0) c.part[blockIdx.x] = p;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_cc_dense_push(CcArgs c) {
  if (c.ctl->mode != MODE_DENSE_PUSH) return;
  CcVisit vis{c.g.out_idx, c.g.in_idx, c.cur, c.nxt, c.g.udeg, c.next};
  dense_push_expand<BT>(c.fr, c.g.n, c.g.out_off, vis, true);
  dense_push_expand<BT>(c.fr, c.g.n, c.g.in_off, vis, false);
  const Part p = block_sum4<BT>(Part{vis.cnt, vis.dsum, vis.work, 0});
  if (threadIdx.x == 0) c.part[blockIdx.x] = p;
}

// Pull, over destination blocks of one adjacency: the block's edge range is
// staged in LDS (coalesced index loads, label gathers), then each row's
// minimum is taken by a power-of-two group of threads.  Pass 0 (in-edges)
// writes nxt[v] = min(cur[v], min over in-neighbours) and clears the next
// frontier words of its rows; pass 1 (out-edges) folds in the out-neighbours
// and records the vertices whose label dropped.
template <int BT>
__global__ __launch_bounds__(BT) void k_cc_pull(CcArgs c, RowBlocks rb, int pass, int cap_e) {
  if (c.ctl->mode != MODE_DENSE_PULL) return;
  extern __shared__ int smem[];
  int* lds_val = smem;
  int* lds_off = smem + cap_e;
  __shared__ int red[BT / kWave];
  long long cnt = 0, dsum = 0, work = 0;
  const int n = c.g.n;
  for (int t = blockIdx.x; t < rb.ntab; t += gridDim.x) {
    const int2 r = rb.table[t];
    const int kb = r.x, ke = r.y, nr = ke - kb;
    const int e0 = rb.off[kb], e1 = rb.off[ke], ne = e1 - e0;
    if (threadIdx.x == 0) work += ne;
    if (pass == 0) {
      const int wb = kb >> 6, we = (ke + 63) >> 6;
      for (int w = wb + (int)threadIdx.x; w < we && w < ((n + 63) >> 6); w += BT) {
        if (c.next.bv) c.next.bv[w] = 0ull;
      }
      if (c.next.bm)
        for (int v = kb + (int)threadIdx.x; v < ke; v += BT) c.next.bm[v] = 0;
    }
    auto finish = [&](int v, int mn) {
      if (pass == 0) {
        const int lv = c.cur[v];
        c.nxt[v] = mn < lv ? mn : lv;
      } else {
        const int x0 = c.nxt[v];
        const int x = mn < x0 ? mn : x0;
        c.nxt[v] = x;
        if (x < c.cur[v]) {
          c.next.insert(v);
          ++cnt;
          dsum += c.g.udeg[v];
        }
      }
    };
    if (ne > cap_e) {  // one long row: workgroup-wide minimum
      int mn = 0x7fffffff;
      for (int e = e0 + (int)threadIdx.x; e < e1; e += BT) mn = min(mn, c.cur[rb.idx[e]]);
      mn = wave_min(mn);
      if (__lane_id() == 0) red[threadIdx.x / kWave] = mn;
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int i = 0; i < BT / kWave; ++i) mn = min(mn, red[i]);
        finish(kb, mn);
      }
      __syncthreads();
      continue;
    }
    for (int j = threadIdx.x; j < ne; j += BT) lds_val[j] = c.cur[rb.idx[e0 + j]];
    for (int k = threadIdx.x; k <= nr; k += BT) lds_off[k] = rb.off[kb + k] - e0;
    __syncthreads();
    int tpv = 1;
    if (nr < BT) {
      tpv = BT / (nr > 0 ? nr : 1);
      tpv = 1 << (31 - __clz(tpv));
      if (tpv > kWave) tpv = kWave;
    }
    const int groups = BT / tpv, grp = threadIdx.x / tpv, gl = threadIdx.x % tpv;
    for (int k0 = 0; k0 < nr; k0 += groups) {
      const int k = k0 + grp;
      int mn = 0x7fffffff;
      if (k < nr) {
        const int lo = lds_off[k], hi = lds_off[k + 1];
        for (int j = lo + gl; j < hi; j += tpv) mn = min(mn, lds_val[j]);
      }
      for (int o = tpv >> 1; o > 0; o >>= 1) mn = min(mn, __shfl_xor(mn, o, kWave));
      if (gl == 0 && k < nr) finish(kb + k, mn);
    }
    __syncthreads();
  }
  if (pass == 1) {
    const Part p = block_sum4<BT>(Part{cnt, dsum, work, 0});
    if (threadIdx.x == 0) c.part[blockIdx.x] = p;
  }
}

// Initial state: both label buffers hold the ids; F = V.
__global__ void k_cc_init(CcArgs c, DenseSet f0, DenseSet f1, int32_t* lab_other) {
  const int n = c.g.n, W = (n + 63) >> 6;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += nt) {
    c.cur[v] = v;
    lab_other[v] = v;
  }
  for (int w = tid; w < W; w += nt) {
    const int rem = n - (w << 6);
    const uint64_t word = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    if (f0.bv) f0.bv[w] = word;
    if (f1.bv) f1.bv[w] = 0ull;
  }
  for (long long i = tid; i < (long long)W * 64; i += nt) {
    if (f0.bm) f0.bm[i] = i < n ? 1 : 0;
    if (f1.bm) f1.bm[i] = 0;
  }
  for (int i = tid; i < kMaxParts; i += nt) c.part[i] = Part{0, 0, 0, 0};
  if (tid == 0) {
    c.part[0] = Part{n, 2 * c.g.m, 0, 0};
    Control* ctl = c.ctl;
    ctl->mode = MODE_NONE;
    ctl->done = 0;
    ctl->steps = 0;
    ctl->dense_steps = 0;
    ctl->edges_examined = 0;
    ctl->error = 0;
  }
}

// ------------------------------------------------------------------ SSSP --

__global__ __launch_bounds__(1024) void k_decide_sssp(SsspArgs a) {
  __shared__ long long s[3][1024];
  const int t = threadIdx.x;
  long long x = 0, y = 0, z = 0;
  for (int i = t; i < kMaxParts; i += 1024) {
    x += a.part[i].a;
    y += a.part[i].b;
    z += a.part[i].c;
  }
  s[0][t] = x;
  s[1][t] = y;
  s[2][t] = z;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      s[0][t] += s[0][t + o];
      s[1][t] += s[1][t + o];
      s[2][t] += s[2][t + o];
    }
    __syncthreads();
  }
  for (int i = t; i < kMaxParts; i += 1024) a.part[i] = Part{0, 0, 0, 0};
  if (t != 0) return;
  Control* c = a.ctl;
  if (c->done) {
    c->mode = MODE_NONE;
    return;
  }
  const long long nn = s[0][0], nfar = s[1][0], work = s[2][0];
  const int k = c->steps;
  if (c->mode == MODE_SSSP_RELAX) {
    if (k > 0 && k <= kMaxLog) c->w_log[k - 1] = work;
    c->edges_examined += work;
    c->far_count += nfar;  // far members added by the relaxation
  } else if (c->mode == MODE_SSSP_SPLIT) {
    c->far_count = nfar;   // far members kept by the split
  }
  if (c->overflow) {
    c->done = 1;
    c->mode = MODE_NONE;
    return;
  }
  if (nn > 0) {
    if (k < kMaxLog) {
      c->dir_log[k] = GI_DIR_SPARSE_PUSH;
      c->f_log[k] = (int)nn;
      c->d_log[k] = 0;
      c->w_log[k] = 0;
    }
    c->steps = k + 1;
    c->nf = nn;
    c->mode = MODE_SSSP_RELAX;
  } else if (c->far_count > 0) {
    c->mode = MODE_SSSP_SPLIT;
  } else {
    c->done = 1;
    c->mode = MODE_NONE;
  }
}

struct SsspVisit {
  const int32_t* idx;
  const uint32_t* w;
  uint32_t* dist;
  DenseSet near;
  DenseSet far;
  unsigned long long thresh;
  int* overflow;
  long long cnt_near = 0, cnt_far = 0, work = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid, bool) {
    if (!valid) return;
    const int v = idx[e];
    ++work;
    const unsigned long long nd = (unsigned long long)dist[u] + (unsigned long long)w[e];
    if (nd >= 0xFFFFFFFFull) {
      __hip_atomic_store(overflow, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    if ((uint32_t)nd >= dist[v]) return;
    const uint32_t old = atomicMin(&dist[v], (uint32_t)nd);
    if ((uint32_t)nd >= old) return;
    if (nd < thresh) {
      if (near.insert(v)) ++cnt_near;
    } else {
      if (far.insert(v)) ++cnt_far;
    }
  }
};

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_sssp_expand(SsspArgs s, ExpandArgs x) {
  Control* ctl = x.ctl;
  if (ctl->mode != MODE_SSSP_RELAX) return;
  SsspVisit vis{s.g.out_idx, s.g.out_w, s.dist, s.next, s.far, ctl->thresh, &ctl->overflow};
  expand_chunks<BT, CH>(x, vis);
  const Part p = block_sum4<BT>(Part{vis.cnt_near, vis.cnt_far, vis.work, 0});
  if (threadIdx.x == 0) s.part[blockIdx.x] = p;
}

// Split, pass 1: smallest far distance at or beyond the threshold (one value
// per workgroup, ~0 when none), and clear the next near set.
template <int BT>
__global__ __launch_bounds__(BT) void k_sssp_far_min(SsspArgs s) {
  Control* ctl = s.ctl;
  if (ctl->mode != MODE_SSSP_SPLIT) return;
  const int n = s.g.n, W = (n + 63) >> 6;
  const unsigned long long th = ctl->thresh;
  unsigned long long mn = ~0ull;
  for (int w = blockIdx.x * BT + threadIdx.x; w < W; w += gridDim.x * BT) {
    if (s.next.bv) s.next.bv[w] = 0ull;
    if (s.next.bm) {
      uint64_t* p = reinterpret_cast<uint64_t*>(s.next.bm + ((size_t)w << 6));
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = 0ull;
    }
    uint64_t x = s.far.word(w);
    while (x) {
      const int b = __ffsll((long long)x) - 1;
      x &= x - 1;
      const unsigned long long d = s.dist[(w << 6) + b];
      if (d >= th && d < mn) mn = d;
    }
  }
  __shared__ unsigned long long red[BT / kWave];
  mn = wave_min(mn);
  if (__lane_id() == 0) red[threadIdx.x / kWave] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < BT / kWave; ++i) mn = red[i] < mn ? red[i] : mn;
    s.part[blockIdx.x].d = (long long)mn;
  }
}

// Split, pass 2 (one workgroup): new threshold.
__global__ __launch_bounds__(1024) void k_sssp_threshold(SsspArgs s, int nparts) {
  Control* ctl = s.ctl;
  if (ctl->mode != MODE_SSSP_SPLIT) return;
  __shared__ unsigned long long red[1024];
  unsigned long long mn = ~0ull;
  for (int i = threadIdx.x; i < nparts; i += 1024) {
    const unsigned long long x = (unsigned long long)s.part[i].d;
    s.part[i].d = 0;
    mn = x < mn ? x : mn;
  }
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < (unsigned)o && red[threadIdx.x + o] < red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mn = red[0];
    const unsigned long long told = ctl->thresh;
    ctl->told = told;
    ctl->thresh = mn == ~0ull ? told : (mn / s.delta + 1ull) * s.delta;
    ctl->buckets++;
  }
}

// Split, pass 3: stale far members (distance below the old threshold, so
// already relaxed) are dropped, members of the new bucket move to the near
// set, the rest stay.
template <int BT>
__global__ __launch_bounds__(BT) void k_sssp_split(SsspArgs s) {
  Control* ctl = s.ctl;
  if (ctl->mode != MODE_SSSP_SPLIT) return;
  const int n = s.g.n, W = (n + 63) >> 6;
  const unsigned long long told = ctl->told, tnew = ctl->thresh;
  long long moved = 0, kept = 0;
  for (int w = blockIdx.x * BT + threadIdx.x; w < W; w += gridDim.x * BT) {
    uint64_t x = s.far.word(w), keep = 0;
    while (x) {
      const int b = __ffsll((long long)x) - 1;
      x &= x - 1;
      const int v = (w << 6) + b;
      const unsigned long long d = s.dist[v];
      if (d < told) continue;
      if (d < tnew) {
        s.next.insert(v);
        ++moved;
      } else {
        keep |= 1ull << b;
        ++kept;
      }
    }
    if (s.far.bv) {
      s.far.bv[w] = keep;
    } else {
      for (int b = 0; b < 64; ++b) s.far.bm[((size_t)w << 6) + b] = (keep >> b) & 1ull;
    }
  }
  const Part p = block_sum4<BT>(Part{moved, kept, 0, 0});
  if (threadIdx.x == 0) s.part[blockIdx.x] = p;
}

__global__ void k_sssp_init(SsspArgs s, int src, DenseSet f0, DenseSet f1) {
  const int n = s.g.n, W = (n + 63) >> 6;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += nt) s.dist[v] = v == src ? 0u : 0xFFFFFFFFu;
  for (int w = tid; w < W; w += nt) {
    const uint64_t word = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    if (f0.bv) f0.bv[w] = word;
    if (f1.bv) f1.bv[w] = 0ull;
    if (s.far.bv) s.far.bv[w] = 0ull;
  }
  for (long long i = tid; i < (long long)W * 64; i += nt) {
    if (f0.bm) f0.bm[i] = i == src ? 1 : 0;
    if (f1.bm) f1.bm[i] = 0;
    if (s.far.bm) s.far.bm[i] = 0;
  }
  for (int i = tid; i < kMaxParts; i += nt) s.part[i] = Part{0, 0, 0, 0};
  if (tid == 0) {
    s.part[0] = Part{1, 0, 0, 0};
    Control* c = s.ctl;
    c->mode = MODE_NONE;
    c->done = 0;
    c->steps = 0;
    c->dense_steps = 0;
    c->edges_examined = 0;
    c->thresh = s.delta;
    c->told = 0;
    c->far_count = 0;
    c->overflow = 0;
    c->buckets = 0;
    c->error = 0;
  }
}

// ------------------------------------------------------- host launchers --

static int grid_for(long long items, int bt, int cap) {
  long long b = (items + bt - 1) / bt;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

#define GI_OK_LAUNCH() (hipGetLastError() == hipSuccess ? 0 : -1)

constexpr int kBT = 256;
constexpr int kCH = 2048;

int expand_chunk_size() { return kCH; }

static CompactArgs compact_args(const Engine& e, DenseSet in, const int32_t* deg, DenseSet clear,
                                const int32_t* fix_src, int32_t* fix_dst, int m1, int m2) {
  CompactArgs a;
  a.in = in;
  a.n = e.n;
  a.tw = e.tw;
  a.deg = deg;
  a.blk_cnt = e.blk_cnt;
  a.blk_deg = e.blk_deg;
  a.ids = e.ids;
  a.excl = e.excl;
  a.chunk_item = e.chunk_item;
  a.chunk = kCH;
  a.chunk_cap = e.chunk_cap;
  a.clear = clear;
  a.fix_src = fix_src;
  a.fix_dst = fix_dst;
  a.ctl = e.ctl;
  a.active_mode = m1;
  a.active_mode2 = m2;
  return a;
}

static int enqueue_compaction(const Engine& e, const CompactArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_count<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, a);
  CompactArgs w = a;
  w.active_mode2 = MODE_NEVER;  // the sparse array is needed by SparsePush only
  w.fix_dst = nullptr;         // fixed up once, in the count pass
  w.clear = DenseSet{nullptr, nullptr};
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, w, e.cgrid);
  hipLaunchKernelGGL(k_compact_write<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, w);
  return GI_OK_LAUNCH();
}

static ExpandArgs expand_args(const Engine& e, const int32_t* off, const int32_t* off2,
                              const int32_t* deg1, int mode) {
  ExpandArgs x;
  x.ids = e.ids;
  x.excl = e.excl;
  x.chunk_item = e.chunk_item;
  x.off = off;
  x.off2 = off2;
  x.deg1 = deg1;
  x.ctl = e.ctl;
  x.active_mode = mode;
  return x;
}

int launch_bfs_init(const BfsArgs& b, int src, DenseSet f0, DenseSet f1, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(b.g.n, 256, 2048)), dim3(256), 0, s, b, src, f0, f1);
  return GI_OK_LAUNCH();
}

int enqueue_bfs_step(const Engine& e, const DecideArgs& d, const BfsArgs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_decide_frontier, dim3(1), dim3(1024), 0, s, d);
  CompactArgs ca = compact_args(e, b.cur, b.g.outdeg, b.next, nullptr, nullptr, MODE_SPARSE_PUSH,
                                MODE_DENSE_PUSH);
  if (enqueue_compaction(e, ca, s)) return -1;
  hipLaunchKernelGGL((k_bfs_expand<kBT, kCH>), dim3(e.xgrid), dim3(kBT), 0, s, b,
                     expand_args(e, b.g.out_off, nullptr, nullptr, MODE_SPARSE_PUSH));
  hipLaunchKernelGGL(k_bfs_dense_push<kBT>, dim3(e.vgrid), dim3(kBT), 0, s, b);
  hipLaunchKernelGGL(k_bfs_pull<kBT>, dim3(e.wgrid), dim3(kBT), 0, s, b);
  return GI_OK_LAUNCH();
}

int launch_cc_init(const CcArgs& c, DenseSet f0, DenseSet f1, int32_t* lab_other, hipStream_t s) {
  hipLaunchKernelGGL(k_cc_init, dim3(grid_for(c.g.n, 256, 2048)), dim3(256), 0, s, c, f0, f1,
                     lab_other);
  return GI_OK_LAUNCH();
}

int enqueue_cc_step(const Engine& e, const DecideArgs& d, const CcArgs& c, const RowBlocks& in_rows,
                    const RowBlocks& out_rows, int cap_e, int cap_v, hipStream_t s) {
  hipLaunchKernelGGL(k_decide_frontier, dim3(1), dim3(1024), 0, s, d);
  CompactArgs ca = compact_args(e, c.fr, c.g.udeg, c.next, c.cur, c.nxt, MODE_SPARSE_PUSH,
                                MODE_DENSE_PUSH);
  if (enqueue_compaction(e, ca, s)) return -1;
  hipLaunchKernelGGL((k_cc_expand<kBT, kCH>), dim3(e.xgrid), dim3(kBT), 0, s, c,
                     expand_args(e, c.g.out_off, c.g.in_off, c.g.outdeg, MODE_SPARSE_PUSH));
  hipLaunchKernelGGL(k_cc_dense_push<kBT>, dim3(e.vgrid), dim3(kBT), 0, s, c);
  const size_t lds = sizeof(int) * (size_t)(cap_e + cap_v + 1);
  hipLaunchKernelGGL(k_cc_pull<kBT>, dim3(std::max(1, std::min(in_rows.ntab, e.rgrid))), dim3(kBT),
                     lds, s, c, in_rows, 0, cap_e);
  hipLaunchKernelGGL(k_cc_pull<kBT>, dim3(std::max(1, std::min(out_rows.ntab, e.rgrid))), dim3(kBT),
                     lds, s, c, out_rows, 1, cap_e);
  return GI_OK_LAUNCH();
}

int launch_sssp_init(const SsspArgs& sa, int src, DenseSet f0, DenseSet f1, hipStream_t s) {
  hipLaunchKernelGGL(k_sssp_init, dim3(grid_for(sa.g.n, 256, 2048)), dim3(256), 0, s, sa, src, f0,
                     f1);
  return GI_OK_LAUNCH();
}

int enqueue_sssp_step(const Engine& e, const SsspArgs& sa, hipStream_t s) {
  hipLaunchKernelGGL(k_decide_sssp, dim3(1), dim3(1024), 0, s, sa);
  hipLaunchKernelGGL(k_sssp_far_min<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, sa);
  hipLaunchKernelGGL(k_sssp_threshold, dim3(1), dim3(1024), 0, s, sa, e.cgrid);
  hipLaunchKernelGGL(k_sssp_split<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, sa);
  CompactArgs ca = compact_args(e, sa.cur, sa.g.outdeg, sa.next, nullptr, nullptr,
                                MODE_SSSP_RELAX, MODE_SSSP_RELAX);
  hipLaunchKernelGGL(k_compact_count<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, ca);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, ca, e.cgrid);
  CompactArgs w = ca;
  w.clear = DenseSet{nullptr, nullptr};
  hipLaunchKernelGGL(k_compact_write<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, w);
  hipLaunchKernelGGL((k_sssp_expand<kBT, kCH>), dim3(e.xgrid), dim3(kBT), 0, s, sa,
                     expand_args(e, sa.g.out_off, nullptr, nullptr, MODE_SSSP_RELAX));
  return GI_OK_LAUNCH();
}

}  // namespace gi
