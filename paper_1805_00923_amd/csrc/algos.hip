// BFS, connected components and delta-stepping SSSP on the frontier engine
// (common.h, traverse.h): per step, count -> decide -> write -> step.
//
// BFS (evaluation, algorithms paragraph; the paper adopts direction-optimized
// BFS): SparsePush claims unvisited out-neighbours with a compare-and-swap on
// the level array, so every vertex enters the next frontier once and no
// de-duplication is needed; DensePull lets every unvisited vertex scan its
// in-edges and stop at the first one whose source is in the frontier (early
// exit); DensePush walks the out-edges of every member of a dense frontier.
//
// CC (synchronous label propagation over edges taken both ways, here as one
// symmetric adjacency: each vertex's out-row followed by its in-row): labels
// are double-buffered.  Push steps lower neighbours' next labels with atomic
// min (the asyncMin reduction of the compiler section); pull steps take the
// minimum over the neighbours' labels without atomics.  The minimum over all
// neighbours equals the minimum over frontier neighbours: a neighbour outside
// the frontier kept the label it had a round earlier, which the vertex has
// already absorbed.
//
// SSSP: delta-stepping (Meyer and Sanders, J. Algorithms 2003) with a near
// set (tentative distance below the current bucket threshold) relaxed by
// SparsePush steps and a far set for everything improved at or beyond it;
// when the near set empties the threshold moves to the end of the bucket of
// the smallest far distance and the far set is split.
#include "bfs_dev.h"
#include "kernels.h"
#include "pr_block.h"
#include "traverse.h"

namespace gi {

constexpr int kBT = 256;
constexpr int kCH = 2048;

int expand_chunk_size() { return kCH; }

// Abandon the run (an internal size check failed).
__device__ __forceinline__ void abandon(Control* c) {
  c->error = 1;
  c->done = 1;
  c->mode = MODE_NONE;
  host_flag(&c->host->error, 1);
  host_flag(&c->host->done, 1);
}

// ---------------------------------------------------------------- decide --

// Reduce the count pass, log the step that just ran, choose the direction of
// the next one (BFS and CC), and prepare the sparse array for SparsePush.
// Every decided step's selector features go to the host trace; with the
// learned direction the attached selector picks the schedule of least
// predicted time among SparsePush, DensePush and DensePull.
__global__ __launch_bounds__(1024) void k_decide_frontier(FrontierArgs f, DecideArgs d) {
  const Blk tot = reduce_blk(f);
  const long long work = reduce_parts(d.part, 2);
  __shared__ int s_mode, s_learn, s_k;
  __shared__ float s_x[kFeat], s_xn[kFeat], s_h1[kHid], s_h2[kHid], s_y[kOut];
  Control* c = d.ctl;
  if (threadIdx.x == 0) {
    int mode = MODE_NONE, learn = 0;
    const int k = c->steps;
    if (!c->done) {
      if (k > 0) {
        if (k <= kMaxLog) c->host->log[k - 1].edges = work;
        c->edges_examined += work;
      }
      if (tot.members == 0 || (d.max_steps > 0 && k >= d.max_steps)) {
        c->done = 1;
        publish_done(c, k);
      } else {
        const float unv = d.is_bfs ? (float)(1.0 - (double)(c->visited + tot.members) / (double)f.n)
                                   : (float)((double)tot.degsum / (double)(d.edges > 0 ? d.edges : 1));
        step_features(d.fc, f.n, d.edges, tot.members, tot.degsum, c->nf, unv, s_x);
        if (k < kMaxLog)
          for (int i = 0; i < kFeat; ++i) c->host->feat[k][i] = s_x[i];
        int dir = d.direction;
        if (d.forced_dir >= 0) dir = d.forced_dir;
        else if (dir == GI_DIR_DENSE_PULL_SPARSE_PUSH)
          dir = hybrid_dense(tot.members, tot.degsum, d.edges, d.divisor) ? GI_DIR_DENSE_PULL
                                                                          : GI_DIR_SPARSE_PUSH;
        else if (dir == GI_DIR_DENSE_PUSH_SPARSE_PUSH)
          dir = hybrid_dense(tot.members, tot.degsum, d.edges, d.divisor) ? GI_DIR_DENSE_PUSH
                                                                          : GI_DIR_SPARSE_PUSH;
        if (dir == GI_DIR_LEARNED) learn = 1;
        else mode = dir;
      }
    }
    s_learn = learn;
    s_mode = mode;
    s_k = k;
  }
  __syncthreads();
  __shared__ int s_seg;
  // the first CC round gathers nothing (labels are still the ids), so
  // segments would only add their merge
  if (threadIdx.x == 0) s_seg = s_mode == MODE_DENSE_PULL && d.seg_pull == 1 && s_k > 0;
  if (s_learn) {  // workgroup-uniform
    mlp_forward_block(d.sel, s_x, s_xn, s_h1, s_h2, s_y);
    if (threadIdx.x == 0) {
      // S0..S2 are the three directions; S3, the pull over the source
      // segments, when the run has them
      const int last = d.seg_pull == 2 ? 3 : GI_DIR_DENSE_PULL;
      int best = GI_DIR_SPARSE_PUSH;
      for (int q = GI_DIR_DENSE_PUSH; q <= last; ++q)
        if (s_y[q] < s_y[best]) best = q;
      // the hybrid rule stays unless the model predicts a clear gain
      const int h = hybrid_dense(tot.members, tot.degsum, d.edges, d.divisor) ? GI_DIR_DENSE_PULL
                                                                              : GI_DIR_SPARSE_PUSH;
      const int pick = s_y[h] - s_y[best] > kLearnedMargin ? best : h;
      s_mode = pick == 3 ? GI_DIR_DENSE_PULL : pick;
      s_seg = pick == 3;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int mode = s_mode;
    c->seg = s_seg;
    if (mode >= 0) {
      const int k = s_k;
      if (k < kMaxLog)
        c->host->log[k] = StepLog{mode + (s_seg ? kLogSegmented : 0), (int)tot.members,
                                  tot.degsum, 0};
      c->steps = k + 1;
      if (mode != GI_DIR_SPARSE_PUSH) c->dense_steps++;
      c->nf = tot.members;
      c->dsum = tot.degsum;
      c->visited += tot.members;
    }
    c->mode = mode;
  }
  __syncthreads();
  if (s_mode == MODE_SPARSE_PUSH && !scan_blk<kCH>(f, tot) && threadIdx.x == 0) abandon(d.ctl);
}

// ------------------------------------------------------------------- BFS --

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_bfs_step(BfsArgs b, ExpandArgs x) {
  __shared__ int lds[expand_lds_ints<CH>()];
  const int mode = b.ctl->mode;
  if (mode == MODE_NONE) return;
  const int l1 = b.ctl->steps;
  long long work = 0;
  if (mode == MODE_DENSE_PULL) {
    const int W = (b.g.n + 63) >> 6;
    work = bfs_pull_range<BT>(b, l1, 0, W, blockIdx.x * (BT / kWave) + (int)(threadIdx.x / kWave),
                              gridDim.x * (BT / kWave), nullptr, nullptr, nullptr);
  } else {
    BfsVisit vis{b.g.out_idx, b.level, b.parent, l1, b.next, b.vis};
    if (mode == MODE_SPARSE_PUSH) expand_chunks<BT, CH>(x, vis, lds);
    else dense_push_expand<BT>(b.cur, b.g.n, b.g.out_off, vis);
    work = vis.work;
  }
  const Part p = block_sum4<BT>(Part{0, 0, work, 0});
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
  for (int i = tid; i < kParts; i += nt) b.part[i] = Part{0, 0, 0, 0};
}

// -------------------------------------------------------------------- CC --

struct CcVisit {
  const int32_t* idx;
  const int32_t* cur;
  int32_t* nxt;
  DenseSet next;
  long long work = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    if (!valid) return;
    const int v = idx[e];
    ++work;
    const int lu = cur[u];
    if (lu >= nxt[v]) return;
    const int old = atomicMin(&nxt[v], lu);
    // the first lowering of this round sees the untouched value cur[v]
    if (lu < old && old == cur[v]) next.insert(v);
  }
};

// SparsePush over the direct adjacency: slot j of vertex u's row is its
// j-th out-neighbour for j < outdeg(u), else its (j - outdeg(u))-th
// in-neighbour, so the frontier's out+in degrees give the slots as with the
// symmetric copy.
struct CcVisitDirect {
  const int32_t* out_off;
  const int32_t* out_idx;
  const int32_t* in_off;
  const int32_t* in_idx;
  const int32_t* cur;
  int32_t* nxt;
  DenseSet next;
  long long work = 0;
  __device__ __forceinline__ void operator()(int u, int j, bool valid) {
    if (!valid) return;
    const int ob = out_off[u], od = out_off[u + 1] - ob;
    const int v = j < od ? out_idx[ob + j] : in_idx[in_off[u] + (j - od)];
    ++work;
    const int lu = cur[u];
    if (lu >= nxt[v]) return;
    const int old = atomicMin(&nxt[v], lu);
    if (lu < old && old == cur[v]) next.insert(v);
  }
};

// Pull over destination blocks of the symmetric adjacency: the block's
// neighbour labels are staged in LDS, then the rows' minima are taken by an
// edge-parallel segmented minimum; vertices whose label drops join the next
// frontier.  Block entries carry their edge range and the next one is
// fetched ahead, and the block's row bounds and current labels are loaded
// together with the gathers, so a block costs one memory latency.
template <int BT>
__device__ long long cc_pull(const CcArgs& c, int* lds) {
  constexpr int kPer = (kCcCapV + 1 + BT - 1) / BT;
  int* lds_val = lds;
  int* lds_off = lds + kCcCapE;
  int* lds_cur = lds_off + kCcCapV + 1;
  int* lds_min = lds_cur + kCcCapV;
  __shared__ int red[BT / kWave];
  long long work = 0;
  // With the direct adjacency the entries of the out-row blocks come first,
  // then those of the in-row blocks; a vertex's two rows are then reduced by
  // different blocks, which merge by atomic minimum.
  const int nt1 = c.rows.ntab, ntab = nt1 + (c.direct ? c.rows_in.ntab : 0);
  auto entry = [&](int t) -> int4 {
    return t < nt1 ? c.rows.table[t] : c.rows_in.table[t - nt1];
  };
  const int32_t* cur = c.cur;
  const int tid = threadIdx.x, lane = __lane_id();
  // In the first round every label is still the vertex id, so a
  // neighbour's label is its id and nothing needs gathering.  (A neighbour
  // outside the frontier cannot lower a label, but testing the frontier bit
  // before the gather measured slower than gathering every label.)
  const bool ids = c.ctl->steps == 1;
  auto label_of = [cur, ids](int u) -> int { return ids ? u : cur[u]; };
  // the next entry is fetched while the current block is processed
  int4 nx = (int)blockIdx.x < ntab ? entry(blockIdx.x) : make_int4(0, 0, 0, 0);
  for (int t = blockIdx.x; t < ntab; t += gridDim.x) {
    const int4 r = nx;
    if (t + (int)gridDim.x < ntab) nx = entry(t + gridDim.x);
    const RowBlocks& rb = t < nt1 ? c.rows : c.rows_in;
    if (r.y < 0) {
      // chunk -(r.y + 1) of the long row r.x: workgroup minimum over at
      // most kCcCapE edges (four loads in flight per thread), merged by an
      // atomic minimum.  At the start of a round nxt equals cur for every
      // vertex (the count pass restores the vertices that changed), so the
      // chunk that first lowers nxt below cur adds the row to the frontier.
      const int row = r.x, eb = r.z, ee = r.w;
      int m0 = 0x7fffffff, m1 = 0x7fffffff;
      int e = eb + tid;
      for (; e + 3 * BT < ee; e += 4 * BT) {
        const int a0 = rb.idx[e], a1 = rb.idx[e + BT], a2 = rb.idx[e + 2 * BT],
                  a3 = rb.idx[e + 3 * BT];
        m0 = min(m0, min(label_of(a0), label_of(a1)));
        m1 = min(m1, min(label_of(a2), label_of(a3)));
      }
      for (; e < ee; e += BT) m0 = min(m0, label_of(rb.idx[e]));
      int mn = wave_min(min(m0, m1));
      if (lane == 0) red[tid / kWave] = mn;
      __syncthreads();
      if (tid == 0) {
        work += ee - eb;
        for (int i = 0; i < BT / kWave; ++i) mn = min(mn, red[i]);
        if (mn < c.nxt[row]) {
          const int old = atomicMin(&c.nxt[row], mn);
          if (mn < old && old == cur[row]) c.next.insert(row);
        }
      }
      __syncthreads();
      continue;
    }
    const int kb = r.x, ke = r.y, nr = ke - kb;
    const int e0 = r.z, ne = r.w - r.z;
    if (tid == 0) work += ne;
    int offv[kPer], curv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = tid + i * BT;
      offv[i] = k <= nr ? rb.off[kb + k] : 0;
      curv[i] = k < nr ? cur[kb + k] : 0;
    }
    gather_block<BT, int>(rb.idx, e0, ne, lds_val, label_of);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = tid + i * BT;
      if (k <= nr) lds_off[k] = offv[i] - e0;
      if (k < nr) {
        lds_cur[k] = curv[i];
        lds_min[k] = 0x7fffffff;
      }
    }
    __syncthreads();
    // Edge-parallel row minima: thread t takes a run of ceil(ne / BT)
    // consecutive edges, finds the row of its first edge by binary search
    // of the row bounds, and merges one partial minimum per row it touches
    // with an LDS atomic.  The block's edges are spread evenly over the
    // threads however skewed its rows are (a block can hold hundreds of
    // empty rows and one row of a thousand edges).
    {
      const int ept = (ne + BT - 1) / BT;
      const int eb = tid * ept, ee = min(ne, eb + ept);
      if (eb < ee) {
        int lo = 0, hi = nr;  // lds_off[lo] <= eb < lds_off[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (lds_off[mid] <= eb) lo = mid;
          else hi = mid;
        }
        int k = lo, rend = lds_off[k + 1], m = 0x7fffffff;
        for (int j = eb; j < ee; ++j) {
          while (j >= rend) {
            atomicMin(&lds_min[k], m);
            m = 0x7fffffff;
            ++k;
            rend = lds_off[k + 1];
          }
          m = min(m, lds_val[j]);
        }
        atomicMin(&lds_min[k], m);
      }
    }
    __syncthreads();
    if (c.direct) {
      // the vertex's other row may be reduced concurrently: only a lower
      // label is written, by atomic minimum (nxt equals cur at the start of
      // the round, so the first lowering sees cur and adds the vertex)
      for (int k = tid; k < nr; k += BT) {
        const int lv = lds_cur[k], mn = lds_min[k];
        if (mn < lv) {
          const int old = atomicMin(&c.nxt[kb + k], mn);
          if (mn < old && old == lv) c.next.insert(kb + k);
        }
      }
      __syncthreads();
      continue;
    }
    // vertex updates, one row per thread: the rows a wave finishes are
    // consecutive, so their frontier bits take at most two atomic ORs
    for (int k0 = 0; k0 < nr; k0 += BT) {
      const int k = k0 + tid;
      bool chg = false;
      if (k < nr) {
        const int lv = lds_cur[k], mn = lds_min[k];
        const int x = mn < lv ? mn : lv;
        c.nxt[kb + k] = x;
        chg = x < lv;
        if (chg && c.next.bm) c.next.bm[kb + k] = 1;
      }
      if (!c.next.bm) {
        const unsigned long long m = __ballot(chg);
        if (m != 0ull && lane == 0) {
          const int r0 = kb + k0 + (tid - lane);
          const int w = r0 >> 6, sh = r0 & 63;
          atomicOr((unsigned long long*)&c.next.bv[w], m << sh);
          if (sh != 0 && (m >> (64 - sh)) != 0ull)
            atomicOr((unsigned long long*)&c.next.bv[w + 1], m >> (64 - sh));
        }
      }
    }
    __syncthreads();
  }
  return work;
}

// Segmented pull (cache-segmented DensePull for CC): workgroup b serves
// segment b mod p, so with p = 8 and the round-robin dispatch of workgroups
// over the XCDs every XCD gathers labels from one segment only, which stays
// in its L2.  Each segment block leaves its rows' minima in that segment's
// partial array; k_cc_seg_merge then takes the minimum over the segments.
template <int BT>
__device__ long long cc_pull_seg(const CcArgs& c, int* lds) {
  constexpr int kPer = (kCcCapV + 1 + BT - 1) / BT;
  int* lds_val = lds;
  int* lds_off = lds + kCcCapE;
  int* lds_min = lds_off + kCcCapV + 1;
  __shared__ int red[BT / kWave];
  long long work = 0;
  const int p = c.nseg, G = (int)gridDim.x / p;
  if ((int)blockIdx.x >= G * p) return 0;
  const int x = (int)blockIdx.x % p, b0 = (int)blockIdx.x / p;
  const CcSeg sg = c.segs[x];
  const RowBlocks& rb = sg.rows;
  uint32_t* part = c.seg_min + (size_t)x * (size_t)c.g.n;
  const int32_t* cur = c.cur;
  const int tid = threadIdx.x, lane = __lane_id();
  const bool ids = c.ctl->steps == 1;
  auto label_of = [cur, ids](int u) -> int { return ids ? u : cur[u]; };
  int4 nx = b0 < rb.ntab ? rb.table[b0] : make_int4(0, 0, 0, 0);
  for (int t = b0; t < rb.ntab; t += G) {
    const int4 r = nx;
    if (t + G < rb.ntab) nx = rb.table[t + G];
    if (r.y < 0) {  // chunk of a long row
      int m0 = 0x7fffffff, m1 = 0x7fffffff;
      int e = r.z + tid;
      for (; e + 3 * BT < r.w; e += 4 * BT) {
        const int a0 = rb.idx[e], a1 = rb.idx[e + BT], a2 = rb.idx[e + 2 * BT],
                  a3 = rb.idx[e + 3 * BT];
        m0 = min(m0, min(label_of(a0), label_of(a1)));
        m1 = min(m1, min(label_of(a2), label_of(a3)));
      }
      for (; e < r.w; e += BT) m0 = min(m0, label_of(rb.idx[e]));
      int mn = wave_min(min(m0, m1));
      if (lane == 0) red[tid / kWave] = mn;
      __syncthreads();
      if (tid == 0) {
        work += r.w - r.z;
        for (int i = 0; i < BT / kWave; ++i) mn = min(mn, red[i]);
        atomicMin(&part[sg.dst[r.x]], (uint32_t)mn);
      }
      __syncthreads();
      continue;
    }
    const int kb = r.x, ke = r.y, nr = ke - kb;
    const int e0 = r.z, ne = r.w - r.z;
    if (tid == 0) work += ne;
    int offv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = tid + i * BT;
      offv[i] = k <= nr ? rb.off[kb + k] : 0;
    }
    gather_block<BT, int>(rb.idx, e0, ne, lds_val, label_of);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = tid + i * BT;
      if (k <= nr) lds_off[k] = offv[i] - e0;
      if (k < nr) lds_min[k] = 0x7fffffff;
    }
    __syncthreads();
    {
      const int ept = (ne + BT - 1) / BT;
      const int eb = tid * ept, ee = min(ne, eb + ept);
      if (eb < ee) {
        int lo = 0, hi = nr;  // lds_off[lo] <= eb < lds_off[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (lds_off[mid] <= eb) lo = mid;
          else hi = mid;
        }
        int k = lo, rend = lds_off[k + 1], m = 0x7fffffff;
        for (int j = eb; j < ee; ++j) {
          while (j >= rend) {
            atomicMin(&lds_min[k], m);
            m = 0x7fffffff;
            ++k;
            rend = lds_off[k + 1];
          }
          m = min(m, lds_val[j]);
        }
        atomicMin(&lds_min[k], m);
      }
    }
    __syncthreads();
    // every row of a segment has a neighbour in it, so every row writes
    for (int k = tid; k < nr; k += BT) part[sg.dst[kb + k]] = (uint32_t)lds_min[k];
    __syncthreads();
  }
  return work;
}

// Merge of the segment minima (dense pull steps of the segmented form): new
// label = min(old, minima), partial arrays reset, next frontier written one
// whole word per wave.
template <int BT>
__global__ __launch_bounds__(BT) void k_cc_seg_merge(CcArgs c) {
  if (c.ctl->mode != MODE_DENSE_PULL || !c.ctl->seg) return;
  const int n = c.g.n, W = (n + 63) >> 6, lane = __lane_id();
  const int wave = (int)((blockIdx.x * BT + threadIdx.x) / kWave);
  const int nw = (int)(gridDim.x * BT / kWave);
  for (int w = wave; w < W; w += nw) {
    const int v = (w << 6) + lane;
    bool chg = false;
    if (v < n) {
      uint32_t mn = 0xffffffffu;
      for (int x = 0; x < c.nseg; ++x) {
        uint32_t* q = c.seg_min + (size_t)x * (size_t)n + v;
        mn = min(mn, *q);
        *q = 0xffffffffu;
      }
      const int lv = c.cur[v];
      const int nl = mn < (uint32_t)lv ? (int)mn : lv;
      c.nxt[v] = nl;
      chg = nl < lv;
      if (c.next.bm) c.next.bm[v] = chg ? 1 : 0;
    }
    const unsigned long long m = __ballot(chg);
    if (!c.next.bm && lane == 0) c.next.bv[w] = m;
  }
}

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_cc_step(CcArgs c, ExpandArgs x) {
  static_assert(kCcCapE + 3 * kCcCapV + 1 <= expand_lds_ints<CH>(), "LDS too small");
  __shared__ int lds[expand_lds_ints<CH>()];
  const int mode = c.ctl->mode;
  if (mode == MODE_NONE) return;
  long long work = 0;
  if (mode == MODE_DENSE_PULL) {
    work = c.nseg > 1 && c.ctl->seg ? cc_pull_seg<BT>(c, lds) : cc_pull<BT>(c, lds);
  } else if (c.direct) {
    if (mode == MODE_SPARSE_PUSH) {
      CcVisitDirect vis{c.g.out_off, c.g.out_idx, c.g.in_off, c.g.in_idx, c.cur, c.nxt, c.next};
      expand_chunks<BT, CH>(x, vis, lds);
      work = vis.work;
    } else {
      // DensePush over the out-rows, then over the in-rows
      CcVisit vo{c.g.out_idx, c.cur, c.nxt, c.next};
      dense_push_expand<BT>(c.fr, c.g.n, c.g.out_off, vo);
      CcVisit vi{c.g.in_idx, c.cur, c.nxt, c.next};
      dense_push_expand<BT>(c.fr, c.g.n, c.g.in_off, vi);
      work = vo.work + vi.work;
    }
  } else {
    CcVisit vis{c.sym_idx, c.cur, c.nxt, c.next};
    if (mode == MODE_SPARSE_PUSH) expand_chunks<BT, CH>(x, vis, lds);
    else dense_push_expand<BT>(c.fr, c.g.n, c.sym_off, vis);
    work = vis.work;
  }
  const Part p = block_sum4<BT>(Part{0, 0, work, 0});
  if (threadIdx.x == 0) c.part[blockIdx.x] = p;
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
  for (int i = tid; i < kParts; i += nt) c.part[i] = Part{0, 0, 0, 0};
}

// Symmetric adjacency: row v = out-row of v, then in-row of v (one wave per
// vertex, grid-stride).
__global__ void k_build_sym(DevGraph g, const int32_t* sym_off, int32_t* sym_idx) {
  const int lane = __lane_id();
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int nw = (int)((gridDim.x * blockDim.x) / kWave);
  for (int v = wave; v < g.n; v += nw) {
    const int o0 = g.out_off[v], o1 = g.out_off[v + 1];
    const int i0 = g.in_off[v], i1 = g.in_off[v + 1];
    const int base = sym_off[v];
    for (int k = lane; k < o1 - o0; k += kWave) sym_idx[base + k] = g.out_idx[o0 + k];
    for (int k = lane; k < i1 - i0; k += kWave) sym_idx[base + (o1 - o0) + k] = g.in_idx[i0 + k];
  }
}

// ------------------------------------------------------------------ SSSP --

__global__ __launch_bounds__(1024) void k_decide_sssp(FrontierArgs f, SsspArgs s) {
  const Blk tot = reduce_blk(f);
  const long long pa = reduce_parts(s.part, 0);
  const long long pc = reduce_parts(s.part, 2);
  __shared__ int s_mode;
  if (threadIdx.x == 0) {
    Control* c = s.ctl;
    const int prev = c->mode;
    const int k = c->steps;
    if (prev == MODE_SSSP_RELAX) {
      c->far_count += pa;  // far members added by the relaxation
      if (k > 0 && k <= kMaxLog) c->host->log[k - 1].edges = pc;
      c->edges_examined += pc;
    } else if (prev == MODE_SSSP_SPLIT) {
      c->far_count = pa;   // far members kept by the split
    }
    int mode = MODE_NONE;
    if (c->done) {
    } else if (c->overflow) {
      c->done = 1;
      host_flag(&c->host->overflow, 1);
      host_flag(&c->host->done, 1);
    } else if (tot.members > 0) {
      if (k < kMaxLog) c->host->log[k] = StepLog{GI_DIR_SPARSE_PUSH, (int)tot.members, tot.degsum, 0};
      c->steps = k + 1;
      c->nf = tot.members;
      mode = MODE_SSSP_RELAX;
    } else if (c->far_count > 0) {
      mode = MODE_SSSP_SPLIT;
    } else {
      c->done = 1;
      publish_done(c, k);
    }
    c->mode = mode;
    s_mode = mode;
  }
  __syncthreads();
  if (s_mode == MODE_SSSP_RELAX && !scan_blk<kCH>(f, tot) && threadIdx.x == 0) abandon(s.ctl);
}

// RELAX: sparse array of the near set.  SPLIT: smallest far distance at or
// beyond the threshold in this workgroup's word range (~0 when none).
template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_sssp_prepare(FrontierArgs f, SsspArgs s) {
  const int mode = s.ctl->mode;
  if (mode == MODE_SSSP_RELAX) {
    write_body<BT, CH>(f);
    return;
  }
  if (mode != MODE_SSSP_SPLIT) return;
  const int W = (f.n + 63) >> 6;
  const int w0 = blockIdx.x * f.tw, w1 = min(W, w0 + f.tw);
  const unsigned long long th = s.ctl->thresh;
  unsigned long long mn = ~0ull;
  for (int w = w0 + (int)threadIdx.x; w < w1; w += BT) {
    uint64_t x = s.far.word(w);
    while (x) {
      const int v = (w << 6) + __ffsll((long long)x) - 1;
      x &= x - 1;
      const unsigned long long d = s.dist[v];
      if (d >= th && d < mn) mn = d;
    }
  }
  __shared__ unsigned long long red[BT / kWave];
  mn = wave_min(mn);
  if (__lane_id() == 0) red[threadIdx.x / kWave] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < BT / kWave; ++i) mn = red[i] < mn ? red[i] : mn;
    s.fmin[blockIdx.x] = mn;
  }
}

// SPLIT: new threshold = end of the bucket of the smallest far distance.
__global__ __launch_bounds__(1024) void k_sssp_threshold(SsspArgs s, int nblk) {
  Control* ctl = s.ctl;
  if (ctl->mode != MODE_SSSP_SPLIT) return;
  __shared__ unsigned long long red[1024];
  unsigned long long mn = ~0ull;
  for (int i = threadIdx.x; i < nblk; i += 1024) mn = s.fmin[i] < mn ? s.fmin[i] : mn;
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

struct SsspVisit {
  const int32_t* idx;
  const uint32_t* w;
  uint32_t* dist;
  DenseSet near;
  DenseSet far;
  unsigned long long thresh;
  int* overflow;
  long long far_new = 0, work = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
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
    if (nd < thresh) near.insert(v);
    else if (far.insert(v)) ++far_new;
  }
};

// RELAX: relax the near set.  SPLIT: stale far members (distance below the
// old threshold, already relaxed) are dropped, members of the new bucket
// move to the next near set, the rest stay.
template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_sssp_step(SsspArgs s, ExpandArgs x) {
  __shared__ int lds[expand_lds_ints<CH>()];
  Control* ctl = s.ctl;
  const int mode = ctl->mode;
  if (mode != MODE_SSSP_RELAX && mode != MODE_SSSP_SPLIT) return;
  Part p{0, 0, 0, 0};
  if (mode == MODE_SSSP_RELAX) {
    SsspVisit vis{s.g.out_idx, s.g.out_w, s.dist, s.next, s.far, ctl->thresh, &ctl->overflow};
    expand_chunks<BT, CH>(x, vis, lds);
    p = Part{vis.far_new, 0, vis.work, 0};
  } else {
    const int W = (s.g.n + 63) >> 6;
    const unsigned long long told = ctl->told, tnew = ctl->thresh;
    long long kept = 0;
    for (int w = blockIdx.x * BT + (int)threadIdx.x; w < W; w += gridDim.x * BT) {
      uint64_t xw = s.far.word(w), keep = 0;
      while (xw) {
        const int b = __ffsll((long long)xw) - 1;
        xw &= xw - 1;
        const int v = (w << 6) + b;
        const unsigned long long d = s.dist[v];
        if (d < told) continue;
        if (d < tnew) {
          s.next.insert(v);
        } else {
          keep |= 1ull << b;
          ++kept;
        }
      }
      s.far.bv[w] = keep;
    }
    p = Part{kept, 0, 0, 0};
  }
  p = block_sum4<BT>(p);
  if (threadIdx.x == 0) s.part[blockIdx.x] = p;
}

__global__ void k_sssp_init(SsspArgs s, int src) {
  const int n = s.g.n, W = (n + 63) >> 6;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += nt) s.dist[v] = v == src ? 0u : 0xFFFFFFFFu;
  for (int w = tid; w < W; w += nt) {
    const uint64_t word = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    s.cur.bv[w] = word;
    s.next.bv[w] = 0ull;
    s.far.bv[w] = 0ull;
  }
  for (int i = tid; i < kParts; i += nt) s.part[i] = Part{0, 0, 0, 0};
}

// ---------------------------------------------------------- PageRankDelta --
//
// The PageRankDelta program of the algorithm-language section, with its
// DensePull-SparsePush schedule and bitvector frontier (scheduling section):
// per round, the active vertices' Delta / OutDegree reaches DeltaSum of
// their out-neighbours (push: FP64 atomic adds from the compacted
// frontier; pull: the PageRank destination-block sum over in-edges, where an
// inactive source contributes an exact zero), then every vertex updates:
//   round 1: Delta = alpha DeltaSum + (1-alpha)/n, Rank += Delta, Delta -= 1/n
//   later:   Delta = alpha DeltaSum,               Rank += Delta
// and stays active when |Delta| > eps Rank.  Delta / OutDegree is kept as one
// FP64 array, the fused layout of the paper's vertex-data optimization.

struct PrdVisit {
  const int32_t* idx;
  const double* contrib;
  double* dsum;
  long long work = 0;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    if (!valid) return;
    ++work;
    atomicAdd(&dsum[idx[e]], contrib[u]);
  }
};

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_prd_step(PrdArgs a, ExpandArgs x) {
  extern __shared__ int smem_i[];
  const int mode = a.ctl->mode;
  if (mode == MODE_NONE) return;
  long long work = 0;
  if (mode == MODE_DENSE_PULL) {
    double* lds_val = reinterpret_cast<double*>(smem_i);
    int* lds_off = reinterpret_cast<int*>(lds_val + a.cap_e);
    PrVertex pv{a.g.outdeg, a.base, a.alpha};
    for (int t = blockIdx.x; t < a.rows.ntab; t += gridDim.x) {
      pr_rows_block<BT, double>(a.rows, t, a.cap_e, a.contrib, 1, pv, nullptr, nullptr, a.dsum,
                                lds_val, lds_off);
    }
    if (threadIdx.x == 0) work = blockIdx.x == 0 ? a.g.m : 0;
  } else {
    PrdVisit vis{a.g.out_idx, a.contrib, a.dsum};
    if (mode == MODE_SPARSE_PUSH) expand_chunks<BT, CH>(x, vis, smem_i);
    else dense_push_expand<BT>(a.cur, a.g.n, a.g.out_off, vis);
    work = vis.work;
  }
  const Part p = block_sum4<BT>(Part{0, 0, work, 0});
  if (threadIdx.x == 0) a.part[blockIdx.x] = p;
}

// Vertex update and next frontier: one wave per 64-vertex word.
__global__ __launch_bounds__(256) void k_prd_update(PrdArgs a) {
  if (a.ctl->mode == MODE_NONE) return;
  const int round = a.ctl->steps;  // 1-based
  const int n = a.g.n, W = (n + 63) >> 6, lane = __lane_id();
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int nw = (int)((gridDim.x * blockDim.x) / kWave);
  for (int w = wave; w < W; w += nw) {
    const int v = (w << 6) + lane;
    bool act = false;
    if (v < n) {
      const double ds = a.dsum[v];
      double d, r = a.rank[v];
      if (round == 1) {
        d = a.alpha * ds + a.base;
        r += d;
        d -= a.inv_n;
      } else {
        d = a.alpha * ds;
        r += d;
      }
      a.dsum[v] = 0.0;
      a.delta[v] = d;
      a.rank[v] = r;
      act = fabs(d) > a.eps * r;
      const int deg = a.g.outdeg[v];
      a.contrib[v] = (act && deg > 0) ? d / (double)deg : 0.0;
    }
    const unsigned long long m = __ballot(act);
    if (lane == 0) a.next.bv[w] = m;
  }
}

// Initial state: Rank = 0, Delta = 1/n, every vertex active.
__global__ void k_prd_init(PrdArgs a) {
  const int n = a.g.n, W = (n + 63) >> 6;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += nt) {
    a.rank[v] = 0.0;
    a.delta[v] = a.inv_n;
    a.dsum[v] = 0.0;
    const int deg = a.g.outdeg[v];
    a.contrib[v] = deg > 0 ? a.inv_n / (double)deg : 0.0;
  }
  for (int w = tid; w < W; w += nt) {
    const int rem = n - (w << 6);
    a.cur.bv[w] = rem >= 64 ? ~0ull : ((1ull << rem) - 1ull);
    a.next.bv[w] = 0ull;
  }
  for (int i = tid; i < kParts; i += nt) a.part[i] = Part{0, 0, 0, 0};
}

// ----------------------------------------------------------- betweenness --
//
// Brandes' dependencies from one source as two labelled sweeps (the paper's
// betweenness program: a forward apply that counts shortest paths, then a
// backward apply over the levels in reverse).  Forward, level by level: the
// listed vertices of level L push their path counts to out-neighbours; the
// first to claim a vertex (compare-and-swap on its level) appends it to the
// level-ordered list with one atomic per wave, and every edge into level
// L+1 adds sigma[u] with an FP64 atomic.  Backward, for L from the deepest
// level down: each vertex w of level L+1 sends (1 + delta[w]) / sigma[w] to
// its in-neighbours at level L, which then set delta = sigma * the sum.

// Degree sum of the next level, for its direction: kept in the control
// block's sa_slots, which the frontier engine's compaction uses and
// betweenness does not.
__device__ __forceinline__ void bc_add_degrees(Control* c, const int32_t* outdeg, bool win, int v) {
  const long long d = wave_sum((long long)(win ? outdeg[v] : 0));
  if (__lane_id() == 0 && d != 0) atomicAdd((unsigned long long*)&c->sa_slots, (unsigned long long)d);
}

struct BcFwdVisit {
  const int32_t* idx;
  int32_t* level;
  double* sigma;
  int32_t* order;
  unsigned long long* count;
  int l1;
  Control* ctl;
  const int32_t* outdeg;
  __device__ __forceinline__ void operator()(int u, int e, bool valid) {
    int v = -1;
    bool win = false, add = false;
    if (valid) {
      v = idx[e];
      const int lv = level[v];
      if (lv < 0) {
        const int old = atomicCAS(&level[v], -1, l1);
        win = old == -1;
        add = win || old == l1;
      } else {
        add = lv == l1;
      }
      if (add) atomicAdd(&sigma[v], sigma[u]);
    }
    // called by whole waves: one reservation per wave for the new vertices
    const unsigned long long m = __ballot(win);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long base = 0;
      if (__lane_id() == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
      base = __shfl(base, leader, kWave);
      if (win) order[base + __popcll(m & lanemask_lt())] = v;
      bc_add_degrees(ctl, outdeg, win, v);
    }
  }
};

// Push level (small frontiers): the listed vertices push their path counts
// to the next level with FP64 atomic adds.
template <int BT>
__global__ __launch_bounds__(BT) void k_bc_forward(BcArgs a) {
  const Control* c = a.ctl;
  if (c->done || c->mode != MODE_SPARSE_PUSH) return;
  const int l1 = c->steps + 1;
  BcFwdVisit vis{a.g.out_idx, a.level, a.sigma, a.order, &a.ctl->bc_count, l1, a.ctl,
                 a.g.outdeg};
  push_list<BT>(a.order, (long long)c->bc_start, (long long)c->bc_end, a.g.out_off, vis);
}

// fs for a pull level: the previous level's entries are cleared, the
// current level's set to their path counts (so fs is nonzero exactly on
// the frontier).
__global__ void k_bc_fs(BcArgs a, int clear_only) {
  const Control* c = a.ctl;
  if (c->done) return;
  const long long prev = a.bounds[c->steps > 0 ? c->steps - 1 : 0];
  const long long b = (long long)c->bc_start, e = (long long)c->bc_end;
  const bool set = !clear_only && c->mode == MODE_DENSE_PULL;
  for (long long i = prev + blockIdx.x * (long long)blockDim.x + threadIdx.x; i < e;
       i += (long long)gridDim.x * blockDim.x) {
    const int u = a.order[i];
    a.fs[u] = (i >= b && set) ? a.sigma[u] : 0.0;
  }
}

// Pull level (large frontiers): every unvisited vertex sums fs over its
// in-edges, atomic-free: destination blocks staged in LDS, rows summed by
// LDS atomics (path counts are integers, exact in any order below 2^53).
// A vertex with a nonzero sum joins the next level.  Hub rows are chunk
// entries whose partial sums meet in sigma by FP64 atomics; the chunk that
// first claims the level appends the vertex.
template <int BT>
__global__ __launch_bounds__(BT) void k_bc_forward_pull(BcArgs a) {
  constexpr int kPer = (kCcCapV + 1 + BT - 1) / BT;
  __shared__ double s_val[kCcCapE];
  __shared__ double s_sum[kCcCapV];
  __shared__ int s_off[kCcCapV + 1];
  __shared__ double red[BT / kWave];
  const Control* c = a.ctl;
  if (c->done || c->mode != MODE_DENSE_PULL) return;
  const int l1 = c->steps + 1, tid = threadIdx.x, lane = __lane_id();
  (void)c;
  const RowBlocks& rb = a.in_rows;
  unsigned long long* count = &a.ctl->bc_count;
  auto append = [&](bool win, int v) {
    const unsigned long long m = __ballot(win);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
      base = __shfl(base, leader, kWave);
      if (win) a.order[base + __popcll(m & lanemask_lt())] = v;
      bc_add_degrees(a.ctl, a.g.outdeg, win, v);
    }
  };
  for (int t = blockIdx.x; t < rb.ntab; t += gridDim.x) {
    const int4 r = rb.table[t];
    if (r.y < 0) {  // chunk of a hub row
      const int v = r.x;
      double sum = 0.0;
      const int lv = a.level[v];  // unvisited, or claimed by another chunk of this level
      if (lv < 0 || lv == l1)
        for (int e = r.z + tid; e < r.w; e += BT) sum += a.fs[rb.idx[e]];
      sum = wave_sum(sum);
      if (lane == 0) red[tid / kWave] = sum;
      __syncthreads();
      bool win = false;
      if (tid < kWave) {
        double tot = 0.0;
        if (tid == 0)
          for (int i = 0; i < BT / kWave; ++i) tot += red[i];
        if (tid == 0 && tot > 0.0) {
          atomicAdd(&a.sigma[v], tot);
          win = atomicCAS(&a.level[v], -1, l1) == -1;
        }
        append(win, v);
      }
      __syncthreads();
      continue;
    }
    const int kb = r.x, ke = r.y, nr = ke - kb, e0 = r.z, ne = r.w - r.z;
    int offv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = tid + i * BT;
      offv[i] = k <= nr ? rb.off[kb + k] : 0;
    }
    gather_block<BT, double>(rb.idx, e0, ne, s_val, [&](int u) { return a.fs[u]; });
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int k = tid + i * BT;
      if (k <= nr) s_off[k] = offv[i] - e0;
      if (k < nr) s_sum[k] = 0.0;
    }
    __syncthreads();
    {
      const int ept = (ne + BT - 1) / BT;
      const int eb = tid * ept, ee = min(ne, eb + ept);
      if (eb < ee) {
        int lo = 0, hi = nr;  // s_off[lo] <= eb < s_off[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_off[mid] <= eb) lo = mid;
          else hi = mid;
        }
        int k = lo, rend = s_off[k + 1];
        double m = 0.0;
        for (int j = eb; j < ee; ++j) {
          while (j >= rend) {
            if (m != 0.0) atomicAdd(&s_sum[k], m);
            m = 0.0;
            ++k;
            rend = s_off[k + 1];
          }
          m += s_val[j];
        }
        if (m != 0.0) atomicAdd(&s_sum[k], m);
      }
    }
    __syncthreads();
    for (int k0 = 0; k0 < nr; k0 += BT) {
      const int k = k0 + tid;
      bool win = false;
      int v = -1;
      if (k < nr) {
        v = kb + k;
        const double sum = s_sum[k];
        if (sum > 0.0 && a.level[v] < 0) {  // rows are this block's alone
          a.level[v] = l1;
          a.sigma[v] = sum;
          win = true;
        }
      }
      append(win, v);
    }
    __syncthreads();
  }
}

// Close the level: log it, and either end the sweep or open the next level,
// choosing its direction by the hybrid rule |F| + sum deg(F) > m / divisor.
__global__ void k_bc_advance(BcArgs a) {
  Control* c = a.ctl;
  if (c->done) return;
  const int k = c->steps;
  const unsigned long long cnt = __hip_atomic_load(&c->bc_count, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
  if (k < kMaxLog)
    c->host->log[k] = StepLog{c->mode, (int)(c->bc_end - c->bc_start), c->dsum, 0};
  if (c->mode != MODE_SPARSE_PUSH) c->dense_steps++;
  c->steps = k + 1;
  a.bounds[k + 1] = c->bc_end;
  if (cnt == c->bc_end) {
    c->done = 1;
    publish_done(c, k + 1);
  } else {
    c->bc_start = c->bc_end;
    c->bc_end = cnt;
    const long long nf = (long long)(cnt - c->bc_start);
    c->dsum = c->sa_slots;
    c->sa_slots = 0;
    c->mode = hybrid_dense(nf, c->dsum, a.g.m, a.divisor) ? MODE_DENSE_PULL : MODE_SPARSE_PUSH;
  }
}

// Backward, level L (deepest first), atomic-free: each vertex u of the level
// sums bw[w] over its out-neighbours w on level L+1 (its successors on
// shortest paths), delta[u] = sigma[u] * sum, and publishes
// bw[u] = (1 + delta[u]) / sigma[u] for level L-1.  A workgroup takes BT
// listed vertices; their out-rows are concatenated (a prefix sum of the
// degrees) and walked BT edges per round, each thread adding into its row's
// LDS sum, so a hub row is shared by the whole workgroup.
// Backward, level L (deepest first), atomic-free: each vertex u of the level
// sums bw[w] over its out-neighbours w on level L+1 (its successors on
// shortest paths), delta[u] = sigma[u] * sum, and publishes
// bw[u] = (1 + delta[u]) / sigma[u] for level L-1.  Rows are binned by
// out-degree: up to kBcSmall edges one thread per vertex, up to kHubDeg one
// wave, longer ones the whole workgroup; each bin's kernel walks the whole
// level list and takes its own vertices (a level of at most 64K vertices
// uses the workgroup kernel for all).
constexpr int kBcSmall = 32;

__device__ __forceinline__ void bc_finish_vertex(const BcArgs& a, int u, double sum) {
  const double dl = u == a.src ? 0.0 : a.sigma[u] * sum;
  a.delta[u] = dl;
  a.bw[u] = (1.0 + dl) / a.sigma[u];
}

__device__ __forceinline__ double bc_succ(const BcArgs& a, int w, int L) {
  const int lw = a.level[w];
  const double c = a.bw[w];
  return lw == L + 1 ? c : 0.0;
}

template <int BT>
__global__ __launch_bounds__(BT) void k_bc_backward_wg(BcArgs a, long long b, long long e, int L,
                                                       int min_deg) {
  for (long long i = b + blockIdx.x; i < e; i += gridDim.x) {
    const int u = a.order[i];
    const int rb = a.g.out_off[u], re = a.g.out_off[u + 1];
    if (re - rb < min_deg) continue;  // workgroup-uniform
    double sum = 0.0, sum2 = 0.0;
    int j = rb + (int)threadIdx.x;
    for (; j + BT < re; j += 2 * BT) {
      const int w0 = a.g.out_idx[j], w1 = a.g.out_idx[j + BT];
      sum += bc_succ(a, w0, L);
      sum2 += bc_succ(a, w1, L);
    }
    if (j < re) sum += bc_succ(a, a.g.out_idx[j], L);
    const double tot = block_sum<BT>(sum + sum2);
    if (threadIdx.x == 0) bc_finish_vertex(a, u, tot);
  }
}

__global__ __launch_bounds__(256) void k_bc_backward_wave(BcArgs a, long long b, long long e,
                                                          int L) {
  const int lane = __lane_id();
  const long long wave = (long long)(blockIdx.x * 256 + threadIdx.x) / kWave;
  const long long nw = (long long)gridDim.x * (256 / kWave);
  for (long long i = b + wave; i < e; i += nw) {
    const int u = a.order[i];
    const int rb = a.g.out_off[u], re = a.g.out_off[u + 1];
    if (re - rb <= kBcSmall || re - rb > kHubDeg) continue;  // wave-uniform
    double sum = 0.0;
    for (int j = rb + lane; j < re; j += kWave) sum += bc_succ(a, a.g.out_idx[j], L);
    sum = wave_sum(sum);
    if (lane == 0) bc_finish_vertex(a, u, sum);
  }
}

__global__ __launch_bounds__(256) void k_bc_backward_thread(BcArgs a, long long b, long long e,
                                                            int L) {
  for (long long i = b + blockIdx.x * 256LL + threadIdx.x; i < e; i += gridDim.x * 256LL) {
    const int u = a.order[i];
    const int rb = a.g.out_off[u], re = a.g.out_off[u + 1];
    if (re - rb > kBcSmall) continue;
    double s0 = 0.0, s1 = 0.0;
    int j = rb;
    for (; j + 1 < re; j += 2) {
      const int w0 = a.g.out_idx[j], w1 = a.g.out_idx[j + 1];
      s0 += bc_succ(a, w0, L);
      s1 += bc_succ(a, w1, L);
    }
    if (j < re) s0 += bc_succ(a, a.g.out_idx[j], L);
    bc_finish_vertex(a, u, s0 + s1);
  }
}


__global__ void k_bc_init(BcArgs a) {
  const int n = a.g.n;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
  for (int v = tid; v < n; v += nt) {
    const bool s = v == a.src;
    a.level[v] = s ? 0 : -1;
    a.sigma[v] = s ? 1.0 : 0.0;
    a.fs[v] = 0.0;
    a.delta[v] = 0.0;
  }
  if (tid == 0) {
    a.order[0] = a.src;
    a.bounds[0] = 0;
    a.ctl->bc_start = 0;
    a.ctl->bc_end = 1;
    a.ctl->bc_count = 1;
    a.ctl->mode = MODE_SPARSE_PUSH;
    a.ctl->dsum = a.g.outdeg[a.src];
    a.ctl->sa_slots = 0;
  }
}

// Control-block reset shared by the runs (one thread).
__global__ void k_ctl_init(Control* c, HostFlags* host, unsigned long long delta) {
  c->mode = MODE_NONE;
  c->done = 0;
  c->steps = 0;
  c->dense_steps = 0;
  c->nf = 0;
  c->dsum = 0;
  c->sa_count = 0;
  c->sa_slots = 0;
  c->nchunks = 0;
  c->chunk = kMinChunk;
  c->visited = 0;
  c->edges_examined = 0;
  c->thresh = delta;
  c->told = 0;
  c->far_count = 0;
  c->overflow = 0;
  c->buckets = 0;
  c->error = 0;
  c->host = host;
}

// ------------------------------------------------------- host launchers --

static int grid_for(long long items, int bt, int cap) {
  long long b = (items + bt - 1) / bt;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

#define GI_OK_LAUNCH() (hipGetLastError() == hipSuccess ? 0 : -1)

static ExpandArgs expand_args(const Engine& e, const int32_t* off) {
  ExpandArgs x;
  x.ids = e.ids;
  x.excl = e.excl;
  x.chunk_item = e.chunk_item;
  x.off = off;
  x.ctl = e.ctl;
  return x;
}

FrontierArgs frontier_args(const Engine& e, DenseSet cur, DenseSet next, const int32_t* deg,
                           const int32_t* fix_src, int32_t* fix_dst) {
  FrontierArgs a;
  a.cur = cur;
  a.next = next;
  a.n = e.n;
  a.tw = e.tw;
  a.cgrid = e.cgrid;
  a.deg = deg;
  a.fix_src = fix_src;
  a.fix_dst = fix_dst;
  a.blk = e.blk;
  a.ids = e.ids;
  a.excl = e.excl;
  a.chunk_item = e.chunk_item;
  a.chunk_cap = e.chunk_cap;
  a.ctl = e.ctl;
  return a;
}

int launch_ctl_init(Control* c, HostFlags* host, unsigned long long delta, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1), 0, s, c, host, delta);
  return GI_OK_LAUNCH();
}

int launch_bfs_init(const BfsArgs& b, int src, DenseSet f0, DenseSet f1, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(b.g.n, 256, 2048)), dim3(256), 0, s, b, src, f0, f1);
  return GI_OK_LAUNCH();
}

static void mark(const StepEvents* te, int which, hipStream_t s) {
  if (!te) return;
  (void)hipEventRecord(which == 0 ? te->start : which == 1 ? te->main : te->end, s);
}

int enqueue_bfs_step(const Engine& e, const FrontierArgs& f, const DecideArgs& d,
                     const BfsArgs& b, const StepEvents* te, hipStream_t s) {
  mark(te, 0, s);
  hipLaunchKernelGGL(k_count<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, f);
  hipLaunchKernelGGL(k_decide_frontier, dim3(1), dim3(1024), 0, s, f, d);
  hipLaunchKernelGGL((k_write<kBT, kCH>), dim3(e.cgrid), dim3(kBT), 0, s, f,
                     (int)MODE_SPARSE_PUSH);
  mark(te, 1, s);
  hipLaunchKernelGGL((k_bfs_step<kBT, kCH>), dim3(kParts), dim3(kBT), 0, s, b,
                     expand_args(e, b.g.out_off));
  mark(te, 2, s);
  return GI_OK_LAUNCH();
}

int launch_cc_init(const CcArgs& c, DenseSet f0, DenseSet f1, int32_t* lab_other, hipStream_t s) {
  hipLaunchKernelGGL(k_cc_init, dim3(grid_for(c.g.n, 256, 2048)), dim3(256), 0, s, c, f0, f1,
                     lab_other);
  return GI_OK_LAUNCH();
}

int launch_build_sym(const DevGraph& g, const int32_t* sym_off, int32_t* sym_idx, hipStream_t s) {
  hipLaunchKernelGGL(k_build_sym, dim3(grid_for((long long)g.n * 64, 256, 8192)), dim3(256), 0, s,
                     g, sym_off, sym_idx);
  return GI_OK_LAUNCH();
}

int enqueue_cc_step(const Engine& e, const FrontierArgs& f, const DecideArgs& d, const CcArgs& c,
                    const StepEvents* te, hipStream_t s) {
  mark(te, 0, s);
  hipLaunchKernelGGL(k_count<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, f);
  hipLaunchKernelGGL(k_decide_frontier, dim3(1), dim3(1024), 0, s, f, d);
  hipLaunchKernelGGL((k_write<kBT, kCH>), dim3(e.cgrid), dim3(kBT), 0, s, f,
                     (int)MODE_SPARSE_PUSH);
  mark(te, 1, s);
  hipLaunchKernelGGL((k_cc_step<kBT, kCH>), dim3(kParts), dim3(kBT), 0, s, c,
                     expand_args(e, c.sym_off));
  if (c.nseg > 1)
    hipLaunchKernelGGL(k_cc_seg_merge<256>,
                       dim3((unsigned)std::max(1, std::min(4096, ((c.g.n + 63) / 64 + 3) / 4))),
                       dim3(256), 0, s, c);
  mark(te, 2, s);
  return GI_OK_LAUNCH();
}

int launch_sssp_init(const SsspArgs& sa, int src, hipStream_t s) {
  hipLaunchKernelGGL(k_sssp_init, dim3(grid_for(sa.g.n, 256, 2048)), dim3(256), 0, s, sa, src);
  return GI_OK_LAUNCH();
}

int enqueue_sssp_step(const Engine& e, const FrontierArgs& f, const SsspArgs& sa,
                      const StepEvents* te, hipStream_t s) {
  mark(te, 0, s);
  hipLaunchKernelGGL(k_count<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, f);
  hipLaunchKernelGGL(k_decide_sssp, dim3(1), dim3(1024), 0, s, f, sa);
  hipLaunchKernelGGL((k_sssp_prepare<kBT, kCH>), dim3(e.cgrid), dim3(kBT), 0, s, f, sa);
  hipLaunchKernelGGL(k_sssp_threshold, dim3(1), dim3(1024), 0, s, sa, e.cgrid);
  mark(te, 1, s);
  hipLaunchKernelGGL((k_sssp_step<kBT, kCH>), dim3(kParts), dim3(kBT), 0, s, sa,
                     expand_args(e, sa.g.out_off));
  mark(te, 2, s);
  return GI_OK_LAUNCH();
}

static size_t prd_lds_bytes(int cap_e) {
  const size_t pull = sizeof(double) * (size_t)cap_e + sizeof(int) * (size_t)(std::min(cap_e, 1024) + 1);
  const size_t push = sizeof(int) * (size_t)expand_lds_ints<kCH>();
  return std::max(pull, push);
}

int launch_prd_init(const PrdArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_prd_init, dim3(grid_for(a.g.n, 256, 2048)), dim3(256), 0, s, a);
  return GI_OK_LAUNCH();
}

int enqueue_prd_step(const Engine& e, const FrontierArgs& f, const DecideArgs& d,
                     const PrdArgs& a, const StepEvents* te, hipStream_t s) {
  mark(te, 0, s);
  hipLaunchKernelGGL(k_count<kBT>, dim3(e.cgrid), dim3(kBT), 0, s, f);
  hipLaunchKernelGGL(k_decide_frontier, dim3(1), dim3(1024), 0, s, f, d);
  hipLaunchKernelGGL((k_write<kBT, kCH>), dim3(e.cgrid), dim3(kBT), 0, s, f,
                     (int)MODE_SPARSE_PUSH);
  mark(te, 1, s);
  hipLaunchKernelGGL((k_prd_step<kBT, kCH>), dim3(kParts), dim3(kBT), prd_lds_bytes(a.cap_e), s,
                     a, expand_args(e, a.g.out_off));
  hipLaunchKernelGGL(k_prd_update, dim3(grid_for((long long)((a.g.n + 63) / 64) * 64, 256, 2048)),
                     dim3(256), 0, s, a);
  mark(te, 2, s);
  return GI_OK_LAUNCH();
}

int launch_bc_init(const BcArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_bc_init, dim3(grid_for(a.g.n, 256, 2048)), dim3(256), 0, s, a);
  return GI_OK_LAUNCH();
}

int enqueue_bc_forward(const BcArgs& a, const StepEvents* te, hipStream_t s) {
  mark(te, 0, s);
  hipLaunchKernelGGL(k_bc_fs, dim3(512), dim3(256), 0, s, a, 0);
  mark(te, 1, s);
  hipLaunchKernelGGL(k_bc_forward<kBT>, dim3(kParts), dim3(kBT), 0, s, a);
  hipLaunchKernelGGL(k_bc_forward_pull<kBT>, dim3(kParts), dim3(kBT), 0, s, a);
  hipLaunchKernelGGL(k_bc_advance, dim3(1), dim3(1), 0, s, a);
  mark(te, 2, s);
  return GI_OK_LAUNCH();
}

int enqueue_bc_backward_level(const BcArgs& a, long long begin, long long end, int level,
                              hipStream_t s) {
  const long long items = end - begin;
  if (items <= 65536) {
    const int blocks = (int)std::max<long long>(1, std::min<long long>(8192, items));
    hipLaunchKernelGGL(k_bc_backward_wg<kBT>, dim3(blocks), dim3(kBT), 0, s, a, begin, end, level,
                       0);
  } else {
    const int tb = (int)std::min<long long>(4096, (items + 255) / 256);
    hipLaunchKernelGGL(k_bc_backward_thread, dim3(tb), dim3(256), 0, s, a, begin, end, level);
    hipLaunchKernelGGL(k_bc_backward_wave, dim3(4096), dim3(256), 0, s, a, begin, end, level);
    hipLaunchKernelGGL(k_bc_backward_wg<kBT>, dim3(2048), dim3(kBT), 0, s, a, begin, end, level,
                       kHubDeg + 1);
  }
  return GI_OK_LAUNCH();
}

}  // namespace gi
