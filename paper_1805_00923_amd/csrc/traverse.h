// Edge-traversal building blocks shared by the BFS, CC and SSSP kernels.
//
// The paper's edgeset.apply comes in three directions (section 2, direction
// optimization): SparsePush walks the out-edges of a sparse-array frontier
// with atomic updates, DensePush walks the out-edges of every vertex whose
// dense-frontier bit is set, DensePull walks the in-edges of every vertex
// and needs no atomics.
//
// Frontiers live as dense sets (bitvector or bool map, the two options of
// configApplyDenseVertexSet).  A SparsePush step first compacts the dense
// set into a sparse array with an exclusive scan of the members' degrees
// (three small kernels, no atomics), and then spreads the frontier's edges
// evenly over all workgroups: chunk c of CH consecutive edge slots starts in
// the frontier item recorded by the compaction (a merge-path split of the
// degree prefix sum), so a handful of hub vertices no longer lands on one
// workgroup.
#pragma once

#include "common.h"

namespace gi {

// Dense vertexset: bitvector (bit v%64 of word v/64) or bool map (byte v).
struct DenseSet {
  uint64_t* bv;
  uint8_t* bm;
  __device__ __forceinline__ bool test(int u) const {
    return bm ? bm[u] != 0 : ((bv[u >> 6] >> (u & 63)) & 1ull) != 0;
  }
  // 64-member mask of word w (members beyond n must be clear)
  __device__ __forceinline__ uint64_t word(int w) const {
    if (!bm) return bv[w];
    const uint64_t* p = reinterpret_cast<const uint64_t*>(bm + ((size_t)w << 6));
    uint64_t m = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t x = p[k];  // bytes are 0 or 1
#pragma unroll
      for (int b = 0; b < 8; ++b) m |= ((x >> (8 * b)) & 1ull) << (8 * k + b);
    }
    return m;
  }
  // set member v; true when it was not a member before
  __device__ __forceinline__ bool insert(int v) const {
    if (bm) {
      const unsigned sh = 8u * (unsigned)(v & 3);
      const unsigned old =
          atomicOr(reinterpret_cast<unsigned*>(bm + (v & ~3)), 1u << sh);
      return ((old >> sh) & 0xffu) == 0;
    }
    const unsigned long long bit = 1ull << (v & 63);
    return (atomicOr((unsigned long long*)&bv[v >> 6], bit) & bit) == 0;
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

// ------------------------------------------------------------ compaction --
//
// Workgroup b owns the words [b*tw, (b+1)*tw) of the dense set; thread t
// visits words b*tw + it*BT + t for it = 0, 1, ... so that the (it, t) order
// is the word order.  Members with degree 0 are left out of the sparse array
// (they own no edge slots).

struct CompactArgs {
  DenseSet in;
  int n;
  int tw;                      // words per workgroup
  const int32_t* deg;          // degree of each vertex
  long long* blk_cnt;          // per-workgroup item counts (pass 1)
  long long* blk_deg;          // per-workgroup degree sums (pass 1)
  int32_t* ids;                // sparse items (pass 3)
  long long* excl;             // exclusive degree prefix per item (pass 3)
  int32_t* chunk_item;         // first item of each chunk of `chunk` slots
  int chunk;
  long long chunk_cap;         // entries allocated for chunk_item
  DenseSet clear;              // dense set to clear (bitvector words), or none
  const int32_t* fix_src;      // optional: fix_dst[v] = fix_src[v] for members
  int32_t* fix_dst;
  Control* ctl;
  int active_mode;             // pass runs only when ctl->mode equals this
  int active_mode2;            // ... or this
};

__device__ __forceinline__ bool mode_on(const Control* ctl, int m1, int m2) {
  const int m = ctl->mode;
  return m == m1 || m == m2;
}

template <int BT>
__device__ __forceinline__ void word_stats(const CompactArgs& a, int w, long long& c,
                                           long long& d) {
  uint64_t x = a.in.word(w);
  while (x) {
    const int b = __ffsll((long long)x) - 1;
    x &= x - 1;
    const int v = (w << 6) + b;
    const int dv = a.deg[v];
    if (dv > 0) {
      c += 1;
      d += dv;
    }
  }
}

template <int BT>
__global__ __launch_bounds__(BT) void k_compact_count(CompactArgs a) {
  if (!mode_on(a.ctl, a.active_mode, a.active_mode2)) return;
  const int W = (a.n + 63) >> 6;
  const int w0 = blockIdx.x * a.tw, w1 = min(W, w0 + a.tw);
  long long c = 0, d = 0;
  for (int w = w0 + threadIdx.x; w < w1; w += BT) {
    if (a.clear.bv) a.clear.bv[w] = 0ull;
    if (a.clear.bm) {
      uint64_t* p = reinterpret_cast<uint64_t*>(a.clear.bm + ((size_t)w << 6));
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = 0ull;
    }
    if (a.fix_dst) {  // CC push: next labels start equal to the current ones on F
      uint64_t x = a.in.word(w);
      while (x) {
        const int v = (w << 6) + __ffsll((long long)x) - 1;
        x &= x - 1;
        a.fix_dst[v] = a.fix_src[v];
      }
    }
    if (a.blk_cnt) word_stats<BT>(a, w, c, d);
  }
  if (!a.blk_cnt) return;
  Part p{c, d, 0, 0};
  p = block_sum4<BT>(p);
  if (threadIdx.x == 0) {
    a.blk_cnt[blockIdx.x] = p.a;
    a.blk_deg[blockIdx.x] = p.b;
  }
}

// Exclusive scan of the per-workgroup counts by one workgroup of 1024.
static __global__ __launch_bounds__(1024) void k_compact_scan(CompactArgs a, int nblk) {
  if (!mode_on(a.ctl, a.active_mode, a.active_mode2)) return;
  __shared__ long long sc[1024], sd[1024];
  const int t = threadIdx.x;
  const int per = (nblk + 1023) / 1024;
  const int b = t * per, e = min(nblk, b + per);
  long long c = 0, d = 0;
  for (int i = b; i < e; ++i) {
    c += a.blk_cnt[i];
    d += a.blk_deg[i];
  }
  sc[t] = c;
  sd[t] = d;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long yc = t >= o ? sc[t - o] : 0, yd = t >= o ? sd[t - o] : 0;
    __syncthreads();
    sc[t] += yc;
    sd[t] += yd;
    __syncthreads();
  }
  long long rc = sc[t] - c, rd = sd[t] - d;
  for (int i = b; i < e; ++i) {
    const long long ci = a.blk_cnt[i], di = a.blk_deg[i];
    a.blk_cnt[i] = rc;
    a.blk_deg[i] = rd;
    rc += ci;
    rd += di;
  }
  if (t == 1023) {
    const long long items = sc[1023], slots = sd[1023];
    const long long nch = (slots + a.chunk - 1) / a.chunk;
    if (items < 0 || items > a.n || nch + 1 > a.chunk_cap) {
      // cannot happen for a consistent dense set; refuse rather than write
      a.ctl->error = 1;
      a.ctl->done = 1;
      a.ctl->mode = MODE_NONE;
      a.ctl->sa_count = 0;
      a.ctl->sa_slots = 0;
      a.ctl->nchunks = 0;
      return;
    }
    a.ctl->sa_count = items;
    a.ctl->sa_slots = slots;
    a.ctl->nchunks = nch;
    a.chunk_item[nch] = (int)items;  // sentinel
  }
}

template <int BT>
__global__ __launch_bounds__(BT) void k_compact_write(CompactArgs a) {
  if (!mode_on(a.ctl, a.active_mode, a.active_mode2) || a.ctl->error) return;
  const int W = (a.n + 63) >> 6;
  const int w0 = blockIdx.x * a.tw, w1 = min(W, w0 + a.tw);
  long long run_c = a.blk_cnt[blockIdx.x], run_d = a.blk_deg[blockIdx.x];
  for (int base = w0; base < w1; base += BT) {
    const int w = base + threadIdx.x;
    long long c = 0, d = 0;
    if (w < w1) word_stats<BT>(a, w, c, d);
    long long tc, td;
    long long pc = block_excl_scan<BT>(c, &tc) + run_c;
    long long pd = block_excl_scan<BT>(d, &td) + run_d;
    if (w < w1) {
      uint64_t x = a.in.word(w);
      while (x) {
        const int b = __ffsll((long long)x) - 1;
        x &= x - 1;
        const int v = (w << 6) + b;
        const int dv = a.deg[v];
        if (dv <= 0) continue;
        a.ids[pc] = v;
        a.excl[pc] = pd;
        // chunks whose first slot falls in [pd, pd + dv) start at this item
        long long c0 = (pd + a.chunk - 1) / a.chunk;
        for (long long k = c0; k * a.chunk < pd + dv; ++k) a.chunk_item[k] = (int)pc;
        ++pc;
        pd += dv;
      }
    }
    run_c += tc;
    run_d += td;
  }
}

// ------------------------------------------------ edge-balanced expansion --
//
// Slots [c*CH, (c+1)*CH) of the frontier's edges belong to chunk c; its items
// are [chunk_item[c], chunk_item[c+1]] (each item owns >= 1 slot, so at most
// CH+1 items).  The items' (vertex, first slot, row start) are staged in LDS,
// then each thread binary-searches its slots.  vis(u, e, valid) is called by
// full waves.

struct ExpandArgs {
  const int32_t* ids;
  const long long* excl;
  const int32_t* chunk_item;
  const int32_t* off;     // row offsets of the adjacency being expanded
  const int32_t* off2;    // CC: second adjacency (slots beyond outdeg)
  const int32_t* deg1;    // CC: degree in the first adjacency
  Control* ctl;
  int active_mode;
};

template <int BT, int CH, class Visit>
__device__ void expand_chunks(const ExpandArgs& a, Visit& vis) {
  __shared__ int s_u[CH + 1];
  __shared__ int s_start[CH + 1];  // first slot of the item, relative to the chunk
  __shared__ int s_row[CH + 1];
  __shared__ int s_n;
  const long long nch = a.ctl->nchunks;
  const long long slots = a.ctl->sa_slots;
  for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
    const long long s0 = c * CH;
    const int s_end = (int)min((long long)CH, slots - s0);
    const int i0 = a.chunk_item[c];
    const int i1 = min(a.chunk_item[c + 1], (int)a.ctl->sa_count - 1);
    const int ni = i1 - i0 + 1;
    for (int k = threadIdx.x; k < ni; k += BT) {
      const int u = a.ids[i0 + k];
      s_u[k] = u;
      s_start[k] = (int)(a.excl[i0 + k] - s0);
      s_row[k] = a.off[u];
    }
    if (threadIdx.x == 0) s_n = ni;
    __syncthreads();
    const int nitems = s_n;
    for (int r = 0; r < s_end; r += BT) {
      const int j = r + threadIdx.x;  // slot within the chunk
      int lo = 0, hi = nitems - 1;      // last item with start <= j
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      const bool valid = j < s_end;
      const int u = s_u[lo];
      int k = j - s_start[lo];
      int e;
      if (a.off2) {  // undirected view: out-edges first, then in-edges
        const int d1 = a.deg1[u];
        e = k < d1 ? s_row[lo] + k : a.off2[u] + (k - d1);
        vis(u, e, valid, k < d1);
      } else {
        e = s_row[lo] + k;
        vis(u, e, valid, true);
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- dense push ----
//
// Every vertex whose bit is set expands its out-edges; rows with >= BT edges
// are walked by the whole workgroup, rows with >= 64 edges by one wave, and
// the remaining short rows of a wave are gathered with a wave prefix sum so
// that 64 consecutive lanes take 64 consecutive edge slots.

template <int BT, class Visit>
__device__ void dense_push_expand(const DenseSet& fr, int n, const int32_t* off, Visit& vis,
                                  bool first_adj) {
  __shared__ int sh_owner, sh_u, sh_b, sh_e;
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  for (int base = blockIdx.x * BT; base < n; base += gridDim.x * BT) {
    const int i = base + tid;
    int u = -1, beg = 0, end = 0;
    if (i < n && fr.test(i)) {
      u = i;
      beg = off[i];
      end = off[i + 1];
    }
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
        vis(cu, e, e < ce, first_adj);
      }
      __syncthreads();
    }
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
        vis(cu, e, e < ce, first_adj);
      }
    }
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
      vis(cu, cb + (j - ex), j < total, first_adj);
    }
  }
}

}  // namespace gi
