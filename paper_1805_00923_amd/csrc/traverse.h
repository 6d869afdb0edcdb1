// Edge-traversal building blocks shared by the BFS, CC and SSSP kernels.
//
// The paper's edgeset.apply comes in three directions (section 2, direction
// optimization): SparsePush walks the out-edges of a sparse-array frontier
// with atomic updates, DensePush walks the out-edges of every vertex whose
// dense-frontier bit is set, DensePull walks the in-edges of every vertex
// and needs no atomics.
//
// Frontiers live as dense sets (bitvector or bool map, the two options of
// configApplyDenseVertexSet).  Each step runs four launches:
//   count  - every workgroup counts the frontier members of its word range
//            (|F|, sum of degrees, and the members that own edges), clears
//            the next frontier and, for CC, copies the current labels of F
//            into the next-label buffer;
//   decide - one workgroup reduces those counts, picks the direction, and
//            for SparsePush turns the counts into exclusive offsets;
//   write  - SparsePush only: the members with edges are written as a sparse
//            array with an exclusive prefix sum of their degrees, and chunk c
//            of CH consecutive edge slots records the item it starts in (a
//            merge-path split of the prefix sum);
//   step   - the edgeset.apply itself in the chosen direction.  SparsePush
//            spreads the frontier's edges evenly over all workgroups, so a
//            few hub vertices do not serialize on one workgroup.
#pragma once

#include "common.h"

namespace gi {

// Dense vertexset: bitvector (bit v%64 of word v/64) or bool map (byte v,
// padded to whole 64-byte words).
struct DenseSet {
  uint64_t* bv;
  uint8_t* bm;
  __device__ __forceinline__ bool test(int u) const {
    return bm ? bm[u] != 0 : ((bv[u >> 6] >> (u & 63)) & 1ull) != 0;
  }
  // 64-member mask of word w (members beyond n are clear)
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
  __device__ __forceinline__ void clear_word(int w) const {
    if (bv) bv[w] = 0ull;
    if (bm) {
      uint64_t* p = reinterpret_cast<uint64_t*>(bm + ((size_t)w << 6));
#pragma unroll
      for (int k = 0; k < 8; ++k) p[k] = 0ull;
    }
  }
  // set member v; true when it was not a member before
  __device__ __forceinline__ bool insert(int v) const {
    if (bm) {
      const unsigned sh = 8u * (unsigned)(v & 3);
      const unsigned old = atomicOr(reinterpret_cast<unsigned*>(bm + (v & ~3)), 1u << sh);
      return ((old >> sh) & 0xffu) == 0;
    }
    const unsigned long long bit = 1ull << (v & 63);
    return (atomicOr((unsigned long long*)&bv[v >> 6], bit) & bit) == 0;
  }
};

// Per-workgroup counts of the count pass.
struct Blk {
  long long items;    // members with degree > 0 (sparse items)
  long long slots;    // their degree sum (edge slots)
  long long members;  // all members (|F|)
  long long degsum;   // degree sum of all members
};

struct FrontierArgs {
  DenseSet cur;                // frontier of the step
  DenseSet next;               // frontier the step produces (cleared by count)
  int n;
  int tw;                      // words per count/write workgroup
  int cgrid;                   // count/write workgroups
  const int32_t* deg;          // degree of each vertex (edge slots it owns)
  const int32_t* fix_src;      // CC: fix_dst[v] = fix_src[v] for members of cur
  int32_t* fix_dst;
  Blk* blk;                    // [cgrid]
  int32_t* ids;                // sparse items
  long long* excl;             // exclusive degree prefix per item
  int32_t* chunk_item;         // first item of each chunk of CH slots
  long long chunk_cap;         // entries allocated for chunk_item
  Control* ctl;
};

template <int BT>
__global__ __launch_bounds__(BT) void k_count(FrontierArgs a) {
  if (a.ctl->done) return;
  const int W = (a.n + 63) >> 6;
  const int w0 = blockIdx.x * a.tw, w1 = min(W, w0 + a.tw);
  long long items = 0, slots = 0, members = 0, degsum = 0;
  for (int w = w0 + (int)threadIdx.x; w < w1; w += BT) {
    a.next.clear_word(w);
    uint64_t x = a.cur.word(w);
    while (x) {
      const int v = (w << 6) + __ffsll((long long)x) - 1;
      x &= x - 1;
      if (a.fix_dst) a.fix_dst[v] = a.fix_src[v];
      const int d = a.deg[v];
      ++members;
      degsum += d;
      if (d > 0) {
        ++items;
        slots += d;
      }
    }
  }
  Part p = block_sum4<BT>(Part{items, slots, members, degsum});
  if (threadIdx.x == 0) a.blk[blockIdx.x] = Blk{p.a, p.b, p.c, p.d};
}

// Sum of the count pass (one workgroup of 1024 threads).
__device__ __forceinline__ Blk reduce_blk(const FrontierArgs& a) {
  __shared__ long long s[4][1024];
  const int t = threadIdx.x;
  long long x0 = 0, x1 = 0, x2 = 0, x3 = 0;
  for (int i = t; i < a.cgrid; i += 1024) {
    const Blk b = a.blk[i];
    x0 += b.items;
    x1 += b.slots;
    x2 += b.members;
    x3 += b.degsum;
  }
  s[0][t] = x0;
  s[1][t] = x1;
  s[2][t] = x2;
  s[3][t] = x3;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) {
      s[0][t] += s[0][t + o];
      s[1][t] += s[1][t + o];
      s[2][t] += s[2][t + o];
      s[3][t] += s[3][t + o];
    }
    __syncthreads();
  }
  const Blk tot{s[0][0], s[1][0], s[2][0], s[3][0]};
  __syncthreads();
  return tot;
}

// Sum of one field over the kParts step-kernel slots (one workgroup of 1024).
__device__ __forceinline__ long long reduce_parts(const Part* part, int field) {
  __shared__ long long s[1024];
  const int t = threadIdx.x;
  long long x = 0;
  for (int i = t; i < kParts; i += 1024) {
    const Part p = part[i];
    x += field == 0 ? p.a : field == 1 ? p.b : field == 2 ? p.c : p.d;
  }
  s[t] = x;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) s[t] += s[t + o];
    __syncthreads();
  }
  const long long r = s[0];
  __syncthreads();
  return r;
}

// Turn the per-workgroup item and slot counts into exclusive offsets and
// publish the expansion shape (one workgroup of 1024, all threads call it).
// Returns false when the sizes break an invariant; the caller then abandons
// the run instead of writing past the arrays.
template <int CH>
__device__ bool scan_blk(const FrontierArgs& a, const Blk& tot) {
  __shared__ long long sc[1024], sd[1024];
  // chunk size: the smallest power of two in [kMinChunk, CH] that needs at
  // most kParts chunks, so that a small step still spreads over the grid
  // with one or two slots per thread
  int cs = kMinChunk;
  while (cs < CH && (long long)cs * kParts < tot.slots) cs <<= 1;
  const long long nch = (tot.slots + cs - 1) / cs;
  if (tot.items < 0 || tot.items > a.n || nch + 1 > a.chunk_cap) return false;
  const int t = threadIdx.x;
  const int per = (a.cgrid + 1023) / 1024;
  const int b = t * per, e = min(a.cgrid, b + per);
  long long c = 0, d = 0;
  for (int i = b; i < e; ++i) {
    c += a.blk[i].items;
    d += a.blk[i].slots;
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
    const long long ci = a.blk[i].items, di = a.blk[i].slots;
    a.blk[i].items = rc;
    a.blk[i].slots = rd;
    rc += ci;
    rd += di;
  }
  if (t == 0) {
    a.ctl->sa_count = tot.items;
    a.ctl->sa_slots = tot.slots;
    a.ctl->nchunks = nch;
    a.ctl->chunk = cs;
    a.chunk_item[nch] = (int)tot.items;  // sentinel
  }
  return true;
}

// Sparse array of the members with edges (after scan_blk turned the counts
// into offsets).  Word order within a workgroup follows (iteration, thread).
template <int BT, int CH>
__device__ void write_body(const FrontierArgs& a) {
  const int W = (a.n + 63) >> 6;
  const int w0 = blockIdx.x * a.tw, w1 = min(W, w0 + a.tw);
  const long long cs = a.ctl->chunk;
  long long run_c = a.blk[blockIdx.x].items, run_d = a.blk[blockIdx.x].slots;
  for (int base = w0; base < w1; base += BT) {
    const int w = base + (int)threadIdx.x;
    uint64_t x = w < w1 ? a.cur.word(w) : 0ull;
    long long c = 0, d = 0;
    for (uint64_t y = x; y;) {
      const int v = (w << 6) + __ffsll((long long)y) - 1;
      y &= y - 1;
      const int dv = a.deg[v];
      if (dv > 0) {
        ++c;
        d += dv;
      }
    }
    long long tc, td;
    long long pc = block_excl_scan<BT>(c, &tc) + run_c;
    long long pd = block_excl_scan<BT>(d, &td) + run_d;
    while (x) {
      const int v = (w << 6) + __ffsll((long long)x) - 1;
      x &= x - 1;
      const int dv = a.deg[v];
      if (dv <= 0) continue;
      a.ids[pc] = v;
      a.excl[pc] = pd;
      // chunks whose first slot falls in [pd, pd + dv) start at this item
      for (long long k = (pd + cs - 1) / cs; k * cs < pd + dv; ++k) a.chunk_item[k] = (int)pc;
      ++pc;
      pd += dv;
    }
    run_c += tc;
    run_d += td;
  }
}

template <int BT, int CH>
__global__ __launch_bounds__(BT) void k_write(FrontierArgs a, int active_mode) {
  if (a.ctl->mode != active_mode) return;
  write_body<BT, CH>(a);
}

// ------------------------------------------------ edge-balanced expansion --
//
// Slots [c*cs, (c+1)*cs) of the frontier's edges belong to chunk c, where
// the chunk size cs <= CH was chosen by the scan; its items are
// [chunk_item[c], chunk_item[c+1]] (each item owns >= 1 slot, so at most
// cs+1 items).  The items' (vertex, first slot, row start) are staged in LDS,
// then each thread binary-searches its slots.  vis(u, e, valid) is called by
// whole workgroups; `valid` is false for padding lanes.

struct ExpandArgs {
  const int32_t* ids;
  const long long* excl;
  const int32_t* chunk_item;
  const int32_t* off;     // row offsets of the adjacency being expanded; NULL:
                          // vis(u, j) gets the slot j within u's row instead
  Control* ctl;
};

// LDS the expansion needs (ints); a step kernel may reuse it for other modes.
template <int CH>
constexpr int expand_lds_ints() { return 3 * (CH + 1); }

template <int BT, int CH, class Visit>
__device__ void expand_chunks(const ExpandArgs& a, Visit& vis, int* lds) {
  int* s_u = lds;
  int* s_start = lds + (CH + 1);  // first slot of the item, relative to the chunk
  int* s_row = lds + 2 * (CH + 1);
  const long long nch = a.ctl->nchunks;
  const long long slots = a.ctl->sa_slots;
  const long long cs = a.ctl->chunk;
  const int last = (int)a.ctl->sa_count - 1;
  for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
    const long long s0 = c * cs;
    const int s_end = (int)min(cs, slots - s0);
    const int i0 = a.chunk_item[c];
    const int ni = min(a.chunk_item[c + 1], last) - i0 + 1;
    for (int k = threadIdx.x; k < ni; k += BT) {
      const int u = a.ids[i0 + k];
      s_u[k] = u;
      s_start[k] = (int)(a.excl[i0 + k] - s0);
      s_row[k] = a.off ? a.off[u] : 0;  // NULL off: visitors get the slot within the row
    }
    __syncthreads();
    for (int r = 0; r < s_end; r += BT) {
      const int j = r + (int)threadIdx.x;  // slot within the chunk
      int lo = 0, hi = ni - 1;             // last item with start <= j
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_start[mid] <= j) lo = mid;
        else hi = mid - 1;
      }
      vis(s_u[lo], s_row[lo] + (j - s_start[lo]), j < s_end);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------- dense push ----
//
// Every vertex whose bit is set expands its row; rows with >= BT edges are
// walked by the whole workgroup, rows with >= 64 edges by one wave, and the
// remaining short rows of a wave are gathered with a wave prefix sum so that
// 64 consecutive lanes take 64 consecutive edge slots.

// Expansion of the rows of one group of BT vertices (u = -1 for lanes
// without a row): rows with >= BT edges by the whole workgroup, rows with
// >= 64 edges by one wave, the remaining short rows of a wave with a wave
// prefix sum.  Every thread of the workgroup must call it.
template <int BT, class Visit>
__device__ __forceinline__ void push_rows(int u, int beg, int end, Visit& vis, int* sh) {
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  while (__syncthreads_or(end - beg >= BT)) {
    if (end - beg >= BT) sh[0] = tid;
    __syncthreads();
    if (tid == sh[0]) {
      sh[1] = u;
      sh[2] = beg;
      sh[3] = end;
      beg = end;
    }
    __syncthreads();
    const int cu = sh[1], cb = sh[2], ce = sh[3];
    for (int k = cb; k < ce; k += BT) {
      const int e = k + tid;
      vis(cu, e, e < ce);
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
      vis(cu, e, e < ce);
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
    vis(cu, cb + (j - ex), j < total);
  }
}

// Vertices [vb, ve) are taken BT at a time by workgroups first_block,
// first_block + nblocks, ...
template <int BT, class Visit>
__device__ void dense_push_range(const DenseSet& fr, int vb, int ve, int first_block, int nblocks,
                                 const int32_t* off, Visit& vis) {
  __shared__ int sh[4];
  const int tid = threadIdx.x;
  for (int base = vb + first_block * BT; base < ve; base += nblocks * BT) {
    const int i = base + tid;
    int u = -1, beg = 0, end = 0;
    if (i < ve && fr.test(i)) {
      u = i;
      beg = off[i];
      end = off[i + 1];
    }
    push_rows<BT>(u, beg, end, vis, sh);
  }
}

// One workgroup over the words [wb, we) of a sparse bitvector frontier.
// Words are read kPushGroup * BT at a time (kPushGroup independent loads in
// flight per thread); a workgroup prefix sum of their popcounts gives each
// member a slot in an LDS list, and the list is expanded BT members per
// group, so one dependent chain (word, list, row bounds, edges) serves the
// whole group and sparse words leave no lanes idle.  Groups with more than
// kList members are listed and expanded in passes of kList.  s_v: LDS for
// kPushList ints, supplied by the caller.
constexpr int kPushList = 4096;
constexpr int kPushGroup = 4;

template <int BT, class Visit>
__device__ void push_words(const uint64_t* bv, int wb, int we, int n, const int32_t* off,
                           Visit& vis, int skip_deg, int* s_v) {
  constexpr int kList = kPushList;
  constexpr int G = kPushGroup;
  __shared__ int sh[4];
  const int tid = threadIdx.x;
  for (int grp = wb; grp < we; grp += G * BT) {
    uint64_t x[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int w = grp + q * BT + tid;
      x[q] = w < we ? bv[w] : 0ull;
    }
    int own = 0;
#pragma unroll
    for (int q = 0; q < G; ++q) own += __popcll(x[q]);
    int total;
    const int first = block_excl_scan<BT, int>(own, &total);  // total: workgroup-uniform
    for (int base = 0; base < total; base += kList) {
      // this thread's members with list index in [base, base + kList)
      int j = first;
#pragma unroll
      for (int q = 0; q < G; ++q) {
        uint64_t y = x[q];
        const int w = grp + q * BT + tid;
        for (; y; ++j) {
          const int b = __ffsll((long long)y) - 1;
          y &= y - 1;
          if (j >= base && j < base + kList) s_v[j - base] = (w << 6) + b;
        }
      }
      __syncthreads();
      const int cnt = min(kList, total - base);
      for (int g = 0; g < cnt; g += BT) {
        int u = -1, beg = 0, end = 0;
        if (g + tid < cnt) {
          u = s_v[g + tid];
          if (u < n) {
            beg = off[u];
            end = off[u + 1];
            if (end - beg > skip_deg) end = beg;  // pushed elsewhere
          }
        }
        push_rows<BT>(u, beg, end, vis, sh);
      }
      __syncthreads();
    }
  }
}

// The rows of the listed vertices ids[begin, end), BT per group, groups
// dealt to workgroups first_block, first_block + nblocks, ...
template <int BT, class Visit>
__device__ void push_list_range(const int32_t* ids, long long begin, long long end,
                                int first_block, int nblocks, const int32_t* off, Visit& vis) {
  __shared__ int sh[4];
  for (long long base = begin + (long long)first_block * BT; base < end;
       base += (long long)nblocks * BT) {
    const long long i = base + threadIdx.x;
    int u = -1, beg = 0, fin = 0;
    if (i < end) {
      u = ids[i];
      beg = off[u];
      fin = off[u + 1];
    }
    push_rows<BT>(u, beg, fin, vis, sh);
  }
}

// The same with the groups dealt over the grid.
template <int BT, class Visit>
__device__ void push_list(const int32_t* ids, long long begin, long long end, const int32_t* off,
                          Visit& vis) {
  push_list_range<BT>(ids, begin, end, blockIdx.x, gridDim.x, off, vis);
}

template <int BT, class Visit>
__device__ void dense_push_expand(const DenseSet& fr, int n, const int32_t* off, Visit& vis) {
  dense_push_range<BT>(fr, 0, n, blockIdx.x, gridDim.x, off, vis);
}

// --------------------------------------------------- row-block gathers ----
//
// A destination block is a run of consecutive rows holding at most cap_e
// edges (or one longer row).  gather_block stages f(idx[e]) for the block's
// edges in LDS with four independent index loads and four independent
// gathers in flight per thread, so a workgroup keeps many requests
// outstanding instead of one dependent chain.

template <int BT, typename T, class F>
__device__ __forceinline__ void gather_block(const int32_t* __restrict__ idx, int e0, int ne,
                                             T* lds, F f) {
  int j = threadIdx.x;
  for (; j + 3 * BT < ne; j += 4 * BT) {
    const int a0 = idx[e0 + j], a1 = idx[e0 + j + BT], a2 = idx[e0 + j + 2 * BT],
              a3 = idx[e0 + j + 3 * BT];
    const T v0 = f(a0), v1 = f(a1), v2 = f(a2), v3 = f(a3);
    lds[j] = v0;
    lds[j + BT] = v1;
    lds[j + 2 * BT] = v2;
    lds[j + 3 * BT] = v3;
  }
  for (; j < ne; j += BT) lds[j] = f(idx[e0 + j]);
}

}  // namespace gi
