// PageRank by DensePull over a degree-ordered copy of the in-adjacency.
//
// Method (section 2, DensePull figure; evaluation: 20 iterations, damping
// 0.85): x_{k+1}[v] = (1-alpha)/n + alpha * sum_{u->v} x_k[u] / outdeg(u),
// contributions stored as FP32 and sums accumulated in FP64, as in
// pagerank.hip.  What differs is the layout and the work split.
//
// Layout.  Vertices are renumbered by decreasing out-degree (ties by id), the
// in-rows are rebuilt under the new numbers and sorted.  A source's id then
// says how often it is gathered: on a power-law graph the first few ten
// thousand ids carry half of all in-edges, the first million nearly all.
// This is the paper's cache partitioning idea (keep the gathered source data
// in the fastest memory that holds it) taken one level further: instead of
// cutting sources into id ranges and sweeping the edges once per range, the
// hottest sources [0, hot) are copied into LDS by every workgroup at the
// start of an iteration and the rest are gathered from global memory, where
// the next million sit in L2.  One sweep, no partial-sum arrays.
//
// Work split (merge path).  The n row ends and m edges of the in-adjacency
// form one sequence of n + m items (the edges of row r, then the end of row
// r).  Tile t holds items [t T, (t+1) T) with T = 64 x items per thread and
// is worked by one wave on its own (no workgroup barrier after the hot
// sources are loaded); its start (row, edge) comes from a host-built table.
// Each lane takes items_per_thread consecutive items, found by a binary
// search of the tile's row offsets staged in the wave's LDS, so every lane
// gets the same amount of
// work however skewed the rows are, and empty rows cost one item.  A thread
// loads all its edges' source ids and contributions first (that many
// independent loads in flight), then walks its items in order, finishing
// each row that starts and ends inside it.  A row that runs across lanes
// is summed by a segmented scan of the lanes' open partial sums; a row
// that runs across tiles adds each tile's part into an FP64 slot, and a
// small kernel after the pass finishes those rows.
//
// The last iteration writes ranks under the caller's vertex numbers
// (rank[old_id[row]]).
#include "kernels.h"

namespace gi {

// Vertex update of row r from its full in-sum.
__device__ __forceinline__ void pr_ord_finish(const PrOrdArgs& a, int r, double s, float* cout,
                                              float* rank) {
  const double x = a.base + a.alpha * s;
  if (rank) {
    rank[a.old_id[r]] = (float)x;
  } else {
    const int d = a.outdeg[r];
    cout[r] = d > 0 ? (float)(x / (double)d) : 0.0f;
  }
}

// One tile's part of a row split over tiles.  Parts meet by atomic add in
// an FP64 slot and k_pr_ord_split finishes the row after the pass: a
// last-arriver scheme would need release and acquire fences, which on this
// chip write back and invalidate the L2 at every tile.
__device__ __forceinline__ void pr_ord_part(const PrOrdArgs& a, int slot, double part) {
  atomicAdd(&a.sacc[slot], part);
}

// LDS written by some lanes of a wave and read by others: LDS operations
// of one wave complete in order, so waiting for the wave's own LDS counter
// and keeping the compiler from moving memory operations across is enough.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// A tile's inputs as one wave holds them in registers: its split slots, and
// lane l keeps the tile's row offsets, row values (out-degree, or caller id
// when the ranks are written) and source ids at positions l, l + 64,
// l + 128, ...  All of them are loads that depend only on the tile table.
template <int U>
struct TileRegs {
  int r0, e0, r1, e1;
  int2 slot;  // split slots of the first and last row
  int off[U + 1];
  int row[U];
  int idx[U];
};

// Every load is issued whatever the tile's shape (addresses past the tile
// are clamped to valid ones and the values ignored), so the number of loads
// in flight after any of them is fixed and the compiler can wait for one
// without draining the rest.  A tile's first row is below n (every row end
// before it lies before the tile's start).
template <int U>
__device__ __forceinline__ void tile_head(const PrOrdArgs& a, int t, TileRegs<U>& R) {
  const int2 ts = a.tiles[t], te = a.tiles[t + 1];
  R.slot = a.tslot[t];
  R.r0 = ts.x;
  R.e0 = ts.y;
  R.r1 = te.x;
  R.e1 = te.y;
}

template <int U>
__device__ __forceinline__ void tile_body(const PrOrdArgs& a, const int32_t* rowsrc, int lane,
                                          TileRegs<U>& R) {
  const int mlast = a.m > 0 ? a.m - 1 : 0;
#pragma unroll
  for (int q = 0; q <= U; ++q) R.off[q] = a.off[min(R.r0 + q * kWave + lane, R.r1)];
#pragma unroll
  for (int q = 0; q < U; ++q) {
    R.row[q] = rowsrc[min(R.r0 + q * kWave + lane, a.n - 1)];
    R.idx[q] = a.idx[min(R.e0 + q * kWave + lane, mlast)];
  }
}

template <int BT, int U>
__global__ __launch_bounds__(BT) void k_pr_ord(PrOrdArgs a, const float* __restrict__ cin,
                                               float* __restrict__ cout, float* __restrict__ rank) {
  constexpr int TW = kWave * U;  // items per tile (one tile per wave at a time)
  constexpr int NW = BT / kWave;
  // LDS: a.hot floats, then per wave the tile's row offsets (TW + 1), its
  // gathered contributions (TW; reused for the finished rows' results) and
  // the finished rows' FP64 in-sums (TW)
  extern __shared__ float lds_hot[];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  int* offs = reinterpret_cast<int*>(lds_hot + a.hot) + wv * (4 * TW + 2);
  float* vals = reinterpret_cast<float*>(offs + TW + 2);  // 8-byte aligned after
  double* sums = reinterpret_cast<double*>(vals + TW);
  const int32_t* rowsrc = rank ? a.old_id : a.outdeg;

  // the hot sources' contributions, once per workgroup and iteration
  {
    const float4* src4 = reinterpret_cast<const float4*>(cin);
    float4* dst4 = reinterpret_cast<float4*>(lds_hot);
    for (int i = threadIdx.x; i < (a.hot >> 2); i += BT) dst4[i] = src4[i];
  }
  __syncthreads();

  const int stride = gridDim.x * NW;
  int t = blockIdx.x * NW + wv;
  if (t >= a.ntiles) return;
  TileRegs<U> cur;
  tile_head<U>(a, t, cur);
  tile_body<U>(a, rowsrc, lane, cur);
  // results of the previous tile, stored at the start of the next iteration
  // (before its gathers, so they never hold back the loads in flight)
  int p_r0 = 0, p_nr = 0, p_skip = -1;
  int p_row[U];
#pragma unroll
  for (int q = 0; q < U; ++q) p_row[q] = 0;
  for (;;) {
    // the next tile (this one again after the last: its loads are issued
    // and ignored, keeping the count of loads in flight fixed); its table
    // entry goes out before this tile's gathers
    const int tn = t + stride;
    TileRegs<U> nxt;
    tile_head<U>(a, tn < a.ntiles ? tn : t, nxt);

    // the previous tile's finished rows (results wait in vals)
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int kk = q * kWave + lane;
      if (q * kWave < p_nr && kk < p_nr && kk != p_skip) {
        if (rank) rank[p_row[q]] = vals[kk];
        else cout[p_r0 + kk] = vals[kk];
      }
    }

    const int r0 = cur.r0, e0 = cur.e0, r1 = cur.r1, e1 = cur.e1;
    const int nr = r1 - r0, ne = e1 - e0;
    // this tile's contributions, edge by edge in coalesced order.  Every
    // lane issues every gather (lanes without a cold source read entry 0),
    // so the count of loads in flight stays fixed; global gathers and LDS
    // reads land in different registers, so the LDS reads do not wait.
    float vg[U], vh[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int k = q * kWave + lane;
      const int uq = cur.idx[q];
      vg[q] = cin[k < ne && uq >= a.hot ? uq : 0];
      vh[q] = lds_hot[k < ne && uq < a.hot ? uq : 0];
    }
    // the next tile's inputs, in flight while this one is reduced
    tile_body<U>(a, rowsrc, lane, nxt);

    wave_lds_sync();  // the previous tile's LDS reads are done
#pragma unroll
    for (int q = 0; q <= U; ++q) {
      const int k = q * kWave + lane;
      if (k <= nr) offs[k] = cur.off[q] - e0;  // offsets relative to the tile's first edge
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int k = q * kWave + lane;
      vals[k] = k >= ne ? 0.0f : (cur.idx[q] < a.hot ? vh[q] : vg[q]);
    }
    wave_lds_sync();

    // this lane's items [ds, ds + steps) of the tile, ds relative to its
    // first item: ks row ends and js edges precede it
    const int ds = min(lane * U, nr + ne);
    const int steps = min(U, nr + ne - ds);
    int lo = 0, hi = nr;  // first k whose row end (item offs[k + 1] + k) is at or after ds
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (offs[mid + 1] + mid < ds) lo = mid + 1;
      else hi = mid;
    }
    const int ks = lo;
    const bool ks_open = offs[ks] < ds - ks;  // the first row began before this lane

    // merge walk: each step takes the next edge of row k or ends row k
    double s = 0.0, first = 0.0;
    bool has_first = false;
    int k = ks, j = ds - ks;
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (q < steps) {
        const int oe = k < nr ? offs[k + 1] : 0x7fffffff;
        if (j < oe) {
          s += (double)vals[j];
          ++j;
        } else {
          if (k == ks && ks_open) {
            first = s;
            has_first = true;
          } else {
            sums[k] = s;
          }
          s = 0.0;
          ++k;
        }
      }
    }

    // segmented inclusive scan of the lanes' open partials (key: the open
    // row; keys never decrease along the wave)
    const int key = k;
    double vs = s;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const double vv = __shfl_up(vs, o);
      const int kk = __shfl_up(key, o);
      if (lane >= o && kk == key) vs += vv;
    }
    const double vprev = __shfl_up(vs, 1);
    const int kprev = __shfl_up(key, 1);
    const int kskip = offs[0] < 0 ? 0 : -1;  // the first row began in an earlier tile
    if (has_first) {
      const double tot = first + (lane > 0 && kprev == ks ? vprev : 0.0);
      if (ks == kskip) pr_ord_part(a, cur.slot.x, tot);
      else sums[ks] = tot;
    }
    // the row open at the tile's end goes on in a later tile
    if (lane == kWave - 1 && r1 < a.n && offs[nr] < ne) pr_ord_part(a, cur.slot.y, vs);
    wave_lds_sync();

    // vertex updates of the rows finished here, row by row in coalesced
    // order; out-degrees (or caller ids) are in this tile's registers
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int kk = q * kWave + lane;
      if (q * kWave < nr && kk < nr && kk != kskip) {
        const double x = a.base + a.alpha * sums[kk];
        const int d = cur.row[q];
        vals[kk] = rank ? (float)x : (d > 0 ? (float)(x / (double)d) : 0.0f);
      }
    }
    p_r0 = r0;
    p_nr = nr;
    p_skip = kskip;
#pragma unroll
    for (int q = 0; q < U; ++q) p_row[q] = cur.row[q];

    if (tn >= a.ntiles) break;
    t = tn;
    cur = nxt;
  }
  // the last tile's rows
  wave_lds_sync();
#pragma unroll
  for (int q = 0; q < U; ++q) {
    const int kk = q * kWave + lane;
    if (q * kWave < p_nr && kk < p_nr && kk != p_skip) {
      if (rank) rank[p_row[q]] = vals[kk];
      else cout[p_r0 + kk] = vals[kk];
    }
  }
}

// Rows split over tiles: the vertex update from the summed parts; the slot
// is cleared for the next pass.  The parts were added by atomics in the
// previous launch, so the reads here are atomic too (a plain load could hit
// a stale line in another XCD's L2).
__global__ void k_pr_ord_split(PrOrdArgs a, float* cout, float* rank) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.nslots; i += gridDim.x * blockDim.x) {
    const double tot = __hip_atomic_load(&a.sacc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&a.sacc[i], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pr_ord_finish(a, a.srow[i], tot, cout, rank);
  }
}

size_t pr_ord_lds_bytes(int hot, int bt, int u) {
  return sizeof(float) * (size_t)hot + sizeof(int) * ((size_t)bt / kWave) * (4 * (size_t)kWave * u + 2);
}

int launch_pr_ord(const PrOrdArgs& a, int bt, int u, int grid, const float* cin, float* cout,
                  float* rank, hipStream_t s) {
  if (a.ntiles == 0) return 0;
  const size_t lds = pr_ord_lds_bytes(a.hot, bt, u);
  const int blocks = std::max(1, std::min(grid, a.ntiles));
#define GI_PR_ORD(B, UU)                                                                       \
  if (bt == B && u == UU) {                                                                    \
    hipLaunchKernelGGL((k_pr_ord<B, UU>), dim3(blocks), dim3(B), lds, s, a, cin, cout, rank); \
    return hipGetLastError() == hipSuccess ? 0 : -1;                                           \
  }
  GI_PR_ORD(256, 4)
  GI_PR_ORD(256, 8)
  GI_PR_ORD(256, 16)
  GI_PR_ORD(512, 4)
  GI_PR_ORD(512, 8)
  GI_PR_ORD(512, 16)
  GI_PR_ORD(1024, 4)
  GI_PR_ORD(1024, 8)
#undef GI_PR_ORD
  return -1;
}

int launch_pr_ord_split(const PrOrdArgs& a, float* cout, float* rank, hipStream_t s) {
  if (a.nslots == 0) return 0;
  const int blocks = std::min(1024, (a.nslots + 255) / 256);
  hipLaunchKernelGGL(k_pr_ord_split, dim3(blocks), dim3(256), 0, s, a, cout, rank);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Workgroups of k_pr_ord<bt, u> resident per CU with `hot` LDS sources.
int pr_ord_occupancy(int hot, int bt, int u) {
  int per = 0;
  const size_t lds = pr_ord_lds_bytes(hot, bt, u);
  hipError_t e = hipErrorInvalidValue;
#define GI_PR_ORD_OCC(B, UU) \
  if (bt == B && u == UU) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_pr_ord<B, UU>, B, lds);
  GI_PR_ORD_OCC(256, 4)
  GI_PR_ORD_OCC(256, 8)
  GI_PR_ORD_OCC(256, 16)
  GI_PR_ORD_OCC(512, 4)
  GI_PR_ORD_OCC(512, 8)
  GI_PR_ORD_OCC(512, 16)
  GI_PR_ORD_OCC(1024, 4)
  GI_PR_ORD_OCC(1024, 8)
#undef GI_PR_ORD_OCC
  return e == hipSuccess ? per : -1;
}

}  // namespace gi
