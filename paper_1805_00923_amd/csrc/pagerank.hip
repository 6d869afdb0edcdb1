// PageRank by DensePull (section 2, DensePull figure; evaluation: 20
// iterations, damping 0.85):
//   x_0 = 1/n,  x_{k+1}[v] = (1-alpha)/n + alpha * sum_{u->v} x_k[u] / outdeg(u).
// Every destination gathers contrib[u] = x_k[u]/outdeg(u) over its in-edges
// without atomics.  contrib and ranks are stored as FP32, sums accumulate in
// FP64.
//
// Destination blocks: the in-edge range of a run of consecutive destinations
// (at most cap_e edges) is staged in LDS with coalesced index loads and
// contrib gathers (four of each in flight per thread), then reduced by a
// deterministic edge-parallel segmented sum (pr_block.h), so skewed rows in
// one block spread over all its threads.  A destination with more
// than cap_e in-edges is cut into chunks of cap_e edges, each summed by one
// workgroup; the chunks' partial sums meet in an FP64 accumulator and the
// last chunk to finish applies the vertex update.  Chunks of long rows come
// first in the table so that they start early.
//
// Segmented (cache-partitioned) form, section 2 and the SSG code of section
// 6: sources are split into segments V_0..V_{p-1}; segment i holds the
// in-edges whose source lies in V_i, grouped by destination.  Segments are
// processed in order, each adding partial sums into an FP64 accumulator, so
// the contrib gathers of one segment touch only |V_i| entries; a final pass
// applies the vertex update.  In the concurrent form workgroup b serves
// segment b mod p into its own FP64 partial array (one segment per XCD for
// p = 8), and the final pass sums the p partials.
#include <type_traits>

#include "kernels.h"
#include "pr_block.h"

namespace gi {

// contrib_0[v] = (1/n)/outdeg(v); with zero iterations the ranks are 1/n.
__device__ __forceinline__ void pr_init_range(int i0, int stride, int n, const int32_t* outdeg,
                                              float* c0, float* rank, bool zero_iters) {
  const double x0 = 1.0 / (double)n;
  for (int v = i0; v < n; v += stride) {
    if (zero_iters) {
      rank[v] = (float)x0;
    } else {
      const int d = outdeg[v];
      c0[v] = d > 0 ? (float)(x0 / (double)d) : 0.0f;
    }
  }
}

__global__ void k_pr_init(int n, const int32_t* outdeg, float* c0, float* rank, int zero_iters) {
  pr_init_range(blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, n, outdeg, c0, rank,
                zero_iters != 0);
}

template <int BT>
__global__ __launch_bounds__(BT) void k_pr_rows(PrRows r, int cap_e, const float* cin, int mode,
                                                PrVertex pv, float* cout, float* rank, double* acc) {
  extern __shared__ float smem[];
  float* lds_val = smem;
  int* lds_off = reinterpret_cast<int*>(smem + cap_e);
  for (int t = blockIdx.x; t < r.ntab; t += gridDim.x)
    pr_rows_block<BT>(r, t, cap_e, cin, mode, pv, cout, rank, acc, lds_val, lds_off);
}

// Segmented epilogue: x = base + alpha*acc[v]; acc[v] = 0.
__global__ void k_pr_seg_final(int n, PrVertex pv, double* acc, float* cout, float* rank) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const double x = pv.base + pv.alpha * acc[v];
    acc[v] = 0.0;
    if (rank) {
      rank[v] = (float)x;
    } else {
      const int d = pv.outdeg[v];
      cout[v] = d > 0 ? (float)(x / (double)d) : 0.0f;
    }
  }
}

// Concurrent segments (one per XCD): workgroup b works on segment b % p, so
// with p = 8 and the round-robin dispatch of workgroups over the eight XCDs
// every XCD gathers from one segment's contributions only, which then stay
// in that XCD's L2.  Segment x adds its rows' partial sums into its own
// FP64 buffer acc + x n; the final pass adds the p partials of each vertex
// (and zeroes them).  Placement only affects speed, never the result.
template <int BT>
__global__ __launch_bounds__(BT) void k_pr_seg_concurrent(const PrRows* segs, int p, int cap_e,
                                                          const float* cin, PrVertex pv,
                                                          double* acc, int n) {
  extern __shared__ float smem[];
  float* lds_val = smem;
  int* lds_off = reinterpret_cast<int*>(smem + cap_e);
  const int x = (int)(blockIdx.x % (unsigned)p);
  const int j = (int)(blockIdx.x / (unsigned)p);
  const int nb = (int)(gridDim.x / (unsigned)p);
  const PrRows r = segs[x];
  double* ax = acc + (size_t)x * (size_t)n;
  for (int t = j; t < r.ntab; t += nb)
    pr_rows_block<BT>(r, t, cap_e, cin, 1, pv, nullptr, nullptr, ax, lds_val, lds_off);
}

__global__ void k_pr_seg_final_multi(int n, int p, PrVertex pv, double* acc, float* cout,
                                     float* rank) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int x = 0; x < p; ++x) {
      double* a = acc + (size_t)x * (size_t)n + v;
      s += *a;
      *a = 0.0;
    }
    const double y = pv.base + pv.alpha * s;
    if (rank) {
      rank[v] = (float)y;
    } else {
      const int d = pv.outdeg[v];
      cout[v] = d > 0 ? (float)(y / (double)d) : 0.0f;
    }
  }
}

// PageRank fused with eigenvector centrality (the paper's loop and apply
// fusion plus its vertex-data layout optimization): one pass over the
// in-edges gathers both kernels' per-source values from one array of
// (contribution, y) pairs, so each edge fetches one 8-byte element instead
// of two 4-byte elements in two arrays.  Eigenvector centrality is the
// L2-normalised power iteration: y_{k+1}[v] = sum_{u->v} y_k[u] / ||y_k||,
// the norm of each new y accumulated in FP64 as it is produced.  Unfused,
// the same kernel gathers y alone and PageRank runs its own pass.
//
// Blocks are reduced by the deterministic edge-parallel segmented sum of
// the PageRank kernel; a row longer than a block is cut into chunks whose
// sums meet in an FP64 slot, finished by k_prec_long after the pass.
template <bool FUSED>
struct PrEcVertex {
  const PrEcArgs& a;
  double inv;
  double n2 = 0.0;
  __device__ __forceinline__ void operator()(int v, double sp, double se) {
    const double y = se * inv;
    n2 += y * y;
    if (FUSED) {
      const double x = a.pv.base + a.pv.alpha * sp;
      const int d = a.pv.outdeg[v];
      a.aos_out[v] = make_float2(d > 0 ? (float)(x / (double)d) : 0.0f, (float)y);
      if (a.ranks) a.ranks[v] = (float)x;
    } else {
      a.y_out[v] = (float)y;
    }
  }
};

__device__ __forceinline__ double inv_norm(const double* n2p) {
  const double n2 = *n2p;
  return n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
}

template <int BT, bool FUSED>
__global__ __launch_bounds__(BT) void k_prec_rows(PrEcArgs a) {
  using V = typename std::conditional<FUSED, float2, float>::type;
  __shared__ V lds_val[kPrEcCapE];
  __shared__ int lds_off[kPrEcCapV + 1];
  __shared__ double head[2][BT], cont[2][BT];
  const int tid = threadIdx.x;
  PrEcVertex<FUSED> fin{a, inv_norm(a.norm2_prev)};
  auto fetch = [&](int u) -> V {
    if constexpr (FUSED) return a.aos_in[u];
    else return a.y_in[u];
  };
  auto add = [](double& sp, double& se, const V& c) {
    if constexpr (FUSED) {
      sp += (double)c.x;
      se += (double)c.y;
    } else {
      se += (double)c;
    }
  };
  int4 nx = blockIdx.x < (unsigned)a.rb.ntab ? a.rb.table[blockIdx.x] : make_int4(0, 0, 0, 0);
  for (int t = blockIdx.x; t < a.rb.ntab; t += gridDim.x) {
    const int4 r = nx;
    if (t + (int)gridDim.x < a.rb.ntab) nx = a.rb.table[t + gridDim.x];
    if (r.y < 0) {
      // a chunk of a long row: workgroup sums into the row's FP64 slot
      double sp = 0.0, se = 0.0, sp2 = 0.0, se2 = 0.0;
      int e = r.z + tid;
      for (; e + BT < r.w; e += 2 * BT) {
        const int u0 = a.rb.idx[e], u1 = a.rb.idx[e + BT];
        const V c0 = fetch(u0), c1 = fetch(u1);
        add(sp, se, c0);
        add(sp2, se2, c1);
      }
      if (e < r.w) add(sp, se, fetch(a.rb.idx[e]));
      const double tp = block_sum<BT>(sp + sp2), te = block_sum<BT>(se + se2);
      if (tid == 0) {
        if (FUSED) atomicAdd(&a.lacc[2 * r.x], tp);
        atomicAdd(&a.lacc[2 * r.x + 1], te);
      }
      continue;
    }
    const int kb = r.x, ke = r.y, nr = ke - kb;
    const int e0 = r.z, ne = r.w - r.z;
    gather_block<BT, V>(a.rb.idx, e0, ne, lds_val, fetch);
    for (int k = tid; k <= nr; k += BT) lds_off[k] = a.rb.off[kb + k] - e0;
    __syncthreads();
    const int ept = (ne + BT - 1) / BT;
    const int eb = tid * ept, ee = min(ne, eb + ept);
    int kl = -1, kl_end = 0;
    if (eb < ee) {
      int lo = 0, hi = nr;  // lds_off[lo] <= eb < lds_off[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (lds_off[mid] <= eb) lo = mid;
        else hi = mid;
      }
      int k = lo, rs = lds_off[k], re = lds_off[k + 1];
      double sp = 0.0, se = 0.0;
      for (int j = eb; j < ee; ++j) {
        if (j >= re) {
          if (rs >= eb) {
            fin(kb + k, sp, se);
          } else {
            cont[0][tid] = sp;
            cont[1][tid] = se;
          }
          sp = 0.0;
          se = 0.0;
          do {
            ++k;
          } while (lds_off[k + 1] <= j);
          rs = lds_off[k];
          re = lds_off[k + 1];
        }
        add(sp, se, lds_val[j]);
      }
      if (re <= ee && rs >= eb) {
        fin(kb + k, sp, se);
      } else if (re > ee && rs >= eb) {
        head[0][tid] = sp;
        head[1][tid] = se;
        kl = k;
        kl_end = re;
      } else {
        cont[0][tid] = sp;
        cont[1][tid] = se;
      }
    }
    __syncthreads();
    if (kl >= 0) {
      double sp = head[0][tid], se = head[1][tid];
      const int t1 = (kl_end - 1) / ept;
      for (int q = tid + 1; q <= t1; ++q) {
        sp += cont[0][q];
        se += cont[1][q];
      }
      fin(kb + kl, sp, se);
    }
    for (int k = tid; k < nr; k += BT)
      if (lds_off[k] == lds_off[k + 1]) fin(kb + k, 0.0, 0.0);
    __syncthreads();
  }
  const double tot = block_sum<BT>(fin.n2);
  if (tid == 0 && tot != 0.0) atomicAdd(a.norm2_next, tot);
}

// Long rows after the pass: apply the vertex update from each slot's sums,
// clear the slot, and add the new y values to the norm.
template <bool FUSED>
__global__ __launch_bounds__(256) void k_prec_long(PrEcArgs a) {
  PrEcVertex<FUSED> fin{a, inv_norm(a.norm2_prev)};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < a.nlong; i += gridDim.x * 256) {
    const double sp = a.lacc[2 * i], se = a.lacc[2 * i + 1];
    a.lacc[2 * i] = 0.0;
    a.lacc[2 * i + 1] = 0.0;
    fin(a.lrow[i], sp, se);
  }
  const double tot = block_sum<256>(fin.n2);
  if (threadIdx.x == 0 && tot != 0.0) atomicAdd(a.norm2_next, tot);
}

// y_0 = 1/n (norm2[0] = 1 so that it is used unscaled), contributions of
// x_0 = 1/n; the later norms start at 0.
__global__ void k_prec_init(int n, const int32_t* outdeg, float2* aos, float* y, double* norm2,
                            int nnorm) {
  const double x0 = 1.0 / (double)n;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    if (aos) {
      const int d = outdeg[v];
      aos[v] = make_float2(d > 0 ? (float)(x0 / (double)d) : 0.0f, (float)x0);
    }
    if (y) y[v] = (float)x0;
  }
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < nnorm; i += blockDim.x) norm2[i] = i == 0 ? 1.0 : 0.0;
}

// x_K = y_K / ||y_K|| (0 when the norm is 0).
__global__ void k_ec_final(int n, const float* y, const float2* aos, const double* norm2,
                           float* out) {
  const double n2 = *norm2;
  const double inv = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const double yv = aos ? (double)aos[v].y : (double)y[v];
    out[v] = (float)(yv * inv);
  }
}

// Results of a run over the degree-ordered numbering back under the
// caller's ids: out[old_id[r]] = tmp[r] (a and b; a may be skipped).
__global__ void k_prec_remap(int n, const int32_t* old_id, const float* ta, float* oa,
                             const float* tb, float* ob) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const int v = old_id[r];
    if (ta) oa[v] = ta[r];
    ob[v] = tb[r];
  }
}

// ------------------------------------------------------- host launchers ----

static size_t pr_lds_bytes(int cap_e, int cap_v) {
  return sizeof(float) * (size_t)cap_e + sizeof(int) * (size_t)(cap_v + 1);
}

int launch_pr_init(int n, const int32_t* outdeg, float* c0, float* rank, bool zero_iters,
                   hipStream_t s) {
  const int blocks = (int)std::min<long long>(2048, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_pr_init, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, outdeg, c0, rank,
                     zero_iters ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pr_rows(const PrRows& r, int cap_e, int cap_v, int bt, int grid, const float* cin,
                   int mode, const PrVertex& pv, float* cout, float* rank, double* acc,
                   hipStream_t s) {
  if (r.ntab == 0) return 0;
  const size_t lds = pr_lds_bytes(cap_e, cap_v);
  const int blocks = grid > 0 ? std::min(grid, r.ntab) : r.ntab;
  switch (bt) {
    case 64: hipLaunchKernelGGL(k_pr_rows<64>, dim3(blocks), dim3(64), lds, s, r, cap_e, cin, mode, pv, cout, rank, acc); break;
    case 128: hipLaunchKernelGGL(k_pr_rows<128>, dim3(blocks), dim3(128), lds, s, r, cap_e, cin, mode, pv, cout, rank, acc); break;
    case 256: hipLaunchKernelGGL(k_pr_rows<256>, dim3(blocks), dim3(256), lds, s, r, cap_e, cin, mode, pv, cout, rank, acc); break;
    case 512: hipLaunchKernelGGL(k_pr_rows<512>, dim3(blocks), dim3(512), lds, s, r, cap_e, cin, mode, pv, cout, rank, acc); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pr_seg_concurrent(const PrRows* segs, int p, int cap_e, int cap_v, int bt,
                             const float* cin, const PrVertex& pv, double* acc, int n,
                             hipStream_t s) {
  const size_t lds = pr_lds_bytes(cap_e, cap_v);
  const int blocks = p * std::max(1, 2048 / p);
  switch (bt) {
    case 64: hipLaunchKernelGGL(k_pr_seg_concurrent<64>, dim3(blocks), dim3(64), lds, s, segs, p, cap_e, cin, pv, acc, n); break;
    case 128: hipLaunchKernelGGL(k_pr_seg_concurrent<128>, dim3(blocks), dim3(128), lds, s, segs, p, cap_e, cin, pv, acc, n); break;
    case 256: hipLaunchKernelGGL(k_pr_seg_concurrent<256>, dim3(blocks), dim3(256), lds, s, segs, p, cap_e, cin, pv, acc, n); break;
    case 512: hipLaunchKernelGGL(k_pr_seg_concurrent<512>, dim3(blocks), dim3(512), lds, s, segs, p, cap_e, cin, pv, acc, n); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pr_seg_final_multi(int n, int p, const PrVertex& pv, double* acc, float* cout,
                              float* rank, hipStream_t s) {
  const int blocks = (int)std::min<long long>(4096, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_pr_seg_final_multi, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, p,
                     pv, acc, cout, rank);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_pr_seg_final(int n, const PrVertex& pv, double* acc, float* cout, float* rank,
                        hipStream_t s) {
  const int blocks = (int)std::min<long long>(4096, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_pr_seg_final, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, pv, acc,
                     cout, rank);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prec_rows(const PrEcArgs& a, bool fused, hipStream_t s) {
  const int blocks = std::max(1, std::min(a.rb.ntab, 2048));
  if (fused) hipLaunchKernelGGL((k_prec_rows<256, true>), dim3(blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_prec_rows<256, false>), dim3(blocks), dim3(256), 0, s, a);
  if (a.nlong > 0) {
    const int lb = std::min(64, (a.nlong + 255) / 256);
    if (fused) hipLaunchKernelGGL((k_prec_long<true>), dim3(lb), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_prec_long<false>), dim3(lb), dim3(256), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prec_init(int n, const int32_t* outdeg, float2* aos, float* y, double* norm2,
                     int nnorm, hipStream_t s) {
  const int blocks = (int)std::min<long long>(2048, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_prec_init, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, outdeg, aos,
                     y, norm2, nnorm);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prec_remap(int n, const int32_t* old_id, const float* ta, float* oa, const float* tb,
                      float* ob, hipStream_t s) {
  const int blocks = (int)std::min<long long>(2048, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_prec_remap, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, old_id, ta,
                     oa, tb, ob);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_ec_final(int n, const float* y, const float2* aos, const double* norm2, float* out,
                    hipStream_t s) {
  const int blocks = (int)std::min<long long>(2048, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_ec_final, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, y, aos, norm2,
                     out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gi
