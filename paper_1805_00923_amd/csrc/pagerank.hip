// PageRank by DensePull (section 2, DensePull figure; evaluation: 20
// iterations, damping 0.85):
//   x_0 = 1/n,  x_{k+1}[v] = (1-alpha)/n + alpha * sum_{u->v} x_k[u] / outdeg(u).
// Every destination gathers contrib[u] = x_k[u]/outdeg(u) over its in-edges
// without atomics.  contrib and ranks are stored as FP32, sums accumulate in
// FP64.
//
// Destination blocks: the in-edge range of a run of consecutive destinations
// (at most cap_e edges) is staged in LDS with coalesced index loads and
// contrib gathers (four of each in flight per thread), then reduced per
// destination by a power-of-two group of threads.  A destination with more
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
// applies the vertex update.
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

}  // namespace gi
