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

namespace gi {

template <int BT>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[BT / kWave];
  v = wave_sum(v);
  if (__lane_id() == 0) part[threadIdx.x / kWave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x < kWave) {
    t = threadIdx.x < BT / kWave ? part[threadIdx.x] : 0.0;
    t = wave_sum(t);
  }
  __syncthreads();
  return t;  // valid in thread 0
}

// Sum over the edge range [eb, ee) of cin[idx[e]] by the whole workgroup,
// four independent loads in flight per thread; result valid in thread 0.
template <int BT>
__device__ __forceinline__ double range_sum(const int32_t* __restrict__ idx,
                                            const float* __restrict__ cin, int eb, int ee) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int e = eb + (int)threadIdx.x;
  for (; e + 3 * BT < ee; e += 4 * BT) {
    const int a0 = idx[e], a1 = idx[e + BT], a2 = idx[e + 2 * BT], a3 = idx[e + 3 * BT];
    s0 += (double)cin[a0];
    s1 += (double)cin[a1];
    s2 += (double)cin[a2];
    s3 += (double)cin[a3];
  }
  for (; e < ee; e += BT) s0 += (double)cin[idx[e]];
  return block_sum<BT>((s0 + s1) + (s2 + s3));
}

// mode 0: final vertex update from the full sum; mode 1: acc[dst] += sum.
template <int BT>
__device__ void pr_rows_block(const PrRows& r, int t, int cap_e, const float* __restrict__ cin,
                              int mode, const PrVertex& pv, float* __restrict__ cout,
                              float* __restrict__ rank, double* __restrict__ acc, float* lds_val,
                              int* lds_off) {
  const int4 en = r.table[t];
  const int tid = threadIdx.x;
  auto finish = [&](int row, double s) {
    const int v = r.dst ? r.dst[row] : row;
    if (mode == 1) {
      acc[v] += s;
    } else {
      const double x = pv.base + pv.alpha * s;
      if (rank) {
        rank[v] = (float)x;
      } else {
        const int d = pv.outdeg[v];
        cout[v] = d > 0 ? (float)(x / (double)d) : 0.0f;
      }
    }
  };
  if (en.z >= 0) {
    // one chunk of a row longer than cap_e: partial sums meet in an FP64
    // accumulator; the chunk that arrives last applies the vertex update
    const int row = en.x;
    const int rb = r.off[row], re = r.off[row + 1];
    const int eb = rb + en.w * cap_e, ee = min(re, eb + cap_e);
    const double s = range_sum<BT>(r.idx, cin, eb, ee);
    if (tid == 0) {
      if (mode == 1) {
        atomicAdd(&acc[r.dst ? r.dst[row] : row], s);
      } else {
        atomicAdd(&r.lr_acc[en.z], s);
        __threadfence();
        const unsigned done = atomicAdd(&r.lr_cnt[en.z], 1u);
        if (done == (unsigned)r.lr_chunks[en.z] - 1u) {
          __threadfence();
          const double tot = atomicAdd(&r.lr_acc[en.z], 0.0);
          __hip_atomic_store(&r.lr_acc[en.z], 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&r.lr_cnt[en.z], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          finish(row, tot);
        }
      }
    }
    return;
  }
  const int kb = en.x, ke = en.y, nr = ke - kb;
  const int e0 = r.off[kb], e1 = r.off[ke], ne = e1 - e0;
  gather_block<BT, float>(r.idx, e0, ne, lds_val, [cin](int u) { return cin[u]; });
  for (int k = tid; k <= nr; k += BT) lds_off[k] = r.off[kb + k] - e0;
  __syncthreads();
  int tpv = 1;
  if (nr < BT) {
    tpv = BT / (nr > 0 ? nr : 1);
    tpv = 1 << (31 - __clz(tpv));
    if (tpv > kWave) tpv = kWave;
  }
  const int groups = BT / tpv, grp = tid / tpv, gl = tid % tpv;
  for (int k0 = 0; k0 < nr; k0 += groups) {
    const int k = k0 + grp;
    double s = 0.0;
    if (k < nr) {
      const int a = lds_off[k], b = lds_off[k + 1];
      for (int j = a + gl; j < b; j += tpv) s += (double)lds_val[j];
    }
    for (int o = tpv >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (gl == 0 && k < nr) finish(kb + k, s);
  }
  __syncthreads();
}

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

int launch_pr_seg_final(int n, const PrVertex& pv, double* acc, float* cout, float* rank,
                        hipStream_t s) {
  const int blocks = (int)std::min<long long>(4096, ((long long)n + 255) / 256);
  hipLaunchKernelGGL(k_pr_seg_final, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, n, pv, acc,
                     cout, rank);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gi
