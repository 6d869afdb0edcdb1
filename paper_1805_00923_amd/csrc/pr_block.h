// PageRank destination-block routine shared by the PageRank kernels and the
// batched persistent kernel (see pagerank.hip for the method).
#pragma once

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
template <int BT, typename TC>
__device__ __forceinline__ double range_sum(const int32_t* __restrict__ idx,
                                            const TC* __restrict__ cin, int eb, int ee) {
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
// TC: type of the gathered contributions (float for PageRank, double for
// PageRankDelta's partial sums).
template <int BT, typename TC = float>
__device__ void pr_rows_block(const PrRows& r, int t, int cap_e, const TC* __restrict__ cin,
                              int mode, const PrVertex& pv, float* __restrict__ cout,
                              float* __restrict__ rank, double* __restrict__ acc, TC* lds_val,
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
    const double s = range_sum<BT, TC>(r.idx, cin, eb, ee);
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
  gather_block<BT, TC>(r.idx, e0, ne, lds_val, [cin](int u) { return cin[u]; });
  for (int k = tid; k <= nr; k += BT) lds_off[k] = r.off[kb + k] - e0;
  __syncthreads();
  // Edge-parallel segmented sum, deterministic: thread t takes a run of
  // ceil(ne / BT) consecutive edges and sums each row piece in order.  A row
  // wholly inside the run is finished by that thread; a row crossing runs
  // leaves its first piece in head[t0] and later pieces in cont[t], and
  // thread t0 adds them in thread order.  The block's edges are spread
  // evenly over the threads however skewed its rows are.
  __shared__ double head[BT], cont[BT];
  const int ept = (ne + BT - 1) / BT;
  const int eb = tid * ept, ee = min(ne, eb + ept);
  int kl = -1, kl_end = 0;  // row whose head this thread holds
  if (eb < ee) {
    int lo = 0, hi = nr;  // lds_off[lo] <= eb < lds_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (lds_off[mid] <= eb) lo = mid;
      else hi = mid;
    }
    int k = lo, rs = lds_off[k], re = lds_off[k + 1];
    double sum = 0.0;
    for (int j = eb; j < ee; ++j) {
      if (j >= re) {  // row k ends inside the run
        if (rs >= eb) finish(kb + k, sum);
        else cont[tid] = sum;
        sum = 0.0;
        do {
          ++k;
        } while (lds_off[k + 1] <= j);
        rs = lds_off[k];
        re = lds_off[k + 1];
      }
      sum += (double)lds_val[j];
    }
    if (re <= ee) {  // the last row ends with the run
      if (rs >= eb) finish(kb + k, sum);
      else cont[tid] = sum;
    } else if (rs >= eb) {  // it starts here and runs on
      head[tid] = sum;
      kl = k;
      kl_end = re;
    } else {  // a run inside one row
      cont[tid] = sum;
    }
  }
  __syncthreads();
  if (kl >= 0) {
    double sum = head[tid];
    const int t1 = (kl_end - 1) / ept;
    for (int t = tid + 1; t <= t1; ++t) sum += cont[t];
    finish(kb + kl, sum);
  }
  for (int k = tid; k < nr; k += BT)
    if (lds_off[k] == lds_off[k + 1]) finish(kb + k, 0.0);
  __syncthreads();
}

}  // namespace gi
