// Stand-alone frontier primitives: conversions between the sparse-array,
// bitvector and bool-map vertexset representations (section 2, direction
// optimization and frontier data structure; configApplyDenseVertexSet of
// the scheduling-language table) and the frontier degree sum that the
// hybrid direction rule compares against its threshold.
#include "kernels.h"

namespace gi {

__global__ void k_clear_words(int W, uint64_t* bv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < W; i += gridDim.x * blockDim.x) bv[i] = 0;
}

__global__ void k_scatter_bits(const int32_t* ids, int count, uint64_t* bv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const int v = ids[i];
    atomicOr((unsigned long long*)&bv[v >> 6], 1ull << (v & 63));
  }
}

// popcount per word
__global__ void k_word_counts(int n, const uint64_t* bv, int32_t* cnt) {
  const int W = (n + 63) >> 6;
  for (int w = blockIdx.x * blockDim.x + threadIdx.x; w < W; w += gridDim.x * blockDim.x) {
    uint64_t x = bv[w];
    const int rem = n - (w << 6);
    if (rem < 64) x &= (1ull << rem) - 1ull;
    cnt[w] = __popcll(x);
  }
}

// Exclusive scan of W word counts by one workgroup of 1024 threads:
// each thread scans a contiguous chunk, chunk totals are scanned in LDS.
__global__ __launch_bounds__(1024) void k_scan_words(int W, int32_t* cnt, int32_t* total) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (W + 1023) / 1024;
  const int b = t * chunk, e = min(W, b + chunk);
  int s = 0;
  for (int i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int y = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = b; i < e; ++i) {
    const int c = cnt[i];
    cnt[i] = run;
    run += c;
  }
  if (t == 1023) *total = part[1023];
}

// one wave per word: members written at scan[w] + rank within the word
__global__ void k_write_sorted(int n, const uint64_t* bv, const int32_t* scan, int32_t* ids) {
  const int W = (n + 63) >> 6;
  const int lane = __lane_id();
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int w = wave; w < W; w += nw) {
    const int v = (w << 6) + lane;
    const uint64_t x = bv[w];
    const bool p = v < n && ((x >> lane) & 1ull);
    if (p) ids[scan[w] + __popcll(x & lanemask_lt())] = v;
  }
}

__global__ void k_bv_to_bm(int n, const uint64_t* bv, uint8_t* bm) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    bm[v] = (uint8_t)((bv[v >> 6] >> (v & 63)) & 1ull);
}

__global__ void k_bm_to_bv(int n, const uint8_t* bm, uint64_t* bv) {
  const int W = (n + 63) >> 6;
  const int lane = __lane_id();
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  for (int w = wave; w < W; w += nw) {
    const int v = (w << 6) + lane;
    const unsigned long long m = __ballot(v < n && bm[v] != 0);
    if (lane == 0) bv[w] = m;
  }
}

__global__ void k_degree_sum(const int32_t* outdeg, const int32_t* ids, int count,
                             unsigned long long* out) {
  long long s = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    s += outdeg[ids[i]];
  s = wave_sum(s);
  if (__lane_id() == 0 && s) atomicAdd(&out[1], (unsigned long long)s);
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&out[0], (unsigned long long)count);
}

static int grid_for(long long items, int bt, int cap = 4096) {
  long long b = (items + bt - 1) / bt;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

#define GI_LAUNCH_OK() (hipGetLastError() == hipSuccess ? 0 : -1)

int launch_sparse_to_bitvec(int n, const int32_t* ids, int count, uint64_t* bv, hipStream_t s) {
  const int W = (n + 63) >> 6;
  hipLaunchKernelGGL(k_clear_words, dim3(grid_for(W, 256)), dim3(256), 0, s, W, bv);
  if (count > 0)
    hipLaunchKernelGGL(k_scatter_bits, dim3(grid_for(count, 256)), dim3(256), 0, s, ids, count, bv);
  return GI_LAUNCH_OK();
}

int launch_bitvec_to_sparse(int n, const uint64_t* bv, int32_t* ids, int32_t* count,
                            int32_t* scratch, hipStream_t s) {
  const int W = (n + 63) >> 6;
  hipLaunchKernelGGL(k_word_counts, dim3(grid_for(W, 256)), dim3(256), 0, s, n, bv, scratch);
  hipLaunchKernelGGL(k_scan_words, dim3(1), dim3(1024), 0, s, W, scratch, count);
  hipLaunchKernelGGL(k_write_sorted, dim3(grid_for((long long)W * 64, 256)), dim3(256), 0, s, n, bv,
                     scratch, ids);
  return GI_LAUNCH_OK();
}

int launch_bitvec_to_boolmap(int n, const uint64_t* bv, uint8_t* bm, hipStream_t s) {
  hipLaunchKernelGGL(k_bv_to_bm, dim3(grid_for(n, 256)), dim3(256), 0, s, n, bv, bm);
  return GI_LAUNCH_OK();
}

int launch_boolmap_to_bitvec(int n, const uint8_t* bm, uint64_t* bv, hipStream_t s) {
  const long long W = (n + 63) >> 6;
  hipLaunchKernelGGL(k_bm_to_bv, dim3(grid_for(W * 64, 256)), dim3(256), 0, s, n, bm, bv);
  return GI_LAUNCH_OK();
}

int launch_degree_sum(const int32_t* outdeg, const int32_t* ids, int count, int64_t* out,
                      hipStream_t s) {
  if (hipMemsetAsync(out, 0, 2 * sizeof(int64_t), s) != hipSuccess) return -1;
  hipLaunchKernelGGL(k_degree_sum, dim3(grid_for(count, 256)), dim3(256), 0, s, outdeg, ids, count,
                     reinterpret_cast<unsigned long long*>(out));
  return GI_LAUNCH_OK();
}

}  // namespace gi
