// Learned schedule selector: a multilayer perceptron 12 -> 64 -> 64 -> 4
// (ReLU) that predicts the natural log of the time, in ms, of the next
// traversal step under each of four schedules:
//   S0 SparsePush (sparse-array frontier), S1 DensePush, S2 DensePull,
//   S3 DensePull over cache segments.
// The paper tunes schedules offline by timing whole runs (autotuning,
// section 6.4) and switches direction per step by a frontier-size rule
// (section 2); the selector replaces that rule with a model trained on the
// library's own per-step timings.  Weights are trained in FP32; inference
// during a run uses BF16 weights with FP32 accumulation.
//
// Parameter layout (fp32, row-major):
//   W1[12][64] b1[64] W2[64][64] b2[64] W3[64][4] b3[4]   (5252 values)
// Features are clamped to the range of the training records, [lo, hi], and
// standardised, x' = (clamp(x) - mu) * isd, before the first layer; the
// clamp keeps the model from extrapolating to graphs larger or more skewed
// than those it was trained on.  Device buffer: parameters, then mu[12],
// isd[12], lo[12], hi[12].
#pragma once

#include "common.h"

namespace gi {

constexpr int kHid = 64;
constexpr int kOut = 4;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kOut;
constexpr int kParams = kOffB3 + kOut;  // 5252
static_assert(kParams == GI_SEL_PARAMS, "parameter count");

// The learned choice replaces the fallback (the hybrid rule; unsegmented
// DensePull for PageRank) only when its predicted log-time is lower by more
// than this (about 15%).
constexpr float kLearnedMargin = 0.14f;

// Device copy of a selector for inference.
struct SelDev {
  const float* p;      // fp32 parameters (biases are read from here)
  const uint16_t* wb;  // bf16 copy of the parameters (weights are read from here)
  const float* mu;     // feature means
  const float* isd;    // reciprocal feature standard deviations
  const float* lo;     // feature range of the training records
  const float* hi;
};

constexpr int kSelBuf = kParams + 4 * kFeat;  // floats of a selector's device buffer

// Clamped, standardised feature f.
__device__ __forceinline__ float sel_input(const SelDev& s, int f, float x) {
  return (fminf(fmaxf(x, s.lo[f]), s.hi[f]) - s.mu[f]) * s.isd[f];
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
  return __uint_as_float((unsigned)h << 16);
}

// Forward pass by the first 64 threads of a workgroup (every thread of the
// workgroup must call it: it synchronises).  x: the 12 raw features in LDS;
// y receives the 4 predicted log-times.  xn, h1, h2: LDS scratch.
__device__ __forceinline__ void mlp_forward_block(const SelDev& s, const float* x, float* xn,
                                                  float* h1, float* h2, float* y) {
  const int t = threadIdx.x;
  if (t < kFeat) xn[t] = sel_input(s, t, x[t]);
  __syncthreads();
  if (t < kHid) {
    float a = s.p[kOffB1 + t];
    for (int f = 0; f < kFeat; ++f) a += xn[f] * bf16_bits_to_f32(s.wb[kOffW1 + f * kHid + t]);
    h1[t] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  if (t < kHid) {
    float a = s.p[kOffB2 + t];
    for (int i = 0; i < kHid; ++i) a += h1[i] * bf16_bits_to_f32(s.wb[kOffW2 + i * kHid + t]);
    h2[t] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  if (t < kOut) {
    float a = s.p[kOffB3 + t];
    for (int i = 0; i < kHid; ++i) a += h2[i] * bf16_bits_to_f32(s.wb[kOffW3 + i * kOut + t]);
    y[t] = a;
  }
  __syncthreads();
}

// Graph-level part of the features (computed once per graph and algorithm
// on the host): log2 n, log2 E, E/n, log2(1 + max degree), degree
// coefficient of variation, algorithm id (BFS 0, CC 0.5, PageRank 1).
struct FeatConst {
  float g[5];
  float alg;
};

// The 12 features of a step (see gi_get_step_features in the header for the
// definitions).  `unvisited` is the BFS unvisited fraction; other
// algorithms pass the fraction of the frontier's degree sum in the edges.
__device__ __forceinline__ void step_features(const FeatConst& c, long long n, long long edges,
                                              long long nf, long long dsum, long long nf_prev,
                                              float unvisited, float* x) {
  x[0] = c.g[0];
  x[1] = c.g[1];
  x[2] = c.g[2];
  x[3] = c.g[3];
  x[4] = c.g[4];
  x[5] = (float)((double)nf / (double)n);
  x[6] = (float)((double)dsum / (double)(edges > 0 ? edges : 1));
  x[7] = unvisited;
  x[8] = log2f(1.0f + (float)nf);
  x[9] = log2f(1.0f + (float)dsum);
  const double r = (double)nf / (double)(nf_prev > 1 ? nf_prev : 1);
  x[10] = (float)(r > 64.0 ? 64.0 : r);
  x[11] = c.alg;
}

}  // namespace gi
