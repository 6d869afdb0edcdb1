// Device training and batch inference of the schedule selector (selector.h).
//
// Training: one workgroup runs every epoch in a single launch.  Each
// minibatch of 32 records is pushed through the network with activations in
// LDS; the gradient of
//   L = (1/V) * sum over valid (record, schedule) pairs of (y - t)^2
// (V = valid pairs in the minibatch) is formed layer by layer, one output
// element per thread, then Adam updates every parameter.  Adam: Kingma and
// Ba, "Adam: A Method for Stochastic Optimization", ICLR 2015, with bias
// correction.
#include "kernels.h"
#include "selector.h"

namespace gi {

constexpr int kTB = 256;  // training workgroup
constexpr int kMB = 32;   // records per minibatch

__device__ __forceinline__ float relu(float a) { return a > 0.0f ? a : 0.0f; }

template <int BT>
__device__ __forceinline__ float block_sum_f(float v, float* sh) {
  v = wave_sum(v);
  if (__lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  float t = 0.0f;
  for (int i = 0; i < BT / kWave; ++i) t += sh[i];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kTB) void k_mlp_train(TrainArgs a) {
  __shared__ float xn[kMB][kFeat];
  __shared__ float h1[kMB][kHid];
  __shared__ float h2[kMB][kHid];
  __shared__ float dy[kMB][kOut];
  __shared__ float dh2[kMB][kHid];
  __shared__ float dh1[kMB][kHid];
  __shared__ int rec[kMB];
  __shared__ float red[kTB / kWave];
  const int t = threadIdx.x;
  float* p = a.p;
  long long step = a.t0;
  for (int ep = 0; ep < a.epochs; ++ep) {
    float ep_loss = 0.0f;
    int nb = 0;
    for (int r0 = 0; r0 < a.n; r0 += kMB) {
      const int bc = min(kMB, a.n - r0);
      if (t < kMB) rec[t] = t < bc ? a.order[r0 + t] : 0;
      __syncthreads();
      for (int i = t; i < kMB * kFeat; i += kTB) {
        const int b = i / kFeat, f = i % kFeat;
        xn[b][f] = b < bc ? (a.x[(size_t)rec[b] * kFeat + f] - a.mu[f]) * a.isd[f] : 0.0f;
      }
      __syncthreads();
      for (int i = t; i < kMB * kHid; i += kTB) {
        const int b = i / kHid, j = i % kHid;
        float acc = p[kOffB1 + j];
        for (int f = 0; f < kFeat; ++f) acc += xn[b][f] * p[kOffW1 + f * kHid + j];
        h1[b][j] = relu(acc);
      }
      __syncthreads();
      for (int i = t; i < kMB * kHid; i += kTB) {
        const int b = i / kHid, j = i % kHid;
        float acc = p[kOffB2 + j];
        for (int k = 0; k < kHid; ++k) acc += h1[b][k] * p[kOffW2 + k * kHid + j];
        h2[b][j] = relu(acc);
      }
      __syncthreads();
      // output layer and loss gradient: thread t < 128 owns (b, s)
      float y = 0.0f, tgt = 0.0f;
      bool val = false;
      if (t < kMB * kOut) {
        const int b = t / kOut, s = t % kOut;
        if (b < bc) {
          val = a.valid[(size_t)rec[b] * kOut + s] != 0;
          y = p[kOffB3 + s];
          for (int k = 0; k < kHid; ++k) y += h2[b][k] * p[kOffW3 + k * kOut + s];
          tgt = a.y[(size_t)rec[b] * kOut + s];
        }
      }
      const int nv = __syncthreads_count(val ? 1 : 0);
      const float inv = nv > 0 ? 1.0f / (float)nv : 0.0f;
      const float diff = val ? y - tgt : 0.0f;
      if (t < kMB * kOut) dy[t / kOut][t % kOut] = 2.0f * diff * inv;
      const float bl = block_sum_f<kTB>(diff * diff * inv, red);
      ep_loss += bl;
      ++nb;
      // W3, b3; then dh2 from the old W3
      for (int i = t; i < kHid * kOut; i += kTB) {
        const int k = i / kOut, s = i % kOut;
        float g = 0.0f;
        for (int b = 0; b < bc; ++b) g += h2[b][k] * dy[b][s];
        a.grad[kOffW3 + i] = g;
      }
      if (t < kOut) {
        float g = 0.0f;
        for (int b = 0; b < bc; ++b) g += dy[b][t];
        a.grad[kOffB3 + t] = g;
      }
      for (int i = t; i < kMB * kHid; i += kTB) {
        const int b = i / kHid, k = i % kHid;
        float g = 0.0f;
        if (h2[b][k] > 0.0f)
          for (int s = 0; s < kOut; ++s) g += dy[b][s] * p[kOffW3 + k * kOut + s];
        dh2[b][k] = g;
      }
      __syncthreads();
      // W2, b2; then dh1 from the old W2
      for (int i = t; i < kHid * kHid; i += kTB) {
        const int k = i / kHid, j = i % kHid;
        float g = 0.0f;
        for (int b = 0; b < bc; ++b) g += h1[b][k] * dh2[b][j];
        a.grad[kOffW2 + i] = g;
      }
      if (t < kHid) {
        float g = 0.0f;
        for (int b = 0; b < bc; ++b) g += dh2[b][t];
        a.grad[kOffB2 + t] = g;
      }
      for (int i = t; i < kMB * kHid; i += kTB) {
        const int b = i / kHid, k = i % kHid;
        float g = 0.0f;
        if (h1[b][k] > 0.0f)
          for (int j = 0; j < kHid; ++j) g += dh2[b][j] * p[kOffW2 + k * kHid + j];
        dh1[b][k] = g;
      }
      __syncthreads();
      // W1, b1
      for (int i = t; i < kFeat * kHid; i += kTB) {
        const int f = i / kHid, j = i % kHid;
        float g = 0.0f;
        for (int b = 0; b < bc; ++b) g += xn[b][f] * dh1[b][j];
        a.grad[kOffW1 + i] = g;
      }
      if (t < kHid) {
        float g = 0.0f;
        for (int b = 0; b < bc; ++b) g += dh1[b][t];
        a.grad[kOffB1 + t] = g;
      }
      __syncthreads();
      if (a.apply) {
        ++step;
        const float c1 = (float)(1.0 - pow((double)a.beta1, (double)step));
        const float c2 = (float)(1.0 - pow((double)a.beta2, (double)step));
        for (int i = t; i < kParams; i += kTB) {
          const float g = a.grad[i];
          const float m = a.beta1 * a.m1[i] + (1.0f - a.beta1) * g;
          const float v = a.beta2 * a.m2[i] + (1.0f - a.beta2) * g * g;
          a.m1[i] = m;
          a.m2[i] = v;
          p[i] -= a.lr * (m / c1) / (sqrtf(v / c2) + a.eps);
        }
      }
      __syncthreads();
    }
    if (t == 0 && a.loss) a.loss[ep] = nb > 0 ? ep_loss / (float)nb : 0.0f;
  }
}

// Batch inference: one 64-thread workgroup per record.
template <bool BF16>
__global__ __launch_bounds__(kWave) void k_mlp_predict(SelDev s, const float* x, long long n,
                                                       float* out) {
  __shared__ float sx[kFeat], xn[kFeat], h1[kHid], h2[kHid], y[kOut];
  for (long long r = blockIdx.x; r < n; r += gridDim.x) {
    const int t = threadIdx.x;
    if (t < kFeat) sx[t] = x[r * kFeat + t];
    __syncthreads();
    if (BF16) {
      mlp_forward_block(s, sx, xn, h1, h2, y);
    } else {
      // same network with the fp32 weights
      if (t < kFeat) xn[t] = sel_input(s, t, sx[t]);
      __syncthreads();
      float acc = s.p[kOffB1 + t];
      for (int f = 0; f < kFeat; ++f) acc += xn[f] * s.p[kOffW1 + f * kHid + t];
      h1[t] = relu(acc);
      __syncthreads();
      acc = s.p[kOffB2 + t];
      for (int k = 0; k < kHid; ++k) acc += h1[k] * s.p[kOffW2 + k * kHid + t];
      h2[t] = relu(acc);
      __syncthreads();
      if (t < kOut) {
        acc = s.p[kOffB3 + t];
        for (int k = 0; k < kHid; ++k) acc += h2[k] * s.p[kOffW3 + k * kOut + t];
        y[t] = acc;
      }
      __syncthreads();
    }
    if (t < kOut) out[r * kOut + t] = y[t];
    __syncthreads();
  }
}

int launch_mlp_train(const TrainArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(kTB), 0, s, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mlp_predict(const SelDev& sd, const float* x, long long n, bool bf16, float* out,
                       hipStream_t s) {
  if (n <= 0) return 0;
  const int blocks = (int)std::min<long long>(n, 65536);
  if (bf16) hipLaunchKernelGGL(k_mlp_predict<true>, dim3(blocks), dim3(kWave), 0, s, sd, x, n, out);
  else hipLaunchKernelGGL(k_mlp_predict<false>, dim3(blocks), dim3(kWave), 0, s, sd, x, n, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gi
