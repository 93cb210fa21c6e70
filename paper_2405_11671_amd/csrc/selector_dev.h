// Device-side inference of the learned edgeMap-variant selector, shared by
// the stand-alone predictor (selector.hip) and the device-side level control
// (graphmode.hip). Network F -> H (ReLU) -> H (ReLU) -> K, FP32, parameters
// packed as W1[F][H] b1[H] W2[H][H] b2[H] W3[H][K] b3[K], then the feature
// means mu[F] and deviations sd[F] the inputs are normalised with.
#pragma once

#include "internal.h"

namespace byo {

constexpr int SEL_F = BYO_MLP_F, SEL_H = BYO_MLP_H, SEL_K = BYO_MLP_K, SEL_P = BYO_MLP_PARAMS;
constexpr int SEL_W1 = 0, SEL_B1 = SEL_W1 + SEL_F * SEL_H, SEL_W2 = SEL_B1 + SEL_H,
              SEL_B2 = SEL_W2 + SEL_H * SEL_H, SEL_W3 = SEL_B2 + SEL_H, SEL_B3 = SEL_W3 + SEL_H * SEL_K;
static_assert(SEL_B3 + SEL_K == SEL_P, "parameter layout");

// Called by all 64 threads of a 64-thread block with the same raw features
// (raw[] may live anywhere the threads can read): normalise, evaluate,
// argmin over the allowed variants (pull variants skipped unless allow_pull).
// Returns the choice in every thread, -1 if any prediction is not finite;
// pred_out (nullable) receives the K predictions.
__device__ inline int sel_pick_block(const float *__restrict__ wts, const float *raw, bool allow_pull,
                                     float *pred_out) {
  __shared__ float x[SEL_F], h1[SEL_H], h2[SEL_H], o[SEL_K];
  __shared__ int best_s;
  const int t = threadIdx.x;
  if (t < SEL_F) x[t] = (raw[t] - wts[SEL_P + t]) / wts[SEL_P + SEL_F + t];
  __syncthreads();
  if (t < SEL_H) {
    float z = wts[SEL_B1 + t];
    for (int i = 0; i < SEL_F; ++i) z += x[i] * wts[SEL_W1 + i * SEL_H + t];
    h1[t] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  if (t < SEL_H) {
    float z = wts[SEL_B2 + t];
    for (int i = 0; i < SEL_H; ++i) z += h1[i] * wts[SEL_W2 + i * SEL_H + t];
    h2[t] = z > 0.f ? z : 0.f;
  }
  __syncthreads();
  if (t < SEL_K) {
    float z = wts[SEL_B3 + t];
    for (int i = 0; i < SEL_H; ++i) z += h2[i] * wts[SEL_W3 + i * SEL_K + t];
    o[t] = z;
    if (pred_out) pred_out[t] = z;
  }
  __syncthreads();
  if (t == 0) {
    int best = -1;
    for (int v = 0; v < SEL_K; ++v) {
      if (!isfinite(o[v])) {
        best = -1;
        break;
      }
      const bool pull = v == BYO_V_PULL_THREAD || v == BYO_V_PULL_WAVE;
      if (pull && !allow_pull) continue;
      if (best < 0 || o[v] < o[best]) best = v;
    }
    best_s = best;
  }
  __syncthreads();
  return best_s;
}

}  // namespace byo
