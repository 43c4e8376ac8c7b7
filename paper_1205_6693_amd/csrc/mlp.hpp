// The scheduler's network: a two-layer perceptron in fp32,
//   y = W2 tanh(W1 x + b1) + b2,
// with parameters packed as W1[H][F], b1[H], W2[O][H], b2[O] (row-major).
// A scheduler model part adds a header and the feature normalisation:
//   [0] kModelTag, [1] F, [2] H, [3] O, mu[F], isd[F], parameters,
// and the network sees (x - mu) * isd.  Each output estimates log2 of the
// time (ms) of one action; the scheduler takes the allowed action with the
// smallest estimate.  The network only chooses between exact methods: it
// never reads or writes supports or truss numbers.
#pragma once

#include "../../include/truss.h"
#include "common.hpp"

namespace truss {

constexpr float kModelTag = 1205.0f;
constexpr int kMlpMaxF = TRUSS_MLP_MAX_F;
constexpr int kMlpMaxH = TRUSS_MLP_MAX_H;
constexpr int kMlpMaxO = TRUSS_MLP_MAX_O;

// features and actions of the two decisions
constexpr int kPeelF = TRUSS_SCHED_PEEL_F;
constexpr int kPeelA = TRUSS_SCHED_PEEL_A;
constexpr int kSupF = TRUSS_SCHED_SUP_F;
constexpr int kSupA = TRUSS_SCHED_SUP_A;
constexpr int kSupBins = TRUSS_SCHED_SUP_BINS;

__host__ __device__ constexpr int mlp_param_count(int F, int H, int O) { return H * F + H + O * H + O; }
__host__ __device__ constexpr int model_part_floats(int F, int H, int O) { return 4 + 2 * F + mlp_param_count(F, H, O); }

// Scores of one feature vector, evaluated by a whole wavefront (hidden unit j
// on lane j).  x (F raw features) must be the same in every lane; the result
// is the same in every lane (lane 0's sums are broadcast).
__device__ __forceinline__ void mlp_scores_wave(const float* __restrict__ part, const float* x, float* out) {
  const int F = (int)part[1], H = (int)part[2], O = (int)part[3];
  const float* mu = part + 4;
  const float* isd = mu + F;
  const float* W1 = isd + F;
  const float* b1 = W1 + H * F;
  const float* W2 = b1 + H;
  const float* b2 = W2 + O * H;
  const int j = lane_id();
  float h = 0.f;
  if (j < H) {
    float z = b1[j];
    for (int i = 0; i < F; ++i) z += W1[j * F + i] * ((x[i] - mu[i]) * isd[i]);
    h = tanhf(z);
  }
  for (int o = 0; o < O; ++o) {
    float p = j < H ? W2[o * H + j] * h : 0.f;
    p = wave_sum(p);
    out[o] = __shfl(p, 0, kWave) + b2[o];
  }
}

// smallest score among the actions allowed by `mask` (bit a = action a);
// ties go to the lower action index
__device__ __forceinline__ int argmin_allowed(const float* s, int n, unsigned mask) {
  int best = -1;
  for (int a = 0; a < n; ++a) {
    if (!(mask >> a & 1u)) continue;
    if (best < 0 || s[a] < s[best]) best = a;
  }
  return best < 0 ? 0 : best;
}

}  // namespace truss
