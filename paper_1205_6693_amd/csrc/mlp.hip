// Forward, backward and training kernels of the scheduler network (fp32).
//
// Shapes are tiny (F <= 16 inputs, H <= 64 hidden units, O <= 8 outputs) and
// the batch is a few thousand traced decisions, so every kernel is a plain
// elementwise or per-parameter loop; nothing here is a dense contraction worth
// the matrix cores.  Gradients are summed in a fixed order (per-chunk partial
// sums, then a serial sum over chunks), so training is deterministic.
#include <math.h>
#include <string.h>

#include "common.hpp"
#include "internal.hpp"
#include "mlp.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kChunk = 256;  // rows per partial gradient sum

inline unsigned blocks_for(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

struct MlpBufs {
  float* hid = nullptr;   // B x H activations tanh(W1 x + b1)
  float* y = nullptr;     // B x O outputs
  float* g = nullptr;     // B x O   dL/dY
  float* dz = nullptr;    // B x H   dL/d(W1 x + b1)
  float* part = nullptr;  // chunks x P partial gradients
  float* grad = nullptr;  // P
  float* scal = nullptr;  // [0] loss, [1] 1 / sum Wt
  int* step = nullptr;    // Adam steps taken
};

void mlp_carve(int F, int H, int O, int B, Arena& a, MlpBufs& b) {
  const int P = mlp_param_count(F, H, O);
  const int nch = (B + kChunk - 1) / kChunk;
  b.hid = a.take<float>((size_t)B * H);
  b.y = a.take<float>((size_t)B * O);
  b.g = a.take<float>((size_t)B * O);
  b.dz = a.take<float>((size_t)B * H);
  b.part = a.take<float>((size_t)nch * P);
  b.grad = a.take<float>(P);
  b.scal = a.take<float>(8);
  b.step = a.take<int>(8);
}

__global__ void k_mlp_hidden(const float* __restrict__ W, int F, int H, const float* __restrict__ X, int B,
                             float* __restrict__ hid) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * H) return;
  const int64_t r = idx / H;
  const int j = (int)(idx % H);
  const float* W1 = W;
  const float* b1 = W + H * F;
  float z = b1[j];
  for (int i = 0; i < F; ++i) z += W1[j * F + i] * X[r * F + i];
  hid[idx] = tanhf(z);
}

__global__ void k_mlp_out(const float* __restrict__ W, int F, int H, int O, const float* __restrict__ hid, int B,
                          float* __restrict__ Y) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * O) return;
  const int64_t r = idx / O;
  const int o = (int)(idx % O);
  const float* W2 = W + H * F + H;
  const float* b2 = W2 + O * H;
  float y = b2[o];
  for (int j = 0; j < H; ++j) y += W2[o * H + j] * hid[r * H + j];
  Y[idx] = y;
}

// dL/dY of the weighted squared error
__global__ void k_mlp_lossgrad(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ Wt,
                               int64_t n, const float* __restrict__ scal, float* __restrict__ G) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx < n) G[idx] = 2.f * Wt[idx] * (Y[idx] - T[idx]) * scal[1];
}

__global__ void k_mlp_dhidden(const float* __restrict__ W, int F, int H, int O, const float* __restrict__ G,
                              const float* __restrict__ hid, int B, float* __restrict__ dz) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)B * H) return;
  const int64_t r = idx / H;
  const int j = (int)(idx % H);
  const float* W2 = W + H * F + H;
  float s = 0.f;
  for (int o = 0; o < O; ++o) s += G[r * O + o] * W2[o * H + j];
  const float h = hid[idx];
  dz[idx] = s * (1.f - h * h);
}

// partial gradient of parameter p over the rows of chunk blockIdx.y
__global__ void k_mlp_wgrad(int F, int H, int O, const float* __restrict__ X, const float* __restrict__ hid,
                            const float* __restrict__ G, const float* __restrict__ dz, int B,
                            float* __restrict__ part) {
  const int P = mlp_param_count(F, H, O);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const int64_t r0 = (int64_t)blockIdx.y * kChunk;
  const int64_t r1 = r0 + kChunk < B ? r0 + kChunk : B;
  float acc = 0.f;
  if (p < H * F) {
    const int j = p / F, i = p % F;
    for (int64_t r = r0; r < r1; ++r) acc += dz[r * H + j] * X[r * F + i];
  } else if (p < H * F + H) {
    const int j = p - H * F;
    for (int64_t r = r0; r < r1; ++r) acc += dz[r * H + j];
  } else if (p < H * F + H + O * H) {
    const int q = p - H * F - H;
    const int o = q / H, j = q % H;
    for (int64_t r = r0; r < r1; ++r) acc += G[r * O + o] * hid[r * H + j];
  } else {
    const int o = p - (H * F + H + O * H);
    for (int64_t r = r0; r < r1; ++r) acc += G[r * O + o];
  }
  part[(int64_t)blockIdx.y * P + p] = acc;
}

__global__ void k_mlp_reduce(const float* __restrict__ part, int nch, int P, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  float s = 0.f;
  for (int c = 0; c < nch; ++c) s += part[(int64_t)c * P + p];
  grad[p] = s;
}

__global__ void k_adam(float* __restrict__ W, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, int P, float lr, const int* __restrict__ step) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float t = (float)(step[0] + 1);
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float c1 = 1.f - powf(b1, t), c2 = 1.f - powf(b2, t);
  W[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_set_step(int* step, int v) {
  if (threadIdx.x == 0) step[0] = v;
}

__global__ void k_step_inc(int* step) {
  if (threadIdx.x == 0) step[0] = step[0] + 1;
}

// fixed-order tree reduction of one double per thread (blockDim.x a power of two <= 1024)
__device__ double block_sum_fixed(double x, double* lds) {
  const int t = threadIdx.x;
  lds[t] = x;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] += lds[t + s];
    __syncthreads();
  }
  const double r = lds[0];
  __syncthreads();
  return r;
}

// scal[1] = 1 / sum(Wt) (0 if the sum is not positive); one workgroup
__global__ void k_wsum(const float* __restrict__ Wt, int64_t n, float* __restrict__ scal) {
  __shared__ double lds[kT];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += (double)Wt[i];
  s = block_sum_fixed(s, lds);
  if (threadIdx.x == 0) scal[1] = s > 0.0 ? (float)(1.0 / s) : 0.f;
}

// scal[0] = sum Wt (Y - T)^2 / sum Wt; one workgroup
__global__ void k_loss(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ Wt,
                       int64_t n, float* __restrict__ scal) {
  __shared__ double lds[kT];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = (double)Y[i] - (double)T[i];
    s += (double)Wt[i] * d * d;
  }
  s = block_sum_fixed(s, lds);
  if (threadIdx.x == 0) scal[0] = (float)(s * (double)scal[1]);
}

int check_dims(int F, int H, int O, int B) {
  if (F < 1 || F > kMlpMaxF || H < 1 || H > kMlpMaxH || O < 1 || O > kMlpMaxO || B < 1) {
    set_last_error("network shape F=%d H=%d O=%d B=%d outside the limits", F, H, O, B);
    return TRUSS_E_INVAL;
  }
  return TRUSS_OK;
}

int mlp_need(int F, int H, int O, int B, size_t* bytes) {
  Arena a;
  a.counting = true;
  MlpBufs b;
  mlp_carve(F, H, O, B, a, b);
  *bytes = a.used;
  return TRUSS_OK;
}

void launch_forward(const float* W, int F, int H, int O, const float* X, int B, float* hid, float* Y, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_hidden, dim3(blocks_for((int64_t)B * H)), dim3(kT), 0, s, W, F, H, X, B, hid);
  hipLaunchKernelGGL(k_mlp_out, dim3(blocks_for((int64_t)B * O)), dim3(kT), 0, s, W, F, H, O, hid, B, Y);
}

// grad = dL/dW given G = dL/dY (hid must hold the forward activations)
void launch_backward(const float* W, int F, int H, int O, const float* X, int B, const float* G, const MlpBufs& b,
                     float* grad, hipStream_t s) {
  const int P = mlp_param_count(F, H, O);
  const int nch = (B + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(k_mlp_dhidden, dim3(blocks_for((int64_t)B * H)), dim3(kT), 0, s, W, F, H, O, G, b.hid, B, b.dz);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for(P), (unsigned)nch), dim3(kT), 0, s, F, H, O, X, b.hid, G, b.dz, B,
                     b.part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(blocks_for(P)), dim3(kT), 0, s, b.part, nch, P, grad);
}

// Adam training on the weighted loss; the buffers come from mlp_carve.
int run_train(float* W, float* am, float* av, int F, int H, int O, const float* X, const float* T, const float* Wt,
              int B, int steps, int step0, float lr, float* loss, const MlpBufs& b, hipStream_t s) {
  const int P = mlp_param_count(F, H, O);
  const int64_t n = (int64_t)B * O;
  hipLaunchKernelGGL(k_wsum, dim3(1), dim3(kT), 0, s, Wt, n, b.scal);
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, b.step, step0);
  float sc[2] = {0.f, 0.f};
  TRUSS_HIP(hipMemcpyAsync(sc, b.scal, sizeof(sc), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  if (!(sc[1] > 0.f)) {
    set_last_error("training weights sum to zero");
    return TRUSS_E_INVAL;
  }
  for (int it = 0; it < steps; ++it) {
    launch_forward(W, F, H, O, X, B, b.hid, b.y, s);
    hipLaunchKernelGGL(k_mlp_lossgrad, dim3(blocks_for(n)), dim3(kT), 0, s, b.y, T, Wt, n, b.scal, b.g);
    launch_backward(W, F, H, O, X, B, b.g, b, b.grad, s);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(P)), dim3(kT), 0, s, W, b.grad, am, av, P, lr, b.step);
    hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, b.step);
  }
  TRUSS_HIP(hipGetLastError());
  if (loss) {
    launch_forward(W, F, H, O, X, B, b.hid, b.y, s);
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(kT), 0, s, b.y, T, Wt, n, b.scal);
    TRUSS_HIP(hipMemcpyAsync(sc, b.scal, sizeof(sc), hipMemcpyDeviceToHost, s));
  }
  TRUSS_HIP(hipStreamSynchronize(s));
  if (loss) *loss = sc[0];
  return TRUSS_OK;
}

// ---- scheduler model fitting -------------------------------------------------------------
int sched_dims(int kind, int* F, int* O) {
  if (kind == 0) { *F = kPeelF; *O = kPeelA; return TRUSS_OK; }
  if (kind == 1) { *F = kSupF; *O = kSupA; return TRUSS_OK; }
  set_last_error("model kind %d is neither 0 (peeling) nor 1 (support)", kind);
  return TRUSS_E_INVAL;
}

struct SchedBufs {
  float* xn;   // B x F normalised features
  float* y;    // B x A log2 times
  float* wt;   // B x A weights
  float* mu;   // F
  float* isd;  // F
  float* w;    // P parameters
  float* am;   // P
  float* av;   // P
  MlpBufs mb;
};

void sched_carve(int F, int H, int A, int B, Arena& a, SchedBufs& sb) {
  const int P = mlp_param_count(F, H, A);
  sb.xn = a.take<float>((size_t)B * F);
  sb.y = a.take<float>((size_t)B * A);
  sb.wt = a.take<float>((size_t)B * A);
  sb.mu = a.take<float>(kMlpMaxF);
  sb.isd = a.take<float>(kMlpMaxF);
  sb.w = a.take<float>(P);
  sb.am = a.take<float>(P);
  sb.av = a.take<float>(P);
  mlp_carve(F, H, A, B, a, sb.mb);
}

// Normalisation, targets and weights; one workgroup of kT threads.
//   mu[f], isd[f]: mean and 1 / max(std, 1e-3) of feature f over the rows;
//   y = log2(T) and weight max(0.05, rowmax / mean rowmax) where T > 0, else 0,
//   rowmax being the slowest measured action of the row.
__global__ void k_sched_prep(const float* __restrict__ X, const float* __restrict__ T, int B, int F, int A,
                             float* __restrict__ xn, float* __restrict__ y, float* __restrict__ wt,
                             float* __restrict__ mu, float* __restrict__ isd) {
  __shared__ double lds[kT];
  __shared__ float s_mu[kMlpMaxF], s_isd[kMlpMaxF];
  for (int f = 0; f < F; ++f) {
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < B; r += blockDim.x) s += (double)X[r * F + f];
    const double mean = block_sum_fixed(s, lds) / (double)B;
    double q = 0.0;
    for (int64_t r = threadIdx.x; r < B; r += blockDim.x) {
      const double d = (double)X[r * F + f] - mean;
      q += d * d;
    }
    const double var = block_sum_fixed(q, lds) / (double)B;
    const double sd = sqrt(var);
    if (threadIdx.x == 0) {
      s_mu[f] = (float)mean;
      s_isd[f] = (float)(1.0 / (sd > 1e-3 ? sd : 1e-3));
    }
  }
  double rs = 0.0, rc = 0.0;
  for (int64_t r = threadIdx.x; r < B; r += blockDim.x) {
    float mx = 0.f;
    for (int a = 0; a < A; ++a) mx = T[r * A + a] > mx ? T[r * A + a] : mx;
    if (mx > 0.f) {
      rs += (double)mx;
      rc += 1.0;
    }
  }
  rs = block_sum_fixed(rs, lds);
  rc = block_sum_fixed(rc, lds);
  const double mean_max = rc > 0.0 ? rs / rc : 1.0;
  __syncthreads();
  if (threadIdx.x < F) {
    mu[threadIdx.x] = s_mu[threadIdx.x];
    isd[threadIdx.x] = s_isd[threadIdx.x];
  }
  for (int64_t r = threadIdx.x; r < B; r += blockDim.x) {
    for (int f = 0; f < F; ++f) xn[r * F + f] = (X[r * F + f] - s_mu[f]) * s_isd[f];
    float mx = 0.f;
    for (int a = 0; a < A; ++a) mx = T[r * A + a] > mx ? T[r * A + a] : mx;
    double wr = (double)mx / mean_max;
    if (wr < 0.05) wr = 0.05;
    for (int a = 0; a < A; ++a) {
      const float t = T[r * A + a];
      const bool ok = t > 0.f;
      y[r * A + a] = ok ? log2f(t) : 0.f;
      wt[r * A + a] = ok ? (float)wr : 0.f;
    }
  }
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ULL;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// Glorot-uniform weights, zero biases and zero Adam moments.
__global__ void k_sched_init(float* __restrict__ W, float* __restrict__ am, float* __restrict__ av, int F, int H,
                             int O, unsigned long long seed) {
  const int P = mlp_param_count(F, H, O);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double u = (double)(splitmix64(seed * 0x100000001b3ULL + (unsigned long long)p) >> 11) * 0x1.0p-53;
  float w = 0.f;
  if (p < H * F) w = (float)((2.0 * u - 1.0) * sqrt(6.0 / (double)(F + H)));
  else if (p >= H * F + H && p < H * F + H + O * H) w = (float)((2.0 * u - 1.0) * sqrt(6.0 / (double)(H + O)));
  W[p] = w;
  am[p] = 0.f;
  av[p] = 0.f;
}

__global__ void k_sched_pack(float* __restrict__ part, int F, int H, int O, const float* __restrict__ mu,
                             const float* __restrict__ isd, const float* __restrict__ W) {
  const int P = mlp_param_count(F, H, O);
  const int total = model_part_floats(F, H, O);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  float v;
  if (i == 0) v = kModelTag;
  else if (i == 1) v = (float)F;
  else if (i == 2) v = (float)H;
  else if (i == 3) v = (float)O;
  else if (i < 4 + F) v = mu[i - 4];
  else if (i < 4 + 2 * F) v = isd[i - 4 - F];
  else v = W[i - 4 - 2 * F];
  (void)P;
  part[i] = v;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws || ws_bytes < need) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
    return TRUSS_E_WORKSPACE;
  }
  return TRUSS_OK;
}

}  // namespace

}  // namespace truss

using namespace truss;

extern "C" {

int truss_mlp_param_count(int32_t F, int32_t H, int32_t O) {
  if (check_dims(F, H, O, 1)) return TRUSS_E_INVAL;
  return mlp_param_count(F, H, O);
}

int truss_mlp_workspace_size(int32_t F, int32_t H, int32_t O, int32_t B, size_t* bytes) {
  int rc = check_dims(F, H, O, B);
  if (rc) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  return mlp_need(F, H, O, B, bytes);
}

int truss_mlp_forward(const float* params, int32_t F, int32_t H, int32_t O, const float* X, int32_t B, float* Y,
                      void* ws, size_t ws_bytes, void* stream) {
  int rc = check_dims(F, H, O, B);
  if (rc) return rc;
  if (!params || !X || !Y) { set_last_error("NULL argument"); return TRUSS_E_INVAL; }
  size_t need = 0;
  mlp_need(F, H, O, B, &need);
  if ((rc = check_ws(ws, ws_bytes, need))) return rc;
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  MlpBufs b;
  mlp_carve(F, H, O, B, a, b);
  hipStream_t s = (hipStream_t)stream;
  launch_forward(params, F, H, O, X, B, b.hid, Y, s);
  TRUSS_HIP(hipGetLastError());
  TRUSS_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

int truss_mlp_backward(const float* params, int32_t F, int32_t H, int32_t O, const float* X, int32_t B,
                       const float* dY, float* grad, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_dims(F, H, O, B);
  if (rc) return rc;
  if (!params || !X || !dY || !grad) { set_last_error("NULL argument"); return TRUSS_E_INVAL; }
  size_t need = 0;
  mlp_need(F, H, O, B, &need);
  if ((rc = check_ws(ws, ws_bytes, need))) return rc;
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  MlpBufs b;
  mlp_carve(F, H, O, B, a, b);
  hipStream_t s = (hipStream_t)stream;
  launch_forward(params, F, H, O, X, B, b.hid, b.y, s);
  launch_backward(params, F, H, O, X, B, dY, b, grad, s);
  TRUSS_HIP(hipGetLastError());
  TRUSS_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

int truss_mlp_train(float* params, float* adam_m, float* adam_v, int32_t F, int32_t H, int32_t O, const float* X,
                    const float* T, const float* Wt, int32_t B, int32_t steps, int32_t step0, float lr, float* loss,
                    void* ws, size_t ws_bytes, void* stream) {
  int rc = check_dims(F, H, O, B);
  if (rc) return rc;
  if (!params || !adam_m || !adam_v || !X || !T || !Wt || steps < 0 || step0 < 0 || !(lr > 0.f)) {
    set_last_error("bad training arguments");
    return TRUSS_E_INVAL;
  }
  size_t need = 0;
  mlp_need(F, H, O, B, &need);
  if ((rc = check_ws(ws, ws_bytes, need))) return rc;
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  MlpBufs b;
  mlp_carve(F, H, O, B, a, b);
  return run_train(params, adam_m, adam_v, F, H, O, X, T, Wt, B, steps, step0, lr, loss, b, (hipStream_t)stream);
}

int truss_sched_part_floats(int32_t kind, int32_t H) {
  int F = 0, O = 0;
  if (sched_dims(kind, &F, &O)) return TRUSS_E_INVAL;
  if (check_dims(F, H, O, 1)) return TRUSS_E_INVAL;
  return model_part_floats(F, H, O);
}

int truss_sched_model_floats(int32_t H) {
  const int a = truss_sched_part_floats(0, H), b = truss_sched_part_floats(1, H);
  if (a < 0 || b < 0) return TRUSS_E_INVAL;
  return a + b;
}

int truss_sched_train_workspace_size(int32_t kind, int32_t H, int32_t B, size_t* bytes) {
  int F = 0, A = 0;
  int rc = sched_dims(kind, &F, &A);
  if (rc) return rc;
  if ((rc = check_dims(F, H, A, B))) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  Arena a;
  a.counting = true;
  SchedBufs sb;
  sched_carve(F, H, A, B, a, sb);
  *bytes = a.used;
  return TRUSS_OK;
}

int truss_sched_train(int32_t kind, const float* X, const float* T_ms, int32_t B, int32_t H, int32_t steps, float lr,
                      uint64_t seed, float* part, float* loss, void* ws, size_t ws_bytes, void* stream) {
  int F = 0, A = 0;
  int rc = sched_dims(kind, &F, &A);
  if (rc) return rc;
  if ((rc = check_dims(F, H, A, B))) return rc;
  if (!X || !T_ms || !part || steps < 0 || !(lr > 0.f)) {
    set_last_error("bad training arguments");
    return TRUSS_E_INVAL;
  }
  size_t need = 0;
  truss_sched_train_workspace_size(kind, H, B, &need);
  if ((rc = check_ws(ws, ws_bytes, need))) return rc;
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  SchedBufs sb;
  sched_carve(F, H, A, B, a, sb);
  hipStream_t s = (hipStream_t)stream;
  const int P = mlp_param_count(F, H, A);
  hipLaunchKernelGGL(k_sched_prep, dim3(1), dim3(kT), 0, s, X, T_ms, B, F, A, sb.xn, sb.y, sb.wt, sb.mu, sb.isd);
  hipLaunchKernelGGL(k_sched_init, dim3(blocks_for(P)), dim3(kT), 0, s, sb.w, sb.am, sb.av, F, H, A,
                     (unsigned long long)seed);
  TRUSS_HIP(hipGetLastError());
  rc = run_train(sb.w, sb.am, sb.av, F, H, A, sb.xn, sb.y, sb.wt, B, steps, 0, lr, loss, sb.mb, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_sched_pack, dim3(blocks_for(model_part_floats(F, H, A))), dim3(kT), 0, s, part, F, H, A,
                     sb.mu, sb.isd, sb.w);
  TRUSS_HIP(hipGetLastError());
  TRUSS_HIP(hipStreamSynchronize(s));
  return TRUSS_OK;
}

}  // extern "C"
