// Core numbers (the c-core is the largest subgraph with minimum degree >= c)
// and the per-vertex sums behind the cohesion statistics of Section 7
// (Table 6: the k_max-truss against the c_max-core).
//
// Core numbers peel vertices level by level, like the edges of Algorithm 2:
// level c takes every live vertex of degree <= c (core number c); removing a
// taken vertex lowers the degree of each live neighbour by one, and a
// neighbour whose degree falls from c+1 to c is taken in the next sub-round
// of the same level.  Taken vertices are not decremented again, so each live
// vertex loses exactly its edges to taken vertices.  An empty level jumps to
// the smallest live degree.  The host drives the sub-rounds (a few hundred
// at these sizes); the work of a sub-round is a wavefront per taken vertex.
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kIntMax = 0x7fffffff;

struct CoreCtl {
  int qn;     // vertices taken by this pass
  int minv;   // smallest degree among live vertices not taken
  int alive;  // live vertices not taken
  int pad;
};

inline unsigned blocks(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

__global__ void k_core_init(const int64_t* __restrict__ row_ptr, int32_t n, int32_t* __restrict__ deg,
                            int32_t* __restrict__ core) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v < n) {
    deg[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
    core[v] = -1;
  }
}

__global__ void k_core_ctl_reset(CoreCtl* c) {
  if (threadIdx.x == 0) {
    c->qn = 0;
    c->minv = kIntMax;
    c->alive = 0;
  }
}

// level start: live vertices of degree <= level are taken
__global__ void __launch_bounds__(kT) k_core_start(const int32_t* __restrict__ deg, int32_t* __restrict__ core,
                                                   int32_t n, int level, int32_t* __restrict__ q, CoreCtl* c) {
  __shared__ int s_min[kT / kWave], s_cnt[kT / kWave];
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool take = false;
  int dmin = kIntMax, alive = 0;
  if (v < n && core[v] < 0) {
    const int d = deg[v];
    if (d <= level) {
      take = true;
      core[v] = level;
    } else {
      dmin = d;
      alive = 1;
    }
  }
  const int pos = wave_append(&c->qn, take);
  if (take) q[pos] = (int32_t)v;
  dmin = wave_min(dmin);
  alive = wave_sum(alive);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_min[w] = dmin;
    s_cnt[w] = alive;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = kIntMax;
    for (int q2 = 0; q2 < kT / kWave; ++q2) {
      a += s_cnt[q2];
      b = s_min[q2] < b ? s_min[q2] : b;
    }
    if (a) atomicAdd(&c->alive, a);
    if (b != kIntMax) atomicMin(&c->minv, b);
  }
}

// a sub-round: every taken vertex removes its edges to live vertices
__global__ void __launch_bounds__(kT) k_core_round(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                   int32_t* __restrict__ deg, int32_t* __restrict__ core,
                                                   const int32_t* __restrict__ q, int qn, int level,
                                                   int32_t* __restrict__ nq, CoreCtl* c) {
  const int lane = lane_id();
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t i = gw; i < qn; i += nw) {
    const int32_t v = q[i];
    const int64_t rb = row_ptr[v], re = row_ptr[v + 1];
    for (int64_t j0 = rb; j0 < re; j0 += kWave) {
      const int64_t j = j0 + lane;
      bool take = false;
      int32_t u = 0;
      if (j < re) {
        u = col[j];
        if (__hip_atomic_load(&core[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 0) {
          const int old = atomicSub(&deg[u], 1);
          if (old == level + 1) {
            __hip_atomic_store(&core[u], level, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            take = true;
          }
        }
      }
      const int pos = wave_append(&c->qn, take);
      if (take) nq[pos] = u;
    }
  }
}

// per-vertex degree and triangle sums over a subgraph's edges (sup = support
// of each subgraph edge inside the subgraph)
__global__ void k_vertex_sums(const int32_t* __restrict__ su, const int32_t* __restrict__ sv,
                              const int32_t* __restrict__ sup, int64_t ms, int32_t* __restrict__ deg,
                              unsigned long long* __restrict__ tri) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ms) return;
  atomicAdd(&deg[su[e]], 1);
  atomicAdd(&deg[sv[e]], 1);
  atomicAdd(&tri[su[e]], (unsigned long long)sup[e]);
  atomicAdd(&tri[sv[e]], (unsigned long long)sup[e]);
}

// local clustering coefficient of every vertex (0 for degree < 2)
__global__ void k_local_cc(const int32_t* __restrict__ deg, const unsigned long long* __restrict__ tri, int32_t n,
                           double* __restrict__ cc) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double d = (double)deg[v];
  cc[v] = deg[v] >= 2 ? (double)(tri[v] / 2) / (d * (d - 1.0) / 2.0) : 0.0;
}

// vertices with degree > 0 and the sum of their coefficients, in a fixed order
__global__ void __launch_bounds__(1024) k_cc_reduce(const int32_t* __restrict__ deg, const double* __restrict__ cc,
                                                    int32_t n, double* __restrict__ out) {
  __shared__ double s_sum[1024];
  __shared__ double s_cnt[1024];
  double a = 0.0, b = 0.0;
  for (int64_t v = threadIdx.x; v < n; v += blockDim.x) {
    if (deg[v] > 0) {
      a += cc[v];
      b += 1.0;
    }
  }
  s_sum[threadIdx.x] = a;
  s_cnt[threadIdx.x] = b;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + st];
      s_cnt[threadIdx.x] += s_cnt[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_cnt[0];
    out[1] = s_sum[0];
  }
}

}  // namespace

size_t core_workspace(int32_t n, Arena& a) {
  a.take<int32_t>((size_t)n + 1);
  a.take<int32_t>((size_t)n + 1);
  a.take<int32_t>((size_t)n + 1);
  a.take<CoreCtl>(1);
  return a.used;
}

int compute_core_numbers(const DevGraph& dg, int32_t* core, int32_t* cmax_out, Arena& a, hipStream_t s) {
  int32_t* deg = a.take<int32_t>((size_t)dg.n + 1);
  int32_t* q[2] = {a.take<int32_t>((size_t)dg.n + 1), a.take<int32_t>((size_t)dg.n + 1)};
  CoreCtl* c = a.take<CoreCtl>(1);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  *cmax_out = 0;
  if (dg.n == 0) return TRUSS_OK;
  hipLaunchKernelGGL(k_core_init, dim3(blocks(dg.n)), dim3(kT), 0, s, dg.row_ptr, dg.n, deg, core);
  int level = 0, cmax = 0;
  CoreCtl h;
  for (;;) {
    hipLaunchKernelGGL(k_core_ctl_reset, dim3(1), dim3(64), 0, s, c);
    hipLaunchKernelGGL(k_core_start, dim3(blocks(dg.n)), dim3(kT), 0, s, deg, core, dg.n, level, q[0], c);
    TRUSS_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    if (h.qn == 0) {
      if (h.alive == 0) break;
      level = h.minv;  // no vertex at this level: the next level is the smallest live degree
      continue;
    }
    cmax = level;
    int cur = 0, qn = h.qn;
    while (qn > 0) {
      hipLaunchKernelGGL(k_core_ctl_reset, dim3(1), dim3(64), 0, s, c);
      const int64_t waves = qn < 65536 ? qn : 65536;
      hipLaunchKernelGGL(k_core_round, dim3(blocks(waves * kWave)), dim3(kT), 0, s, dg.row_ptr, dg.col, deg, core,
                         q[cur], qn, level, q[cur ^ 1], c);
      TRUSS_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, s));
      TRUSS_HIP(hipStreamSynchronize(s));
      cur ^= 1;
      qn = h.qn;
    }
    ++level;
  }
  TRUSS_HIP(hipGetLastError());
  *cmax_out = cmax;
  return TRUSS_OK;
}

int subgraph_vertex_stats(int32_t n, const int32_t* su, const int32_t* sv, const int32_t* sup, int64_t ms, Arena& a,
                          double* nv_out, double* cc_out, hipStream_t s) {
  int32_t* deg = a.take<int32_t>((size_t)n + 1);
  unsigned long long* tri = a.take<unsigned long long>((size_t)n + 1);
  double* cc = a.take<double>((size_t)n + 1);
  double* red = a.take<double>(4);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  TRUSS_HIP(hipMemsetAsync(deg, 0, sizeof(int32_t) * ((size_t)n + 1), s));
  TRUSS_HIP(hipMemsetAsync(tri, 0, sizeof(unsigned long long) * ((size_t)n + 1), s));
  if (ms > 0) hipLaunchKernelGGL(k_vertex_sums, dim3(blocks(ms)), dim3(kT), 0, s, su, sv, sup, ms, deg, tri);
  hipLaunchKernelGGL(k_local_cc, dim3(blocks(n)), dim3(kT), 0, s, deg, tri, n, cc);
  hipLaunchKernelGGL(k_cc_reduce, dim3(1), dim3(1024), 0, s, deg, cc, n, red);
  double h[2] = {0.0, 0.0};
  TRUSS_HIP(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  *nv_out = h[0];
  *cc_out = h[0] > 0.0 ? h[1] / h[0] : 0.0;
  return TRUSS_OK;
}

}  // namespace truss
