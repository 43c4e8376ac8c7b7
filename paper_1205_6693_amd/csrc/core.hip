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
// the smallest live degree.  Each level start and each sub-round is one
// launch of the same step kernel (a thread per vertex at a level start, a
// wavefront per taken vertex in a sub-round); the step's last workgroup
// decides the next step, so launches are queued without host round trips.
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kIntMax = 0x7fffffff;

// The peeling runs as a sequence of identical launches (steps) of one kernel;
// the state below says what a step does.  The last workgroup to finish a step
// decides the next one, so launches follow each other without a host round
// trip; the host checks for the end every kStepsPerCheck launches.
enum CorePhase : int { kStart = 0, kRound = 1, kDone = 2 };

struct CoreState {
  int phase;  // kStart: take live vertices of degree <= level; kRound: remove the queue's vertices
  int level;
  int cur;    // queue holding the current frontier
  int qn;     // its length (kRound)
  int cmax;
  int steps;
  // counters of the running step, cleared by the workgroup that decides
  int next;   // vertices appended by this step
  int alive;  // kStart: live vertices left
  int minv;   // kStart: their smallest degree
  unsigned arrived;
};

constexpr unsigned kStepBlocks = 1024;
constexpr int kStepsPerCheck = 16;

inline unsigned blocks(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

__global__ void k_core_init(const int64_t* __restrict__ row_ptr, int32_t n, int32_t* __restrict__ deg,
                            int32_t* __restrict__ core, CoreState* st) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v < n) {
    deg[v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
    core[v] = -1;
  }
  if (v == 0) {
    st->phase = kStart;
    st->level = 0;
    st->cur = 0;
    st->qn = 0;
    st->cmax = 0;
    st->steps = 0;
    st->next = 0;
    st->alive = 0;
    st->minv = kIntMax;
    st->arrived = 0;
  }
}

__global__ void __launch_bounds__(kT) k_core_step(const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col, int32_t* __restrict__ deg,
                                                  int32_t* __restrict__ core, int32_t n, int32_t* __restrict__ q0,
                                                  int32_t* __restrict__ q1, CoreState* st) {
  __shared__ int s_min[kT / kWave], s_cnt[kT / kWave];
  __shared__ int s_last;
  const int phase = st->phase;  // written by an earlier launch
  if (phase == kDone) return;
  const int level = st->level, cur = st->cur;
  int32_t* qc = cur ? q1 : q0;
  int32_t* qx = cur ? q0 : q1;
  const int lane = lane_id();
  if (phase == kStart) {
    // live vertices of degree <= level are taken (core number = level)
    int dmin = kIntMax, alive = 0;
    for (int64_t v0 = (int64_t)blockIdx.x * kT; v0 < n; v0 += (int64_t)gridDim.x * kT) {
      const int64_t v = v0 + threadIdx.x;
      bool take = false;
      if (v < n && core[v] < 0) {
        const int d = deg[v];
        if (d <= level) {
          take = true;
          core[v] = level;
        } else {
          dmin = d < dmin ? d : dmin;
          alive += 1;
        }
      }
      const int pos = wave_append(&st->next, take);
      if (take) qc[pos] = (int32_t)v;
    }
    dmin = wave_min(dmin);
    alive = wave_sum(alive);
    const int w = threadIdx.x / kWave;
    if (lane == 0) {
      s_min[w] = dmin;
      s_cnt[w] = alive;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int x = 0, y = kIntMax;
      for (int i = 0; i < kT / kWave; ++i) {
        x += s_cnt[i];
        y = s_min[i] < y ? s_min[i] : y;
      }
      if (x) atomicAdd(&st->alive, x);
      if (y != kIntMax) atomicMin(&st->minv, y);
    }
  } else {
    // every queued vertex removes its edges to live vertices; a neighbour
    // whose degree falls from level + 1 to level joins the next queue
    const int qn = st->qn;
    const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t i = gw; i < qn; i += nw) {
      const int32_t v = qc[i];
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
        const int pos = wave_append(&st->next, take);
        if (take) qx[pos] = u;
      }
    }
  }
  // the last workgroup of the step decides the next one
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&st->arrived, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    __threadfence();
    const int next = __hip_atomic_load(&st->next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (phase == kStart) {
      if (next == 0) {
        if (__hip_atomic_load(&st->alive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          st->phase = kDone;
        } else {
          // no vertex at this level: the next level is the smallest live degree
          st->level = __hip_atomic_load(&st->minv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else {
        st->cmax = level;
        st->qn = next;
        st->phase = kRound;
      }
    } else if (next == 0) {
      st->level = level + 1;
      st->phase = kStart;
    } else {
      st->cur = cur ^ 1;
      st->qn = next;
    }
    st->next = 0;
    st->alive = 0;
    st->minv = kIntMax;
    st->steps += 1;
    st->arrived = 0;
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
  a.take<CoreState>(1);
  return a.used;
}

int compute_core_numbers(const DevGraph& dg, int32_t* core, int32_t* cmax_out, Arena& a, hipStream_t s) {
  int32_t* deg = a.take<int32_t>((size_t)dg.n + 1);
  int32_t* q0 = a.take<int32_t>((size_t)dg.n + 1);
  int32_t* q1 = a.take<int32_t>((size_t)dg.n + 1);
  CoreState* st = a.take<CoreState>(1);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  *cmax_out = 0;
  if (dg.n == 0) return TRUSS_OK;
  hipLaunchKernelGGL(k_core_init, dim3(blocks(dg.n)), dim3(kT), 0, s, dg.row_ptr, dg.n, deg, core, st);
  // a level with takes costs its start, at most one empty start before it and
  // at most one sub-round per vertex taken: at most 3n + 1 steps in all (a
  // guard against a stuck loop)
  const long long max_steps = 4LL * dg.n + 2 * kStepsPerCheck;
  CoreState h;
  for (long long launched = 0;;) {
    for (int i = 0; i < kStepsPerCheck; ++i)
      hipLaunchKernelGGL(k_core_step, dim3(kStepBlocks), dim3(kT), 0, s, dg.row_ptr, dg.col, deg, core, dg.n, q0,
                         q1, st);
    launched += kStepsPerCheck;
    TRUSS_HIP(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    if (h.phase == kDone) break;
    if (launched > max_steps) {
      set_last_error("core numbers did not finish within %lld steps", max_steps);
      return TRUSS_E_INTERNAL;
    }
  }
  TRUSS_HIP(hipGetLastError());
  *cmax_out = h.cmax;
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
