// Algorithm 1 (Cohen's truss decomposition, Section 3.1) on the device, as a
// comparator for the in-memory path of Algorithm 2.
//
// Support: sup(e) = |nb(u) ∩ nb(v)| by merging the two full sorted
// rows.  Peeling: for k = 3, 4, ... every edge with sup < k-2
// leaves (its truss number is k-1); W = nb(u) ∩ nb(v) is again a merge of the
// two full rows, reading removed edges as deleted (the implicit deletion of
// Section 3.1: rows are never compacted), and the two other edges of each
// triangle lose one.  Both merges cost deg(u) + deg(v) per edge, which is what
// separates Algorithm 1 from Algorithm 2 (Section 3.2): summed over the edges
// that is the sum over vertices of deg(v)^2, and the counters below report it.
//
// Removal is level-synchronous like the main path: round r takes a frontier
// snapshot (stamp r); a triangle with no edge removed before round r and at
// least one frontier edge is destroyed by its frontier edge of smallest id,
// which decrements each of its other edges that is not in the frontier once.
// An edge whose support falls from k-2 to k-3 joins the next round.
//
// One wavefront per edge; a merge of lengths a and b is split over the 64
// lanes by merge path (each lane binary-searches its diagonal, then merges
// (a + b) / 64 steps).
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kIntMax = 0x7fffffff;

struct CohenCtl {
  int qn;                   // next-frontier length
  int live;                 // live edges seen by a level start
  int minsup;               // their smallest support
  int pad;
  unsigned long long work;  // row entries merged
};

inline unsigned grid_for(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : (b > 65535 * 4 ? 65535 * 4 : b));
}

__device__ __forceinline__ int ld_stamp(const int2* p) {
  return __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Visits the common entries of the sorted rows col[a0, a1) and col[b0, b1):
// f(ja, jb) with col[ja] == col[jb].  Wave-cooperative (every lane calls it
// with the same rows); each match is visited by exactly one lane.
template <typename F>
__device__ __forceinline__ void wave_merge_common(const int32_t* __restrict__ col, int64_t a0, int64_t a1, int64_t b0,
                                                  int64_t b1, F&& f) {
  const int64_t la = a1 - a0, lb = b1 - b0, len = la + lb;
  const int64_t per = (len + kWave - 1) / kWave;
  const int lane = lane_id();
  const int64_t d0 = lane * per < len ? lane * per : len;
  const int64_t d1 = d0 + per < len ? d0 + per : len;
  if (d0 >= d1) return;
  // merge-path split at diagonal d0 (ties take A first)
  int64_t lo = d0 - lb > 0 ? d0 - lb : 0, hi = d0 < la ? d0 : la;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[a0 + mid] <= col[b0 + d0 - mid - 1]) lo = mid + 1;
    else hi = mid;
  }
  int64_t i = lo, j = d0 - lo;
  int32_t bj = j < lb ? col[b0 + j] : kIntMax;
  for (int64_t t = d0; t < d1; ++t) {
    if (i < la) {
      const int32_t ai = col[a0 + i];
      if (ai <= bj) {  // A's element is consumed; a match is counted here
        if (ai == bj) f(a0 + i, b0 + j);
        ++i;
        continue;
      }
    }
    ++j;
    bj = j < lb ? col[b0 + j] : kIntMax;
  }
}

__global__ void __launch_bounds__(kT) k_cohen_support(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, const int32_t* __restrict__ eu,
                                                      const int32_t* __restrict__ ev, int64_t m,
                                                      int2* __restrict__ sr, CohenCtl* c) {
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  unsigned long long work = 0;
  for (int64_t e = gw; e < m; e += nw) {
    const int32_t u = eu[e], v = ev[e];
    const int64_t a0 = row_ptr[u], a1 = row_ptr[u + 1], b0 = row_ptr[v], b1 = row_ptr[v + 1];
    int cnt = 0;
    wave_merge_common(col, a0, a1, b0, b1, [&](int64_t, int64_t) { ++cnt; });
    cnt = wave_sum(cnt);
    if (lane_id() == 0) sr[e] = make_int2(cnt, 0);
    work += (unsigned long long)((a1 - a0) + (b1 - b0));
  }
  if (lane_id() == 0 && work) atomicAdd(&c->work, work);
}

__global__ void k_cohen_reset(CohenCtl* c, int full) {
  if (threadIdx.x == 0) {
    c->qn = 0;
    c->live = 0;
    c->minsup = kIntMax;
    if (full) c->work = 0ULL;
  }
}

// Level start (a new k): live edges with sup < k-2 form the frontier
// of round r; also counts the live edges left and their smallest support.
__global__ void __launch_bounds__(kT) k_cohen_start(int2* __restrict__ sr, int64_t m, int k, int r,
                                                    int32_t* __restrict__ q, int32_t* __restrict__ truss,
                                                    CohenCtl* c) {
  __shared__ int s_live[kT / kWave], s_min[kT / kWave];
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool take = false;
  int live = 0, mins = kIntMax;
  if (e < m) {
    const int2 s = sr[e];
    if (s.y == 0) {
      if (s.x < k - 2) {
        take = true;
        sr[e].y = r;
        truss[e] = k - 1;
      } else {
        live = 1;
        mins = s.x;
      }
    }
  }
  const int pos = wave_append(&c->qn, take);
  if (take) q[pos] = (int32_t)e;
  live = wave_sum(live);
  mins = wave_min(mins);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    s_live[w] = live;
    s_min[w] = mins;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = kIntMax;
    for (int i = 0; i < kT / kWave; ++i) {
      a += s_live[i];
      b = s_min[i] < b ? s_min[i] : b;
    }
    if (a) atomicAdd(&c->live, a);
    if (b != kIntMax) atomicMin(&c->minsup, b);
  }
}

// One round: every frontier edge (stamp r) finds W by merging the full rows
// and breaks the triangles it owns.
__global__ void __launch_bounds__(kT) k_cohen_round(const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col, const int32_t* __restrict__ seid,
                                                    const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                                    int2* __restrict__ sr, const int32_t* __restrict__ q, int qn, int k,
                                                    int r, int32_t* __restrict__ nq, int32_t* __restrict__ truss,
                                                    CohenCtl* c) {
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  unsigned long long work = 0;
  for (int64_t i = gw; i < qn; i += nw) {
    const int32_t e = q[i];
    const int32_t u = eu[e], v = ev[e];
    const int64_t a0 = row_ptr[u], a1 = row_ptr[u + 1], b0 = row_ptr[v], b1 = row_ptr[v + 1];
    work += (unsigned long long)((a1 - a0) + (b1 - b0));
    wave_merge_common(col, a0, a1, b0, b1, [&](int64_t ja, int64_t jb) {
      const int32_t e1 = seid[ja], e2 = seid[jb];
      const int s1 = ld_stamp(&sr[e1]), s2 = ld_stamp(&sr[e2]);
      if ((s1 != 0 && s1 < r) || (s2 != 0 && s2 < r)) return;  // destroyed in an earlier round
      if ((s1 == r && e1 < e) || (s2 == r && e2 < e)) return;  // another frontier edge owns it
      const int32_t f[2] = {e1, e2};
      const int sf[2] = {s1, s2};
      for (int t = 0; t < 2; ++t) {
        if (sf[t] == r) continue;
        const int old = atomicSub(&sr[f[t]].x, 1);
        if (old == k - 2) {  // sup falls below k-2: the edge joins the next round
          __hip_atomic_store(&sr[f[t]].y, r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          truss[f[t]] = k - 1;
          nq[atomicAdd(&c->qn, 1)] = f[t];
        }
      }
    });
  }
  if (lane_id() == 0 && work) atomicAdd(&c->work, work);
}

}  // namespace

size_t cohen_workspace(int64_t m, Arena& a) {
  a.take<int32_t>((size_t)m + 1);
  a.take<int32_t>((size_t)m + 1);
  a.take<CohenCtl>(1);
  return a.used;
}

int cohen_decompose(const DevGraph& dg, int2* sr, int32_t* truss, Arena& a, CohenResult* res, hipStream_t s) {
  int32_t* q[2] = {a.take<int32_t>((size_t)dg.m + 1), a.take<int32_t>((size_t)dg.m + 1)};
  CohenCtl* c = a.take<CohenCtl>(1);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  *res = CohenResult();
  if (dg.m == 0) return TRUSS_OK;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (auto& x : ev) TRUSS_HIP(hipEventCreate(&x));
  CohenCtl h;
  hipLaunchKernelGGL(k_cohen_reset, dim3(1), dim3(64), 0, s, c, 1);
  TRUSS_HIP(hipEventRecord(ev[0], s));
  const int64_t waves = dg.m < 262144 ? dg.m : 262144;
  hipLaunchKernelGGL(k_cohen_support, dim3(grid_for(waves * kWave)), dim3(kT), 0, s, dg.row_ptr, dg.col, dg.eu,
                     dg.ev, dg.m, sr, c);
  TRUSS_HIP(hipEventRecord(ev[1], s));
  TRUSS_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  res->support_work = (int64_t)h.work;
  int k = 3, r = 1, kmax = 2;
  for (;;) {
    hipLaunchKernelGGL(k_cohen_reset, dim3(1), dim3(64), 0, s, c, 0);
    hipLaunchKernelGGL(k_cohen_start, dim3((unsigned)((dg.m + kT - 1) / kT)), dim3(kT), 0, s, sr, dg.m, k, r, q[0],
                       truss, c);
    TRUSS_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    if (h.qn == 0) {
      if (h.live == 0) break;
      k = h.minsup + 3;  // the live edges form the (k-1)-truss for every k up to minsup + 2
      continue;
    }
    kmax = k - 1;
    res->levels += 1;
    int cur = 0, qn = h.qn;
    while (qn > 0) {
      hipLaunchKernelGGL(k_cohen_reset, dim3(1), dim3(64), 0, s, c, 0);
      const int64_t w = qn < 262144 ? qn : 262144;
      hipLaunchKernelGGL(k_cohen_round, dim3(grid_for(w * kWave)), dim3(kT), 0, s, dg.row_ptr, dg.col, dg.seid,
                         dg.eu, dg.ev, sr, q[cur], qn, k, r, q[cur ^ 1], truss, c);
      TRUSS_HIP(hipMemcpyAsync(&h, c, sizeof(h), hipMemcpyDeviceToHost, s));
      TRUSS_HIP(hipStreamSynchronize(s));
      res->rounds += 1;
      cur ^= 1;
      qn = h.qn;
      r += 1;
    }
    r += 1;
    k += 1;  // the live edges now form the k-truss
  }
  TRUSS_HIP(hipEventRecord(ev[2], s));
  TRUSS_HIP(hipEventSynchronize(ev[2]));
  float t0 = 0.f, t1 = 0.f;
  (void)hipEventElapsedTime(&t0, ev[0], ev[1]);
  (void)hipEventElapsedTime(&t1, ev[1], ev[2]);
  for (auto& x : ev) (void)hipEventDestroy(x);
  res->ms_support = t0;
  res->ms_peel = t1;
  res->peel_work = (int64_t)h.work - res->support_work;
  res->kmax = kmax;
  TRUSS_HIP(hipGetLastError());
  return TRUSS_OK;
}

}  // namespace truss
