// Upper bound of the truss number (Procedure 6; Lemma 2: phi(e) <= psi(e)).
//
// psi(e) = min{sup(e), x_u, x_v} + 2, where x_w is the largest x such that at
// least x edges incident to w other than e have support >= x.  With h(w) the
// largest x such that at least x edges incident to w have support >= x (all of
// them, e included) and c(w) the number of incident edges with support >= h(w),
// leaving e out changes the answer only when e is one of exactly h(w) edges at
// or above h(w):
//   x_w = h(w) - 1  if sup(e) >= h(w) and c(w) == h(w),  else  x_w = h(w).
// (If c(w) > h(w), h(w) edges other than e still reach h(w); if sup(e) < h(w),
// e is not counted at h(w).  And h(w) - 1 is always reached: at least h(w) - 1
// other edges have support >= h(w) >= h(w) - 1.)
//
// k_hindex: a wavefront per vertex finds h and c (see below).  k_psi: an edge
// a thread.
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// h(v) and c(v) for every vertex.  Rows of up to 64 entries: binary search on
// x with ballots over registers.  Longer rows: counts of min(sup, deg) in the
// vertex's slice of hs (deg+1 counters starting at row_ptr[v] + v), then a
// scan from the top finds the largest y with at least y supports >= y.
__global__ void __launch_bounds__(kT) k_hindex(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ seid,
                                               const int2* __restrict__ sr, int32_t n, int32_t* __restrict__ h,
                                               int32_t* __restrict__ ch, int32_t* __restrict__ hs) {
  const int lane = lane_id();
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = gw; v < n; v += nw) {
    const int64_t rb = row_ptr[v];
    const int64_t d = row_ptr[v + 1] - rb;
    int64_t hv = 0, cv = 0;
    if (d <= kWave) {
      const int s = lane < d ? sr[seid[rb + lane]].x : -1;
      int64_t lo = 0, hi = d;
      while (lo < hi) {
        const int64_t x = (lo + hi + 1) >> 1;
        const int64_t c = __popcll(ballot(s >= x));
        if (c >= x) lo = x; else hi = x - 1;
      }
      hv = lo;
      cv = __popcll(ballot(s >= lo));
    } else {
      int32_t* cnt = hs + rb + v;  // d + 1 counters
      for (int64_t y = lane; y <= d; y += kWave) cnt[y] = 0;
      wait_memory();
      wave_sync();
      for (int64_t j = lane; j < d; j += kWave) {
        const int64_t sv = sr[seid[rb + j]].x;
        atomicAdd(&cnt[sv < d ? sv : d], 1);
      }
      wait_memory();
      wave_sync();
      // lane i of a step covers y = top - i; suffix counts accumulate downwards
      int64_t run = 0;
      for (int64_t top = d;; top -= kWave) {
        const int64_t y = top - lane;
        const int64_t c = y >= 0 ? __hip_atomic_load(&cnt[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        const int64_t suf = run + wave_inclusive_sum(c);
        const uint64_t ok = ballot(y >= 0 && suf >= y);
        if (ok) {
          const int first = __builtin_ctzll(ok);
          hv = __shfl(y, first, kWave);
          cv = __shfl(suf, first, kWave);
          break;
        }
        run = __shfl(suf, kWave - 1, kWave);
      }
    }
    if (lane == 0) {
      h[v] = (int32_t)hv;
      ch[v] = (int32_t)(cv < 0x7fffffff ? cv : 0x7fffffff);
    }
  }
}

__global__ void __launch_bounds__(kT) k_psi(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                                            const int2* __restrict__ sr, const int32_t* __restrict__ h,
                                            const int32_t* __restrict__ ch, int64_t m, int32_t* __restrict__ psi) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int s = sr[e].x;
  const int u = eu[e], v = ev[e];
  const int hu = h[u], hv = h[v];
  const int xu = (s >= hu && ch[u] == hu) ? hu - 1 : hu;
  const int xv = (s >= hv && ch[v] == hv) ? hv - 1 : hv;
  int x = s < xu ? s : xu;
  x = x < xv ? x : xv;
  psi[e] = x + 2;
}

}  // namespace

void compute_upper_bound(const DevGraph& dg, const int2* sr, int32_t* h, int32_t* ch, int32_t* psi, int32_t* hs,
                         hipStream_t s) {
  if (dg.m == 0) return;
  const unsigned gw = 256 * 8;
  hipLaunchKernelGGL(k_hindex, dim3(gw), dim3(kT), 0, s, dg.row_ptr, dg.seid, sr, dg.n, h, ch, hs);
  const int64_t b = (dg.m + kT - 1) / kT;
  hipLaunchKernelGGL(k_psi, dim3((unsigned)b), dim3(kT), 0, s, dg.eu, dg.ev, sr, h, ch, dg.m, psi);
}

}  // namespace truss
