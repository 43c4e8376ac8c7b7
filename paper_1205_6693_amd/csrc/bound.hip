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
// k_hindex: a wavefront per vertex finds h by binary search over x in
// [0, deg], counting the row's supports >= x with ballots (rows of up to 64
// entries stay in registers).  k_psi: an edge a thread.
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;

__global__ void __launch_bounds__(kT) k_hindex(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ seid,
                                               const int2* __restrict__ sr, int32_t n, int32_t* __restrict__ h,
                                               int32_t* __restrict__ ch) {
  const int lane = lane_id();
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = gw; v < n; v += nw) {
    const int64_t rb = row_ptr[v];
    const int64_t d = row_ptr[v + 1] - rb;
    int64_t lo = 0, hi = d, cnt_lo = d;
    if (d <= kWave) {
      const int s = lane < d ? sr[seid[rb + lane]].x : -1;
      while (lo < hi) {
        const int64_t x = (lo + hi + 1) >> 1;
        const int64_t c = __popcll(ballot(s >= x));
        if (c >= x) lo = x; else hi = x - 1;
      }
      cnt_lo = __popcll(ballot(s >= lo));
    } else {
      auto count = [&](int64_t x) {
        int64_t c = 0;
        for (int64_t j0 = 0; j0 < d; j0 += kWave) {
          const int64_t j = j0 + lane;
          const bool ge = j < d && sr[seid[rb + j]].x >= x;
          c += __popcll(ballot(ge));
        }
        return c;
      };
      while (lo < hi) {
        const int64_t x = (lo + hi + 1) >> 1;
        if (count(x) >= x) lo = x; else hi = x - 1;
      }
      cnt_lo = count(lo);
    }
    if (lane == 0) {
      h[v] = (int32_t)lo;
      ch[v] = (int32_t)(cnt_lo < 0x7fffffff ? cnt_lo : 0x7fffffff);
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

void compute_upper_bound(const DevGraph& dg, const int2* sr, int32_t* h, int32_t* ch, int32_t* psi, hipStream_t s) {
  if (dg.m == 0) return;
  const unsigned gw = 256 * 8;
  hipLaunchKernelGGL(k_hindex, dim3(gw), dim3(kT), 0, s, dg.row_ptr, dg.seid, sr, dg.n, h, ch);
  const int64_t b = (dg.m + kT - 1) / kT;
  hipLaunchKernelGGL(k_psi, dim3((unsigned)b), dim3(kT), 0, s, dg.eu, dg.ev, sr, h, ch, dg.m, psi);
}

}  // namespace truss
