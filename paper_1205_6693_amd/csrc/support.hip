// Support counting (Definition 1): sup(e) = number of triangles containing e.
//
// Every triangle {a, b, c} is listed exactly once through the (degree, id)
// orientation: with a before b before c, it is found from a as b in N+(a) and
// c in N+(a) ∩ N+(b).  This is the in-memory triangle counting that Algorithm 2,
// Step 2 relies on, and the orientation bounds |N+(a)| by 2*sqrt(m) as in the
// proof of Theorem 1, so N+(a) fits in LDS for every vertex of the target
// graphs.  The three edges of a found triangle get +1: (a,b) and (a,c) in LDS
// counters private to the workgroup that owns a (flushed once per edge), and
// (b,c) with one device-scope atomic.
//
// Work decomposition: vertices with |N+(a)| >= 2 are binned by |N+(a)|; a
// wavefront owns a vertex of the small bin, a workgroup one of the larger bins.
// The (b, c) pairs of a vertex are flattened (prefix sums over |N+(b)|) so the
// lanes stay busy whatever the individual out-degrees are.  Membership of c in
// N+(a) is an LDS hash probe (TRUSS_SUP_HASH) or a binary search of N+(a) in
// global memory (TRUSS_SUP_BSEARCH).  TRUSS_SUP_MERGE uses one lane per
// oriented edge and merges N+(a) with N+(b).
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kBins = 4;
constexpr int kWaveMax = 64;     // bin 0: 2 <= d <= 64, a wavefront per vertex
constexpr int kBlockMax1 = 1024; // bin 1: d <= 1024, a workgroup per vertex
constexpr int kBlockMax2 = 4096; // bin 2: d <= 4096, a workgroup per vertex
                                 // bin 3: larger, chunked binary search

enum { kHash = 0, kBsearch = 1 };

__device__ __forceinline__ uint32_t hslot(int32_t c, int logsz) {
  return ((uint32_t)c * 2654435769u) >> (32 - logsz);
}

struct SupCtl {
  int cnt[kBins];
  int fetch[kBins];
};

__global__ void k_sup_zero(int2* __restrict__ sr, int64_t m, SupCtl* ctl) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < m) sr[i] = make_int2(0, 0);
  if (i < kBins) { ctl->cnt[i] = 0; ctl->fetch[i] = 0; }
}

__global__ void k_sup_bin(const int64_t* __restrict__ orow, int32_t n, int32_t* __restrict__ vlist, SupCtl* ctl,
                          int all_bsearch) {
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int d = 0;
  if (a < n) d = (int)(orow[a + 1] - orow[a]);
  int bin = -1;
  if (d >= 2) bin = d <= kWaveMax ? 0 : d <= kBlockMax1 ? 1 : d <= kBlockMax2 ? 2 : 3;
  if (all_bsearch && bin > 0) bin = 3;
#pragma unroll
  for (int q = 0; q < kBins; ++q) {
    int pos = wave_append(&ctl->cnt[q], bin == q);
    if (bin == q) vlist[(int64_t)q * n + pos] = (int32_t)a;
  }
}

__device__ __forceinline__ int* sup_ptr(int2* sr, int32_t e) { return &sr[e].x; }

// ---- bin 0: a wavefront per vertex --------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(kT) k_sup_wave(const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol,
                                                 const int32_t* __restrict__ oeid, int32_t n,
                                                 const int32_t* __restrict__ vlist, SupCtl* ctl,
                                                 int2* __restrict__ sr) {
  constexpr int W = kT / kWave;
  __shared__ int s_nb[W][kWaveMax];
  __shared__ int s_cnt[W][kWaveMax];
  __shared__ int s_pre[W][kWaveMax + 1];
  __shared__ int64_t s_off[W][kWaveMax];
  __shared__ int s_tab[W][2 * kWaveMax];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int count = atomic_load_relaxed(&ctl->cnt[0]);
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = atomicAdd(&ctl->fetch[0], 1);
    idx = __shfl(idx, 0, kWave);
    if (idx >= count) break;
    const int32_t a = vlist[idx];
    const int64_t base = orow[a];
    const int d = (int)(orow[a + 1] - base);
    const bool valid = lane < d;
    const int32_t b = valid ? ocol[base + lane] : 0;
    const int64_t ob = valid ? orow[b] : 0;
    const int db = valid ? (int)(orow[b + 1] - ob) : 0;
    const int inc = wave_inclusive_sum(db);
    const int total = __shfl(inc, kWave - 1, kWave);
    if (valid) {
      s_nb[w][lane] = b;
      s_off[w][lane] = ob;
    }
    s_cnt[w][lane] = 0;
    s_pre[w][lane + 1] = inc;
    if (lane == 0) s_pre[w][0] = 0;
    if (MODE == kHash) {
      s_tab[w][lane] = -1;
      s_tab[w][lane + kWave] = -1;
    }
    wave_sync();
    if (MODE == kHash && valid) {
      uint32_t h = hslot(b, 7);
      while (atomicCAS(&s_tab[w][h], -1, lane) != -1) h = (h + 1) & 127;
    }
    wave_sync();
    for (int t0 = 0; t0 < total; t0 += kWave) {
      const int t = t0 + lane;
      if (t < total) {
        int lo = 0, hi = d;  // last i with pre[i] <= t
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_pre[w][mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int i = lo;
        const int64_t j = s_off[w][i] + (t - s_pre[w][i]);
        const int32_t c = ocol[j];
        int p = -1;
        if (MODE == kHash) {
          uint32_t h = hslot(c, 7);
          for (;;) {
            const int x = s_tab[w][h];
            if (x < 0) break;
            if (s_nb[w][x] == c) { p = x; break; }
            h = (h + 1) & 127;
          }
        } else {
          const int64_t q = lower_bound_i32<int64_t>(ocol, base, base + d, c);
          if (q < base + d && ocol[q] == c) p = (int)(q - base);
        }
        if (p >= 0) {
          atomicAdd(&s_cnt[w][i], 1);
          atomicAdd(&s_cnt[w][p], 1);
          atomicAdd(sup_ptr(sr, oeid[j]), 1);
        }
      }
    }
    wave_sync();
    if (valid) {
      const int cc = s_cnt[w][lane];
      if (cc) atomicAdd(sup_ptr(sr, oeid[base + lane]), cc);
    }
    wave_sync();
  }
}

// ---- bins 1, 2: a workgroup per vertex, N+(a) staged in LDS --------------------------------
template <int MODE, int MAXD>
__global__ void __launch_bounds__(kT) k_sup_block(const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol,
                                                  const int32_t* __restrict__ oeid, int32_t n,
                                                  const int32_t* __restrict__ vlist, int bin, SupCtl* ctl,
                                                  int2* __restrict__ sr) {
  constexpr int TAB = 2 * MAXD;
  constexpr int LOGTAB = MAXD == 1024 ? 11 : 13;
  __shared__ int s_nb[MAXD];
  __shared__ int s_cnt[MAXD];
  __shared__ int s_pre[MAXD + 1];
  __shared__ int64_t s_off[MAXD];
  __shared__ int s_tab[MODE == kHash ? TAB : 1];
  __shared__ int s_wt[kT / kWave];
  __shared__ int s_idx;
  const int count = atomic_load_relaxed(&ctl->cnt[bin]);
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(&ctl->fetch[bin], 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= count) break;
    const int32_t a = vlist[(int64_t)bin * n + idx];
    const int64_t base = orow[a];
    const int d = (int)(orow[a + 1] - base);
    // stage N+(a), |N+(b)| prefix sums
    int run = 0;
    for (int c0 = 0; c0 < d; c0 += kT) {
      const int i = c0 + threadIdx.x;
      const bool valid = i < d;
      int db = 0;
      if (valid) {
        const int32_t b = ocol[base + i];
        const int64_t ob = orow[b];
        db = (int)(orow[b + 1] - ob);
        s_nb[i] = b;
        s_off[i] = ob;
        s_cnt[i] = 0;
      }
      const int inc = wave_inclusive_sum(db);
      const int w = threadIdx.x / kWave;
      if (lane_id() == kWave - 1) s_wt[w] = inc;
      __syncthreads();
      int wbase = 0, ctot = 0;
      for (int q = 0; q < kT / kWave; ++q) {
        const int x = s_wt[q];
        if (q < w) wbase += x;
        ctot += x;
      }
      if (valid) s_pre[i + 1] = run + wbase + inc;
      run += ctot;
      __syncthreads();
    }
    if (threadIdx.x == 0) s_pre[0] = 0;
    if (MODE == kHash) {
      for (int i = threadIdx.x; i < TAB; i += kT) s_tab[i] = -1;
      __syncthreads();
      for (int i = threadIdx.x; i < d; i += kT) {
        uint32_t h = hslot(s_nb[i], LOGTAB);
        while (atomicCAS(&s_tab[h], -1, i) != -1) h = (h + 1) & (TAB - 1);
      }
    }
    __syncthreads();
    const int total = run;
    for (int t = threadIdx.x; t < total; t += kT) {
      int lo = 0, hi = d;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= t) lo = mid; else hi = mid - 1;
      }
      const int i = lo;
      const int64_t j = s_off[i] + (t - s_pre[i]);
      const int32_t c = ocol[j];
      int p = -1;
      if (MODE == kHash) {
        uint32_t h = hslot(c, LOGTAB);
        for (;;) {
          const int x = s_tab[h];
          if (x < 0) break;
          if (s_nb[x] == c) { p = x; break; }
          h = (h + 1) & (TAB - 1);
        }
      } else {
        const int64_t q = lower_bound_i32<int64_t>(ocol, base, base + d, c);
        if (q < base + d && ocol[q] == c) p = (int)(q - base);
      }
      if (p >= 0) {
        atomicAdd(&s_cnt[i], 1);
        atomicAdd(&s_cnt[p], 1);
        atomicAdd(sup_ptr(sr, oeid[j]), 1);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += kT) {
      const int cc = s_cnt[i];
      if (cc) atomicAdd(sup_ptr(sr, oeid[base + i]), cc);
    }
    __syncthreads();
  }
}

// ---- bin 3: a workgroup per vertex, N+(a) searched in global memory, chunks of 256 b's --------
__global__ void __launch_bounds__(kT) k_sup_chunked(const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol,
                                                    const int32_t* __restrict__ oeid, int32_t n,
                                                    const int32_t* __restrict__ vlist, SupCtl* ctl,
                                                    int2* __restrict__ sr) {
  __shared__ int s_cnt[kT];
  __shared__ int s_pre[kT + 1];
  __shared__ int64_t s_off[kT];
  __shared__ int s_wt[kT / kWave];
  __shared__ int s_idx;
  const int count = atomic_load_relaxed(&ctl->cnt[3]);
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(&ctl->fetch[3], 1);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= count) break;
    const int32_t a = vlist[(int64_t)3 * n + idx];
    const int64_t base = orow[a];
    const int d = (int)(orow[a + 1] - base);
    for (int c0 = 0; c0 < d; c0 += kT) {
      const int i = c0 + threadIdx.x;
      const bool valid = i < d;
      int db = 0;
      if (valid) {
        const int32_t b = ocol[base + i];
        const int64_t ob = orow[b];
        db = (int)(orow[b + 1] - ob);
        s_off[threadIdx.x] = ob;
      }
      s_cnt[threadIdx.x] = 0;
      const int inc = wave_inclusive_sum(db);
      const int w = threadIdx.x / kWave;
      if (lane_id() == kWave - 1) s_wt[w] = inc;
      __syncthreads();
      int wbase = 0, ctot = 0;
      for (int q = 0; q < kT / kWave; ++q) {
        const int x = s_wt[q];
        if (q < w) wbase += x;
        ctot += x;
      }
      s_pre[threadIdx.x + 1] = wbase + inc;
      if (threadIdx.x == 0) s_pre[0] = 0;
      __syncthreads();
      const int nb = d - c0 < kT ? d - c0 : kT;
      for (int t = threadIdx.x; t < ctot; t += kT) {
        int lo = 0, hi = nb;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const int64_t j = s_off[lo] + (t - s_pre[lo]);
        const int32_t c = ocol[j];
        const int64_t q = lower_bound_i32<int64_t>(ocol, base, base + d, c);
        if (q < base + d && ocol[q] == c) {
          atomicAdd(&s_cnt[lo], 1);
          atomicAdd(sup_ptr(sr, oeid[q]), 1);
          atomicAdd(sup_ptr(sr, oeid[j]), 1);
        }
      }
      __syncthreads();
      if (valid && s_cnt[threadIdx.x]) atomicAdd(sup_ptr(sr, oeid[base + i]), s_cnt[threadIdx.x]);
      __syncthreads();
    }
  }
}

// ---- merge: one lane per oriented edge a->b, two-pointer merge of N+(a) and N+(b) ------------
__global__ void __launch_bounds__(kT) k_sup_merge(const int64_t* __restrict__ row_ptr,
                                                  const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol,
                                                  const int32_t* __restrict__ oeid, const int32_t* __restrict__ eu,
                                                  const int32_t* __restrict__ ev, int64_t m, int2* __restrict__ sr) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t u = eu[e], v = ev[e];
  const bool ub = vertex_before(row_ptr[u + 1] - row_ptr[u], u, row_ptr[v + 1] - row_ptr[v], v);
  const int32_t a = ub ? u : v, b = ub ? v : u;
  int64_t i = orow[a], ie = orow[a + 1], j = orow[b], je = orow[b + 1];
  int cnt = 0;
  while (i < ie && j < je) {
    const int32_t ci = ocol[i], cj = ocol[j];
    if (ci < cj) ++i;
    else if (ci > cj) ++j;
    else {
      ++cnt;
      atomicAdd(sup_ptr(sr, oeid[i]), 1);
      atomicAdd(sup_ptr(sr, oeid[j]), 1);
      ++i; ++j;
    }
  }
  if (cnt) atomicAdd(sup_ptr(sr, (int32_t)e), cnt);
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

struct SupLayout {
  SupCtl* ctl;
  int32_t* vlist;
};

void carve(const DevGraph& dg, Arena& a, SupLayout& L) {
  L.ctl = a.take<SupCtl>(1);
  L.vlist = a.take<int32_t>((size_t)kBins * (dg.n + 1));
}

}  // namespace

size_t support_workspace(const DevGraph& dg, Arena& a) {
  SupLayout L;
  carve(dg, a, L);
  return a.used;
}

int compute_support(const DevGraph& dg, int strategy, int2* sr, Arena& a, hipStream_t s) {
  SupLayout L;
  carve(dg, a, L);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  const int64_t m = dg.m;
  const int32_t n = dg.n;
  hipLaunchKernelGGL(k_sup_zero, dim3(grid_for(m > kBins ? m : kBins)), dim3(kT), 0, s, sr, m, L.ctl);
  if (m == 0) return TRUSS_OK;
  if (strategy == TRUSS_SUP_MERGE) {
    hipLaunchKernelGGL(k_sup_merge, dim3(grid_for(m)), dim3(kT), 0, s, dg.row_ptr, dg.orow, dg.ocol, dg.oeid, dg.eu, dg.ev, m,
                       sr);
    TRUSS_HIP(hipGetLastError());
    return TRUSS_OK;
  }
  const bool bs = strategy == TRUSS_SUP_BSEARCH;
  hipLaunchKernelGGL(k_sup_bin, dim3(grid_for(n)), dim3(kT), 0, s, dg.orow, n, L.vlist, L.ctl, bs ? 1 : 0);
  // persistent-style grids: workers fetch vertices from the bin lists
  const unsigned gw = 256 * 8, gb = 256 * 4;
  if (bs) {
    hipLaunchKernelGGL(k_sup_wave<kBsearch>, dim3(gw), dim3(kT), 0, s, dg.orow, dg.ocol, dg.oeid, n, L.vlist, L.ctl,
                       sr);
  } else {
    hipLaunchKernelGGL(k_sup_wave<kHash>, dim3(gw), dim3(kT), 0, s, dg.orow, dg.ocol, dg.oeid, n, L.vlist, L.ctl, sr);
    hipLaunchKernelGGL((k_sup_block<kHash, kBlockMax1>), dim3(gb), dim3(kT), 0, s, dg.orow, dg.ocol, dg.oeid, n,
                       L.vlist, 1, L.ctl, sr);
    hipLaunchKernelGGL((k_sup_block<kHash, kBlockMax2>), dim3(256), dim3(kT), 0, s, dg.orow, dg.ocol, dg.oeid, n,
                       L.vlist, 2, L.ctl, sr);
  }
  hipLaunchKernelGGL(k_sup_chunked, dim3(256), dim3(kT), 0, s, dg.orow, dg.ocol, dg.oeid, n, L.vlist, L.ctl, sr);
  TRUSS_HIP(hipGetLastError());
  return TRUSS_OK;
}

}  // namespace truss
