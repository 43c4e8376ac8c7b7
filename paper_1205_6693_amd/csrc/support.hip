// Support counting (Definition 1): sup(e) = number of triangles containing e.
//
// Every triangle {a, b, c} is listed exactly once through the (degree, id)
// orientation: with a before b before c, it is found from a as b in N+(a) and
// c in N+(a) ∩ N+(b).  This is the in-memory triangle counting that Algorithm 2,
// starts from, and the orientation bounds |N+(a)| by 2*sqrt(m) as in the
// proof of Theorem 1, so N+(a) fits in LDS for every vertex of the target
// graphs.  The three edges of a found triangle get +1: (a,b) and (a,c) in LDS
// counters private to the workgroup that owns a (flushed once per edge), and
// (b,c) with one device-scope atomic.
//
// Work decomposition: vertices with |N+(a)| >= 2 are binned by |N+(a)|; a
// wavefront owns a vertex of the small bin, a workgroup one of the larger bins.
// The (b, c) pairs of a vertex are flattened (prefix sums over |N+(b)|) so the
// lanes stay busy whatever the individual out-degrees are.  Each bin takes one
// of three intersection methods, chosen per bin on the device (k_sup_decide):
// membership of c in N+(a) by an LDS hash probe, by a binary search of N+(a)
// in global memory, or a merge of N+(a) with N+(b), one lane per oriented edge
// a -> b.  The kernels of the methods not chosen exit at once.
//
// Counts accumulate by position in the oriented CSR (an edge a -> b at
// position j of ocol counts into supo[j]): the pairs (b, c) a wavefront walks
// sit at consecutive positions of N+(b), so their increments land on the same
// few lines, and the per-vertex flushes of the (a, b), (a, c) counts are
// contiguous.  One pass at the end moves supo into edge-id order.
#include "common.hpp"
#include "internal.hpp"
#include "mlp.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kBins = 4;
constexpr int kWaveMax = 64;     // bin 0: 2 <= d <= 64, a wavefront per vertex
constexpr int kBlockMax1 = 1024; // bin 1: d <= 1024, a workgroup per vertex
constexpr int kBlockMax2 = 4096; // bin 2: d <= 4096, a workgroup per vertex
                                 // bin 3: larger, chunked binary search

static_assert(kBins == kSupBins, "support bins");

// bin actions (the scheduler's support outputs)
enum { kHash = 0, kBsearch = 1, kMerge = 2 };

__device__ __forceinline__ uint32_t hslot(int32_t c, int logsz) {
  return ((uint32_t)c * 2654435769u) >> (32 - logsz);
}

struct SupCtl {
  int cnt[kBins];    // vertices per bin
  int fetch[kBins];  // next vertex of the bin to take
  int act[kBins];    // method chosen for the bin
  unsigned long long sd[kBins], sd2[kBins];  // sum of d+ and of d+^2 over the bin
  float feat[kBins][kSupF];                  // the decision's features
};

__global__ void k_sup_zero(int32_t* __restrict__ supo, int64_t m, SupCtl* ctl) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < m) supo[i] = 0;
  if (i < kBins) {
    ctl->cnt[i] = 0;
    ctl->fetch[i] = 0;
    ctl->act[i] = 0;
    ctl->sd[i] = 0ULL;
    ctl->sd2[i] = 0ULL;
  }
}

// Bins the vertices by d+ = |N+(a)| and sums d+ and d+^2 per bin; counts are
// gathered per wavefront, then per workgroup, so each bin counter sees one
// atomic per workgroup.  A bin's list comes out roughly in id order; with ids
// ranked by degree, the hash kernels take it backwards, so the vertices with
// the most pairs start first and the short ones fill the tail.
constexpr int kBinT = 1024;
__global__ void __launch_bounds__(kBinT) k_sup_bin(const int64_t* __restrict__ orow, int32_t n,
                                                   int32_t* __restrict__ vlist, SupCtl* ctl) {
  __shared__ int s_c[kBins], s_base[kBins];
  __shared__ unsigned long long s_d[kBins], s_d2[kBins];
  if (threadIdx.x < kBins) {
    s_c[threadIdx.x] = 0;
    s_d[threadIdx.x] = 0ULL;
    s_d2[threadIdx.x] = 0ULL;
  }
  __syncthreads();
  const int64_t a = blockIdx.x * (int64_t)kBinT + threadIdx.x;
  int d = 0;
  if (a < n) d = (int)(orow[a + 1] - orow[a]);
  int bin = -1;
  if (d >= 2) bin = d <= kWaveMax ? 0 : d <= kBlockMax1 ? 1 : d <= kBlockMax2 ? 2 : 3;
  int local = 0;
  const int lane = lane_id();
#pragma unroll
  for (int q = 0; q < kBins; ++q) {
    const uint64_t msk = ballot(bin == q);
    if (msk == 0) continue;
    const unsigned long long x = bin == q ? (unsigned long long)d : 0ULL;
    const unsigned long long sd = wave_sum(x), sd2 = wave_sum(x * x);
    const int leader = __builtin_ctzll(msk);
    int wb = 0;
    if (lane == leader) {
      wb = atomicAdd(&s_c[q], __popcll(msk));
      atomicAdd(&s_d[q], sd);
      atomicAdd(&s_d2[q], sd2);
    }
    wb = __shfl(wb, leader, kWave);
    if (bin == q) local = wb + rank_below(msk);
  }
  __syncthreads();
  if (threadIdx.x < kBins) {
    const int q = threadIdx.x;
    if (s_c[q] > 0) {
      s_base[q] = atomicAdd(&ctl->cnt[q], s_c[q]);
      atomicAdd(&ctl->sd[q], s_d[q]);
      atomicAdd(&ctl->sd2[q], s_d2[q]);
    }
  }
  __syncthreads();
  if (bin >= 0) vlist[(int64_t)bin * n + s_base[bin] + local] = (int32_t)a;
}

// One wavefront per bin picks the bin's method.  force >= 0: that method for
// every bin (hash becomes binary search in the last bin); otherwise by
// scheduler: plain = merge; heuristic = hash, binary search in the last bin;
// learned = the allowed method with the smallest model score if that score is
// below the heuristic method's by more than kSupMargin (log2 ms), else the
// heuristic method.
constexpr float kSupMargin = 0.25f;
__global__ void __launch_bounds__(kBins * kWave) k_sup_decide(SupCtl* ctl, int64_t m, int sched, int force,
                                                               const float* __restrict__ model) {
  const int b = threadIdx.x / kWave;
  const int lane = lane_id();
  const float cnt = (float)ctl->cnt[b];
  const float sd = (float)ctl->sd[b], sd2 = (float)ctl->sd2[b];
  float x[kSupF];
  x[0] = log2f(1.f + cnt);
  x[1] = log2f(1.f + sd);
  x[2] = log2f(1.f + sd2);
  x[3] = log2f(1.f + sd / (cnt > 1.f ? cnt : 1.f));
  x[4] = log2f(1.f + (float)m);
  x[5] = log2f(1.f + sd2 / (sd > 1.f ? sd : 1.f));
  const unsigned allowed = b == kBins - 1 ? 0x6u : 0x7u;
  int act;
  if (force >= 0) {
    act = (force == kHash && b == kBins - 1) ? kBsearch : force;
  } else if (sched == TRUSS_SCHED_PLAIN) {
    act = kMerge;
  } else if (sched == TRUSS_SCHED_LEARNED && model != nullptr) {
    // the network's choice replaces the heuristic's only when it predicts a
    // clear gain (a bin decides a large share of the support time at once)
    float sc[kSupA];
    mlp_scores_wave(model, x, sc);
    const int best = argmin_allowed(sc, kSupA, allowed);
    const int pref = b == kBins - 1 ? kBsearch : kHash;
    act = sc[best] < sc[pref] - kSupMargin ? best : pref;
  } else {
    act = b == kBins - 1 ? kBsearch : kHash;
  }
  if (lane == 0) {
    ctl->act[b] = act;
    for (int i = 0; i < kSupF; ++i) ctl->feat[b][i] = x[i];
  }
}

// sup(e) in edge-id order, round stamp 0, from the counts by oriented position
__global__ void k_sup_finish(const int32_t* __restrict__ supo, const int32_t* __restrict__ oeid, int64_t m,
                             int2* __restrict__ sr) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < m) sr[oeid[j]] = make_int2(supo[j], 0);
}

// ---- the hash method: N+(a) in an LDS hash table, the (b, c) pairs walked by
// wavefronts in windows of 64 consecutive pairs -----------------------------------------
// Rows of the walk are the b in N+(a) with |N+(b)| > 0, in N+(a) order; row k
// covers pairs [pre[k], pre[k+1]), its pair t is c = ocol[offj[k] + t], and
// wi[k] is the position of b in N+(a).  The table maps c to its position in
// N+(a) (key -1: empty slot).
struct WalkTabs {
  const int* pre;   // nrows + 1
  const int* offj;  // nrows
  const int* wi;    // nrows
  const int2* tab;  // (key, position), 2^LOGTAB slots, linear probing
  int* cnt;         // per position of N+(a): triangles found on (a, that vertex)
  int* own;         // 64 ints private to the wavefront
};

template <int LOGTAB>
__device__ __forceinline__ void tab_insert(int2* tab, int32_t key, int pos) {
  uint32_t h = hslot(key, LOGTAB);
  while (atomicCAS(&tab[h].x, -1, key) != -1) h = (h + 1) & ((1u << LOGTAB) - 1);
  tab[h].y = pos;
}

template <int LOGTAB>
__device__ __forceinline__ int tab_find(const int2* tab, int32_t key) {
  uint32_t h = hslot(key, LOGTAB);
  for (;;) {
    const int2 x = tab[h];
    if (x.x == key) return x.y;
    if (x.x < 0) return -1;
    h = (h + 1) & ((1u << LOGTAB) - 1);
  }
}

// Inclusive maximum over the lanes 0..lane (DPP row shifts within rows of 16,
// then the row broadcasts 15 and 31 of the gfx9 wave64 scan).
__device__ __forceinline__ int wave_incl_max(int x) {
  constexpr int lo = (int)0x80000000;
  int y;
  y = __builtin_amdgcn_update_dpp(lo, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x = y > x ? y : x;
  y = __builtin_amdgcn_update_dpp(lo, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x = y > x ? y : x;
  y = __builtin_amdgcn_update_dpp(lo, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x = y > x ? y : x;
  y = __builtin_amdgcn_update_dpp(lo, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x = y > x ? y : x;
  y = __builtin_amdgcn_update_dpp(lo, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x = y > x ? y : x;
  y = __builtin_amdgcn_update_dpp(lo, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  x = y > x ? y : x;
  return x;
}

// One wavefront walks pairs [lo, hi) of a vertex's flattened list, 64 pairs
// (one per lane) a window.  Every lane needs the row of its pair.  Inside a
// row (the common case: most pairs lie in long rows) that is the row in
// progress, and kU windows are taken together so that their loads are in
// flight at once; the triangles found on (a, b) of that row are summed in a
// register and added to its LDS count when the row ends.  A window where rows
// start has each starting row mark its first pair in the wavefront's `own`
// array, and an inclusive maximum scan carries each row over the pairs that
// follow it.
constexpr int kU = 4;
template <int LOGTAB>
__device__ void walk_pairs(const WalkTabs& W, int nrows, int lo, int hi, const int32_t* __restrict__ ocol,
                           int32_t* __restrict__ supo) {
  if (lo >= hi || nrows <= 0) return;
  const int lane = lane_id();
  // kc: the row holding pair lo - 1 (the last row starting at or before it), -1 if none
  int x = -1, y = nrows - 1;
  while (x < y) {
    const int mid = (x + y + 1) >> 1;
    if (W.pre[mid] <= lo - 1) x = mid; else y = mid - 1;
  }
  int kc = x;
  int nx = kc + 1 < nrows ? W.pre[kc + 1] : 0x7fffffff;  // first pair of row kc + 1
  int oj = kc >= 0 ? W.offj[kc] : 0;                    // pair t of row kc: ocol[oj + t]
  int acc = 0;                                          // triangles on (a, row kc's b) not yet counted
  int t0 = lo;
  while (t0 < hi) {
    if (nx >= t0 + kU * kWave) {
      // kU windows inside row kc
      int32_t c[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int t = t0 + u * kWave + lane;
        c[u] = t < hi ? ocol[(int64_t)oj + t] : -1;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int t = t0 + u * kWave + lane;
        bool hit = false;
        if (c[u] >= 0) {
          const int pos = tab_find<LOGTAB>(W.tab, c[u]);
          if (pos >= 0) {
            hit = true;
            atomicAdd(&W.cnt[pos], 1);
            atomicAdd(&supo[(int64_t)oj + t], 1);
          }
        }
        acc += __popcll(ballot(hit));
      }
      t0 += kU * kWave;
      continue;
    }
    if (nx >= t0 + kWave) {
      // one window inside row kc
      const int t = t0 + lane;
      bool hit = false;
      if (t < hi) {
        const int pos = tab_find<LOGTAB>(W.tab, ocol[(int64_t)oj + t]);
        if (pos >= 0) {
          hit = true;
          atomicAdd(&W.cnt[pos], 1);
          atomicAdd(&supo[(int64_t)oj + t], 1);
        }
      }
      acc += __popcll(ballot(hit));
      t0 += kWave;
      continue;
    }
    // rows start inside the window: settle row kc's count, then find each
    // lane's row
    if (lane == 0 && acc && kc >= 0) atomicAdd(&W.cnt[W.wi[kc]], acc);
    acc = 0;
    const int idx = kc + 1 + lane;
    const int p = idx < nrows ? W.pre[idx] : 0x7fffffff;
    wave_sync();
    W.own[lane] = -1;
    wave_sync();
    if (p < t0 + kWave) W.own[p - t0] = idx;  // rows after kc start at or after t0
    wave_sync();
    int o = W.own[lane];
    o = o > kc ? o : kc;
    o = wave_incl_max(o);
    o = o < 0 ? 0 : o >= nrows ? nrows - 1 : o;
    const int t = t0 + lane;
    if (t < hi) {
      const int64_t j = (int64_t)W.offj[o] + t;
      const int pos = tab_find<LOGTAB>(W.tab, ocol[j]);
      if (pos >= 0) {
        atomicAdd(&W.cnt[pos], 1);
        atomicAdd(&supo[j], 1);
        atomicAdd(&W.cnt[W.wi[o]], 1);
      }
    }
    kc = __shfl(o, kWave - 1, kWave);
    nx = kc + 1 < nrows ? W.pre[kc + 1] : 0x7fffffff;
    oj = W.offj[kc];
    t0 += kWave;
  }
  if (lane == 0 && acc && kc >= 0) atomicAdd(&W.cnt[W.wi[kc]], acc);
}

// Stages N+(a) for the hash method: the table, the list nb, zeroed counts and
// the rows.  A b with |N+(b)| > kRev |N+(a)| is a searched row instead of a
// walked one: rather than walking its pairs, each c in N+(a) is looked up in
// the sorted N+(b) (see search_rows).  Walked rows (non-empty, compacted by a
// scan) fill pre, offj, wi from index 0; searched rows fill them from the top
// (searched row r: position wi[MAXD-1-r], N+(b) at ocol[offj[MAXD-1-r] ..] of
// length pre[MAXD-r]); as walked + searched <= |N+(a)| <= MAXD they never
// meet.  nth threads take part (a wavefront or the whole workgroup; scratch:
// NTH / kWave entries); *nrev (LDS, zero on entry) receives the searched rows.
// Returns the number of walked rows; pre[nrows] is the number of their pairs.
constexpr int kRev = 8;
template <int LOGTAB, int NTH, int MAXD>
__device__ int stage_rows(const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol, int64_t base, int d,
                          int2* tab, int* nb, int* pre, int* offj, int* wi, int* cnt, int* nrev,
                          unsigned long long* scratch) {
  const int tid = NTH == kWave ? lane_id() : (int)threadIdx.x;
  constexpr int NW = NTH / kWave;
  const int w = tid / kWave;
  for (int i = tid; i < (1 << LOGTAB); i += NTH) tab[i] = make_int2(-1, 0);
  if (NTH == kWave) wave_sync(); else __syncthreads();
  unsigned long long run = 0;  // (pairs << 32) | rows over the chunks done
  for (int c0 = 0; c0 < d; c0 += NTH) {
    const int i = c0 + tid;
    int32_t b = 0;
    int64_t ob = 0;
    int db = 0;
    if (i < d) {
      b = ocol[base + i];
      ob = orow[b];
      db = (int)(orow[b + 1] - ob);
      tab_insert<LOGTAB>(tab, b, i);
      nb[i] = b;
      cnt[i] = 0;
      if (db > kRev * d) {
        const int r = atomicAdd(nrev, 1);
        pre[MAXD - r] = db;
        offj[MAXD - 1 - r] = (int)ob;
        wi[MAXD - 1 - r] = i;
        db = 0;  // not walked
      }
    }
    const unsigned long long v = db > 0 ? (((unsigned long long)db) << 32) | 1ULL : 0ULL;
    const unsigned long long inc = wave_inclusive_sum(v);
    unsigned long long wbase = 0, tot = 0;
    if (NW > 1) {
      if (lane_id() == kWave - 1) scratch[w] = inc;
      __syncthreads();
      for (int q = 0; q < NW; ++q) {
        const unsigned long long z = scratch[q];
        if (q < w) wbase += z;
        tot += z;
      }
      __syncthreads();
    } else {
      tot = __shfl(inc, kWave - 1, kWave);
    }
    if (db > 0) {
      const unsigned long long ex = run + wbase + inc - v;
      const int k = (int)(uint32_t)ex;
      const int pr = (int)(ex >> 32);
      pre[k] = pr;
      offj[k] = (int)(ob - pr);
      wi[k] = i;
    }
    run += tot;
  }
  const int nrows = (int)(uint32_t)run;
  if (tid == 0) pre[nrows] = (int)(run >> 32);
  if (NTH == kWave) wave_sync(); else __syncthreads();
  return nrows;
}

// One wavefront checks pairs [lo, hi) of the searched rows: pair t is
// (searched row t / d, c = nb[t % d]); c in N+(b) closes the triangle
// {a, b, c}, counted on (a, b), (a, c) in LDS and on (b, c) at its oriented
// position.  Each triangle is still found once: c must be an out-neighbour of
// b, as in the walk.
template <int MAXD>
__device__ void search_rows(const int* nb, const int* pre, const int* offj, const int* wi, int* cnt, int d, int lo,
                            int hi, const int32_t* __restrict__ ocol, int32_t* __restrict__ supo) {
  for (int t = lo + lane_id(); t < hi; t += kWave) {
    const int r = t / d, j = t - r * d;
    const int i = wi[MAXD - 1 - r];
    if (j == i) continue;
    const int32_t c = nb[j];
    const int64_t off = offj[MAXD - 1 - r];
    const int64_t end = off + pre[MAXD - r];
    const int64_t p = lower_bound_i32<int64_t>(ocol, off, end, c);
    if (p < end && ocol[p] == c) {
      atomicAdd(&cnt[i], 1);
      atomicAdd(&cnt[j], 1);
      atomicAdd(&supo[p], 1);
    }
  }
}

// bin 0, hash: a wavefront per vertex, vertices fetched kFetch0 at a time
constexpr int kFetch0 = 16;
__global__ void __launch_bounds__(kT) k_sup_hash_wave(const int64_t* __restrict__ orow,
                                                      const int32_t* __restrict__ ocol,
                                                      const int32_t* __restrict__ vlist, SupCtl* ctl,
                                                      int32_t* __restrict__ supo) {
  constexpr int W = kT / kWave;
  constexpr int LOGTAB = 7;
  __shared__ int2 s_tab[W][1 << LOGTAB];
  __shared__ int s_nb[W][kWaveMax];
  __shared__ int s_pre[W][kWaveMax + 1];
  __shared__ int s_offj[W][kWaveMax];
  __shared__ int s_wi[W][kWaveMax];
  __shared__ int s_cnt[W][kWaveMax];
  __shared__ int s_own[W][kWave];
  __shared__ int s_nrev[W];
  if (ctl->act[0] != kHash) return;
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int count = atomic_load_relaxed(&ctl->cnt[0]);
  WalkTabs T{s_pre[w], s_offj[w], s_wi[w], s_tab[w], s_cnt[w], s_own[w]};
  for (;;) {
    int first = 0;
    if (lane == 0) first = atomicAdd(&ctl->fetch[0], kFetch0);
    first = __shfl(first, 0, kWave);
    if (first >= count) break;
    const int last = first + kFetch0 < count ? first + kFetch0 : count;
    for (int idx = first; idx < last; ++idx) {
      const int32_t a = vlist[count - 1 - idx];  // the bin's list backwards: see k_sup_bin
      const int64_t base = orow[a];
      const int d = (int)(orow[a + 1] - base);
      if (lane == 0) s_nrev[w] = 0;
      wave_sync();
      const int nrows = stage_rows<LOGTAB, kWave, kWaveMax>(orow, ocol, base, d, s_tab[w], s_nb[w], s_pre[w],
                                                            s_offj[w], s_wi[w], s_cnt[w], &s_nrev[w], nullptr);
      walk_pairs<LOGTAB>(T, nrows, 0, s_pre[w][nrows], ocol, supo);
      search_rows<kWaveMax>(s_nb[w], s_pre[w], s_offj[w], s_wi[w], s_cnt[w], d, 0, s_nrev[w] * d, ocol, supo);
      wave_sync();
      if (lane < d) {
        const int cc = s_cnt[w][lane];
        if (cc) atomicAdd(&supo[base + lane], cc);
      }
      wave_sync();
    }
  }
}

// bins 1 and 2, hash: a workgroup of NTH threads per vertex; its wavefronts
// split the vertex's pairs into equal contiguous ranges
template <int MAXD, int NTH>
__global__ void __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(8, 8))) k_sup_hash_block(const int64_t* __restrict__ orow,
                                                        const int32_t* __restrict__ ocol, int32_t n,
                                                        const int32_t* __restrict__ vlist, int bin, SupCtl* ctl,
                                                        int32_t* __restrict__ supo) {
  constexpr int LOGTAB = MAXD == 1024 ? 11 : 13;
  constexpr int NW = NTH / kWave;
  __shared__ int2 s_tab[1 << LOGTAB];
  __shared__ int s_nb[MAXD];
  __shared__ int s_pre[MAXD + 1];
  __shared__ int s_offj[MAXD];
  __shared__ int s_wi[MAXD];
  __shared__ int s_cnt[MAXD];
  __shared__ int s_own[NW][kWave];
  __shared__ unsigned long long s_scr[NW];
  __shared__ int s_idx, s_nrev;
  if (ctl->act[bin] != kHash) return;
  const int w = threadIdx.x / kWave;
  const int count = atomic_load_relaxed(&ctl->cnt[bin]);
  WalkTabs T{s_pre, s_offj, s_wi, s_tab, s_cnt, s_own[w]};
  for (;;) {
    if (threadIdx.x == 0) {
      s_idx = atomicAdd(&ctl->fetch[bin], 1);
      s_nrev = 0;
    }
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= count) break;
    const int32_t a = vlist[(int64_t)bin * n + (count - 1 - idx)];
    const int64_t base = orow[a];
    const int d = (int)(orow[a + 1] - base);
    const int nrows = stage_rows<LOGTAB, NTH, MAXD>(orow, ocol, base, d, s_tab, s_nb, s_pre, s_offj, s_wi, s_cnt,
                                                    &s_nrev, s_scr);
    const int64_t total = s_pre[nrows];
    walk_pairs<LOGTAB>(T, nrows, (int)(total * w / NW), (int)(total * (w + 1) / NW), ocol, supo);
    const int64_t stot = (int64_t)s_nrev * d;
    search_rows<MAXD>(s_nb, s_pre, s_offj, s_wi, s_cnt, d, (int)(stot * w / NW), (int)(stot * (w + 1) / NW), ocol,
                      supo);
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += NTH) {
      const int cc = s_cnt[i];
      if (cc) atomicAdd(&supo[base + i], cc);
    }
    __syncthreads();
  }
}

// ---- bin 0, binary search: a wavefront per vertex --------------------------------------------------------
// (the (b, c) pairs flattened over the lanes, c searched in N+(a) in global memory)
__global__ void __launch_bounds__(kT) k_sup_wave_bs(const int64_t* __restrict__ orow,
                                                    const int32_t* __restrict__ ocol,
                                                    const int32_t* __restrict__ vlist, SupCtl* ctl,
                                                    int32_t* __restrict__ supo) {
  constexpr int MODE = kBsearch;
  constexpr int W = kT / kWave;
  __shared__ int s_nb[W][kWaveMax];
  __shared__ int s_cnt[W][kWaveMax];
  __shared__ int s_pre[W][kWaveMax + 1];
  __shared__ int64_t s_off[W][kWaveMax];
  if (ctl->act[0] != MODE) return;
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
        const int64_t q = lower_bound_i32<int64_t>(ocol, base, base + d, c);
        if (q < base + d && ocol[q] == c) p = (int)(q - base);
        if (p >= 0) {
          atomicAdd(&s_cnt[w][i], 1);
          atomicAdd(&s_cnt[w][p], 1);
          atomicAdd(&supo[j], 1);
        }
      }
    }
    wave_sync();
    if (valid) {
      const int cc = s_cnt[w][lane];
      if (cc) atomicAdd(&supo[base + lane], cc);
    }
    wave_sync();
  }
}

// ---- bins 1-3, binary search: a workgroup per vertex, N+(a) searched in global memory,
// chunks of 256 b's ------------------------------------------------------------------------
__global__ void __launch_bounds__(kT) k_sup_chunked(const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol,
                                                    int32_t n, const int32_t* __restrict__ vlist, int bin,
                                                    SupCtl* ctl, int32_t* __restrict__ supo) {
  __shared__ int s_cnt[kT];
  __shared__ int s_pre[kT + 1];
  __shared__ int64_t s_off[kT];
  __shared__ int s_wt[kT / kWave];
  __shared__ int s_idx;
  if (ctl->act[bin] != kBsearch) return;
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
          atomicAdd(&supo[q], 1);
          atomicAdd(&supo[j], 1);
        }
      }
      __syncthreads();
      if (valid && s_cnt[threadIdx.x]) atomicAdd(&supo[base + i], s_cnt[threadIdx.x]);
      __syncthreads();
    }
  }
}

// ---- merge: a wavefront per vertex a of the bin, one lane per oriented edge a -> b,
// two-pointer merge of N+(a) and N+(b) ---------------------------------------------------------
__global__ void __launch_bounds__(kT) k_sup_merge(const int64_t* __restrict__ orow, const int32_t* __restrict__ ocol,
                                                  int32_t n, const int32_t* __restrict__ vlist, int bin, SupCtl* ctl,
                                                  int32_t* __restrict__ supo) {
  if (ctl->act[bin] != kMerge) return;
  const int lane = lane_id();
  const int count = atomic_load_relaxed(&ctl->cnt[bin]);
  for (;;) {
    int idx = 0;
    if (lane == 0) idx = atomicAdd(&ctl->fetch[bin], 1);
    idx = __shfl(idx, 0, kWave);
    if (idx >= count) break;
    const int32_t a = vlist[(int64_t)bin * n + idx];
    const int64_t base = orow[a], end = orow[a + 1];
    for (int64_t e0 = base; e0 < end; e0 += kWave) {
      const int64_t i = e0 + lane;
      if (i >= end) continue;
      const int32_t b = ocol[i];
      int64_t p = base, q = orow[b];
      const int64_t qe = orow[b + 1];
      int cnt = 0;
      while (p < end && q < qe) {
        const int32_t cp = ocol[p], cq = ocol[q];
        if (cp < cq) {
          ++p;
        } else if (cp > cq) {
          ++q;
        } else {
          ++cnt;
          atomicAdd(&supo[p], 1);
          atomicAdd(&supo[q], 1);
          ++p;
          ++q;
        }
      }
      if (cnt) atomicAdd(&supo[i], cnt);
    }
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

struct SupLayout {
  SupCtl* ctl;
  int32_t* vlist;
  int32_t* supo;  // counts by oriented position
};

void carve(const DevGraph& dg, Arena& a, SupLayout& L) {
  L.ctl = a.take<SupCtl>(1);
  L.vlist = a.take<int32_t>((size_t)kBins * (dg.n + 1));
  L.supo = a.take<int32_t>((size_t)dg.m + 1);
}

// workgroup sizes of the hash kernels of bins 1 and 2
constexpr int kHashT1 = 512, kHashT2 = 1024;

}  // namespace

size_t support_workspace(const DevGraph& dg, Arena& a) {
  SupLayout L;
  carve(dg, a, L);
  return a.used;
}

int compute_support(const DevGraph& dg, const SupPlan& plan, int2* sr, Arena& a, hipStream_t s,
                    truss_trace* trace) {
  SupLayout L;
  carve(dg, a, L);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  const int64_t m = dg.m;
  const int32_t n = dg.n;
  hipLaunchKernelGGL(k_sup_zero, dim3(grid_for(m > kBins ? m : kBins)), dim3(kT), 0, s, L.supo, m, L.ctl);
  if (m == 0) return TRUSS_OK;
  hipLaunchKernelGGL(k_sup_bin, dim3((unsigned)((n + kBinT - 1) / kBinT > 0 ? (n + kBinT - 1) / kBinT : 1)),
                     dim3(kBinT), 0, s, dg.orow, n, L.vlist, L.ctl);
  hipLaunchKernelGGL(k_sup_decide, dim3(1), dim3(kBins * kWave), 0, s, L.ctl, m, plan.sched, plan.force,
                     plan.model);
  hipEvent_t ev[kBins + 1] = {};
  bool timed = trace != nullptr;
  for (int b = 0; timed && b <= kBins; ++b)
    if (hipEventCreate(&ev[b]) != hipSuccess) timed = false;
  // persistent-style grids: workers fetch vertices from the bin lists
  const unsigned gw = 256 * 8, gb = 256 * 4, g2 = 256;
  for (int b = 0; b < kBins; ++b) {
    if (timed) (void)hipEventRecord(ev[b], s);
    if (b == 0) {
      hipLaunchKernelGGL(k_sup_hash_wave, dim3(gw), dim3(kT), 0, s, dg.orow, dg.ocol, L.vlist, L.ctl, L.supo);
      hipLaunchKernelGGL(k_sup_wave_bs, dim3(gw), dim3(kT), 0, s, dg.orow, dg.ocol, L.vlist, L.ctl, L.supo);
    } else if (b == 1) {
      hipLaunchKernelGGL((k_sup_hash_block<kBlockMax1, kHashT1>), dim3(gb), dim3(kHashT1), 0, s, dg.orow, dg.ocol, n,
                         L.vlist, 1, L.ctl, L.supo);
    } else if (b == 2) {
      hipLaunchKernelGGL((k_sup_hash_block<kBlockMax2, kHashT2>), dim3(g2), dim3(kHashT2), 0, s, dg.orow, dg.ocol,
                         n, L.vlist, 2, L.ctl, L.supo);
    }
    if (b > 0)
      hipLaunchKernelGGL(k_sup_chunked, dim3(b == 1 ? gb : g2), dim3(kT), 0, s, dg.orow, dg.ocol, n, L.vlist, b,
                         L.ctl, L.supo);
    hipLaunchKernelGGL(k_sup_merge, dim3(b == 0 ? gw : gb), dim3(kT), 0, s, dg.orow, dg.ocol, n, L.vlist, b, L.ctl,
                       L.supo);
  }
  hipLaunchKernelGGL(k_sup_finish, dim3(grid_for(m)), dim3(kT), 0, s, L.supo, dg.oeid, m, sr);
  if (timed) (void)hipEventRecord(ev[kBins], s);
  TRUSS_HIP(hipGetLastError());
  if (trace) {
    SupCtl h;
    TRUSS_HIP(hipMemcpyAsync(&h, L.ctl, sizeof(SupCtl), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < kBins; ++b) {
      trace->sup_action[b] = h.act[b];
      for (int i = 0; i < kSupF; ++i) trace->sup_feat[b][i] = h.feat[b][i];
      float t = 0.f;
      if (timed && hipEventElapsedTime(&t, ev[b], ev[b + 1]) != hipSuccess) t = 0.f;
      trace->sup_ms[b] = t;
    }
  }
  for (int b = 0; b <= kBins; ++b)
    if (ev[b]) (void)hipEventDestroy(ev[b]);
  return TRUSS_OK;
}

}  // namespace truss
