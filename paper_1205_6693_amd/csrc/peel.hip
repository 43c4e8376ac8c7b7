// Peeling (Algorithm 2, Steps 4-15, made level-synchronous).
//
// Level k removes every live edge whose support is at most k-2 and gives it
// truss number k.  Within a level the frontier F_r of sub-round r is a snapshot:
// an edge joins F_r by having its round stamp set to r, and an edge counts as
// removed once its stamp is non-zero and below the current round.  A triangle
// whose three edges are not removed and which has at least one edge in F_r is
// destroyed in round r; only its F_r edge of smallest id processes it, and that
// edge decrements each of the triangle's other edges that is not in F_r exactly
// once (the two decrements of Algorithm 2, Step 9).  After round r every live
// edge's support therefore equals its support in the graph without
// F_0 ∪ ... ∪ F_r, which is the sequential invariant, so the truss numbers
// match Algorithm 2 whatever the order of removals inside a level.
//
// Triangles through a frontier edge e = (u, v) are found as in Algorithm 2,
// Steps 6-8: walk the adjacency row of the endpoint with the shorter live row,
// and look each neighbour w up in the other endpoint's sorted row by binary
// search.  Deleted edges are only marked (Section 3.1), and the rows are
// compacted in place whenever the live edge count has halved.
//
// The whole loop runs in one persistent cooperative kernel.  Phases are
// separated by a grid barrier; the last workgroup to arrive runs the control
// step (next phase, next level k = max(k+1, min live support + 2), queue sizes)
// before releasing the others, so the host is not involved until the end.
//
// Frontier modes per level: SPARSE enqueues an edge the moment its support
// drops from k-1 to k-2 (the queue of Section 3.1); DENSE re-scans the live
// edges after every sub-round.
#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;
constexpr int kWaves = kT / kWave;
constexpr int kHeavy = 2048;   // frontier edges with a longer walk are split into pieces
constexpr int kPiece = 1024;   // adjacency entries per piece
constexpr int kIntMax = 0x7fffffff;

enum Phase : int {
  PH_SWEEP = 0,   // compact the live-edge list, minimum live support
  PH_START = 1,   // level start: collect live edges with sup <= k-2
  PH_PROC = 2,    // destroy triangles of F_r (light edges; heavy ones queued)
  PH_HEAVY = 3,   // split walks of heavy frontier edges
  PH_DENSE = 4,   // dense mode: collect next frontier by re-scan
  PH_COMPACT = 5, // drop removed entries from the adjacency rows
  PH_DONE = 6
};

struct alignas(256) PeelCtl {
  unsigned bar_count;
  unsigned pad0[63];
  unsigned bar_gen;
  unsigned pad1[63];
  // working counters, reset by the control step
  int w_fetch;
  int w_qlen;
  int w_alive;
  int w_minsup;
  int w_pfetch;   // piece fetch counter
  int pad2;
  unsigned long long w_pieces;  // pieces appended this round (may exceed capacity)
  unsigned long long w_work;
  int pad3[54];
  // published control state, written only by the control step
  int phase;
  int k;
  int r;
  int qlen;
  int acnt;
  int acur;
  int first;
  int mode;
  int pcount;     // pieces to process in PH_HEAVY
  int pcap;       // piece-list capacity
  long long removed_level;
  long long csr_live;
  int kmax;
  int levels;
  long long subrounds;
  long long work;
  int err;
  int abort;
  long long max_subrounds;
  int force_mode;
};

struct PeelArgs {
  int32_t n;
  int64_t m;
  const int64_t* row_ptr;
  int32_t* col;
  int32_t* seid;
  int32_t* rlen;
  const int32_t* eu;
  const int32_t* ev;
  int2* sr;
  int32_t* truss;
  int32_t* alist[2];
  int32_t* fq[2];
  int32_t* pe;   // piece: frontier edge
  int32_t* pb;   // piece: endpoint whose row is searched
  int64_t* pj;   // piece: first adjacency entry
  int32_t* pn;   // piece: entry count
  PeelCtl* ctl;
};

__device__ __forceinline__ int ld(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ long long ld(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- control step: runs on one thread of the last workgroup at each barrier ----------------
__device__ void control_step(PeelCtl* c) {
  int phase = ld(&c->phase);
  const int r = ld(&c->r);
  long long subrounds = ld(&c->subrounds);
  const long long maxsr = ld(&c->max_subrounds);
  auto next_round = [&](void) {
    const int q = ld(&c->w_qlen);
    st(&c->w_qlen, 0);
    st(&c->w_fetch, 0);
    if (q > 0) {
      st(&c->qlen, q);
      st(&c->r, r + 1);
      st(&c->removed_level, ld(&c->removed_level) + q);
      subrounds += 1;
      st(&c->subrounds, subrounds);
      phase = PH_PROC;
    } else {
      // level finished: compact rows when the live count has halved
      const long long alive_after = (long long)ld(&c->acnt) - ld(&c->removed_level);
      const long long live = ld(&c->csr_live);
      if (alive_after > 0 && alive_after * 2 < live) {
        st(&c->csr_live, alive_after);
        phase = PH_COMPACT;
      } else {
        phase = PH_SWEEP;
      }
    }
  };
  switch (phase) {
    case PH_SWEEP: {
      const int alive = ld(&c->w_alive);
      const int minsup = ld(&c->w_minsup);
      st(&c->w_alive, 0);
      st(&c->w_minsup, kIntMax);
      st(&c->acnt, alive);
      st(&c->acur, ld(&c->acur) ^ 1);
      st(&c->first, 0);
      if (alive == 0) { phase = PH_DONE; break; }
      int k = ld(&c->k) + 1;
      if (minsup + 2 > k) k = minsup + 2;
      st(&c->k, k);
      st(&c->kmax, k);
      st(&c->levels, ld(&c->levels) + 1);
      st(&c->r, r + 1);
      st(&c->removed_level, 0LL);
      const int fm = ld(&c->force_mode);
      st(&c->mode, fm == TRUSS_PEEL_DENSE ? (int)TRUSS_PEEL_DENSE : (int)TRUSS_PEEL_SPARSE);
      st(&c->w_qlen, 0);
      st(&c->w_fetch, 0);
      phase = PH_START;
      break;
    }
    case PH_START: {
      const int q = ld(&c->w_qlen);
      st(&c->w_qlen, 0);
      st(&c->w_fetch, 0);
      st(&c->qlen, q);
      st(&c->removed_level, (long long)q);
      subrounds += 1;
      st(&c->subrounds, subrounds);
      phase = q > 0 ? PH_PROC : PH_SWEEP;
      break;
    }
    case PH_PROC:
    case PH_HEAVY: {
      if (phase == PH_PROC) {
        const unsigned long long pw = ld(&c->w_pieces);
        const int cap = ld(&c->pcap);
        const int pc = pw > (unsigned long long)cap ? cap : (int)pw;
        st(&c->w_pieces, 0ULL);
        st(&c->w_pfetch, 0);
        if (pc > 0) {
          st(&c->pcount, pc);
          phase = PH_HEAVY;
          break;
        }
      }
      if (ld(&c->mode) == TRUSS_PEEL_DENSE) {
        st(&c->w_qlen, 0);
        st(&c->w_fetch, 0);
        phase = PH_DENSE;
        break;
      }
      next_round();
      break;
    }
    case PH_DENSE:
      next_round();
      break;
    case PH_COMPACT:
      phase = PH_SWEEP;
      break;
    default:
      phase = PH_DONE;
  }
  if (maxsr > 0 && subrounds > maxsr && phase != PH_DONE) {
    st(&c->err, (int)TRUSS_E_INTERNAL);
    phase = PH_DONE;
  }
  st(&c->phase, phase);
}

// Grid barrier; the last workgroup to arrive runs control_step before release.
// Returns false if the wait timed out (the kernel then winds down).
__device__ bool phase_barrier(PeelCtl* c) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const unsigned gen = __hip_atomic_load(&c->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (prev == gridDim.x - 1) {
      __threadfence();
      control_step(c);
      __hip_atomic_store(&c->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      __hip_atomic_fetch_add(&c->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&c->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
        if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0; break; }
        // 100 MHz constant clock: give up after 30 s
        if (wall_clock64() - t0 > 3000000000ULL) {
          __hip_atomic_store(&c->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ bool removed_at(int rnd, int r) { return rnd != 0 && rnd < r; }

// One adjacency entry j of the walk of frontier edge e = (a, b).  Returns the
// (up to two) edges whose support crossed k-1 -> k-2 and must be enqueued.
__device__ __forceinline__ void process_entry(const PeelArgs& P, int32_t e, int32_t b, int64_t j, int r, int l, int k,
                                              bool sparse, int32_t& f1, int32_t& f2) {
  f1 = -1;
  f2 = -1;
  const int32_t w = P.col[j];
  if (w == b) return;
  const int32_t e1 = P.seid[j];
  const int rnd1 = P.sr[e1].y;
  if (removed_at(rnd1, r)) return;
  const int64_t rb = P.row_ptr[b];
  const int64_t re = rb + P.rlen[b];
  const int64_t p = lower_bound_i32<int64_t>(P.col, rb, re, w);
  if (p >= re || P.col[p] != w) return;
  const int32_t e2 = P.seid[p];
  const int rnd2 = P.sr[e2].y;
  if (removed_at(rnd2, r)) return;
  // the triangle belongs to its frontier edge of smallest id
  if (rnd1 == r && e1 < e) return;
  if (rnd2 == r && e2 < e) return;
  if (rnd1 != r) {
    const int old = atomicSub(&P.sr[e1].x, 1);
    if (sparse && old == l + 1) {
      P.sr[e1].y = r + 1;
      P.truss[e1] = k;
      f1 = e1;
    }
  }
  if (rnd2 != r) {
    const int old = atomicSub(&P.sr[e2].x, 1);
    if (sparse && old == l + 1) {
      P.sr[e2].y = r + 1;
      P.truss[e2] = k;
      f2 = e2;
    }
  }
}

__device__ __forceinline__ void push_next(const PeelArgs& P, int32_t* q, int32_t f1, int32_t f2) {
  const int p1 = wave_append(&P.ctl->w_qlen, f1 >= 0);
  if (f1 >= 0) q[p1] = f1;
  const int p2 = wave_append(&P.ctl->w_qlen, f2 >= 0);
  if (f2 >= 0) q[p2] = f2;
}

__global__ void __launch_bounds__(kT) k_peel(PeelArgs P) {
  __shared__ int s_pre[kWaves][kWave + 1];
  __shared__ int s_e[kWaves][kWave];
  __shared__ int s_b[kWaves][kWave];
  __shared__ int64_t s_base[kWaves][kWave];
  PeelCtl* c = P.ctl;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const int64_t gwave = (blockIdx.x * (int64_t)kT + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  unsigned long long my_work = 0;

  for (;;) {
    const int phase = ld(&c->phase);
    if (phase == PH_DONE) break;
    const int k = ld(&c->k);
    const int l = k - 2;
    const int r = ld(&c->r);
    const int acur = ld(&c->acur);
    if (phase == PH_SWEEP) {
      // live-edge list of the new level; minimum live support
      const int first = ld(&c->first);
      const int64_t cnt = first ? P.m : (int64_t)ld(&c->acnt);
      const int32_t* A = P.alist[acur];
      int32_t* B = P.alist[acur ^ 1];
      int mins = kIntMax;
      for (int64_t base = gwave * kWave; base < cnt; base += nwaves * kWave) {
        const int64_t i = base + lane;
        bool live = false;
        int32_t e = 0;
        if (i < cnt) {
          e = first ? (int32_t)i : A[i];
          const int2 s = P.sr[e];
          live = s.y == 0;
          if (live && s.x < mins) mins = s.x;
        }
        const int pos = wave_append(&c->w_alive, live);
        if (live) B[pos] = e;
      }
      mins = wave_min(mins);
      if (lane == 0 && mins != kIntMax) atomicMin(&c->w_minsup, mins);
    } else if (phase == PH_START || phase == PH_DENSE) {
      // collect live edges with sup <= k-2 (level start, or dense re-scan)
      const int64_t cnt = ld(&c->acnt);
      const int32_t* A = P.alist[acur];
      const int stamp = phase == PH_START ? r : r + 1;
      int32_t* Q = P.fq[stamp & 1];
      for (int64_t base = gwave * kWave; base < cnt; base += nwaves * kWave) {
        const int64_t i = base + lane;
        bool take = false;
        int32_t e = 0;
        if (i < cnt) {
          e = A[i];
          const int2 s = P.sr[e];
          take = s.y == 0 && s.x <= l;
          if (take) {
            P.sr[e].y = stamp;
            P.truss[e] = k;
          }
        }
        const int pos = wave_append(&c->w_qlen, take);
        if (take) Q[pos] = e;
      }
    } else if (phase == PH_PROC) {
      const int qn = ld(&c->qlen);
      const bool sparse = ld(&c->mode) == TRUSS_PEEL_SPARSE;
      const int32_t* Q = P.fq[r & 1];
      int32_t* Qn = P.fq[(r + 1) & 1];
      for (;;) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&c->w_fetch, kWave);
        base = __shfl(base, 0, kWave);
        if (base >= qn) break;
        const int i = base + lane;
        const bool valid = i < qn;
        int32_t e = 0, a = 0, b = 0;
        int work = 0;
        if (valid) {
          e = Q[i];
          const int32_t u = P.eu[e], v = P.ev[e];
          const int du = P.rlen[u], dv = P.rlen[v];
          const bool ua = du < dv || (du == dv && u < v);
          a = ua ? u : v;
          b = ua ? v : u;
          work = ua ? du : dv;
        }
        // heavy walks are cut into pieces for PH_HEAVY; pieces past the list's
        // capacity are walked here
        const bool heavy = work > kHeavy;
        int64_t inl_lo = 0, inl_hi = 0;
        if (ballot(heavy)) {
          const int np = heavy ? (work + kPiece - 1) / kPiece : 0;
          const int pinc = wave_inclusive_sum(np);
          const int ptot = __shfl(pinc, kWave - 1, kWave);
          unsigned long long pbase = 0;
          if (lane == 0) pbase = atomicAdd(&c->w_pieces, (unsigned long long)ptot);
          pbase = __shfl(pbase, 0, kWave);
          const int cap = ld(&c->pcap);
          const int64_t ra = P.row_ptr[a];
          if (heavy) {
            const unsigned long long first = pbase + (unsigned long long)(pinc - np);
            for (int q = 0; q < np; ++q) {
              const int64_t j0 = ra + (int64_t)q * kPiece;
              const int len = work - q * kPiece < kPiece ? work - q * kPiece : kPiece;
              if (first + q < (unsigned long long)cap) {
                P.pe[first + q] = e;
                P.pb[first + q] = b;
                P.pj[first + q] = j0;
                P.pn[first + q] = len;
              } else {
                if (inl_hi == 0) inl_lo = j0;
                inl_hi = j0 + len;
              }
            }
          }
          work = heavy ? 0 : work;
          // overflow pieces: the wave walks them one heavy edge at a time
          uint64_t om = ballot(inl_hi > inl_lo);
          while (om) {
            const int src = __builtin_ctzll(om);
            om &= om - 1;
            const int32_t oe = __shfl(e, src, kWave), ob = __shfl(b, src, kWave);
            const int64_t lo = __shfl(inl_lo, src, kWave), hi = __shfl(inl_hi, src, kWave);
            for (int64_t j0 = lo; j0 < hi; j0 += kWave) {
              int32_t f1 = -1, f2 = -1;
              if (j0 + lane < hi) process_entry(P, oe, ob, j0 + lane, r, l, k, sparse, f1, f2);
              push_next(P, Qn, f1, f2);
            }
            my_work += (unsigned long long)(hi - lo);
          }
        }
        const int inc = wave_inclusive_sum(work);
        const int W = __shfl(inc, kWave - 1, kWave);
        s_pre[wv][lane + 1] = inc;
        if (lane == 0) s_pre[wv][0] = 0;
        s_e[wv][lane] = e;
        s_b[wv][lane] = b;
        s_base[wv][lane] = P.row_ptr[a];
        wave_sync();
        my_work += (unsigned long long)W;
        for (int t0 = 0; t0 < W; t0 += kWave) {
          const int t = t0 + lane;
          int32_t f1 = -1, f2 = -1;
          if (t < W) {
            int lo = 0, hi = kWave - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (s_pre[wv][mid] <= t) lo = mid; else hi = mid - 1;
            }
            process_entry(P, s_e[wv][lo], s_b[wv][lo], s_base[wv][lo] + (t - s_pre[wv][lo]), r, l, k, sparse, f1,
                          f2);
          }
          push_next(P, Qn, f1, f2);
        }
        wave_sync();
      }
    } else if (phase == PH_HEAVY) {
      const int pc = ld(&c->pcount);
      const bool sparse = ld(&c->mode) == TRUSS_PEEL_SPARSE;
      int32_t* Qn = P.fq[(r + 1) & 1];
      for (;;) {
        int q = 0;
        if (lane == 0) q = atomicAdd(&c->w_pfetch, 1);
        q = __shfl(q, 0, kWave);
        if (q >= pc) break;
        const int32_t e = P.pe[q], b = P.pb[q];
        const int64_t j0 = P.pj[q];
        const int len = P.pn[q];
        for (int t0 = 0; t0 < len; t0 += kWave) {
          int32_t f1 = -1, f2 = -1;
          if (t0 + lane < len) process_entry(P, e, b, j0 + t0 + lane, r, l, k, sparse, f1, f2);
          push_next(P, Qn, f1, f2);
        }
        my_work += (unsigned long long)len;
      }
    } else if (phase == PH_COMPACT) {
      // stable in-place compaction of every row to its live entries
      for (int64_t v = gwave; v < P.n; v += nwaves) {
        const int64_t rb = P.row_ptr[v];
        const int len = P.rlen[v];
        int wpos = 0;
        for (int c0 = 0; c0 < len; c0 += kWave) {
          const int i = c0 + lane;
          int32_t x = 0, ed = 0;
          bool keep = false;
          if (i < len) {
            x = P.col[rb + i];
            ed = P.seid[rb + i];
            keep = P.sr[ed].y == 0;
          }
          const uint64_t km = ballot(keep);
          if (keep) {
            const int64_t dst = rb + wpos + rank_below(km);
            P.col[dst] = x;
            P.seid[dst] = ed;
          }
          wpos += __popcll(km);
        }
        if (lane == 0) P.rlen[v] = wpos;
      }
    }
    if (!phase_barrier(c)) break;
  }
  // statistics
  my_work = wave_sum(my_work);
  if (lane == 0 && my_work) atomicAdd(&c->w_work, my_work);
}

__global__ void k_peel_init(PeelCtl* c, const int64_t* __restrict__ row_ptr, int32_t* __restrict__ rlen, int32_t n,
                            int64_t m, long long max_subrounds, int force_mode, int pcap) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rlen[i] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
  if (i == 0) {
    c->bar_count = 0;
    c->bar_gen = 0;
    c->w_fetch = 0;
    c->w_qlen = 0;
    c->w_alive = 0;
    c->w_minsup = kIntMax;
    c->w_pieces = 0ULL;
    c->w_pfetch = 0;
    c->w_work = 0;
    c->phase = PH_SWEEP;
    c->k = 1;
    c->r = 0;
    c->qlen = 0;
    c->acnt = (int)m;
    c->acur = 0;
    c->first = 1;
    c->mode = TRUSS_PEEL_SPARSE;
    c->pcount = 0;
    c->pcap = pcap;
    c->removed_level = 0;
    c->csr_live = m;
    c->kmax = 0;
    c->levels = 0;
    c->subrounds = 0;
    c->work = 0;
    c->err = 0;
    c->abort = 0;
    c->max_subrounds = max_subrounds;
    c->force_mode = force_mode;
  }
}

struct PeelLayout {
  PeelCtl* ctl;
  int32_t* rlen;
  int32_t* alist[2];
  int32_t* fq[2];
  int32_t *pe, *pb, *pn;
  int64_t* pj;
  int pcap;
};

void carve(const DevGraph& dg, Arena& a, PeelLayout& L) {
  const int64_t m = dg.m;
  L.ctl = a.take<PeelCtl>(1);
  L.rlen = a.take<int32_t>(dg.n + 1);
  for (int i = 0; i < 2; ++i) L.alist[i] = a.take<int32_t>(m + 1);
  for (int i = 0; i < 2; ++i) L.fq[i] = a.take<int32_t>(m + 1);
  L.pcap = (int)(m < (1 << 22) ? m : (1 << 22));
  L.pe = a.take<int32_t>(L.pcap + 1);
  L.pb = a.take<int32_t>(L.pcap + 1);
  L.pn = a.take<int32_t>(L.pcap + 1);
  L.pj = a.take<int64_t>(L.pcap + 1);
}

int g_peel_blocks = 0;

}  // namespace

size_t peel_workspace(const DevGraph& dg, Arena& a) {
  PeelLayout L;
  carve(dg, a, L);
  return a.used;
}

int peel(const DevGraph& dg, const truss_options* opts, int2* sr, int32_t* truss_canon, Arena& a, PeelResult* res,
         hipStream_t s) {
  PeelLayout L;
  carve(dg, a, L);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  *res = PeelResult();
  if (dg.m == 0) return TRUSS_OK;
  const int force = opts ? opts->peel_mode : TRUSS_PEEL_AUTO;
  const long long maxsr = opts ? opts->max_subrounds : 0;
  const int64_t initn = dg.n > 1 ? dg.n : 1;
  hipLaunchKernelGGL(k_peel_init, dim3((unsigned)((initn + kT - 1) / kT)), dim3(kT), 0, s, L.ctl, dg.row_ptr, L.rlen,
                     dg.n, dg.m, maxsr, force, L.pcap);
  if (g_peel_blocks == 0) g_peel_blocks = device_grid_blocks((const void*)k_peel, kT, 0);
  int blocks = g_peel_blocks;
  if (opts && opts->grid_blocks > 0 && opts->grid_blocks < blocks) blocks = opts->grid_blocks;
  PeelArgs P;
  P.n = dg.n;
  P.m = dg.m;
  P.row_ptr = dg.row_ptr;
  P.col = dg.col;
  P.seid = dg.seid;
  P.rlen = L.rlen;
  P.eu = dg.eu;
  P.ev = dg.ev;
  P.sr = sr;
  P.truss = truss_canon;
  P.alist[0] = L.alist[0];
  P.alist[1] = L.alist[1];
  P.fq[0] = L.fq[0];
  P.fq[1] = L.fq[1];
  P.pe = L.pe;
  P.pb = L.pb;
  P.pj = L.pj;
  P.pn = L.pn;
  P.ctl = L.ctl;
  void* args[] = {&P};
  TRUSS_HIP(hipLaunchCooperativeKernel((const void*)k_peel, dim3(blocks), dim3(kT), args, 0, s));
  PeelCtl h;
  TRUSS_HIP(hipMemcpyAsync(&h, L.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  res->kmax = h.kmax;
  res->levels = h.levels;
  res->subrounds = h.subrounds;
  res->work = (int64_t)h.w_work;
  if (h.abort) {
    set_last_error("peeling kernel barrier timed out");
    return TRUSS_E_INTERNAL;
  }
  if (h.err) {
    set_last_error("peeling exceeded the sub-round cap (%lld)", (long long)h.max_subrounds);
    return h.err;
  }
  return TRUSS_OK;
}

}  // namespace truss
