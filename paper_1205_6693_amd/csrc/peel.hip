// Peeling (Algorithm 2, made level-synchronous).
//
// Level k removes every live edge whose support is at most k-2 and gives it
// truss number k.  Within a level the frontier F_r of sub-round r is a snapshot:
// an edge joins F_r by having its round stamp set to r, and an edge counts as
// removed once its stamp is non-zero and below the current round.  A triangle
// whose three edges are not removed and which has at least one edge in F_r is
// destroyed in round r; only its F_r edge of smallest id processes it, and that
// edge decrements each of the triangle's other edges that is not in F_r exactly
// once (the two decrements of Algorithm 2).  After round r every live
// edge's support therefore equals its support in the graph without
// F_0 ∪ ... ∪ F_r, which is the sequential invariant, so the truss numbers
// match Algorithm 2 whatever the order of removals inside a level.
//
// Triangles through a frontier edge e = (u, v) are found as in Algorithm 2,
// by its triangle walk: walk the adjacency row of the endpoint with the shorter live row,
// and look each neighbour w up in the other endpoint's sorted row by binary
// search.  Deleted edges are only marked (Section 3.1); the rows are compacted
// in place whenever the live edge count has halved.
//
// The level loop runs in a persistent kernel, one 1024-thread workgroup per
// compute unit.  The grid is never larger than the number of workgroups the
// device holds at once (one per compute unit, checked against the occupancy
// of the kernel before the first launch), so every workgroup is resident and
// the grid barrier can complete; the launch is an ordinary one on the
// caller's stream (a cooperative launch goes through a queue of its own,
// which profilers tear down at exit after the run's results are written, and
// adds nothing here).  Phases are separated by a grid barrier; the last
// workgroup to arrive runs the control step (next phase, next level
// k = max(k+1, min live support + 2), queue sizes) before releasing the others.
// The kernel returns to the host only to compact the rows (a separate kernel)
// or when every edge is removed.
//
// Memory coherence: the L2 caches of the XCDs are not coherent with each
// other, and an agent-scope fence writes back and invalidates a whole L2.  The
// barrier therefore uses no fences: every value that one phase writes and a
// later phase of another workgroup reads (queues, live lists, round stamps,
// supports, pieces) is written and read with agent-scope relaxed atomics, which
// go to the coherent level, and each lane waits for its outstanding memory
// operations before its workgroup arrives.  Adjacency rows, offsets and row
// lengths are immutable inside a launch and use ordinary cached loads.
//
// Each level runs in one of four ways, decided when its first frontier is
// known: the frontier mode (SPARSE enqueues an edge the moment its support
// drops from k-1 to k-2, the queue of Section 3.1; DENSE re-scans the live
// edges after every sub-round) and the membership probe (the edge
// hash table, or a binary search of the other endpoint's sorted row).  The scheduler
// (plain, a fixed heuristic, or the learned network evaluated by the control
// wavefront) only picks among these exact methods.
#include "common.hpp"
#include "internal.hpp"
#include "mlp.hpp"

namespace truss {

namespace {

constexpr int kT = 1024;
constexpr int kWaves = kT / kWave;
// adjacency entries per segment of a chunk's walks: smaller segments spread
// mid-size rounds over more workgroups, larger ones cut the announcement
// traffic of rounds with big frontiers
constexpr int kSegSmall = 1 * 1024, kSegLarge = 8 * 1024;
constexpr int kSegLargeFrontier = 8192;  // frontiers of at least this many edges use kSegLarge
constexpr int kIntMax = 0x7fffffff;
constexpr int kHistBins = 6;
constexpr long long kCompactNum = 8, kCompactDen = 10;  // row compaction threshold
constexpr int kStageA = 8192;  // LDS staging of live-list appends (entries)
constexpr int kStageQ = 2048;  // LDS staging of frontier-queue appends
static_assert(4 * kT <= kStageA && 2 * kT <= kStageQ, "sweep staging capacity");
constexpr int kMinChunk = 64;  // smallest frontier chunk

// Frontier edges per chunk in a round with qn frontier edges: the frontier is
// spread over all workgroups, with between kMinChunk and kT edges a chunk.
__device__ __forceinline__ int chunk_size(int qn, int groups) {
  int cs = (qn + groups - 1) / groups;
  cs = (cs + kMinChunk - 1) / kMinChunk * kMinChunk;
  return cs < kMinChunk ? kMinChunk : cs > kT ? kT : cs;
}

enum Phase : int {
  PH_SWEEP = 0,    // compact the live-edge list, minimum live support
  PH_START = 1,    // level start: collect live edges with sup <= k-2
  PH_PROC = 2,     // destroy the triangles of F_r
  PH_UNUSED = 3,
  PH_DENSE = 4,    // dense mode: collect the next frontier by re-scan
  PH_COMPACT = 5,  // return to the host: drop removed entries from the rows
  PH_DONE = 6
};

constexpr int kGroups = 8;  // barrier arrival groups (workgroup id mod 8: one per XCD under round-robin dispatch)

struct alignas(256) PeelCtl {
  unsigned bar_count;          // groups arrived
  unsigned pad0[63];
  unsigned bar_gen;
  unsigned pad1[63];
  unsigned grp_count[kGroups][32];  // workgroups arrived, per group (one 128-byte line each)
  // working counters, reset by the control step; each on its own 128-byte
  // line so that polling one does not slow the atomics on another
  alignas(128) int w_fetch;               // frontier chunk fetch
  alignas(128) int w_qlen;                // next-frontier queue length
  alignas(128) int w_alive;               // live-list length
  alignas(128) int w_minsup;              // minimum live support
  alignas(128) unsigned long long w_pfetch;  // segment indices drawn
  alignas(128) int w_chunks;              // frontier chunks finished
  alignas(128) unsigned long long w_pieces;  // segments announced (may exceed the slot capacity)
  alignas(128) unsigned long long w_work;
  alignas(128) unsigned long long w_fwork;  // level start: sum over F_0 of the shorter live row
  alignas(128) int pad3;
  // published control state, written only by the control step
  int phase;
  int k;
  int r;
  int qlen;
  int acnt;
  int acur;
  int first;
  int mode;
  int pcap;
  int kmax;
  int levels;
  long long removed_level;
  long long csr_live;
  long long subrounds;
  long long heavy_rounds;
  long long max_subrounds;
  long long hist[kHistBins];
  unsigned long long t_last;            // wall clock at the previous barrier
  unsigned long long t_phase[8];        // time spent per phase (100 MHz ticks)
  int err;
  int abort;
  int launches;
  // scheduling
  int probe;               // membership probe of the current level: 0 row hash table, 1 binary search
  int sched;               // TRUSS_SCHED_* in effect
  int fix_bits, fix_vals;  // action bits fixed by the options
  int m_edges;
  int stop_level;          // > 0: no level above it is started
  long long lvl_sub0;      // sub-rounds before the current level
  long long prev_sub;      // sub-rounds of the previous level
  unsigned long long t_dec;  // wall clock at the current level's decision
};

struct PeelArgs {
  int32_t n;
  int64_t m;
  const int64_t* row_ptr;
  const int32_t* col;
  const int32_t* seid;
  const int32_t* rlen;
  const int32_t* eu;
  const int32_t* ev;
  int2* sr;
  int32_t* truss;
  int32_t* alist[2];
  int32_t* fq[2];
  unsigned long long* pslot;  // segment slots: 0 = free, ((chunk start + 1) << 32) | segment = announced
  int32_t* rec_e;             // per frontier position: edge, search endpoint, row start, prefix
  int32_t* rec_b;
  int64_t* rec_base;
  int32_t* rec_pre;
  int32_t* rec_tot;           // per chunk of 64 positions: total walk length
  const int2* rtab;           // row hash tables
  const int64_t* rtoff;
  PeelCtl* ctl;
  const float* model;         // peeling model part (learned scheduler), or null
  float* tr_feat;             // per-level trace (tr_cap rows), or null
  float* tr_ms;
  int32_t* tr_act;
  int tr_cap;
};

// ---- coherent (agent-scope relaxed) accesses ---------------------------------------
template <typename T>
__device__ __forceinline__ T ldc(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void stc(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int2 ldc2(const int2* p) {
  const unsigned long long x = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int)(uint32_t)x, (int)(uint32_t)(x >> 32));
}
__device__ __forceinline__ int ldc_stamp(const int2* p) { return ldc(&p->y); }
__device__ __forceinline__ void stc_stamp(int2* p, int v) { stc(&p->y, v); }

// wait until this lane's global loads, stores and atomics have completed
__device__ __forceinline__ void mem_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int hist_bin(long long q) {
  return q <= 1 ? 0 : q <= 16 ? 1 : q <= 256 ? 2 : q <= 4096 ? 3 : q <= 65536 ? 4 : 5;
}

// The heuristic's action for a level (bit 0 probe, bit 1 mode).
__device__ __forceinline__ int heuristic_action(const float* x) {
  (void)x;
  return 0;
}

// ---- control step: the first wavefront of the last workgroup to reach a barrier ---------------
// All inputs are loaded first (independent loads in flight together), the
// decision is made in registers, and lane 0 stores the outputs at the end.
// Every value is the same in all lanes; the lanes evaluate the scheduler's
// network together (one hidden unit each).
__device__ void control_step(PeelCtl* c, const PeelArgs& P) {
  const bool lead = lane_id() == 0;
  int phase = ldc(&c->phase);
  int k = ldc(&c->k);
  int r = ldc(&c->r);
  int acnt = ldc(&c->acnt);
  int acur = ldc(&c->acur);
  const int mode_in = ldc(&c->mode);
  int levels = ldc(&c->levels);
  long long removed_level = ldc(&c->removed_level);
  long long csr_live = ldc(&c->csr_live);
  long long subrounds = ldc(&c->subrounds);
  long long heavy_rounds = ldc(&c->heavy_rounds);
  const long long maxsr = ldc(&c->max_subrounds);
  const unsigned long long t_last = ldc(&c->t_last);
  const int w_qlen = ldc(&c->w_qlen);
  const int w_alive = ldc(&c->w_alive);
  const int w_minsup = ldc(&c->w_minsup);
  const unsigned long long w_pieces = ldc(&c->w_pieces);
  const unsigned long long w_fwork = ldc(&c->w_fwork);
  const int sched = ldc(&c->sched);
  const int fix_bits = ldc(&c->fix_bits);
  const int fix_vals = ldc(&c->fix_vals);
  const int stop_level = ldc(&c->stop_level);
  long long lvl_sub0 = ldc(&c->lvl_sub0);
  long long prev_sub = ldc(&c->prev_sub);
  unsigned long long t_dec = ldc(&c->t_dec);
  const int phase_in = phase;
  const unsigned long long now = wall_clock64();
  int qlen_out = -1, mode_out = -1, probe_out = -1, first_out = -1, hist_bin_out = -1;
  bool reset_sweep = false, reset_queue = false, reset_proc = false;

  auto begin_round = [&](int q) {
    qlen_out = q;
    subrounds += 1;
    hist_bin_out = hist_bin(q);
    phase = PH_PROC;
  };
  auto next_round = [&]() {
    reset_queue = true;
    if (w_qlen > 0) {
      r += 1;
      removed_level += w_qlen;
      begin_round(w_qlen);
    } else {
      // level finished
      const int li = levels - 1;
      if (lead && li < P.tr_cap && P.tr_ms) P.tr_ms[li] = (float)((double)(now - t_dec) * 1e-5);
      prev_sub = subrounds - lvl_sub0;
      // compact the rows when the live count has dropped below kCompactNum /
      // kCompactDen of the entries they hold
      const long long alive_after = (long long)acnt - removed_level;
      if (alive_after > 0 && alive_after * kCompactDen < csr_live * kCompactNum) {
        csr_live = alive_after;
        phase = PH_COMPACT;
      } else {
        phase = PH_SWEEP;
      }
    }
  };
  // the level's decision, from features that are the same whatever earlier
  // levels chose; then the level's first round
  auto start_level = [&]() {
        float x[kPeelF];
        const float live = (float)acnt, f0 = (float)w_qlen, wk = (float)w_fwork;
        x[0] = log2f(1.f + live);
        x[1] = log2f(1.f + f0);
        x[2] = f0 / (live > 1.f ? live : 1.f);
        x[3] = log2f((float)k);
        x[4] = log2f(1.f + wk);
        x[5] = log2f(1.f + wk / (f0 > 1.f ? f0 : 1.f));
        x[6] = live / (float)(csr_live > 1 ? csr_live : 1);
        x[7] = log2f(1.f + (float)prev_sub);
        int act;
        if (sched == TRUSS_SCHED_LEARNED && P.model) {
          float sc[kPeelA];
          mlp_scores_wave(P.model, x, sc);
          unsigned mask = 0;
          for (int a = 0; a < kPeelA; ++a)
            if ((a & fix_bits) == fix_vals) mask |= 1u << a;
          act = argmin_allowed(sc, kPeelA, mask);
        } else {
          const int pref = sched == TRUSS_SCHED_PLAIN ? 3 : heuristic_action(x);
          act = (pref & ~fix_bits) | fix_vals;
        }
        mode_out = (act & 2) ? (int)TRUSS_PEEL_DENSE : (int)TRUSS_PEEL_SPARSE;
        probe_out = act & 1;
        const int li = levels - 1;  // trace row of the level
        if (lead && li < P.tr_cap && P.tr_feat) {
          for (int i = 0; i < kPeelF; ++i) P.tr_feat[(int64_t)li * kPeelF + i] = x[i];
          P.tr_act[li] = act;
        }
        lvl_sub0 = subrounds;
        t_dec = now;
        begin_round(w_qlen);
  };
  switch (phase) {
    case PH_SWEEP:
      // the sweep has also taken the live edges with sup <= k-1, the frontier
      // of level k+1 (stamped r+1); it is the level's F_0 unless empty, which
      // happens exactly when the minimum live support is at least k, so that
      // the next level is min + 2 and needs its own start phase
      reset_sweep = true;
      reset_queue = true;
      acnt = w_alive;
      acur ^= 1;
      first_out = 0;
      if (w_alive == 0 || (stop_level > 0 && (w_qlen > 0 ? k + 1 : w_minsup + 2) > stop_level)) {
        phase = PH_DONE;
        break;
      }
      levels += 1;
      r += 1;
      if (w_qlen > 0) {
        k = k + 1;
        removed_level = w_qlen;
        start_level();
      } else {
        k = w_minsup + 2;
        removed_level = 0;
        phase = PH_START;
      }
      break;
    case PH_START:
      reset_queue = true;
      removed_level = w_qlen;
      if (w_qlen > 0) start_level();
      else phase = PH_SWEEP;
      break;
    case PH_PROC:
      reset_proc = true;
      if (w_pieces != 0ULL) heavy_rounds += 1;
      if (mode_in == TRUSS_PEEL_DENSE) {
        reset_queue = true;
        phase = PH_DENSE;
        break;
      }
      next_round();
      break;
    case PH_DENSE:
      next_round();
      break;
    default:
      phase = PH_DONE;
  }
  if (maxsr > 0 && subrounds > maxsr && phase != PH_DONE) {
    if (lead) stc(&c->err, (int)TRUSS_E_INTERNAL);
    phase = PH_DONE;
  }
  if (!lead) return;
  // outputs
  if (t_last != 0 && phase_in >= 0 && phase_in < 8)
    stc(&c->t_phase[phase_in], ldc(&c->t_phase[phase_in]) + (now - t_last));
  stc(&c->t_last, now);
  if (hist_bin_out >= 0) stc(&c->hist[hist_bin_out], ldc(&c->hist[hist_bin_out]) + 1);
  if (reset_sweep) {
    stc(&c->w_alive, 0);
    stc(&c->w_minsup, kIntMax);
    stc(&c->w_fwork, 0ULL);
  }
  if (reset_queue) {
    stc(&c->w_qlen, 0);
    stc(&c->w_fetch, 0);
  }
  if (reset_proc) {
    stc(&c->w_pieces, 0ULL);
    stc(&c->w_pfetch, 0ULL);
    stc(&c->w_chunks, 0);
  }
  if (qlen_out >= 0) stc(&c->qlen, qlen_out);
  if (mode_out >= 0) stc(&c->mode, mode_out);
  if (probe_out >= 0) stc(&c->probe, probe_out);
  if (first_out >= 0) stc(&c->first, first_out);
  stc(&c->k, k);
  stc(&c->kmax, k);
  stc(&c->r, r);
  stc(&c->acnt, acnt);
  stc(&c->acur, acur);
  stc(&c->levels, levels);
  stc(&c->removed_level, removed_level);
  stc(&c->csr_live, csr_live);
  stc(&c->subrounds, subrounds);
  stc(&c->heavy_rounds, heavy_rounds);
  stc(&c->lvl_sub0, lvl_sub0);
  stc(&c->prev_sub, prev_sub);
  stc(&c->t_dec, t_dec);
  stc(&c->phase, phase);
}

// Grid barrier without cache maintenance (see the coherence note above); the
// first wavefront of the last workgroup to arrive runs control_step before
// release.  Returns false if the wait timed out, and the kernel then winds down.
__device__ bool phase_barrier(PeelCtl* c, const PeelArgs& P) {
  __shared__ int s_ok, s_last;
  mem_wait();
  __syncthreads();
  unsigned gen = 0;
  if (threadIdx.x == 0) {
    gen = ldc(&c->bar_gen);
    // two-level arrival: the last workgroup of a group arrives for the group
    const unsigned g = blockIdx.x % kGroups;
    const unsigned gsize = (gridDim.x - g + kGroups - 1) / kGroups;
    const unsigned ngroups = gridDim.x < (unsigned)kGroups ? gridDim.x : (unsigned)kGroups;
    bool last = false;
    const unsigned pg = __hip_atomic_fetch_add(&c->grp_count[g][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (pg == gsize - 1) {
      stc(&c->grp_count[g][0], 0u);
      mem_wait();
      const unsigned prev = __hip_atomic_fetch_add(&c->bar_count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = prev == ngroups - 1;
    }
    s_last = last ? 1 : 0;
  }
  __syncthreads();
  if (s_last) {
    if (threadIdx.x < kWave) control_step(c, P);
    if (threadIdx.x == 0) {
      stc(&c->bar_count, 0u);
      mem_wait();
      __hip_atomic_fetch_add(&c->bar_gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_ok = 1;
    }
  } else if (threadIdx.x == 0) {
    int ok = 1;
    const uint64_t t0 = wall_clock64();
    while (ldc(&c->bar_gen) == gen) {
      __builtin_amdgcn_s_sleep(1);
      if (ldc(&c->abort)) { ok = 0; break; }
      // 100 MHz constant clock: give up after 30 s
      if (wall_clock64() - t0 > 3000000000ULL) {
        stc(&c->abort, 1);
        ok = 0;
        break;
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ bool removed_at(int rnd, int r) { return rnd != 0 && rnd < r; }

// NI adjacency entries of walks, one step at a time for all of them so that
// their memory accesses are in flight together.  Entry q is position j[q] of
// the row walked for frontier edge e[q] = (a, b[q]), valid if ok[q].  Outputs
// the (up to two) edges per entry whose support crossed k-1 -> k-2 and must be
// enqueued.
template <int NI>
__device__ __forceinline__ void process_entries(const PeelArgs& P, const int32_t (&e)[NI], const int32_t (&b)[NI],
                                                const int64_t (&j)[NI], bool (&ok)[NI], int r, int l, int k,
                                                bool sparse, int probe, int32_t (&f1)[NI], int32_t (&f2)[NI]) {
  int32_t w[NI], e1[NI], e2[NI], s1[NI], s2[NI];
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    f1[q] = -1;
    f2[q] = -1;
    w[q] = -1;
    e1[q] = 0;
    e2[q] = 0;
    s1[q] = 0;
    s2[q] = 0;
    if (ok[q]) {
      w[q] = P.col[j[q]];
      e1[q] = P.seid[j[q]];
    }
  }
  // the first other edge (a, w) must not be removed
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    ok[q] = ok[q] && w[q] != b[q];
    if (ok[q]) s1[q] = ldc_stamp(&P.sr[e1[q]]);
  }
#pragma unroll
  for (int q = 0; q < NI; ++q) ok[q] = ok[q] && !removed_at(s1[q], r);
  // the second other edge (b, w): b's row hash table, or a binary search of
  // b's sorted row (the entries of one walk look up the same row, so they
  // touch the same few cached lines either way)
  if (probe == 0) {
    const int2* tb[NI];
    uint32_t h[NI], mask[NI];
    int2 sl[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {  // the first slots of all lookups in flight together
      tb[q] = P.rtab;
      h[q] = 0;
      mask[q] = 0;
      sl[q] = make_int2(-1, 0);
      if (ok[q]) {
        const int64_t off = P.rtoff[b[q]];
        const int lg = row_table_lg(P.rtoff[b[q] + 1] - off);
        tb[q] = P.rtab + off;
        mask[q] = (1u << lg) - 1u;
        h[q] = row_slot(w[q], lg);
        sl[q] = tb[q][h[q]];
      }
    }
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      if (!ok[q]) continue;
      while (sl[q].x != w[q] && sl[q].x >= 0) {
        h[q] = (h[q] + 1) & mask[q];
        sl[q] = tb[q][h[q]];
      }
      e2[q] = sl[q].y;
      ok[q] = sl[q].x == w[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      if (!ok[q]) continue;
      const int64_t rb = P.row_ptr[b[q]];
      const int64_t re = rb + P.rlen[b[q]];
      const int64_t p = lower_bound_i32<int64_t>(P.col, rb, re, w[q]);
      if (p < re && P.col[p] == w[q]) e2[q] = P.seid[p];
      else ok[q] = false;
    }
  }
#pragma unroll
  for (int q = 0; q < NI; ++q)
    if (ok[q]) s2[q] = ldc_stamp(&P.sr[e2[q]]);
  // the triangle is destroyed now unless an edge is removed, and it belongs
  // to its frontier edge of smallest id; each other edge not in F_r loses one
  bool d1[NI], d2[NI];
  int old1[NI], old2[NI];
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    const bool live = ok[q] && !removed_at(s2[q], r) && !(s1[q] == r && e1[q] < e[q]) &&
                      !(s2[q] == r && e2[q] < e[q]);
    d1[q] = live && s1[q] != r;
    d2[q] = live && s2[q] != r;
    old1[q] = 0;
    old2[q] = 0;
    if (d1[q]) old1[q] = atomicSub(&P.sr[e1[q]].x, 1);
    if (d2[q]) old2[q] = atomicSub(&P.sr[e2[q]].x, 1);
  }
  if (!sparse) return;
#pragma unroll
  for (int q = 0; q < NI; ++q) {
    if (d1[q] && old1[q] == l + 1) {
      stc_stamp(&P.sr[e1[q]], r + 1);
      P.truss[e1[q]] = k;
      f1[q] = e1[q];
    }
    if (d2[q] && old2[q] == l + 1) {
      stc_stamp(&P.sr[e2[q]], r + 1);
      P.truss[e2[q]] = k;
      f2[q] = e2[q];
    }
  }
}

// Next-frontier edges are gathered per wavefront in LDS and appended to the
// global queue 64 or more at a time, so the queue counter sees one atomic per
// flush instead of one per wavefront iteration.
constexpr int kWq = 192;  // capacity: a flush happens before 64 + 2 * 64 entries are exceeded
struct WaveQueue {
  int* buf;     // LDS, kWq entries, private to the wavefront
  int cnt;      // wave-uniform fill level
  int32_t* q;   // global next-frontier queue
  int* count;   // its length
};

__device__ __forceinline__ void wq_flush(WaveQueue& wq) {
  if (wq.cnt == 0) return;
  wave_sync();
  int base = 0;
  if (lane_id() == 0) base = atomicAdd(wq.count, wq.cnt);
  base = __shfl(base, 0, kWave);
  for (int i = lane_id(); i < wq.cnt; i += kWave) stc(&wq.q[base + i], wq.buf[i]);
  wq.cnt = 0;
  wave_sync();
}

__device__ __forceinline__ void wq_push(WaveQueue& wq, int32_t f1, int32_t f2) {
  const uint64_t m1 = ballot(f1 >= 0);
  if (f1 >= 0) wq.buf[wq.cnt + rank_below(m1)] = f1;
  wq.cnt += __popcll(m1);
  const uint64_t m2 = ballot(f2 >= 0);
  if (f2 >= 0) wq.buf[wq.cnt + rank_below(m2)] = f2;
  wq.cnt += __popcll(m2);
  if (wq.cnt >= kWave) wq_flush(wq);
}

// Appends of a whole workgroup gathered in LDS and written to a global list in
// bulk, so that the list's counter sees one atomic per flush rather than one
// per 1024 entries.  Every thread of the workgroup calls append() and flush().
struct StagedList {
  int* buf;       // LDS, cap entries
  int cap;
  int* fill;      // LDS: entries held
  int* base;      // LDS: list position of a flush
  int* counter;   // global list length
  int32_t* out;   // global list
};

__device__ __forceinline__ void staged_flush(StagedList& L) {
  __syncthreads();
  const int n = *L.fill;
  if (n == 0) return;
  if (threadIdx.x == 0) *L.base = atomicAdd(L.counter, n);
  __syncthreads();
  const int b = *L.base;
  for (int i = threadIdx.x; i < n; i += kT) stc(&L.out[b + i], L.buf[i]);
  __syncthreads();
  if (threadIdx.x == 0) *L.fill = 0;
  __syncthreads();
}

// tmp: kWaves ints of LDS
__device__ __forceinline__ void staged_append(StagedList& L, bool want, int32_t val, int* tmp) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint64_t m = ballot(want);
  if (lane == 0) tmp[w] = __popcll(m);
  __syncthreads();
  int wbase = 0, tot = 0;
  for (int q = 0; q < kWaves; ++q) {
    const int x = tmp[q];
    if (q < w) wbase += x;
    tot += x;
  }
  if (*L.fill + tot > L.cap) staged_flush(L);
  const int f = *L.fill;
  if (want) L.buf[f + wbase + rank_below(m)] = val;
  __syncthreads();
  if (threadIdx.x == 0) *L.fill = f + tot;
  __syncthreads();
}

// The same for U candidate entries per thread (vals[u] kept where want[u]);
// a thread's kept entries stay in order and follow the previous thread's.
// U * kT must not exceed the list's LDS capacity.
template <int U>
__device__ __forceinline__ void staged_append_n(StagedList& L, const bool (&want)[U], const int32_t (&vals)[U],
                                                int* tmp) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int cnt = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) cnt += want[u] ? 1 : 0;
  const int incl = wave_inclusive_sum(cnt);
  if (lane == kWave - 1) tmp[w] = incl;
  __syncthreads();
  int wbase = 0, tot = 0;
  for (int q = 0; q < kWaves; ++q) {
    const int x = tmp[q];
    if (q < w) wbase += x;
    tot += x;
  }
  if (*L.fill + tot > L.cap) staged_flush(L);
  int pos = *L.fill + wbase + incl - cnt;
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (want[u]) L.buf[pos++] = vals[u];
  __syncthreads();
  if (threadIdx.x == 0) *L.fill += tot;
  __syncthreads();
}

// minimum over the workgroup into *dst (one atomic per workgroup); tmp: kWaves ints
__device__ __forceinline__ void block_min_to(int x, int* tmp, int* dst) {
  x = wave_min(x);
  if (lane_id() == 0) tmp[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int v = kIntMax;
    for (int q = 0; q < kWaves; ++q) v = tmp[q] < v ? tmp[q] : v;
    if (v != kIntMax) atomicMin(dst, v);
  }
  __syncthreads();
}

// sum over the workgroup into *dst (one atomic per workgroup); tmp: kWaves entries
__device__ __forceinline__ void block_sum_to(unsigned long long x, unsigned long long* tmp,
                                             unsigned long long* dst) {
  x = wave_sum(x);
  if (lane_id() == 0) tmp[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long v = 0;
    for (int q = 0; q < kWaves; ++q) v += tmp[q];
    if (v) atomicAdd(dst, v);
  }
  __syncthreads();
}

// Block-wide inclusive prefix sum of one int per thread; total in *total.
__device__ __forceinline__ int block_inclusive_sum(int x, int* tmp, int* total) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int inc = wave_inclusive_sum(x);
  if (lane == kWave - 1) tmp[w] = inc;
  __syncthreads();
  int base = 0, all = 0;
  for (int q = 0; q < kWaves; ++q) {
    const int v = tmp[q];
    if (q < w) base += v;
    all += v;
  }
  *total = all;
  __syncthreads();
  return base + inc;
}

// NI: walk entries in flight per thread; SU (2 or 4): live-list entries per
// thread and step of the level sweep
template <int NI, int SU>
__device__ __forceinline__ void peel_body(const PeelArgs& P) {
  static_assert(SU == 2 || SU == 4, "sweep step");
  __shared__ int s_pre[kT + 1];
  __shared__ int s_e[kT];
  __shared__ int s_b[kT];
  __shared__ int64_t s_base[kT];
  __shared__ int s_wq[kWaves][kWq];
  __shared__ int s_tmp[kWaves + 2];
  __shared__ int s_c0;
  __shared__ unsigned long long s_pv;
  __shared__ unsigned long long s_w64[kWaves];
  __shared__ int s_stage_a[kStageA];
  __shared__ int s_stage_q[kStageQ];
  __shared__ int s_fill[4];
  PeelCtl* c = P.ctl;
  if (threadIdx.x == 0) {
    s_fill[0] = 0;
    s_fill[2] = 0;
  }
  __syncthreads();
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wv = tid / kWave;
  unsigned long long my_work = 0;

  for (;;) {
    const int phase = ldc(&c->phase);
    if (phase == PH_DONE || phase == PH_COMPACT) break;
    const int k = ldc(&c->k);
    const int l = k - 2;
    const int r = ldc(&c->r);
    const int acur = ldc(&c->acur);
    if (phase == PH_SWEEP) {
      // live-edge list of the new level and its minimum support; the live
      // edges with sup <= k-1 are taken at once as the frontier of level k+1
      // (the control step keeps them only if that level is not skipped, in
      // which case none is taken)
      const int first = ldc(&c->first);
      const int64_t cnt = first ? P.m : (int64_t)ldc(&c->acnt);
      const int32_t* A = P.alist[acur];
      StagedList LA{s_stage_a, kStageA, &s_fill[0], &s_fill[1], &c->w_alive, P.alist[acur ^ 1]};
      StagedList LQ{s_stage_q, kStageQ, &s_fill[2], &s_fill[3], &c->w_qlen, P.fq[(r + 1) & 1]};
      const int kt = k + 1, stamp = r + 1;
      int mins = kIntMax;
      unsigned long long wsum = 0;
      // SU consecutive list entries a thread, their loads in flight together
      for (int64_t base = (int64_t)blockIdx.x * kT * SU; base < cnt; base += (int64_t)gridDim.x * kT * SU) {
        const int64_t i0 = base + (int64_t)tid * SU;
        int32_t e[SU];
        int2 sv[SU];
        bool live[SU], take[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          e[u] = 0;
          if (i0 + u < cnt) e[u] = first ? (int32_t)(i0 + u) : ldc(&A[i0 + u]);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          sv[u] = make_int2(0, 1);
          if (i0 + u < cnt) sv[u] = ldc2(&P.sr[e[u]]);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          live[u] = sv[u].y == 0;
          take[u] = false;
          if (live[u]) {
            mins = sv[u].x < mins ? sv[u].x : mins;
            take[u] = sv[u].x <= kt - 2;
            if (take[u]) {
              stc_stamp(&P.sr[e[u]], stamp);
              P.truss[e[u]] = kt;
              const int du = P.rlen[P.eu[e[u]]], dv = P.rlen[P.ev[e[u]]];
              wsum += (unsigned long long)(du < dv ? du : dv);
            }
          }
        }
        staged_append_n<SU>(LA, live, e, s_tmp);
        // the frontier stage holds two entries a thread per append
#pragma unroll
        for (int h = 0; h < SU; h += 2) {
          const bool th[2] = {take[h], take[h + 1]};
          const int32_t eh[2] = {e[h], e[h + 1]};
          staged_append_n<2>(LQ, th, eh, s_tmp);
        }
      }
      staged_flush(LA);
      staged_flush(LQ);
      block_min_to(mins, s_tmp, &c->w_minsup);
      block_sum_to(wsum, s_w64, &c->w_fwork);
    } else if (phase == PH_START || phase == PH_DENSE) {
      // collect live edges with sup <= k-2 (level start after a skip, or dense re-scan)
      const int64_t cnt = ldc(&c->acnt);
      const int32_t* A = P.alist[acur];
      const int stamp = phase == PH_START ? r : r + 1;
      StagedList LQ{s_stage_q, kStageQ, &s_fill[2], &s_fill[3], &c->w_qlen, P.fq[stamp & 1]};
      unsigned long long wsum = 0;  // level start: shorter live row over the frontier
      for (int64_t base = (int64_t)blockIdx.x * kT; base < cnt; base += (int64_t)gridDim.x * kT) {
        const int64_t i = base + tid;
        bool take = false;
        int32_t e = 0;
        if (i < cnt) {
          e = ldc(&A[i]);
          const int2 sv = ldc2(&P.sr[e]);
          take = sv.y == 0 && sv.x <= l;
          if (take) {
            stc_stamp(&P.sr[e], stamp);
            P.truss[e] = k;
            if (phase == PH_START) {
              const int du = P.rlen[P.eu[e]], dv = P.rlen[P.ev[e]];
              wsum += (unsigned long long)(du < dv ? du : dv);
            }
          }
        }
        staged_append(LQ, take, e, s_tmp);
      }
      staged_flush(LQ);
      if (phase == PH_START) block_sum_to(wsum, s_w64, &c->w_fwork);
    } else if (phase == PH_PROC) {
      const int qn = ldc(&c->qlen);
      const bool sparse = ldc(&c->mode) == TRUSS_PEEL_SPARSE;
      const int probe = ldc(&c->probe);
      const int32_t* Q = P.fq[r & 1];
      WaveQueue wq{s_wq[wv], 0, P.fq[(r + 1) & 1], &c->w_qlen};
      const unsigned long long cap = (unsigned long long)ldc(&c->pcap);
      unsigned long long* slots = P.pslot;
      // walk items [lo, hi) of the chunk held in the workgroup's LDS tables
      auto walk = [&](int lo, int hi) {
        for (int t0 = lo; t0 < hi; t0 += NI * kT) {
          int32_t e[NI], b[NI], f1[NI], f2[NI];
          int64_t j[NI];
          bool ok[NI];
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            const int t = t0 + q * kT + tid;
            ok[q] = t < hi;
            e[q] = 0;
            b[q] = 0;
            j[q] = 0;
            if (ok[q]) {
              int x = 0, y = kT - 1;  // last edge whose range starts at or before t
              while (x < y) {
                const int mid = (x + y + 1) >> 1;
                if (s_pre[mid] <= t) x = mid; else y = mid - 1;
              }
              e[q] = s_e[x];
              b[q] = s_b[x];
              j[q] = s_base[x] + (t - s_pre[x]);
            }
          }
          process_entries<NI>(P, e, b, j, ok, r, l, k, sparse, probe, f1, f2);
#pragma unroll
          for (int q = 0; q < NI; ++q) wq_push(wq, f1[q], f2[q]);
        }
        if (tid == 0) my_work += (unsigned long long)(hi - lo);
      };
      // (1) frontier edges in chunks of cs <= kT, one edge a thread (the first
      // chunk of every workgroup is static, the rest are fetched).  Small
      // frontiers are spread over all workgroups (cs ~ |F| / workgroups, at
      // least 64).  The walks of a chunk are laid end to end and cut into
      // segments of seg entries; the workgroup walks segment 0 and announces
      // the others for any workgroup to take.  A segment is announced by one
      // 64-bit store into a slot.
      const int cs = chunk_size(qn, (int)gridDim.x);
      const int seg = qn >= kSegLargeFrontier ? kSegLarge : kSegSmall;
      bool first_chunk = true;
      for (;;) {
        if (tid == 0) s_c0 = first_chunk ? (int)blockIdx.x * cs : (int)gridDim.x * cs + atomicAdd(&c->w_fetch, cs);
        first_chunk = false;
        __syncthreads();
        const int c0 = s_c0;
        if (c0 >= qn) break;
        const int i = c0 + tid;
        int32_t e = 0, a = 0, b = 0;
        int work = 0;
        if (tid < cs && i < qn) {
          e = ldc(&Q[i]);
          const int32_t u = P.eu[e], v = P.ev[e];
          const int du = P.rlen[u], dv = P.rlen[v];
          const bool ua = du < dv || (du == dv && u < v);
          a = ua ? u : v;
          b = ua ? v : u;
          work = ua ? du : dv;
        }
        const int64_t ra = P.row_ptr[a];
        int W = 0;
        const int inc = block_inclusive_sum(work, s_tmp, &W);
        s_pre[tid + 1] = inc;
        if (tid == 0) s_pre[0] = 0;
        s_e[tid] = e;
        s_b[tid] = b;
        s_base[tid] = ra;
        const int nseg = (W + seg - 1) / seg;
        int npub = 0;  // segments 1..npub are announced
        if (nseg > 1) {
          // chunk tables for other workgroups, then the segment announcements
          if (tid < cs) {
            stc(&P.rec_e[i], e);
            stc(&P.rec_b[i], b);
            stc(&P.rec_base[i], ra);
            stc(&P.rec_pre[i], inc - work);
          }
          if (tid == 0) stc(&P.rec_tot[c0 / cs], W);
          mem_wait();
          __syncthreads();
          if (tid == 0) s_pv = atomicAdd(&c->w_pieces, (unsigned long long)(nseg - 1));
          __syncthreads();
          const unsigned long long pbase = s_pv;
          const unsigned long long room = pbase < cap ? cap - pbase : 0ULL;
          npub = room < (unsigned long long)(nseg - 1) ? (int)room : nseg - 1;
          const unsigned long long code0 = (unsigned long long)(c0 + 1) << 32;
          for (int sg = 1 + tid; sg <= npub; sg += kT)
            stc(&slots[pbase + (unsigned long long)(sg - 1)], code0 | (unsigned)sg);
        }
        __syncthreads();
        walk(0, W < seg ? W : seg);
        // segments that found no slot
        for (int sg = npub + 1; sg < nseg; ++sg) walk(sg * seg, (sg + 1) * seg < W ? (sg + 1) * seg : W);
        if (tid == 0) atomicAdd(&c->w_chunks, 1);
        __syncthreads();
      }
      // (2) take announced segments.  A workgroup draws one index of the
      // announcement order at a time and keeps it until that slot is
      // announced (then takes and clears it) or until every chunk is finished
      // with fewer announcements than the index (then stops).  Indices are
      // drawn in order and never dropped, so each announced slot is taken
      // exactly once.
      const int nchunks = (qn + cs - 1) / cs;
      for (;;) {
        if (tid == 0) {
          unsigned long long pv = ~0ULL;
          // nothing announced and nothing left to announce: skip the draw
          bool draw = true;
          const uint64_t t0 = wall_clock64();
          for (;;) {
            if (ldc(&c->w_chunks) >= nchunks && ldc(&c->w_pieces) == 0ULL) {
              draw = false;
              break;
            }
            if (ldc(&c->w_pieces) != 0ULL) break;
            __builtin_amdgcn_s_sleep(2);
            if (wall_clock64() - t0 > 3000000000ULL) {  // 30 s: give up, wind down
              stc(&c->abort, 1);
              draw = false;
              break;
            }
          }
          if (draw) {
            const unsigned long long q = atomicAdd(&c->w_pfetch, 1ULL);
            for (;;) {
              const unsigned long long cl = ldc(&c->w_pieces);
              const unsigned long long limit = cl < cap ? cl : cap;
              if (q < limit) {
                // the owner announces right after claiming the slot range
                unsigned long long v;
                while ((v = ldc(&slots[q])) == 0ULL) {
                  __builtin_amdgcn_s_sleep(1);
                  if (wall_clock64() - t0 > 3000000000ULL) break;
                }
                if (v == 0ULL) {
                  stc(&c->abort, 1);
                  break;
                }
                stc(&slots[q], 0ULL);
                pv = v;
                break;
              }
              if (ldc(&c->w_chunks) >= nchunks) {
                const unsigned long long cl2 = ldc(&c->w_pieces);
                if (q >= (cl2 < cap ? cl2 : cap)) break;  // final count reached: stop
                continue;
              }
              __builtin_amdgcn_s_sleep(2);
              if (wall_clock64() - t0 > 3000000000ULL) {  // 30 s: give up, wind down
                stc(&c->abort, 1);
                break;
              }
            }
          }
          s_pv = pv;
        }
        __syncthreads();
        const unsigned long long pv = s_pv;
        __syncthreads();
        if (pv == ~0ULL) break;
        const int c0 = (int)(pv >> 32) - 1;
        const int sg = (int)(pv & 0xffffffffu);
        const int i = c0 + tid;
        const bool ok = tid < cs && i < qn;
        s_pre[tid] = ok ? ldc(&P.rec_pre[i]) : kIntMax;
        s_e[tid] = ok ? ldc(&P.rec_e[i]) : 0;
        s_b[tid] = ok ? ldc(&P.rec_b[i]) : 0;
        s_base[tid] = ok ? ldc(&P.rec_base[i]) : 0;
        const int W = ldc(&P.rec_tot[c0 / cs]);
        if (tid == 0) s_pre[kT] = W;
        __syncthreads();
        walk(sg * seg, (sg + 1) * seg < W ? (sg + 1) * seg : W);
        __syncthreads();
      }
      wq_flush(wq);
    }
    if (!phase_barrier(c, P)) break;
  }
  if (tid == 0 && my_work) atomicAdd(&c->w_work, my_work);
}

// The persistent peeling kernel in two shapes over the same state machine:
// one 1024-thread workgroup per compute unit with four walk entries in flight
// per thread, or two workgroups per compute unit (registers capped for eight
// wavefronts per SIMD) with two entries per thread, which hides more latency
// when walks are long.  All state lives in global memory between launches.
__global__ void __launch_bounds__(kT) k_peel(PeelArgs P) { peel_body<4, 4>(P); }
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(8, 8))) k_peel_wide(PeelArgs P) {
  peel_body<2, 2>(P);
}

// One bit per edge, set when the edge is removed: the liveness test of the
// row compaction reads this bitmap (m/8 bytes, cache-resident) instead of
// one scattered support/stamp pair per row entry.
__global__ void __launch_bounds__(256) k_dead_bits(const int2* __restrict__ sr, int64_t m,
                                                   unsigned long long* __restrict__ dead) {
  const int lane = lane_id();
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t base = gw * kWave; base < m; base += nw * kWave) {
    const int64_t e = base + lane;
    const unsigned long long bits = ballot(e < m && sr[e].y != 0);
    if (lane == 0) dead[base / kWave] = bits;
  }
}

// Stable in-place compaction of every row to its live entries (a wavefront a row).
constexpr int kCompactUnroll = 4;
__global__ void __launch_bounds__(256) k_compact(const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                 int32_t* __restrict__ seid, int32_t* __restrict__ rlen, int32_t n,
                                                 const unsigned long long* __restrict__ dead, PeelCtl* c) {
  const int lane = lane_id();
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  if (gw == 0 && lane == 0) {
    c->phase = PH_SWEEP;
    c->t_last = 0;
  }
  for (int64_t v = gw; v < n; v += nw) {
    const int64_t rb = row_ptr[v];
    const int len = rlen[v];
    int wpos = 0;
    // kCompactUnroll chunks of kWave entries are read before any is written
    // back, so their loads overlap; entries only move to lower positions, so
    // the writes never reach an entry that has not been read
    for (int c0 = 0; c0 < len; c0 += kCompactUnroll * kWave) {
      int32_t x[kCompactUnroll], ed[kCompactUnroll];
      bool keep[kCompactUnroll];
#pragma unroll
      for (int u = 0; u < kCompactUnroll; ++u) {
        const int i = c0 + u * kWave + lane;
        x[u] = 0;
        ed[u] = 0;
        if (i < len) {
          x[u] = col[rb + i];
          ed[u] = seid[rb + i];
        }
      }
#pragma unroll
      for (int u = 0; u < kCompactUnroll; ++u) {
        const int i = c0 + u * kWave + lane;
        keep[u] = i < len && ((dead[ed[u] >> 6] >> (ed[u] & 63)) & 1ULL) == 0;
      }
#pragma unroll
      for (int u = 0; u < kCompactUnroll; ++u) {
        const uint64_t km = ballot(keep[u]);
        if (keep[u]) {
          const int64_t dst = rb + wpos + rank_below(km);
          col[dst] = x[u];
          seid[dst] = ed[u];
        }
        wpos += __popcll(km);
      }
    }
    if (lane == 0) rlen[v] = wpos;
  }
}

__global__ void k_peel_init(PeelCtl* c, const int64_t* __restrict__ row_ptr, int32_t* __restrict__ rlen, int32_t n,
                            int64_t m, long long max_subrounds, int sched, int fix_bits, int fix_vals, int pcap,
                            unsigned long long* __restrict__ pslot, int first_level, int stop_level) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rlen[i] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
  if (i < pcap) pslot[i] = 0ULL;
  if (i == 0) {
    c->bar_count = 0;
    c->bar_gen = 0;
    for (int g = 0; g < kGroups; ++g) c->grp_count[g][0] = 0;
    c->w_fetch = 0;
    c->w_qlen = 0;
    c->w_alive = 0;
    c->w_minsup = kIntMax;
    c->w_pfetch = 0ULL;
    c->w_chunks = 0;
    c->w_pieces = 0ULL;
    c->w_work = 0ULL;
    c->w_fwork = 0ULL;
    c->phase = PH_SWEEP;
    c->k = first_level - 1;  // the first sweep takes the frontier of level first_level
    c->r = 0;
    c->qlen = 0;
    c->acnt = (int)m;
    c->acur = 0;
    c->first = 1;
    c->mode = TRUSS_PEEL_SPARSE;
    c->pcap = pcap;
    c->kmax = 0;
    c->levels = 0;
    c->removed_level = 0;
    c->csr_live = m;
    c->subrounds = 0;
    c->heavy_rounds = 0;
    c->max_subrounds = max_subrounds;
    for (int b = 0; b < kHistBins; ++b) c->hist[b] = 0;
    c->t_last = 0;
    for (int b = 0; b < 8; ++b) c->t_phase[b] = 0;
    c->err = 0;
    c->abort = 0;
    c->launches = 0;
    c->probe = 0;
    c->sched = sched;
    c->fix_bits = fix_bits;
    c->fix_vals = fix_vals;
    c->stop_level = stop_level;
    c->m_edges = (int)m;
    c->lvl_sub0 = 0;
    c->prev_sub = 0;
    c->t_dec = 0;
  }
}

struct PeelLayout {
  PeelCtl* ctl;
  int32_t* rlen;
  int32_t* alist[2];
  int32_t* fq[2];
  unsigned long long* pslot;
  int32_t *rec_e, *rec_b, *rec_pre, *rec_tot;
  int64_t* rec_base;
  unsigned long long* dead;  // removed-edge bitmap for the row compaction
  int pcap;
};

void carve(const DevGraph& dg, Arena& a, PeelLayout& L) {
  const int64_t m = dg.m;
  L.ctl = a.take<PeelCtl>(1);
  L.rlen = a.take<int32_t>(dg.n + 1);
  for (int i = 0; i < 2; ++i) L.alist[i] = a.take<int32_t>(m + 1);
  for (int i = 0; i < 2; ++i) L.fq[i] = a.take<int32_t>(m + 1);
  L.pcap = (int)(m < (1 << 22) ? m : (1 << 22));
  L.pslot = a.take<unsigned long long>(L.pcap + 1);
  L.rec_e = a.take<int32_t>(m + kT);
  L.rec_b = a.take<int32_t>(m + kT);
  L.rec_pre = a.take<int32_t>(m + kT);
  L.rec_base = a.take<int64_t>(m + kT);
  L.rec_tot = a.take<int32_t>(m / kMinChunk + 2);
  L.dead = a.take<unsigned long long>(m / kWave + 2);
}

int g_peel_blocks = 0;       // grid of k_peel: one workgroup per compute unit
int g_peel_wide_blocks = -1;  // grid of k_peel_wide (two per compute unit), 0 if it does not fit

// TRUSS_SHAPE_AUTO takes the wide shape from this many edges on: there its
// extra wavefronts hide the latency of long walks in every launch, while on
// smaller graphs the shorter rounds favour the narrow shape (fewer workgroups
// at each barrier, more entries in flight per thread).
constexpr long long kWideMinEdges = 1LL << 27;

}  // namespace

size_t peel_workspace(const DevGraph& dg, Arena& a) {
  PeelLayout L;
  carve(dg, a, L);
  return a.used;
}

int peel(const DevGraph& dg, const PeelPlan& plan, int2* sr, int32_t* truss_canon, Arena& a, PeelResult* res,
         hipStream_t s, truss_trace* trace) {
  PeelLayout L;
  carve(dg, a, L);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  *res = PeelResult();
  if (dg.m == 0) return TRUSS_OK;
  const long long maxsr = plan.max_subrounds;
  int64_t initn = dg.n > L.pcap ? dg.n : L.pcap;
  if (initn < 1) initn = 1;
  hipLaunchKernelGGL(k_peel_init, dim3((unsigned)((initn + 255) / 256)), dim3(256), 0, s, L.ctl, dg.row_ptr, L.rlen,
                     dg.n, dg.m, maxsr, plan.sched, plan.fix_bits, plan.fix_vals, L.pcap, L.pslot,
                     plan.first_level < 2 ? 2 : plan.first_level, plan.stop_level);
  if (g_peel_blocks == 0) {
    int dev = 0, cus = 0, occ = 0;
    TRUSS_HIP(hipGetDevice(&dev));
    TRUSS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    TRUSS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_peel, kT, 0));
    if (occ < 1) {
      set_last_error("peeling kernel does not fit on a compute unit");
      return TRUSS_E_DEVICE;
    }
    g_peel_blocks = cus;
    int occw = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occw, (const void*)k_peel_wide, kT, 0) != hipSuccess) occw = 0;
    g_peel_wide_blocks = occw >= 2 ? 2 * cus : 0;
  }
  int blocks = g_peel_blocks;
  if (plan.grid_blocks > 0 && plan.grid_blocks < blocks) blocks = plan.grid_blocks;
  // a caller-fixed grid keeps the narrow shape
  const bool wide = plan.grid_blocks <= 0 && g_peel_wide_blocks > 0 &&
                    (plan.shape == TRUSS_SHAPE_WIDE || (plan.shape == TRUSS_SHAPE_AUTO && dg.m >= kWideMinEdges));
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
  for (int i = 0; i < 2; ++i) {
    P.alist[i] = L.alist[i];
    P.fq[i] = L.fq[i];
  }
  P.pslot = L.pslot;
  P.rec_e = L.rec_e;
  P.rec_b = L.rec_b;
  P.rec_pre = L.rec_pre;
  P.rec_base = L.rec_base;
  P.rec_tot = L.rec_tot;
  P.rtab = dg.rtab;
  P.rtoff = dg.rtoff;
  P.ctl = L.ctl;
  P.model = plan.sched == TRUSS_SCHED_LEARNED ? plan.model : nullptr;
  P.tr_cap = trace && trace->level_feat && trace->level_ms && trace->level_action ? trace->level_cap : 0;
  P.tr_feat = P.tr_cap > 0 ? trace->level_feat : nullptr;
  P.tr_ms = P.tr_cap > 0 ? trace->level_ms : nullptr;
  P.tr_act = P.tr_cap > 0 ? trace->level_action : nullptr;
  PeelCtl h;
  int launches = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  const bool timed = plan.timed && hipEventCreate(&ev0) == hipSuccess && hipEventCreate(&ev1) == hipSuccess;
  double kernel_ms = 0.0;
  for (;;) {
    if (timed) (void)hipEventRecord(ev0, s);
    if (wide)
      hipLaunchKernelGGL(k_peel_wide, dim3(g_peel_wide_blocks), dim3(kT), 0, s, P);
    else
      hipLaunchKernelGGL(k_peel, dim3(blocks), dim3(kT), 0, s, P);
    TRUSS_HIP(hipGetLastError());
    if (timed) (void)hipEventRecord(ev1, s);
    ++launches;
    TRUSS_HIP(hipMemcpyAsync(&h, L.ctl, sizeof(PeelCtl), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    if (timed) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev0, ev1) == hipSuccess) kernel_ms += t;
    }
    if (h.abort || h.err || h.phase != PH_COMPACT) break;
    hipLaunchKernelGGL(k_dead_bits, dim3(4096), dim3(256), 0, s, sr, dg.m, L.dead);
    hipLaunchKernelGGL(k_compact, dim3(2048), dim3(256), 0, s, dg.row_ptr, dg.col, dg.seid, L.rlen, dg.n, L.dead,
                       L.ctl);
  }
  if (ev0) (void)hipEventDestroy(ev0);
  if (ev1) (void)hipEventDestroy(ev1);
  res->kernel_ms = kernel_ms;
  if (trace) trace->levels = h.levels < P.tr_cap ? h.levels : P.tr_cap;
  res->kmax = h.kmax;
  res->levels = h.levels;
  res->subrounds = h.subrounds;
  res->work = (int64_t)h.w_work;
  res->launches = launches;
  res->heavy_rounds = h.heavy_rounds;
  for (int b = 0; b < kHistBins; ++b) res->hist[b] = h.hist[b];
  for (int b = 0; b < 6; ++b) res->phase_ms[b] = (double)h.t_phase[b] * 1e-5;
  if (h.abort) {
    set_last_error("peeling kernel barrier timed out");
    return TRUSS_E_INTERNAL;
  }
  if (h.err) {
    set_last_error("peeling exceeded the sub-round cap (%lld)", (long long)h.max_subrounds);
    return h.err;
  }
  if (h.phase != PH_DONE) {
    set_last_error("peeling stopped in phase %d", h.phase);
    return TRUSS_E_INTERNAL;
  }
  return TRUSS_OK;
}

}  // namespace truss
