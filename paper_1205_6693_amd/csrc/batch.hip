// Batched truss decomposition: many independent graphs in one persistent launch.
//
// Triangles never cross graphs (Definitions 1 and 2 are per connected piece),
// so each graph is decomposed on its own.  One workgroup takes one graph at a
// time from a queue ordered largest first, and runs the whole method on it with
// workgroup barriers only: canonical edges and validation, a symmetric CSR in
// the workgroup's scratch slot, rows sorted by neighbour id (a rank sort that
// also finds duplicate edges), the support of every edge by intersecting the
// shorter endpoint row with the longer one (Definition 1), and
// level-synchronous peeling of Algorithm 2, with the same
// snapshot frontier, smallest-id ownership and exactly-once decrements as the
// device-wide path.  Edge ids are the graph's input positions, so truss
// numbers land directly in the caller's packed output.
//
// All the scratch a graph touches belongs to one workgroup, which runs on one
// compute unit; workgroup barriers order its global-memory traffic, and no
// other workgroup reads it.
//
// Shapes: T threads per workgroup and NI walk entries in flight per thread
// (peeling walks are flattened over the workgroup; each thread advances NI
// entries step by step so their memory accesses overlap).  Both are template
// parameters picked by the autotuner.
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kIntMax = 0x7fffffff;
constexpr int64_t kBatchMaxM = 1 << 21;  // larger graphs take the device-wide path
constexpr int64_t kBatchMaxN = 1 << 22;

struct BatchCtl {
  int next;        // queue head
  int err_g;       // smallest failing graph index
  int kmax;
  int pad;
  unsigned long long levels, subrounds, triangles3;
  unsigned long long sup_work, peel_work;  // row entries walked (support, peeling)
  unsigned long long t_phase[3];            // workgroup time in CSR build, support, peeling (10 ns ticks)
};

struct BatchArgs {
  int G;                   // graphs in the queue
  const int32_t* order;    // queue: graph ids, largest first
  const int64_t* vo;       // G+1 vertex offsets (device copy)
  const int64_t* eo;       // G+1 edge offsets (device copy)
  const int32_t* src;
  const int32_t* dst;
  int32_t* out;
  int32_t* gerr;           // per graph status
  char* scratch;
  size_t slot_bytes;
  int32_t max_n;
  int64_t max_m;
  BatchCtl* ctl;
};

struct Slot {
  int32_t *rp, *cur, *col, *eid, *eu, *ev, *sup, *stamp;
  int32_t *colA, *eidA;  // unsorted rows; later the frontier queues and live lists
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ inline size_t slot_bytes_for(int64_t max_n, int64_t max_m) {
  const size_t nb = align256((size_t)(max_n + 1) * 4), mb = align256((size_t)(max_m + 1) * 4),
               m2 = align256((size_t)(2 * max_m + 1) * 4);
  return 2 * nb + 4 * m2 + 4 * mb;
}

__device__ inline Slot slot_at(const BatchArgs& A, int s) {
  char* p = A.scratch + (size_t)s * A.slot_bytes;
  const size_t nb = align256((size_t)(A.max_n + 1) * 4), mb = align256((size_t)(A.max_m + 1) * 4),
               m2 = align256((size_t)(2 * A.max_m + 1) * 4);
  Slot S;
  S.rp = (int32_t*)p;
  p += nb;
  S.cur = (int32_t*)p;
  p += nb;
  S.col = (int32_t*)p;
  p += m2;
  S.eid = (int32_t*)p;
  p += m2;
  S.colA = (int32_t*)p;
  p += m2;
  S.eidA = (int32_t*)p;
  p += m2;
  S.eu = (int32_t*)p;
  p += mb;
  S.ev = (int32_t*)p;
  p += mb;
  S.sup = (int32_t*)p;
  p += mb;
  S.stamp = (int32_t*)p;
  return S;
}

// Reads of scratch that the workgroup itself writes: atomic loads are never
// turned into scalar-cache loads.
__device__ __forceinline__ int ldw(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

constexpr int kSweepNI = 4;                    // live-list entries per thread per sweep step
constexpr int kBitmapWords = 256;              // per wavefront: graphs with up to 8192 vertices
constexpr int kBitmapBits = kBitmapWords * 32;
constexpr int kStageRow = 4096;                // longest row ranked from an LDS copy
constexpr int kLongRows = 512;                 // rows longer than kBitmapWords listed per graph

template <int T>
struct Lds {
  unsigned bits[T / kWave][kBitmapWords];
  int pre[T / kWave][kWave];
  int rowst[T / kWave][kWave];
  int cnt64[T / kWave][kWave];
  int stage[kStageRow];   // a long row being ranked
  int longrow[kLongRows];
  int nlong;
  long long wpre[T + 1];  // flattened walk of a frontier chunk: prefix of walk lengths
  long long wtot[T / kWave];
  int we[T], wb[T], wra[T], wrb[T], wlb[T];
  int tmp[T / kWave + 2];
  int err;
  int cnt;
  int minv;
  int qn;
  int g;
};

// exclusive prefix sum of in[0..n) into out[0..n], out[n] = total
template <int T>
__device__ void block_scan(const int32_t* in, int32_t* out, int n, Lds<T>& L) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int carry = 0;
  for (int t0 = 0; t0 < n; t0 += T) {
    const int x = t0 + threadIdx.x;
    const int v = x < n ? ldw(&in[x]) : 0;
    const int inc = wave_inclusive_sum(v);
    if (lane == kWave - 1) L.tmp[w] = inc;
    __syncthreads();
    int base = 0, tot = 0;
    for (int q = 0; q < T / kWave; ++q) {
      const int y = L.tmp[q];
      if (q < w) base += y;
      tot += y;
    }
    if (x < n) out[x] = carry + base + inc - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

// inclusive prefix sum over the workgroup of one value per thread
template <int T>
__device__ long long block_scan64(long long v, Lds<T>& L) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const long long inc = wave_inclusive_sum(v);
  if (lane == kWave - 1) L.wtot[w] = inc;
  __syncthreads();
  long long base = 0;
  for (int q = 0; q < w; ++q) base += L.wtot[q];
  __syncthreads();
  return base + inc;
}

// slot in an LDS counter for each lane with `want` (one LDS atomic per wavefront)
__device__ __forceinline__ int lds_append(int* counter, bool want) {
  const uint64_t m = ballot(want);
  if (m == 0) return 0;
  const int leader = __builtin_ctzll(m);
  int base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, __popcll(m));
  base = __shfl(base, leader, kWave);
  return base + rank_below(m);
}

__device__ __forceinline__ bool removed_at(int s, int r) { return s != 0 && s < r; }

// position of `key` in the sorted row [lo, hi), or -1
__device__ __forceinline__ int row_find(const int32_t* col, int lo, int hi, int key) {
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if (ldw(&col[mid]) < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <int T, int NI>
__device__ void process_graph(const BatchArgs& A, const Slot& S, int g, Lds<T>& L) {
  const int tid = threadIdx.x, lane = lane_id(), wv = tid / kWave;
  constexpr int kWavesT = T / kWave;
  const int n = (int)(A.vo[g + 1] - A.vo[g]);
  const int m = (int)(A.eo[g + 1] - A.eo[g]);
  const int32_t* src = A.src + A.eo[g];
  const int32_t* dst = A.dst + A.eo[g];
  int32_t* out = A.out + A.eo[g];
  if (m == 0) {
    if (tid == 0) A.gerr[g] = 0;
    return;
  }
  const unsigned long long t0 = wall_clock64();
  // 1. degrees of the canonical edges; range and self-loop checks (Section 2: simple graphs)
  for (int x = tid; x <= n; x += T) S.cur[x] = 0;
  if (tid == 0) L.err = kNoErr;
  __syncthreads();
  for (int i = tid; i < m; i += T) {
    const int u = src[i], v = dst[i];
    int e = 0;
    if (u < 0 || u >= n || v < 0 || v >= n) e = kErrRange;
    else if (u == v) e = kErrSelfloop;
    if (e) {
      atomicMin(&L.err, e);
      continue;
    }
    const int a = u < v ? u : v, b = u < v ? v : u;
    S.eu[i] = a;
    S.ev[i] = b;
    atomicAdd(&S.cur[a], 1);
    atomicAdd(&S.cur[b], 1);
  }
  __syncthreads();
  if (L.err != kNoErr) {
    if (tid == 0) {
      A.gerr[g] = -L.err;
      atomicMin(&A.ctl->err_g, g);
    }
    return;
  }
  // 2. symmetric CSR: offsets, then every edge into both rows (unordered)
  block_scan<T>(S.cur, S.rp, n, L);
  __syncthreads();
  for (int x = tid; x < n; x += T) S.cur[x] = ldw(&S.rp[x]);
  __syncthreads();
  for (int i = tid; i < m; i += T) {
    const int a = ldw(&S.eu[i]), b = ldw(&S.ev[i]);
    const int p = atomicAdd(&S.cur[a], 1);
    S.colA[p] = b;
    S.eidA[p] = i;
    const int q = atomicAdd(&S.cur[b], 1);
    S.colA[q] = a;
    S.eidA[q] = i;
  }
  __syncthreads();
  // 3. rows sorted by neighbour id: each entry's rank in its row is the count
  // of smaller neighbours; an equal neighbour is a duplicated edge.  A
  // wavefront per row: up to 64 entries compared in registers, up to
  // kBitmapWords staged in the wavefront's LDS; longer rows are listed and
  // ranked afterwards by the whole workgroup from an LDS copy.
  if (tid == 0) L.nlong = 0;
  __syncthreads();
  for (int x = wv; x < n; x += kWavesT) {
    const int base = ldw(&S.rp[x]);
    const int len = ldw(&S.rp[x + 1]) - base;
    if (len <= kWave) {
      const bool ok = lane < len;
      const int cj = ok ? ldw(&S.colA[base + lane]) : kIntMax;
      const int ej = ok ? ldw(&S.eidA[base + lane]) : 0;
      int rank = 0, eq = 0;
      for (int t = 0; t < len; ++t) {
        const int ct = __shfl(cj, t, kWave);
        rank += ct < cj;
        eq += ct == cj;
      }
      if (ok) {
        S.col[base + rank] = cj;
        S.eid[base + rank] = ej;
        if (eq > 1) atomicMin(&L.err, kErrDup);
      }
    } else if (len <= kBitmapWords) {
      int* st = reinterpret_cast<int*>(L.bits[wv]);
      for (int j = lane; j < len; j += kWave) st[j] = ldw(&S.colA[base + j]);
      wave_sync();
      for (int j = lane; j < len; j += kWave) {
        const int cj = st[j];
        int rank = 0, eq = 0;
        for (int t = 0; t < len; ++t) {
          const int ct = st[t];
          rank += ct < cj;
          eq += ct == cj;
        }
        S.col[base + rank] = cj;
        S.eid[base + rank] = ldw(&S.eidA[base + j]);
        if (eq > 1) atomicMin(&L.err, kErrDup);
      }
      wave_sync();
    } else if (lane == 0) {
      const int q = atomicAdd(&L.nlong, 1);
      if (q < kLongRows) L.longrow[q] = x;
    }
  }
  __syncthreads();
  const int nlong = L.nlong < kLongRows ? L.nlong : kLongRows;
  const bool long_overflow = L.nlong > kLongRows;
  for (int q = 0; q < nlong + (long_overflow ? 1 : 0); ++q) {
    // q == nlong (after an overflow of the list): every long row not listed
    int x0 = 0, x1 = 0;
    if (q < nlong) {
      x0 = L.longrow[q];
      x1 = x0 + 1;
    } else {
      x0 = 0;
      x1 = n;
    }
    for (int x = x0; x < x1; ++x) {
      const int base = ldw(&S.rp[x]);
      const int len = ldw(&S.rp[x + 1]) - base;
      if (len <= kBitmapWords) continue;
      if (q == nlong) {
        bool listed = false;
        for (int y = 0; y < nlong; ++y) listed = listed || L.longrow[y] == x;
        if (listed) continue;
      }
      const bool staged = len <= kStageRow;
      if (staged)
        for (int j = tid; j < len; j += T) L.stage[j] = ldw(&S.colA[base + j]);
      __syncthreads();
      for (int j = tid; j < len; j += T) {
        const int cj = staged ? L.stage[j] : ldw(&S.colA[base + j]);
        int rank = 0, eq = 0;
        for (int t = 0; t < len; ++t) {
          const int ct = staged ? L.stage[t] : ldw(&S.colA[base + t]);
          rank += ct < cj;
          eq += ct == cj;
        }
        S.col[base + rank] = cj;
        S.eid[base + rank] = ldw(&S.eidA[base + j]);
        if (eq > 1) atomicMin(&L.err, kErrDup);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  if (L.err != kNoErr) {
    if (tid == 0) {
      A.gerr[g] = -L.err;
      atomicMin(&A.ctl->err_g, g);
    }
    return;
  }
  const unsigned long long t1 = wall_clock64();
  // live row lengths for peeling (cur is free after the scatter)
  for (int x = tid; x < n; x += T) S.cur[x] = ldw(&S.rp[x + 1]) - ldw(&S.rp[x]);
  // 4. support (Definition 1): each edge walks its shorter endpoint row and
  // looks every neighbour up in the other row
  unsigned long long tri3 = 0, wsup = 0, wpeel = 0;
  if (n <= kBitmapBits) {
    // the longer endpoint u's row as a bitmap in LDS (a wavefront per u):
    // every shorter neighbour v walks its row and tests the bits
    unsigned* bm = L.bits[wv];
    for (int x = lane; x < kBitmapWords; x += kWave) bm[x] = 0u;
    wave_sync();
    for (int u = wv; u < n; u += kWavesT) {
      const int ru = ldw(&S.rp[u]), du = ldw(&S.rp[u + 1]) - ru;
      if (du == 0) continue;
      for (int j = lane; j < du; j += kWave) {
        const int w = ldw(&S.col[ru + j]);
        atomicOr(&bm[w >> 5], 1u << (w & 31));
      }
      wave_sync();
      for (int c0 = 0; c0 < du; c0 += kWave) {
        // shorter neighbours among this 64-entry chunk of the row, their rows flattened
        const int j = c0 + lane;
        int v = 0, rv = 0, dv = 0, e = 0;
        bool shorter = false;
        if (j < du) {
          v = ldw(&S.col[ru + j]);
          e = ldw(&S.eid[ru + j]);
          rv = ldw(&S.rp[v]);
          dv = ldw(&S.rp[v + 1]) - rv;
          shorter = dv < du || (dv == du && v < u);
        }
        const int len = shorter ? dv : 0;
        const int inc = wave_inclusive_sum(len);
        const int tot = __shfl(inc, kWave - 1, kWave);
        // the flattened walk: slot q covers [pre[q], pre[q] + len of lane q)
        // and starts at row offset rowst[q]
        L.pre[wv][lane] = inc - len;
        L.rowst[wv][lane] = rv;
        L.cnt64[wv][lane] = 0;
        wave_sync();
        for (int t0 = 0; t0 < tot; t0 += kWave) {
          const int t = t0 + lane;
          if (t < tot) {
            int lo = 0, hi = kWave - 1;  // last slot whose range starts at or before t
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (L.pre[wv][mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int w = ldw(&S.col[L.rowst[wv][lo] + (t - L.pre[wv][lo])]);
            if (bm[w >> 5] >> (w & 31) & 1u) atomicAdd(&L.cnt64[wv][lo], 1);
          }
        }
        wave_sync();
        if (shorter) {
          const int cnt = L.cnt64[wv][lane];
          S.sup[e] = cnt;
          S.stamp[e] = 0;
          tri3 += (unsigned long long)cnt;
          wsup += (unsigned long long)dv;
        }
        wave_sync();
      }
      for (int j = lane; j < du; j += kWave) {
        const int w = ldw(&S.col[ru + j]);
        bm[w >> 5] = 0u;
      }
      wave_sync();
    }
  } else {
    // larger graphs: a thread per edge, binary search of the longer row
    for (int i = tid; i < m; i += T) {
      const int u = ldw(&S.eu[i]), v = ldw(&S.ev[i]);
      const int ru = ldw(&S.rp[u]), du = ldw(&S.rp[u + 1]) - ru;
      const int rv = ldw(&S.rp[v]), dv = ldw(&S.rp[v + 1]) - rv;
      const bool ua = du < dv || (du == dv && u < v);
      const int wa = ua ? ru : rv, la = ua ? du : dv;
      const int wb = ua ? rv : ru, lb = ua ? dv : du;
      int cnt = 0;
      for (int j = 0; j < la; ++j) {
        const int w = ldw(&S.col[wa + j]);
        const int p = row_find(S.col, wb, wb + lb, w);
        cnt += (p < wb + lb && ldw(&S.col[p]) == w) ? 1 : 0;
      }
      S.sup[i] = cnt;
      S.stamp[i] = 0;
      tri3 += (unsigned long long)cnt;
      wsup += (unsigned long long)la;
    }
  }
  __syncthreads();
  const unsigned long long t2 = wall_clock64();
  // 5. peeling, level by level (Algorithm 2, level-synchronous)
  int32_t* alist[2] = {S.colA, S.colA + A.max_m};
  int32_t* fq[2] = {S.eidA, S.eidA + A.max_m};
  int acnt = m, acur = 0, csr_live = m;
  bool first = true;
  int k = 1, r = 0, levels = 0, subrounds = 0;
  __syncthreads();
  for (;;) {
    // live list of the level, its minimum support, and at once the live edges
    // with sup <= k-1: the frontier F_0 of level k+1 (stamped r+1).  If none
    // is taken, the minimum is at least k and the next level is min + 2.
    __syncthreads();  // every thread has read the previous level's counters
    if (tid == 0) {
      L.cnt = 0;
      L.minv = kIntMax;
      L.qn = 0;
    }
    __syncthreads();
    const int kt = k + 1, st = r + 1;
    int mins = kIntMax;
    for (int t0 = 0; t0 < acnt; t0 += kSweepNI * T) {
      int e[kSweepNI], sv[kSweepNI], sk[kSweepNI];
      bool live[kSweepNI], take[kSweepNI];
#pragma unroll
      for (int q = 0; q < kSweepNI; ++q) {
        const int t = t0 + q * T + tid;
        e[q] = 0;
        live[q] = t < acnt;
        if (live[q]) e[q] = first ? t : ldw(&alist[acur][t]);
      }
#pragma unroll
      for (int q = 0; q < kSweepNI; ++q) {
        sk[q] = live[q] ? ldw(&S.stamp[e[q]]) : 1;
        sv[q] = live[q] ? ldw(&S.sup[e[q]]) : kIntMax;
      }
#pragma unroll
      for (int q = 0; q < kSweepNI; ++q) {
        live[q] = live[q] && sk[q] == 0;
        take[q] = live[q] && sv[q] <= kt - 2;
        if (live[q]) mins = sv[q] < mins ? sv[q] : mins;
        if (take[q]) {
          S.stamp[e[q]] = st;
          out[e[q]] = kt;
        }
      }
#pragma unroll
      for (int q = 0; q < kSweepNI; ++q) {
        const int pos = lds_append(&L.cnt, live[q]);
        if (live[q]) alist[acur ^ 1][pos] = e[q];
        const int qpos = lds_append(&L.qn, take[q]);
        if (take[q]) fq[st & 1][qpos] = e[q];
      }
    }
    mins = wave_min(mins);
    if (lane == 0 && mins != kIntMax) atomicMin(&L.minv, mins);
    __syncthreads();
    acnt = L.cnt;
    acur ^= 1;
    first = false;
    if (acnt == 0) break;
    ++levels;
    ++r;
    if (L.qn > 0) {
      k = kt;
    } else {
      // frontier F_0 of level min + 2: live edges with sup <= k-2 get truss number k
      k = L.minv + 2;
      __syncthreads();
      for (int t0 = 0; t0 < acnt; t0 += T) {
        const int t = t0 + tid;
        bool take = false;
        int e = 0;
        if (t < acnt) {
          e = ldw(&alist[acur][t]);
          take = ldw(&S.sup[e]) <= k - 2;
          if (take) {
            S.stamp[e] = r;
            out[e] = k;
          }
        }
        const int pos = lds_append(&L.qn, take);
        if (take) fq[r & 1][pos] = e;
      }
      __syncthreads();
    }
    const int l = k - 2;
    int qn = L.qn;
    int removed = qn;
    while (qn > 0) {
      ++subrounds;
      __syncthreads();
      if (tid == 0) L.qn = 0;
      __syncthreads();
      const int32_t* Q = fq[r & 1];
      int32_t* NQ = fq[(r + 1) & 1];
      // frontier edges in chunks of T; the chunk's walks (shorter live row of
      // each edge) are laid end to end and every thread takes NI entries of
      // the flattened range at a time, so long and short walks share the lanes
      for (int c0 = 0; c0 < qn; c0 += T) {
        const int i = c0 + tid;
        int e = 0, b = 0, ra = 0, la = 0, rb = 0, lb = 0;
        if (i < qn) {
          e = ldw(&Q[i]);
          const int u = ldw(&S.eu[e]), v = ldw(&S.ev[e]);
          const int ru = ldw(&S.rp[u]), du = ldw(&S.cur[u]);
          const int rv = ldw(&S.rp[v]), dv = ldw(&S.cur[v]);
          const bool ua = du < dv || (du == dv && u < v);
          b = ua ? v : u;
          ra = ua ? ru : rv;
          la = ua ? du : dv;
          rb = ua ? rv : ru;
          lb = ua ? dv : du;
          wpeel += (unsigned long long)la;
        }
        const long long Wc = block_scan64<T>((long long)la, L);
        L.wpre[tid + 1] = Wc;
        if (tid == 0) L.wpre[0] = 0;
        L.we[tid] = e;
        L.wb[tid] = b;
        L.wra[tid] = ra;
        L.wrb[tid] = rb;
        L.wlb[tid] = lb;
        __syncthreads();
        const long long W = L.wpre[T];
        for (long long t0 = 0; t0 < W; t0 += (long long)NI * T) {
          int ee[NI], bb[NI], jj[NI], rbb[NI], lbb[NI], w[NI], e1[NI], s1[NI], e2[NI], s2[NI];
          bool ok[NI];
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            const long long t = t0 + (long long)q * T + tid;
            ok[q] = t < W;
            ee[q] = bb[q] = jj[q] = rbb[q] = lbb[q] = 0;
            if (ok[q]) {
              int x = 0, y = T - 1;  // last edge whose range starts at or before t
              while (x < y) {
                const int mid = (x + y + 1) >> 1;
                if (L.wpre[mid] <= t) x = mid; else y = mid - 1;
              }
              ee[q] = L.we[x];
              bb[q] = L.wb[x];
              jj[q] = L.wra[x] + (int)(t - L.wpre[x]);
              rbb[q] = L.wrb[x];
              lbb[q] = L.wlb[x];
            }
          }
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            w[q] = ok[q] ? ldw(&S.col[jj[q]]) : -1;
            e1[q] = ok[q] ? ldw(&S.eid[jj[q]]) : 0;
          }
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            ok[q] = ok[q] && w[q] != bb[q];
            s1[q] = ok[q] ? ldw(&S.stamp[e1[q]]) : 0;
          }
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            ok[q] = ok[q] && !removed_at(s1[q], r);
            e2[q] = 0;
            if (ok[q]) {
              const int p = row_find(S.col, rbb[q], rbb[q] + lbb[q], w[q]);
              if (p < rbb[q] + lbb[q] && ldw(&S.col[p]) == w[q]) e2[q] = ldw(&S.eid[p]);
              else ok[q] = false;
            }
          }
#pragma unroll
          for (int q = 0; q < NI; ++q) s2[q] = ok[q] ? ldw(&S.stamp[e2[q]]) : 0;
#pragma unroll
          for (int q = 0; q < NI; ++q) {
            int f1 = -1, f2 = -1;
            const bool live = ok[q] && !removed_at(s2[q], r) && !(s1[q] == r && e1[q] < ee[q]) &&
                              !(s2[q] == r && e2[q] < ee[q]);
            if (live && s1[q] != r) {
              const int old = atomicSub(&S.sup[e1[q]], 1);
              if (old == l + 1) {
                S.stamp[e1[q]] = r + 1;
                out[e1[q]] = k;
                f1 = e1[q];
              }
            }
            if (live && s2[q] != r) {
              const int old = atomicSub(&S.sup[e2[q]], 1);
              if (old == l + 1) {
                S.stamp[e2[q]] = r + 1;
                out[e2[q]] = k;
                f2 = e2[q];
              }
            }
            const int p1 = lds_append(&L.qn, f1 >= 0);
            if (f1 >= 0) NQ[p1] = f1;
            const int p2 = lds_append(&L.qn, f2 >= 0);
            if (f2 >= 0) NQ[p2] = f2;
          }
        }
        __syncthreads();  // the chunk tables are reused by the next chunk
      }
      __syncthreads();
      qn = L.qn;
      removed += qn;
      ++r;
    }
    if (2 * (acnt - removed) < csr_live) {
      // drop removed entries from the rows once the live edge count has halved
      // (stable, so rows stay sorted; a wavefront per row)
      csr_live = acnt - removed;
      for (int x = wv; x < n; x += kWavesT) {
        const int base = ldw(&S.rp[x]);
        const int len = ldw(&S.cur[x]);
        int wpos = 0;
        for (int c0 = 0; c0 < len; c0 += kWave) {
          const int j = c0 + lane;
          int c = 0, ed = 0;
          bool keep = false;
          if (j < len) {
            c = ldw(&S.col[base + j]);
            ed = ldw(&S.eid[base + j]);
            keep = ldw(&S.stamp[ed]) == 0;
          }
          const uint64_t km = ballot(keep);
          wave_sync();
          if (keep) {
            S.col[base + wpos + rank_below(km)] = c;
            S.eid[base + wpos + rank_below(km)] = ed;
          }
          wpos += __popcll(km);
          wave_sync();
        }
        if (lane == 0) S.cur[x] = wpos;
      }
      __syncthreads();
    }
  }
  // per-graph totals
  tri3 = wave_sum(tri3);
  wsup = wave_sum(wsup);
  wpeel = wave_sum(wpeel);
  if (lane == 0) {
    if (tri3) atomicAdd(&A.ctl->triangles3, tri3);
    if (wsup) atomicAdd(&A.ctl->sup_work, wsup);
    if (wpeel) atomicAdd(&A.ctl->peel_work, wpeel);
  }
  if (tid == 0) {
    const unsigned long long t3 = wall_clock64();
    atomicAdd(&A.ctl->t_phase[0], t1 - t0);
    atomicAdd(&A.ctl->t_phase[1], t2 - t1);
    atomicAdd(&A.ctl->t_phase[2], t3 - t2);
    A.gerr[g] = 0;
    atomicMax(&A.ctl->kmax, k);
    atomicAdd(&A.ctl->levels, (unsigned long long)levels);
    atomicAdd(&A.ctl->subrounds, (unsigned long long)subrounds);
  }
}

template <int T, int NI>
__global__ void __launch_bounds__(T) k_batch(BatchArgs A) {
  __shared__ Lds<T> L;
  const Slot S = slot_at(A, blockIdx.x);
  for (;;) {
    if (threadIdx.x == 0) L.g = atomicAdd(&A.ctl->next, 1);
    __syncthreads();
    const int gi = L.g;
    if (gi >= A.G) break;
    process_graph<T, NI>(A, S, A.order[gi], L);
    __syncthreads();
  }
}

// gerr = 1 (not run) for every graph; counters cleared.  A fill kernel rather
// than a memset, so that the plan's graph holds kernels only.
__global__ void k_batch_init(BatchCtl* c, int32_t* gerr, int G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < G) gerr[i] = 1;
  if (i == 0) {
    c->next = 0;
    c->err_g = kIntMax;
    c->kmax = 0;
    c->levels = 0;
    c->subrounds = 0;
    c->triangles3 = 0;
    c->sup_work = 0;
    c->peel_work = 0;
    for (int q = 0; q < 3; ++q) c->t_phase[q] = 0;
  }
}

using BatchKernel = void (*)(BatchArgs);

BatchKernel batch_kernel(int T, int NI) {
#define TRUSS_BK(t, g) \
  if (T == t && NI == g) return &k_batch<t, g>;
  TRUSS_BK(256, 1) TRUSS_BK(256, 2) TRUSS_BK(256, 4)
  TRUSS_BK(512, 1) TRUSS_BK(512, 2) TRUSS_BK(512, 4)
  TRUSS_BK(1024, 1) TRUSS_BK(1024, 2) TRUSS_BK(1024, 4)
#undef TRUSS_BK
  return nullptr;
}

constexpr int kDefaultT = 1024, kDefaultG = 2;

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 256;
  return cus;
}

// The batch split: graphs for the persistent kernel (largest first) and graphs
// for the device-wide path; scratch shapes.
struct BatchSplit {
  std::vector<int32_t> order, big;
  int64_t max_n = 0, max_m = 0;
  int slots = 0;
  size_t slot_bytes = 0, big_ws = 0;
};

int split_batch(int32_t G, const int64_t* vo, const int64_t* eo, const truss_options* opts, BatchSplit& B) {
  if (G < 0 || (G > 0 && (!vo || !eo))) {
    set_last_error("bad batch arguments");
    return TRUSS_E_INVAL;
  }
  const int orc = validate_options(opts);
  if (orc) return orc;
  for (int32_t i = 0; i < G; ++i) {
    const int64_t n = vo[i + 1] - vo[i], m = eo[i + 1] - eo[i];
    if (n < 0 || m < 0 || n > 0x7fffffffLL) {
      set_last_error("batch offsets of graph %d are not monotone", i);
      return TRUSS_E_INVAL;
    }
    if (m > 0x7fffffffLL) {
      set_last_error("graph %d has more than INT32_MAX edges", i);
      return TRUSS_E_TOOBIG;
    }
    if (m <= kBatchMaxM && n <= kBatchMaxN) {
      B.order.push_back(i);
      B.max_n = std::max(B.max_n, n);
      B.max_m = std::max(B.max_m, m);
    } else {
      B.big.push_back(i);
      truss_graph g;
      memset(&g, 0, sizeof(g));
      g.fmt = TRUSS_FMT_EDGES;
      g.n = (int32_t)n;
      g.m = m;
      g.src = g.dst = reinterpret_cast<const int32_t*>(1);
      size_t b = 0;
      const int rc = truss_workspace_size(&g, opts, &b);
      if (rc) return rc;
      B.big_ws = std::max(B.big_ws, b);
    }
  }
  std::stable_sort(B.order.begin(), B.order.end(),
                   [&](int32_t a, int32_t b) { return eo[a + 1] - eo[a] > eo[b + 1] - eo[b]; });
  const int maxslots = 4 * device_cus();
  B.slots = (int)std::min<int64_t>((int64_t)B.order.size(), maxslots);
  B.slot_bytes = slot_bytes_for(B.max_n, B.max_m);
  return TRUSS_OK;
}

struct BatchLayout {
  BatchCtl* ctl;
  int64_t *vo, *eo;
  int32_t *order, *gerr;
  char* scratch;
  char* big_ws;
};

size_t batch_layout(int32_t G, const BatchSplit& B, char* base, BatchLayout* L) {
  Arena a;
  a.base = base;
  a.counting = base == nullptr;
  a.cap = ~size_t(0);
  BatchLayout l;
  l.ctl = a.take<BatchCtl>(1);
  l.vo = a.take<int64_t>((size_t)G + 1);
  l.eo = a.take<int64_t>((size_t)G + 1);
  l.order = a.take<int32_t>((size_t)G + 1);
  l.gerr = a.take<int32_t>((size_t)G + 1);
  l.scratch = a.take<char>((size_t)B.slots * B.slot_bytes + 256);
  l.big_ws = a.take<char>(B.big_ws + 256);
  if (L) *L = l;
  return a.used;
}

int check_cfg(int T, int G) {
  if (!batch_kernel(T, G)) {
    set_last_error("batch shape %d threads x %d walk entries per thread is not built", T, G);
    return TRUSS_E_INVAL;
  }
  return TRUSS_OK;
}

int launch_batch(const BatchArgs& A, int T, int G, int slots, hipStream_t s) {
  BatchKernel k = batch_kernel(T, G);
  int occ = 0;
  TRUSS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k, T, 0));
  if (occ < 1) {
    set_last_error("batch kernel does not fit on a compute unit");
    return TRUSS_E_DEVICE;
  }
  const int grid = std::max(1, std::min(slots, occ * device_cus()));
  BatchArgs a = A;
  void* args[] = {&a};
  TRUSS_HIP(hipLaunchKernel((const void*)k, dim3(grid), dim3(T), args, 0, s));
  return TRUSS_OK;
}

}  // namespace
}  // namespace truss

using namespace truss;

struct truss_batch_plan {
  int32_t G = 0;
  int T = kDefaultT, Gl = kDefaultG;
  std::vector<int64_t> vo, eo;
  BatchSplit split;
  BatchLayout lay;
  const int32_t *src = nullptr, *dst = nullptr;
  int32_t* out = nullptr;
  truss_options opts;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchArgs args;
};

namespace truss {
namespace {

void plan_free(truss_batch_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  delete p;
}

// Reads the kernel's status and runs the device-wide path on the big graphs.
int plan_finish(truss_batch_plan* p, truss_stats* stats, hipStream_t s, hipEvent_t done) {
  if (stats) memset(stats, 0, sizeof(*stats));
  int first_bad = kIntMax, bad_code = 0;
  truss_stats acc;
  memset(&acc, 0, sizeof(acc));
  for (int32_t gi : p->split.big) {
    truss_graph g;
    memset(&g, 0, sizeof(g));
    g.fmt = TRUSS_FMT_EDGES;
    g.n = (int32_t)(p->vo[gi + 1] - p->vo[gi]);
    g.m = p->eo[gi + 1] - p->eo[gi];
    g.src = p->src + p->eo[gi];
    g.dst = p->dst + p->eo[gi];
    truss_stats st;
    const int rc = truss_decompose(&g, p->out + p->eo[gi], &p->opts, &st, p->lay.big_ws, p->split.big_ws + 256, s);
    if (rc) {
      if (gi < first_bad) {
        first_bad = gi;
        bad_code = rc;
      }
      break;
    }
    acc.triangles += st.triangles;
    acc.kmax = std::max(acc.kmax, st.kmax);
    acc.levels += st.levels;
    acc.subrounds += st.subrounds;
    acc.peel_work += st.peel_work;
  }
  if (done) (void)hipEventRecord(done, s);
  BatchCtl h;
  TRUSS_HIP(hipMemcpyAsync(&h, p->lay.ctl, sizeof(h), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  if (h.err_g != kIntMax && h.err_g < first_bad) {
    int code = 0;
    TRUSS_HIP(hipMemcpy(&code, p->lay.gerr + h.err_g, sizeof(int), hipMemcpyDeviceToHost));
    first_bad = h.err_g;
    bad_code = code;
    set_last_error("graph %d of the batch failed: %s", h.err_g, truss_strerror(code));
  }
  if (first_bad != kIntMax) return bad_code;
  if (stats) {
    stats->n = p->vo[p->G] - p->vo[0];
    stats->m = p->eo[p->G] - p->eo[0];
    stats->triangles = (int64_t)(h.triangles3 / 3) + acc.triangles;
    stats->kmax = std::max(h.kmax, acc.kmax);
    stats->levels = (int32_t)(h.levels + (unsigned long long)acc.levels);
    stats->subrounds = (int64_t)h.subrounds + acc.subrounds;
    stats->launches = 1 + (int32_t)p->split.big.size();
    stats->support_work = (int64_t)h.sup_work;
    // workgroup time per phase (CSR build, support, peeling), summed over graphs
    for (int q = 0; q < 3; ++q) stats->ms_phase[q] = (double)h.t_phase[q] * 1e-5;
    stats->peel_work = (int64_t)h.peel_work + acc.peel_work;
  }
  return TRUSS_OK;
}

int plan_build(int32_t G, const int64_t* vo, const int64_t* eo, const int32_t* src, const int32_t* dst,
               int32_t* out, const truss_options* opts, void* ws, size_t ws_bytes, hipStream_t s, bool capture,
               truss_batch_plan** planp) {
  *planp = nullptr;
  truss_batch_plan* p = new truss_batch_plan();
  truss_default_options(&p->opts);
  if (opts) p->opts = *opts;
  int rc = split_batch(G, vo, eo, opts, p->split);
  if (rc) { plan_free(p); return rc; }
  const int64_t M = G > 0 ? eo[G] - eo[0] : 0;
  if (M > 0 && (!src || !dst || !out)) {
    set_last_error("src, dst or truss_out is NULL");
    plan_free(p);
    return TRUSS_E_INVAL;
  }
  if (G > 0 && eo[0] != 0) {
    set_last_error("edge_off[0] must be 0");
    plan_free(p);
    return TRUSS_E_INVAL;
  }
  p->T = opts && opts->batch_block > 0 ? opts->batch_block : kDefaultT;
  p->Gl = opts && opts->batch_ilp > 0 ? opts->batch_ilp : kDefaultG;
  if ((rc = check_cfg(p->T, p->Gl))) { plan_free(p); return rc; }
  const size_t need = batch_layout(G, p->split, nullptr, nullptr);
  if (!ws || ws_bytes < need) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
    plan_free(p);
    return TRUSS_E_WORKSPACE;
  }
  batch_layout(G, p->split, static_cast<char*>(ws), &p->lay);
  p->G = G;
  p->vo.assign(vo, vo + G + 1);
  p->eo.assign(eo, eo + G + 1);
  p->src = src;
  p->dst = dst;
  p->out = out;
  const int Q = (int)p->split.order.size();
  if (G > 0) {
    if (hipMemcpyAsync(p->lay.vo, vo, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(p->lay.eo, eo, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        (Q > 0 && hipMemcpyAsync(p->lay.order, p->split.order.data(), sizeof(int32_t) * Q, hipMemcpyHostToDevice,
                                 s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_last_error("copying the batch offsets failed");
      plan_free(p);
      return TRUSS_E_DEVICE;
    }
  }
  BatchArgs& A = p->args;
  A.G = Q;
  A.order = p->lay.order;
  A.vo = p->lay.vo;
  A.eo = p->lay.eo;
  A.src = src;
  A.dst = dst;
  A.out = out;
  A.gerr = p->lay.gerr;
  A.scratch = p->lay.scratch;
  A.slot_bytes = p->split.slot_bytes;
  A.max_n = (int32_t)p->split.max_n;
  A.max_m = p->split.max_m;
  A.ctl = p->lay.ctl;
  if (capture) {
    // the plan's work on the device: init, then the persistent kernel, as one graph
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      set_last_error("stream creation failed");
      plan_free(p);
      return TRUSS_E_DEVICE;
    }
    rc = TRUSS_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = TRUSS_E_DEVICE;
    if (!rc) {
      hipLaunchKernelGGL(k_batch_init, dim3((unsigned)((G + 256) / 256)), dim3(256), 0, cs, p->lay.ctl, p->lay.gerr,
                         G);
      if (Q > 0) rc = launch_batch(A, p->T, p->Gl, p->split.slots, cs);
      hipGraph_t gr = nullptr;
      if (hipStreamEndCapture(cs, &gr) != hipSuccess || !gr) rc = rc ? rc : TRUSS_E_DEVICE;
      p->graph = gr;
      if (!rc && hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) rc = TRUSS_E_DEVICE;
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
      set_last_error("capturing the batch graph failed");
      plan_free(p);
      return rc;
    }
  }
  *planp = p;
  return TRUSS_OK;
}

}  // namespace
}  // namespace truss

extern "C" {

int truss_batch_workspace_size(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off,
                               const truss_options* opts, size_t* bytes) {
  if (!bytes) {
    set_last_error("bytes is NULL");
    return TRUSS_E_INVAL;
  }
  BatchSplit B;
  const int rc = split_batch(num_graphs, vtx_off, edge_off, opts, B);
  if (rc) return rc;
  *bytes = batch_layout(num_graphs, B, nullptr, nullptr);
  return TRUSS_OK;
}

int truss_batch_plan_create(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off, const int32_t* src,
                            const int32_t* dst, int32_t* truss_out, const truss_options* opts, void* ws,
                            size_t ws_bytes, void* stream, truss_batch_plan** plan) {
  if (!plan) {
    set_last_error("plan is NULL");
    return TRUSS_E_INVAL;
  }
  return plan_build(num_graphs, vtx_off, edge_off, src, dst, truss_out, opts, ws, ws_bytes, (hipStream_t)stream, true,
                    plan);
}

int truss_batch_plan_run(truss_batch_plan* plan, truss_stats* stats, void* stream) {
  if (!plan) {
    set_last_error("plan is NULL");
    return TRUSS_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e[3] = {nullptr, nullptr, nullptr};
  bool timed = stats != nullptr;
  for (auto& x : e)
    if (timed && hipEventCreate(&x) != hipSuccess) timed = false;
  if (timed) (void)hipEventRecord(e[0], s);
  if (plan->exec) TRUSS_HIP(hipGraphLaunch(plan->exec, s));
  if (timed) (void)hipEventRecord(e[1], s);
  int rc = plan_finish(plan, stats, s, timed ? e[2] : nullptr);
  if (!rc && timed) {
    float k = 0.f, t = 0.f;
    if (hipEventElapsedTime(&k, e[0], e[1]) == hipSuccess) stats->ms_peel_kernel = k;
    if (hipEventElapsedTime(&t, e[0], e[2]) == hipSuccess) stats->ms_total = t;
  }
  for (auto& x : e)
    if (x) (void)hipEventDestroy(x);
  return rc;
}

void truss_batch_plan_destroy(truss_batch_plan* plan) { plan_free(plan); }

int truss_batch(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off, const int32_t* src,
                const int32_t* dst, int32_t* truss_out, const truss_options* opts, truss_stats* stats, void* ws,
                size_t ws_bytes, void* stream) {
  truss_batch_plan* p = nullptr;
  int rc = truss_batch_plan_create(num_graphs, vtx_off, edge_off, src, dst, truss_out, opts, ws, ws_bytes, stream, &p);
  if (rc) return rc;
  rc = truss_batch_plan_run(p, stats, stream);
  truss_batch_plan_destroy(p);
  return rc;
}

int truss_batch_autotune(int32_t num_graphs, const int64_t* vtx_off, const int64_t* edge_off, const int32_t* src,
                         const int32_t* dst, int32_t* truss_out, const truss_options* opts, void* ws, size_t ws_bytes,
                         void* stream, int32_t* best_block, int32_t* best_ilp, float* best_ms) {
  if (!best_block || !best_ilp) {
    set_last_error("NULL output");
    return TRUSS_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  truss_batch_plan* p = nullptr;
  int rc = plan_build(num_graphs, vtx_off, edge_off, src, dst, truss_out, opts, ws, ws_bytes, s, false, &p);
  if (rc) return rc;
  // a stratified sample of the queue: every stride-th graph in size order
  const std::vector<int32_t>& q = p->split.order;
  const int want = 512;
  std::vector<int32_t> sample;
  const size_t stride = q.size() > (size_t)want ? q.size() / want : 1;
  for (size_t i = 0; i < q.size(); i += stride) sample.push_back(q[i]);
  *best_block = kDefaultT;
  *best_ilp = kDefaultG;
  if (best_ms) *best_ms = 0.f;
  if (sample.empty()) {
    plan_free(p);
    return TRUSS_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TRUSS_HIP(hipEventCreate(&e0));
  TRUSS_HIP(hipEventCreate(&e1));
  // time one shape on the first `count` queue entries (order already on the device)
  auto time_shape = [&](int T, int Gl, int count, int reps, float* ms) -> int {
    BatchArgs A = p->args;
    A.G = count;
    float t = 0.f;
    for (int rep = 0; rep < reps; ++rep) {
      hipLaunchKernelGGL(k_batch_init, dim3((unsigned)((num_graphs + 256) / 256)), dim3(256), 0, s, p->lay.ctl,
                         p->lay.gerr, num_graphs);
      (void)hipEventRecord(e0, s);
      int r = launch_batch(A, T, Gl, (int)std::min<size_t>((size_t)count, (size_t)p->split.slots), s);
      if (r) return r;
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        return TRUSS_E_DEVICE;
    }
    *ms = t;
    return TRUSS_OK;
  };
  // stage 1: every shape on the sample (the first run of each warms the caches)
  TRUSS_HIP(hipMemcpyAsync(p->lay.order, sample.data(), sizeof(int32_t) * sample.size(), hipMemcpyHostToDevice, s));
  const int Ts[3] = {256, 512, 1024}, Gs[3] = {1, 2, 4};
  struct Cand { float ms; int T, G; };
  std::vector<Cand> cands;
  for (int ti = 0; ti < 3 && !rc; ++ti)
    for (int gi = 0; gi < 3 && !rc; ++gi) {
      float t = 0.f;
      rc = time_shape(Ts[ti], Gs[gi], (int)sample.size(), 2, &t);
      if (!rc) cands.push_back({t, Ts[ti], Gs[gi]});
    }
  // stage 2: the three fastest on the whole queue, where the largest graphs
  // (which set the tail) count at their full weight
  float best = -1.f;
  if (!rc) {
    std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
    TRUSS_HIP(hipMemcpyAsync(p->lay.order, q.data(), sizeof(int32_t) * q.size(), hipMemcpyHostToDevice, s));
    for (size_t c = 0; c < cands.size() && c < 3 && !rc; ++c) {
      float t = 0.f;
      rc = time_shape(cands[c].T, cands[c].G, (int)q.size(), 1, &t);
      if (!rc && (best < 0.f || t < best)) {
        best = t;
        *best_block = cands[c].T;
        *best_ilp = cands[c].G;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!rc) {
    BatchCtl h;
    TRUSS_HIP(hipMemcpy(&h, p->lay.ctl, sizeof(h), hipMemcpyDeviceToHost));
    if (h.err_g != kIntMax) {
      int code = 0;
      TRUSS_HIP(hipMemcpy(&code, p->lay.gerr + h.err_g, sizeof(int), hipMemcpyDeviceToHost));
      set_last_error("graph %d of the batch failed: %s", h.err_g, truss_strerror(code));
      rc = code;
    }
  }
  if (best_ms) *best_ms = best;
  plan_free(p);
  return rc;
}

}  // extern "C"
