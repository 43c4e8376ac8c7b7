// Graph build: validation of the simple-graph contract (Section 2), canonical
// edge ids, the symmetric CSR with edge ids, and the (degree, id) orientation
// used for triangle listing (the in-memory triangle counting that Algorithm 2,
// starts from; the smaller-degree rule of its triangle walk and Theorem 1).
#include <utility>

#include "common.hpp"
#include "internal.hpp"

namespace truss {

namespace {

constexpr int kT = 256;

inline unsigned grid_for(int64_t n, int per_block = kT) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (1LL << 30)) b = 1LL << 30;
  return (unsigned)b;
}

inline int bits_for(int64_t n) {
  int b = 0;
  while (b < 62 && (1LL << b) < n) ++b;
  return b;
}

__device__ __forceinline__ void report(int* err, int code) { atomicMin(err, code); }

__global__ void k_init_err(int* err) { *err = kNoErr; }

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---- row hash tables (the membership test of Algorithm 2) -----------------------------------

// slots of v's table: the power of two >= 2 deg(v) (0 for an isolated vertex)
__global__ void k_rtab_sizes(const int64_t* __restrict__ row_ptr, int32_t n, int32_t* __restrict__ tsz) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t d = row_ptr[v + 1] - row_ptr[v];
  int64_t sz = 0;
  if (d > 0) {
    sz = 2;
    while (sz < 2 * d) sz <<= 1;
  }
  tsz[v] = (int32_t)sz;
}

__global__ void k_rtab_clear(int2* __restrict__ rtab, const int64_t* __restrict__ rtoff, int32_t n, int64_t cap) {
  const int64_t total = rtoff[n];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total && i < cap;
       i += (int64_t)gridDim.x * blockDim.x)
    rtab[i] = make_int2(-1, 0);
}

__device__ __forceinline__ void rtab_put(int2* __restrict__ rtab, const int64_t* __restrict__ rtoff, int32_t v,
                                         int32_t w, int32_t e) {
  const int64_t off = rtoff[v];
  const int lg = row_table_lg(rtoff[v + 1] - off);
  const uint32_t mask = (1u << lg) - 1u;
  uint32_t h = row_slot(w, lg);
  // neighbours are distinct and the table is at most half full: a free slot is found
  while (atomicCAS(&rtab[off + h].x, -1, w) != -1) h = (h + 1) & mask;
  rtab[off + h].y = e;
}

// a thread per edge (u, v) inserts v into u's table and u into v's table (CSR
// input used as it is; the sorted builds insert while placing the row entries)
__global__ void k_rtab_insert(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev, int64_t m,
                              const int64_t* __restrict__ rtoff, int2* __restrict__ rtab) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int32_t u = eu[e], v = ev[e];
  rtab_put(rtab, rtoff, u, v, (int32_t)e);
  rtab_put(rtab, rtoff, v, u, (int32_t)e);
}

// capacity bound: 2^ceil(log2(2d)) < 4d for d >= 1, so all tables fit in 8m slots
inline int64_t rtab_capacity(int64_t m) { return 8 * m + 2; }

// ---- edge-list input ----------------------------------------------------------------

__global__ void k_canon(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t m, int32_t n,
                        int vb, uint64_t* __restrict__ key, int32_t* __restrict__ val, int* err) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  int32_t u = src[i], v = dst[i];
  int code = 0;
  if (u < 0 || u >= n || v < 0 || v >= n) code = kErrRange;
  else if (u == v) code = kErrSelfloop;
  if (code) { report(err, code); u = 0; v = 0; }
  uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
  key[i] = (a << vb) | b;
  val[i] = (int32_t)i;
}

__device__ __forceinline__ int64_t deg_of(const int64_t* __restrict__ rp, int32_t v) { return rp[v + 1] - rp[v]; }

__global__ void k_edges_from_keys(const uint64_t* __restrict__ key, const int32_t* __restrict__ val, int64_t m,
                                  int vb, int32_t* __restrict__ eu, int32_t* __restrict__ ev,
                                  int32_t* __restrict__ perm, int* err) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  uint64_t k = key[e];
  if (e > 0 && key[e - 1] == k) report(err, kErrDup);
  eu[e] = (int32_t)(k >> vb);
  ev[e] = (int32_t)(k & ((1ULL << vb) - 1));
  perm[e] = val[e];
}

// Row offsets without counters: the canonical edges are sorted by their
// smaller endpoint (eu) and, in a second copy, by their larger one (lo_v), so
// uppre[x] / lowpre[x] = edges whose smaller / larger endpoint is below x
// are lower bounds in those arrays; row x of the symmetric CSR starts at
// uppre[x] + lowpre[x] and holds its lower neighbours, then its upper ones.
__global__ void k_row_bounds(const int32_t* __restrict__ eu, const int32_t* __restrict__ lo_v, int64_t m, int32_t n,
                             int64_t* __restrict__ uppre, int64_t* __restrict__ lowpre,
                             int64_t* __restrict__ row_ptr) {
  const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (x > n) return;
  const int64_t a = lower_bound_i32<int64_t>(eu, 0, m, (int)x);
  const int64_t b = lower_bound_i32<int64_t>(lo_v, 0, m, (int)x);
  uppre[x] = a;
  lowpre[x] = b;
  row_ptr[x] = a + b;
}

// upper entry of canonical edge e = (u, v): the tail of u's row, after its
// lower entries (row_ptr[u+1] = uppre[u+1] + lowpre[u+1]); and v into u's row table
// (the threads of a block share u, so their inserts land in one table)
__global__ void k_sym_upper(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev, int64_t m,
                            const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ lowpre,
                            int32_t* __restrict__ col, int32_t* __restrict__ seid, int32_t* __restrict__ kf,
                            const int64_t* __restrict__ rtoff, int2* __restrict__ rtab) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  int32_t u = eu[e], v = ev[e];
  int64_t pos = lowpre[u + 1] + e;
  col[pos] = v;
  seid[pos] = (int32_t)e;
  kf[pos] = vertex_before(deg_of(row_ptr, u), u, deg_of(row_ptr, v), v) ? 1 : 0;
  rtab_put(rtab, rtoff, u, v, (int32_t)e);
}

__global__ void k_copy_ev(const int32_t* __restrict__ ev, int64_t m, uint32_t* __restrict__ tkey,
                          int32_t* __restrict__ tval) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= m) return;
  tkey[e] = (uint32_t)ev[e];
  tval[e] = (int32_t)e;
}

// lower entry of edge tval[t] = (u, v) with v = tkey[t]: the head of v's row,
// in canonical order (row_ptr[v] = uppre[v] + lowpre[v]); and u into v's row
// table (threads sorted by v, so again one table per run of threads)
__global__ void k_sym_lower(const uint32_t* __restrict__ tkey, const int32_t* __restrict__ tval, int64_t m,
                            const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ uppre,
                            const int32_t* __restrict__ eu, int32_t* __restrict__ col,
                            int32_t* __restrict__ seid, int32_t* __restrict__ kf,
                            const int64_t* __restrict__ rtoff, int2* __restrict__ rtab) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m) return;
  int32_t e = tval[t];
  int32_t v = (int32_t)tkey[t];
  int32_t u = eu[e];
  int64_t pos = uppre[v] + t;
  col[pos] = u;
  seid[pos] = e;
  kf[pos] = vertex_before(deg_of(row_ptr, v), v, deg_of(row_ptr, u), u) ? 1 : 0;
  rtab_put(rtab, rtoff, v, u, e);
}

// ---- locality relabelling ------------------------------------------------------------
// Vertices are renumbered by (degree, id) ascending before the graph is built:
// the orientation order of triangle listing becomes the id order, and the edges
// among high-degree vertices -- the ones the late levels of peeling walk over
// and over -- get the highest canonical ids, so that their supports, stamps and
// rows share lines and stay in cache.  perm maps each relabelled edge back to
// the caller's edge (input pair, or canonical CSR position), so outputs keep
// the caller's order.

// edge-list input: range and self-loop checks, degrees over the valid pairs
__global__ void k_edge_degrees(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t m,
                               int32_t n, int32_t* __restrict__ deg, int* err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t u = src[i], v = dst[i];
  if (u < 0 || u >= n || v < 0 || v >= n) { report(err, kErrRange); return; }
  if (u == v) { report(err, kErrSelfloop); return; }
  atomicAdd(&deg[u], 1);
  atomicAdd(&deg[v], 1);
}

// sort keys (degree, id) of the vertices; degrees from the CSR offsets or from deg
__global__ void k_degree_keys(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ deg, int32_t n, int vb,
                              uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v >= n) return;
  int64_t d = row_ptr ? row_ptr[v + 1] - row_ptr[v] : deg[v];
  const int64_t dmax = (1LL << vb) - 1;  // a simple graph has d < n <= 2^vb; larger only on invalid input
  d = d < 0 ? 0 : d > dmax ? dmax : d;
  key[v] = ((uint64_t)d << vb) | (uint64_t)v;
  val[v] = (int32_t)v;
}

__global__ void k_ranks(const int32_t* __restrict__ order, int32_t n, int32_t* __restrict__ rank) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rank[order[i]] = (int32_t)i;
}

// canonical keys of the relabelled edges (ids already checked)
__global__ void k_canon_relabel(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t m, int vb,
                                const int32_t* __restrict__ rank, uint64_t* __restrict__ key,
                                int32_t* __restrict__ val) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t u = rank[src[i]], v = rank[dst[i]];
  const uint64_t a = (uint64_t)(u < v ? u : v), b = (uint64_t)(u < v ? v : u);
  key[i] = (a << vb) | b;
  val[i] = (int32_t)i;
}

// ---- CSR input -------------------------------------------------------------------------

__global__ void k_rowptr_check(const int64_t* __restrict__ row_ptr, int32_t n, int64_t m2, int* err) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v > n) return;
  int64_t r = row_ptr[v];
  if (v == 0 && r != 0) report(err, kErrRowptr);
  if (v == n && r != m2) report(err, kErrRowptr);
  if (v < n && row_ptr[v + 1] < r) report(err, kErrRowptr);
  if (r < 0 || r > m2) report(err, kErrRowptr);
}

// one wavefront per row writes the row id of each entry
__global__ void k_rowid(const int64_t* __restrict__ row_ptr, int32_t n, int32_t* __restrict__ rowid) {
  const int lane = lane_id();
  const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t v = wid; v < n; v += nw) {
    const int64_t b = row_ptr[v], e = row_ptr[v + 1];
    for (int64_t j = b + lane; j < e; j += kWave) rowid[j] = (int32_t)v;
  }
}

__global__ void k_csr_check(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int32_t n,
                            int64_t m2, const int32_t* __restrict__ rowid, int32_t* __restrict__ uf, int* err) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m2) return;
  const int32_t v = rowid[j], w = col[j];
  int code = 0;
  if (w < 0 || w >= n) code = kErrRange;
  else if (w == v) code = kErrSelfloop;
  else if (j + 1 < row_ptr[v + 1]) {
    const int32_t x = col[j + 1];
    if (x == w) code = kErrDup;
    else if (x < w && x >= 0) code = kErrUnsorted;
  }
  if (code) report(err, code);
  uf[j] = (w > v && w < n) ? 1 : 0;
}

__global__ void k_csr_upper(const int32_t* __restrict__ col, const int32_t* __restrict__ rowid,
                            const int64_t* __restrict__ upos, int64_t m2, int32_t* __restrict__ colcopy,
                            int32_t* __restrict__ seid, int32_t* __restrict__ eu, int32_t* __restrict__ ev) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m2) return;
  const int32_t v = rowid[j], w = col[j];
  if (colcopy) {
    colcopy[j] = w;
    if (w > v) seid[j] = (int32_t)upos[j];
  }
  if (w > v) {
    const int64_t e = upos[j];
    eu[e] = v;
    ev[e] = w;
  }
}

__global__ void k_csr_lower(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ rowid, const int64_t* __restrict__ upos, int64_t m2,
                            int32_t* __restrict__ seid, int32_t* __restrict__ kf, int* err) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m2) return;
  const int32_t v = rowid[j], w = col[j];
  if (w < v) {
    const int64_t lo = row_ptr[w], hi = row_ptr[w + 1];
    const int64_t p = lower_bound_i32<int64_t>(col, lo, hi, v);
    if (p >= hi || col[p] != v) report(err, kErrAsym);
    else seid[j] = (int32_t)upos[p];
  }
  kf[j] = vertex_before(deg_of(row_ptr, v), v, deg_of(row_ptr, w), w) ? 1 : 0;
}

// Symmetry of a CSR input built through the relabelled path: the graph was
// built from the upper entries alone (m of them, no repeats), so the input is
// symmetric iff every lower entry (v, w), w < v, is an edge of that graph --
// looked up in the row table of v's new id.
__global__ void k_csr_sym_check(const int32_t* __restrict__ col_in, const int32_t* __restrict__ rowid, int64_t m2,
                                const int32_t* __restrict__ rank, const int2* __restrict__ rtab,
                                const int64_t* __restrict__ rtoff, int* err) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m2) return;
  const int32_t v = rowid[j], w = col_in[j];
  if (w >= v) return;
  const int32_t x = rank[v];
  const int64_t off = rtoff[x], slots = rtoff[x + 1] - off;
  if (slots == 0 || row_lookup(rtab, off, row_table_lg(slots), rank[w]) < 0) report(err, kErrAsym);
}

__global__ void k_check_total(const int64_t* __restrict__ upos, int64_t m2, int64_t m, int* err) {
  if (upos[m2] != m) report(err, kErrAsym);
}

// ---- orientation ------------------------------------------------------------------------

__global__ void k_orow(const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ opos, int32_t n,
                       int64_t* __restrict__ orow) {
  int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (v <= n) orow[v] = opos[row_ptr[v]];
}

__global__ void k_ocsr(const int32_t* __restrict__ col, const int32_t* __restrict__ seid,
                       const int32_t* __restrict__ kf, const int64_t* __restrict__ opos, int64_t m2,
                       int32_t* __restrict__ ocol, int32_t* __restrict__ oeid) {
  int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= m2) return;
  if (kf[j]) {
    const int64_t p = opos[j];
    ocol[p] = col[j];
    oeid[p] = seid[j];
  }
}

int read_err(const int* d_err, hipStream_t s) {
  int h = kNoErr;
  TRUSS_HIP(hipMemcpyAsync(&h, d_err, sizeof(int), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  if (h == kNoErr) return TRUSS_OK;
  switch (h) {
    case kErrRowptr: set_last_error("CSR row_ptr is not a valid offset array for 2m entries"); break;
    case kErrRange: set_last_error("vertex id outside [0, n)"); break;
    case kErrSelfloop: set_last_error("self-loop in input (simple graphs only)"); break;
    case kErrUnsorted: set_last_error("CSR row not strictly ascending"); break;
    case kErrDup: set_last_error("edge listed more than once"); break;
    case kErrAsym: set_last_error("CSR is not symmetric"); break;
    default: set_last_error("validation failed (%d)", h); break;
  }
  return -h;
}

// buffers of the build, laid out identically for the size query and the run
struct Layout {
  // resident
  int32_t *col, *seid, *eu, *ev, *perm, *ocol, *oeid;
  int64_t *row_ptr, *orow;
  // temporaries
  uint64_t *key, *key_alt;
  int32_t *val, *val_alt;
  int64_t *uppre, *lowpre;
  int32_t *rowid, *kf;
  int64_t *opos;
  int32_t *rtmp;
  int64_t *stmp;
  int2* rtab;
  int64_t* rtoff;
  int32_t* tsz;
  // relabelling: vertex sort keys and values (ping-pong), their radix scratch, ranks, degrees
  uint64_t *vkey, *vkey_alt;
  int32_t *vval, *vval_alt, *vtmp, *rank, *vdeg;
};

void carve(const truss_graph* g, bool relabel, Arena& a, Layout& L) {
  const int64_t n = g->n, m = g->m, m2 = 2 * m;
  // the edge-list build runs for edge-list input and, after validation, for
  // relabelled CSR input
  const bool edges = g->fmt == TRUSS_FMT_EDGES || relabel;
  L.col = a.take<int32_t>(m2 + 1);
  L.seid = a.take<int32_t>(m2 + 1);
  L.eu = a.take<int32_t>(m + 1);
  L.ev = a.take<int32_t>(m + 1);
  L.ocol = a.take<int32_t>(m + 1);
  L.oeid = a.take<int32_t>(m + 1);
  L.orow = a.take<int64_t>(n + 1);
  L.perm = edges ? a.take<int32_t>(m + 1) : nullptr;
  L.rtab = a.take<int2>((size_t)rtab_capacity(m));
  L.rtoff = a.take<int64_t>(n + 1);
  L.tsz = a.take<int32_t>(n + 1);
  L.row_ptr = edges ? a.take<int64_t>(n + 1) : nullptr;
  // temporaries (could alias peeling state; kept separate for clarity)
  L.kf = a.take<int32_t>(m2 + 1);
  L.opos = a.take<int64_t>(m2 + 1);
  L.stmp = a.take<int64_t>(scan_tmp_elems(m2 + 1) + scan_tmp_elems(n + 1));
  if (edges) {
    L.key = a.take<uint64_t>(m + 1);
    L.key_alt = a.take<uint64_t>(m + 1);
    L.val = a.take<int32_t>(m + 1);
    L.val_alt = a.take<int32_t>(m + 1);
    L.uppre = a.take<int64_t>(n + 1);
    L.lowpre = a.take<int64_t>(n + 1);
    L.rtmp = a.take<int32_t>(radix_tmp_elems(m + 1));
    L.rowid = g->fmt == TRUSS_FMT_CSR ? a.take<int32_t>(m2 + 1) : nullptr;
  } else {
    L.rowid = a.take<int32_t>(m2 + 1);
    L.key = L.key_alt = nullptr;
    L.val = L.val_alt = nullptr;
    L.uppre = L.lowpre = nullptr;
    L.rtmp = nullptr;
  }
  if (relabel) {
    L.vkey = a.take<uint64_t>(n + 1);
    L.vkey_alt = a.take<uint64_t>(n + 1);
    L.vval = a.take<int32_t>(n + 1);
    L.vval_alt = a.take<int32_t>(n + 1);
    L.vtmp = a.take<int32_t>(radix_tmp_elems(n + 1));
    L.rank = a.take<int32_t>(n + 1);
    L.vdeg = a.take<int32_t>(n + 1);
  } else {
    L.vkey = L.vkey_alt = nullptr;
    L.vval = L.vval_alt = L.vtmp = L.rank = L.vdeg = nullptr;
  }
}

// ranks of the vertices in (degree, id) order; degrees from row_ptr, else from deg
void degree_ranks(const int64_t* row_ptr, const int32_t* deg, int32_t n, int vb, Layout& L, hipStream_t s) {
  hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(n > 0 ? n : 1)), dim3(kT), 0, s, row_ptr, deg, n, vb, L.vkey,
                     L.vval);
  const bool alt = radix_sort_u64(L.vkey, L.vval, L.vkey_alt, L.vval_alt, n, 2 * vb, L.vtmp, s);
  hipLaunchKernelGGL(k_ranks, dim3(grid_for(n > 0 ? n : 1)), dim3(kT), 0, s, alt ? L.vval_alt : L.vval, n, L.rank);
}

// sizes, offsets and cleared slots of the row tables for the rows at row_ptr
void table_layout(const int64_t* row_ptr, int32_t n, int64_t m, Layout& L, hipStream_t s) {
  hipLaunchKernelGGL(k_rtab_sizes, dim3(grid_for(n > 0 ? n : 1)), dim3(kT), 0, s, row_ptr, n, L.tsz);
  scan_exclusive_i32_to_i64(L.tsz, L.rtoff, n, L.stmp, s);
  const int64_t cap = rtab_capacity(m);
  hipLaunchKernelGGL(k_rtab_clear, dim3(grid_for(cap) < 65536 ? grid_for(cap) : 65536), dim3(kT), 0, s, L.rtab,
                     L.rtoff, n, cap);
}

// symmetric CSR, canonical edges, perm and the row tables from the unsorted
// canonical keys in L.key / L.val (val: the caller's index of each edge)
int rows_from_keys(int32_t n, int64_t m, int vb, Layout& L, int* d_err, hipStream_t s) {
  if (radix_sort_u64(L.key, L.val, L.key_alt, L.val_alt, m, 2 * vb, L.rtmp, s)) {
    std::swap(L.key, L.key_alt);
    std::swap(L.val, L.val_alt);
  }
  hipLaunchKernelGGL(k_edges_from_keys, dim3(grid_for(m)), dim3(kT), 0, s, L.key, L.val, m, vb, L.eu, L.ev, L.perm,
                     d_err);
  const int rc = read_err(d_err, s);
  if (rc) return rc;
  // the canonical order, stably sorted by the larger endpoint (lower halves of the rows)
  uint32_t* tkey = reinterpret_cast<uint32_t*>(L.key);
  uint32_t* tkey_alt = reinterpret_cast<uint32_t*>(L.key_alt);
  hipLaunchKernelGGL(k_copy_ev, dim3(grid_for(m)), dim3(kT), 0, s, L.ev, m, tkey, L.val);
  if (radix_sort_u32(tkey, L.val, tkey_alt, L.val_alt, m, vb, L.rtmp, s)) {
    std::swap(tkey, tkey_alt);
    std::swap(L.val, L.val_alt);
  }
  hipLaunchKernelGGL(k_row_bounds, dim3(grid_for((int64_t)n + 1)), dim3(kT), 0, s, L.eu,
                     reinterpret_cast<const int32_t*>(tkey), m, n, L.uppre, L.lowpre, L.row_ptr);
  table_layout(L.row_ptr, n, m, L, s);
  hipLaunchKernelGGL(k_sym_upper, dim3(grid_for(m)), dim3(kT), 0, s, L.eu, L.ev, m, L.row_ptr, L.lowpre, L.col,
                     L.seid, L.kf, L.rtoff, L.rtab);
  hipLaunchKernelGGL(k_sym_lower, dim3(grid_for(m)), dim3(kT), 0, s, tkey, L.val, m, L.row_ptr, L.uppre, L.eu,
                     L.col, L.seid, L.kf, L.rtoff, L.rtab);
  return TRUSS_OK;
}

}  // namespace

size_t build_workspace(const truss_graph* g, Arena& a, bool relabel) {
  Layout L;
  carve(g, relabel, a, L);
  return a.used;
}

int build_graph(const truss_graph* g, Arena& a, DevGraph& dg, int* d_err, hipStream_t s, bool relabel) {
  Layout L;
  carve(g, relabel, a, L);
  if (a.overflow()) return TRUSS_E_WORKSPACE;
  const int32_t n = g->n;
  const int64_t m = g->m, m2 = 2 * m;
  const int vb = bits_for(n) > 0 ? bits_for(n) : 1;
  dg.n = n;
  dg.m = m;
  hipLaunchKernelGGL(k_init_err, dim3(1), dim3(1), 0, s, d_err);

  if (g->fmt == TRUSS_FMT_EDGES) {
    int rc;
    if (relabel) {
      hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n + 1)), dim3(kT), 0, s, L.vdeg, (int64_t)n + 1, 0);
      hipLaunchKernelGGL(k_edge_degrees, dim3(grid_for(m)), dim3(kT), 0, s, g->src, g->dst, m, n, L.vdeg, d_err);
      if ((rc = read_err(d_err, s))) return rc;
      degree_ranks(nullptr, L.vdeg, n, vb, L, s);
      hipLaunchKernelGGL(k_canon_relabel, dim3(grid_for(m)), dim3(kT), 0, s, g->src, g->dst, m, vb, L.rank, L.key,
                         L.val);
    } else {
      hipLaunchKernelGGL(k_canon, dim3(grid_for(m)), dim3(kT), 0, s, g->src, g->dst, m, n, vb, L.key, L.val, d_err);
      if ((rc = read_err(d_err, s))) return rc;
    }
    if ((rc = rows_from_keys(n, m, vb, L, d_err, s))) return rc;
    dg.row_ptr = L.row_ptr;
    dg.perm = L.perm;
  } else {
    hipLaunchKernelGGL(k_rowptr_check, dim3(grid_for((int64_t)n + 1)), dim3(kT), 0, s, g->row_ptr, n, m2, d_err);
    int rc = read_err(d_err, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_rowid, dim3(grid_for((int64_t)n * kWave > 0 ? (int64_t)n * kWave : 1)), dim3(kT), 0, s,
                       g->row_ptr, n, L.rowid);
    int32_t* uf = L.kf;  // upper flags, later reused for orientation flags
    hipLaunchKernelGGL(k_csr_check, dim3(grid_for(m2)), dim3(kT), 0, s, g->row_ptr, g->col, n, m2, L.rowid, uf,
                       d_err);
    rc = read_err(d_err, s);
    if (rc) return rc;
    int64_t* upos = L.opos;
    scan_exclusive_i32_to_i64(uf, upos, m2, L.stmp, s);
    hipLaunchKernelGGL(k_check_total, dim3(1), dim3(1), 0, s, upos, m2, m, d_err);
    rc = read_err(d_err, s);
    if (rc) return rc;
    // canonical edges; the entries themselves are kept only when the input rows are used as they are
    hipLaunchKernelGGL(k_csr_upper, dim3(grid_for(m2)), dim3(kT), 0, s, g->col, L.rowid, upos, m2,
                       relabel ? nullptr : L.col, L.seid, L.eu, L.ev);
    if (relabel) {
      // the canonical edges (the upper entries), renamed, go through the
      // edge-list build; perm then maps each edge to its canonical CSR
      // position.  Symmetry is checked on the row tables at the end.
      degree_ranks(g->row_ptr, nullptr, n, vb, L, s);
      hipLaunchKernelGGL(k_canon_relabel, dim3(grid_for(m)), dim3(kT), 0, s, L.eu, L.ev, m, vb, L.rank, L.key,
                         L.val);
      if ((rc = rows_from_keys(n, m, vb, L, d_err, s))) return rc;
      dg.row_ptr = L.row_ptr;
      dg.perm = L.perm;
    } else {
      hipLaunchKernelGGL(k_csr_lower, dim3(grid_for(m2)), dim3(kT), 0, s, g->row_ptr, g->col, L.rowid, upos, m2,
                         L.seid, L.kf, d_err);
      if ((rc = read_err(d_err, s))) return rc;
      dg.row_ptr = g->row_ptr;
      dg.perm = nullptr;
    }
  }
  // oriented CSR: stable compaction of the symmetric rows by the orientation flag
  scan_exclusive_i32_to_i64(L.kf, L.opos, m2, L.stmp, s);
  hipLaunchKernelGGL(k_orow, dim3(grid_for((int64_t)n + 1)), dim3(kT), 0, s, dg.row_ptr, L.opos, n, L.orow);
  hipLaunchKernelGGL(k_ocsr, dim3(grid_for(m2)), dim3(kT), 0, s, L.col, L.seid, L.kf, L.opos, m2, L.ocol, L.oeid);
  TRUSS_HIP(hipGetLastError());
  dg.col = L.col;
  dg.seid = L.seid;
  dg.eu = L.eu;
  dg.ev = L.ev;
  dg.orow = L.orow;
  dg.ocol = L.ocol;
  dg.oeid = L.oeid;
  // row hash tables for the membership tests of peeling (the sorted builds
  // filled them while placing the row entries)
  if (dg.perm == nullptr) {
    table_layout(dg.row_ptr, n, m, L, s);
    if (m > 0) hipLaunchKernelGGL(k_rtab_insert, dim3(grid_for(m)), dim3(kT), 0, s, L.eu, L.ev, m, L.rtoff, L.rtab);
  }
  TRUSS_HIP(hipGetLastError());
  dg.rtab = L.rtab;
  dg.rtoff = L.rtoff;
  if (relabel && g->fmt == TRUSS_FMT_CSR && m2 > 0) {
    hipLaunchKernelGGL(k_csr_sym_check, dim3(grid_for(m2)), dim3(kT), 0, s, g->col, L.rowid, m2, L.rank, L.rtab,
                       L.rtoff, d_err);
    return read_err(d_err, s);
  }
  return TRUSS_OK;
}

}  // namespace truss
