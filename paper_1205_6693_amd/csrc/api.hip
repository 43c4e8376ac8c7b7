// C ABI of libtruss.so (declarations and contracts in include/truss.h).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "mlp.hpp"

namespace truss {

namespace {
thread_local char g_last_error[512] = "";

constexpr int kT = 256;

__global__ void k_scatter_out(const int32_t* __restrict__ val, const int32_t* __restrict__ perm, int64_t m,
                              int32_t* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < m) out[perm ? perm[e] : e] = val[e];
}

__global__ void k_scatter_sup(const int2* __restrict__ sr, const int32_t* __restrict__ perm, int64_t m,
                              int32_t* __restrict__ out, unsigned long long* total) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long x = 0;
  if (e < m) {
    const int s = sr[e].x;
    out[perm ? perm[e] : e] = s;
    x = (unsigned long long)s;
  }
  x = wave_sum(x);
  if (lane_id() == 0 && x) atomicAdd(total, x);
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0; }

// supports out of reach of every level for edges that must not be peeled
constexpr int kFrozenSup = 1 << 29;
__global__ void k_freeze(int2* __restrict__ sr, const int32_t* __restrict__ perm, const uint8_t* __restrict__ frozen,
                         int64_t m) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < m && frozen[perm ? perm[e] : e]) sr[e].x = kFrozenSup;
}

__global__ void k_fill_i32(int32_t* __restrict__ x, int64_t m, int32_t v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < m) x[i] = v;
}

__global__ void k_sum_sup(const int2* __restrict__ sr, int64_t m, unsigned long long* total) {
  unsigned long long x = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
    x += (unsigned long long)sr[e].x;
  x = wave_sum(x);
  if (lane_id() == 0 && x) atomicAdd(total, x);
}

inline unsigned grid_for(int64_t n) {
  const int64_t b = (n + kT - 1) / kT;
  return (unsigned)(b < 1 ? 1 : b);
}

int check_graph(const truss_graph* g) {
  if (!g) { set_last_error("graph is NULL"); return TRUSS_E_INVAL; }
  if (g->n < 0 || g->m < 0) { set_last_error("negative n or m"); return TRUSS_E_INVAL; }
  if (g->m > 0x7fffffffLL) { set_last_error("m exceeds INT32_MAX"); return TRUSS_E_TOOBIG; }
  if (g->fmt == TRUSS_FMT_EDGES) {
    if (g->m > 0 && (!g->src || !g->dst)) { set_last_error("src/dst is NULL"); return TRUSS_E_INVAL; }
  } else if (g->fmt == TRUSS_FMT_CSR) {
    if (!g->row_ptr || (g->m > 0 && !g->col)) { set_last_error("row_ptr/col is NULL"); return TRUSS_E_INVAL; }
  } else {
    set_last_error("unknown graph format %d", g->fmt);
    return TRUSS_E_INVAL;
  }
  return TRUSS_OK;
}

}  // namespace

int validate_options(const truss_options* o) {
  if (!o) return TRUSS_OK;
  if (o->version != TRUSS_VERSION) { set_last_error("options version mismatch"); return TRUSS_E_INVAL; }
  if (o->support_strategy < TRUSS_SUP_AUTO || o->support_strategy > TRUSS_SUP_MERGE ||
      o->peel_mode < TRUSS_PEEL_AUTO || o->peel_mode > TRUSS_PEEL_DENSE ||
      o->scheduler < TRUSS_SCHED_PLAIN || o->scheduler > TRUSS_SCHED_LEARNED ||
      o->peel_probe < TRUSS_PROBE_AUTO || o->peel_probe > TRUSS_PROBE_BSEARCH ||
      o->peel_shape < TRUSS_SHAPE_AUTO || o->peel_shape > TRUSS_SHAPE_WIDE ||
      !(o->batch_block == 0 || o->batch_block == 256 || o->batch_block == 512 || o->batch_block == 1024) ||
      !(o->batch_ilp == 0 || o->batch_ilp == 1 || o->batch_ilp == 2 || o->batch_ilp == 4)) {
    set_last_error("option out of range");
    return TRUSS_E_INVAL;
  }
  return TRUSS_OK;
}

namespace {

// Checks a learned model's two part headers (device memory) against the
// network shapes the scheduler evaluates and, when the caller states how many
// floats the model holds (nfloats > 0), against that length: both headers
// must lie inside it and the two parts must fill it exactly.  Fills the part
// pointers.
bool model_parts(const float* model, int64_t nfloats, const float** peel_part, const float** sup_part,
                 hipStream_t s) {
  if (!model) return false;
  if (nfloats > 0 && nfloats < 4) return false;
  float h[4];
  if (hipMemcpyAsync(h, model, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  if (h[0] != kModelTag || h[1] != (float)kPeelF || h[3] != (float)kPeelA || !(h[2] >= 1.f) ||
      !(h[2] <= (float)kMlpMaxH) || h[2] != (float)(int)h[2])
    return false;
  const int off = model_part_floats(kPeelF, (int)h[2], kPeelA);
  if (nfloats > 0 && (int64_t)off + 4 > nfloats) return false;
  float g[4];
  if (hipMemcpyAsync(g, model + off, sizeof(g), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  if (g[0] != kModelTag || g[1] != (float)kSupF || g[3] != (float)kSupA || !(g[2] >= 1.f) ||
      !(g[2] <= (float)kMlpMaxH) || g[2] != (float)(int)g[2])
    return false;
  if (nfloats > 0 && (int64_t)off + model_part_floats(kSupF, (int)g[2], kSupA) != nfloats) return false;
  *peel_part = model;
  *sup_part = model + off;
  return true;
}

// Resolves the options into the support and peeling plans.  A learned
// scheduler without a well-formed model falls back to the heuristic.
void resolve(const truss_options* in, SupPlan* sp, PeelPlan* pp, int* fallback, hipStream_t s) {
  truss_options o;
  truss_default_options(&o);
  if (in) o = *in;
  *fallback = 0;
  int sched = o.scheduler;
  const float *peel_part = nullptr, *sup_part = nullptr;
  if (sched == TRUSS_SCHED_LEARNED && !model_parts(o.model, o.model_floats, &peel_part, &sup_part, s)) {
    *fallback = 1;
    sched = TRUSS_SCHED_HEURISTIC;
  }
  *sp = SupPlan();
  sp->sched = sched;
  sp->force = o.support_strategy == TRUSS_SUP_AUTO ? -1 : o.support_strategy - 1;
  sp->model = sup_part;
  *pp = PeelPlan();
  pp->sched = sched;
  pp->model = peel_part;
  if (o.peel_probe != TRUSS_PROBE_AUTO) {
    pp->fix_bits |= 1;
    pp->fix_vals |= o.peel_probe == TRUSS_PROBE_BSEARCH ? 1 : 0;
  }
  if (o.peel_mode != TRUSS_PEEL_AUTO) {
    pp->fix_bits |= 2;
    pp->fix_vals |= o.peel_mode == TRUSS_PEEL_DENSE ? 2 : 0;
  }
  pp->max_subrounds = o.max_subrounds;
  pp->grid_blocks = o.grid_blocks;
  pp->shape = o.peel_shape;
}

struct Plan {
  int* d_err = nullptr;
  unsigned long long* d_total = nullptr;
  int2* sr = nullptr;
  int32_t* truss_canon = nullptr;
  int32_t *h = nullptr, *ch = nullptr, *psi = nullptr;  // upper bound (Procedure 6)
};

// what run_single produces
enum Mode { kModeSupport, kModeDecompose, kModeBound };

void take_bound(const truss_graph* g, Arena& a, Plan& p) {
  p.h = a.take<int32_t>((size_t)g->n + 1);
  p.ch = a.take<int32_t>((size_t)g->n + 1);
  p.psi = a.take<int32_t>((size_t)g->m + 1);
}

// One layout for size queries and runs: header, build, per-edge state, support, peel.
void layout(const truss_graph* g, Arena& a, Plan& p, DevGraph* dg_for_sizes) {
  p.d_err = a.take<int>(64);
  p.d_total = a.take<unsigned long long>(8);
  build_workspace(g, a, true);
  p.sr = a.take<int2>((size_t)g->m + 1);
  p.truss_canon = a.take<int32_t>((size_t)g->m + 1);
  take_bound(g, a, p);
  DevGraph dg;
  dg.n = g->n;
  dg.m = g->m;
  if (dg_for_sizes) dg = *dg_for_sizes;
  support_workspace(dg, a);
  peel_workspace(dg, a);
}

struct Timer {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool on = false;
  hipStream_t s;
  explicit Timer(bool enable, hipStream_t st) : on(enable), s(st) {
    if (on)
      for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) on = false;
  }
  void mark(int i) {
    if (on) (void)hipEventRecord(ev[i], s);
  }
  double ms(int a, int b) {
    float t = 0.f;
    if (!on) return 0.0;
    if (hipEventSynchronize(ev[b]) != hipSuccess) return 0.0;
    if (hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0.0;
    return t;
  }
  ~Timer() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Runs build + support, then either scatters sup (want_truss false) or peels.
// sub (nullable): the neighbourhood-subgraph extras of run_subgraph (decompose mode)
int run_single(const truss_graph* g, Mode mode, int32_t* out, int64_t* triangles,
               const truss_options* opts_in, truss_stats* stats, void* ws, size_t ws_bytes, hipStream_t s,
               truss_trace* trace, const SubgraphRun* sub = nullptr, bool timed = true) {
  int rc = check_graph(g);
  if (rc) return rc;
  rc = validate_options(opts_in);
  if (rc) return rc;
  if (g->m > 0 && !out) { set_last_error("output is NULL"); return TRUSS_E_INVAL; }
  if (trace && trace->level_cap < 0) { set_last_error("negative trace capacity"); return TRUSS_E_INVAL; }
  if (trace) {
    trace->levels = 0;
    for (int b = 0; b < kSupBins; ++b) {
      trace->sup_action[b] = -1;
      trace->sup_ms[b] = 0.f;
      for (int i = 0; i < kSupF; ++i) trace->sup_feat[b][i] = 0.f;
    }
  }
  Arena need;
  need.counting = true;
  Plan dummy;
  layout(g, need, dummy, nullptr);
  if (!ws || ws_bytes < need.used) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, need.used);
    return TRUSS_E_WORKSPACE;
  }
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  Plan p;
  p.d_err = a.take<int>(64);
  p.d_total = a.take<unsigned long long>(8);
  SupPlan sp;
  PeelPlan pp;
  int fallback = 0;
  resolve(opts_in, &sp, &pp, &fallback, s);
  pp.timed = timed;
  Timer tm(stats != nullptr && timed, s);
  tm.mark(0);
  DevGraph dg;
  rc = build_graph(g, a, dg, p.d_err, s, true);
  if (rc) return rc;
  tm.mark(1);
  p.sr = a.take<int2>((size_t)g->m + 1);
  p.truss_canon = a.take<int32_t>((size_t)g->m + 1);
  take_bound(g, a, p);
  rc = compute_support(dg, sp, p.sr, a, s, trace);
  if (rc) return rc;
  tm.mark(2);
  PeelResult pr;
  unsigned long long tot = 0;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, p.d_total);
  if (mode == kModeBound) {
    // the counters of long rows live in the (unused) peeling region
    int32_t* hs = a.take<int32_t>((size_t)(2 * g->m + g->n + 1));
    if (a.overflow()) { set_last_error("workspace too small for the upper bound"); return TRUSS_E_WORKSPACE; }
    compute_upper_bound(dg, p.sr, p.h, p.ch, p.psi, hs, s);
    if (g->m > 0)
      hipLaunchKernelGGL(k_scatter_out, dim3(grid_for(g->m)), dim3(kT), 0, s, p.psi, dg.perm, g->m, out);
    TRUSS_HIP(hipGetLastError());
    TRUSS_HIP(hipStreamSynchronize(s));
    tm.mark(3);
  } else if (mode == kModeSupport) {
    if (g->m > 0)
      hipLaunchKernelGGL(k_scatter_sup, dim3(grid_for(g->m)), dim3(kT), 0, s, p.sr, dg.perm, g->m, out, p.d_total);
    TRUSS_HIP(hipMemcpyAsync(&tot, p.d_total, sizeof(tot), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    if (triangles) *triangles = (int64_t)(tot / 3);
    tm.mark(3);
  } else {
    if (stats && g->m > 0) hipLaunchKernelGGL(k_sum_sup, dim3(1024), dim3(kT), 0, s, p.sr, g->m, p.d_total);
    int32_t* tc = dg.perm ? p.truss_canon : out;
    if (sub && g->m > 0) {
      if (sub->sup_out)
        hipLaunchKernelGGL(k_scatter_sup, dim3(grid_for(g->m)), dim3(kT), 0, s, p.sr, dg.perm, g->m, sub->sup_out,
                           p.d_total);
      if (sub->frozen)
        hipLaunchKernelGGL(k_freeze, dim3(grid_for(g->m)), dim3(kT), 0, s, p.sr, dg.perm, sub->frozen, g->m);
      if (sub->stop_level > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(g->m)), dim3(kT), 0, s, tc, g->m, 0);
      pp.first_level = sub->first_level;
      pp.stop_level = sub->stop_level;
    }
    rc = peel(dg, pp, p.sr, tc, a, &pr, s, trace);
    if (rc) return rc;
    if (dg.perm && g->m > 0)
      hipLaunchKernelGGL(k_scatter_out, dim3(grid_for(g->m)), dim3(kT), 0, s, tc, dg.perm, g->m, out);
    tm.mark(3);
    TRUSS_HIP(hipGetLastError());
    if (stats) TRUSS_HIP(hipMemcpyAsync(&tot, p.d_total, sizeof(tot), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
  }
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n = g->n;
    stats->m = g->m;
    stats->kmax = pr.kmax;
    stats->levels = pr.levels;
    stats->subrounds = pr.subrounds;
    stats->peel_work = pr.work;
    stats->ms_build = tm.ms(0, 1);
    stats->ms_support = tm.ms(1, 2);
    stats->ms_peel = tm.ms(2, 3);
    stats->ms_total = tm.ms(0, 3);
    stats->sched_fallback = fallback;
    stats->triangles = (int64_t)(tot / 3);
    stats->launches = pr.launches;
    stats->heavy_rounds = pr.heavy_rounds;
    for (int b = 0; b < 6; ++b) stats->frontier_hist[b] = pr.hist[b];
    for (int b = 0; b < 6; ++b) stats->ms_phase[b] = pr.phase_ms[b];
    stats->ms_peel_kernel = pr.kernel_ms;
  }
  return TRUSS_OK;
}

// ---- top-down: the top-t k-classes (Algorithm 7) ----------------------------------------
// Every edge with phi(e) >= k has psi(e) >= k (Lemma 2), so the k-truss of G
// lies in E_k = {e : psi(e) >= k}; and the k-truss of E_k is a k-truss of G.
// Hence the truss numbers >= k of G and of the subgraph E_k agree, and the
// top-t classes come from decomposing E_k for any k <= k_max - t + 1.  k
// starts at max psi and moves down (by the exact amount once k_max is known,
// otherwise by doubling steps) until that holds.
__global__ void k_max_i32(const int32_t* __restrict__ x, int64_t m, int* __restrict__ out) {
  int v = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    v = x[i] > v ? x[i] : v;
  v = wave_max(v);
  if (lane_id() == 0 && v) atomicMax(out, v);
}

// edges with psi >= k, as an edge list over the same vertex ids
__global__ void k_select(const int32_t* __restrict__ psi, const int32_t* __restrict__ eu,
                         const int32_t* __restrict__ ev, int64_t m, int k, int32_t* __restrict__ ssrc,
                         int32_t* __restrict__ sdst, int32_t* __restrict__ sid, int* __restrict__ count) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool take = e < m && psi[e] >= k;
  const int pos = wave_append(count, take);
  if (take) {
    ssrc[pos] = eu[e];
    sdst[pos] = ev[e];
    sid[pos] = (int32_t)e;
  }
}

// truss numbers of the subgraph at or above kmin, written to the caller's indexing
__global__ void k_topdown_out(const int32_t* __restrict__ sub_out, const int32_t* __restrict__ sid, int64_t cnt,
                              int kmin, const int32_t* __restrict__ perm, int32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int v = sub_out[i];
  if (v >= kmin) {
    const int32_t e = sid[i];
    out[perm ? perm[e] : e] = v;
  }
}

// histogram of psi (hist zeroed, psimax + 1 bins); small values counted in LDS first
constexpr int kHistLds = 2048;
__global__ void __launch_bounds__(kT) k_psi_hist(const int32_t* __restrict__ psi, int64_t m,
                                                 int32_t* __restrict__ hist) {
  __shared__ int lh[kHistLds];
  for (int b = threadIdx.x; b < kHistLds; b += blockDim.x) lh[b] = 0;
  __syncthreads();
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int p = psi[e];
    if (p < kHistLds) atomicAdd(&lh[p], 1);
    else atomicAdd(&hist[p], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kHistLds; b += blockDim.x)
    if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

struct TopDownBufs {
  int* d_scalar;
  int32_t* hist;
  int32_t *ssrc, *sdst, *sid, *sout;
  char* sub_ws;
  size_t sub_ws_bytes;
};

size_t topdown_layout(const truss_graph* g, const truss_options* opts, Arena& a, Plan* p, TopDownBufs* b) {
  Plan dummy;
  layout(g, a, p ? *p : dummy, nullptr);
  TopDownBufs t;
  t.d_scalar = a.take<int>(64);
  t.hist = a.take<int32_t>((size_t)g->n + 3);
  t.ssrc = a.take<int32_t>((size_t)g->m + 1);
  t.sdst = a.take<int32_t>((size_t)g->m + 1);
  t.sid = a.take<int32_t>((size_t)g->m + 1);
  t.sout = a.take<int32_t>((size_t)g->m + 1);
  truss_graph sg;
  memset(&sg, 0, sizeof(sg));
  sg.fmt = TRUSS_FMT_EDGES;
  sg.n = g->n;
  sg.m = g->m;
  sg.src = sg.dst = reinterpret_cast<const int32_t*>(1);
  Arena sa;
  sa.counting = true;
  Plan sp;
  layout(&sg, sa, sp, nullptr);
  t.sub_ws_bytes = sa.used;
  t.sub_ws = a.take<char>(sa.used);
  if (b) *b = t;
  (void)opts;
  return a.used;
}

int run_topdown(const truss_graph* g, int32_t t, int32_t* out, int32_t* kmin_out, int32_t* kmax_out,
                const truss_options* opts, truss_stats* stats, void* ws, size_t ws_bytes, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if ((rc = validate_options(opts))) return rc;
  if (t < 1) { set_last_error("t must be at least 1"); return TRUSS_E_INVAL; }
  if (g->m > 0 && !out) { set_last_error("truss_out is NULL"); return TRUSS_E_INVAL; }
  Arena need;
  need.counting = true;
  const size_t bytes = topdown_layout(g, opts, need, nullptr, nullptr);
  if (!ws || ws_bytes < bytes) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, bytes);
    return TRUSS_E_WORKSPACE;
  }
  if (kmin_out) *kmin_out = 0;
  if (kmax_out) *kmax_out = 0;
  if (stats) memset(stats, 0, sizeof(*stats));
  if (g->m == 0) return TRUSS_OK;
  // main region: build, support, upper bound (the same carving order as layout())
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  Plan p;
  p.d_err = a.take<int>(64);
  p.d_total = a.take<unsigned long long>(8);
  SupPlan sp;
  PeelPlan pp;
  int fallback = 0;
  resolve(opts, &sp, &pp, &fallback, s);
  Timer tm(stats != nullptr, s);
  tm.mark(0);
  DevGraph dg;
  rc = build_graph(g, a, dg, p.d_err, s);
  if (rc) return rc;
  p.sr = a.take<int2>((size_t)g->m + 1);
  p.truss_canon = g->fmt == TRUSS_FMT_EDGES ? a.take<int32_t>((size_t)g->m + 1) : nullptr;
  take_bound(g, a, p);
  rc = compute_support(dg, sp, p.sr, a, s, nullptr);
  if (rc) return rc;
  {
    int32_t* hs = a.take<int32_t>((size_t)(2 * g->m + g->n + 1));
    if (a.overflow()) { set_last_error("workspace too small for the upper bound"); return TRUSS_E_WORKSPACE; }
    compute_upper_bound(dg, p.sr, p.h, p.ch, p.psi, hs, s);
  }
  // the top-down region follows the whole single-graph layout
  Arena full;
  full.counting = true;
  Plan dummy;
  layout(g, full, dummy, nullptr);
  Arena b;
  b.base = static_cast<char*>(ws) + full.used;
  b.cap = ws_bytes - full.used;
  TopDownBufs tb;
  tb.d_scalar = b.take<int>(64);
  tb.hist = b.take<int32_t>((size_t)g->n + 3);
  tb.ssrc = b.take<int32_t>((size_t)g->m + 1);
  tb.sdst = b.take<int32_t>((size_t)g->m + 1);
  tb.sid = b.take<int32_t>((size_t)g->m + 1);
  tb.sout = b.take<int32_t>((size_t)g->m + 1);
  {
    truss_graph sg;
    memset(&sg, 0, sizeof(sg));
    sg.fmt = TRUSS_FMT_EDGES;
    sg.n = g->n;
    sg.m = g->m;
    sg.src = sg.dst = reinterpret_cast<const int32_t*>(1);
    Arena sa;
    sa.counting = true;
    Plan sp2;
    layout(&sg, sa, sp2, nullptr);
    tb.sub_ws_bytes = sa.used;
    tb.sub_ws = b.take<char>(sa.used);
  }
  const unsigned gm = grid_for(g->m);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, tb.d_scalar, (int64_t)64, 0);
  hipLaunchKernelGGL(k_max_i32, dim3(1024), dim3(kT), 0, s, p.psi, g->m, tb.d_scalar);
  int psimax = 0;
  TRUSS_HIP(hipMemcpyAsync(&psimax, tb.d_scalar, sizeof(int), hipMemcpyDeviceToHost, s));
  TRUSS_HIP(hipStreamSynchronize(s));
  // |E_k| for every k from the histogram of psi (psi <= max sup + 2 <= n + 1)
  std::vector<int64_t> ek((size_t)psimax + 2, 0);
  {
    std::vector<int32_t> hh((size_t)psimax + 1, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((psimax + kT) / kT)), dim3(kT), 0, s, tb.hist,
                       (int64_t)psimax + 1, 0);
    hipLaunchKernelGGL(k_psi_hist, dim3(1024), dim3(kT), 0, s, p.psi, g->m, tb.hist);
    TRUSS_HIP(hipMemcpyAsync(hh.data(), tb.hist, sizeof(int32_t) * ((size_t)psimax + 1), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    for (int q = psimax; q >= 0; --q) ek[q] = ek[q + 1] + hh[q];
  }
  // largest k' <= kcap with |E_k'| >= size (2 if none)
  auto pick = [&](int kcap, int64_t size) {
    for (int q = kcap; q > 2; --q)
      if (ek[q] >= size) return q;
    return 2;
  };
  int64_t want = ek[psimax] > (1 << 17) ? ek[psimax] : (1 << 17);
  int k = pick(psimax, want), iters = 0, kmax = 0, cnt = 0;
  truss_stats sst;
  memset(&sst, 0, sizeof(sst));
  for (;;) {
    ++iters;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, tb.d_scalar, (int64_t)64, 0);
    hipLaunchKernelGGL(k_select, dim3(gm), dim3(kT), 0, s, p.psi, dg.eu, dg.ev, g->m, k, tb.ssrc, tb.sdst, tb.sid,
                       tb.d_scalar);
    TRUSS_HIP(hipMemcpyAsync(&cnt, tb.d_scalar, sizeof(int), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
    truss_graph sg;
    memset(&sg, 0, sizeof(sg));
    sg.fmt = TRUSS_FMT_EDGES;
    sg.n = g->n;
    sg.m = cnt;
    sg.src = tb.ssrc;
    sg.dst = tb.sdst;
    rc = run_single(&sg, kModeDecompose, tb.sout, nullptr, opts, &sst, tb.sub_ws, tb.sub_ws_bytes, s, nullptr);
    if (rc) return rc;
    const int km = cnt > 0 ? sst.kmax : 0;
    if (km >= k) {
      // k <= k_max: the classes >= k are exact; one more pass if k is above k_max - t + 1
      kmax = km;
      const int kmin = kmax - t + 1 > 2 ? kmax - t + 1 : 2;
      if (k <= kmin) break;
      k = kmin;
    } else if (k <= 2) {
      kmax = km;
      break;
    } else {
      // no k-truss: grow the subgraph about fourfold
      want = 4 * (ek[k] > 1 ? ek[k] : 1);
      k = pick(k - 1, want);
    }
  }
  const int kmin = kmax - t + 1 > 2 ? kmax - t + 1 : 2;
  hipLaunchKernelGGL(k_fill_i32, dim3(gm), dim3(kT), 0, s, out, g->m, 0);
  if (cnt > 0)
    hipLaunchKernelGGL(k_topdown_out, dim3(grid_for(cnt)), dim3(kT), 0, s, tb.sout, tb.sid, (int64_t)cnt, kmin,
                       dg.perm, out);
  TRUSS_HIP(hipGetLastError());
  tm.mark(1);
  TRUSS_HIP(hipStreamSynchronize(s));
  if (kmin_out) *kmin_out = kmin;
  if (kmax_out) *kmax_out = kmax;
  if (stats) {
    *stats = sst;
    stats->n = g->n;
    stats->m = cnt;  // edges of the subgraph decomposed last
    stats->kmax = kmax;
    stats->launches = iters;  // subgraph decompositions
    stats->ms_total = tm.ms(0, 1);
    stats->sched_fallback = fallback;
  }
  return TRUSS_OK;
}

// ---- Algorithm 1 as a comparator ---------------------------------------------------
size_t cohen_layout(const truss_graph* g, Arena& a) {
  a.take<int>(64);
  build_workspace(g, a);
  a.take<int2>((size_t)g->m + 1);
  a.take<int32_t>((size_t)g->m + 1);
  cohen_workspace(g->m, a);
  return a.used;
}

int run_cohen(const truss_graph* g, int32_t* out, truss_stats* stats, void* ws, size_t ws_bytes, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (g->m > 0 && !out) { set_last_error("truss_out is NULL"); return TRUSS_E_INVAL; }
  Arena need;
  need.counting = true;
  const size_t bytes = cohen_layout(g, need);
  if (!ws || ws_bytes < bytes) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, bytes);
    return TRUSS_E_WORKSPACE;
  }
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  int* d_err = a.take<int>(64);
  Timer tm(stats != nullptr, s);
  tm.mark(0);
  DevGraph dg;
  if ((rc = build_graph(g, a, dg, d_err, s))) return rc;
  tm.mark(1);
  int2* sr = a.take<int2>((size_t)g->m + 1);
  int32_t* tc = a.take<int32_t>((size_t)g->m + 1);
  CohenResult cr;
  if ((rc = cohen_decompose(dg, sr, g->fmt == TRUSS_FMT_EDGES ? tc : out, a, &cr, s))) return rc;
  if (g->fmt == TRUSS_FMT_EDGES && g->m > 0)
    hipLaunchKernelGGL(k_scatter_out, dim3(grid_for(g->m)), dim3(kT), 0, s, tc, dg.perm, g->m, out);
  tm.mark(2);
  TRUSS_HIP(hipGetLastError());
  TRUSS_HIP(hipStreamSynchronize(s));
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n = g->n;
    stats->m = g->m;
    stats->kmax = cr.kmax;
    stats->levels = cr.levels;
    stats->subrounds = cr.rounds;
    stats->peel_work = cr.peel_work;
    stats->support_work = cr.support_work;
    stats->ms_build = tm.ms(0, 1);
    stats->ms_support = cr.ms_support;
    stats->ms_peel = cr.ms_peel;
    stats->ms_total = tm.ms(0, 2);
  }
  return TRUSS_OK;
}

// ---- core numbers and the cohesion statistics of Table 6 ---------------------------
size_t core_layout(const truss_graph* g, Arena& a) {
  a.take<int>(64);
  build_workspace(g, a);
  core_workspace(g->n, a);
  return a.used;
}

int run_core(const truss_graph* g, int32_t* core_out, int32_t* cmax_out, void* ws, size_t ws_bytes, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (g->n > 0 && !core_out) { set_last_error("core_out is NULL"); return TRUSS_E_INVAL; }
  Arena need;
  need.counting = true;
  const size_t bytes = core_layout(g, need);
  if (!ws || ws_bytes < bytes) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, bytes);
    return TRUSS_E_WORKSPACE;
  }
  if (cmax_out) *cmax_out = 0;
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  int* d_err = a.take<int>(64);
  DevGraph dg;
  rc = build_graph(g, a, dg, d_err, s);
  if (rc) return rc;
  int32_t cmax = 0;
  rc = compute_core_numbers(dg, core_out, &cmax, a, s);
  if (rc) return rc;
  if (cmax_out) *cmax_out = cmax;
  return TRUSS_OK;
}

// canonical edges whose truss number (given in the caller's indexing) is k
__global__ void k_select_truss(const int32_t* __restrict__ phi, const int32_t* __restrict__ perm,
                               const int32_t* __restrict__ eu, const int32_t* __restrict__ ev, int64_t m, int k,
                               int32_t* __restrict__ ssrc, int32_t* __restrict__ sdst, int* __restrict__ count) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool take = e < m && phi[perm ? perm[e] : e] == k;
  const int pos = wave_append(count, take);
  if (take) {
    ssrc[pos] = eu[e];
    sdst[pos] = ev[e];
  }
}

// canonical edges with both ends of core number c
__global__ void k_select_core(const int32_t* __restrict__ core, const int32_t* __restrict__ eu,
                              const int32_t* __restrict__ ev, int64_t m, int c, int32_t* __restrict__ ssrc,
                              int32_t* __restrict__ sdst, int* __restrict__ count) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool take = false;
  int32_t u = 0, v = 0;
  if (e < m) {
    u = eu[e];
    v = ev[e];
    take = core[u] == c && core[v] == c;
  }
  const int pos = wave_append(count, take);
  if (take) {
    ssrc[pos] = u;
    sdst[pos] = v;
  }
}

struct CohesionBufs {
  int* d_count;
  int32_t *phi, *core, *tsrc, *tdst, *csrc, *cdst, *ssup;
  char* stats_ws;
  size_t stats_bytes;
  char* region;  // decomposition, then build + core numbers, then subgraph support
  size_t region_bytes;
};

// the edge-list graph of up to m edges over n vertices (workspace sizes only)
truss_graph edge_list_shape(int32_t n, int64_t m) {
  truss_graph sg;
  memset(&sg, 0, sizeof(sg));
  sg.fmt = TRUSS_FMT_EDGES;
  sg.n = n;
  sg.m = m;
  sg.src = sg.dst = reinterpret_cast<const int32_t*>(1);
  return sg;
}

size_t cohesion_layout(const truss_graph* g, Arena& a, CohesionBufs* out) {
  CohesionBufs b;
  const size_t m1 = (size_t)g->m + 1, n1 = (size_t)g->n + 1;
  b.d_count = a.take<int>(64);
  b.phi = a.take<int32_t>(m1);
  b.core = a.take<int32_t>(n1);
  b.tsrc = a.take<int32_t>(m1);
  b.tdst = a.take<int32_t>(m1);
  b.csrc = a.take<int32_t>(m1);
  b.cdst = a.take<int32_t>(m1);
  b.ssup = a.take<int32_t>(m1);
  {
    Arena sa;
    sa.counting = true;
    sa.take<int32_t>(n1);
    sa.take<unsigned long long>(n1);
    sa.take<double>(n1);
    sa.take<double>(4);
    b.stats_bytes = sa.used;
  }
  b.stats_ws = a.take<char>(b.stats_bytes);
  size_t r = 0;
  {
    Arena x;
    x.counting = true;
    Plan p;
    layout(g, x, p, nullptr);
    r = x.used;
  }
  {
    Arena x;
    x.counting = true;
    const size_t c = core_layout(g, x);
    r = c > r ? c : r;
  }
  {
    const truss_graph sg = edge_list_shape(g->n, g->m);
    Arena x;
    x.counting = true;
    Plan p;
    layout(&sg, x, p, nullptr);
    r = x.used > r ? x.used : r;
  }
  b.region_bytes = r;
  b.region = a.take<char>(r);
  if (out) *out = b;
  return a.used;
}

int subgraph_cohesion(const truss_graph* g, const CohesionBufs& b, const int32_t* src, const int32_t* dst,
                      int64_t cnt, int64_t* nv, double* cc, hipStream_t s) {
  truss_graph sg;
  memset(&sg, 0, sizeof(sg));
  sg.fmt = TRUSS_FMT_EDGES;
  sg.n = g->n;
  sg.m = cnt;
  sg.src = src;
  sg.dst = dst;
  int rc = run_single(&sg, kModeSupport, b.ssup, nullptr, nullptr, nullptr, b.region, b.region_bytes, s, nullptr);
  if (rc) return rc;
  Arena sa;
  sa.base = b.stats_ws;
  sa.cap = b.stats_bytes;
  double v = 0.0;
  rc = subgraph_vertex_stats(g->n, src, dst, b.ssup, cnt, sa, &v, cc, s);
  *nv = (int64_t)v;
  return rc;
}

int run_cohesion(const truss_graph* g, const truss_options* opts, truss_cohesion_stats* out, void* ws,
                 size_t ws_bytes, hipStream_t s) {
  int rc = check_graph(g);
  if (rc) return rc;
  if ((rc = validate_options(opts))) return rc;
  if (!out) { set_last_error("out is NULL"); return TRUSS_E_INVAL; }
  Arena need;
  need.counting = true;
  const size_t bytes = cohesion_layout(g, need, nullptr);
  if (!ws || ws_bytes < bytes) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, bytes);
    return TRUSS_E_WORKSPACE;
  }
  memset(out, 0, sizeof(*out));
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  CohesionBufs b;
  cohesion_layout(g, a, &b);
  // truss numbers (k_max from the stats)
  truss_stats st;
  rc = run_single(g, kModeDecompose, b.phi, nullptr, opts, &st, b.region, b.region_bytes, s, nullptr);
  if (rc) return rc;
  const int kmax = g->m > 0 ? st.kmax : 0;
  // core numbers; the graph built for them also lists the canonical edges
  Arena r;
  r.base = b.region;
  r.cap = b.region_bytes;
  int* d_err = r.take<int>(64);
  DevGraph dg;
  if ((rc = build_graph(g, r, dg, d_err, s))) return rc;
  int32_t cmax = 0;
  if ((rc = compute_core_numbers(dg, b.core, &cmax, r, s))) return rc;
  int cnt[2] = {0, 0};
  if (g->m > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, b.d_count, (int64_t)64, 0);
    hipLaunchKernelGGL(k_select_truss, dim3(grid_for(g->m)), dim3(kT), 0, s, b.phi, dg.perm, dg.eu, dg.ev, g->m, kmax,
                       b.tsrc, b.tdst, b.d_count);
    hipLaunchKernelGGL(k_select_core, dim3(grid_for(g->m)), dim3(kT), 0, s, b.core, dg.eu, dg.ev, g->m, cmax, b.csrc,
                       b.cdst, b.d_count + 1);
    TRUSS_HIP(hipGetLastError());
    TRUSS_HIP(hipMemcpyAsync(cnt, b.d_count, sizeof(cnt), hipMemcpyDeviceToHost, s));
    TRUSS_HIP(hipStreamSynchronize(s));
  }
  // the region is reused below: the graph built above is no longer needed
  out->kmax = kmax;
  out->cmax = cmax;
  out->e_t = cnt[0];
  out->e_c = cnt[1];
  if ((rc = subgraph_cohesion(g, b, b.tsrc, b.tdst, cnt[0], &out->v_t, &out->cc_t, s))) return rc;
  if ((rc = subgraph_cohesion(g, b, b.csrc, b.cdst, cnt[1], &out->v_c, &out->cc_c, s))) return rc;
  return TRUSS_OK;
}

}  // namespace

size_t subgraph_workspace(int32_t n, int64_t m) {
  truss_graph sg;
  memset(&sg, 0, sizeof(sg));
  sg.fmt = TRUSS_FMT_EDGES;
  sg.n = n;
  sg.m = m;
  sg.src = sg.dst = reinterpret_cast<const int32_t*>(1);
  Arena a;
  a.counting = true;
  Plan p;
  layout(&sg, a, p, nullptr);
  return a.used;
}

int run_subgraph(const SubgraphRun& r, const truss_options* opts, void* ws, size_t ws_bytes, hipStream_t s) {
  truss_graph sg;
  memset(&sg, 0, sizeof(sg));
  sg.fmt = TRUSS_FMT_EDGES;
  sg.n = r.n;
  sg.m = r.m;
  sg.src = r.src;
  sg.dst = r.dst;
  return run_single(&sg, kModeDecompose, r.truss_out, nullptr, opts, nullptr, ws, ws_bytes, s, nullptr, &r);
}

void set_last_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

int device_grid_blocks(const void* kernel, int block, size_t lds) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, block, lds) != hipSuccess || occ < 1) occ = 1;
  if (occ > 4) occ = 4;
  return cus * occ;
}

}  // namespace truss

using namespace truss;

// ---- scratch of truss_decompose_noalloc ---------------------------------------------------
// A fixed device array (one per GPU, held until the process ends) for callers
// that cannot allocate.  Host code never passes the array's name to a kernel:
// it looks up the device address once per device and uses that.
static __device__ __align__(256) unsigned char scratch[TRUSS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, found once per
// device with that device current.
int scratch_address(void** out) {
  int dev = -1;
  TRUSS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_last_error("device %d is beyond the %d devices the scratch table covers", dev, kMaxDevices);
    return TRUSS_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_last_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
      return TRUSS_E_DEVICE;
    }
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return TRUSS_OK;
}
}  // namespace

extern "C" {

void truss_default_options(truss_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->version = TRUSS_VERSION;
  o->support_strategy = TRUSS_SUP_AUTO;
  o->peel_mode = TRUSS_PEEL_AUTO;
  o->scheduler = TRUSS_SCHED_HEURISTIC;
}

int truss_workspace_size(const truss_graph* g, const truss_options* opts, size_t* bytes) {
  int rc = check_graph(g);
  if (rc) return rc;
  rc = validate_options(opts);
  if (rc) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  Arena a;
  a.counting = true;
  Plan p;
  layout(g, a, p, nullptr);
  *bytes = a.used;
  return TRUSS_OK;
}

int truss_support(const truss_graph* g, int32_t* sup_out, int64_t* triangles, void* ws, size_t ws_bytes,
                  void* stream) {
  if (triangles) *triangles = 0;
  if (g && g->m > 0 && !sup_out) { set_last_error("sup_out is NULL"); return TRUSS_E_INVAL; }
  return run_single(g, kModeSupport, sup_out, triangles, nullptr, nullptr, ws, ws_bytes, (hipStream_t)stream,
                    nullptr);
}

int truss_decompose(const truss_graph* g, int32_t* truss_out, const truss_options* opts, truss_stats* stats,
                    void* ws, size_t ws_bytes, void* stream) {
  if (g && g->m > 0 && !truss_out) { set_last_error("truss_out is NULL"); return TRUSS_E_INVAL; }
  return run_single(g, kModeDecompose, truss_out, nullptr, opts, stats, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

int truss_decompose_noalloc(const truss_graph* g, int32_t* truss_out, const truss_options* opts, truss_stats* stats,
                            void* stream) {
  int rc = check_graph(g);
  if (rc) return rc;
  rc = validate_options(opts);
  if (rc) return rc;
  if (g->m > 0 && !truss_out) { set_last_error("truss_out is NULL"); return TRUSS_E_INVAL; }
  Arena need;
  need.counting = true;
  Plan dummy;
  layout(g, need, dummy, nullptr);
  if (need.used > TRUSS_NOALLOC_SCRATCH_BYTES) {
    set_last_error("graph needs %zu bytes of scratch; the fixed array holds %zu", need.used,
                   (size_t)TRUSS_NOALLOC_SCRATCH_BYTES);
    return TRUSS_E_WORKSPACE;
  }
  void* ws = nullptr;
  rc = scratch_address(&ws);
  if (rc) return rc;
  return run_single(g, kModeDecompose, truss_out, nullptr, opts, stats, ws, TRUSS_NOALLOC_SCRATCH_BYTES,
                    (hipStream_t)stream, nullptr, nullptr, false);
}

int truss_decompose_traced(const truss_graph* g, int32_t* truss_out, const truss_options* opts, truss_stats* stats,
                           truss_trace* trace, void* ws, size_t ws_bytes, void* stream) {
  if (!trace) { set_last_error("trace is NULL"); return TRUSS_E_INVAL; }
  if (g && g->m > 0 && !truss_out) { set_last_error("truss_out is NULL"); return TRUSS_E_INVAL; }
  return run_single(g, kModeDecompose, truss_out, nullptr, opts, stats, ws, ws_bytes, (hipStream_t)stream, trace);
}

int truss_upper_bound(const truss_graph* g, int32_t* psi_out, void* ws, size_t ws_bytes, void* stream) {
  if (g && g->m > 0 && !psi_out) { set_last_error("psi_out is NULL"); return TRUSS_E_INVAL; }
  return run_single(g, kModeBound, psi_out, nullptr, nullptr, nullptr, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

int truss_topdown_workspace_size(const truss_graph* g, const truss_options* opts, size_t* bytes) {
  int rc = check_graph(g);
  if (rc) return rc;
  if ((rc = validate_options(opts))) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  Arena a;
  a.counting = true;
  *bytes = topdown_layout(g, opts, a, nullptr, nullptr);
  return TRUSS_OK;
}

int truss_topdown(const truss_graph* g, int32_t t, int32_t* truss_out, int32_t* kmin_out, int32_t* kmax_out,
                  const truss_options* opts, truss_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  return run_topdown(g, t, truss_out, kmin_out, kmax_out, opts, stats, ws, ws_bytes, (hipStream_t)stream);
}

int truss_cohen_workspace_size(const truss_graph* g, size_t* bytes) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  Arena a;
  a.counting = true;
  *bytes = cohen_layout(g, a);
  return TRUSS_OK;
}

int truss_cohen(const truss_graph* g, int32_t* truss_out, truss_stats* stats, void* ws, size_t ws_bytes,
                void* stream) {
  return run_cohen(g, truss_out, stats, ws, ws_bytes, (hipStream_t)stream);
}

int truss_core_workspace_size(const truss_graph* g, size_t* bytes) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  Arena a;
  a.counting = true;
  *bytes = core_layout(g, a);
  return TRUSS_OK;
}

int truss_core_numbers(const truss_graph* g, int32_t* core_out, int32_t* cmax_out, void* ws, size_t ws_bytes,
                       void* stream) {
  return run_core(g, core_out, cmax_out, ws, ws_bytes, (hipStream_t)stream);
}

int truss_cohesion_workspace_size(const truss_graph* g, size_t* bytes) {
  int rc = check_graph(g);
  if (rc) return rc;
  if (!bytes) { set_last_error("bytes is NULL"); return TRUSS_E_INVAL; }
  Arena a;
  a.counting = true;
  *bytes = cohesion_layout(g, a, nullptr);
  return TRUSS_OK;
}

int truss_cohesion(const truss_graph* g, const truss_options* opts, truss_cohesion_stats* out, void* ws,
                   size_t ws_bytes, void* stream) {
  return run_cohesion(g, opts, out, ws, ws_bytes, (hipStream_t)stream);
}

const char* truss_strerror(int code) {
  switch (code) {
    case TRUSS_OK: return "success";
    case TRUSS_E_INVAL: return "invalid argument";
    case TRUSS_E_TOOBIG: return "graph too large (m > INT32_MAX)";
    case TRUSS_E_ROWPTR: return "invalid CSR row_ptr";
    case TRUSS_E_RANGE: return "vertex id out of range";
    case TRUSS_E_SELFLOOP: return "self-loop";
    case TRUSS_E_UNSORTED: return "CSR row not strictly ascending";
    case TRUSS_E_DUP: return "duplicate edge";
    case TRUSS_E_ASYM: return "CSR not symmetric";
    case TRUSS_E_NOMEM: return "out of device memory";
    case TRUSS_E_WORKSPACE: return "workspace too small";
    case TRUSS_E_DEVICE: return "HIP runtime error";
    case TRUSS_E_INTERNAL: return "internal limit reached";
    default: return "unknown error";
  }
}

const char* truss_last_error(void) { return g_last_error; }

int truss_version(void) { return TRUSS_VERSION; }

}  // extern "C"
