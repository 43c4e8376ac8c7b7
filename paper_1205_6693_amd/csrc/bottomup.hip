// Bottom-up truss decomposition of a graph held in host memory (Section 5):
// LowerBounding (Algorithm 3), then Algorithm 4 with Procedure 5, or
// Procedure 9 (Appendix) when a candidate subgraph exceeds the budget.
//
// Host memory plays the part of the paper's disk and the device that of its
// main memory: the graph, the bounds and the outputs stay on the host, and
// each neighbourhood subgraph NS(P) (Definition 4) is relabelled, copied to
// the device and decomposed there by the in-memory path.  The budget is the
// most edges a subgraph sent to the device may hold.
//
// Partition of a vertex set (Algorithm 3 and Procedure 9):
// parts are grown breadth-first over the edges of the graph being partitioned
// (the current G; H' in Procedure 9).  A part starts at the smallest-id
// unplaced vertex that has such an edge and takes, from each vertex it holds
// in the order added, every unplaced neighbour (ascending id) whose weight
// still fits; when its growth stops it goes on from the next such vertex by id
// if that one fits, else a new part starts there.  A vertex weighs its degree
// in the graph the subgraphs are taken from, so |NS(P)| <= the part's weight
// sum <= the budget.
//
// The 2-class: only the first pass of Algorithm 3 sees the input graph, so
// only there does an internal edge of support 0 go to Phi_2; internal edges of
// later passes go to G_new with their bound, and Algorithm 4 then starts at
// k = 2.  Algorithm 4 skips each k for which no remaining edge has a bound
// <= k (U_k and Phi_k are empty there).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <exception>
#include <new>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace truss {

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// The input graph on the host: rows sorted by neighbour id, with edge ids.
struct HostGraph {
  int32_t n = 0;
  int64_t m = 0;
  const int32_t* src = nullptr;
  const int32_t* dst = nullptr;
  std::vector<int64_t> off, end;  // row v holds entries off[v] .. end[v]
  std::vector<int32_t> nbr, eid;
  int64_t stored = 0;             // entries held over all rows

  // Keeps only the entries of edges with flag[e] == live once the live edges
  // fill less than 70% of the entries held; rows keep their ascending order.
  void compact(const uint8_t* flag, uint8_t live, int64_t live_edges) {
    if (10 * (2 * live_edges) >= 7 * stored) return;
    stored = 0;
    for (int32_t v = 0; v < n; ++v) {
      int64_t w = off[v];
      for (int64_t j = off[v]; j < end[v]; ++j)
        if (flag[eid[(size_t)j]] == live) {
          nbr[(size_t)w] = nbr[(size_t)j];
          eid[(size_t)w++] = eid[(size_t)j];
        }
      end[v] = w;
      stored += w - off[v];
    }
  }
};

bool verbose() {
  const char* v = getenv("TRUSS_VERBOSE");
  return v && *v && *v != '0';
}

// Host threads for the scans over a subgraph (at most 16).
int host_threads() {
  static const int t = [] {
    const unsigned h = std::thread::hardware_concurrency();
    const int x = h ? (int)h : 4;
    return x < 16 ? x : 16;
  }();
  return t;
}

// f(lo, hi, t) over [0, n) cut into at most host_threads() contiguous
// pieces of at least `grain` items; piece t is [lo, hi).  Returns the pieces.
template <typename F>
int parallel_pieces(int64_t n, int64_t grain, F&& f) {
  int64_t parts = (n + grain - 1) / grain;
  if (parts > host_threads()) parts = host_threads();
  if (parts <= 1) {
    if (n > 0) f((int64_t)0, n, 0);
    return n > 0 ? 1 : 0;
  }
  const int64_t chunk = (n + parts - 1) / parts;
  // an exception in a piece (a failed allocation) is carried to the caller
  // once every started thread has been joined
  std::vector<std::exception_ptr> err((size_t)parts);
  auto piece = [&f, &err](int64_t lo, int64_t hi, int t) {
    try {
      f(lo, hi, t);
    } catch (...) {
      err[(size_t)t] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  try {
    th.reserve((size_t)parts);
    for (int t = 1; t < parts; ++t) {
      const int64_t lo = t * chunk, hi = lo + chunk < n ? lo + chunk : n;
      if (lo < hi) th.emplace_back(piece, lo, hi, t);
    }
  } catch (...) {
    for (auto& x : th) x.join();
    throw;
  }
  piece((int64_t)0, chunk < n ? chunk : n, 0);
  for (auto& x : th) x.join();
  for (auto& x : err)
    if (x) std::rethrow_exception(x);
  return (int)parts;
}
constexpr int64_t kGrain = 1 << 16;

template <typename T>
void atomic_add(T* p, T v) {
  __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}

int build_host_graph(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, HostGraph& g) {
  g.n = n;
  g.m = m;
  g.src = src;
  g.dst = dst;
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = src[e], v = dst[e];
    if (u < 0 || u >= n || v < 0 || v >= n) {
      set_last_error("edge %lld has an endpoint outside [0, n)", (long long)e);
      return TRUSS_E_RANGE;
    }
    if (u == v) {
      set_last_error("edge %lld is a self-loop", (long long)e);
      return TRUSS_E_SELFLOOP;
    }
  }
  g.off.assign((size_t)n + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    g.off[(size_t)src[e] + 1]++;
    g.off[(size_t)dst[e] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) g.off[(size_t)v + 1] += g.off[v];
  // rows in edge order, then transposed row by row: row y receives its
  // neighbours x in ascending x
  std::vector<int32_t> tn((size_t)(2 * m)), te((size_t)(2 * m));
  std::vector<int64_t> fill(g.off.begin(), g.off.end() - 1);
  for (int64_t e = 0; e < m; ++e) {
    const int32_t u = src[e], v = dst[e];
    tn[(size_t)fill[u]] = v;
    te[(size_t)fill[u]++] = (int32_t)e;
    tn[(size_t)fill[v]] = u;
    te[(size_t)fill[v]++] = (int32_t)e;
  }
  g.nbr.resize((size_t)(2 * m));
  g.eid.resize((size_t)(2 * m));
  std::copy(g.off.begin(), g.off.end() - 1, fill.begin());
  for (int32_t x = 0; x < n; ++x)
    for (int64_t j = g.off[x]; j < g.off[(size_t)x + 1]; ++j) {
      const int32_t y = tn[(size_t)j];
      g.nbr[(size_t)fill[y]] = x;
      g.eid[(size_t)fill[y]++] = te[(size_t)j];
    }
  for (int32_t v = 0; v < n; ++v)
    for (int64_t j = g.off[v] + 1; j < g.off[(size_t)v + 1]; ++j)
      if (g.nbr[(size_t)j] == g.nbr[(size_t)j - 1]) {
        set_last_error("edge (%d, %d) is given twice", v, g.nbr[(size_t)j]);
        return TRUSS_E_DUP;
      }
  g.end.assign(g.off.begin() + 1, g.off.end());
  g.stored = 2 * m;
  return TRUSS_OK;
}

// A partition: vertices in placement order, part p = order[start[p] .. start[p+1]).
struct Parts {
  std::vector<int32_t> part;   // n: part id, -1 if not placed
  std::vector<int32_t> order;  // placed vertices, part by part
  std::vector<int64_t> start;  // parts + 1
  int64_t count() const { return (int64_t)start.size() - 1; }
};

// Rows of a graph: vertex v's entries (neighbour, edge index) are
// off[v] .. end[v], ascending by neighbour.
struct Rows {
  int32_t n;
  const int64_t* off;
  const int64_t* end;
  const int32_t* nbr;
  const int32_t* eid;
};

Rows rows_of(const HostGraph& g) {
  return Rows{g.n, g.off.data(), g.end.data(), g.nbr.data(), g.eid.data()};
}

// Parts grown breadth-first (see the file comment).  mask: by edge index, the
// edges of the graph being partitioned.  Returns false if a vertex alone
// weighs more than cap.
bool grow_parts(const Rows& g, const uint8_t* mask, const int64_t* w, int64_t cap, Parts& P) {
  P.part.assign((size_t)g.n, -1);
  P.order.clear();
  P.start.assign(1, 0);
  int64_t sum = 0, parts = 0;
  for (int32_t r = 0; r < g.n; ++r) {
    if (P.part[r] >= 0) continue;
    bool has = false;
    for (int64_t j = g.off[r]; j < g.end[r] && !has; ++j) has = mask[g.eid[j]] != 0;
    if (!has) continue;
    if (w[r] > cap) {
      set_last_error("vertex %d alone needs %lld edges, more than the budget of %lld", r, (long long)w[r],
                     (long long)cap);
      return false;
    }
    if (parts == 0 || sum + w[r] > cap) {  // a new part starts at r
      if (parts > 0) P.start.push_back((int64_t)P.order.size());
      parts += 1;
      sum = 0;
    }
    const int32_t p = (int32_t)(parts - 1);
    size_t head = P.order.size();
    sum += w[r];
    P.part[r] = p;
    P.order.push_back(r);
    while (head < P.order.size()) {
      const int32_t v = P.order[head++];
      for (int64_t j = g.off[v]; j < g.end[v]; ++j) {
        const int32_t x = g.nbr[j];
        if (!mask[g.eid[j]] || P.part[x] >= 0 || sum + w[x] > cap) continue;
        P.part[x] = p;
        sum += w[x];
        P.order.push_back(x);
      }
    }
  }
  if (parts > 0) P.start.push_back((int64_t)P.order.size());
  return true;
}

// A subgraph sent to the device: global edge ids and relabelled endpoints.
struct Staged {
  std::vector<int32_t> ids;  // global edge ids, in staging order
  std::vector<uint8_t> flag;  // per staged edge (meaning set by the caller)
};

// Device side: staging buffers and the subgraph workspace, carved from the
// caller's workspace; pinned host mirrors.
struct Device {
  int64_t cap = 0;
  int32_t *d_src = nullptr, *d_dst = nullptr, *d_out = nullptr, *d_sup = nullptr;
  uint8_t* d_frozen = nullptr;
  void* sub_ws = nullptr;
  size_t sub_bytes = 0;
  int32_t *h_src = nullptr, *h_dst = nullptr, *h_out = nullptr, *h_sup = nullptr;
  uint8_t* h_frozen = nullptr;
  std::vector<int32_t> lid;      // n: local id of a vertex in the current subgraph, -1 otherwise
  std::vector<int32_t> touched;  // vertices with a local id
  int64_t calls = 0, h2d = 0, d2h = 0;
  double ms_relabel = 0.0, ms_device = 0.0;  // host relabelling; copies and subgraph runs
  ~Device() {
    if (h_src) (void)hipHostFree(h_src);
  }
};

size_t device_layout(int64_t cap, Arena& a, Device* d) {
  const size_t c = (size_t)(cap > 0 ? cap : 1);
  int32_t* s = a.take<int32_t>(c);
  int32_t* t = a.take<int32_t>(c);
  int32_t* o = a.take<int32_t>(c);
  int32_t* p = a.take<int32_t>(c);
  uint8_t* f = a.take<uint8_t>(c);
  const size_t sub = subgraph_workspace((int32_t)std::min<int64_t>(2 * cap + 1, 0x7fffffff), cap);
  char* w = a.take<char>(sub);
  if (d) {
    d->d_src = s;
    d->d_dst = t;
    d->d_out = o;
    d->d_sup = p;
    d->d_frozen = f;
    d->sub_ws = w;
    d->sub_bytes = sub;
  }
  return a.used;
}

// Relabels the staged edges, copies them to the device, runs the subgraph
// and brings back the per-edge truss level (and supports when want_sup).
int run_staged(const HostGraph& g, Device& D, const Staged& S, bool frozen, int first_level, int stop_level,
               bool want_sup, const truss_options* opts, hipStream_t s) {
  const int64_t h = (int64_t)S.ids.size();
  const auto t0 = Clock::now();
  int32_t nl = 0;
  if (h >= 4 * kGrain && 8 * h >= (int64_t)g.n) {
    // large subgraphs: mark the vertices in parallel, number them in id
    // order, then map the edges in parallel
    int32_t* lid = D.lid.data();
    parallel_pieces(h, kGrain, [&](int64_t lo, int64_t hi, int) {
      for (int64_t i = lo; i < hi; ++i) {
        const int32_t e = S.ids[(size_t)i];
        __atomic_store_n(&lid[g.src[e]], -2, __ATOMIC_RELAXED);
        __atomic_store_n(&lid[g.dst[e]], -2, __ATOMIC_RELAXED);
      }
    });
    for (int32_t v = 0; v < g.n; ++v)
      if (lid[v] == -2) lid[v] = nl++;
    parallel_pieces(h, kGrain, [&](int64_t lo, int64_t hi, int) {
      for (int64_t i = lo; i < hi; ++i) {
        const int32_t e = S.ids[(size_t)i];
        D.h_src[i] = lid[g.src[e]];
        D.h_dst[i] = lid[g.dst[e]];
        if (frozen) D.h_frozen[i] = S.flag[(size_t)i] ? 0 : 1;
      }
    });
    parallel_pieces(g.n, kGrain, [&](int64_t lo, int64_t hi, int) {
      for (int64_t v = lo; v < hi; ++v) lid[v] = -1;
    });
  } else {
    for (int64_t i = 0; i < h; ++i) {
      const int32_t e = S.ids[(size_t)i];
      const int32_t u = g.src[e], v = g.dst[e];
      if (D.lid[u] < 0) {
        D.lid[u] = nl++;
        D.touched.push_back(u);
      }
      if (D.lid[v] < 0) {
        D.lid[v] = nl++;
        D.touched.push_back(v);
      }
      D.h_src[i] = D.lid[u];
      D.h_dst[i] = D.lid[v];
      if (frozen) D.h_frozen[i] = S.flag[(size_t)i] ? 0 : 1;
    }
    for (int32_t v : D.touched) D.lid[v] = -1;
    D.touched.clear();
  }
  const auto t1 = Clock::now();
  D.ms_relabel += std::chrono::duration<double, std::milli>(t1 - t0).count();
  const size_t b = sizeof(int32_t) * (size_t)h;
  TRUSS_HIP(hipMemcpyAsync(D.d_src, D.h_src, b, hipMemcpyHostToDevice, s));
  TRUSS_HIP(hipMemcpyAsync(D.d_dst, D.h_dst, b, hipMemcpyHostToDevice, s));
  D.h2d += 2 * (int64_t)b;
  if (frozen) {
    TRUSS_HIP(hipMemcpyAsync(D.d_frozen, D.h_frozen, (size_t)h, hipMemcpyHostToDevice, s));
    D.h2d += h;
  }
  SubgraphRun r;
  r.src = D.d_src;
  r.dst = D.d_dst;
  r.n = nl;
  r.m = h;
  r.truss_out = D.d_out;
  r.sup_out = want_sup ? D.d_sup : nullptr;
  r.frozen = frozen ? D.d_frozen : nullptr;
  r.first_level = first_level;
  r.stop_level = stop_level;
  const int rc = run_subgraph(r, opts, D.sub_ws, D.sub_bytes, s);
  if (rc) return rc;
  TRUSS_HIP(hipMemcpyAsync(D.h_out, D.d_out, b, hipMemcpyDeviceToHost, s));
  D.d2h += (int64_t)b;
  if (want_sup) {
    TRUSS_HIP(hipMemcpyAsync(D.h_sup, D.d_sup, b, hipMemcpyDeviceToHost, s));
    D.d2h += (int64_t)b;
  }
  TRUSS_HIP(hipStreamSynchronize(s));
  D.calls += 1;
  D.ms_device += ms_since(t1);
  return TRUSS_OK;
}

struct Run {
  HostGraph& g;
  Device& D;
  const truss_options* opts;
  hipStream_t s;
  int64_t cap;
  int32_t* truss;  // host output
  truss_bottomup_stats st;
};

// ---- LowerBounding (Algorithm 3) -------------------------------------------------
int lower_bounding(Run& R, const int32_t* first_part, std::vector<int32_t>& lb, std::vector<uint8_t>& phi2) {
  const HostGraph& g = R.g;
  const auto t0 = Clock::now();
  std::vector<uint8_t> alive((size_t)g.m, 1);
  std::vector<int64_t> deg((size_t)g.n);
  for (int32_t v = 0; v < g.n; ++v) deg[v] = g.end[v] - g.off[v];
  lb.assign((size_t)g.m, 2);  // the bound starts at 2, as in Example 3
  phi2.assign((size_t)g.m, 0);
  Parts P;
  Staged S;
  int64_t left = g.m;
  while (left > 0) {  // one pass over the remaining graph
    const bool first = R.st.passes == 0;
    R.st.passes += 1;
    if (first && first_part) {  // the caller's partition
      int32_t parts = 0;
      P.part.assign((size_t)g.n, -1);
      for (int32_t v = 0; v < g.n; ++v) {
        if (deg[v] == 0) continue;
        if (first_part[v] < 0 || first_part[v] >= g.n) {
          set_last_error("vertex %d has edges but no part id in [0, n)", v);
          return TRUSS_E_INVAL;
        }
        P.part[v] = first_part[v];
        parts = std::max(parts, first_part[v] + 1);
      }
      std::vector<int64_t> cnt((size_t)parts + 1, 0);
      for (int32_t v = 0; v < g.n; ++v)
        if (P.part[v] >= 0) cnt[(size_t)P.part[v] + 1]++;
      for (int32_t p = 0; p < parts; ++p) cnt[(size_t)p + 1] += cnt[p];
      P.start = cnt;
      P.order.assign((size_t)cnt[(size_t)parts], 0);
      for (int32_t v = 0; v < g.n; ++v)
        if (P.part[v] >= 0) P.order[(size_t)cnt[P.part[v]]++] = v;
    } else if (!grow_parts(rows_of(g), alive.data(), deg.data(), R.cap, P)) {
      return TRUSS_E_WORKSPACE;
    }
    int64_t removed = 0;
    for (int64_t p = 0; p < P.count(); ++p) {
      // H = NS(P_p) in the current G; flag = internal
      S.ids.clear();
      S.flag.clear();
      for (int64_t i = P.start[(size_t)p]; i < P.start[(size_t)p + 1]; ++i) {
        const int32_t v = P.order[(size_t)i];
        for (int64_t j = g.off[v]; j < g.end[v]; ++j) {
          const int32_t e = g.eid[(size_t)j], w = g.nbr[(size_t)j];
          if (!alive[(size_t)e]) continue;
          const bool inside = P.part[w] == p;
          if (inside && w < v) continue;  // listed from its smaller end
          S.ids.push_back(e);
          S.flag.push_back(inside ? 1 : 0);
        }
      }
      const int64_t h = (int64_t)S.ids.size();
      if (h == 0) continue;
      if (h > R.cap) {
        set_last_error("the neighbourhood subgraph of part %lld has %lld edges, more than the budget of %lld",
                       (long long)p, (long long)h, (long long)R.cap);
        return TRUSS_E_WORKSPACE;
      }
      R.st.subgraphs += 1;
      R.st.max_subgraph = std::max(R.st.max_subgraph, h);
      int rc = run_staged(g, R.D, S, false, 2, 0, true, R.opts, R.s);  // local truss numbers
      if (rc) return rc;
      for (int64_t i = 0; i < h; ++i) {
        const int32_t e = S.ids[(size_t)i];
        lb[(size_t)e] = std::max(lb[(size_t)e], R.D.h_out[i]);  // Lemma 1
        if (!S.flag[(size_t)i]) continue;
        if (first && R.D.h_sup[i] == 0) {  // Phi_2
          phi2[(size_t)e] = 1;
          R.st.phi2_edges += 1;
        } else {  // G_new
          R.st.gnew_edges += 1;
        }
        alive[(size_t)e] = 0;
        deg[g.src[e]] -= 1;
        deg[g.dst[e]] -= 1;
        removed += 1;
      }
    }
    if (removed == 0) {
      set_last_error("no part holds an internal edge: the budget of %lld edges is too small for this graph",
                     (long long)R.cap);
      return TRUSS_E_WORKSPACE;
    }
    left -= removed;  // (rows are not compacted here: Algorithm 4 reads every edge of G_new from them)
    if (verbose())
      fprintf(stderr, "truss_bottomup: lower bounding pass %lld: %lld parts, %lld edges left, %.0f ms\n",
              (long long)R.st.passes, (long long)P.count(), (long long)left, ms_since(t0));
  }
  return TRUSS_OK;
}

// ---- Algorithm 4 -------------------------------------------------------------------
struct BottomUp {
  Run& R;
  std::vector<uint8_t> gone;
  std::vector<int32_t> cnt;  // per vertex: remaining edges with bound <= k (U_k = cnt > 0)
  int64_t left = 0, active_left = 0;

  void output(int32_t e, int32_t k) {
    R.truss[e] = k;
    gone[(size_t)e] = 1;
    left -= 1;
    active_left -= 1;
    cnt[R.g.src[e]] -= 1;
    cnt[R.g.dst[e]] -= 1;
  }
  // the same from several threads on distinct edges; the caller subtracts
  // the number of edges output from left and active_left afterwards
  void output_shared(int32_t e, int32_t k) {
    R.truss[e] = k;
    gone[(size_t)e] = 1;
    atomic_add(&cnt[R.g.src[e]], -1);
    atomic_add(&cnt[R.g.dst[e]], -1);
  }
  void count_outputs(int64_t c) {
    left -= c;
    active_left -= c;
  }
};

// Sum of per-piece counts.
struct PieceSums {
  int64_t v[16] = {0};
  int64_t total() const {
    int64_t t = 0;
    for (int64_t x : v) t += x;
    return t;
  }
};

// Procedure 5 on the candidate subgraph H (flag = internal).
int procedure5(BottomUp& B, const Staged& H, int32_t k, int64_t* found) {
  int rc = run_staged(B.R.g, B.R.D, H, true, k, k, false, B.R.opts, B.R.s);
  if (rc) return rc;
  PieceSums c;
  parallel_pieces((int64_t)H.ids.size(), kGrain, [&](int64_t lo, int64_t hi, int t) {
    for (int64_t i = lo; i < hi; ++i)
      if (H.flag[(size_t)i] && B.R.D.h_out[i] == k) {
        B.output_shared(H.ids[(size_t)i], k);
        c.v[t] += 1;
      }
  });
  B.count_outputs(c.total());
  *found += c.total();
  return TRUSS_OK;
}

// The candidate subgraph H as rows of its own: local vertex ids in ascending
// global id (so the partition visits vertices and neighbours in the same order
// as on the whole graph), edge indices into H.
struct LocalRows {
  std::vector<int32_t> gid;  // local vertex -> global vertex
  std::vector<int64_t> off, end;
  std::vector<int32_t> nbr, eid;
  std::vector<int32_t> lu, lv;  // local endpoints of H's edges
  Rows view() const {
    return Rows{(int32_t)gid.size(), off.data(), end.data(), nbr.data(), eid.data()};
  }
};

void build_local_rows(const HostGraph& g, const Staged& H, std::vector<int32_t>& lid, LocalRows& L) {
  const size_t h = H.ids.size();
  L.gid.clear();
  for (size_t i = 0; i < h; ++i)
    for (const int32_t v : {g.src[H.ids[i]], g.dst[H.ids[i]]})
      if (lid[v] < 0) {
        lid[v] = 0;
        L.gid.push_back(v);
      }
  std::sort(L.gid.begin(), L.gid.end());
  const int32_t nl = (int32_t)L.gid.size();
  for (int32_t x = 0; x < nl; ++x) lid[L.gid[x]] = x;
  L.lu.resize(h);
  L.lv.resize(h);
  L.off.assign((size_t)nl + 1, 0);
  for (size_t i = 0; i < h; ++i) {
    L.lu[i] = lid[g.src[H.ids[i]]];
    L.lv[i] = lid[g.dst[H.ids[i]]];
    L.off[(size_t)L.lu[i] + 1]++;
    L.off[(size_t)L.lv[i] + 1]++;
  }
  for (int32_t x = 0; x < nl; ++x) L.off[(size_t)x + 1] += L.off[x];
  for (const int32_t v : L.gid) lid[v] = -1;
  // rows in edge order, then transposed so each row is ascending
  std::vector<int32_t> tn(2 * h), te(2 * h);
  std::vector<int64_t> fill(L.off.begin(), L.off.end() - 1);
  for (size_t i = 0; i < h; ++i) {
    tn[(size_t)fill[L.lu[i]]] = L.lv[i];
    te[(size_t)fill[L.lu[i]]++] = (int32_t)i;
    tn[(size_t)fill[L.lv[i]]] = L.lu[i];
    te[(size_t)fill[L.lv[i]]++] = (int32_t)i;
  }
  L.nbr.resize(2 * h);
  L.eid.resize(2 * h);
  std::copy(L.off.begin(), L.off.end() - 1, fill.begin());
  for (int32_t x = 0; x < nl; ++x)
    for (int64_t j = L.off[x]; j < L.off[(size_t)x + 1]; ++j) {
      const int32_t y = tn[(size_t)j];
      L.nbr[(size_t)fill[y]] = x;
      L.eid[(size_t)fill[y]++] = te[(size_t)j];
    }
  L.end.assign(L.off.begin() + 1, L.off.end());
}

// Procedure 9: H exceeds the budget; its internal edges are examined part by
// part until a whole scan adds nothing to Phi_k.
int procedure9(BottomUp& B, const Staged& H, int32_t k, std::vector<int32_t>& lid, int64_t* found_total) {
  Run& R = B.R;
  const HostGraph& g = R.g;
  const size_t h = H.ids.size();
  LocalRows L;
  build_local_rows(g, H, lid, L);
  const Rows rows = L.view();
  std::vector<uint8_t> inh(h, 1), cov(h, 0), mask(h, 0);
  std::vector<int64_t> deg((size_t)rows.n, 0);
  std::vector<int32_t> fidx;
  std::vector<std::vector<int32_t>> piece((size_t)host_threads());
  std::vector<int64_t> moff((size_t)rows.n + 1);
  std::vector<int32_t> mnbr(2 * h), meid(2 * h);
  Parts P;
  Staged F;
  R.st.proc9_calls += 1;
  for (;;) {  // scans of H until one adds nothing to Phi_k
    int64_t found = 0;
    for (size_t i = 0; i < h; ++i) cov[i] = !inh[i];  // H' = H
    for (;;) {
      std::fill(deg.begin(), deg.end(), 0);
      PieceSums lc;
      parallel_pieces((int64_t)h, kGrain, [&](int64_t lo, int64_t hi, int t) {
        for (int64_t i = lo; i < hi; ++i) {
          mask[(size_t)i] = inh[(size_t)i] && !cov[(size_t)i];
          if (!inh[(size_t)i]) continue;
          atomic_add(&deg[(size_t)L.lu[(size_t)i]], (int64_t)1);
          atomic_add(&deg[(size_t)L.lv[(size_t)i]], (int64_t)1);
          lc.v[t] += !cov[(size_t)i];
        }
      });
      const int64_t left = lc.total();
      if (left == 0) break;
      R.st.proc9_scans += 1;
      // rows of H' alone (same order), so that the partition walks only its edges
      parallel_pieces(rows.n, kGrain, [&](int64_t lo, int64_t hi, int) {
        for (int64_t x = lo; x < hi; ++x) {
          int64_t c = 0;
          for (int64_t j = rows.off[x]; j < rows.end[x]; ++j) c += mask[(size_t)rows.eid[j]];
          moff[(size_t)x + 1] = c;
        }
      });
      moff[0] = 0;
      for (int32_t x = 0; x < rows.n; ++x) moff[(size_t)x + 1] += moff[(size_t)x];
      parallel_pieces(rows.n, kGrain, [&](int64_t lo, int64_t hi, int) {
        for (int64_t x = lo; x < hi; ++x) {
          int64_t w = moff[(size_t)x];
          for (int64_t j = rows.off[x]; j < rows.end[x]; ++j)
            if (mask[(size_t)rows.eid[j]]) {
              mnbr[(size_t)w] = rows.nbr[j];
              meid[(size_t)w++] = rows.eid[j];
            }
        }
      });
      const Rows hrows{rows.n, moff.data(), moff.data() + 1, mnbr.data(), meid.data()};
      if (!grow_parts(hrows, mask.data(), deg.data(), R.cap, P)) return TRUSS_E_WORKSPACE;
      int64_t covered = 0;
      for (int64_t p = 0; p < P.count(); ++p) {
        // F = NS(P_p) in the current H; flag = eligible (internal to F and to H)
        // local edge indices of F, gathered piecewise over the part's vertices
        const int64_t p0 = P.start[(size_t)p], np = P.start[(size_t)p + 1] - p0;
        for (auto& x : piece) x.clear();
        const int pieces = parallel_pieces(np, 4096, [&](int64_t lo, int64_t hi, int t) {
          std::vector<int32_t>& out = piece[(size_t)t];
          for (int64_t q = lo; q < hi; ++q) {
            const int32_t v = P.order[(size_t)(p0 + q)];
            for (int64_t j = rows.off[v]; j < rows.end[v]; ++j) {
              const int32_t i = rows.eid[j], w = rows.nbr[j];
              if (!inh[(size_t)i]) continue;
              const bool inside = P.part[w] == p;
              if (inside && w < v) continue;
              out.push_back(inside ? i : ~i);  // ~i: an edge leaving the part
            }
          }
        });
        fidx.clear();
        for (int t = 0; t < pieces; ++t) fidx.insert(fidx.end(), piece[(size_t)t].begin(), piece[(size_t)t].end());
        if (fidx.empty()) continue;
        const int64_t nf = (int64_t)fidx.size();
        F.ids.resize((size_t)nf);
        F.flag.resize((size_t)nf);
        parallel_pieces(nf, kGrain, [&](int64_t lo, int64_t hi, int) {
          for (int64_t j = lo; j < hi; ++j) {
            const int32_t x = fidx[(size_t)j];
            const bool inside = x >= 0;
            const size_t i = (size_t)(inside ? x : ~x);
            F.ids[(size_t)j] = H.ids[i];
            F.flag[(size_t)j] = inside && H.flag[i] ? 1 : 0;
          }
        });
        const int rc = run_staged(g, R.D, F, true, k, k, false, R.opts, R.s);  // peel level k of F
        if (rc) return rc;
        PieceSums fc, cc;
        parallel_pieces(nf, kGrain, [&](int64_t lo, int64_t hi, int t) {
          for (int64_t j = lo; j < hi; ++j) {
            const int32_t x = fidx[(size_t)j];
            const size_t i = (size_t)(x >= 0 ? x : ~x);
            if (F.flag[(size_t)j] && R.D.h_out[j] == k) {  // joins Phi_k
              B.output_shared(F.ids[(size_t)j], k);
              inh[i] = 0;
              fc.v[t] += 1;
            }
            if (x >= 0 && !cov[i]) {  // leaves H' (each internal edge of F appears once)
              cov[i] = 1;
              cc.v[t] += 1;
            }
          }
        });
        B.count_outputs(fc.total());
        found += fc.total();
        covered += cc.total();
      }
      if (covered == 0) {
        set_last_error("procedure 9 made no progress: the budget of %lld edges is too small", (long long)R.cap);
        return TRUSS_E_WORKSPACE;
      }
    }
    *found_total += found;
    if (found == 0) break;
  }
  return TRUSS_OK;
}

int bottom_up(Run& R, const std::vector<int32_t>& lb, const std::vector<uint8_t>& phi2) {
  HostGraph& g = R.g;
  const auto t0 = Clock::now();
  BottomUp B{R, {}, {}, 0, 0};
  B.gone.assign((size_t)g.m, 0);
  B.cnt.assign((size_t)g.n, 0);
  int32_t maxlb = 2;
  for (int64_t e = 0; e < g.m; ++e) {
    if (phi2[(size_t)e]) {
      B.gone[(size_t)e] = 1;
      R.truss[e] = 2;
    } else {
      R.truss[e] = 0;
      B.left += 1;
      maxlb = std::max(maxlb, lb[(size_t)e]);
    }
  }
  // G_new's edges by bound (counting sort); activated in that order as k grows
  std::vector<int64_t> byb((size_t)maxlb + 2, 0);
  for (int64_t e = 0; e < g.m; ++e)
    if (!phi2[(size_t)e]) byb[(size_t)lb[(size_t)e] + 1]++;
  for (int32_t b = 0; b <= maxlb; ++b) byb[(size_t)b + 1] += byb[b];
  std::vector<int32_t> sorted((size_t)B.left);
  for (int64_t e = 0; e < g.m; ++e)
    if (!phi2[(size_t)e]) sorted[(size_t)byb[lb[(size_t)e]]++] = (int32_t)e;
  std::vector<int32_t> ulist, lid((size_t)g.n, -1);
  std::vector<std::vector<int32_t>> hpiece((size_t)host_threads());
  std::vector<uint8_t> inlist((size_t)g.n, 0);
  size_t ap = 0;
  Staged H;
  int32_t k = R.st.kstart;
  while (B.left > 0) {  // one level k at a time
    // U_k = ends of the remaining edges with bound <= k
    for (;;) {
      while (ap < sorted.size() && lb[(size_t)sorted[ap]] <= k) {
        const int32_t e = sorted[ap++];
        for (const int32_t v : {g.src[e], g.dst[e]}) {
          if (B.cnt[v]++ == 0 && !inlist[v]) {
            inlist[v] = 1;
            ulist.push_back(v);
          }
        }
        B.active_left += 1;
      }
      if (B.active_left > 0) break;
      k = lb[(size_t)sorted[ap]];  // no candidate at this k: Phi_k is empty
    }
    // H = NS(U_k); flag = internal
    size_t keep = 0;
    for (size_t i = 0; i < ulist.size(); ++i) {
      const int32_t u = ulist[i];
      if (B.cnt[u] > 0) ulist[keep++] = u;
      else inlist[u] = 0;
    }
    ulist.resize(keep);
    for (auto& x : hpiece) x.clear();
    const int hp = parallel_pieces((int64_t)ulist.size(), 4096, [&](int64_t lo, int64_t hi, int t) {
      std::vector<int32_t>& out = hpiece[(size_t)t];
      for (int64_t q = lo; q < hi; ++q) {
        const int32_t u = ulist[(size_t)q];
        for (int64_t j = g.off[u]; j < g.end[u]; ++j) {
          const int32_t e = g.eid[(size_t)j], w = g.nbr[(size_t)j];
          if (B.gone[(size_t)e]) continue;
          const bool inside = B.cnt[w] > 0;
          if (inside && w < u) continue;
          out.push_back(inside ? e : ~e);  // ~e: an external edge
        }
      }
    });
    H.ids.clear();
    H.flag.clear();
    for (int t = 0; t < hp; ++t)
      for (const int32_t x : hpiece[(size_t)t]) {
        H.ids.push_back(x >= 0 ? x : ~x);
        H.flag.push_back(x >= 0 ? 1 : 0);
      }
    R.st.candidates += 1;
    R.st.max_candidate = std::max(R.st.max_candidate, (int64_t)H.ids.size());
    int64_t found = 0;
    const int rc = (int64_t)H.ids.size() <= R.cap ? procedure5(B, H, k, &found)
                                                   : procedure9(B, H, k, lid, &found);
    if (rc) return rc;
    if (found > 0) R.st.kmax = k;
    if (verbose())
      fprintf(stderr, "truss_bottomup: k %d: candidate of %zu edges (procedure %d), %lld in Phi_k, %lld left, %.0f ms\n",
              k, H.ids.size(), (int64_t)H.ids.size() <= R.cap ? 5 : 9, (long long)found, (long long)B.left,
              ms_since(t0));
    g.compact(B.gone.data(), 0, B.left);
    k += 1;
  }
  return TRUSS_OK;
}

}  // namespace

}  // namespace truss

using namespace truss;

extern "C" {

int truss_bottomup_workspace_size(int64_t cap, size_t* bytes) {
  if (!bytes || cap < 1) {
    set_last_error(!bytes ? "bytes is NULL" : "the budget must be at least one edge");
    return TRUSS_E_INVAL;
  }
  if (cap > 0x7fffffffLL) {
    set_last_error("the budget exceeds INT32_MAX edges");
    return TRUSS_E_TOOBIG;
  }
  Arena a;
  a.counting = true;
  *bytes = device_layout(cap, a, nullptr);
  return TRUSS_OK;
}

}  // extern "C"

namespace {

int bottomup_entry(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const int32_t* first_part,
                   int64_t cap, int32_t* truss_out, int32_t* lower_out, const truss_options* opts,
                   truss_bottomup_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  const auto t0 = Clock::now();
  if (n < 0 || m < 0 || (m > 0 && (!src || !dst || !truss_out))) {
    set_last_error("invalid graph or NULL output");
    return TRUSS_E_INVAL;
  }
  if (m > 0x7fffffffLL) {
    set_last_error("m exceeds INT32_MAX");
    return TRUSS_E_TOOBIG;
  }
  int rc = validate_options(opts);
  if (rc) return rc;
  size_t need = 0;
  if ((rc = truss_bottomup_workspace_size(cap, &need))) return rc;
  if (!ws || ws_bytes < need) {
    set_last_error("workspace of %zu bytes given, %zu needed", ws_bytes, need);
    return TRUSS_E_WORKSPACE;
  }
  truss_bottomup_stats st;
  memset(&st, 0, sizeof(st));
  if (stats) *stats = st;
  HostGraph g;
  if ((rc = build_host_graph(n, m, src, dst, g))) return rc;
  Device D;
  D.cap = cap;
  Arena a;
  a.base = static_cast<char*>(ws);
  a.cap = ws_bytes;
  device_layout(cap, a, &D);
  const size_t c = (size_t)cap;
  void* pin = nullptr;
  if (hipHostMalloc(&pin, c * (4 * sizeof(int32_t) + 1), hipHostMallocDefault) != hipSuccess) {
    set_last_error("pinned staging of %zu bytes failed", c * (4 * sizeof(int32_t) + 1));
    return TRUSS_E_NOMEM;
  }
  D.h_src = static_cast<int32_t*>(pin);
  D.h_dst = D.h_src + c;
  D.h_out = D.h_dst + c;
  D.h_sup = D.h_out + c;
  D.h_frozen = reinterpret_cast<uint8_t*>(D.h_sup + c);
  D.lid.assign((size_t)n, -1);
  Run R{g, D, opts, (hipStream_t)stream, cap, truss_out, st};
  std::vector<int32_t> lb;
  std::vector<uint8_t> phi2;
  const auto t1 = Clock::now();
  if ((rc = lower_bounding(R, first_part, lb, phi2))) return rc;
  R.st.ms_lower = ms_since(t1);
  if (lower_out)
    for (int64_t e = 0; e < m; ++e) lower_out[e] = lb[(size_t)e];
  R.st.kstart = R.st.passes > 1 ? 2 : 3;
  const auto t2 = Clock::now();
  if ((rc = bottom_up(R, lb, phi2))) return rc;
  R.st.ms_bottomup = ms_since(t2);
  R.st.device_calls = D.calls;
  R.st.bytes_h2d = D.h2d;
  R.st.bytes_d2h = D.d2h;
  R.st.ms_total = ms_since(t0);
  if (R.st.kmax == 0 && m > 0) R.st.kmax = 2;
  if (verbose())
    fprintf(stderr, "truss_bottomup: %.0f ms in all: %.0f ms relabelling on the host, %.0f ms of copies and "
            "device runs over %lld subgraphs, the rest partitioning and extraction on the host\n",
            R.st.ms_total, D.ms_relabel, D.ms_device, (long long)D.calls);
  if (stats) *stats = R.st;
  return TRUSS_OK;
}

}  // namespace

extern "C" {

// The host side holds memory in proportion to the graph (its adjacency, the
// bounds, the candidate rows) and runs host threads: a failed allocation or
// thread start is reported as a status, never thrown across the C ABI.
int truss_bottomup(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const int32_t* first_part,
                   int64_t cap, int32_t* truss_out, int32_t* lower_out, const truss_options* opts,
                   truss_bottomup_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  try {
    return bottomup_entry(n, m, src, dst, first_part, cap, truss_out, lower_out, opts, stats, ws, ws_bytes, stream);
  } catch (const std::bad_alloc&) {
    set_last_error("host memory allocation failed");
    return TRUSS_E_NOMEM;
  } catch (const std::exception& e) {
    set_last_error("host error: %s", e.what());
    return TRUSS_E_INTERNAL;
  } catch (...) {
    set_last_error("host error");
    return TRUSS_E_INTERNAL;
  }
}

}  // extern "C"
