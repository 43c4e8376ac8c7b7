// Host-side interfaces between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/truss.h"

namespace truss {

// error magnitudes reported by device validation (smallest wins)
enum : int {
  kErrRowptr = 3, kErrRange = 4, kErrSelfloop = 5, kErrUnsorted = 6, kErrDup = 7, kErrAsym = 8
};
constexpr int kNoErr = 0x7fffffff;

// ---- bump allocator over the caller's workspace --------------------------------
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool counting = false;  // size query only
  template <typename T>
  T* take(size_t count) {
    size_t bytes = ((count * sizeof(T)) + 255) & ~size_t(255);
    size_t at = used;
    used += bytes;
    if (counting || base == nullptr) return nullptr;
    return reinterpret_cast<T*>(base + at);
  }
  bool overflow() const { return !counting && used > cap; }
};

// ---- scan (exclusive prefix sum) ---------------------------------------------
// out[i] = sum_{j<i} in[i]; out[count] = total (out has count+1 entries).
// tmp must hold scan_tmp_elems(count) elements of OutT.
size_t scan_tmp_elems(int64_t count);
void scan_exclusive_i32_to_i64(const int32_t* in, int64_t* out, int64_t count, int64_t* tmp,
                               hipStream_t s);
void scan_exclusive_i32_to_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* tmp,
                               hipStream_t s);

// ---- radix sort (LSD, 8-bit digits, stable) -------------------------------------
// Sorts (keys, vals) of length n by the low `bits` bits of the keys, passing
// back and forth between the two buffer pairs: returns true when the sorted
// result ended in keys_alt/vals_alt (an odd number of passes), false when it
// is in keys/vals.
size_t radix_tmp_elems(int64_t n);
bool radix_sort_u64(uint64_t* keys, int32_t* vals, uint64_t* keys_alt, int32_t* vals_alt,
                    int64_t n, int bits, int32_t* tmp, hipStream_t s);
bool radix_sort_u32(uint32_t* keys, int32_t* vals, uint32_t* keys_alt, int32_t* vals_alt,
                    int64_t n, int bits, int32_t* tmp, hipStream_t s);

// ---- the resident graph ---------------------------------------------------------
struct DevGraph {
  int32_t n = 0;
  int64_t m = 0;
  const int64_t* row_ptr = nullptr;  // n+1, symmetric CSR offsets
  int32_t* col = nullptr;            // 2m neighbours (rows ascending; compacted in place)
  int32_t* seid = nullptr;           // 2m edge id of each CSR entry
  int32_t* rlen = nullptr;           // n live row lengths (peeling)
  int32_t* eu = nullptr;             // m smaller-id endpoint
  int32_t* ev = nullptr;             // m larger-id endpoint
  int64_t* orow = nullptr;           // n+1 oriented CSR offsets
  int32_t* ocol = nullptr;           // m out-neighbours, ascending
  int32_t* oeid = nullptr;           // m edge ids of oriented entries
  int32_t* perm = nullptr;           // m canonical edge -> input index (EDGES only)
  int2* rtab = nullptr;               // row hash tables (neighbour, edge id), back to back
  const int64_t* rtoff = nullptr;    // n+1 offsets of the tables in rtab (slots; sizes are powers of two)
};

// Build: validation + canonical edge ids + symmetric and oriented CSR.
// Returns TRUSS_OK or a TRUSS_E_* code; syncs on the stream for the checks.
struct BuildBufs;
// relabel: vertices renumbered by (degree, id) inside the build (dg.perm then
// always maps the build's edges to the caller's); off where the caller reads
// vertex ids back out of dg
size_t build_workspace(const truss_graph* g, Arena& a, bool relabel = false);
int build_graph(const truss_graph* g, Arena& a, DevGraph& dg, int* d_err, hipStream_t s, bool relabel = false);

// Scheduling of the exact methods (the scheduler never changes results).
struct SupPlan {
  int sched = TRUSS_SCHED_HEURISTIC;  // effective scheduler for the bins
  int force = -1;                     // >= 0: this method (0 hash, 1 bsearch, 2 merge) in every bin
  const float* model = nullptr;       // (device) support model part when learned
};
struct PeelPlan {
  int sched = TRUSS_SCHED_HEURISTIC;  // effective scheduler for the levels
  int fix_bits = 0;                   // action bits fixed by the options (bit 0 probe, bit 1 mode)
  int fix_vals = 0;                   // their values
  const float* model = nullptr;       // (device) peeling model part when learned
  long long max_subrounds = 0;
  int grid_blocks = 0;
  int shape = TRUSS_SHAPE_AUTO;  // kernel shape (TRUSS_SHAPE_*)
  int first_level = 2;  // the first level peeled takes every live edge with sup <= first_level - 2
  int stop_level = 0;   // > 0: stop once the next level would exceed it (later edges keep no truss number)
  bool timed = true;    // time the kernel's launches with HIP events
};

// Support: sr[e].x = sup(e) for every canonical edge (sr must be zeroed inside).
// trace (nullable): receives each bin's method, features and time.
size_t support_workspace(const DevGraph& dg, Arena& a);
int compute_support(const DevGraph& dg, const SupPlan& plan, int2* sr, Arena& a, hipStream_t s,
                    truss_trace* trace);

// Peeling: truss[e] for every canonical edge; sr holds sup on entry.
struct PeelResult {
  int32_t kmax = 0, levels = 0;
  int64_t subrounds = 0, work = 0;
  int32_t launches = 0;
  int64_t heavy_rounds = 0;
  int64_t hist[6] = {0, 0, 0, 0, 0, 0};
  double phase_ms[6] = {0, 0, 0, 0, 0, 0};
  double kernel_ms = 0;  // time inside the persistent peeling kernel (all launches)
};
size_t peel_workspace(const DevGraph& dg, Arena& a);
int peel(const DevGraph& dg, const PeelPlan& plan, int2* sr, int32_t* truss_canon, Arena& a,
         PeelResult* res, hipStream_t s, truss_trace* trace);

// Upper bound psi(e) (Procedure 6) for every canonical edge; sr holds sup.
// h, ch: n entries of scratch each; psi: m entries; hs: 2m + n + 1 entries.
void compute_upper_bound(const DevGraph& dg, const int2* sr, int32_t* h, int32_t* ch, int32_t* psi, int32_t* hs,
                         hipStream_t s);

// Core numbers of every vertex (k-cores); syncs the stream once per peeling
// step.  core: n entries.  Workspace: core_workspace(n) after the build's.
size_t core_workspace(int32_t n, Arena& a);
int compute_core_numbers(const DevGraph& dg, int32_t* core, int32_t* cmax_out, Arena& a, hipStream_t s);
// Vertices of degree > 0 in the subgraph given by ms edges (su, sv) and
// their mean local clustering coefficient; sup[i] = triangles of edge i in the
// subgraph.  Syncs the stream.
int subgraph_vertex_stats(int32_t n, const int32_t* su, const int32_t* sv, const int32_t* sup, int64_t ms, Arena& a,
                          double* nv_out, double* cc_out, hipStream_t s);

// Algorithm 1 (comparator): truss[e] for every canonical edge; sr is scratch
// (support, removal round).  Workspace: cohen_workspace(m) after the build's.
struct CohenResult {
  int32_t kmax = 0, levels = 0;
  int64_t rounds = 0, support_work = 0, peel_work = 0;  // work: row entries merged
  double ms_support = 0, ms_peel = 0;
};
size_t cohen_workspace(int64_t m, Arena& a);
int cohen_decompose(const DevGraph& dg, int2* sr, int32_t* truss, Arena& a, CohenResult* res, hipStream_t s);

// One neighbourhood subgraph on the device, given as a device edge list of m
// edges over vertices 0..n-1 (validated like truss_decompose's input).
// Outputs are indexed like the edge list.  sup_out (nullable): sup(e) in the
// subgraph.  frozen (nullable, one byte per edge): a frozen edge is never
// peeled (its support is set out of reach before peeling).  Peeling starts at
// first_level and stops after stop_level (0: all levels); truss_out holds the
// level at which each peeled edge left, 0 for edges never peeled when
// stop_level > 0.  ws: subgraph_workspace(n, m) bytes.
struct SubgraphRun {
  const int32_t* src = nullptr;
  const int32_t* dst = nullptr;
  int32_t n = 0;
  int64_t m = 0;
  int32_t* truss_out = nullptr;
  int32_t* sup_out = nullptr;
  const uint8_t* frozen = nullptr;
  int first_level = 2;
  int stop_level = 0;
};
size_t subgraph_workspace(int32_t n, int64_t m);
int run_subgraph(const SubgraphRun& r, const truss_options* opts, void* ws, size_t ws_bytes, hipStream_t s);

void set_last_error(const char* fmt, ...);
int validate_options(const truss_options* o);  // TRUSS_OK or TRUSS_E_INVAL (message set)
int device_grid_blocks(const void* kernel, int block, size_t lds);

}  // namespace truss

#define TRUSS_HIP(call)                                                         \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::truss::set_last_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                              __FILE__, __LINE__);                              \
      return TRUSS_E_DEVICE;                                                    \
    }                                                                           \
  } while (0)
