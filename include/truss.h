/*
 * truss.h — C ABI of the MI355X truss-decomposition library (libtruss.so).
 *
 * Problem (Wang & Cheng, "Truss Decomposition in Massive Networks", PVLDB 2012):
 *   the input is an undirected, unweighted simple graph G = (V, E) (Section 2);
 *   sup(e) is the number of triangles of G that contain e (Definition 1);
 *   the k-truss T_k is the largest subgraph in which every edge lies in at least
 *   k-2 triangles of T_k (Definition 2); the truss number phi(e) is the largest k
 *   with e in T_k, and the k-class Phi_k is the set of edges with phi(e) = k
 *   (Definition 3).  Truss decomposition computes every k-truss, equivalently
 *   phi(e) for every edge, since T_k is the union of the classes Phi_j, j >= k
 *   (the problem statement of Section 2).
 *
 * Conventions shared by every entry point
 *   - Pointers marked (device) are HIP device pointers; (host) are host
 *     pointers.  The caller owns every buffer; the library never frees or
 *     keeps caller memory and holds no state between calls.  The library
 *     checks device pointers for NULL only: a host pointer, or a buffer
 *     shorter than an entry point states, is the caller's error and is not
 *     detected (the Python binding checks these before every call).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is ordered on it, and every call returns only after the
 *     stream has synchronised, so the returned status is final.
 *   - Vertex ids, supports, truss numbers and edge ids are int32; offsets,
 *     edge counts and triangle counts are int64.  m must not exceed INT32_MAX.
 *   - Duplicated edges and self-loops are rejected, not repaired.
 *   - Return value: TRUSS_OK (0) or a negative TRUSS_E_* code.  When the input
 *     violates several rules, the code of smallest magnitude among the
 *     TRUSS_E_ROWPTR .. TRUSS_E_ASYM group is reported.  Output contents are
 *     unspecified after an error.  truss_last_error() gives a message for the
 *     calling thread's last failure.
 *
 * Output indexing
 *   - TRUSS_FMT_EDGES: out[i] belongs to input pair (src[i], dst[i]).
 *   - TRUSS_FMT_CSR:   out[i] belongs to the i-th edge in canonical upper-CSR
 *     order: vertices u ascending, and within row u the neighbours v > u in
 *     row order.
 */
#ifndef TRUSS_H
#define TRUSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRUSS_VERSION 10000

/* ---- status codes ------------------------------------------------------- */
#define TRUSS_OK 0
#define TRUSS_E_INVAL (-1)      /* null pointer, negative size, bad option     */
#define TRUSS_E_TOOBIG (-2)     /* m > INT32_MAX                                */
#define TRUSS_E_ROWPTR (-3)     /* CSR row_ptr[0] != 0, decreasing, or != 2m    */
#define TRUSS_E_RANGE (-4)      /* vertex id outside [0, n)                     */
#define TRUSS_E_SELFLOOP (-5)   /* edge (v, v)                                  */
#define TRUSS_E_UNSORTED (-6)   /* CSR row not ascending                        */
#define TRUSS_E_DUP (-7)        /* edge listed twice (either orientation)       */
#define TRUSS_E_ASYM (-8)       /* CSR has (u,v) without (v,u)                  */
#define TRUSS_E_NOMEM (-9)      /* device (or bottom-up host) allocation failed */
#define TRUSS_E_WORKSPACE (-10) /* workspace missing or smaller than required   */
#define TRUSS_E_DEVICE (-11)    /* HIP runtime error                            */
#define TRUSS_E_INTERNAL (-12)  /* internal limit hit (e.g. sub-round cap)      */

/* ---- graph description -------------------------------------------------- */
#define TRUSS_FMT_EDGES 0 /* src[m], dst[m]: each undirected edge once, any orientation */
#define TRUSS_FMT_CSR 1   /* row_ptr[n+1], col[2m]: symmetric, rows strictly ascending  */

typedef struct truss_graph {
  int32_t n;              /* number of vertices (ids 0..n-1)                  */
  int32_t fmt;            /* TRUSS_FMT_EDGES or TRUSS_FMT_CSR                 */
  int64_t m;              /* number of undirected edges                       */
  const int32_t *src;     /* (device) EDGES: m endpoints                      */
  const int32_t *dst;     /* (device) EDGES: m endpoints                      */
  const int64_t *row_ptr; /* (device) CSR: n+1 offsets into col               */
  const int32_t *col;     /* (device) CSR: 2m neighbour ids                   */
} truss_graph;

/* ---- options ------------------------------------------------------------ */
/* Intersection strategy for support counting (Definition 1 by triangle
 * listing over the (degree, id) orientation; any exact method gives the same
 * sup, the choice only changes speed). */
#define TRUSS_SUP_AUTO 0    /* per vertex bin: LDS hash, global binary search   */
#define TRUSS_SUP_HASH 1    /* N+(u) staged in an LDS hash table                */
#define TRUSS_SUP_BSEARCH 2 /* binary search of N+(u) in global memory          */
#define TRUSS_SUP_MERGE 3   /* one wavefront merges N+(u) and N+(v) per edge    */

/* Frontier extraction for peeling. */
#define TRUSS_PEEL_AUTO 0   /* scheduler decides per level                      */
#define TRUSS_PEEL_SPARSE 1 /* worklist: enqueue an edge when its support drops to k-2 */
#define TRUSS_PEEL_DENSE 2  /* re-scan every live edge after each sub-round      */

/* Membership test (is (v, w) an edge of E_G?) while peeling (Algorithm 2). */
#define TRUSS_PROBE_AUTO 0    /* hash table                                      */
#define TRUSS_PROBE_HASH 1    /* hash table over the edges, as Section 3.2 keeps E_G */
#define TRUSS_PROBE_BSEARCH 2 /* binary search of the other endpoint's sorted row  */

/* Shape of the persistent peeling kernel (a tuning choice; results are the
 * same): one 1024-thread workgroup per compute unit with four walk entries in
 * flight per thread, or two workgroups per compute unit with two entries per
 * thread (more wavefronts to hide memory latency).  AUTO takes the wide shape
 * for graphs of at least 2^27 edges, where it measured faster. */
#define TRUSS_SHAPE_AUTO 0
#define TRUSS_SHAPE_NARROW 1
#define TRUSS_SHAPE_WIDE 2

/* Scheduler used for the AUTO decisions: the intersection strategy of each
 * support bin (vertices grouped by out-degree) and, for each peeling level, the
 * frontier mode and the membership probe.  Every choice computes the same
 * supports and truss numbers; only the speed differs. */
#define TRUSS_SCHED_PLAIN 0     /* fixed: merge support, dense sweep, bsearch probes */
#define TRUSS_SCHED_HEURISTIC 1 /* fixed thresholds                                  */
#define TRUSS_SCHED_LEARNED 2   /* MLP scores (see "Learned scheduler" below); the
                                   heuristic is used when the model is absent or
                                   malformed (truss_stats.sched_fallback = 1)       */

typedef struct truss_options {
  int32_t version;          /* must be TRUSS_VERSION                           */
  int32_t support_strategy; /* TRUSS_SUP_*                                      */
  int32_t peel_mode;        /* TRUSS_PEEL_*                                     */
  int32_t scheduler;        /* TRUSS_SCHED_*                                    */
  const float *model;       /* (device) learned-scheduler model (both parts, see
                               truss_sched_model_floats), or NULL             */
  int64_t max_subrounds;    /* > 0: fail with TRUSS_E_INTERNAL past this many  */
  int32_t grid_blocks;      /* > 0: persistent-kernel workgroups (tuning)      */
  int32_t peel_probe;       /* TRUSS_PROBE_*                                    */
  int32_t batch_block;      /* truss_batch: threads per workgroup (256, 512, 1024; 0 = 1024) */
  int32_t batch_ilp;        /* truss_batch: walk entries in flight per thread (1, 2, 4; 0 = 2) */
  int32_t model_floats;     /* floats readable at *model; > 0: a model whose two
                               part headers ask for more (or for a different
                               total) is rejected like a malformed one (the
                               heuristic runs, sched_fallback = 1); 0: the
                               caller vouches for the length              */
  int32_t peel_shape;       /* TRUSS_SHAPE_* (ignored when grid_blocks > 0: the
                               narrow shape runs with that grid)             */
  int32_t reserved[2];
} truss_options;

/* Filled when a stats pointer is passed (host). */
typedef struct truss_stats {
  int64_t n, m;
  int64_t triangles;        /* |triangles of G|                                  */
  int32_t kmax;             /* largest truss number (0 when m = 0)               */
  int32_t levels;           /* non-empty k-classes visited                       */
  int64_t subrounds;        /* frontier rounds over all levels                   */
  int64_t peel_work;        /* adjacency entries walked while peeling            */
  double ms_build;          /* validation + CSR build + orientation              */
  double ms_support;        /* support counting                                  */
  double ms_peel;           /* peeling                                           */
  double ms_total;
  int32_t sched_fallback;   /* 1 if the learned model was absent or invalid      */
  int32_t launches;         /* peeling kernel launches (one more per row compaction) */
  int64_t frontier_hist[6]; /* sub-rounds by frontier size: 1, 2-16, 17-256,
                               257-4096, 4097-65536, larger                      */
  int64_t heavy_rounds;     /* sub-rounds in which long walks were cut into pieces */
  double ms_phase[6];       /* peeling time by phase: live-list sweep, level start,
                               frontier rounds, unused, dense re-scan, unused     */
  double ms_peel_kernel;    /* time inside the persistent peeling kernel, all launches
                               (truss_batch: the batch kernel's graph launch)     */
  int64_t support_work;     /* truss_batch: row entries walked while counting support */
} truss_stats;

/* Fills *opts with defaults: AUTO strategies, heuristic scheduler. */
void truss_default_options(truss_options *opts);

/* Bytes of device workspace that truss_support / truss_decompose need for a
 * graph of this shape (only n, m and fmt are read).  bytes: (host). */
int truss_workspace_size(const truss_graph *g, const truss_options *opts, size_t *bytes);

/* Support of every edge (Definition 1).
 *   sup_out   (device) int32[m], indexed as in "Output indexing" above.
 *   triangles (host, nullable) receives |triangles of G| = sum(sup) / 3.
 *   ws, ws_bytes (device) workspace of at least truss_workspace_size bytes. */
int truss_support(const truss_graph *g, int32_t *sup_out, int64_t *triangles,
                  void *ws, size_t ws_bytes, void *stream);

/* Truss number of every edge (Definition 2; the k-classes of Definition 3).
 *   truss_out (device) int32[m], values in [2, k_max], indexed as above.
 *   opts (host, nullable) options; NULL = truss_default_options.
 *   stats (host, nullable) filled on success. */
int truss_decompose(const truss_graph *g, int32_t *truss_out, const truss_options *opts,
                    truss_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* Truss decomposition of many independent graphs at once.
 *   num_graphs  G >= 0.
 *   vtx_off     (host) int64[G+1]: graph g has vertices 0..vtx_off[g+1]-vtx_off[g]-1.
 *   edge_off    (host) int64[G+1], edge_off[0] = 0: graph g owns packed edges
 *               edge_off[g]..edge_off[g+1]-1.
 *   src, dst    (device) int32[edge_off[G]]: graph-local endpoint ids.
 *   truss_out   (device) int32[edge_off[G]]: truss number of each packed edge.
 * Triangles never cross graphs, so the result equals decomposing each graph
 * alone (Definitions 1-2 per graph).  Graphs with at most 2^21 edges and 2^22
 * vertices are decomposed by one persistent kernel, one workgroup per graph
 * (largest first); larger graphs take the device-wide path after it.  Each
 * graph is validated as an edge list; the failing graph of smallest index
 * decides the returned code (the other graphs' outputs are then unspecified).
 * The workspace holds the offsets, a scratch slot per concurrent workgroup
 * (about 8 bytes per vertex and 48 per edge of the largest batched graph, for
 * up to four workgroups per compute unit) and the device-wide path's workspace
 * for the largest remaining graph. */
int truss_batch_workspace_size(int32_t num_graphs, const int64_t *vtx_off, const int64_t *edge_off,
                               const truss_options *opts, size_t *bytes);
int truss_batch(int32_t num_graphs, const int64_t *vtx_off, const int64_t *edge_off,
                const int32_t *src, const int32_t *dst, int32_t *truss_out,
                const truss_options *opts, truss_stats *stats, void *ws, size_t ws_bytes,
                void *stream);

/* A reusable batch: the offsets are copied to the workspace once and the
 * device work (counter reset and the persistent kernel) is captured in a HIP
 * graph, replayed by each truss_batch_plan_run.  The plan refers to src, dst,
 * truss_out and ws, which must stay valid (and unchanged in shape) until
 * truss_batch_plan_destroy.  The caller owns the plan (host memory). */
typedef struct truss_batch_plan truss_batch_plan;
int truss_batch_plan_create(int32_t num_graphs, const int64_t *vtx_off, const int64_t *edge_off,
                            const int32_t *src, const int32_t *dst, int32_t *truss_out,
                            const truss_options *opts, void *ws, size_t ws_bytes, void *stream,
                            truss_batch_plan **plan);
int truss_batch_plan_run(truss_batch_plan *plan, truss_stats *stats, void *stream);
void truss_batch_plan_destroy(truss_batch_plan *plan);

/* Autotuner of the batch shape (threads per workgroup x walk entries in flight
 * per thread): every
 * built shape is timed on a size-stratified sample of at most 512 of the
 * batch's graphs, then the three fastest on the whole batch; the fastest of
 * those is returned in *best_block, *best_ilp (host) with its whole-batch
 * time in *best_ms (host, nullable).  Leaves valid truss numbers in truss_out. */
int truss_batch_autotune(int32_t num_graphs, const int64_t *vtx_off, const int64_t *edge_off,
                         const int32_t *src, const int32_t *dst, int32_t *truss_out,
                         const truss_options *opts, void *ws, size_t ws_bytes, void *stream,
                         int32_t *best_block, int32_t *best_ilp, float *best_ms);

/* ---- upper bound and top-down classes (Procedure 6, Algorithm 7) -------- */
/* psi(e) = min{sup(e), x_u, x_v} + 2 for every edge, where x_w is the largest x
 * such that at least x edges incident to w other than e have support >= x
 * (Procedure 6, the whole graph as one neighbourhood subgraph); phi(e) <= psi(e)
 * (Lemma 2).  psi_out (device) int32[m], indexed as in "Output indexing".  The
 * workspace is truss_workspace_size's. */
int truss_upper_bound(const truss_graph *g, int32_t *psi_out, void *ws, size_t ws_bytes, void *stream);

/* The top-t k-classes (Algorithm 7's output): truss_out[e] = phi(e) for every
 * edge with phi(e) > k_max - t, and 0 for the others; *kmin_out = max(2,
 * k_max - t + 1) and *kmax_out = k_max (host, nullable).  Only the subgraph of
 * edges with psi(e) >= k is decomposed, for k stepping down from max psi until
 * k <= k_max - t + 1 (by Lemma 2 that subgraph holds every k-truss).
 * stats (host, nullable): those of the last subgraph decomposition, with m =
 * its edge count and launches = the number of subgraphs decomposed. */
int truss_topdown_workspace_size(const truss_graph *g, const truss_options *opts, size_t *bytes);
int truss_topdown(const truss_graph *g, int32_t t, int32_t *truss_out, int32_t *kmin_out, int32_t *kmax_out,
                  const truss_options *opts, truss_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- Algorithm 1 (Section 3.1) as a comparator ------------------------------- */
/* The decomposition of Algorithm 1 (Cohen): sup(e) = |nb(u) ∩ nb(v)| by
 * merging the two full sorted rows; then for k = 3, 4, ... the
 * edges with sup < k-2 leave, each finding its triangles by merging the two
 * full rows again (removed edges are only marked) and decrementing the
 * two other edges of each.  truss_out (device) int32[m] as in
 * "Output indexing" — the same truss numbers as truss_decompose.  stats
 * (host, nullable): support_work and peel_work = row entries merged (for
 * each edge deg(u) + deg(v) once in each stage, i.e. the sum over vertices of
 * deg(v)^2 per stage), subrounds = frontier rounds, levels = non-empty
 * levels.  Workspace from truss_cohen_workspace_size.  This entry point is
 * the reference point of Algorithm 2's improvement (Table 3), not a fast path. */
int truss_cohen_workspace_size(const truss_graph *g, size_t *bytes);
int truss_cohen(const truss_graph *g, int32_t *truss_out, truss_stats *stats, void *ws, size_t ws_bytes,
                void *stream);

/* ---- k-cores and the cohesion comparison of Section 7 (Table 6) ---------- */
/* Core numbers: the c-core is the largest subgraph whose vertices all have
 * degree >= c; core(v) is the largest c whose c-core holds v (0 for isolated
 * vertices).  core_out (device) int32[n], indexed by vertex id in both
 * formats; *cmax_out (host, nullable) = max core(v).  The graph is validated
 * as for truss_decompose.  Workspace from truss_core_workspace_size; the
 * call synchronises the stream (the host steps the peeling levels). */
int truss_core_workspace_size(const truss_graph *g, size_t *bytes);
int truss_core_numbers(const truss_graph *g, int32_t *core_out, int32_t *cmax_out, void *ws, size_t ws_bytes,
                       void *stream);

/* Table 6's columns for T = the k_max-truss (the edges with phi(e) = k_max;
 * k_max is the largest truss number) and C = the c_max-core (the edges whose
 * two ends have core number c_max): vertex and edge counts, k_max and c_max,
 * and the mean local clustering coefficient over the subgraph's vertices,
 * where a vertex of degree d >= 2 in the subgraph with t triangles there has
 * coefficient t / (d (d - 1) / 2) and a vertex of degree 1 has 0.  Counts are
 * exact; the means are fp64 sums taken in a tree order (their last bits can
 * differ from a sequential sum). */
typedef struct truss_cohesion_stats {
  int64_t v_t, e_t;  /* |V_T|, |E_T|                                */
  int32_t kmax, pad0;
  double cc_t;       /* mean clustering coefficient of T            */
  int64_t v_c, e_c;  /* |V_C|, |E_C|                                */
  int32_t cmax, pad1;
  double cc_c;       /* mean clustering coefficient of C            */
} truss_cohesion_stats;

/* Runs the truss decomposition (opts as for truss_decompose, nullable), the
 * core numbers and the support of T and of C inside themselves.  out (host)
 * receives the statistics.  Synchronises the stream. */
int truss_cohesion_workspace_size(const truss_graph *g, size_t *bytes);
int truss_cohesion(const truss_graph *g, const truss_options *opts, truss_cohesion_stats *out, void *ws,
                   size_t ws_bytes, void *stream);

/* ---- bottom-up decomposition of a graph in host memory (Section 5) ------- */
/* Host memory holds the graph, the bounds and the results (the paper's disk);
 * the device holds one neighbourhood subgraph NS(P) (Definition 4) at a time
 * (the paper's main memory), of at most `cap` edges.  LowerBounding
 * (Algorithm 3) partitions the vertices of the shrinking graph into parts
 * whose neighbourhood subgraphs fit, decomposes each on the device and keeps
 * the largest local truss number of every edge as its lower bound (Lemma 1);
 * Algorithm 4 then computes Phi_3, Phi_4, ... from the candidate subgraphs
 * NS(U_k) by Procedure 5, or by Procedure 9 when a candidate exceeds cap.
 * Parts are grown breadth-first from the smallest-id unplaced vertex, a
 * vertex weighing its degree, a part's weight at most cap.  Only the first
 * pass of Algorithm 3 sees the input graph, so only it outputs internal edges
 * of support 0 as Phi_2; Algorithm 4 starts at k = 2 after a second pass. */
typedef struct truss_bottomup_stats {
  int64_t passes;        /* LowerBounding passes (Algorithm 3)                        */
  int64_t subgraphs;     /* neighbourhood subgraphs decomposed by LowerBounding       */
  int64_t phi2_edges;    /* |Phi_2| output by LowerBounding                           */
  int64_t gnew_edges;    /* |G_new|                                                   */
  int64_t max_subgraph;  /* most edges in one neighbourhood subgraph of LowerBounding  */
  int64_t candidates;    /* candidate subgraphs NS(U_k) (Algorithm 4)                 */
  int64_t proc9_calls;   /* candidates above cap (Procedure 9)                        */
  int64_t proc9_scans;   /* partitions of H' made by Procedure 9                      */
  int64_t max_candidate; /* most edges in a candidate subgraph                        */
  int64_t device_calls;  /* subgraphs run on the device                               */
  int64_t bytes_h2d, bytes_d2h;
  int32_t kstart, kmax;  /* first k of Algorithm 4; largest truss number              */
  double ms_lower, ms_bottomup, ms_total;
} truss_bottomup_stats;

/* Device workspace for a budget of cap edges per subgraph (1 <= cap <= INT32_MAX). */
int truss_bottomup_workspace_size(int64_t cap, size_t *bytes);
/* src, dst (host): the m edges over vertices 0..n-1 (validated: ids in range,
 * no self-loop, no pair twice).  first_part (host, nullable): part id in [0, n)
 * of every vertex with an edge, for the first LowerBounding pass instead of the
 * grown parts (each part's neighbourhood subgraph must fit in cap).
 * truss_out (host) int32[m]: phi(e) by input index; lower_out (host,
 * nullable) int32[m]: the bound from LowerBounding.  opts as for
 * truss_decompose (nullable).  ws (device): truss_bottomup_workspace_size
 * bytes.  Synchronises the stream; allocates pinned host staging of 17 bytes
 * per budget edge for the call, and host memory in proportion to m (the
 * adjacency, the bounds, the candidate rows), used by up to 16 host threads.
 * TRUSS_E_WORKSPACE when a vertex alone, a given part, or every part of a
 * pass leaves no internal edge within cap; TRUSS_E_NOMEM when host memory
 * runs out (TRUSS_E_INTERNAL if a host thread cannot start). */
int truss_bottomup(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *first_part,
                   int64_t cap, int32_t *truss_out, int32_t *lower_out, const truss_options *opts,
                   truss_bottomup_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ---- tracing: the per-decision record behind the learned scheduler ----- */
/* Peeling level actions: bit 0 = probe (0 hash table, 1 binary search),
 * bit 1 = frontier mode (0 sparse worklist, 1 dense re-scan). */
#define TRUSS_SCHED_PEEL_F 8 /* features of a level, taken when its first frontier is known:
                                log2(1+live edges), log2(1+|F_0|), |F_0|/live edges,
                                log2(k), log2(1+W_0), log2(1+W_0/|F_0|) where W_0 is the
                                summed shorter live row length over F_0,
                                live edges / row entries kept, log2(1+sub-rounds of the
                                previous level) */
#define TRUSS_SCHED_PEEL_A 4
/* Support bin actions: 0 LDS hash, 1 binary search, 2 merge (hash is not
 * available to the last bin, whose out-neighbourhoods exceed the LDS).  The
 * learned scheduler departs from the heuristic's method for a bin only when
 * the network predicts it at least 2^0.25 times faster. */
#define TRUSS_SCHED_SUP_BINS 4 /* out-degree 2..64, 65..1024, 1025..4096, larger */
#define TRUSS_SCHED_SUP_F 6  /* log2(1+vertices), log2(1+sum d), log2(1+sum d^2),
                                log2(1+mean d), log2(1+m), log2(1+sum d^2 / sum d) */
#define TRUSS_SCHED_SUP_A 3

typedef struct truss_trace {
  int32_t level_cap;      /* (in) rows available in the level arrays (may be 0)        */
  int32_t levels;         /* (out) levels recorded: min(levels peeled, level_cap)      */
  float *level_feat;      /* (device) level_cap x TRUSS_SCHED_PEEL_F raw features      */
  float *level_ms;        /* (device) level_cap: time from the level's decision to its
                             last sub-round's end (same state at that point under
                             every action, so times of different runs compare)        */
  int32_t *level_action;  /* (device) level_cap: action taken                          */
  int32_t sup_action[TRUSS_SCHED_SUP_BINS];              /* (out) action per bin       */
  float sup_feat[TRUSS_SCHED_SUP_BINS][TRUSS_SCHED_SUP_F]; /* (out) raw features      */
  float sup_ms[TRUSS_SCHED_SUP_BINS];                    /* (out) time of each bin     */
} truss_trace;

/* truss_decompose that also records every scheduling decision, its features
 * and its time (trace: host struct; its arrays are device memory).  The
 * extra timing events make it slightly slower than truss_decompose. */
int truss_decompose_traced(const truss_graph *g, int32_t *truss_out, const truss_options *opts,
                           truss_stats *stats, truss_trace *trace, void *ws, size_t ws_bytes,
                           void *stream);

/* ---- decomposition without allocation ------------------------------------ */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * decomposition as truss_decompose (same kernels, same output), with its
 * scratch taken from a fixed device array of TRUSS_NOALLOC_SCRATCH_BYTES
 * bytes instead of a caller workspace.  Each GPU the library runs on holds
 * one such array from its first call on that GPU until the process ends.
 *   g, truss_out, opts: as for truss_decompose.
 *   stats (host, nullable): as for truss_decompose, except that every time
 *     field is 0 (no timing events are created).
 * Graphs whose truss_workspace_size exceeds the array are refused with
 * TRUSS_E_WORKSPACE before any device work.  The call allocates nothing: no
 * hipMalloc, hipFree, events or streams.  Every call on one GPU uses that
 * GPU's array and leaves its contents behind; calls that overlap on one GPU
 * (two threads, or two streams of one thread) race and give undefined
 * results. */
#define TRUSS_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int truss_decompose_noalloc(const truss_graph *g, int32_t *truss_out, const truss_options *opts,
                            truss_stats *stats, void *stream);

/* ---- learned scheduler: the network and its training ----------------- */
/* Two-layer perceptron y = W2 tanh(W1 x + b1) + b2 in fp32.  params packs
 * W1[H][F], b1[H], W2[O][H], b2[O], row-major; X is B x F and Y is B x O,
 * row-major.  Limits: 1 <= F <= 16, 1 <= H <= 64, 1 <= O <= 8, B >= 1. */
#define TRUSS_MLP_MAX_F 16
#define TRUSS_MLP_MAX_H 64
#define TRUSS_MLP_MAX_O 8

/* Number of floats in params, or TRUSS_E_INVAL. */
int truss_mlp_param_count(int32_t F, int32_t H, int32_t O);
int truss_mlp_workspace_size(int32_t F, int32_t H, int32_t O, int32_t B, size_t *bytes);
/* Y = network(X). */
int truss_mlp_forward(const float *params, int32_t F, int32_t H, int32_t O, const float *X,
                      int32_t B, float *Y, void *ws, size_t ws_bytes, void *stream);
/* grad = d(sum_{r,o} dY[r,o] * Y[r,o]) / d params (the vector-Jacobian product). */
int truss_mlp_backward(const float *params, int32_t F, int32_t H, int32_t O, const float *X,
                       int32_t B, const float *dY, float *grad, void *ws, size_t ws_bytes,
                       void *stream);
/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, step size
 * lr) on the loss L = sum_{r,o} Wt[r,o] (Y[r,o] - T[r,o])^2 / sum Wt, where Y
 * = network(X).  params, adam_m, adam_v (device, param_count floats each) are
 * updated in place; step0 is the number of Adam steps already taken (bias
 * correction).  loss (host, nullable) receives L after the last step.  The sum
 * of Wt must be positive. */
int truss_mlp_train(float *params, float *adam_m, float *adam_v, int32_t F, int32_t H, int32_t O,
                    const float *X, const float *T, const float *Wt, int32_t B, int32_t steps,
                    int32_t step0, float lr, float *loss, void *ws, size_t ws_bytes, void *stream);

/* The model passed in truss_options.model is two parts back to back, peeling
 * first, then support.  A part is [1205, F, H, O, mu[F], isd[F], params] in
 * floats; the network sees (x - mu) * isd and each output estimates log2 of
 * the action's time in ms.  kind: 0 = peeling, 1 = support. */
int truss_sched_part_floats(int32_t kind, int32_t H);
int truss_sched_model_floats(int32_t H);
int truss_sched_train_workspace_size(int32_t kind, int32_t H, int32_t B, size_t *bytes);
/* Fits one model part on B traced decisions: X (device) B x F raw features,
 * T_ms (device) B x A times of every action (<= 0 where not measured).  Sets
 * the normalisation from X, initialises the weights from `seed`, and trains
 * with a weighted log2-time loss in which a row's weight grows with its
 * slowest measured time.  part (device) receives truss_sched_part_floats. */
int truss_sched_train(int32_t kind, const float *X, const float *T_ms, int32_t B, int32_t H,
                      int32_t steps, float lr, uint64_t seed, float *part, float *loss,
                      void *ws, size_t ws_bytes, void *stream);

const char *truss_strerror(int code);
const char *truss_last_error(void);
int truss_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TRUSS_H */
