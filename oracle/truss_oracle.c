/*
 * Serial CPU oracle for truss decomposition (Wang & Cheng, "Truss Decomposition
 * in Massive Networks", PVLDB 2012).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library includes, links or
 * calls this file; it shares no header, table or helper with it.  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * What it computes (all integer, exact):
 *   - validation of a simple undirected graph given as an edge list or as a
 *     symmetric CSR (Section 2: undirected, unweighted, simple graphs);
 *   - sup(e), the number of triangles containing e (Definition 1), by two
 *     independent routines:
 *       (i)  oracle_support_def: |nb(u) ∩ nb(v)| for every edge by a two-pointer
 *            merge of the full sorted adjacency lists (the support of Algorithm 1);
 *       (ii) oracle_support_fwd: every triangle listed once through the
 *            degree orientation (deg, id) and counted on its three edges — the
 *            in-memory triangle counting Algorithm 2 starts from
 *            (Section 3.2);
 *   - phi(e), the truss number (Definition 2 and the text after it), by
 *     Algorithm 2 (Section 3.2): bin sort of edges by support, then repeatedly
 *     take the lowest-support edge e=(u,v) while sup(e) <= k-2, walk the
 *     smaller-degree endpoint's neighbours w, and for each live triangle
 *     decrement (u,w) and (v,w) and re-bin them; e joins the k-class.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - Algorithm 2 decrements the two other edges unconditionally.  Here an edge whose
 *     support is already <= k-2 is not decremented: it is removed at this level
 *     anyway (so its truss number is k either way) and the guard keeps the bin
 *     array sorted without moving an edge left of the pointer.
 *   - "w in nb(u)" and "(v,w) in E_G" are read on the current graph: both
 *     (u,w) and (v,w) must not have been removed yet.
 *   - The endpoint whose neighbours are walked is chosen by original degree;
 *     ties go to the smaller id.
 *   - Edge identity: edge i is the i-th input pair; outputs are per input pair.
 *
 * Error codes are returned as negative numbers; when several violations exist
 * the one of smallest magnitude is reported.  Codes (magnitudes):
 *   1 INVAL, 2 TOOBIG, 3 ROWPTR, 4 RANGE, 5 SELFLOOP, 6 UNSORTED, 7 DUP, 8 ASYM.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum {
  OR_OK = 0,
  OR_INVAL = 1,
  OR_TOOBIG = 2,
  OR_ROWPTR = 3,
  OR_RANGE = 4,
  OR_SELFLOOP = 5,
  OR_UNSORTED = 6,
  OR_DUP = 7,
  OR_ASYM = 8,
  OR_NOMEM = 9
};

/* ------------------------------------------------------------------------- */
/* Adjacency: for every vertex its neighbours sorted by id, with edge ids.    */
/* ------------------------------------------------------------------------- */
typedef struct {
  int32_t n;
  int64_t m;
  int64_t *off;  /* n+1 */
  int32_t *nbr;  /* 2m, sorted within each vertex */
  int64_t *eid;  /* 2m, edge index of (v, nbr) */
} adj_t;

typedef struct { int32_t w; int64_t e; } pair_t;

static int cmp_pair(const void *a, const void *b) {
  int32_t x = ((const pair_t *)a)->w, y = ((const pair_t *)b)->w;
  return (x > y) - (x < y);
}

static void adj_free(adj_t *g) {
  free(g->off); free(g->nbr); free(g->eid);
  memset(g, 0, sizeof(*g));
}

/* Build sorted adjacency lists from a validated edge list. */
static int adj_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, adj_t *g) {
  g->n = n; g->m = m;
  g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  g->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m + 1));
  g->eid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m + 1));
  int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  pair_t *tmp = NULL;
  if (!g->off || !g->nbr || !g->eid || !fill) { free(fill); adj_free(g); return -OR_NOMEM; }
  for (int64_t i = 0; i < m; ++i) { g->off[src[i] + 1]++; g->off[dst[i] + 1]++; }
  for (int32_t v = 0; v < n; ++v) g->off[v + 1] += g->off[v];
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = src[i], v = dst[i];
    int64_t pu = g->off[u] + fill[u]++, pv = g->off[v] + fill[v]++;
    g->nbr[pu] = v; g->eid[pu] = i;
    g->nbr[pv] = u; g->eid[pv] = i;
  }
  free(fill);
  int64_t maxdeg = 0;
  for (int32_t v = 0; v < n; ++v) {
    int64_t d = g->off[v + 1] - g->off[v];
    if (d > maxdeg) maxdeg = d;
  }
  tmp = (pair_t *)malloc(sizeof(pair_t) * (size_t)(maxdeg + 1));
  if (!tmp) { adj_free(g); return -OR_NOMEM; }
  for (int32_t v = 0; v < n; ++v) {
    int64_t b = g->off[v], d = g->off[v + 1] - b;
    for (int64_t j = 0; j < d; ++j) { tmp[j].w = g->nbr[b + j]; tmp[j].e = g->eid[b + j]; }
    qsort(tmp, (size_t)d, sizeof(pair_t), cmp_pair);
    for (int64_t j = 0; j < d; ++j) { g->nbr[b + j] = tmp[j].w; g->eid[b + j] = tmp[j].e; }
  }
  free(tmp);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Validation (Section 2: simple undirected graph).                            */
/* ------------------------------------------------------------------------- */
static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return (x > y) - (x < y);
}

/* Edge list: ids in [0,n), no self-loop, no pair given twice in either
 * orientation.  Returns 0 or -code. */
int oracle_validate_edges(int32_t n, int64_t m, const int32_t *src, const int32_t *dst) {
  if (n < 0 || m < 0) return -OR_INVAL;
  if (m > 0 && (!src || !dst)) return -OR_INVAL;
  if (m > INT32_MAX) return -OR_TOOBIG;
  int worst = 0;
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = src[i], v = dst[i];
    int c = 0;
    if (u < 0 || u >= n || v < 0 || v >= n) c = OR_RANGE;
    else if (u == v) c = OR_SELFLOOP;
    if (c && (!worst || c < worst)) worst = c;
  }
  if (worst) return -worst;
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m + 1));
  if (!key) return -OR_NOMEM;
  for (int64_t i = 0; i < m; ++i) {
    uint64_t a = (uint64_t)(src[i] < dst[i] ? src[i] : dst[i]);
    uint64_t b = (uint64_t)(src[i] < dst[i] ? dst[i] : src[i]);
    key[i] = (a << 32) | b;
  }
  qsort(key, (size_t)m, sizeof(uint64_t), cmp_u64);
  for (int64_t i = 1; i < m; ++i)
    if (key[i] == key[i - 1]) { free(key); return -OR_DUP; }
  free(key);
  return OR_OK;
}

/* Symmetric CSR: row_ptr[0]=0, non-decreasing, row_ptr[n]=2m; neighbours in
 * range, no self-loop, strictly ascending per row; (u,v) present iff (v,u). */
int oracle_validate_csr(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col) {
  if (n < 0 || m < 0 || !row_ptr) return -OR_INVAL;
  if (m > 0 && !col) return -OR_INVAL;
  if (m > INT32_MAX) return -OR_TOOBIG;
  if (row_ptr[0] != 0 || row_ptr[n] != 2 * m) return -OR_ROWPTR;
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return -OR_ROWPTR;
  int worst = 0;
  for (int32_t v = 0; v < n; ++v) {
    for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
      int32_t w = col[j];
      int c = 0;
      if (w < 0 || w >= n) c = OR_RANGE;
      else if (w == v) c = OR_SELFLOOP;
      else if (j + 1 < row_ptr[v + 1]) {
        if (col[j + 1] == w) c = OR_DUP;
        else if (col[j + 1] < w && col[j + 1] >= 0) c = OR_UNSORTED;
      }
      if (c && (!worst || c < worst)) worst = c;
    }
  }
  if (worst) return -worst;
  /* every (v,w) needs (w,v): binary search in the sorted row of w */
  for (int32_t v = 0; v < n; ++v) {
    for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
      int32_t w = col[j];
      int64_t lo = row_ptr[w], hi = row_ptr[w + 1];
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (lo >= row_ptr[w + 1] || col[lo] != v) return -OR_ASYM;
    }
  }
  return OR_OK;
}

/* Canonical upper-CSR edge list of a symmetric CSR: for u ascending, the
 * neighbours v > u in row order.  src/dst must hold m entries. */
int oracle_csr_to_edges(int32_t n, int64_t m, const int64_t *row_ptr, const int32_t *col,
                        int32_t *src, int32_t *dst) {
  int64_t k = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
      if (col[j] > u) {
        if (k >= m) return -OR_ASYM;
        src[k] = u; dst[k] = col[j]; ++k;
      }
  return k == m ? OR_OK : -OR_ASYM;
}

/* ------------------------------------------------------------------------- */
/* Support (Definition 1).                                                   */
/* ------------------------------------------------------------------------- */

/* (i) |nb(u) ∩ nb(v)| for every edge, by merging the two full sorted lists
 * (the support computation of Algorithm 1).  O(sum_v deg(v)^2). */
int oracle_support_def(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       int32_t *sup, int64_t *triangles) {
  adj_t g;
  int rc = adj_build(n, m, src, dst, &g);
  if (rc) return rc;
  int64_t total = 0;
  for (int64_t i = 0; i < m; ++i) {
    int32_t u = src[i], v = dst[i];
    int64_t a = g.off[u], ae = g.off[u + 1], b = g.off[v], be = g.off[v + 1];
    int32_t c = 0;
    while (a < ae && b < be) {
      if (g.nbr[a] < g.nbr[b]) ++a;
      else if (g.nbr[a] > g.nbr[b]) ++b;
      else { ++c; ++a; ++b; }
    }
    sup[i] = c;
    total += c;
  }
  if (triangles) *triangles = total / 3;
  adj_free(&g);
  return OR_OK;
}

/* Vertex order used for orientation: by degree, ties by id. */
static int before(const adj_t *g, int32_t a, int32_t b) {
  int64_t da = g->off[a + 1] - g->off[a], db = g->off[b + 1] - g->off[b];
  return da < db || (da == db && a < b);
}

/* (ii) forward triangle listing: orient every edge from the earlier to the
 * later endpoint in (deg, id) order; each triangle a<b<c is found once as
 * c in N+(a) ∩ N+(b) for the edge a->b and adds 1 to its three edges. */
int oracle_support_fwd(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       int32_t *sup, int64_t *triangles) {
  adj_t g;
  int rc = adj_build(n, m, src, dst, &g);
  if (rc) return rc;
  /* out-lists: the later neighbours of each vertex, kept in id order */
  int64_t *ooff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *onbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  int64_t *oeid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
  if (!ooff || !onbr || !oeid) { free(ooff); free(onbr); free(oeid); adj_free(&g); return -OR_NOMEM; }
  for (int32_t u = 0; u < n; ++u) {
    ooff[u + 1] = ooff[u];
    for (int64_t j = g.off[u]; j < g.off[u + 1]; ++j)
      if (before(&g, u, g.nbr[j])) {
        onbr[ooff[u + 1]] = g.nbr[j];
        oeid[ooff[u + 1]] = g.eid[j];
        ooff[u + 1]++;
      }
  }
  memset(sup, 0, sizeof(int32_t) * (size_t)m);
  int64_t tri = 0;
  for (int32_t a = 0; a < n; ++a) {
    for (int64_t j = ooff[a]; j < ooff[a + 1]; ++j) {
      int32_t b = onbr[j];
      int64_t eab = oeid[j];
      int64_t x = ooff[a], xe = ooff[a + 1], y = ooff[b], ye = ooff[b + 1];
      while (x < xe && y < ye) {
        if (onbr[x] < onbr[y]) ++x;
        else if (onbr[x] > onbr[y]) ++y;
        else {
          sup[eab]++; sup[oeid[x]]++; sup[oeid[y]]++;
          ++tri; ++x; ++y;
        }
      }
    }
  }
  if (triangles) *triangles = tri;
  free(ooff); free(onbr); free(oeid);
  adj_free(&g);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Truss numbers by Algorithm 2 (Section 3.2).                                */
/* ------------------------------------------------------------------------- */

/* Position of w in the sorted neighbour list of v, or -1. */
static int64_t find_nbr(const adj_t *g, int32_t v, int32_t w) {
  int64_t lo = g->off[v], hi = g->off[v + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->nbr[mid] < w) lo = mid + 1; else hi = mid;
  }
  return (lo < g->off[v + 1] && g->nbr[lo] == w) ? lo : -1;
}

/* Edges kept sorted by current support (the bin sort of Algorithm 2):
 * order[] lists the edges by support, pos[e] is e's place in it and start[s]
 * the first place holding support s.  Lowering an edge's support by one swaps
 * it with the first edge of its bin and moves that bin's start past it, so
 * order[] stays sorted. */
typedef struct {
  int64_t *order, *pos, *start;
  int32_t *sup;
} bins_t;

static void bins_free(bins_t *b) {
  free(b->order); free(b->pos); free(b->start);
  memset(b, 0, sizeof(*b));
}

static int bins_build(int64_t m, int32_t *sup, bins_t *b) {
  int32_t maxsup = 0;
  for (int64_t i = 0; i < m; ++i) if (sup[i] > maxsup) maxsup = sup[i];
  b->sup = sup;
  b->start = (int64_t *)calloc((size_t)maxsup + 2, sizeof(int64_t));
  b->order = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
  b->pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)maxsup + 1));
  if (!b->start || !b->order || !b->pos || !fill) { free(fill); bins_free(b); return -OR_NOMEM; }
  for (int64_t i = 0; i < m; ++i) b->start[sup[i] + 1]++;
  for (int32_t s = 0; s <= maxsup; ++s) b->start[s + 1] += b->start[s];
  for (int32_t s = 0; s <= maxsup; ++s) fill[s] = b->start[s];
  for (int64_t i = 0; i < m; ++i) { b->pos[i] = fill[sup[i]]++; b->order[b->pos[i]] = i; }
  free(fill);
  return OR_OK;
}

static void bins_lower(bins_t *b, int64_t f) {
  const int32_t s = b->sup[f];
  const int64_t here = b->pos[f], first = b->start[s];
  const int64_t other = b->order[first];
  b->order[first] = f; b->pos[f] = first;
  b->order[here] = other; b->pos[other] = here;
  b->start[s]++;
  b->sup[f] = s - 1;
}

/* Removes e = (u, v) at level k: every triangle (u, v, w) whose other two
 * edges are still present loses e, so each of those edges loses one support
 * -- unless its support is already at most k - 2 (it leaves at this level
 * whatever happens; the guard keeps it from moving before the current
 * position of the bin order).  The triangles are found from the endpoint
 * that comes first in (degree, id) order, each w looked up in the other's
 * sorted list (Section 3.2's choice of the smaller-degree endpoint). */
static void remove_edge(const adj_t *g, bins_t *b, unsigned char *removed, const int32_t *src,
                        const int32_t *dst, int64_t e, int32_t k) {
  int32_t near = src[e], far = dst[e];
  if (!before(g, near, far)) { int32_t t = near; near = far; far = t; }
  for (int64_t j = g->off[near]; j < g->off[near + 1]; ++j) {
    const int32_t w = g->nbr[j];
    const int64_t e1 = g->eid[j];
    if (w == far || removed[e1]) continue;
    const int64_t q = find_nbr(g, far, w);
    if (q < 0 || removed[g->eid[q]]) continue;
    const int64_t e2 = g->eid[q];
    if (b->sup[e1] > k - 2) bins_lower(b, e1);
    if (b->sup[e2] > k - 2) bins_lower(b, e2);
  }
  removed[e] = 1;
}

/* Truss numbers by Algorithm 2 (Section 3.2): supports from triangle
 * counting, edges in bin order, and a level k that rises whenever the next
 * edge in that order has support above k - 2; an edge taken at level k has
 * truss number k.  phi[i] for every input edge i; kmax_out (nullable) gets
 * the largest phi (0 when m = 0). */
int oracle_truss(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 int32_t *phi, int32_t *kmax_out) {
  if (kmax_out) *kmax_out = 0;
  if (m == 0) return OR_OK;
  int32_t *sup = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  if (!sup) return -OR_NOMEM;
  int rc = oracle_support_fwd(n, m, src, dst, sup, NULL);
  if (rc) { free(sup); return rc; }
  adj_t g;
  rc = adj_build(n, m, src, dst, &g);
  if (rc) { free(sup); return rc; }
  bins_t b;
  rc = bins_build(m, sup, &b);
  unsigned char *removed = (unsigned char *)calloc((size_t)m, 1);
  if (rc || !removed) {
    if (!rc) bins_free(&b);
    free(removed); free(sup); adj_free(&g);
    return -OR_NOMEM;
  }
  int32_t k = 2;
  for (int64_t p = 0; p < m;) {
    const int64_t e = b.order[p];
    if (b.sup[e] > k - 2) { ++k; continue; }
    remove_edge(&g, &b, removed, src, dst, e, k);
    phi[e] = k;
    ++p;
  }
  if (kmax_out) *kmax_out = k;
  bins_free(&b); free(removed); free(sup);
  adj_free(&g);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Upper bound of the truss number (Procedure 6, Lemma 2).                   */
/* ------------------------------------------------------------------------- */
/* For an end vertex w of e, x_w is the largest x such that at least x edges
 * incident to w, other than e, have support at least x; then
 * psi(e) = min{sup(e), x_u, x_v} + 2.  The whole graph is taken as one
 * neighbourhood subgraph, so every edge is internal.  Per vertex the incident
 * supports are sorted in descending order; the number of edges other than e
 * with support >= x is a binary search (minus e itself when sup(e) >= x), and
 * x_w is the last x for which that number is >= x (it never increases with x),
 * found by a second binary search over x in [0, deg(w) - 1]. */
static int cmp_desc_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x < y) - (x > y);
}

/* entries >= x in the descending array s[0..d) */
static int64_t count_at_least(const int32_t *s, int64_t d, int32_t x) {
  int64_t lo = 0, hi = d;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (s[mid] >= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

int oracle_upper_bound(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *sup,
                       int32_t *psi) {
  adj_t g;
  int rc = adj_build(n, m, src, dst, &g);
  if (rc) return rc;
  int64_t maxdeg = 0;
  for (int32_t v = 0; v < n; ++v)
    if (g.off[v + 1] - g.off[v] > maxdeg) maxdeg = g.off[v + 1] - g.off[v];
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxdeg + 1));
  if (!s) { adj_free(&g); return -OR_NOMEM; }
  for (int64_t i = 0; i < m; ++i) psi[i] = sup[i];
  for (int32_t w = 0; w < n; ++w) {
    int64_t b = g.off[w], d = g.off[w + 1] - b;
    for (int64_t j = 0; j < d; ++j) s[j] = sup[g.eid[b + j]];
    qsort(s, (size_t)d, sizeof(int32_t), cmp_desc_i32);
    for (int64_t j = 0; j < d; ++j) {
      int64_t e = g.eid[b + j];
      int64_t lo = 0, hi = d - 1;
      while (lo < hi) {
        int64_t x = (lo + hi + 1) / 2;
        int64_t c = count_at_least(s, d, (int32_t)x) - (sup[e] >= x ? 1 : 0);
        if (c >= x) lo = x; else hi = x - 1;
      }
      if ((int32_t)lo < psi[e]) psi[e] = (int32_t)lo;
    }
  }
  for (int64_t i = 0; i < m; ++i) psi[i] += 2;
  free(s);
  adj_free(&g);
  return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Core numbers and the cohesion statistics of the k_max-truss and the       */
/* c_max-core (Section 7, Table 6).                                          */
/* ------------------------------------------------------------------------- */
/* core[v] = the largest c such that v lies in the c-core (the largest
 * subgraph with minimum degree >= c).  Vertices are kept in buckets by
 * current degree and taken in order of increasing degree; taking v removes
 * its edges, which lowers each later neighbour's degree by one and moves it
 * one bucket down (the bucket method of Batagelj and Zaversnik, 2003). */
int oracle_core_numbers(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *core,
                        int32_t *cmax_out) {
  adj_t g;
  int rc = adj_build(n, m, src, dst, &g);
  if (rc) return rc;
  int64_t md = 0;
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *vert = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  if (!deg || !pos || !vert) { free(deg); free(pos); free(vert); adj_free(&g); return -OR_NOMEM; }
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = g.off[v + 1] - g.off[v];
    if (deg[v] > md) md = deg[v];
  }
  int64_t *bin = (int64_t *)calloc((size_t)md + 2, sizeof(int64_t));
  if (!bin) { free(deg); free(pos); free(vert); adj_free(&g); return -OR_NOMEM; }
  for (int32_t v = 0; v < n; ++v) bin[deg[v]]++;
  for (int64_t d = 0, start = 0; d <= md; ++d) {  /* bucket starts */
    int64_t c = bin[d];
    bin[d] = start;
    start += c;
  }
  for (int32_t v = 0; v < n; ++v) {
    pos[v] = bin[deg[v]]++;
    vert[pos[v]] = v;
  }
  for (int64_t d = md; d > 0; --d) bin[d] = bin[d - 1];
  bin[0] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t v = vert[i];
    for (int64_t j = g.off[v]; j < g.off[v + 1]; ++j) {
      int32_t u = g.nbr[j];
      if (deg[u] > deg[v]) {
        /* swap u with the first vertex of its bucket, then shrink the bucket */
        int64_t du = deg[u], pu = pos[u], pw = bin[du];
        int32_t w = vert[pw];
        if (u != w) {
          pos[u] = pw; vert[pw] = u;
          pos[w] = pu; vert[pu] = w;
        }
        bin[du]++;
        deg[u]--;
      }
    }
  }
  int32_t cmax = 0;
  for (int32_t v = 0; v < n; ++v) {
    core[v] = (int32_t)deg[v];
    if (core[v] > cmax) cmax = core[v];
  }
  if (cmax_out) *cmax_out = cmax;
  free(bin); free(deg); free(pos); free(vert);
  adj_free(&g);
  return OR_OK;
}

/* Statistics of the subgraph S given by a mask over the edges: out[0] = its
 * vertices (those touching an edge of S), out[1] = its edges, out[2] = the
 * mean over those vertices of the local clustering coefficient within S:
 * triangles of S at v divided by deg_S(v)(deg_S(v)-1)/2 (0 when deg_S < 2).
 * Triangles at v are counted by merging the sorted S-neighbour lists of the
 * two ends of each S-edge at v. */
static int subgraph_stats(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const uint8_t *in,
                          double *out) {
  int64_t ms = 0;
  for (int64_t i = 0; i < m; ++i) ms += in[i];
  int32_t *s2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ms + 1));
  int32_t *d2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ms + 1));
  if (!s2 || !d2) { free(s2); free(d2); return -OR_NOMEM; }
  for (int64_t i = 0, j = 0; i < m; ++i)
    if (in[i]) { s2[j] = src[i]; d2[j] = dst[i]; ++j; }
  adj_t g;
  int rc = adj_build(n, ms, s2, d2, &g);
  if (rc) { free(s2); free(d2); return rc; }
  int64_t *tri = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!tri) { free(s2); free(d2); adj_free(&g); return -OR_NOMEM; }
  for (int64_t i = 0; i < ms; ++i) {
    int32_t u = s2[i], v = d2[i];
    int64_t a = g.off[u], ae = g.off[u + 1], b = g.off[v], be = g.off[v + 1], c = 0;
    while (a < ae && b < be) {
      if (g.nbr[a] < g.nbr[b]) ++a;
      else if (g.nbr[a] > g.nbr[b]) ++b;
      else { ++c; ++a; ++b; }
    }
    tri[u] += c;  /* each triangle at u is seen from both of its edges at u */
    tri[v] += c;
  }
  int64_t nv = 0;
  double cc = 0.0;
  for (int32_t v = 0; v < n; ++v) {
    int64_t d = g.off[v + 1] - g.off[v];
    if (d == 0) continue;
    ++nv;
    if (d >= 2) cc += (double)(tri[v] / 2) / ((double)d * (double)(d - 1) / 2.0);
  }
  out[0] = (double)nv;
  out[1] = (double)ms;
  out[2] = nv ? cc / (double)nv : 0.0;
  free(tri); free(s2); free(d2);
  adj_free(&g);
  return OR_OK;
}

/* Table 6's columns for T = the k_max-truss (edges with phi = k_max) and C =
 * the c_max-core (edges with both ends of core number c_max):
 * out = {V_T, E_T, k_max, CC_T, V_C, E_C, c_max, CC_C}. */
int oracle_cohesion(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *phi,
                    const int32_t *core, double *out) {
  int32_t kmax = 0, cmax = 0;
  for (int64_t i = 0; i < m; ++i) if (phi[i] > kmax) kmax = phi[i];
  for (int32_t v = 0; v < n; ++v) if (core[v] > cmax) cmax = core[v];
  uint8_t *in = (uint8_t *)calloc((size_t)m + 1, 1);
  if (!in) return -OR_NOMEM;
  double st[3];
  for (int64_t i = 0; i < m; ++i) in[i] = (uint8_t)(phi[i] == kmax);
  int rc = subgraph_stats(n, m, src, dst, in, st);
  if (!rc) { out[0] = st[0]; out[1] = st[1]; out[2] = kmax; out[3] = st[2]; }
  for (int64_t i = 0; !rc && i < m; ++i) in[i] = (uint8_t)(core[src[i]] == cmax && core[dst[i]] == cmax);
  if (!rc) rc = subgraph_stats(n, m, src, dst, in, st);
  if (!rc) { out[4] = st[0]; out[5] = st[1]; out[6] = cmax; out[7] = st[2]; }
  free(in);
  return rc;
}

/* ------------------------------------------------------------------------- */
/* Bottom-up truss decomposition (Section 5): LowerBounding (Algorithm 3),    */
/* then Algorithm 4 with Procedure 5, or Procedure 9 (Appendix) when the      */
/* candidate subgraph exceeds the memory budget.                              */
/* ------------------------------------------------------------------------- */
/* Readings (the paper leaves the partition open and is at odds with itself
 * on the 2-class; the design notes list these):
 *   - Memory budget: cap = the most edges a neighbourhood subgraph may hold.
 *   - Partition of a vertex set (Algorithm 3 and Procedure 9): parts grown breadth-first over the edges of the graph being
 *     partitioned (the current G; H' in Procedure 9), each vertex weighted
 *     by its degree in the graph the neighbourhood subgraphs are taken from
 *     (the current G; the current H), a part's weight sum at most cap
 *     (grow_partition below; a vertex alone above cap is an error).
 *     |NS(P)| <= the weight sum, so every part fits.  A pass that leaves
 *     every edge between parts stalls (an error: the budget is too small for
 *     this graph).  The first pass of Algorithm 3 may use a partition given
 *     by the caller (Example 3's {a,b,c,l}, {d,e,f,g}, {h,i,j,k}).
 *   - The 2-class: an internal edge's support in the current graph is its
 *     support in the input graph only in the first pass (later passes lack the
 *     internal edges removed before), so only the first pass outputs internal
 *     edges of support 0 as Phi_2; internal edges of later passes go to G_new
 *     with their bound, and Algorithm 4 then starts from k = 2 instead of 3.
 *     Example 3 likewise stops stage 1 after one pass.
 *   - The bound starts at 2 (Example 3; Algorithm 3 starts it at 0): every edge lies in
 *     some neighbourhood subgraph, where its local truss number is >= 2, so
 *     the two starts give the same bounds.
 *   - Algorithm 4 skips a k for which no edge of G_new has bound <= k: U_k
 *     and hence Phi_k are empty there.  k starts at the smallest bound >= the
 *     start value.
 *   - Procedure 9: F = NS(P_i) is taken in the current H (so that supports of
 *     its internal edges are exact); the edges eligible for Phi_k are those
 *     internal to both F and H; P ranges over the vertices that still have an
 *     edge of H' (not yet internal to an F in this scan), weighted by their
 *     degree in H.  A scan without new Phi_k edges ends the procedure. */
enum { OR_CAP = 10, OR_STALL = 11 };

/* Parts grown breadth-first (the partitions of Algorithm 3 and Procedure 9).
 * Vertices qualify when they have an edge with mask[e] set.  A part starts
 * at the smallest-id qualifying vertex not yet placed and grows
 * breadth-first: from each vertex it holds (in the order added) it takes
 * every unplaced neighbour over such edges, by ascending id, whose weight
 * still fits (weight sum <= cap); a neighbour that does not fit is left for
 * a later part.  When the growth stops, the part goes on from the next
 * unplaced qualifying vertex by id if that one still fits, else a new part
 * starts there.  part[v] = part id, -1 for vertices that do not qualify.
 * Returns the number of parts or a negative error. */
static int64_t grow_partition(const adj_t *g, const uint8_t *mask, const int64_t *w, int64_t cap, int32_t *part,
                              int32_t *queue) {
  int64_t parts = 0, sum = 0;
  for (int32_t v = 0; v < g->n; ++v) part[v] = -1;
  for (int32_t r = 0; r < g->n; ++r) {
    if (part[r] >= 0) continue;
    int has = 0;
    for (int64_t j = g->off[r]; j < g->off[r + 1] && !has; ++j) has = mask[g->eid[j]];
    if (!has) continue;
    if (w[r] > cap) return -OR_CAP;
    if (parts == 0 || sum + w[r] > cap) { ++parts; sum = 0; }
    const int32_t p = (int32_t)(parts - 1);
    int32_t head = 0, tail = 0;
    sum += w[r];
    part[r] = p;
    queue[tail++] = r;
    while (head < tail) {
      const int32_t v = queue[head++];
      for (int64_t j = g->off[v]; j < g->off[v + 1]; ++j) {
        const int32_t x = g->nbr[j];
        if (!mask[g->eid[j]] || part[x] >= 0 || sum + w[x] > cap) continue;
        part[x] = p;
        sum += w[x];
        queue[tail++] = x;
      }
    }
  }
  return parts;
}

/* Local truss numbers and supports of the subgraph given by the edge ids
 * ids[0..h) (Algorithm 2 and Definition 1 on that subgraph). */
static int local_truss(int32_t n, const int32_t *src, const int32_t *dst, const int64_t *ids, int64_t h,
                       int32_t *phi_h, int32_t *sup_h) {
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(h + 1));
  int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)(h + 1));
  if (!s || !d) { free(s); free(d); return -OR_NOMEM; }
  for (int64_t i = 0; i < h; ++i) { s[i] = src[ids[i]]; d[i] = dst[ids[i]]; }
  int rc = oracle_support_fwd(n, h, s, d, sup_h, NULL);
  if (!rc && phi_h) rc = oracle_truss(n, h, s, d, phi_h, NULL);
  free(s); free(d);
  return rc;
}

/* LowerBounding (Algorithm 3).  lb[e] = the bound of every edge; phi2[e] = 1
 * for the edges output as Phi_2.  info (nullable) = {passes, neighbourhood
 * subgraphs, |Phi_2|, |G_new|, largest subgraph}. */
int oracle_lower_bounding(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                          const int32_t *first_part, int64_t cap, int32_t *lb, uint8_t *phi2, int64_t *info) {
  uint8_t *alive = (uint8_t *)malloc((size_t)m + 1);
  uint8_t *active = (uint8_t *)malloc((size_t)n + 1);
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  int32_t *part = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
  int32_t *phi_h = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
  int32_t *sup_h = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m + 1));
  int64_t st[5] = {0, 0, 0, 0, 0};
  adj_t g;
  memset(&g, 0, sizeof(g));
  int rc = OR_OK;
  if (!alive || !active || !deg || !part || !order || !ids || !phi_h || !sup_h) { rc = -OR_NOMEM; goto out; }
  if ((rc = adj_build(n, m, src, dst, &g))) goto out;
  for (int64_t e = 0; e < m; ++e) { alive[e] = 1; lb[e] = 2; phi2[e] = 0; }
  int64_t left = m;
  /* passes over the shrinking graph: partition, decompose each part's
   * neighbourhood subgraph, raise the bounds, drop the internal edges */
  while (left > 0) {
    const int first = st[0] == 0;
    st[0]++;
    for (int32_t v = 0; v < n; ++v) deg[v] = 0;
    for (int64_t e = 0; e < m; ++e)
      if (alive[e]) { deg[src[e]]++; deg[dst[e]]++; }
    for (int32_t v = 0; v < n; ++v) active[v] = deg[v] > 0;
    int64_t parts;
    if (first && first_part) {
      parts = 0;
      for (int32_t v = 0; v < n; ++v) {
        part[v] = active[v] ? first_part[v] : -1;
        if (active[v] && (first_part[v] < 0 || first_part[v] >= n)) { rc = -OR_INVAL; goto out; }
        if (part[v] + 1 > parts) parts = part[v] + 1;
      }
    } else {
      parts = grow_partition(&g, alive, deg, cap, part, order);
      if (parts < 0) { rc = (int)parts; goto out; }
    }
    int64_t removed = 0;
    for (int64_t p = 0; p < parts; ++p) {
      int64_t h = 0;  /* NS(P_p): live edges with an end in part p */
      for (int64_t e = 0; e < m; ++e)
        if (alive[e] && (part[src[e]] == p || part[dst[e]] == p)) ids[h++] = e;
      if (h == 0) continue;
      if (h > cap) { rc = -OR_CAP; goto out; }
      st[1]++;
      if (h > st[4]) st[4] = h;
      rc = local_truss(n, src, dst, ids, h, phi_h, sup_h);
      if (rc) goto out;
      for (int64_t i = 0; i < h; ++i) {
        const int64_t e = ids[i];
        if (phi_h[i] > lb[e]) lb[e] = phi_h[i];  /* Lemma 1: a local truss number is a lower bound */
        if (part[src[e]] == p && part[dst[e]] == p) {
          /* an internal edge leaves the graph: to Phi_2 if it closes no
           * triangle (first pass only), else to G_new with its bound */
          if (first && sup_h[i] == 0) { phi2[e] = 1; st[2]++; }
          else st[3]++;
          alive[e] = 0;
          ++removed;
        }
      }
    }
    if (removed == 0) { rc = -OR_STALL; goto out; }
    left -= removed;
  }
  if (info) for (int i = 0; i < 5; ++i) info[i] = st[i];
out:
  adj_free(&g);
  free(alive); free(active); free(deg); free(part); free(order); free(ids); free(phi_h); free(sup_h);
  return rc;
}

/* Peel the eligible edges of the subgraph ids[0..h) at level k (Procedure 5;
 * the inner peel of Procedure 9): while an eligible edge has support
 * <= k-2, it joins Phi_k and the two other edges of each of its triangles in
 * the subgraph lose one.  Removed edges get phi = k and gone = 1.  Returns the
 * number of edges output, or a negative error. */
static int64_t peel_level(int32_t n, const int32_t *src, const int32_t *dst, const int64_t *ids, int64_t h,
                          const uint8_t *elig, int32_t k, int32_t *phi, uint8_t *gone) {
  int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(h + 1));
  int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)(h + 1));
  int32_t *sup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(h + 1));
  uint8_t *out = (uint8_t *)calloc((size_t)h + 1, 1);
  uint8_t *inq = (uint8_t *)calloc((size_t)h + 1, 1);
  int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(h + 1));
  adj_t g;
  memset(&g, 0, sizeof(g));
  int64_t count = 0;
  if (!s || !d || !sup || !out || !inq || !queue) { count = -OR_NOMEM; goto done; }
  for (int64_t i = 0; i < h; ++i) { s[i] = src[ids[i]]; d[i] = dst[ids[i]]; }
  int rc = oracle_support_fwd(n, h, s, d, sup, NULL);
  if (!rc) rc = adj_build(n, h, s, d, &g);
  if (rc) { count = rc; goto done; }
  int64_t qh = 0, qt = 0;
  for (int64_t i = 0; i < h; ++i)
    if (elig[i] && sup[i] <= k - 2) { queue[qt++] = i; inq[i] = 1; }
  while (qh < qt) {
    const int64_t e = queue[qh++];
    const int32_t u = s[e], v = d[e];
    for (int64_t j = g.off[u]; j < g.off[u + 1]; ++j) {
      const int32_t w = g.nbr[j];
      const int64_t euw = g.eid[j];
      if (w == v || out[euw]) continue;
      const int64_t q = find_nbr(&g, v, w);
      if (q < 0 || out[g.eid[q]]) continue;
      const int64_t f2[2] = {euw, g.eid[q]};
      for (int t = 0; t < 2; ++t) {
        const int64_t f = f2[t];
        sup[f] -= 1;
        if (elig[f] && !inq[f] && sup[f] <= k - 2) { queue[qt++] = f; inq[f] = 1; }
      }
    }
    out[e] = 1;
    phi[ids[e]] = k;
    gone[ids[e]] = 1;
    ++count;
  }
done:
  adj_free(&g);
  free(s); free(d); free(sup); free(out); free(inq); free(queue);
  return count;
}

/* Procedure 9: Phi_k of the candidate subgraph ids[0..h) (internal[i] = both
 * ends in U_k) when it exceeds cap.  Returns edges output or an error;
 * scans_out accumulates the scans made. */
static int64_t proc9(const adj_t *g, const int32_t *src, const int32_t *dst, const int64_t *ids, int64_t h,
                     const uint8_t *internal, int32_t k, int64_t cap, int32_t *phi, uint8_t *gone,
                     int64_t *scans_out) {
  const int32_t n = g->n;
  uint8_t *mask = (uint8_t *)calloc((size_t)g->m + 1, 1);   /* edges of H' (by edge id) */
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  uint8_t *inh = (uint8_t *)calloc((size_t)h + 1, 1);       /* still in H */
  uint8_t *cov = (uint8_t *)calloc((size_t)h + 1, 1);       /* removed from H' */
  int64_t *deg = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  uint8_t *active = (uint8_t *)malloc((size_t)n + 1);
  int32_t *part = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int64_t *fid = (int64_t *)malloc(sizeof(int64_t) * ((size_t)h + 1));
  int64_t *fpos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)h + 1));
  uint8_t *elig = (uint8_t *)malloc((size_t)h + 1);
  int64_t total = 0;
  if (!mask || !order || !inh || !cov || !deg || !active || !part || !fid || !fpos || !elig) {
    total = -OR_NOMEM;
    goto done;
  }
  for (int64_t i = 0; i < h; ++i) inh[i] = 1;
  /* scans of H until one adds nothing to Phi_k; each scan partitions H'
   * (the edges of H not yet internal to a part of this scan) and peels the
   * eligible edges of every part's neighbourhood subgraph in H */
  for (;;) {
    int64_t found = 0;
    for (int64_t i = 0; i < h; ++i) cov[i] = !inh[i];
    for (;;) {
      int64_t left = 0;
      for (int32_t v = 0; v < n; ++v) deg[v] = 0;
      for (int64_t i = 0; i < h; ++i) {
        mask[ids[i]] = inh[i] && !cov[i];
        if (!inh[i]) continue;
        deg[src[ids[i]]]++; deg[dst[ids[i]]]++;
        left += !cov[i];
      }
      if (left == 0) break;
      (*scans_out)++;
      const int64_t parts = grow_partition(g, mask, deg, cap, part, order);
      if (parts < 0) { total = parts; goto done; }
      int64_t covered = 0;
      for (int64_t p = 0; p < parts; ++p) {
        int64_t f = 0;  /* F = NS(P_p) in H */
        for (int64_t i = 0; i < h; ++i) {
          if (!inh[i]) continue;
          const int32_t a = part[src[ids[i]]], b = part[dst[ids[i]]];
          if (a == p || b == p) { fpos[f] = i; fid[f] = ids[i]; elig[f] = a == p && b == p && internal[i]; ++f; }
        }
        if (f == 0) continue;
        if (f > cap) { total = -OR_CAP; goto done; }
        const int64_t c = peel_level(n, src, dst, fid, f, elig, k, phi, gone);
        if (c < 0) { total = c; goto done; }
        found += c;
        for (int64_t j = 0; j < f; ++j) {
          const int64_t i = fpos[j];
          if (gone[ids[i]]) inh[i] = 0;
          const int32_t a = part[src[ids[i]]], b = part[dst[ids[i]]];
          if (a == p && b == p && !cov[i]) { cov[i] = 1; ++covered; }
        }
      }
      if (covered == 0) { total = -OR_STALL; goto done; }
    }
    total += found;
    if (found == 0) break;
  }
done:
  free(mask); free(order);
  free(inh); free(cov); free(deg); free(active); free(part); free(fid); free(fpos); free(elig);
  return total;
}

/* Algorithm 4 on the output of LowerBounding: phi[e] for every edge.
 * kstart = 3, or 2 when LowerBounding took more than one pass.  info
 * (nullable) = {candidate subgraphs, Procedure 9 calls, Procedure 9 scans,
 * largest candidate subgraph, k_max}. */
int oracle_bottom_up(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int32_t *lb,
                     const uint8_t *phi2, int32_t kstart, int64_t cap, int32_t *phi, int64_t *info) {
  uint8_t *gone = (uint8_t *)malloc((size_t)m + 1);
  uint8_t *inu = (uint8_t *)malloc((size_t)n + 1);
  int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
  uint8_t *internal = (uint8_t *)malloc((size_t)m + 1);
  int64_t st[5] = {0, 0, 0, 0, 0};
  adj_t g;
  memset(&g, 0, sizeof(g));
  int rc = OR_OK;
  if (!gone || !inu || !ids || !internal) { rc = -OR_NOMEM; goto out; }
  if ((rc = adj_build(n, m, src, dst, &g))) goto out;
  int64_t left = 0;
  for (int64_t e = 0; e < m; ++e) {
    gone[e] = phi2[e];
    phi[e] = phi2[e] ? 2 : 0;
    left += !phi2[e];
  }
  /* one level k at a time: U_k = the ends of the G_new edges with bound <= k,
   * Phi_k from the candidate subgraph NS(U_k) */
  int32_t k = kstart;
  while (left > 0) {
    int32_t lmin = 0x7fffffff;
    for (int64_t e = 0; e < m; ++e)
      if (!gone[e] && lb[e] < lmin) lmin = lb[e];
    if (lmin > k) k = lmin;
    for (int32_t v = 0; v < n; ++v) inu[v] = 0;
    for (int64_t e = 0; e < m; ++e)
      if (!gone[e] && lb[e] <= k) { inu[src[e]] = 1; inu[dst[e]] = 1; }
    int64_t h = 0;  /* NS(U_k) */
    for (int64_t e = 0; e < m; ++e)
      if (!gone[e] && (inu[src[e]] || inu[dst[e]])) {
        internal[h] = inu[src[e]] && inu[dst[e]];
        ids[h++] = e;
      }
    st[0]++;
    if (h > st[3]) st[3] = h;
    int64_t c;
    if (h <= cap) {
      c = peel_level(n, src, dst, ids, h, internal, k, phi, gone);  /* Procedure 5 */
    } else {
      st[1]++;
      c = proc9(&g, src, dst, ids, h, internal, k, cap, phi, gone, &st[2]);
    }
    if (c < 0) { rc = (int)c; goto out; }
    left -= c;
    st[4] = k;
    k += 1;
  }
  if (info) for (int i = 0; i < 5; ++i) info[i] = st[i];
out:
  adj_free(&g);
  free(gone); free(inu); free(ids); free(internal);
  return rc;
}
