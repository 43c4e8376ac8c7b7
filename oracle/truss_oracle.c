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
 *            merge of the full sorted adjacency lists (Algorithm 1, Steps 2-3);
 *       (ii) oracle_support_fwd: every triangle listed once through the
 *            degree orientation (deg, id) and counted on its three edges — the
 *            in-memory triangle counting cited for Algorithm 2, Step 2
 *            (Section 3.2);
 *   - phi(e), the truss number (Definition 2 and the text after it), by
 *     Algorithm 2 (Section 3.2): bin sort of edges by support, then repeatedly
 *     take the lowest-support edge e=(u,v) while sup(e) <= k-2, walk the
 *     smaller-degree endpoint's neighbours w, and for each live triangle
 *     decrement (u,w) and (v,w) and re-bin them; e joins the k-class.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - Algorithm 2, Step 9 decrements unconditionally.  Here an edge whose
 *     support is already <= k-2 is not decremented: it is removed at this level
 *     anyway (so its truss number is k either way) and the guard keeps the bin
 *     array sorted without moving an edge left of the pointer.
 *   - "w in nb(u)" and "(v,w) in E_G" are read on the current graph: both
 *     (u,w) and (v,w) must not have been removed yet.
 *   - deg() in Step 6 is the original degree; ties go to the smaller id.
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
 * (Algorithm 1, Step 3).  O(sum_v deg(v)^2). */
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

/* phi[i] for every input edge i; kmax_out (nullable) gets the largest phi
 * (2 for an edgeless graph is not reported: kmax_out = 0 when m = 0). */
int oracle_truss(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 int32_t *phi, int32_t *kmax_out) {
  if (kmax_out) *kmax_out = 0;
  if (m == 0) return OR_OK;
  int32_t *sup = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
  if (!sup) return -OR_NOMEM;
  /* Step 2: support by triangle counting */
  int rc = oracle_support_fwd(n, m, src, dst, sup, NULL);
  if (rc) { free(sup); return rc; }
  adj_t g;
  rc = adj_build(n, m, src, dst, &g);
  if (rc) { free(sup); return rc; }

  /* Step 3: bin sort by support.  order[] is the sorted edge array, pos[e]
   * the position of e in it, bin[s] the first position holding support s. */
  int32_t maxsup = 0;
  for (int64_t i = 0; i < m; ++i) if (sup[i] > maxsup) maxsup = sup[i];
  int64_t *bin = (int64_t *)calloc((size_t)maxsup + 2, sizeof(int64_t));
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
  unsigned char *removed = (unsigned char *)calloc((size_t)m, 1);
  if (!bin || !order || !pos || !removed) {
    free(bin); free(order); free(pos); free(removed); free(sup); adj_free(&g);
    return -OR_NOMEM;
  }
  for (int64_t i = 0; i < m; ++i) bin[sup[i] + 1]++;
  for (int32_t s = 0; s <= maxsup; ++s) bin[s + 1] += bin[s];
  {
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * ((size_t)maxsup + 1));
    if (!next) {
      free(bin); free(order); free(pos); free(removed); free(sup); adj_free(&g);
      return -OR_NOMEM;
    }
    for (int32_t s = 0; s <= maxsup; ++s) next[s] = bin[s];
    for (int64_t i = 0; i < m; ++i) { pos[i] = next[sup[i]]++; order[pos[i]] = i; }
    free(next);
  }

  /* Steps 4-15 */
  int32_t k = 2;
  int64_t p = 0;
  while (p < m) {
    int64_t e = order[p];
    if (sup[e] > k - 2) { ++k; continue; }          /* Steps 13-15 */
    int32_t u = src[e], v = dst[e];
    if (!before(&g, u, v)) { int32_t t = u; u = v; v = t; }  /* Step 6 */
    for (int64_t j = g.off[u]; j < g.off[u + 1]; ++j) {     /* Step 7 */
      int32_t w = g.nbr[j];
      int64_t euw = g.eid[j];
      if (w == v || removed[euw]) continue;
      int64_t q = find_nbr(&g, v, w);                       /* Step 8 */
      if (q < 0) continue;
      int64_t evw = g.eid[q];
      if (removed[evw]) continue;
      int64_t f2[2] = {euw, evw};
      for (int t = 0; t < 2; ++t) {                         /* Steps 9-10 */
        int64_t f = f2[t];
        if (sup[f] > k - 2) {
          int32_t s = sup[f];
          int64_t pf = pos[f], pb = bin[s];
          int64_t g2 = order[pb];
          order[pb] = f; pos[f] = pb;
          order[pf] = g2; pos[g2] = pf;
          bin[s]++;
          sup[f] = s - 1;
        }
      }
    }
    phi[e] = k;                                             /* Step 11 */
    removed[e] = 1;                                         /* Step 12 */
    ++p;
  }
  if (kmax_out) *kmax_out = k;
  free(bin); free(order); free(pos); free(removed); free(sup);
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
