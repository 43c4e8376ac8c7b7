/*
 * Seeded synthetic graph generators (inputs only; no truss arithmetic here).
 *
 * Every random number is SplitMix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: draw i of stream s under seed x is mix(x ^ (s * C1) + (i + 1) * GAMMA),
 * so samples can be produced in any order or in parallel and stay identical.
 *
 * Families (all simple undirected, self-loops dropped, duplicates merged,
 * output canonical: u < v, sorted by (u, v)):
 *   gg_er        Erdos-Renyi G(n, p), pairs visited in order with geometric skips
 *   gg_rmat      R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with a seeded vertex
 *                permutation
 *   gg_chung_lu  Chung-Lu with power-law weights, capped, plus planted cliques
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL
#define C1 0xD1B54A32D192ED03ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64((seed ^ (stream * C1)) + (i + 1) * GAMMA);
}

/* uniform double in [0,1) from the top 53 bits */
static inline double unif(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

typedef struct {
  int32_t n;
  int64_t m;
  int32_t *src;
  int32_t *dst;
} gg_graph;

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->src); free(g->dst); free(g);
}

int64_t gg_m(const gg_graph *g) { return g->m; }
int32_t gg_n(const gg_graph *g) { return g->n; }

void gg_copy(const gg_graph *g, int32_t *src, int32_t *dst) {
  memcpy(src, g->src, sizeof(int32_t) * (size_t)g->m);
  memcpy(dst, g->dst, sizeof(int32_t) * (size_t)g->m);
}

/* LSD radix sort of 64-bit keys on their low `bits` bits, 16 bits a pass. */
static int radix_u64(uint64_t *a, int64_t n, int bits) {
  if (n <= 1) return 0;
  uint64_t *buf = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * 65536);
  if (!buf || !cnt) { free(buf); free(cnt); return -1; }
  uint64_t *from = a, *to = buf;
  for (int shift = 0; shift < bits; shift += 16) {
    memset(cnt, 0, sizeof(int64_t) * 65536);
    for (int64_t i = 0; i < n; ++i) cnt[(from[i] >> shift) & 0xFFFF]++;
    int64_t s = 0;
    for (int d = 0; d < 65536; ++d) { int64_t c = cnt[d]; cnt[d] = s; s += c; }
    for (int64_t i = 0; i < n; ++i) to[cnt[(from[i] >> shift) & 0xFFFF]++] = from[i];
    uint64_t *t = from; from = to; to = t;
  }
  if (from != a) memcpy(a, from, sizeof(uint64_t) * (size_t)n);
  free(buf); free(cnt);
  return 0;
}

static int bits_for(int64_t n) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < n) ++b;
  return b;
}

/* Canonicalise, drop self loops, sort and deduplicate; keys hold (u<<32)|v. */
static gg_graph *finish(int32_t n, uint64_t *key, int64_t cnt) {
  int64_t w = 0;
  for (int64_t i = 0; i < cnt; ++i) {
    uint32_t u = (uint32_t)(key[i] >> 32), v = (uint32_t)key[i];
    if (u == v) continue;
    uint64_t a = u < v ? u : v, b = u < v ? v : u;
    key[w++] = (a << 32) | b;
  }
  int vb = bits_for(n);
  /* pack (a, b) into 2*vb bits for a shorter sort, then unpack */
  for (int64_t i = 0; i < w; ++i) key[i] = ((key[i] >> 32) << vb) | (key[i] & 0xFFFFFFFFULL);
  int tb = 2 * vb;
  tb = ((tb + 15) / 16) * 16;
  if (radix_u64(key, w, tb ? tb : 16)) return NULL;
  gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
  if (!g) return NULL;
  int64_t m = 0;
  for (int64_t i = 0; i < w; ++i)
    if (i == 0 || key[i] != key[i - 1]) key[m++] = key[i];
  g->n = n; g->m = m;
  g->src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  g->dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m + 1));
  if (!g->src || !g->dst) { gg_free(g); return NULL; }
  uint64_t mask = vb ? ((1ULL << vb) - 1) : 0;
  for (int64_t i = 0; i < m; ++i) {
    g->src[i] = (int32_t)(key[i] >> vb);
    g->dst[i] = (int32_t)(key[i] & mask);
  }
  return g;
}

/* Erdos-Renyi: pairs (i<j) in row-major order; the gap to the next chosen pair
 * is geometric with parameter p (inverse-CDF).  stream 1. */
gg_graph *gg_er(int32_t n, double p, uint64_t seed) {
  if (n < 0) return NULL;
  int64_t total = (int64_t)n * (n - 1) / 2;
  int64_t cap = (int64_t)(total * p + 8.0 * sqrt(total * p + 1.0) + 16.0);
  if (p >= 1.0) cap = total;
  if (cap > total) cap = total;
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(cap + 1));
  if (!key) return NULL;
  int64_t cnt = 0, idx = -1, draws = 0;
  double lq = (p > 0.0 && p < 1.0) ? log1p(-p) : 0.0;
  int64_t row = 0, rowstart = 0; /* rowstart = linear index of (row, row+1) */
  while (p > 0.0) {
    if (p >= 1.0) idx += 1;
    else {
      double u = unif(draw(seed, 1, (uint64_t)draws++));
      double g = floor(log1p(-u) / lq);
      if (g > (double)total) break;
      idx += 1 + (int64_t)g;
    }
    if (idx >= total) break;
    while (idx >= rowstart + (n - 1 - row)) { rowstart += n - 1 - row; ++row; }
    int64_t col = row + 1 + (idx - rowstart);
    if (cnt >= cap) {
      cap = cap * 2 + 16;
      uint64_t *k2 = (uint64_t *)realloc(key, sizeof(uint64_t) * (size_t)(cap + 1));
      if (!k2) { free(key); return NULL; }
      key = k2;
    }
    key[cnt++] = ((uint64_t)row << 32) | (uint64_t)col;
  }
  gg_graph *g = finish(n, key, cnt);
  free(key);
  return g;
}

/* Fisher-Yates permutation of [0, n) from the given stream. */
static int32_t *perm_n(int32_t n, uint64_t seed, uint64_t stream) {
  int32_t *pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!pi) return NULL;
  for (int32_t i = 0; i < n; ++i) pi[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    uint64_t r = draw(seed, stream, (uint64_t)i);
    int32_t j = (int32_t)(((unsigned __int128)r * (uint64_t)(i + 1)) >> 64);
    int32_t t = pi[i]; pi[i] = pi[j]; pi[j] = t;
  }
  return pi;
}

/* R-MAT: `samples` edges of a 2^scale vertex grid; each sample descends `scale`
 * levels, choosing quadrant (0,0),(0,1),(1,0),(1,1) with probabilities
 * a, b, c, 1-a-b-c, one 32-bit uniform per level (stream 2, two levels per
 * draw).  Endpoints >= n are rejected (n <= 2^scale).  If permute, vertex ids
 * are relabelled by a seeded permutation (stream 3). */
gg_graph *gg_rmat(int32_t scale, int64_t samples, int32_t n, double a, double b, double c,
                  uint64_t seed, int permute) {
  if (scale < 0 || scale > 30 || n < 0 || n > (1 << scale) || samples < 0) return NULL;
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(samples + 1));
  if (!key) return NULL;
  const double ab = a + b, abc = a + b + c;
  const uint32_t tA = (uint32_t)(a * 4294967296.0), tAB = (uint32_t)(ab * 4294967296.0),
                 tABC = (uint32_t)(abc * 4294967296.0 > 4294967295.0 ? 4294967295.0 : abc * 4294967296.0);
  const int per = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < samples; ++s) {
    uint32_t u = 0, v = 0;
    for (int d = 0; d < per; ++d) {
      uint64_t r = draw(seed, 2, (uint64_t)s * (uint64_t)per + (uint64_t)d);
      for (int h = 0; h < 2; ++h) {
        int lvl = 2 * d + h;
        if (lvl >= scale) break;
        uint32_t x = (uint32_t)(h ? (r >> 32) : r);
        uint32_t bu = 0, bv = 0;
        if (x < tA) { bu = 0; bv = 0; }
        else if (x < tAB) { bu = 0; bv = 1; }
        else if (x < tABC) { bu = 1; bv = 0; }
        else { bu = 1; bv = 1; }
        u = (u << 1) | bu; v = (v << 1) | bv;
      }
    }
    key[s] = ((uint64_t)u << 32) | v;
  }
  int64_t cnt = 0;
  for (int64_t s = 0; s < samples; ++s) {
    uint32_t u = (uint32_t)(key[s] >> 32), v = (uint32_t)key[s];
    if ((int64_t)u >= n || (int64_t)v >= n) continue;
    key[cnt++] = key[s];
  }
  if (permute && n > 1) {
    int32_t *pi = perm_n(n, seed, 3);
    if (!pi) { free(key); return NULL; }
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < cnt; ++s) {
      uint32_t u = (uint32_t)(key[s] >> 32), v = (uint32_t)key[s];
      key[s] = ((uint64_t)(uint32_t)pi[u] << 32) | (uint32_t)pi[v];
    }
    free(pi);
  }
  gg_graph *g = finish(n, key, cnt);
  free(key);
  return g;
}

/* Chung-Lu: weight w_i = min(cap, C * (i+1)^(-1/(gamma-1))) with C found by
 * bisection so that the mean weight is mean_deg; round(n*mean_deg/2) endpoint
 * pairs are drawn, each endpoint by inverse CDF over the weights (stream 4).
 * Then n_cliques cliques with sizes uniform in [cmin, cmax] (stream 5) are
 * planted on disjoint vertex sets taken from a seeded permutation (stream 6). */
gg_graph *gg_chung_lu(int32_t n, double gamma, double mean_deg, double cap,
                      int32_t n_cliques, int32_t cmin, int32_t cmax, uint64_t seed) {
  if (n <= 1 || gamma <= 1.0 || mean_deg <= 0) return NULL;
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  double *cdf = (double *)malloc(sizeof(double) * (size_t)n);
  if (!w || !cdf) { free(w); free(cdf); return NULL; }
  const double alpha = 1.0 / (gamma - 1.0);
  double lo = 0.0, hi = cap * 4.0 + mean_deg * 4.0;
  for (int it = 0; it < 200; ++it) {
    double C = 0.5 * (lo + hi), s = 0.0;
    for (int32_t i = 0; i < n; ++i) {
      double x = C * pow((double)(i + 1), -alpha);
      s += x > cap ? cap : x;
    }
    if (s / n < mean_deg) lo = C; else hi = C;
  }
  {
    double C = 0.5 * (lo + hi), s = 0.0;
    for (int32_t i = 0; i < n; ++i) {
      double x = C * pow((double)(i + 1), -alpha);
      w[i] = x > cap ? cap : x;
      s += w[i];
      cdf[i] = s;
    }
    for (int32_t i = 0; i < n; ++i) cdf[i] /= s;
  }
  int64_t pairs = (int64_t)llround((double)n * mean_deg / 2.0);
  int64_t csize_total = 0;
  int32_t *csz = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_cliques + 1));
  if (!csz) { free(w); free(cdf); return NULL; }
  for (int32_t q = 0; q < n_cliques; ++q) {
    uint64_t r = draw(seed, 5, (uint64_t)q);
    csz[q] = cmin + (int32_t)(((unsigned __int128)r * (uint64_t)(cmax - cmin + 1)) >> 64);
    csize_total += csz[q];
  }
  if (csize_total > n) { free(w); free(cdf); free(csz); return NULL; }
  int64_t cedges = 0;
  for (int32_t q = 0; q < n_cliques; ++q) cedges += (int64_t)csz[q] * (csz[q] - 1) / 2;
  uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(pairs + cedges + 1));
  if (!key) { free(w); free(cdf); free(csz); return NULL; }
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < pairs; ++s) {
    uint32_t ends[2];
    for (int h = 0; h < 2; ++h) {
      double u = unif(draw(seed, 4, (uint64_t)(2 * s + h)));
      int32_t l = 0, r = n - 1;
      while (l < r) {
        int32_t mid = l + (r - l) / 2;
        if (cdf[mid] <= u) l = mid + 1; else r = mid;
      }
      ends[h] = (uint32_t)l;
    }
    key[s] = ((uint64_t)ends[0] << 32) | ends[1];
  }
  int64_t cnt = pairs;
  if (n_cliques > 0) {
    int32_t *pi = perm_n(n, seed, 6);
    if (!pi) { free(w); free(cdf); free(csz); free(key); return NULL; }
    int64_t base = 0;
    for (int32_t q = 0; q < n_cliques; ++q) {
      for (int32_t x = 0; x < csz[q]; ++x)
        for (int32_t y = x + 1; y < csz[q]; ++y)
          key[cnt++] = ((uint64_t)(uint32_t)pi[base + x] << 32) | (uint32_t)pi[base + y];
      base += csz[q];
    }
    free(pi);
  }
  free(w); free(cdf); free(csz);
  gg_graph *g = finish(n, key, cnt);
  free(key);
  return g;
}

/* Planted clique sizes of gg_chung_lu (for tests of the clique bound). */
void gg_chung_lu_clique_sizes(int32_t n_cliques, int32_t cmin, int32_t cmax, uint64_t seed,
                              int32_t *out) {
  for (int32_t q = 0; q < n_cliques; ++q) {
    uint64_t r = draw(seed, 5, (uint64_t)q);
    out[q] = cmin + (int32_t)(((unsigned __int128)r * (uint64_t)(cmax - cmin + 1)) >> 64);
  }
}

/* Symmetric CSR from a canonical sorted edge list (u < v, sorted by (u, v)):
 * row v holds its neighbours in ascending order.  row_ptr has n+1 entries,
 * col 2m. */
void gg_to_csr(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
               int64_t *row_ptr, int32_t *col) {
  memset(row_ptr, 0, sizeof(int64_t) * ((size_t)n + 1));
  for (int64_t i = 0; i < m; ++i) { row_ptr[src[i] + 1]++; row_ptr[dst[i] + 1]++; }
  for (int32_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  memcpy(fill, row_ptr, sizeof(int64_t) * ((size_t)n + 1));
  /* lower neighbours first (u < v, visited in ascending u), then upper ones */
  for (int64_t i = 0; i < m; ++i) col[fill[dst[i]]++] = src[i];
  for (int64_t i = 0; i < m; ++i) col[fill[src[i]]++] = dst[i];
  free(fill);
}

/* Seeded shuffle of edge order and orientation (stream 7), in place. */
void gg_shuffle(int64_t m, int32_t *src, int32_t *dst, uint64_t seed) {
  for (int64_t i = m - 1; i > 0; --i) {
    uint64_t r = draw(seed, 7, (uint64_t)i);
    int64_t j = (int64_t)(((unsigned __int128)r * (uint64_t)(i + 1)) >> 64);
    int32_t t = src[i]; src[i] = src[j]; src[j] = t;
    t = dst[i]; dst[i] = dst[j]; dst[j] = t;
  }
  for (int64_t i = 0; i < m; ++i) {
    if (draw(seed, 8, (uint64_t)i) >> 63) { int32_t t = src[i]; src[i] = dst[i]; dst[i] = t; }
  }
}
