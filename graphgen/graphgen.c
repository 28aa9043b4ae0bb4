/*
 * graphgen.c -- seeded synthetic graph generators.
 *
 * Shared input module: both the oracle tests and the GPU path draw their
 * inputs from here.  It holds no arithmetic of the maximum-clique method, only
 * random graph models and CSR assembly.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), used as a counter-based generator: every
 * independent stream (a row of the Chung-Lu sampler, an R-MAT sample, the
 * permutation) is seeded by hashing (seed, stream id).
 *
 * Models:
 *   Chung-Lu expected-degree graphs, sampled in O(n+m) with the skipping method
 *     of Miller and Hagberg (WAW 2011): weights sorted in decreasing order, and
 *     for each u a geometric skip over v > u driven by an upper bound on the
 *     pair probability, followed by an accept test with the true probability.
 *   G(n,p) with geometric skipping (Batagelj and Brandes, Phys. Rev. E 2005).
 *   R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004), per-level quadrant choice.
 *   Planted cliques on disjoint, uniformly random vertex sets.
 * Finishing: a seeded uniform relabelling of the background graph, union with
 * the plants, symmetrisation, self-loop removal, de-duplication, sorted rows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ rng */
static inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t sm64_next(uint64_t *s) {
  *s += 0x9E3779B97F4A7C15ULL;
  return sm64_mix(*s);
}
/* Start of stream `id` of generator `seed`. */
static inline uint64_t sm64_stream(uint64_t seed, uint64_t id) {
  return sm64_mix(seed ^ sm64_mix(id + 0x632BE59BD9B4E019ULL));
}
/* Uniform double in [0,1). */
static inline double u01(uint64_t *s) { return (double)(sm64_next(s) >> 11) * 0x1.0p-53; }
/* Uniform double in (0,1]. */
static inline double u01_open0(uint64_t *s) { return ((double)(sm64_next(s) >> 11) + 1.0) * 0x1.0p-53; }
/* Uniform integer in [0, m) (m >= 1), by 128-bit multiply-shift. */
static inline uint64_t ubelow(uint64_t *s, uint64_t m) {
  return (uint64_t)(((__uint128_t)sm64_next(s) * (__uint128_t)m) >> 64);
}

uint64_t gg_splitmix64(uint64_t x) { return sm64_mix(x + 0x9E3779B97F4A7C15ULL); }

/* ------------------------------------------------------------- edge list */
typedef struct {
  int64_t len, cap;
  int32_t *uv; /* pairs */
} edgebuf;

static int eb_push(edgebuf *e, int64_t u, int64_t v) {
  if (e->len == e->cap) {
    int64_t nc = e->cap ? e->cap * 2 : 1 << 16;
    int32_t *p = (int32_t *)realloc(e->uv, (size_t)nc * 2 * sizeof(int32_t));
    if (!p) return -1;
    e->uv = p;
    e->cap = nc;
  }
  e->uv[2 * e->len] = (int32_t)u;
  e->uv[2 * e->len + 1] = (int32_t)v;
  e->len++;
  return 0;
}

/* ---------------------------------------------------------------- graph */
typedef struct {
  int64_t n, nnz;
  int64_t *off;
  int32_t *idx;
} gg_graph;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Build a simple symmetric CSR from an undirected edge list (any order,
 * duplicates and loops allowed; they are removed). */
static gg_graph *build_csr(int64_t n, const edgebuf *e) {
  gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
  if (!g) return NULL;
  g->n = n;
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) { free(g); return NULL; }
  for (int64_t i = 0; i < e->len; i++) {
    int32_t u = e->uv[2 * i], v = e->uv[2 * i + 1];
    if (u == v) continue;
    cnt[u + 1]++;
    cnt[v + 1]++;
  }
  for (int64_t i = 0; i < n; i++) cnt[i + 1] += cnt[i];
  int64_t tot = cnt[n];
  int32_t *tmp = (int32_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
  int64_t *pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!tmp || !pos) { free(cnt); free(tmp); free(pos); free(g); return NULL; }
  memcpy(pos, cnt, (size_t)n * sizeof(int64_t));
  for (int64_t i = 0; i < e->len; i++) {
    int32_t u = e->uv[2 * i], v = e->uv[2 * i + 1];
    if (u == v) continue;
    tmp[pos[u]++] = v;
    tmp[pos[v]++] = u;
  }
  free(pos);
  g->off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!g->off) { free(cnt); free(tmp); free(g); return NULL; }
  int64_t w = 0;
  g->off[0] = 0;
  for (int64_t u = 0; u < n; u++) {
    int64_t b = cnt[u], en = cnt[u + 1];
    qsort(tmp + b, (size_t)(en - b), sizeof(int32_t), cmp_i32);
    int32_t last = -1;
    for (int64_t j = b; j < en; j++) {
      if (tmp[j] != last) { tmp[w++] = tmp[j]; last = tmp[j]; }
    }
    g->off[u + 1] = w;
  }
  free(cnt);
  g->nnz = w;
  g->idx = (int32_t *)realloc(tmp, (size_t)(w > 0 ? w : 1) * sizeof(int32_t));
  if (!g->idx) g->idx = tmp;
  return g;
}

/* ----------------------------------------------------------- permutation */
static int32_t *random_perm(int64_t n, uint64_t seed) {
  int32_t *p = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!p) return NULL;
  for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
  uint64_t s = sm64_stream(seed, 0xFEEDULL);
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = (int64_t)ubelow(&s, (uint64_t)i + 1);
    int32_t t = p[i]; p[i] = p[j]; p[j] = t;
  }
  return p;
}

static void relabel(edgebuf *e, const int32_t *perm) {
  for (int64_t i = 0; i < 2 * e->len; i++) e->uv[i] = perm[e->uv[i]];
}

/* Plant cliques of the given sizes on disjoint uniformly random vertices.
 * members (optional) receives the vertices, plant after plant. */
static int plant_cliques(edgebuf *e, int64_t n, const int32_t *sizes, int32_t nplants,
                         uint64_t seed, int32_t *members) {
  int64_t tot = 0;
  for (int32_t i = 0; i < nplants; i++) tot += sizes[i];
  if (tot > n) return -2;
  if (tot == 0) return 0;
  /* partial Fisher-Yates over a sparse swap map would save memory; a dense
   * array is fine for the sizes used here. */
  int32_t *p = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!p) return -1;
  for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
  uint64_t s = sm64_stream(seed, 0xC11CULL);
  for (int64_t i = 0; i < tot; i++) {
    int64_t j = i + (int64_t)ubelow(&s, (uint64_t)(n - i));
    int32_t t = p[i]; p[i] = p[j]; p[j] = t;
  }
  int64_t base = 0;
  for (int32_t c = 0; c < nplants; c++) {
    for (int32_t a = 0; a < sizes[c]; a++)
      for (int32_t b = a + 1; b < sizes[c]; b++)
        if (eb_push(e, p[base + a], p[base + b])) { free(p); return -1; }
    base += sizes[c];
  }
  if (members) memcpy(members, p, (size_t)tot * sizeof(int32_t));
  free(p);
  return 0;
}

static gg_graph *finish(int64_t n, edgebuf *e, const int32_t *plants, int32_t nplants,
                        uint64_t seed, int32_t permute, int32_t *members) {
  if (permute && n > 1) {
    int32_t *perm = random_perm(n, seed);
    if (!perm) return NULL;
    relabel(e, perm);
    free(perm);
  }
  if (plant_cliques(e, n, plants, nplants, seed, members)) return NULL;
  return build_csr(n, e);
}

/* -------------------------------------------------------------- models */

/* Chung-Lu weights w_i = w_max * ((i + i0) / i0)^(-1/(gamma-1)), i0 chosen by
 * bisection (on log i0) so that the mean weight is mean_deg. */
static double cl_mean(int64_t n, double gamma, double wmax, double i0) {
  double a = -1.0 / (gamma - 1.0), s = 0.0;
  for (int64_t i = 0; i < n; i++) s += wmax * pow((i + i0) / i0, a);
  return s / (double)n;
}

int gg_chung_lu_weights(int64_t n, double gamma, double mean_deg, double wmax, double *w) {
  if (n <= 0 || gamma <= 1.0 || mean_deg <= 0 || wmax < mean_deg) return -1;
  double lo = -30.0, hi = 40.0; /* log i0 */
  for (int it = 0; it < 200; it++) {
    double mid = 0.5 * (lo + hi);
    if (cl_mean(n, gamma, wmax, exp(mid)) < mean_deg) lo = mid; else hi = mid;
  }
  double i0 = exp(0.5 * (lo + hi)), a = -1.0 / (gamma - 1.0);
  for (int64_t i = 0; i < n; i++) w[i] = wmax * pow((i + i0) / i0, a);
  return 0;
}

static int chung_lu_edges(int64_t n, const double *w, uint64_t seed, edgebuf *e) {
  double S = 0.0;
  for (int64_t i = 0; i < n; i++) S += w[i];
  if (S <= 0) return 0;
  for (int64_t u = 0; u + 1 < n; u++) {
    uint64_t s = sm64_stream(seed, (uint64_t)u);
    int64_t v = u + 1;
    double p = fmin(w[u] * w[v] / S, 1.0);
    while (v < n && p > 0.0) {
      if (p < 1.0) {
        double r = u01_open0(&s);
        double skip = floor(log(r) / log1p(-p));
        if (skip >= (double)(n - v)) break;
        v += (int64_t)skip;
      }
      if (v >= n) break;
      double q = fmin(w[u] * w[v] / S, 1.0);
      if (u01(&s) < q / p)
        if (eb_push(e, u, v)) return -1;
      p = q;
      v++;
    }
  }
  return 0;
}

static int gnp_edges(int64_t n, double p, uint64_t seed, edgebuf *e) {
  if (p <= 0.0 || n < 2) return 0;
  uint64_t s = sm64_stream(seed, 0x6E70ULL);
  if (p >= 1.0) {
    for (int64_t u = 1; u < n; u++)
      for (int64_t v = 0; v < u; v++)
        if (eb_push(e, u, v)) return -1;
    return 0;
  }
  /* walk the lower triangle (u > w) in row-major order with geometric gaps */
  double lq = log1p(-p);
  int64_t u = 1, w = -1;
  while (u < n) {
    double r = u01_open0(&s);
    w += 1 + (int64_t)floor(log(r) / lq);
    while (w >= u && u < n) { w -= u; u++; }
    if (u < n)
      if (eb_push(e, u, w)) return -1;
  }
  return 0;
}

static int rmat_edges(int32_t scale, int64_t nsamples, double a, double b, double c,
                      uint64_t seed, edgebuf *e) {
  double ab = a + b, abc = a + b + c;
  for (int64_t i = 0; i < nsamples; i++) {
    uint64_t s = sm64_stream(seed, (uint64_t)i);
    int64_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; l++) {
      double r = u01(&s);
      int bu = 0, bv = 0;
      if (r < a) { }
      else if (r < ab) bv = 1;
      else if (r < abc) bu = 1;
      else { bu = 1; bv = 1; }
      u = (u << 1) | bu;
      v = (v << 1) | bv;
    }
    if (eb_push(e, u, v)) return -1;
  }
  return 0;
}

/* ---------------------------------------------------------------- API */

void *gg_chung_lu(int64_t n, double gamma, double mean_deg, double wmax, uint64_t seed,
                  const int32_t *plants, int32_t nplants, int32_t *members) {
  if (n <= 0 || n >= (1LL << 31)) return NULL;
  double *w = (double *)malloc((size_t)n * sizeof(double));
  if (!w) return NULL;
  if (gg_chung_lu_weights(n, gamma, mean_deg, wmax, w)) { free(w); return NULL; }
  edgebuf e = {0, 0, NULL};
  if (chung_lu_edges(n, w, seed, &e)) { free(w); free(e.uv); return NULL; }
  free(w);
  gg_graph *g = finish(n, &e, plants, nplants, seed, 1, members);
  free(e.uv);
  return g;
}

void *gg_gnp(int64_t n, double p, uint64_t seed, const int32_t *plants, int32_t nplants,
             int32_t *members) {
  if (n < 0 || n >= (1LL << 31)) return NULL;
  edgebuf e = {0, 0, NULL};
  if (gnp_edges(n, p, seed, &e)) { free(e.uv); return NULL; }
  gg_graph *g = finish(n, &e, plants, nplants, seed, 1, members);
  free(e.uv);
  return g;
}

void *gg_rmat(int32_t scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
              const int32_t *plants, int32_t nplants, int32_t *members) {
  if (scale < 1 || scale > 30) return NULL;
  int64_t n = 1LL << scale;
  edgebuf e = {0, 0, NULL};
  if (rmat_edges(scale, edge_factor * n, a, b, c, seed, &e)) { free(e.uv); return NULL; }
  gg_graph *g = finish(n, &e, plants, nplants, seed, 1, members);
  free(e.uv);
  return g;
}

/* Simple graph from an explicit undirected edge list (pairs). */
void *gg_from_edges(int64_t n, const int32_t *uv, int64_t m) {
  edgebuf e = {0, 0, NULL};
  for (int64_t i = 0; i < m; i++) {
    if (uv[2 * i] < 0 || uv[2 * i] >= n || uv[2 * i + 1] < 0 || uv[2 * i + 1] >= n) {
      free(e.uv);
      return NULL;
    }
    if (eb_push(&e, uv[2 * i], uv[2 * i + 1])) { free(e.uv); return NULL; }
  }
  gg_graph *g = build_csr(n, &e);
  free(e.uv);
  return g;
}

int64_t gg_n(void *h) { return ((gg_graph *)h)->n; }
int64_t gg_nnz(void *h) { return ((gg_graph *)h)->nnz; }
void gg_copy(void *h, int64_t *off, int32_t *idx) {
  gg_graph *g = (gg_graph *)h;
  memcpy(off, g->off, ((size_t)g->n + 1) * sizeof(int64_t));
  if (g->nnz) memcpy(idx, g->idx, (size_t)g->nnz * sizeof(int32_t));
}
void gg_free(void *h) {
  gg_graph *g = (gg_graph *)h;
  if (!g) return;
  free(g->off);
  free(g->idx);
  free(g);
}
