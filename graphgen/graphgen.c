/*
 * Seeded synthetic graph generators (RMAT and capped-Zipf out-degree graphs).
 *
 * This module produces INPUTS only: it holds none of the traversal, load
 * balancing or label arithmetic that the library and the CPU oracle compute.
 * Both of those consume the CSR arrays built here.
 *
 * Randomness comes from one counter-based generator: value(seed, stream, i)
 * is the SplitMix64 finaliser (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) applied to a linear mix of
 * the key and the counter.  Every draw is addressed by its counter, so the
 * output does not depend on the thread count.
 *
 * Output graphs are CSR with int32 row offsets and int32 columns, rows sorted
 * by destination, with self-loops and duplicate edges removed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Counter-based draw: independent 64-bit values addressed by (seed, stream, i).
 * The key of a (seed, stream) pair is computed once per loop (draw_key), the
 * draw itself is one more finaliser call (draw_at). */
static inline uint64_t draw_key(uint64_t seed, uint64_t stream) {
  return mix64(seed * 0x9e3779b97f4a7c15ULL + stream * 0xd1b54a32d192ed03ULL + 0x632be59bd9b4e019ULL);
}
static inline uint64_t draw_at(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * 0x9e3779b97f4a7c15ULL); }

uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t i) { return draw_at(draw_key(seed, stream), i); }

/* Uniform double in [0, 1) with 53 random bits. */
static inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

/* Uniform integer in [0, n) by the multiply-high method on 32 bits (n < 2^32). */
static inline uint32_t below(uint64_t x, uint32_t n) { return (uint32_t)(((x >> 32) * (uint64_t)n) >> 32); }

typedef struct {
  int32_t n;
  int64_t m;
  int32_t *off; /* n + 1 */
  int32_t *col; /* m */
} gg_graph;

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->off);
  free(g->col);
  free(g);
}

int32_t gg_n(const gg_graph *g) { return g->n; }
int64_t gg_m(const gg_graph *g) { return g->m; }

/* Copy the CSR out into caller-owned arrays (off: n+1, col: m). */
void gg_fetch(const gg_graph *g, int32_t *off, int32_t *col) {
  memcpy(off, g->off, sizeof(int32_t) * ((size_t)g->n + 1));
  if (g->m) memcpy(col, g->col, sizeof(int32_t) * (size_t)g->m);
}

/* Ascending sort of non-negative int32 values: insertion sort for short rows,
 * else least-significant-digit radix sort (11-bit digits) through `tmp`. */
static void sort_row(int32_t *a, int64_t len, int32_t *tmp) {
  if (len <= 48) {
    for (int64_t i = 1; i < len; ++i) {
      int32_t x = a[i];
      int64_t j = i - 1;
      while (j >= 0 && a[j] > x) {
        a[j + 1] = a[j];
        --j;
      }
      a[j + 1] = x;
    }
    return;
  }
  uint32_t mx = 0;
  for (int64_t i = 0; i < len; ++i) mx |= (uint32_t)a[i];
  int32_t *src = a, *dst = tmp;
  for (int shift = 0; shift < 32 && (mx >> shift) != 0; shift += 11) {
    int64_t cnt[2048];
    memset(cnt, 0, sizeof cnt);
    for (int64_t i = 0; i < len; ++i) cnt[((uint32_t)src[i] >> shift) & 2047u]++;
    int64_t sum = 0;
    for (int k = 0; k < 2048; ++k) {
      int64_t c = cnt[k];
      cnt[k] = sum;
      sum += c;
    }
    for (int64_t i = 0; i < len; ++i) dst[cnt[((uint32_t)src[i] >> shift) & 2047u]++] = src[i];
    int32_t *t = src;
    src = dst;
    dst = t;
  }
  if (src != a) memcpy(a, src, sizeof(int32_t) * (size_t)len);
}

/*
 * Given raw rows (raw_off: n+1 int64 offsets into raw, unsorted, may hold
 * duplicates and self-loops), sort each row, drop self-loops and duplicates,
 * and build the final CSR.  raw is modified in place.  Returns NULL on
 * allocation failure or when the result would not fit int32 offsets.
 */
static gg_graph *finish_rows(int32_t n, const int64_t *raw_off, int32_t *raw) {
  int64_t *keep = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
  if (!keep) return NULL;
  int64_t maxlen = 0;
  for (int64_t v = 0; v < n; ++v) maxlen = raw_off[v + 1] - raw_off[v] > maxlen ? raw_off[v + 1] - raw_off[v] : maxlen;
  int failed = 0;
#pragma omp parallel
  {
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxlen ? maxlen : 1));
    if (!tmp) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
      int32_t *row = raw + raw_off[v];
      int64_t len = raw_off[v + 1] - raw_off[v];
      if (len > 1 && tmp) sort_row(row, len, tmp);
      int64_t w = 0;
      for (int64_t i = 0; i < len; ++i) {
        int32_t d = row[i];
        if (d == (int32_t)v) continue;
        if (w > 0 && row[w - 1] == d) continue;
        row[w++] = d;
      }
      keep[v] = w;
    }
    free(tmp);
  }
  if (failed) { free(keep); return NULL; }
  gg_graph *g = (gg_graph *)calloc(1, sizeof(gg_graph));
  if (!g) { free(keep); return NULL; }
  g->n = n;
  g->off = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  if (!g->off) { free(keep); gg_free(g); return NULL; }
  int64_t total = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (total > INT32_MAX) break;
    g->off[v] = (int32_t)total;
    total += keep[v];
  }
  if (total > INT32_MAX) { free(keep); gg_free(g); return NULL; }
  g->off[n] = (int32_t)total;
  g->m = total;
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total ? total : 1));
  if (!g->col) { free(keep); gg_free(g); return NULL; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v)
    memcpy(g->col + g->off[v], raw + raw_off[v], sizeof(int32_t) * (size_t)keep[v]);
  free(keep);
  return g;
}

/*
 * RMAT (Chakrabarti, Zhan and Faloutsos, SDM 2004), Graph500 style without
 * noise or vertex permutation: each of the ef * 2^scale edges picks one of
 * four quadrants per bit level with probabilities a, b, c and 1-a-b-c, from
 * the most significant bit down.  Vertex 0 is therefore the hub.
 */
static inline void rmat_edge(int scale, double a, double ab, double abc, uint64_t key, uint64_t i,
                             int32_t *s, int32_t *d) {
  uint32_t src = 0, dst = 0;
  for (int l = 0; l < scale; ++l) {
    double u = u01(draw_at(key, i * (uint64_t)scale + (uint64_t)l));
    uint32_t bs = 0, bd = 0;
    if (u < a) {
    } else if (u < ab) {
      bd = 1;
    } else if (u < abc) {
      bs = 1;
    } else {
      bs = 1;
      bd = 1;
    }
    src = (src << 1) | bs;
    dst = (dst << 1) | bd;
  }
  *s = (int32_t)src;
  *d = (int32_t)dst;
}

gg_graph *gg_rmat(int scale, int edge_factor, double a, double b, double c, uint64_t seed) {
  if (scale < 1 || scale > 30 || edge_factor < 1) return NULL;
  int32_t n = (int32_t)1 << scale;
  int64_t raw_m = (int64_t)edge_factor * (int64_t)n;
  double ab = a + b, abc = a + b + c;
  const uint64_t key = draw_key(seed, 1);
  int64_t *raw_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *es = (int32_t *)malloc(sizeof(int32_t) * (size_t)raw_m);
  int32_t *ed = (int32_t *)malloc(sizeof(int32_t) * (size_t)raw_m);
  if (!raw_off || !es || !ed) { free(raw_off); free(es); free(ed); return NULL; }
  /* pass 1: draw every edge, count raw out-degrees per source */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < raw_m; ++i) {
    rmat_edge(scale, a, ab, abc, key, (uint64_t)i, &es[i], &ed[i]);
    __atomic_fetch_add(&raw_off[es[i] + 1], 1, __ATOMIC_RELAXED);
  }
  for (int64_t v = 0; v < n; ++v) raw_off[v + 1] += raw_off[v];
  int32_t *raw = (int32_t *)malloc(sizeof(int32_t) * (size_t)raw_m);
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!raw || !cur) { free(raw_off); free(raw); free(cur); free(es); free(ed); return NULL; }
  memcpy(cur, raw_off, sizeof(int64_t) * (size_t)n);
  /* pass 2: scatter destinations into their rows (row order fixed by the sort below) */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < raw_m; ++i) {
    int64_t p = __atomic_fetch_add(&cur[es[i]], 1, __ATOMIC_RELAXED);
    raw[p] = ed[i];
  }
  free(cur);
  free(es);
  free(ed);
  gg_graph *g = finish_rows(n, raw_off, raw);
  free(raw_off);
  free(raw);
  return g;
}

/*
 * Out-degree law: P(k) proportional to k^-s for k >= 1 (Zipf), with every
 * draw above `cap` replaced by cap.  Inverse-CDF sampling against a table of
 * the cumulative probabilities for k = 1 .. cap-1; the remaining mass goes to
 * cap.  The normaliser zeta(s) is the direct sum up to cap-1 plus the
 * Euler-Maclaurin estimate of the tail from cap on.
 */
typedef struct {
  int64_t cap;
  double *cdf; /* cdf[k-1] = P(X <= k), k = 1 .. cap-1 */
} zipf_table;

static int zipf_init(zipf_table *z, double s, int64_t cap) {
  z->cap = cap;
  z->cdf = NULL;
  if (cap < 1 || s <= 1.0) return -1;
  if (cap == 1) return 0;
  z->cdf = (double *)malloc(sizeof(double) * (size_t)(cap - 1));
  if (!z->cdf) return -1;
  double capd = (double)cap;
  double tail = pow(capd, 1.0 - s) / (s - 1.0) + 0.5 * pow(capd, -s) + s * pow(capd, -s - 1.0) / 12.0;
  double head = 0.0;
  for (int64_t k = cap - 1; k >= 1; --k) head += pow((double)k, -s); /* small terms first */
  double zeta = head + tail;
  double acc = 0.0;
  for (int64_t k = 1; k < cap; ++k) {
    acc += pow((double)k, -s);
    z->cdf[k - 1] = acc / zeta;
  }
  return 0;
}

static inline int64_t zipf_sample(const zipf_table *z, double u) {
  if (z->cap == 1) return 1;
  /* smallest k with cdf[k-1] > u; cap if none */
  int64_t lo = 0, hi = z->cap - 1; /* search in cdf[0 .. cap-2] */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (z->cdf[mid] > u)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo + 1; /* lo == cap-1 means no entry exceeded u: value cap */
}

/* Out-degrees alone (before dedup), for tests of the sampler. */
int gg_zipf_degrees(int32_t n, double s, int64_t cap, uint64_t seed, int64_t *deg) {
  zipf_table z;
  if (zipf_init(&z, s, cap) != 0) return -1;
  const uint64_t key = draw_key(seed, 2);
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < n; ++v) deg[v] = zipf_sample(&z, u01(draw_at(key, (uint64_t)v)));
  free(z.cdf);
  return 0;
}

/*
 * Graph with capped-Zipf out-degrees and uniform random targets drawn with
 * replacement; self-loops and duplicates are then removed.
 */
gg_graph *gg_zipf(int32_t n, double s, int64_t cap, uint64_t seed) {
  if (n < 1) return NULL;
  int64_t *raw_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!raw_off) return NULL;
  if (gg_zipf_degrees(n, s, cap, seed, raw_off + 1) != 0) { free(raw_off); return NULL; }
  for (int64_t v = 0; v < n; ++v) raw_off[v + 1] += raw_off[v];
  int64_t raw_m = raw_off[n];
  int32_t *raw = (int32_t *)malloc(sizeof(int32_t) * (size_t)(raw_m ? raw_m : 1));
  if (!raw) { free(raw_off); return NULL; }
  const uint64_t key = draw_key(seed, 3);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v)
    for (int64_t p = raw_off[v]; p < raw_off[v + 1]; ++p) raw[p] = (int32_t)below(draw_at(key, (uint64_t)p), (uint32_t)n);
  gg_graph *g = finish_rows(n, raw_off, raw);
  free(raw_off);
  free(raw);
  return g;
}

/* Edge weights: uniform integers in [lo, hi] (inclusive), one draw per CSR position. */
void gg_uniform_weights(int64_t m, int32_t lo, int32_t hi, uint64_t seed, int32_t *w) {
  uint32_t span = (uint32_t)((int64_t)hi - (int64_t)lo + 1);
  const uint64_t key = draw_key(seed, 4);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) w[i] = lo + (int32_t)below(draw_at(key, (uint64_t)i), span);
}

/* Uniform integers in [0, n) (source draws and the like). */
void gg_uniform_ints(int64_t count, uint32_t n, uint64_t seed, uint64_t stream, int32_t *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = (int32_t)below(gg_draw(seed, 16 + stream, (uint64_t)i), n);
}

/* Uniform doubles in [0, 1). */
void gg_uniform_doubles(int64_t count, uint64_t seed, uint64_t stream, double *out) {
  for (int64_t i = 0; i < count; ++i) out[i] = u01(gg_draw(seed, 32 + stream, (uint64_t)i));
}
