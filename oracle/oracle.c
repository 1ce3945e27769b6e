/*
 * CPU oracle for the adaptive load balancer (ALB) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may call,
 * link or load this file; only the test suite, the smoke check and the CPU
 * baseline of the benchmark do.  It shares no code with the GPU library.
 *
 * What the path computes, and where the paper defines it
 * (Jatala et al., "An Adaptive Load Balancer For Graph Analytics on GPUs"):
 *
 *  - Section 2 (Background): labels are updated by an operator applied to
 *    active vertices until quiescence; push operators update neighbours.
 *    ALB only changes which thread applies the operator to which edge
 *    (Algorithm 2), so for the monotone push operators the converged labels
 *    are the plain results below:
 *      bfs  : hop distance from the source (FIFO queue search),
 *      sssp : shortest path distance with non-negative integer weights
 *             (Dijkstra with a binary heap and lazy deletion, int64 sums),
 *      cc   : weakly connected components, labelled by the minimum vertex id
 *             (union-find: union by size, path halving),
 *      pr   : PageRank by synchronous (Jacobi) power iteration in fp64.
 *    The paper names the applications (Section 5) but prints no formulas;
 *    the textbook definitions are used.
 *
 *  - Algorithm 1 (inspection): a frontier vertex with out-degree >= THRESHOLD
 *    is pushed to the huge worklist `work`; any other vertex is sent to the
 *    thread / warp / CTA bin of TWC by its degree (Section 3, TWC).
 *  - Section 4.1 (Search): `prefixWork` is the prefix sum of the out-degrees
 *    of the vertices in `work`; the source of edge k is found by a binary
 *    search in it.
 *  - Section 4.1 (Distribution): cyclic assigns edge k to thread k mod p;
 *    blocked assigns each thread one contiguous chunk.
 *
 * Integer results are exact.  Unreachable distances are INT32_MAX.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_INF INT32_MAX

/* ------------------------------------------------------------------ */
/* BFS: level[s] = 0, every other vertex INF; a FIFO queue visits vertices in
 * order of hop distance and sets each newly seen neighbour to level + 1.    */
/* ------------------------------------------------------------------ */
int oracle_bfs(int32_t n, const int32_t *off, const int32_t *col, int32_t src, int32_t *level) {
  if (n < 1 || src < 0 || src >= n) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -2;
  for (int32_t v = 0; v < n; ++v) level[v] = ORACLE_INF;
  int64_t head = 0, tail = 0;
  level[src] = 0;
  queue[tail++] = src;
  while (head < tail) {
    int32_t u = queue[head++];
    for (int32_t p = off[u]; p < off[u + 1]; ++p) {
      int32_t v = col[p];
      if (level[v] == ORACLE_INF) {
        level[v] = level[u] + 1;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return 0;
}

/* ------------------------------------------------------------------ */
/* SSSP: Dijkstra.  A binary min-heap of (distance, vertex) entries; a popped
 * entry whose distance is stale (larger than the settled one) is skipped.   */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t d;
  int32_t v;
} heap_item;

static void heap_push(heap_item *h, int64_t *size, heap_item x) {
  int64_t i = (*size)++;
  while (i > 0) {
    int64_t parent = (i - 1) / 2;
    if (h[parent].d <= x.d) break;
    h[i] = h[parent];
    i = parent;
  }
  h[i] = x;
}

static heap_item heap_pop(heap_item *h, int64_t *size) {
  heap_item top = h[0];
  heap_item last = h[--(*size)];
  int64_t i = 0, n = *size;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= n) break;
    if (c + 1 < n && h[c + 1].d < h[c].d) c++;
    if (last.d <= h[c].d) break;
    h[i] = h[c];
    i = c;
  }
  if (n > 0) h[i] = last;
  return top;
}

int oracle_sssp(int32_t n, const int32_t *off, const int32_t *col, const int32_t *w, int32_t src, int32_t *dist) {
  if (n < 1 || src < 0 || src >= n) return -1;
  int64_t m = off[n];
  int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  /* every push follows a strict improvement, so at most m + 1 pushes happen */
  heap_item *h = (heap_item *)malloc(sizeof(heap_item) * (size_t)(m + 1));
  if (!d || !h) { free(d); free(h); return -2; }
  for (int32_t v = 0; v < n; ++v) d[v] = INT64_MAX;
  int64_t size = 0;
  d[src] = 0;
  heap_push(h, &size, (heap_item){0, src});
  while (size > 0) {
    heap_item it = heap_pop(h, &size);
    if (it.d > d[it.v]) continue; /* stale entry */
    int32_t u = it.v;
    for (int32_t p = off[u]; p < off[u + 1]; ++p) {
      int32_t v = col[p];
      int64_t nd = it.d + (int64_t)w[p];
      if (nd < d[v]) {
        d[v] = nd;
        heap_push(h, &size, (heap_item){nd, v});
      }
    }
  }
  int rc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (d[v] == INT64_MAX)
      dist[v] = ORACLE_INF;
    else if (d[v] >= ORACLE_INF) {
      dist[v] = ORACLE_INF;
      rc = -3; /* a distance does not fit int32 */
    } else
      dist[v] = (int32_t)d[v];
  }
  free(d);
  free(h);
  return rc;
}

/* ------------------------------------------------------------------ */
/* CC: union-find over every directed edge (so components are the weakly
 * connected ones), union by size, path halving.  Each vertex is labelled with
 * the smallest vertex id of its component.                                  */
/* ------------------------------------------------------------------ */
static int32_t uf_find(int32_t *parent, int32_t x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

int oracle_cc(int32_t n, const int32_t *off, const int32_t *col, int32_t *label) {
  if (n < 1) return -1;
  int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *size = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *minid = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!parent || !size || !minid) { free(parent); free(size); free(minid); return -2; }
  for (int32_t v = 0; v < n; ++v) {
    parent[v] = v;
    size[v] = 1;
  }
  for (int32_t u = 0; u < n; ++u) {
    for (int32_t p = off[u]; p < off[u + 1]; ++p) {
      int32_t a = uf_find(parent, u), b = uf_find(parent, col[p]);
      if (a == b) continue;
      if (size[a] < size[b]) { int32_t t = a; a = b; b = t; }
      parent[b] = a;
      size[a] += size[b];
    }
  }
  for (int32_t v = 0; v < n; ++v) minid[v] = ORACLE_INF;
  for (int32_t v = 0; v < n; ++v) {
    int32_t r = uf_find(parent, v);
    if (v < minid[r]) minid[r] = v;
  }
  for (int32_t v = 0; v < n; ++v) label[v] = minid[uf_find(parent, v)];
  free(parent);
  free(size);
  free(minid);
  return 0;
}

/* ------------------------------------------------------------------ */
/* The undirected graph of a CSR: both directions of every edge, self-loops
 * and duplicates dropped, each row sorted.  Two calls: with out_col == NULL
 * only the row lengths (out_off) are computed; then the columns. */
static int cmp_i32(const void *a, const void *b) {
  const int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

int64_t oracle_symmetrise(int32_t n, const int32_t *off, const int32_t *col, int64_t *out_off, int32_t *out_col) {
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
  for (int32_t u = 0; u < n; ++u)
    for (int32_t p = off[u]; p < off[u + 1]; ++p) {
      ++cnt[u + 1];
      ++cnt[col[p] + 1];
    }
  for (int32_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  const int64_t total = cnt[n];
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!tmp || !cur) { free(cnt); free(tmp); free(cur); return -2; }
  for (int32_t v = 0; v < n; ++v) cur[v] = cnt[v];
  for (int32_t u = 0; u < n; ++u)
    for (int32_t p = off[u]; p < off[u + 1]; ++p) {
      const int32_t v = col[p];
      tmp[cur[u]++] = v;
      tmp[cur[v]++] = u;
    }
  int64_t m = 0;
  out_off[0] = 0;
  for (int32_t v = 0; v < n; ++v) {
    int32_t *row = tmp + cnt[v];
    const int64_t len = cnt[v + 1] - cnt[v];
    qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
    for (int64_t i = 0; i < len; ++i) {
      if (row[i] == v || (i > 0 && row[i] == row[i - 1])) continue;
      if (out_col) out_col[m] = row[i];
      ++m;
    }
    out_off[v + 1] = m;
  }
  free(cnt);
  free(tmp);
  free(cur);
  return m;
}

/* ------------------------------------------------------------------ */
/* k-core (the paper's kcore application, Section 5): the k-core of an
 * undirected graph is its largest subgraph in which every vertex has at least
 * k neighbours.  Peeling: every vertex of degree < k is removed; removing a
 * vertex lowers its neighbours' degrees; a neighbour whose degree falls
 * below k is removed in turn, until none is left to remove.  The input is
 * the symmetric CSR (both directions of every edge, no self-loops);
 * in_core[v] = 1 for the vertices that remain, else 0.
 * ------------------------------------------------------------------ */
int oracle_kcore(int32_t n, const int32_t *off, const int32_t *col, int32_t k, int32_t *in_core) {
  if (n < 1 || k < 0) return -1;
  int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!deg || !queue) { free(deg); free(queue); return -2; }
  int64_t head = 0, tail = 0;
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = off[v + 1] - off[v];
    in_core[v] = 1;
    if (deg[v] < k) {
      in_core[v] = 0;
      queue[tail++] = v;
    }
  }
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int32_t p = off[u]; p < off[u + 1]; ++p) {
      const int32_t v = col[p];
      if (!in_core[v]) continue;
      if (--deg[v] < k) {
        in_core[v] = 0;
        queue[tail++] = v;
      }
    }
  }
  free(deg);
  free(queue);
  return 0;
}

/* ------------------------------------------------------------------ */
/* PageRank, fp64, synchronous iteration with uniform teleport and the rank
 * of dangling vertices (out-degree 0) spread uniformly:
 *   x_0(v) = 1/N
 *   x_{t+1}(v) = (1-d)/N + d * ( sum_{(u,v) in E} x_t(u)/outdeg(u) + D_t/N ),
 *   D_t = sum_{outdeg(u)=0} x_t(u),
 * for exactly `iters` iterations.  The sum over in-edges of v is taken in
 * ascending order of the source u, from a transposed copy of the CSR, so the
 * result does not depend on the thread count (OpenMP over v when threads>1).
 * ------------------------------------------------------------------ */
int oracle_pagerank(int32_t n, const int32_t *off, const int32_t *col, double d, int32_t iters, int32_t threads,
                    double *x) {
  if (n < 1 || iters < 0 || !(d > 0.0 && d < 1.0)) return -1;
  int64_t m = off[n];
  int64_t *toff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *tsrc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  double *contrib = (double *)malloc(sizeof(double) * (size_t)n);
  double *nx = (double *)malloc(sizeof(double) * (size_t)n);
  if (!toff || !tsrc || !cur || !contrib || !nx) {
    free(toff); free(tsrc); free(cur); free(contrib); free(nx);
    return -2;
  }
  /* transpose: in-edges of v grouped, in ascending source order */
  for (int64_t p = 0; p < m; ++p) toff[col[p] + 1]++;
  for (int32_t v = 0; v < n; ++v) toff[v + 1] += toff[v];
  memcpy(cur, toff, sizeof(int64_t) * (size_t)n);
  for (int32_t u = 0; u < n; ++u)
    for (int32_t p = off[u]; p < off[u + 1]; ++p) tsrc[cur[col[p]]++] = u;
#ifdef _OPENMP
  if (threads < 1) threads = 1;
#endif
  const double N = (double)n;
  for (int32_t v = 0; v < n; ++v) x[v] = 1.0 / N;
  for (int32_t it = 0; it < iters; ++it) {
    double dangling = 0.0;
    for (int32_t u = 0; u < n; ++u) {
      int32_t deg = off[u + 1] - off[u];
      if (deg == 0) {
        dangling += x[u];
        contrib[u] = 0.0;
      } else {
        contrib[u] = x[u] / (double)deg;
      }
    }
    const double base = (1.0 - d) / N + d * dangling / N;
#pragma omp parallel for schedule(dynamic, 4096) num_threads(threads)
    for (int32_t v = 0; v < n; ++v) {
      double s = 0.0;
      for (int64_t q = toff[v]; q < toff[v + 1]; ++q) s += contrib[tsrc[q]];
      nx[v] = base + d * s;
    }
    memcpy(x, nx, sizeof(double) * (size_t)n);
  }
  free(toff); free(tsrc); free(cur); free(contrib); free(nx);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, inspection.  For frontier entry i (vertex v = frontier[i]):
 *   bin[i] = 3 (huge)   if deg(v) >= threshold and deg(v) >= 1
 *            2 (CTA)    else if deg(v) >= cta_cutoff
 *            1 (warp)   else if deg(v) >= warp_cutoff
 *            0 (thread) otherwise.
 * Huge vertices are appended to `work` in frontier order; *nwork is their
 * count.  A zero-degree vertex has no edge to distribute and is never huge
 * (this is the reading taken for threshold 0, where the paper places every
 * vertex in the huge bin).                                                  */
/* ------------------------------------------------------------------ */
int64_t oracle_inspect(int64_t nf, const int32_t *frontier, const int32_t *off, int64_t threshold,
                       int64_t warp_cutoff, int64_t cta_cutoff, int8_t *bin, int32_t *work) {
  int64_t nwork = 0;
  for (int64_t i = 0; i < nf; ++i) {
    int32_t v = frontier[i];
    int64_t deg = (int64_t)off[v + 1] - off[v];
    int8_t b;
    if (deg >= threshold && deg >= 1) {
      b = 3;
      work[nwork++] = v;
    } else if (deg >= cta_cutoff) {
      b = 2;
    } else if (deg >= warp_cutoff) {
      b = 1;
    } else {
      b = 0;
    }
    bin[i] = b;
  }
  return nwork;
}

/* prefixWork: exclusive prefix sum of the out-degrees of work[0..nwork-1];
 * prefix has nwork + 1 entries and prefix[nwork] is the total huge edge count. */
void oracle_prefix_work(int64_t nwork, const int32_t *work, const int32_t *off, int64_t *prefix) {
  prefix[0] = 0;
  for (int64_t j = 0; j < nwork; ++j) prefix[j + 1] = prefix[j] + ((int64_t)off[work[j] + 1] - off[work[j]]);
}

/* Source search: the huge-list index s whose edge range [prefix[s], prefix[s+1])
 * holds edge k, i.e. the last s with prefix[s] <= k (binary search). */
int64_t oracle_owner(int64_t nwork, const int64_t *prefix, int64_t k) {
  int64_t lo = 0, hi = nwork; /* answer in [0, nwork) */
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if (prefix[mid] <= k)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

/* Distribution (Section 4.1).  Thread that handles huge edge k out of w with p
 * threads: cyclic gives k mod p; blocked gives k / ceil(w / p). */
int64_t oracle_cyclic_thread(int64_t k, int64_t p) { return k % p; }
int64_t oracle_blocked_thread(int64_t k, int64_t w, int64_t p) {
  int64_t c = (w + p - 1) / p;
  return k / c;
}

/* Algorithm 2 for every huge edge k in [0, w): its source vertex, its CSR
 * position and the thread that processes it under the cyclic distribution. */
void oracle_lb_edges(int64_t nwork, const int32_t *work, const int64_t *prefix, const int32_t *off, int64_t p,
                     int32_t *src, int64_t *pos, int64_t *thread) {
  int64_t w = prefix[nwork];
  for (int64_t k = 0; k < w; ++k) {
    int64_t s = oracle_owner(nwork, prefix, k);
    src[k] = work[s];
    pos[k] = (int64_t)off[work[s]] + (k - prefix[s]);
    thread[k] = oracle_cyclic_thread(k, p);
  }
}
