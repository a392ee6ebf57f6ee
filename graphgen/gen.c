/*
 * Seeded synthetic graph generators and CSR/CSC construction.
 *
 * This file holds input preparation only: random graph families (R-MAT,
 * 2-D lattice with deletions and shortcuts, Erdos-Renyi G(n,m)), vertex
 * relabelling, edge-list -> CSR conversion, transposition and the largest
 * weakly connected component.  It contains none of the breadth-first-search
 * arithmetic; both the HIP library's tests/benchmarks and the CPU oracle read
 * the graphs it writes.
 *
 * Random numbers are counter based: value i of stream s under seed k is
 * splitmix64(splitmix64(k ^ s*phi) + (i+1)*phi), where splitmix64 is the
 * finaliser published by Steele, Lea and Flood ("Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Every output therefore
 * depends only on (seed, stream, index), never on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PHI 0x9e3779b97f4a7c15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static inline uint64_t rng_at(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64(mix64(seed ^ (stream * PHI)) + (i + 1) * PHI);
}

static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

/* Uniform integer in [0, bound) by 128-bit multiply-shift (Lemire 2019). */
static inline uint64_t below(uint64_t x, uint64_t bound) {
  return (uint64_t)(((__uint128_t)x * bound) >> 64);
}

uint64_t gg_rng(uint64_t seed, uint64_t stream, uint64_t i) { return rng_at(seed, stream, i); }

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each of m tuples descends
 * `scale` levels of the adjacency matrix, picking quadrant (0,0),(0,1),(1,0),
 * (1,1) with probabilities a, b, c, 1-a-b-c.  Bit `scale-1-l` of the source
 * and destination is set at level l. */
void gg_rmat_edges(int32_t scale, int64_t m, double a, double b, double c,
                   uint64_t seed, int32_t *src, int32_t *dst) {
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    uint32_t s = 0, d = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double r = u01(rng_at(seed, 1, (uint64_t)i * (uint64_t)scale + (uint64_t)l));
      uint32_t bs = (r >= ab) ? 1u : 0u;
      uint32_t bd = (r >= a && r < ab) || (r >= abc) ? 1u : 0u;
      s = (s << 1) | bs;
      d = (d << 1) | bd;
    }
    src[i] = (int32_t)s;
    dst[i] = (int32_t)d;
  }
}

/* Uniform random permutation of [0,n) by Fisher-Yates with stream 2. */
void gg_permutation(int64_t n, uint64_t seed, int32_t *perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)below(rng_at(seed, 2, (uint64_t)i), (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

void gg_apply_perm(int64_t m, const int32_t *perm, int32_t *ids) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) ids[i] = perm[ids[i]];
}

/* side x side 4-neighbour lattice.  Vertex (r,c) has id r*side+c.  Lattice
 * edge e (horizontal ones first, then vertical ones) is deleted when its
 * stream-3 uniform draw is below p_delete.  Then `shortcuts` uniform random
 * pairs (stream 4) are appended.  Returns the number of tuples written. */
int64_t gg_lattice_edges(int32_t side, double p_delete, int64_t shortcuts,
                         uint64_t seed, int32_t *src, int32_t *dst) {
  const int64_t L = side;
  const int64_t nh = L * (L - 1);      /* horizontal edges */
  const int64_t ne = 2 * nh;           /* all lattice edges */
  int64_t w = 0;
  for (int64_t e = 0; e < ne; ++e) {
    if (u01(rng_at(seed, 3, (uint64_t)e)) < p_delete) continue;
    int64_t u, v;
    if (e < nh) {
      int64_t r = e / (L - 1), c = e % (L - 1);
      u = r * L + c; v = u + 1;
    } else {
      int64_t f = e - nh;
      int64_t r = f / L, c = f % L;
      u = r * L + c; v = u + L;
    }
    src[w] = (int32_t)u; dst[w] = (int32_t)v; ++w;
  }
  const uint64_t n = (uint64_t)(L * L);
  for (int64_t j = 0; j < shortcuts; ++j) {
    src[w] = (int32_t)below(rng_at(seed, 4, 2 * (uint64_t)j), n);
    dst[w] = (int32_t)below(rng_at(seed, 4, 2 * (uint64_t)j + 1), n);
    ++w;
  }
  return w;
}

/* G(n,m): m uniform ordered pairs (stream 5). */
void gg_uniform_pairs(int64_t n, int64_t m, uint64_t seed, uint64_t stream,
                      int32_t *src, int32_t *dst) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    src[i] = (int32_t)below(rng_at(seed, stream, 2 * (uint64_t)i), (uint64_t)n);
    dst[i] = (int32_t)below(rng_at(seed, stream, 2 * (uint64_t)i + 1), (uint64_t)n);
  }
}

static int cmp_i32(const void *x, const void *y) {
  int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
  return (a > b) - (a < b);
}

static void sort_row(int32_t *p, int64_t len) {
  if (len < 24) {
    for (int64_t i = 1; i < len; ++i) {
      int32_t k = p[i];
      int64_t j = i - 1;
      while (j >= 0 && p[j] > k) { p[j + 1] = p[j]; --j; }
      p[j + 1] = k;
    }
  } else {
    qsort(p, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

/*
 * Edge list -> CSR with rows sorted ascending.
 *   symmetrize: add (d,s) for each (s,d)
 *   drop_self:  drop tuples with s == d
 *   dedup:      keep one copy of repeated (s,d)
 * row_ptr must hold n+1 entries; col must hold (symmetrize ? 2m : m).
 * Returns nnz, or -1 when nnz would not fit int32.
 */
int64_t gg_build_csr(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     int32_t symmetrize, int32_t drop_self, int32_t dedup,
                     int32_t *row_ptr, int32_t *col) {
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[i], d = dst[i];
    if (drop_self && s == d) continue;
#pragma omp atomic
    cnt[s + 1]++;
    if (symmetrize) {
#pragma omp atomic
      cnt[d + 1]++;
    }
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  const int64_t total = cnt[n];
  int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!cur) { free(cnt); return -2; }
  memcpy(cur, cnt, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[i], d = dst[i];
    if (drop_self && s == d) continue;
    int64_t p;
#pragma omp atomic capture
    p = cur[s]++;
    col[p] = d;
    if (symmetrize) {
#pragma omp atomic capture
      p = cur[d]++;
      col[p] = s;
    }
  }
  free(cur);
  /* Sort each row, then deduplicate in place; the kept length goes to deg. */
  int64_t *deg = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  if (!deg) { free(cnt); return -2; }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < n; ++v) {
    int32_t *p = col + cnt[v];
    int64_t len = cnt[v + 1] - cnt[v];
    sort_row(p, len);
    if (dedup && len > 1) {
      int64_t k = 1;
      for (int64_t j = 1; j < len; ++j)
        if (p[j] != p[k - 1]) p[k++] = p[j];
      len = k;
    }
    deg[v] = len;
  }
  /* Compact rows to the front (sequential: each row moves left only). */
  int64_t w = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t beg = cnt[v], len = deg[v];
    if (w != beg) memmove(col + w, col + beg, (size_t)len * sizeof(int32_t));
    if (w > INT32_MAX) { free(cnt); free(deg); return -1; }
    row_ptr[v] = (int32_t)w;
    w += len;
  }
  free(cnt);
  free(deg);
  if (w > INT32_MAX) return -1;
  row_ptr[n] = (int32_t)w;
  (void)total;
  return w;
}

/* CSC of a CSR (the transpose); columns within each CSC row ascend because
 * rows are visited in ascending order. */
void gg_transpose(int64_t n, const int32_t *row_ptr, const int32_t *col,
                  int32_t *t_ptr, int32_t *t_col) {
  int64_t nnz = row_ptr[n];
  int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t j = 0; j < nnz; ++j) cnt[col[j] + 1]++;
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  for (int64_t v = 0; v <= n; ++v) t_ptr[v] = (int32_t)cnt[v];
  for (int64_t u = 0; u < n; ++u)
    for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
      t_col[cnt[col[j]]++] = (int32_t)u;
  free(cnt);
}

static int64_t uf_find(int64_t *p, int64_t x) {
  while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
  return x;
}

/* Marks (mask[v]=1) the vertices of the largest weakly connected component,
 * by union-find with path halving and union by size.  Returns its size. */
int64_t gg_largest_component(int64_t n, const int32_t *row_ptr, const int32_t *col,
                             uint8_t *mask) {
  int64_t *p = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  int64_t *sz = (int64_t *)malloc((size_t)n * sizeof(int64_t));
  for (int64_t v = 0; v < n; ++v) { p[v] = v; sz[v] = 1; }
  for (int64_t u = 0; u < n; ++u)
    for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
      int64_t a = uf_find(p, u), b = uf_find(p, col[j]);
      if (a == b) continue;
      if (sz[a] < sz[b]) { int64_t t = a; a = b; b = t; }
      p[b] = a; sz[a] += sz[b];
    }
  int64_t best = 0, root = 0;
  for (int64_t v = 0; v < n; ++v)
    if (p[v] == v && sz[v] > best) { best = sz[v]; root = v; }
  for (int64_t v = 0; v < n; ++v) mask[v] = (uf_find(p, v) == root) ? 1 : 0;
  free(p); free(sz);
  return best;
}

/* Draws k distinct vertices uniformly (stream 6) from those with mask[v]=1
 * and at least two neighbours other than v itself.  Returns the number drawn
 * (less than k only if fewer candidates exist). */
int32_t gg_pick_sources(int64_t n, const int32_t *row_ptr, const int32_t *col,
                        const uint8_t *mask, int32_t k, uint64_t seed, int32_t *out) {
  int32_t *cand = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int64_t nc = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (!mask[v]) continue;
    int64_t d = 0;
    for (int64_t j = row_ptr[v]; j < row_ptr[v + 1] && d < 2; ++j)
      if (col[j] != v) ++d;
    if (d >= 2) cand[nc++] = (int32_t)v;
  }
  int32_t got = 0;
  uint64_t t = 0;
  while (got < k && (int64_t)got < nc) {
    int32_t v = cand[below(rng_at(seed, 6, t++), (uint64_t)nc)];
    int dup = 0;
    for (int32_t i = 0; i < got; ++i) if (out[i] == v) { dup = 1; break; }
    if (!dup) out[got++] = v;
  }
  free(cand);
  return got;
}
