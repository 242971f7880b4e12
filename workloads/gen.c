/*
 * Seeded synthetic graph workloads (input generation only).
 *
 * This file draws the inputs that both the plain CPU oracle and the GPU
 * library consume: R-MAT edge lists, a preferential-attachment temporal edge
 * stream and duplicate removal of raw edge draws.  It contains none of the
 * PageRank arithmetic.  Every random number comes from a counter-based
 * splitmix64 stream, so a draw depends only on (seed, stream, counter) and the
 * result is independent of the number of OpenMP threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ---- counter-based random numbers (splitmix64 output function) ---------- */
static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t ctr) {
  uint64_t s = mix64(seed * 0x9E3779B97F4A7C15ULL + mix64(stream + 0x632BE59BD9B4E019ULL));
  return mix64(s + (ctr + 1) * 0x9E3779B97F4A7C15ULL);
}
/* uniform integer in [0, k) by multiply-high (Lemire) */
static inline uint64_t below(uint64_t r, uint64_t k) {
  return (uint64_t)(((__uint128_t)r * (__uint128_t)k) >> 64);
}
static inline double unit(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/*
 * R-MAT draws.  Each draw descends `scale` levels; at each level the quadrant
 * (src bit, dst bit) is (0,0) w.p. a, (0,1) w.p. b, (1,0) w.p. c, (1,1)
 * otherwise.  Draws whose endpoints are >= n_limit are redrawn from the next
 * attempt counter.  Self-draws are kept here; gen_dedupe drops them.
 * If perm != NULL every endpoint x is relabelled to perm[x].
 */
void gen_rmat(int32_t scale, int64_t n_draws, int32_t n_limit, double a, double b,
              double c, uint64_t seed, const int32_t* perm, int32_t* src, int32_t* dst) {
  const uint64_t ta = (uint64_t)(a * 4294967296.0);
  const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
  const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
  const int64_t words = (scale + 1) / 2;
#pragma omp parallel for schedule(static, 65536)
  for (int64_t i = 0; i < n_draws; i++) {
    for (uint64_t attempt = 0;; attempt++) {
      uint64_t u = 0, v = 0;
      uint64_t base = ((uint64_t)i * 64 + attempt) * (uint64_t)words;
      for (int32_t lv = 0; lv < scale; lv++) {
        uint64_t w = rnd(seed, 1, base + (uint64_t)(lv >> 1));
        uint64_t r = (lv & 1) ? (w >> 32) : (w & 0xFFFFFFFFULL);
        uint64_t sb, db;
        if (r < ta) { sb = 0; db = 0; }
        else if (r < tb) { sb = 0; db = 1; }
        else if (r < tc) { sb = 1; db = 0; }
        else { sb = 1; db = 1; }
        u = (u << 1) | sb;
        v = (v << 1) | db;
      }
      if ((int64_t)u < n_limit && (int64_t)v < n_limit) {
        src[i] = perm ? perm[u] : (int32_t)u;
        dst[i] = perm ? perm[v] : (int32_t)v;
        break;
      }
      if (attempt == 63) { /* practically unreachable for n_limit >= 2^(scale-1) */
        src[i] = (int32_t)below(rnd(seed, 3, (uint64_t)i * 2), (uint64_t)n_limit);
        dst[i] = (int32_t)below(rnd(seed, 3, (uint64_t)i * 2 + 1), (uint64_t)n_limit);
        break;
      }
    }
  }
}

/* Seeded Fisher-Yates permutation of [0, n). */
void gen_permutation(int32_t n, uint64_t seed, int32_t* perm) {
  for (int32_t i = 0; i < n; i++) perm[i] = i;
  for (int32_t i = n - 1; i > 0; i--) {
    int32_t j = (int32_t)below(rnd(seed, 2, (uint64_t)i), (uint64_t)i + 1);
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

static int cmp_i32(const void* x, const void* y) {
  int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}

/*
 * Remove self-draws and duplicate (src,dst) pairs.  Output is sorted by
 * (src, dst).  `out_src`/`out_dst` need room for m pairs.  Returns the number
 * of distinct non-self pairs.  Scratch: counts (n+1) and a row buffer (m).
 */
int64_t gen_dedupe(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   int32_t* out_src, int32_t* out_dst) {
  int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int64_t* cur = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
  int64_t* kept = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* rows = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!start || !cur || !kept || !rows) { free(start); free(cur); free(kept); free(rows); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; i++) __atomic_fetch_add(&start[src[i] + 1], 1, __ATOMIC_RELAXED);
  for (int32_t u = 0; u < n; u++) start[u + 1] += start[u];
  memcpy(cur, start, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; i++) {
    int64_t p = __atomic_fetch_add(&cur[src[i]], 1, __ATOMIC_RELAXED);
    rows[p] = dst[i];
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; u++) {
    int64_t s = start[u], e = start[u + 1], k = s;
    if (e - s > 1) qsort(rows + s, (size_t)(e - s), sizeof(int32_t), cmp_i32);
    for (int64_t p = s; p < e; p++) {
      if (rows[p] == u) continue;
      if (k > s && rows[k - 1] == rows[p]) continue;
      rows[k++] = rows[p];
    }
    kept[u + 1] = k - s;
  }
  for (int32_t u = 0; u < n; u++) kept[u + 1] += kept[u];
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; u++) {
    int64_t s = start[u], o = kept[u], len = kept[u + 1] - kept[u];
    for (int64_t j = 0; j < len; j++) { out_src[o + j] = u; out_dst[o + j] = rows[s + j]; }
  }
  int64_t total = kept[n];
  free(start); free(cur); free(kept); free(rows);
  return total;
}

/*
 * Temporal edge stream by preferential attachment (Polya urn).
 * Vertices 0..n-1 arrive in order; arriving vertex u emits k ~ Poisson(mean)
 * edges.  Each edge is, with probability p_repeat, an exact copy of a
 * uniformly chosen earlier stream edge; otherwise it is (u, w) with w drawn
 * from an urn holding every arrived vertex once plus once per in-edge it has
 * received (redrawn while w == u).  After all n vertices have arrived, further
 * edges (up to `total`) come from uniformly chosen sources.  Endpoints are
 * relabelled through perm when perm != NULL.  Returns the number of edges
 * written (always `total` when n >= 2).
 */
int64_t gen_temporal(int32_t n, int64_t total, double mean_deg, double p_repeat,
                     uint64_t seed, const int32_t* perm, int32_t* src, int32_t* dst) {
  if (n < 2 || total <= 0) return 0;
  int32_t* urn = (int32_t*)malloc(((size_t)n + (size_t)total) * sizeof(int32_t));
  if (!urn) return -1;
  int64_t urn_len = 0, e = 0;
  uint64_t ctr = 0;
  const double el = exp(-mean_deg);
  int32_t arrived = 0;
  while (e < total) {
    int32_t u;
    int64_t k;
    if (arrived < n) {
      u = arrived++;
      urn[urn_len++] = u;
      double p = 1.0;
      k = -1;
      do { k++; p *= unit(rnd(seed, 4, ctr++)); } while (p > el);
    } else {
      u = (int32_t)below(rnd(seed, 4, ctr++), (uint64_t)n);
      k = 1;
    }
    for (int64_t j = 0; j < k && e < total; j++) {
      if (e > 0 && unit(rnd(seed, 5, ctr++)) < p_repeat) {
        int64_t q = (int64_t)below(rnd(seed, 6, ctr++), (uint64_t)e);
        src[e] = src[q]; dst[e] = dst[q];
        e++;
        continue;
      }
      if (urn_len < 2 && arrived < 2) continue;
      int32_t w;
      int tries = 0;
      do {
        w = urn[below(rnd(seed, 7, ctr++), (uint64_t)urn_len)];
      } while (w == u && ++tries < 64);
      if (w == u) continue;
      src[e] = u; dst[e] = w;
      urn[urn_len++] = w;
      e++;
    }
  }
  free(urn);
  if (perm) {
    for (int64_t i = 0; i < e; i++) { src[i] = perm[src[i]]; dst[i] = perm[dst[i]]; }
  }
  return e;
}
