/*
 * Plain FP64 CPU oracle for Static, Naive-dynamic (ND), Dynamic Frontier (DF)
 * and Dynamic Frontier with Pruning (DF-P) PageRank
 * (Sahu, "DF* PageRank", arXiv 2401.15870).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code with the GPU
 * library and is written to be read against the paper, not to be fast:
 * sets are sorted arrays, every sum is a left fold in ascending source order,
 * every per-edge contribution R[u]/|out(u)| is divided inline.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *  - Synchronous (Jacobi) iteration: every rank read in iteration i sees the
 *    ranks of iteration i; prunes and marks take effect in iteration i+1.
 *    The paper runs DF/DF-P asynchronously on one rank vector (Section 4.4);
 *    the fixed point, the formulas and the stop rule are the same.
 *  - Initial marking follows Algorithm 1 literally: for every edge (u,v) of
 *    the batch, all of out(u) in G^{t-1} and in G^t is marked, which includes
 *    u itself through its self-loop.
 *  - A pruned vertex may be re-marked by an expanding in-neighbour in the
 *    same iteration; marks win over prunes.
 *  - Prune iff relative change <= tau_p, expand iff > tau_f (Algorithm 1),
 *    relative change = |r - R[v]| / max(r, R[v]) (Section 4.2).
 *  - C0 = (1 - alpha)/|V| (Equation 1), not the garbled form in the appendix.
 *  - Batch semantics (Section 3.2): deletions and insertions are sets; the
 *    effective batch is Delta- = E^{t-1} \ E^t and Delta+ = E^t \ E^{t-1}.
 *    A pair both deleted and inserted is present in E^t.  Deleting a
 *    self-loop is ignored: every vertex keeps its self-loop (Section 5.1.3).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math, no
 * FMA contraction, IEEE binary64 round-to-nearest-even).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"

/* ------------------------------------------------------------------------ */
/* Edge sets as (src,dst) pairs sorted lexicographically, no duplicates.     */
/* ------------------------------------------------------------------------ */

static int cmp_pair(const void* x, const void* y) {
  const int32_t* a = (const int32_t*)x;
  const int32_t* b = (const int32_t*)y;
  if (a[0] != b[0]) return (a[0] > b[0]) - (a[0] < b[0]);
  return (a[1] > b[1]) - (a[1] < b[1]);
}
static int cmp_i32(const void* x, const void* y) {
  int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
  return (a > b) - (a < b);
}
static int pair_less(int32_t au, int32_t av, int32_t bu, int32_t bv) {
  return au < bu || (au == bu && av < bv);
}

/* Sort pairs (interleaved u,v), drop duplicates and self pairs (v,v).
 * Returns the new count; *n_self receives the number of distinct self pairs
 * that were dropped. */
static int64_t sort_unique_pairs(int32_t* pv, int64_t k, int64_t* n_self) {
  if (k > 1) qsort(pv, (size_t)k, 2 * sizeof(int32_t), cmp_pair);
  int64_t w = 0, selfs = 0;
  for (int64_t i = 0; i < k; i++) {
    const int32_t u = pv[2 * i], v = pv[2 * i + 1];
    /* pv[i-1] still holds input pair i-1: writes never pass the read index */
    if (i > 0 && pv[2 * (i - 1)] == u && pv[2 * (i - 1) + 1] == v) continue;
    if (u == v) { selfs++; continue; }
    pv[2 * w] = u;
    pv[2 * w + 1] = v;
    w++;
  }
  *n_self = selfs;
  return w;
}

/*
 * Canonical edge set of a graph: E = {(u,v) : input pairs} U {(v,v) : v in V},
 * sorted by (u,v) without duplicates.  Rows are gathered per source, sorted
 * and de-duplicated one by one (a counting sort by source followed by a sort
 * of each row), which is the plain definition of the sorted set.
 * esrc/edst need room for m + n pairs.  Returns |E|, or -1 if an id is out of
 * range, -2 on allocation failure.
 */
int64_t orc_canonical(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      int32_t* esrc, int32_t* edst) {
  for (int64_t i = 0; i < m; i++)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return -1;
  int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* rows = (int32_t*)malloc((size_t)(m + n) * sizeof(int32_t));
  if (!start || !rows) { free(start); free(rows); return -2; }
  for (int64_t i = 0; i < m; i++) start[src[i] + 1]++;
  for (int32_t v = 0; v < n; v++) start[v + 1] += 1; /* the self-loop */
  for (int32_t v = 0; v < n; v++) start[v + 1] += start[v];
  int64_t* fill = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!fill) { free(start); free(rows); return -2; }
  for (int32_t v = 0; v < n; v++) { fill[v] = start[v]; rows[fill[v]++] = v; }
  for (int64_t i = 0; i < m; i++) rows[fill[src[i]]++] = dst[i];
  int64_t out = 0;
  for (int32_t u = 0; u < n; u++) {
    int64_t s = start[u], e = start[u + 1];
    qsort(rows + s, (size_t)(e - s), sizeof(int32_t), cmp_i32);
    for (int64_t p = s; p < e; p++) {
      if (p > s && rows[p] == rows[p - 1]) continue;
      esrc[out] = u;
      edst[out] = rows[p];
      out++;
    }
  }
  free(fill); free(rows); free(start);
  return out;
}

/*
 * CSR of a canonical edge list (sorted by (src,dst)).
 * by_dst == 0: out-adjacency, row u lists out(u) ascending.
 * by_dst == 1: in-adjacency, row v lists in(v) ascending (a stable counting
 *              sort by destination of the (src,dst)-sorted list).
 * off has n+1 entries, idx has m entries.
 */
void orc_csr(int32_t n, int64_t m, const int32_t* esrc, const int32_t* edst, int by_dst,
             int32_t* off, int32_t* idx) {
  const int32_t* key = by_dst ? edst : esrc;
  const int32_t* val = by_dst ? esrc : edst;
  for (int32_t v = 0; v <= n; v++) off[v] = 0;
  for (int64_t i = 0; i < m; i++) off[key[i] + 1]++;
  for (int32_t v = 0; v < n; v++) off[v + 1] += off[v];
  int32_t* fill = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int32_t v = 0; v < n; v++) fill[v] = off[v];
  for (int64_t i = 0; i < m; i++) idx[fill[key[i]]++] = val[i];
  free(fill);
}

/*
 * Apply a batch update (Section 3.2).  The batch is read as two sets:
 *   Ins' = set(ins) minus self pairs,  Del' = set(del) minus self pairs.
 *   E^t  = (E^{t-1} \ Del') U Ins'            (self-loops stay on all vertices)
 *   Delta+ = E^t \ E^{t-1},  Delta- = E^{t-1} \ E^t   (the paper's definitions)
 * old: canonical E^{t-1} (sorted pairs).  new_src/new_dst need room for
 * m_old + n_ins pairs, dm_* for n_del, dp_* for n_ins.
 * info[5] = {ins_in, ins_effective, del_in, del_effective, self_loop_dels_ignored}.
 * Returns 0, -1 on an out-of-range id (nothing written), -2 on allocation failure.
 */
int orc_apply(int32_t n, int64_t m_old, const int32_t* osrc, const int32_t* odst,
              int64_t n_del, const int32_t* del_src, const int32_t* del_dst,
              int64_t n_ins, const int32_t* ins_src, const int32_t* ins_dst,
              int32_t* new_src, int32_t* new_dst, int64_t* m_new,
              int32_t* dm_src, int32_t* dm_dst, int64_t* n_dm,
              int32_t* dp_src, int32_t* dp_dst, int64_t* n_dp, int64_t* info) {
  for (int64_t i = 0; i < n_del; i++)
    if (del_src[i] < 0 || del_src[i] >= n || del_dst[i] < 0 || del_dst[i] >= n) return -1;
  for (int64_t i = 0; i < n_ins; i++)
    if (ins_src[i] < 0 || ins_src[i] >= n || ins_dst[i] < 0 || ins_dst[i] >= n) return -1;
  int32_t* D = (int32_t*)malloc((size_t)(2 * n_del + 2) * sizeof(int32_t));
  int32_t* I = (int32_t*)malloc((size_t)(2 * n_ins + 2) * sizeof(int32_t));
  if (!D || !I) { free(D); free(I); return -2; }
  for (int64_t i = 0; i < n_del; i++) { D[2 * i] = del_src[i]; D[2 * i + 1] = del_dst[i]; }
  for (int64_t i = 0; i < n_ins; i++) { I[2 * i] = ins_src[i]; I[2 * i + 1] = ins_dst[i]; }
  int64_t self_del = 0, self_ins = 0;
  int64_t nd = sort_unique_pairs(D, n_del, &self_del);
  int64_t ni = sort_unique_pairs(I, n_ins, &self_ins);

  /* E^t = (E^{t-1} \ Del') U Ins' by a three-way walk over sorted lists */
  int64_t a = 0, d = 0, b = 0, w = 0;
  while (a < m_old || b < ni) {
    int take_old;
    if (a >= m_old) take_old = 0;
    else if (b >= ni) take_old = 1;
    else take_old = pair_less(osrc[a], odst[a], I[2 * b], I[2 * b + 1]) ||
                    (osrc[a] == I[2 * b] && odst[a] == I[2 * b + 1]);
    if (take_old) {
      int32_t u = osrc[a], v = odst[a];
      if (b < ni && I[2 * b] == u && I[2 * b + 1] == v) b++; /* also inserted: keep once */
      else {
        while (d < nd && pair_less(D[2 * d], D[2 * d + 1], u, v)) d++;
        if (d < nd && D[2 * d] == u && D[2 * d + 1] == v) { a++; continue; } /* deleted */
      }
      new_src[w] = u; new_dst[w] = v; w++; a++;
    } else {
      new_src[w] = I[2 * b]; new_dst[w] = I[2 * b + 1]; w++; b++;
    }
  }
  *m_new = w;

  /* Delta- = E^{t-1} \ E^t and Delta+ = E^t \ E^{t-1} (merge walk) */
  int64_t i = 0, j = 0, km = 0, kp = 0;
  while (i < m_old || j < w) {
    if (j >= w || (i < m_old && pair_less(osrc[i], odst[i], new_src[j], new_dst[j]))) {
      dm_src[km] = osrc[i]; dm_dst[km] = odst[i]; km++; i++;
    } else if (i >= m_old || pair_less(new_src[j], new_dst[j], osrc[i], odst[i])) {
      dp_src[kp] = new_src[j]; dp_dst[kp] = new_dst[j]; kp++; j++;
    } else { i++; j++; }
  }
  *n_dm = km;
  *n_dp = kp;
  if (info) {
    info[0] = n_ins; info[1] = kp; info[2] = n_del; info[3] = km; info[4] = self_del;
  }
  free(D); free(I);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Rank computation: Static, ND, DF, DF-P (Algorithm 1, Equations 1 and 2). */
/* ------------------------------------------------------------------------ */

/*
 * criterion: ORC_CRIT_RELATIVE (dr / max(r, R[v])), ORC_CRIT_ABSOLUTE (dr) or
 * ORC_CRIT_CONTRIB (dr / |out(v)|), the measure compared with tau_f and tau_p.
 * n: |V^t|; out_off/out_idx and in_off/in_idx: G^t; prev_off/prev_idx:
 * G^{t-1}.out (needed by DF and DF-P only).  dm / dp: the effective deletions
 * and insertions.  r_prev: R^{t-1} (ignored by STATIC).
 * stats[5] = {iterations, converged, ever_affected, vertex_updates, edges_pulled}.
 * frontier (nullable, max_iters entries): |A_i| per iteration.
 * Returns 0, or -2 on allocation failure.
 */
int orc_rank(int32_t n, int32_t mode,
             const int32_t* prev_off, const int32_t* prev_idx,
             const int32_t* out_off, const int32_t* out_idx,
             const int32_t* in_off, const int32_t* in_idx,
             int64_t n_dm, const int32_t* dm_src, const int32_t* dm_dst,
             int64_t n_dp, const int32_t* dp_src, const int32_t* dp_dst,
             const double* r_prev, double alpha, double tol, double tol_f, double tol_p,
             int32_t criterion, int32_t max_iters, double* r_out, int64_t* stats, double* last_delta,
             int32_t* frontier) {
  (void)dm_dst; (void)dp_dst;
  const int dynamic = (mode == ORC_DF || mode == ORC_DFP);
  double* R = r_out;                                   /* current ranks R_i       */
  double* Rn = (double*)malloc((size_t)n * sizeof(double)); /* next ranks R_{i+1} */
  uint8_t* A = (uint8_t*)calloc((size_t)n, 1);         /* affected in iteration i */
  uint8_t* An = (uint8_t*)calloc((size_t)n, 1);        /* affected in i+1         */
  uint8_t* X = (uint8_t*)calloc((size_t)n, 1);         /* expands in iteration i  */
  uint8_t* ever = (uint8_t*)calloc((size_t)n, 1);
  if (!Rn || !A || !An || !X || !ever) {
    free(Rn); free(A); free(An); free(X); free(ever);
    return -2;
  }

  /* Initialisation of ranks: 1/|V| for Static (Section 3.1), R^{t-1} otherwise
   * (Section 4.1.1; Algorithm 1, initialisation). */
  for (int32_t v = 0; v < n; v++) R[v] = (mode == ORC_STATIC) ? 1.0 / (double)n : r_prev[v];

  /* Affected set.  Static and ND process every vertex.  DF/DF-P: for every
   * (u,v) in Delta- U Delta+, mark (G^{t-1} U G^t).out(u) (Algorithm 1,
   * initial marking; Section 4.1.1). */
  if (!dynamic) {
    for (int32_t v = 0; v < n; v++) A[v] = 1;
  } else {
    for (int64_t e = 0; e < n_dm + n_dp; e++) {
      int32_t u = (e < n_dm) ? dm_src[e] : dp_src[e - n_dm];
      for (int32_t p = prev_off[u]; p < prev_off[u + 1]; p++) A[prev_idx[p]] = 1;
      for (int32_t p = out_off[u]; p < out_off[u + 1]; p++) A[out_idx[p]] = 1;
    }
  }

  const double C0 = (1.0 - alpha) / (double)n;      /* Algorithm 1: C0 = (1-a)/|V^t| */
  int64_t vertex_updates = 0, edges_pulled = 0;
  int32_t it = 0, converged = 0;
  double dR = 0.0;

  for (it = 0; it < max_iters; it++) {
    dR = 0.0;
    int64_t cnt = 0, pulled = 0;
    for (int32_t v = 0; v < n; v++) { Rn[v] = R[v]; An[v] = 0; X[v] = 0; }

#pragma omp parallel for schedule(dynamic, 2048) reduction(max : dR) reduction(+ : cnt, pulled)
    for (int32_t v = 0; v < n; v++) {
      if (!A[v]) continue;
      ever[v] = 1;
      cnt++;
      pulled += in_off[v + 1] - in_off[v];
      /* c = sum over u in in(v) of R[u] / |out(u)|, ascending u, left fold */
      double c = 0.0;
      for (int32_t p = in_off[v]; p < in_off[v + 1]; p++) {
        int32_t u = in_idx[p];
        c = c + R[u] / (double)(out_off[u + 1] - out_off[u]);
      }
      const double d = (double)(out_off[v + 1] - out_off[v]);
      double r;
      if (mode == ORC_DFP)
        r = (1.0 / (1.0 - alpha / d)) * (C0 + alpha * (c - R[v] / d)); /* Equation 2 */
      else
        r = C0 + alpha * c;                                             /* Equation 1 */
      const double dr = fabs(r - R[v]);
      if (dr > dR) dR = dr;
      if (dynamic) {
        /* Section 4.2: the change measured as dr / max(previous, current rank)
         * (the method's choice), as dr, or as the change dr/d of the
         * contribution factor; the same measure decides pruning (DF-P). */
        double rel;
        if (criterion == ORC_CRIT_ABSOLUTE) rel = dr;
        else if (criterion == ORC_CRIT_CONTRIB) rel = dr / d;
        else rel = dr / fmax(r, R[v]);
        An[v] = (mode == ORC_DFP && rel <= tol_p) ? 0 : 1; /* prune (DF-P only) */
        if (rel > tol_f) X[v] = 1;                         /* expand             */
      } else {
        An[v] = 1;
      }
      Rn[v] = r;
    }
    /* Expansion: mark out(v) of every vertex whose relative change exceeded
     * tau_f.  Applied after the prunes, so marks win. */
    if (dynamic) {
#pragma omp parallel for schedule(dynamic, 2048)
      for (int32_t v = 0; v < n; v++) {
        if (!X[v]) continue;
        for (int32_t p = out_off[v]; p < out_off[v + 1]; p++) {
#pragma omp atomic write
          An[out_idx[p]] = 1;
        }
      }
    }
    if (frontier) frontier[it] = (int32_t)cnt;
    vertex_updates += cnt;
    edges_pulled += pulled;
    memcpy(R, Rn, (size_t)n * sizeof(double));
    uint8_t* t = A; A = An; An = t;
    if (dR <= tol) { converged = 1; it++; break; } /* Algorithm 1: stop when dR <= tau */
  }

  int64_t ever_n = 0;
  for (int32_t v = 0; v < n; v++) ever_n += ever[v];
  if (stats) {
    stats[0] = it; stats[1] = converged; stats[2] = ever_n;
    stats[3] = vertex_updates; stats[4] = edges_pulled;
  }
  if (last_delta) *last_delta = dR;
  free(Rn); free(A); free(An); free(X); free(ever);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
