// Rank engine: Static, Naive-dynamic, Dynamic Frontier and Dynamic Frontier
// with Pruning (Algorithm 1; Equations 1 and 2), pull-based (Section 4.4),
// iterated synchronously: every read of iteration i sees the ranks of
// iteration i; prunes and marks take effect in iteration i+1.
//
// Per iteration:
//   pull     one fused launch over the affected set, binned by in-degree:
//            c = sum of contrib[u] over in(v), the rank of Equation 1 or 2,
//            |r - R[v]| folded into a spread max
//   commit   contrib[v] = R[v]/|out(v)| for the processed vertices (DF, DF-P)
//            and marking of out(v) where the relative change exceeds tau_f
//   bin      next affected flags -> worklist split in degree bins
// Static and ND process every vertex and ping-pong two rank/contribution
// buffers instead of committing.
//
// Memory-level parallelism is the design rule: every lane keeps up to four
// independent gathers in flight, short rows are processed by sub-wave groups,
// out-row marking is balanced across the wave by a prefix sum of row lengths,
// and no reduction funnels the whole chip into one atomic address.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <mutex>

#include "prim.hpp"

namespace dfpr {

enum : int { kSync = 0, kDF = 2, kDFP = 3 };  // kSync = Static and ND (Equation 1, no flags)

struct PullArgs {
  const int32_t* __restrict__ in_off;
  const int32_t* __restrict__ in_idx;
  const int32_t* __restrict__ in_deg;   // row v of the in-CSR: in_idx[in_off[v], in_off[v] + in_deg[v])
  const int32_t* __restrict__ out_deg;  // |out(v)|
  const double* __restrict__ contrib;
  double* R;       // ranks of this iteration (frontier DF/DF-P: written in place)
  double* Rw;      // Static/ND and dense DF/DF-P: ranks of the next iteration
  double* cw;      // Static/ND and dense DF/DF-P: contributions of the next iteration
  uint8_t* next;   // frontier DF/DF-P: affected in the next iteration
  uint8_t* xflag;  // frontier DF/DF-P: expands
  // dense DF/DF-P: v is affected iff stay_in[v] or an in-neighbour u has x_in[u]
  const uint8_t* stay_in;
  const uint8_t* x_in;
  uint8_t* stay_out;
  uint8_t* x_out;
  uint8_t* ever;    // processed in this update: the stamp of the last dense iteration that did (else 1)
  int stamp;        // dense: this iteration's stamp (1 .. 255)
  int carry;        // dense: the previous dense iteration's stamp, 0 before the first one
  int use_x;
  unsigned long long* gslots;  // spread L-inf slots: member g, sub j at (g * gsub + j) * kSlotStride
  int gsub;
  const int32_t* gid;          // member of each vertex (null: plain graph)
  const int32_t* nk;           // vertex count of each member
  const uint8_t* done;         // member already converged (null: none)
  unsigned long long* acc;   // spread accumulator rows (dense counts)
  double* partial;           // bin 5: per-chunk partial sums
  int32_t* partial_x;        // bin 5: per-chunk "an in-neighbour expanded" (dense)
  int32_t* arrive;           // bin 5: chunks finished per vertex
  const int64_t* chunk_pre;  // bin 5: first chunk of each vertex (exclusive scan)
  double alpha, C0, tf, tp;
  int crit;      // DFPR_CRIT_*
  double* cmut;  // frontier form, asynchronous: contributions updated in the pull (else null)
};

// Stamp of dense iteration `it` in the ever array: nonzero, 254 values in turn
// (a vertex last processed 254 iterations back only costs a needless copy).
__host__ __device__ inline int dense_stamp(int it) { return 2 + it % 254; }

// Bin k covers worklist [lo[k], hi[k]) and workgroups [blk[k], blk[k+1]).
struct PullLayout {
  int64_t lo[kBins], hi[kBins];
  int32_t blk[kBins + 1];
};

struct Bounds {
  int32_t b[5];
};

// What a vertex needs besides its in-neighbour sum.  The self-loop term
// R[v]/|out(v)| is taken from R[v] instead of gathering contrib[v]: the same
// correctly rounded quotient.
struct VCtx {
  int32_t v, s, e, g;
  double Rv, d, selfc;
};
__device__ __forceinline__ VCtx load_vertex(const PullArgs& a, int32_t v) {
  VCtx c;
  c.v = v;
  c.g = a.gid ? a.gid[v] : 0;
  c.s = a.in_off[v];
  c.e = c.s + a.in_deg[v];
  c.d = (double)a.out_deg[v];
  c.Rv = a.R[v];
  c.selfc = c.Rv / c.d;
  return c;
}
__device__ __forceinline__ int32_t ld_idx(const PullArgs& a, int32_t p) {
  return __builtin_nontemporal_load(&a.in_idx[p]);  // streamed once: keep L2 for the gathers
}
__device__ __forceinline__ double gx(const PullArgs& a, int32_t u, const VCtx& c) {
  return u == c.v ? c.selfc : a.contrib[u];
}

// Per-member maxima of one workgroup, in LDS: a small open-addressing table
// (member -> bit pattern of the max), flushed to the spread slots at the end.
// A batch's worklist is sorted by vertex and members are vertex ranges, so a
// workgroup meets few members; when the table is full the update goes
// straight to the member's slot.
constexpr int kGTab = 32;
struct GTab {
  int key[kGTab];
  unsigned long long val[kGTab];
};
__device__ __forceinline__ void gtab_max(GTab* t, int g, double x, unsigned long long* gslots, int gsub) {
  if (!(x > 0.0)) return;
  const unsigned long long bits = (unsigned long long)__double_as_longlong(x);
#pragma unroll 1
  for (int i = 0; i < kGTab; i++) {
    const int sl = (g + i) & (kGTab - 1);
    const int cur = atomicCAS(&t->key[sl], -1, g);
    if (cur == -1 || cur == g) {
      atomicMax(&t->val[sl], bits);
      return;
    }
  }
  atomicMax(&gslots[((size_t)g * gsub + blockIdx.x % gsub) * kSlotStride], bits);
}

// Per-thread accumulators of one pull launch.
struct Acc {
  double mx = 0.0;                          // L-inf change (plain graph)
  int64_t cnt = 0, aedges = 0, xedges = 0, sedges = 0;  // dense: affected, their in-edges, expander
                                                        // out-edges, kept vertices' in-edges
  int64_t carry = 0;                                    // dense: unprocessed vertices copied over
  GTab* tab = nullptr;                      // per-member maxima (batch)
};
__device__ __forceinline__ void acc_dr(Acc& acc, const PullArgs& a, int g, double dr) {
  if (acc.tab) gtab_max(acc.tab, g, dr, a.gslots, a.gsub); else acc.mx = fmax(acc.mx, dr);
}
__device__ __forceinline__ bool member_done(const PullArgs& a, int g) { return a.done && a.done[g]; }

// Equation 1 (DF, Static, ND) or Equation 2 (DF-P) for the vertex from its
// in-neighbour sum c.  Same operation order as the algorithm states it; the
// library is built without FMA contraction.  DENSE: aff tells whether the
// vertex is affected; unaffected vertices carry their rank over.
template <int MODE, bool DENSE>
__device__ __forceinline__ void vertex_finish(const PullArgs& a, const VCtx& x, double c, bool aff, Acc& acc) {
  if (!aff) {  // not processed (unaffected, or its member converged): carry over
    // The dense form ping-pongs its rank and contribution vectors, so the
    // vector written now already holds the vertex's current values unless
    // the previous iteration processed it (its ever stamp) or this is the
    // first dense iteration since the vectors were last in step (carry 0).
    if (MODE == kSync) {
      a.Rw[x.v] = x.Rv;
      a.cw[x.v] = x.selfc;
    } else if (DENSE && (a.carry == 0 || a.ever[x.v] == (uint8_t)a.carry)) {
      a.Rw[x.v] = x.Rv;
      a.cw[x.v] = x.selfc;
      acc.carry++;
    }
    if (DENSE) {
      a.stay_out[x.v] = 0;
      a.x_out[x.v] = 0;
    }
    return;
  }
  const double d = x.d, Rv = x.Rv;
  const double C0 = a.gid ? (1.0 - a.alpha) / (double)a.nk[x.g] : a.C0;  // (1-alpha)/|V| of the member
  double r;
  if (MODE == kDFP)
    r = (1.0 / (1.0 - a.alpha / d)) * (C0 + a.alpha * (c - Rv / d));
  else
    r = C0 + a.alpha * c;
  const double dr = fabs(r - Rv);
  acc_dr(acc, a, x.g, dr);
  if (MODE == kSync) {
    a.Rw[x.v] = r;
    a.cw[x.v] = r / d;
    return;
  }
  // change measure (Section 4.2): relative (default), absolute, or of the contribution factor
  const double rel = a.crit == DFPR_CRIT_ABSOLUTE ? dr : a.crit == DFPR_CRIT_CONTRIB ? dr / d : dr / fmax(r, Rv);
  const bool stay = !(MODE == kDFP && rel <= a.tp);  // prune (DF-P) or keep
  const bool expand = rel > a.tf;
  if (DENSE) {
    a.Rw[x.v] = r;
    a.cw[x.v] = r / d;
    a.stay_out[x.v] = stay;
    a.x_out[x.v] = expand;
    a.ever[x.v] = (uint8_t)a.stamp;
    acc.cnt++;
    acc.aedges += x.e - x.s;
    if (expand) acc.xedges += (int64_t)d;
    if (stay) acc.sedges += x.e - x.s;
  } else {
    a.R[x.v] = r;
    if (a.cmut) a.cmut[x.v] = r / d;  // asynchronous: visible to the vertices processed after this one
    if (stay) a.next[x.v] = 1;
    if (expand) {
      a.xflag[x.v] = 1;
      acc.xedges += (int64_t)d;  // out-edges the commit will mark
    }
  }
}

// Workgroup reduction of the accumulators into spread slots (the bit pattern
// of a non-negative IEEE double orders like the value).
template <bool DENSE>
__device__ __forceinline__ void block_acc_to_slots(Acc acc, const PullArgs& a) {
  __shared__ double shm[1024 / kWave];
  __shared__ int64_t shc[5][1024 / kWave];
  const int w = threadIdx.x / kWave;
  const double m = wave_max(acc.mx);
  int64_t c0 = 0, c1 = 0, c3 = 0, c4 = 0;
  const int64_t c2 = wave_sum_i64(acc.xedges);  // both forms: out-degree sum of the expanding vertices
  if (DENSE) {
    c0 = wave_sum_i64(acc.cnt);
    c1 = wave_sum_i64(acc.aedges);
    c3 = wave_sum_i64(acc.sedges);
    c4 = wave_sum_i64(acc.carry);
  }
  if (lane_id() == 0) {
    shm[w] = m;
    shc[0][w] = c0;
    shc[1][w] = c1;
    shc[2][w] = c2;
    shc[3][w] = c3;
    shc[4][w] = c4;
  }
  __syncthreads();
  if (acc.tab) {  // batch: flush the per-member maxima (all threads reached the barrier above)
    for (int i = threadIdx.x; i < kGTab; i += blockDim.x)
      if (acc.tab->key[i] >= 0 && acc.tab->val[i])
        atomicMax(&a.gslots[((size_t)acc.tab->key[i] * a.gsub + blockIdx.x % a.gsub) * kSlotStride], acc.tab->val[i]);
  }
  if (threadIdx.x == 0) {
    double mm = 0.0;
    int64_t t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
      mm = fmax(mm, shm[i]);
      t0 += shc[0][i];
      t1 += shc[1][i];
      t2 += shc[2][i];
      t3 += shc[3][i];
      t4 += shc[4][i];
    }
    const int slot = (blockIdx.x % kSlots) * kSlotStride;
    if (mm > 0.0)
      atomicMax(&a.gslots[(blockIdx.x % a.gsub) * kSlotStride], (unsigned long long)__double_as_longlong(mm));
    constexpr int kRow = kSlots * kSlotStride;
    if (t2) atomicAdd(&a.acc[kAccXEdges * kRow + slot], (unsigned long long)t2);
    if (DENSE) {
      if (t0) atomicAdd(&a.acc[kAccCnt * kRow + slot], (unsigned long long)t0);
      if (t1) atomicAdd(&a.acc[kAccAffEdges * kRow + slot], (unsigned long long)t1);
      if (t3) atomicAdd(&a.acc[kAccStayEdges * kRow + slot], (unsigned long long)t3);
      if (t4) atomicAdd(&a.acc[kAccCarry * kRow + slot], (unsigned long long)t4);
    }
  }
}

// ---- bins 0-3: groups of G lanes per vertex.  G = 1 folds in ascending
// source order (the order of the algorithm's sum); G > 1 lanes take strided
// edges and combine with a butterfly.  Up to four gathers in flight per lane.
// DENSE: a vertex not kept by its own flag first checks its in-neighbours'
// expand flags (same strided sweep), and gathers contributions only if it is
// affected.
template <int MODE, int G, bool DENSE>
__device__ __forceinline__ void pull_groups(const PullArgs& a, const int32_t* __restrict__ wl, int64_t lo, int64_t hi,
                                            int lb, int nb, Acc& acc) {
  constexpr int kGroups = 256 / G;
  const int gl = threadIdx.x % G;
  for (int64_t k = lo + (int64_t)lb * kGroups + threadIdx.x / G; k < hi; k += (int64_t)nb * kGroups) {
    const VCtx x = load_vertex(a, wl[k]);
    bool aff = !member_done(a, x.g);
    if (DENSE && aff) {
      aff = a.stay_in[x.v] != 0;
      if (!aff && a.use_x) {
        // any in-neighbour expanded?  Rounds of 4G edges with a group vote after
        // each, stopping at the first hit (in-rows start with the high-degree
        // sources, which expand most often).  The trip count is the same for
        // the G lanes of a group, so the vote only reads active lanes.
        int any = 0;
        for (int32_t base = x.s; base < x.e && !any; base += 4 * G) {
          int f = 0;
#pragma unroll
          for (int t = 0; t < 4; t++) {
            const int32_t p = base + t * G + gl;
            if (p < x.e) f |= a.x_in[ld_idx(a, p)];
          }
#pragma unroll
          for (int o = G / 2; o >= 1; o >>= 1) f |= __shfl_xor(f, o, kWave);
          any = f;
        }
        aff = any != 0;
      }
    }
    double c = 0.0;
    if (aff) {
      if (G == 1) {
        int32_t p = x.s;
        for (; p + 8 <= x.e; p += 8) {  // eight gathers in flight, then folded in order
          int32_t u[8];
          double xv[8];
#pragma unroll
          for (int t = 0; t < 8; t++) u[t] = ld_idx(a, p + t);
#pragma unroll
          for (int t = 0; t < 8; t++) xv[t] = gx(a, u[t], x);
#pragma unroll
          for (int t = 0; t < 8; t++) c = c + xv[t];
        }
        for (; p + 4 <= x.e; p += 4) {
          const int32_t u0 = ld_idx(a, p), u1 = ld_idx(a, p + 1), u2 = ld_idx(a, p + 2), u3 = ld_idx(a, p + 3);
          const double x0 = gx(a, u0, x), x1 = gx(a, u1, x), x2 = gx(a, u2, x), x3 = gx(a, u3, x);
          c = c + x0;
          c = c + x1;
          c = c + x2;
          c = c + x3;
        }
        const int32_t r = x.e - p;  // 0..3 left
        const int32_t u0 = r > 0 ? ld_idx(a, p) : x.v;
        const int32_t u1 = r > 1 ? ld_idx(a, p + 1) : x.v;
        const int32_t u2 = r > 2 ? ld_idx(a, p + 2) : x.v;
        const double x0 = gx(a, u0, x), x1 = gx(a, u1, x), x2 = gx(a, u2, x);
        if (r > 0) c = c + x0;
        if (r > 1) c = c + x1;
        if (r > 2) c = c + x2;
      } else {
        int32_t p = x.s + gl;
        for (; p + 3 * G < x.e; p += 4 * G) {
          const int32_t u0 = ld_idx(a, p), u1 = ld_idx(a, p + G), u2 = ld_idx(a, p + 2 * G), u3 = ld_idx(a, p + 3 * G);
          const double x0 = gx(a, u0, x), x1 = gx(a, u1, x), x2 = gx(a, u2, x), x3 = gx(a, u3, x);
          c += x0;
          c += x1;
          c += x2;
          c += x3;
        }
        for (; p < x.e; p += G) c += gx(a, ld_idx(a, p), x);
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) c += __shfl_xor(c, o, kWave);
      }
    }
    if (gl == 0) vertex_finish<MODE, DENSE>(a, x, c, aff, acc);
  }
}

// Strided sum (and expand-flag OR when want_x) over in_idx[s, e) by the 256
// threads of a workgroup, combined in a fixed order; valid in thread 0.
template <bool DEEP>
__device__ __forceinline__ double block_row_sum(const PullArgs& a, const VCtx& x, int32_t s, int32_t e, bool want_sum,
                                                bool want_x, int* any_out, double* sh, int* shx) {
  double part = 0.0;
  int any = 0;
  int32_t p = s + (int32_t)threadIdx.x;
  // DEEP: eight loads in flight per thread (a workgroup on one long row has no
  // other work to hide its latency; the dense form keeps four, its flag checks
  // leave no registers for more); the thread's additions keep the order of its
  // elements, so the sum is the same either way
  for (; DEEP && p + 7 * 256 < e; p += 8 * 256) {
    int32_t u[8];
#pragma unroll
    for (int t = 0; t < 8; t++) u[t] = ld_idx(a, p + t * 256);
    if (want_x) {
#pragma unroll
      for (int t = 0; t < 8; t++) any |= a.x_in[u[t]];
    }
    if (want_sum) {
      double xs[8];
#pragma unroll
      for (int t = 0; t < 8; t++) xs[t] = gx(a, u[t], x);
#pragma unroll
      for (int t = 0; t < 8; t++) part += xs[t];
    }
  }
  for (; p + 3 * 256 < e; p += 4 * 256) {
    const int32_t u0 = ld_idx(a, p), u1 = ld_idx(a, p + 256), u2 = ld_idx(a, p + 512), u3 = ld_idx(a, p + 768);
    if (want_x) any |= a.x_in[u0] | a.x_in[u1] | a.x_in[u2] | a.x_in[u3];
    if (want_sum) {
      const double x0 = gx(a, u0, x), x1 = gx(a, u1, x), x2 = gx(a, u2, x), x3 = gx(a, u3, x);
      part += x0;
      part += x1;
      part += x2;
      part += x3;
    }
  }
  for (; p < e; p += 256) {
    const int32_t u = ld_idx(a, p);
    if (want_x) any |= a.x_in[u];
    if (want_sum) part += gx(a, u, x);
  }
  part = wave_sum(part);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) any |= __shfl_xor(any, o, kWave);
  if (lane_id() == 0) {
    sh[threadIdx.x / kWave] = part;
    shx[threadIdx.x / kWave] = any;
  }
  __syncthreads();
  double c = 0.0;
  if (threadIdx.x == 0) {
    c = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    *any_out = shx[0] | shx[1] | shx[2] | shx[3];
  }
  __syncthreads();
  return c;
}

// ---- bin 4: one workgroup per vertex
template <int MODE, bool DENSE>
__device__ __forceinline__ void pull_block(const PullArgs& a, const int32_t* __restrict__ wl, int64_t lo, int64_t hi,
                                           int lb, int nb, Acc& acc) {
  __shared__ double sh[256 / kWave];
  __shared__ int shx[256 / kWave];
  for (int64_t k = lo + lb; k < hi; k += nb) {
    const VCtx x = load_vertex(a, wl[k]);
    bool aff = !member_done(a, x.g);
    if (DENSE && aff) {
      aff = a.stay_in[x.v] != 0;
      if (!aff && a.use_x) {  // in-neighbour expand flags, stopping at the first hit
        int any = 0;
        for (int32_t base = x.s; base < x.e; base += 4 * 256) {
          int f = 0;
#pragma unroll
          for (int t = 0; t < 4; t++) {
            const int32_t p = base + t * 256 + (int32_t)threadIdx.x;
            if (p < x.e) f |= a.x_in[ld_idx(a, p)];
          }
          if (__syncthreads_or(f)) {
            any = 1;
            break;
          }
        }
        aff = any != 0;
      }
    }
    int dummy;
    const double c = aff ? block_row_sum<!DENSE>(a, x, x.s, x.e, true, false, &dummy, sh, shx) : 0.0;
    if (threadIdx.x == 0) vertex_finish<MODE, DENSE>(a, x, c, aff, acc);
  }
}

// ---- bin 5: rows split in kPullChunk-edge chunks.  chunk_pre[j] is the
// first chunk of the bin's j-th vertex (exclusive scan of the chunk counts);
// workgroup lb takes the contiguous chunk range [lb*T/nb, (lb+1)*T/nb).  Each
// chunk's sum goes to `partial`.  A row's partials are added by 256 threads
// (thread t takes chunks t, t+256, ..., then a fixed reduction tree) before
// the rank is computed: in a launch of its own after the pull (DEFER; the
// launch boundary orders the partials before the reads), or, inside the
// single-launch loop, by the workgroup that finishes the row's last chunk
// (arrival counter; a device-scope fence before each arrival).  Both add in
// the same order, so give the same bits.  DENSE: each chunk also reports
// whether an in-neighbour expanded.
__device__ __forceinline__ int64_t upper_bound_i64(const int64_t* a, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <int MODE, bool DENSE, bool DEFER>
__device__ __forceinline__ void pull_chunks(const PullArgs& a, const int32_t* __restrict__ wl, int64_t lo, int64_t hi,
                                            int lb, int nb, Acc& acc) {
  __shared__ double sh[256 / kWave];
  __shared__ int shx[256 / kWave];
  __shared__ int last;
  const int64_t nv = hi - lo;
  const int64_t* pre = a.chunk_pre;
  const int64_t T = pre[nv];
  const int64_t q0 = (int64_t)lb * T / nb, q1 = (int64_t)(lb + 1) * T / nb;
  if (q0 >= q1) return;
  int64_t j = upper_bound_i64(pre, 0, nv + 1, q0) - 1;
  int64_t cj = pre[j], cj1 = pre[j + 1];
  VCtx x = load_vertex(a, wl[lo + j]);
  for (int64_t q = q0; q < q1; q++) {
    while (q >= cj1) {
      j++;
      cj = cj1;
      cj1 = pre[j + 1];
      x = load_vertex(a, wl[lo + j]);
    }
    const bool want_x = DENSE && a.use_x && !a.stay_in[x.v] && !member_done(a, x.g);
    const int32_t cs = x.s + (int32_t)((q - cj) * kPullChunk);
    const int32_t ce = min(cs + kPullChunk, x.e);
    int any = 0;
    const double part = block_row_sum<!DENSE>(a, x, cs, ce, true, want_x, &any, sh, shx);
    if (DEFER) {
      if (threadIdx.x == 0) {
        a.partial[q] = part;
        if (DENSE) a.partial_x[q] = any;
      }
      continue;
    }
    if (threadIdx.x == 0) {
      a.partial[q] = part;
      if (DENSE) a.partial_x[q] = any;
      __threadfence();
      last = atomicAdd(&a.arrive[j], 1) == (int)(cj1 - cj - 1);
    }
    __syncthreads();
    if (last) {  // the same in every thread: the whole workgroup adds the row's partials
      __threadfence();
      double c = 0.0;
      int anyx = 0;
      for (int64_t t = cj + threadIdx.x; t < cj1; t += blockDim.x) {
        c += __hip_atomic_load(&a.partial[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (DENSE) anyx |= __hip_atomic_load(&a.partial_x[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      c = wave_sum(c);
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) anyx |= __shfl_xor(anyx, o, kWave);
      if (lane_id() == 0) {
        sh[threadIdx.x / kWave] = c;
        shx[threadIdx.x / kWave] = anyx;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        c = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        anyx = shx[0] | shx[1] | shx[2] | shx[3];
        a.arrive[j] = 0;
        const bool aff = !member_done(a, x.g) && (!DENSE || a.stay_in[x.v] || (a.use_x && anyx));
        vertex_finish<MODE, DENSE>(a, x, aff ? c : 0.0, aff, acc);
      }
    }
    __syncthreads();
  }
}

// The chunked rows of a pull launch that deferred them: one workgroup per row
// adds its partials and updates the vertex.
template <int MODE, bool DENSE>
__global__ void __launch_bounds__(256) k_chunk_finish(PullArgs a, const int32_t* __restrict__ wl, int64_t lo,
                                                      int64_t nv) {
  __shared__ double sh[256 / kWave];
  __shared__ int shx[256 / kWave];
  __shared__ GTab tab;
  Acc acc;
  if (a.gid) {
    for (int i = threadIdx.x; i < kGTab; i += blockDim.x) {
      tab.key[i] = -1;
      tab.val[i] = 0ull;
    }
    __syncthreads();
    acc.tab = &tab;
  }
  for (int64_t j = blockIdx.x; j < nv; j += gridDim.x) {
    const int64_t cj = a.chunk_pre[j], cj1 = a.chunk_pre[j + 1];
    double c = 0.0;
    int anyx = 0;
    for (int64_t t = cj + threadIdx.x; t < cj1; t += blockDim.x) {
      c += a.partial[t];
      if (DENSE) anyx |= a.partial_x[t];
    }
    c = wave_sum(c);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) anyx |= __shfl_xor(anyx, o, kWave);
    if (lane_id() == 0) {
      sh[threadIdx.x / kWave] = c;
      shx[threadIdx.x / kWave] = anyx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      c = ((sh[0] + sh[1]) + sh[2]) + sh[3];
      anyx = shx[0] | shx[1] | shx[2] | shx[3];
      const VCtx x = load_vertex(a, wl[lo + j]);
      const bool aff = !member_done(a, x.g) && (!DENSE || a.stay_in[x.v] || (a.use_x && anyx));
      vertex_finish<MODE, DENSE>(a, x, aff ? c : 0.0, aff, acc);
    }
    __syncthreads();
  }
  block_acc_to_slots<DENSE>(acc, a);
}

// Dense form with the two-phase pull (dfpr_set_two_phase): the in-neighbour
// sums and "an in-neighbour expanded" bits come from the phase-two
// accumulators; one thread per vertex converts its sum and updates the
// vertex as the gather pull would.  A block's 256 vertices are 8 whole flag
// words, so the words of split buckets are cleared after the barrier.
template <int MODE>
__global__ void __launch_bounds__(256) k_tp_finish(PullArgs a, int32_t n, uint64_t* glo, uint64_t* ghi, uint32_t* gfl,
                                                   const uint8_t* __restrict__ split) {
  Acc acc;
  const int32_t v = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  const bool in = v < n;
  double c = 0.0;
  bool anyx = false;
  if (in) {
    c = unfix128(glo[v], ghi[v]);
    anyx = ((gfl[v >> 5] >> (v & 31)) & 1u) != 0;
  }
  __syncthreads();
  if (in) {
    if (split[v >> kTpDstBits]) {  // several workgroups added into these: clear for the next iteration
      glo[v] = 0;
      ghi[v] = 0;
      if ((v & 31) == 0) gfl[v >> 5] = 0u;
    }
    const VCtx x = load_vertex(a, v);
    const bool aff = a.stay_in[v] != 0 || (a.use_x && anyx);
    vertex_finish<MODE, true>(a, x, aff ? c : 0.0, aff, acc);
  }
  block_acc_to_slots<true>(acc, a);
}

template <int MODE, bool DENSE, bool DEFER = false>
__device__ __forceinline__ void pull_virtual_block(const PullArgs& a, const int32_t* __restrict__ wl,
                                                   const PullLayout& L, int b);

// The layout lists the bins from the one-lane bin to the chunked rows; the
// workgroups take them in reverse, so the heaviest work items (long rows,
// whole-workgroup rows) are dispatched first and the light ones fill in
// behind them (1-3 % per launch at scale 24).  Which workgroup takes an item
// does not change how the item is summed.
template <int MODE, bool DENSE>
__global__ void __launch_bounds__(256, 8) k_pull(PullArgs a, const int32_t* __restrict__ wl, PullLayout L) {
  pull_virtual_block<MODE, DENSE, true>(a, wl, L, (int)(gridDim.x - 1 - blockIdx.x));
}

// Whole update in one cooperative launch (small graphs, where launch and
// readback latency dominate): every iteration runs the pull of the layout's
// workgroups (the same code and work split as k_pull, so the sums and ranks
// are the same bits) spread over the resident workgroups, then one grid
// barrier; every workgroup reads the iteration's L-inf change and stops at the
// same iteration.  Ranks, contributions and (DF, DF-P, dense form) keep/expand
// flags ping-pong.  The change of iteration i goes to slot i % 3: workgroup 0
// clears slot i+1 at the start of iteration i, which no workgroup reads or
// writes until after the barrier that ends iteration i.
// Grid barrier for a launch whose workgroups are all resident (cooperative
// launch): workgroups arrive at one of 32 group counters, the last of each
// group at the root counter, and the last of all bumps the generation the
// others wait on.  Two levels keep each counter's atomics few (one counter for
// the whole grid serialises every workgroup's atomic).  Memory ordering: the
// workgroup barrier completes the workgroup's stores, thread 0's arrival is a
// release at device scope (it publishes them), the wait polls with relaxed
// loads and ends with one acquire fence (so the workgroup then reads the other
// workgroups' stores).  The wait is bounded: on a timeout it raises
// c->fused_err and every workgroup leaves the loop.
constexpr int kBarGroups = 32;
__device__ __forceinline__ bool grid_barrier(IterCtl* c, unsigned nb) {
  __syncthreads();
  __shared__ int ok_sh;
  if (threadIdx.x == 0) {
    int ok = 1;
    unsigned* gen = &c->bar_gen[0];
    const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned grp = blockIdx.x % kBarGroups;
    const unsigned groups = nb < (unsigned)kBarGroups ? nb : (unsigned)kBarGroups;
    const unsigned gsize = nb / kBarGroups + (grp < nb % kBarGroups ? 1u : 0u);
    unsigned* leaf = &c->bar_leaf[grp * 32];
    bool released = false;
    if (__hip_atomic_fetch_add(leaf, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
      __hip_atomic_store(leaf, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned* root = &c->bar_root[0];
      if (__hip_atomic_fetch_add(root, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == groups - 1) {
        __hip_atomic_store(root, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        released = true;
      }
    }
    if (!released) {
      int64_t spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > ((int64_t)1 << 26) ||
            __hip_atomic_load(&c->fused_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          __hip_atomic_store(&c->fused_err, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

// One part of the all-vertex pull as the single-launch loop sees it: the
// part's layout, its worklist and its chunk prefix (see pull_parts).
constexpr int kFusedMaxParts = 16;  // parts of one single-launch loop (64M+ vertices)
struct FusedPart {
  PullLayout L;
  const int32_t* wl;
  const int64_t* chunk_pre;
  // the long-row bin's chunk partial sums and arrival counters of this part
  // (the parts' pulls run concurrently in one launch, so each has its own)
  double* partial;
  int32_t* partial_x;
  int32_t* arrive;
};
static_assert(sizeof(FusedPart) % sizeof(int32_t) == 0, "the part table is copied to LDS word by word");

// Member convergence inside the single-launch loop (batch handles): every
// member's spread L-inf slots are folded and cleared, its change and iteration
// count recorded, and it retires once the change is within tolerance (the
// stopping rule of Algorithm 1, per member graph, as k_dr_finish does between
// launches).  A wavefront per member; the members still running and the
// largest change among them go to the iteration's slots.
__device__ __forceinline__ void fused_fold_members(const PullArgs& a, IterCtl* c, int32_t G, int it, double tol,
                                                   double* g_dr, int32_t* g_iters, uint8_t* done) {
  const int lane = lane_id();
  const int waves = (int)(blockDim.x / kWave);
  int64_t active = 0;
  unsigned long long mx = 0ull;
  for (int64_t gg = (int64_t)blockIdx.x * waves + threadIdx.x / kWave; gg < G; gg += (int64_t)gridDim.x * waves) {
    const int32_t g = (int32_t)gg;
    unsigned long long m = 0ull;
    if (lane < a.gsub) {
      unsigned long long* sl = &a.gslots[((size_t)g * a.gsub + lane) * kSlotStride];
      m = *sl;
      *sl = 0ull;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const unsigned long long y = __shfl_xor(m, o, kWave);
      m = y > m ? y : m;
    }
    if (lane == 0 && !done[g]) {
      double d;
      __builtin_memcpy(&d, &m, sizeof d);
      g_dr[g] = d;
      g_iters[g] = it + 1;
      if (d <= tol) done[g] = 1; else active++;
      mx = m > mx ? m : mx;
    }
  }
  if (lane == 0 && active) atomicAdd(&c->fused_act[(it % 3) * kSlotStride], (unsigned long long)active);
  if (lane == 0 && mx) atomicMax(&c->fused_dr[(it % 3) * kSlotStride], mx);
}

// Whole update in one cooperative launch: every iteration runs the pull of
// every part's layout (the same code and work split as k_pull, so the sums
// and ranks are the same bits), spread over the resident workgroups, then one
// grid barrier; every workgroup reads the iteration's outcome and stops at the
// same iteration.  Plain graph: the outcome is the L-inf change, the change of
// iteration i goes to slot i % 3 (workgroup 0 clears slot i+1 at the start of
// iteration i, which no workgroup touches until after the barrier that ends
// iteration i).  Batch (G members): a second barrier follows the member fold,
// and the outcome is the number of members still running, in the same
// rotation of slots.  Ranks, contributions and (DF, DF-P, dense form)
// keep/expand flags ping-pong.
template <int MODE, bool BATCH>
__global__ void __launch_bounds__(256) k_fused_loop(PullArgs a0, const int32_t* __restrict__ wl0, PullLayout L0,
                                                       const FusedPart* __restrict__ parts, int nparts,
                                                       IterCtl* c, int max_iters, double tol, double* r_out,
                                                       const int32_t* __restrict__ inv, int32_t n, int32_t G,
                                                       double* g_dr, int32_t* g_iters) {
  constexpr bool DENSE = MODE != kSync;
  constexpr bool batch = BATCH;  // a plain graph: one part (wl0, L0) and one member
  PullArgs a = a0;
  if (!batch) {
    a.gsub = 1;
    a.gid = nullptr;
    a.done = nullptr;
  }
  uint8_t* done = const_cast<uint8_t*>(a0.done);
  // the part table lives in LDS for the whole loop: every work item reads its
  // part's layout, and a chain of global loads per item would lengthen every
  // iteration of this latency-bound loop
  __shared__ FusedPart sp[BATCH ? kFusedMaxParts : 1];
  int total = L0.blk[kBins];
  if (BATCH) {
    for (int i = threadIdx.x; i < nparts * (int)(sizeof(FusedPart) / sizeof(int32_t)); i += blockDim.x)
      reinterpret_cast<int32_t*>(sp)[i] = reinterpret_cast<const int32_t*>(parts)[i];
    __syncthreads();
    total = 0;
    for (int p = 0; p < nparts; p++) total += sp[p].L.blk[kBins];
  }
  for (int it = 0; it < max_iters; it++) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      c->fused_dr[((it + 1) % 3) * kSlotStride] = 0ull;
      c->fused_act[((it + 1) % 3) * kSlotStride] = 0ull;
    }
    if (!batch) a.gslots = &c->fused_dr[(it % 3) * kSlotStride];
    a.stamp = dense_stamp(it);
    a.carry = it == 0 ? 0 : dense_stamp(it - 1);  // the vectors are in step after the first iteration
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
      if (BATCH) {
        int p = 0, b = vb;
        while (p + 1 < nparts && b >= sp[p].L.blk[kBins]) b -= sp[p++].L.blk[kBins];
        b = sp[p].L.blk[kBins] - 1 - b;  // within a part, the heaviest work items first (as k_pull)
        a.chunk_pre = sp[p].chunk_pre;
        a.partial = sp[p].partial;
        a.partial_x = sp[p].partial_x;
        a.arrive = sp[p].arrive;
        pull_virtual_block<MODE, DENSE>(a, sp[p].wl, sp[p].L, b);
      } else {
        pull_virtual_block<MODE, DENSE>(a, wl0, L0, total - 1 - vb);
      }
      __syncthreads();
    }
    if (!grid_barrier(c, gridDim.x)) return;
    bool stop;
    if (batch) {
      fused_fold_members(a, c, G, it, tol, g_dr, g_iters, done);
      if (!grid_barrier(c, gridDim.x)) return;
      stop = __hip_atomic_load(&c->fused_act[(it % 3) * kSlotStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
             0ull;
    } else {
      const unsigned long long m =
          __hip_atomic_load(&c->fused_dr[(it % 3) * kSlotStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      double d;
      __builtin_memcpy(&d, &m, sizeof d);
      stop = d <= tol;
    }
    const unsigned long long last =
        __hip_atomic_load(&c->fused_dr[(it % 3) * kSlotStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // next iteration reads what this one wrote
    double* t = a.R;
    a.R = a.Rw;
    a.Rw = t;
    t = const_cast<double*>(a.contrib);
    a.contrib = a.cw;
    a.cw = t;
    if (DENSE) {
      uint8_t* f = const_cast<uint8_t*>(a.stay_in);
      a.stay_in = a.stay_out;
      a.stay_out = f;
      f = const_cast<uint8_t*>(a.x_in);
      a.x_in = a.x_out;
      a.x_out = f;
      a.use_x = 1;
    }
    if (stop || it + 1 == max_iters) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->fused_iters = it + 1;
        c->fused_converged = stop ? 1 : 0;
        c->fused_last = last;
      }
      break;
    }
  }
  // Epilogue, after the last barrier (nothing reads the ranks or flags any
  // more): the ranks go out in the caller's order, and DF/DF-P clear the four
  // flag arrays and (plain graph) count and clear the processed vertices, so
  // the host reads the outcome back once.  A batch counts its processed
  // vertices per member afterwards (k_count_ever_members).
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t cnt = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const double r = a.R[v];
    if (inv)
      r_out[inv[v]] = r;
    else if (r_out != a.R)
      r_out[v] = r;
    if (DENSE) {
      const_cast<uint8_t*>(a.stay_in)[v] = 0;
      a.stay_out[v] = 0;
      const_cast<uint8_t*>(a.x_in)[v] = 0;
      a.x_out[v] = 0;
      if (!batch && a.ever[v]) {
        cnt++;
        a.ever[v] = 0;
      }
    }
  }
  if (DENSE && !batch) {
    cnt = wave_sum_i64(cnt);
    if (lane_id() == 0 && cnt)
      atomicAdd(&a.acc[kAccEver * (kSlots * kSlotStride) + ((blockIdx.x * 4 + threadIdx.x / kWave) % kSlots) *
                                                             kSlotStride],
                (unsigned long long)cnt);
  }
}

template <int MODE, bool DENSE, bool DEFER>
__device__ __forceinline__ void pull_virtual_block(const PullArgs& a, const int32_t* __restrict__ wl,
                                                   const PullLayout& L, int b) {
  int k = 0;
  while (k < kBins - 1 && b >= L.blk[k + 1]) k++;
  const int lb = b - L.blk[k], nb = L.blk[k + 1] - L.blk[k];
  Acc acc;
  __shared__ GTab tab;
  if (a.gid) {
    for (int i = threadIdx.x; i < kGTab; i += blockDim.x) {
      tab.key[i] = -1;
      tab.val[i] = 0ull;
    }
    __syncthreads();
    acc.tab = &tab;
  }
  switch (k) {
    case 0: pull_groups<MODE, 1, DENSE>(a, wl, L.lo[0], L.hi[0], lb, nb, acc); break;
    case 1: pull_groups<MODE, 4, DENSE>(a, wl, L.lo[1], L.hi[1], lb, nb, acc); break;
    case 2: pull_groups<MODE, 16, DENSE>(a, wl, L.lo[2], L.hi[2], lb, nb, acc); break;
    case 3: pull_groups<MODE, 64, DENSE>(a, wl, L.lo[3], L.hi[3], lb, nb, acc); break;
    case 4: pull_block<MODE, DENSE>(a, wl, L.lo[4], L.hi[4], lb, nb, acc); break;
    default: pull_chunks<MODE, DENSE, DEFER>(a, wl, L.lo[5], L.hi[5], lb, nb, acc); break;
  }
  block_acc_to_slots<DENSE>(acc, a);
}

// ---- marking of out-rows, balanced over the wave: every lane that wants its
// row [os, oe) marked contributes its length to a wave prefix sum, then the
// 64 lanes sweep the concatenated rows four edges at a time, locating each
// edge's row by a binary search over the lanes' start offsets (cross-lane
// reads).  Rows longer than big_row go to big_list for the chunked pass.
// Must be called with all 64 lanes active.
__device__ __forceinline__ int seg_of(int32_t st, int32_t e) {
  int lo = 0, hi = kWave;
#pragma unroll
  for (int i = 0; i < 6; i++) {
    const int mid = (lo + hi) >> 1;
    const int32_t sm = __shfl(st, mid, kWave);
    if (sm <= e) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ void wave_mark_rows(bool want, int32_t v, int32_t os, int32_t oe,
                                               const int32_t* __restrict__ out_idx, uint8_t* flags,
                                               int32_t* big_list, int64_t* big_count, int32_t big_row) {
  const int lane = lane_id();
  int32_t len = want ? oe - os : 0;
  if (len > big_row) {
    const int64_t pos = (int64_t)atomicAdd((unsigned long long*)big_count, 1ull);
    big_list[pos] = v;
    len = 0;
  }
  int32_t incl = len;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  const int32_t total = __shfl(incl, kWave - 1, kWave);
  const int32_t st = incl - len;
  for (int32_t e0 = 0; e0 < total; e0 += 4 * kWave) {
    int32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int32_t e = e0 + lane + t * kWave;
      const bool ok = e < total;
      const int j = seg_of(st, ok ? e : 0);
      const int32_t p = __shfl(os, j, kWave) + (e - __shfl(st, j, kWave));
      w[t] = ok ? out_idx[p] : -1;
    }
#pragma unroll
    for (int t = 0; t < 4; t++)
      if (w[t] >= 0) flags[w[t]] = 1;
  }
}

// Initial marking (Algorithm 1): for every pending source u mark out(u) in
// G^t; the targets of effective deletions (the rest of out(u) in G^{t-1})
// were set in `flags` when the batch was applied.  The batch's sources
// include the high-degree vertices, which sit together in the first
// wavefronts: rows over kPendBigRow go to the chunked pass, so no wavefront
// sweeps more than a few hundred edges.
constexpr int32_t kPendBigRow = 128;
__global__ void __launch_bounds__(256) k_mark_pending(uint8_t* pend_src, int32_t n, const int32_t* __restrict__ out_off,
                                                      const int32_t* __restrict__ out_deg,
                                                      const int32_t* __restrict__ out_idx, uint8_t* flags,
                                                      int32_t* big_list, int64_t* big_count, int32_t big_row) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < n; base += stride) {
    const int64_t u = base + lane_id();
    bool want = false;
    int32_t os = 0, oe = 0;
    if (u < n && pend_src[u]) {
      pend_src[u] = 0;
      want = true;
      os = out_off[u];
      oe = os + out_deg[u];
    }
    wave_mark_rows(want, (int32_t)u, os, oe, out_idx, flags, big_list, big_count, big_row);
  }
}

// Commit (Jacobi reading): contrib[v] = R[v]/|out(v)| for the processed
// vertices, clear their current flag, and expand out(v) where flagged.
__global__ void __launch_bounds__(256) k_commit_expand(const int32_t* __restrict__ wl, int64_t cnt, const double* R,
                                                       double* contrib, const int32_t* __restrict__ out_off,
                                                       const int32_t* __restrict__ out_deg,
                                                       const int32_t* __restrict__ out_idx, uint8_t* cur,
                                                       uint8_t* next, uint8_t* xflag, int32_t* big_list,
                                                       int64_t* big_count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < cnt; base += stride) {
    const int64_t k = base + lane_id();
    bool want = false;
    int32_t v = 0, os = 0, oe = 0;
    if (k < cnt) {
      v = wl[k];
      os = out_off[v];
      oe = os + out_deg[v];
      contrib[v] = R[v] / (double)(oe - os);
      cur[v] = 0;
      if (xflag[v]) {
        xflag[v] = 0;
        want = true;
      }
    }
    wave_mark_rows(want, v, os, oe, out_idx, next, big_list, big_count, kBigRow);
  }
}

// Chunk prefix of the long out-row list (one workgroup; the list is short).
__global__ void __launch_bounds__(1024) k_big_scan(const int32_t* big_list, const int64_t* big_count,
                                                   const int32_t* out_deg, int64_t* big_pre) {
  __shared__ int64_t sh[1024 / kWave + 1];
  const int64_t nb = *big_count;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = min(lo + per, nb);
  int64_t local = 0;
  for (int64_t i = lo; i < hi; i++) {
    const int32_t v = big_list[i];
    local += ((int64_t)out_deg[v] + kMarkChunk - 1) / kMarkChunk;
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(local, sh, &tot);
  for (int64_t i = lo; i < hi; i++) {
    big_pre[i] = run;
    const int32_t v = big_list[i];
    run += ((int64_t)out_deg[v] + kMarkChunk - 1) / kMarkChunk;
  }
  if (threadIdx.x == 0) big_pre[nb] = tot;
}

__global__ void __launch_bounds__(256) k_big_mark(const int32_t* big_list, const int64_t* big_count,
                                                  const int64_t* big_pre, const int32_t* __restrict__ out_off,
                                                  const int32_t* __restrict__ out_deg,
                                                  const int32_t* __restrict__ out_idx, uint8_t* flags) {
  const int64_t nb = *big_count;
  const int64_t total = big_pre[nb];
  for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
    const int64_t j = upper_bound_i64(big_pre, 0, nb + 1, q) - 1;
    const int32_t v = big_list[j];
    const int32_t s = out_off[v] + (int32_t)((q - big_pre[j]) * kMarkChunk);
    const int32_t e = min(s + kMarkChunk, out_off[v] + out_deg[v]);
    for (int32_t p = s + (int32_t)threadIdx.x; p < e; p += 4 * (int32_t)blockDim.x) {
      int32_t w[4];
#pragma unroll
      for (int t = 0; t < 4; t++) w[t] = p + t * (int32_t)blockDim.x < e ? out_idx[p + t * blockDim.x] : -1;
#pragma unroll
      for (int t = 0; t < 4; t++)
        if (w[t] >= 0) flags[w[t]] = 1;
    }
  }
}

// ---- binning: affected vertices (flags == nullptr: all) -> worklist in
// ascending vertex order within each bin, bins back to back.  Each thread
// owns 8 consecutive vertices (one 8-byte flag load).
constexpr int kBinItems = 8;
constexpr int kBinTile = 256 * kBinItems;
constexpr int kBinShift = 20;  // three 20-bit counters per int64

__device__ __forceinline__ int bin_of(int32_t d, const Bounds& B) {
  return d <= B.b[0] ? 0 : d <= B.b[1] ? 1 : d <= B.b[2] ? 2 : d <= B.b[3] ? 3 : d <= B.b[4] ? 4 : 5;
}

// Flags of vertices base..base+7 as a bit mask; in a batch, vertices of
// members that have converged drop out.
struct MemberMask {
  const int32_t* gid;   // null: plain graph
  const uint8_t* done;
};
__device__ __forceinline__ unsigned tile_flags(const uint8_t* flags, int64_t base, int32_t n, MemberMask mm) {
  unsigned m = 0;
  if (base + kBinItems <= n) {
    if (flags == nullptr) {
      m = 0xFFu;
    } else {
      const uint64_t w = *reinterpret_cast<const uint64_t*>(flags + base);
#pragma unroll
      for (int j = 0; j < kBinItems; j++) m |= ((w >> (8 * j)) & 0xFFull) ? (1u << j) : 0u;
    }
  } else {
    for (int j = 0; j < kBinItems; j++)
      if (base + j < n && (flags == nullptr || flags[base + j])) m |= 1u << j;
  }
  if (mm.gid && m) {
    for (int j = 0; j < kBinItems; j++)
      if ((m & (1u << j)) && mm.done[mm.gid[base + j]]) m &= ~(1u << j);
  }
  return m;
}

// Vertices [lo, n) are binned (n: end of the range).
__global__ void __launch_bounds__(256) k_bin_count(const uint8_t* flags, const int32_t* __restrict__ in_deg,
                                                   const int32_t* __restrict__ out_deg, int64_t lo, int32_t n,
                                                   MemberMask mm, Bounds B, int64_t* blk, int64_t nb,
                                                   unsigned long long* acc) {
  __shared__ int64_t sh[256 / kWave + 1];
  __shared__ int64_t she[256 / kWave][kBins + 1];
  const int64_t base = lo + (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinItems;
  const unsigned m = tile_flags(flags, base, n, mm);
  int64_t p0 = 0, p1 = 0;
  int64_t ed[kBins + 1] = {0, 0, 0, 0, 0, 0, 0};  // per-bin in-degree sums, then the out-degree sum
  if (m) {
    int32_t o[kBinItems], q[kBinItems];
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
      o[j] = base + j < n ? in_deg[base + j] : 0;
      q[j] = base + j < n ? out_deg[base + j] : 0;
    }
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
      if (m & (1u << j)) {
        const int32_t d = o[j];
        const int b = bin_of(d, B);
        if (b < 3) p0 += (int64_t)1 << (kBinShift * b); else p1 += (int64_t)1 << (kBinShift * (b - 3));
#pragma unroll
        for (int t = 0; t < kBins; t++) ed[t] += (t == b) ? d : 0;
        ed[kBins] += q[j];
      }
    }
  }
  int64_t t0, t1;
  block_exclusive_scan(p0, sh, &t0);
  block_exclusive_scan(p1, sh, &t1);
  if (threadIdx.x == 0) {
    const int64_t mk = ((int64_t)1 << kBinShift) - 1;
    for (int b = 0; b < 3; b++) {
      blk[b * nb + blockIdx.x] = (t0 >> (kBinShift * b)) & mk;
      blk[(b + 3) * nb + blockIdx.x] = (t1 >> (kBinShift * b)) & mk;
    }
  }
#pragma unroll
  for (int t = 0; t <= kBins; t++) ed[t] = wave_sum_i64(ed[t]);
  if (lane_id() == 0)
    for (int t = 0; t <= kBins; t++) she[threadIdx.x / kWave][t] = ed[t];
  __syncthreads();
  if (threadIdx.x <= kBins) {
    const int64_t s = she[0][threadIdx.x] + she[1][threadIdx.x] + she[2][threadIdx.x] + she[3][threadIdx.x];
    const int row = threadIdx.x < kBins ? kAccEdges0 + (int)threadIdx.x : kAccOutEdges;
    if (s) atomicAdd(&acc[row * (kSlots * kSlotStride) + (blockIdx.x % kSlots) * kSlotStride], (unsigned long long)s);
  }
}

__global__ void __launch_bounds__(256) k_bin_scatter(const uint8_t* flags, const int32_t* __restrict__ in_deg,
                                                     int64_t lo, int32_t n, MemberMask mm, Bounds B, const int64_t* offs,
                                                     int64_t nb, int32_t* wl, uint8_t* ever, int64_t* bin_end) {
  __shared__ int64_t sh[256 / kWave + 1];
  const int64_t base = lo + (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinItems;
  const unsigned m = tile_flags(flags, base, n, mm);
  uint8_t bins[kBinItems];
  int64_t p0 = 0, p1 = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; j++) bins[j] = 0xFF;
  if (m) {
    int32_t o[kBinItems];
#pragma unroll
    for (int j = 0; j < kBinItems; j++) o[j] = base + j < n ? in_deg[base + j] : 0;
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
      if (m & (1u << j)) {
        const int b = bin_of(o[j], B);
        bins[j] = (uint8_t)b;
        if (b < 3) p0 += (int64_t)1 << (kBinShift * b); else p1 += (int64_t)1 << (kBinShift * (b - 3));
      }
    }
  }
  int64_t t0, t1;
  const int64_t e0 = block_exclusive_scan(p0, sh, &t0);
  const int64_t e1 = block_exclusive_scan(p1, sh, &t1);
  if (m) {
    const int64_t mk = ((int64_t)1 << kBinShift) - 1;
    int64_t pos[kBins];
#pragma unroll
    for (int b = 0; b < 3; b++) {
      pos[b] = offs[b * nb + blockIdx.x] + ((e0 >> (kBinShift * b)) & mk);
      pos[b + 3] = offs[(b + 3) * nb + blockIdx.x] + ((e1 >> (kBinShift * b)) & mk);
    }
#pragma unroll
    for (int j = 0; j < kBinItems; j++) {
      if (bins[j] != 0xFF) {
        const int32_t v = (int32_t)(base + j);
        int64_t ps = 0;
#pragma unroll
        for (int b = 0; b < kBins; b++)
          if (bins[j] == b) ps = pos[b]++;
        wl[ps] = v;
        if (ever) ever[v] = 1;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kBins) bin_end[threadIdx.x] = offs[(threadIdx.x + 1) * nb];
}

// ---- control block
// Per-member convergence after a pull: fold each member's spread slots (and
// clear them), record its change and iteration count, and retire it once the
// change is within tolerance (Algorithm 1's stopping rule, applied to every
// member graph on its own).  head.dR = largest change among the members still
// running, head.active = members not yet converged.  One workgroup; a wave
// per member, a lane per slot.
__device__ __forceinline__ void dr_fold(unsigned long long* gslots, int gsub, int32_t G, uint8_t* done,
                                        double* g_dr, int32_t* g_iters, int32_t it, double tol, IterCtl* c) {
  __shared__ unsigned long long shm[256 / kWave];
  __shared__ int64_t sha[256 / kWave];
  const int w = threadIdx.x / kWave, lane = lane_id();
  unsigned long long mx = 0ull;
  int64_t active = 0;
  for (int32_t g = w; g < G; g += 256 / kWave) {
    unsigned long long m = 0ull;
    if (lane < gsub) {
      unsigned long long* sl = &gslots[((size_t)g * gsub + lane) * kSlotStride];
      m = *sl;
      *sl = 0ull;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const unsigned long long y = __shfl_xor(m, o, kWave);
      m = y > m ? y : m;
    }
    if (lane == 0 && !done[g]) {
      double d;
      __builtin_memcpy(&d, &m, sizeof d);
      g_dr[g] = d;
      g_iters[g] = it + 1;
      if (d <= tol) done[g] = 1; else active++;
      mx = m > mx ? m : mx;
    }
  }
  if (lane == 0) {
    shm[w] = mx;
    sha[w] = active;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 256 / kWave; i++) {
      mx = shm[i] > mx ? shm[i] : mx;
      active += sha[i];
    }
    c->dR = mx;
    c->active = active;
  }
}
__global__ void __launch_bounds__(256) k_dr_finish(unsigned long long* gslots, int gsub, int32_t G, uint8_t* done,
                                                   double* g_dr, int32_t* g_iters, int32_t it, double tol,
                                                   IterCtl* c) {
  dr_fold(gslots, gsub, G, done, g_dr, g_iters, it, tol, c);
}

// Reset of the per-member state at the start of an update.
__global__ void k_member_reset(int32_t G, int gsub, unsigned long long* gslots, uint8_t* done, double* g_dr,
                               int32_t* g_iters, int64_t* g_ever) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)G * gsub; i += stride)
    gslots[i * kSlotStride] = 0ull;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < G; i += stride) {
    done[i] = 0;
    g_dr[i] = 0.0;
    g_iters[i] = 0;
    g_ever[i] = 0;
  }
}

// Fold the spread accumulator rows into the compact head and clear them; also
// clears the long-row list count for the next marking pass.
__device__ __forceinline__ void iter_finish_body(IterCtl* c) {  // one wavefront (kSlots lanes)
  const int t = threadIdx.x;
  int64_t r[kAccRows];
#pragma unroll
  for (int a = 0; a < kAccRows; a++) {
    r[a] = (int64_t)c->acc_slots[a][t * kSlotStride];
    c->acc_slots[a][t * kSlotStride] = 0ull;
    r[a] = wave_sum_i64(r[a]);
  }
  if (t == 0) {
    for (int b = 0; b < kBins; b++) c->bin_edges[b] = r[kAccEdges0 + b];
    c->ever_count = r[kAccEver];
    c->dense_cnt = r[kAccCnt];
    c->dense_edges = r[kAccAffEdges];
    c->dense_xedges = r[kAccXEdges];
    c->dense_sedges = r[kAccStayEdges];
    c->bin_out_edges = r[kAccOutEdges];
    c->dense_carry = r[kAccCarry];
    c->big_count = 0;
  }
}
__global__ void __launch_bounds__(kSlots) k_iter_finish(IterCtl* c) { iter_finish_body(c); }
// The same for a plain graph together with the L-inf change of iteration `it`
// (a batch folds the members' changes before binning instead, so that
// converged members drop out of it).
__global__ void __launch_bounds__(256) k_iter_finish_dr(unsigned long long* gslots, int gsub, uint8_t* done,
                                                        double* g_dr, int32_t* g_iters, int32_t it, double tol,
                                                        IterCtl* c) {
  dr_fold(gslots, gsub, 1, done, g_dr, g_iters, it, tol, c);
  if (threadIdx.x < kSlots) iter_finish_body(c);
}

__global__ void k_reset_ctl(IterCtl* c) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(c);
  const int64_t nw = (int64_t)(sizeof(IterCtl) / sizeof(unsigned long long));
  const int64_t keep0 = offsetof(IterCtl, n_apply) / 8, keep1 = keep0 + 6;  // apply counters stay
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nw; i += (int64_t)gridDim.x * blockDim.x)
    if (i < keep0 || i >= keep1) w[i] = 0ull;
}

// ---- small helpers
// Uniform start 1/|V| (of the vertex's member graph in a batch).
__global__ void k_init_static(double* R, double* contrib, const int32_t* __restrict__ out_deg, int32_t n,
                              const int32_t* gid, const int32_t* nk) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const double r = 1.0 / (double)(gid ? nk[gid[v]] : n);
    R[v] = r;
    contrib[v] = r / (double)out_deg[v];
  }
}
__global__ void k_init_prev(const double* r_prev, double* R, double* contrib, const int32_t* __restrict__ out_deg,
                            int32_t n, int copy) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const double r = r_prev[v];
    if (copy) R[v] = r;
    contrib[v] = r / (double)out_deg[v];
  }
}
// Caller order <-> internal order of the rank vector.
__global__ void k_gather_ranks(const double* r_ext, const int32_t* __restrict__ inv, double* R, double* contrib,
                               const int32_t* __restrict__ out_deg, int32_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double r = r_ext[inv[i]];
    R[i] = r;
    contrib[i] = r / (double)out_deg[i];
  }
}
__global__ void k_scatter_ranks(const double* R, const int32_t* __restrict__ inv, double* r_ext, int32_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r_ext[inv[i]] = R[i];
}
// Nonzero bytes of a word.
__device__ __forceinline__ int nonzero_bytes(unsigned long long w) {
  w |= w >> 4;
  w |= w >> 2;
  w |= w >> 1;
  return __popcll(w & 0x0101010101010101ull);
}
// End of an update: clears up to four byte-flag arrays of n entries (null ones
// skipped) and, when `ever` is given, counts its nonzero entries (processed
// vertices; a dense iteration leaves its stamp) into the ever accumulator and
// clears it, 16 bytes per thread (the arrays are 256-byte aligned), in one pass.
__global__ void __launch_bounds__(256) k_clear_flags(uint8_t* f0, uint8_t* f1, uint8_t* f2, uint8_t* f3, uint8_t* ever,
                                                     int32_t n, unsigned long long* acc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n16 = n / 16;
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  int64_t c = 0;
  for (int64_t i = t0; i < n16; i += stride) {
    if (f0) reinterpret_cast<uint4*>(f0)[i] = z;
    if (f1) reinterpret_cast<uint4*>(f1)[i] = z;
    if (f2) reinterpret_cast<uint4*>(f2)[i] = z;
    if (f3) reinterpret_cast<uint4*>(f3)[i] = z;
    if (ever) {
      const uint4 e = reinterpret_cast<const uint4*>(ever)[i];
      c += nonzero_bytes(((unsigned long long)e.y << 32) | e.x) + nonzero_bytes(((unsigned long long)e.w << 32) | e.z);
      reinterpret_cast<uint4*>(ever)[i] = z;
    }
  }
  for (int64_t v = n16 * 16 + t0; v < n; v += stride) {
    if (f0) f0[v] = 0;
    if (f1) f1[v] = 0;
    if (f2) f2[v] = 0;
    if (f3) f3[v] = 0;
    if (ever) {
      c += ever[v] != 0;
      ever[v] = 0;
    }
  }
  c = wave_sum_i64(c);
  if (ever && lane_id() == 0 && c)
    atomicAdd(&acc[kAccEver * (kSlots * kSlotStride) + ((blockIdx.x * 4 + threadIdx.x / kWave) % kSlots) * kSlotStride],
              (unsigned long long)c);
}

// Batch: count (and clear) the processed vertices of each member.  A thread
// walks 64 consecutive vertices (members are vertex ranges) and issues one
// atomic per member run.
__global__ void __launch_bounds__(256) k_count_ever_members(uint8_t* ever, int32_t n, const int32_t* __restrict__ gid,
                                                            int64_t* g_ever) {
  constexpr int64_t kRun = 64;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t * kRun < n; t += stride) {
    const int64_t lo = t * kRun, hi = min(lo + kRun, (int64_t)n);
    int32_t cg = -1;
    int64_t c = 0;
    for (int64_t v = lo; v < hi; v++) {
      if (!ever[v]) continue;
      ever[v] = 0;
      const int32_t gv = gid[v];
      if (gv != cg) {
        if (c) atomicAdd((unsigned long long*)&g_ever[cg], (unsigned long long)c);
        cg = gv;
        c = 0;
      }
      c++;
    }
    if (c) atomicAdd((unsigned long long*)&g_ever[cg], (unsigned long long)c);
  }
}
__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// ------------------------------------------------------------------ host side
static double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

static Bounds bounds_of(const dfpr_graph* g) {
  Bounds B;
  for (int i = 0; i < 5; i++) B.b[i] = g->bounds[i];
  return B;
}

// Bin the vertices [lo, hi) (default: all) into wl[0 ..), bins back to back.
static int bin_vertices(dfpr_graph* g, const uint8_t* flags, int32_t* wl, uint8_t* ever, hipStream_t s,
                        int64_t lo = 0, int64_t hi = -1) {
  if (hi < 0) hi = g->n;
  size_t tok;
  DFPR_TRY(g->pool.start(&tok));
  const int64_t nb = std::max<int64_t>(1, (hi - lo + kBinTile - 1) / kBinTile);
  // the cached all-vertex bins (flags == null) never drop converged members
  const MemberMask mm{flags ? g->gidv : nullptr, flags ? g->done : nullptr};
  k_bin_count<<<(unsigned)nb, 256, 0, s>>>(flags, g->in_deg, g->out_deg, lo, (int32_t)hi, mm, bounds_of(g), g->bin_blk,
                                           nb, &g->ctl->acc_slots[0][0]);
  DFPR_TRY(scan_i64(g->bin_blk, g->bin_blk, kBins * nb, g->scan_tmp, s));
  k_bin_scatter<<<(unsigned)nb, 256, 0, s>>>(flags, g->in_deg, lo, (int32_t)hi, mm, bounds_of(g), g->bin_blk, nb, wl,
                                             ever, g->ctl->bin_end);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(g->pool.stop(kTBin, tok));
  return DFPR_OK;
}

// Per-member convergence of iteration `it` (sets head.dR and head.active).
static int dr_finish(dfpr_graph* g, const dfpr_params& p, int it, hipStream_t s) {
  k_dr_finish<<<1, 256, 0, s>>>(g->gslots, g->gsub, g->ngraphs, g->done, g->g_dr, g->g_iters, it, p.tol, g->ctl);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

// p (plain graphs): also fold the L-inf change of iteration it (dr_finish).
static int finish_and_read(dfpr_graph* g, hipStream_t s, const dfpr_params* p = nullptr, int it = 0) {
  if (p)
    k_iter_finish_dr<<<1, 256, 0, s>>>(g->gslots, g->gsub, g->done, g->g_dr, g->g_iters, it, p->tol, g->ctl);
  else
    k_iter_finish<<<1, kSlots, 0, s>>>(g->ctl);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, kCtlHead, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  return DFPR_OK;
}

// Chunked marking of the rows collected in big_list.
static int mark_big(dfpr_graph* g, uint8_t* flags, hipStream_t s) {
  k_big_scan<<<1, 1024, 0, s>>>(g->big_list, &g->ctl->big_count, g->out_deg, g->big_pre);
  k_big_mark<<<1024, 256, 0, s>>>(g->big_list, &g->ctl->big_count, g->big_pre, g->out.off, g->out_deg, g->out.idx,
                                  flags);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

// Launch layout of the fused pull kernel from the bin ends and edge counts.
static bool make_layout(const int64_t* be, const int64_t* bedges, PullLayout* L) {
  static const int per_block[kBins - 1] = {256, 64, 16, 4, 1};
  const int64_t cap = 2048;
  L->blk[0] = 0;
  for (int k = 0; k < kBins; k++) {
    L->lo[k] = k ? be[k - 1] : 0;
    L->hi[k] = be[k];
    const int64_t cnt = L->hi[k] - L->lo[k];
    int64_t nb = 0;
    if (cnt > 0) {
      if (k < kBins - 1)
        nb = std::min(cap, (cnt + per_block[k] - 1) / per_block[k]);
      else
        nb = std::min<int64_t>(1024, bedges[k] / kPullChunk + cnt);
    }
    L->blk[k + 1] = L->blk[k] + (int32_t)nb;
  }
  return L->blk[kBins] > 0;
}

struct LoadChunks {
  const int32_t* wl;
  const int32_t* in_deg;
  int64_t lo;
  __device__ int64_t operator()(int64_t i) const {
    const int32_t v = wl[lo + i];
    return ((int64_t)in_deg[v] + kPullChunk - 1) / kPullChunk;
  }
};
struct StoreChunk {
  int64_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = v; }
};

// chunk_ready: chunk_pre already holds the scan for this worklist (cached
// all-vertex bins of Static/ND).
template <int MODE, bool DENSE = false>
static int pull_all(dfpr_graph* g, PullArgs a, const int32_t* wl, const int64_t* be, const int64_t* bedges,
                    int64_t* chunk_pre, bool chunk_ready, hipStream_t s, dfpr_stats* st) {
  PullLayout L;
  if (!make_layout(be, bedges, &L)) return DFPR_OK;
  size_t tok;
  DFPR_TRY(g->pool.start(&tok));
  const int64_t n5 = L.hi[kBins - 1] - L.lo[kBins - 1];
  if (n5 > 0 && !chunk_ready)
    DFPR_TRY(scan_generic(LoadChunks{wl, g->in_deg, L.lo[kBins - 1]}, StoreChunk{chunk_pre}, n5, g->scan_tmp, s));
  a.chunk_pre = chunk_pre;
  k_pull<MODE, DENSE><<<(unsigned)L.blk[kBins], 256, 0, s>>>(a, wl, L);
  if (n5 > 0)  // the chunked rows' sums and updates, after every chunk's partial is stored
    k_chunk_finish<MODE, DENSE><<<(unsigned)std::min<int64_t>(n5, 4096), 256, 0, s>>>(a, wl, L.lo[kBins - 1], n5);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(g->pool.stop(kTPull0, tok));
  st->pull_launches++;
  return DFPR_OK;
}

static void add_bins(dfpr_stats* st, const int64_t* be, const int64_t* bedges) {
  for (int k = 0; k < kBins; k++) {
    st->bin_vertices[k] += be[k] - (k ? be[k - 1] : 0);
    st->bin_edges[k] += bedges[k];
  }
}

static PullArgs make_args(dfpr_graph* g, const dfpr_params& p) {
  PullArgs a{};
  a.in_off = g->in.off;
  a.in_deg = g->in_deg;
  a.out_deg = g->out_deg;
  a.in_idx = g->in.idx;
  a.gslots = g->gslots;
  a.gsub = g->gsub;
  a.gid = g->gidv;
  a.nk = g->nk;
  a.done = g->ngraphs > 1 ? g->done : nullptr;
  a.acc = &g->ctl->acc_slots[0][0];
  a.partial = g->partial;
  a.partial_x = g->partial_x;
  a.arrive = g->arrive;
  a.alpha = p.alpha;
  a.C0 = (1.0 - p.alpha) / (double)g->n;
  a.tf = p.frontier_tol;
  a.tp = p.prune_tol;
  a.crit = p.criterion;
  a.stamp = 1;
  a.carry = 0;  // every unprocessed vertex is copied over unless a dense loop says otherwise
  return a;
}

static int ensure_all_bins(dfpr_graph* g, hipStream_t s);
template <int MODE, bool DENSE>
static int pull_parts(dfpr_graph* g, const PullArgs& a, hipStream_t s, dfpr_stats* st, bool count_bins);

// Whole-update single launch (see k_fused_loop) for graphs and batch arenas
// of at most fused_limit edges.
static bool use_fused(const dfpr_graph* g) {
  return g->fused_limit > 0 && g->m <= g->fused_limit && g->parts.size() <= (size_t)kFusedMaxParts;
}

struct FusedResult {
  int iters = 0;
  bool converged = false;
  double last = 0.0;
};

// Resident workgroups of k_fused_loop<MODE, BATCH> on the current device
// (queried once; the serving form's lanes may get here concurrently).
template <int MODE, bool BATCH>
static int fused_resident() {
  static const int resident = [] {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_fused_loop<MODE, BATCH>),
                                                     256, 0) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    return per_cu * cus;
  }();
  return resident;
}

// Resident-workgroup budget of single-launch loops on one device.  Its
// capacity is the resident grid of the most demanding single-launch kernel
// (the fewest workgroups per compute unit), and every loop is charged one
// unit per workgroup: loops whose grids fit the capacity together can all be
// resident at once, whichever kernels they run.
struct FusedBudget {
  std::mutex mu;
  std::condition_variable cv;
  int64_t capacity = 0, free = 0;
  struct Hold {
    FusedBudget& b;
    int64_t n;
    Hold(FusedBudget& bb, int64_t nn) : b(bb), n(nn) {
      std::unique_lock<std::mutex> lk(b.mu);
      b.cv.wait(lk, [&] { return b.free >= n; });
      b.free -= n;
    }
    ~Hold() {
      {
        std::lock_guard<std::mutex> lk(b.mu);
        b.free += n;
      }
      b.cv.notify_all();
    }
  };
};
static FusedBudget& fused_budget(int dev) {
  static FusedBudget budgets[64];
  static std::once_flag once[64];
  FusedBudget& b = budgets[dev & 63];
  std::call_once(once[dev & 63], [&] {
    const int r[] = {fused_resident<kSync, false>(), fused_resident<kDF, false>(), fused_resident<kDFP, false>(),
                     fused_resident<kSync, true>(),  fused_resident<kDF, true>(),  fused_resident<kDFP, true>()};
    int64_t c = r[0];
    for (int x : r) c = std::min<int64_t>(c, x);
    b.capacity = b.free = c;
  });
  return b;
}

// r_out: the final ranks in the caller's order (through g->inv when the graph
// is renumbered), written by the kernel's epilogue.
template <int MODE>
static int fused_run(dfpr_graph* g, const dfpr_params& p, PullArgs a, hipStream_t s, dfpr_stats* st,
                     FusedResult* out, double* r_out) {
  DFPR_TRY(ensure_all_bins(g, s));
  // one layout per part, with the chunk prefix of its long rows
  int nparts = (int)g->parts.size();  // <= kFusedMaxParts (use_fused)
  std::vector<FusedPart> fp(nparts);
  int64_t total = 0, chunk_base = 0, arrive_base = 0;
  for (int k = 0; k < nparts; k++) {
    const auto& pt = g->parts[k];
    make_layout(pt.bin_end, pt.bin_edges, &fp[k].L);
    fp[k].wl = g->all_bins + pt.lo;
    int64_t* pre = g->all_chunk_pre + pt.lo + (int64_t)k;
    fp[k].chunk_pre = pre;
    const int64_t n5 = fp[k].L.hi[kBins - 1] - fp[k].L.lo[kBins - 1];
    // a row of d in-edges has ceil(d / chunk) <= d / chunk + 1 chunks
    fp[k].partial = g->partial + chunk_base;
    fp[k].partial_x = g->partial_x + chunk_base;
    fp[k].arrive = g->arrive + arrive_base;
    chunk_base += pt.bin_edges[kBins - 1] / kPullChunk + n5 + 1;
    arrive_base += n5;
    if (chunk_base > g->partial_n || arrive_base > g->n) {
      set_error("single-launch loop: chunk partial sums of %lld parts exceed their arrays", (long long)nparts);
      return DFPR_EHIP;
    }
    if (n5 > 0 && !g->all_chunks_valid)
      DFPR_TRY(scan_generic(LoadChunks{fp[k].wl, g->in_deg, fp[k].L.lo[kBins - 1]}, StoreChunk{pre}, n5, g->scan_tmp,
                            s));
    total += fp[k].L.blk[kBins];
  }
  g->all_chunks_valid = true;
  if (g->ngraphs > 1) {
    // batch: the part table goes to the device through a pinned mirror, and
    // only when it changed (the layouts change with the bins, after a batch)
    const size_t tb = (size_t)nparts * sizeof(FusedPart);
    if (!g->fused_parts) {
      if (hipMalloc(&g->fused_parts, tb) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of the single-launch part table failed");
        return DFPR_ENOMEM;
      }
      DFPR_HIP(hipHostMalloc(&g->fused_parts_host, tb, hipHostMallocDefault));
      std::memset(g->fused_parts_host, 0, tb);
      g->fused_parts_stale = true;
    }
    if (g->fused_parts_stale || std::memcmp(g->fused_parts_host, fp.data(), tb) != 0) {
      DFPR_HIP(hipStreamSynchronize(s));  // the mirror may still feed an earlier copy
      std::memcpy(g->fused_parts_host, fp.data(), tb);
      DFPR_HIP(hipMemcpyAsync(g->fused_parts, g->fused_parts_host, tb, hipMemcpyHostToDevice, s));
      g->fused_parts_stale = false;
    }
  }
  const bool batch = g->ngraphs > 1;
  const int resident = batch ? fused_resident<MODE, true>() : fused_resident<MODE, false>();
  FusedBudget& budget = fused_budget(g->device);
  if (resident < 1 || budget.capacity < 1) {
    set_error("occupancy query for the single-launch loop failed");
    return DFPR_EHIP;
  }
  // the loop's share of the device: all of it alone, 1/fused_share of the
  // budget when the caller runs several updates side by side (serving lanes)
  int64_t cap = std::min<int64_t>(resident, budget.capacity);
  if (g->fused_share > 1) cap = std::max<int64_t>(1, cap / g->fused_share);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(cap, total));
  const FusedPart* parts = static_cast<const FusedPart*>(g->fused_parts);
  const int32_t* wl0 = fp[0].wl;  // a plain graph's one part, passed by value
  PullLayout L0 = fp[0].L;
  a.chunk_pre = fp[0].chunk_pre;
  a.partial = fp[0].partial;
  a.partial_x = fp[0].partial_x;
  a.arrive = fp[0].arrive;
  IterCtl* c = g->ctl;
  int mi = p.max_iters;
  double tol = p.tol;
  const int32_t* inv = g->perm ? g->inv : nullptr;
  int32_t nv = g->n;
  int32_t G = g->ngraphs;
  double* gdr = g->g_dr;
  int32_t* git = g->g_iters;
  void* args[] = {&a, &wl0, &L0, &parts, &nparts, &c, &mi, &tol, &r_out, &inv, &nv, &G, &gdr, &git};
  // The grid barrier needs all of the loop's workgroups resident at once.
  // Loops on concurrent streams (the serving form's lanes) therefore draw
  // their grids from the device's budget of resident workgroups and wait
  // while it cannot hold them; the grids are held until the loop has
  // finished on the device.  Ordinary kernels on other streams only delay a
  // loop: their workgroups finish and free their slots.
  FusedBudget::Hold hold(budget, grid);
  size_t tok;
  DFPR_TRY(g->pool.start(&tok));
  const void* fn = batch ? reinterpret_cast<const void*>(&k_fused_loop<MODE, true>)
                         : reinterpret_cast<const void*>(&k_fused_loop<MODE, false>);
  DFPR_HIP(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(256), args, 0, s));
  DFPR_TRY(g->pool.stop(kTPull0, tok));
  st->pull_launches++;
  if (G > 1 && MODE != kSync)  // processed vertices per member (the epilogue left `ever` set)
    k_count_ever_members<<<grid_for((g->n + 63) / 64, 256, 2048), 256, 0, s>>>(g->ever, g->n, g->gidv, g->g_ever);
  // fold the dense counters and read the loop's outcome
  k_iter_finish<<<1, kSlots, 0, s>>>(g->ctl);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, kCtlHead, hipMemcpyDeviceToHost, s));  // outcome in the head
  DFPR_HIP(hipStreamSynchronize(s));
  if (g->ctl_host->fused_err) {
    set_error("single-launch rank loop: grid barrier timed out");
    return DFPR_EHIP;
  }
  out->iters = (int)g->ctl_host->fused_iters;
  out->converged = g->ctl_host->fused_converged != 0;
  out->last = bits_to_double(g->ctl_host->fused_last);
  return DFPR_OK;
}

static int run_sync(dfpr_graph* g, bool cold, const dfpr_params& p, const double* r_prev, double* r_out,
                    hipStream_t s, dfpr_stats* st) {
  const int32_t n = g->n;
  k_reset_ctl<<<64, 256, 0, s>>>(g->ctl);
  DFPR_TRY(ensure_all_bins(g, s));
  const unsigned gi = grid_for(n, 256, 2048);
  double* R0 = g->perm ? g->rint : r_out;  // ranks in internal order
  if (cold)
    k_init_static<<<gi, 256, 0, s>>>(R0, g->contrib, g->out_deg, n, g->gidv, g->nk);
  else if (g->perm)
    k_gather_ranks<<<gi, 256, 0, s>>>(r_prev, g->inv, R0, g->contrib, g->out_deg, n);
  else
    k_init_prev<<<gi, 256, 0, s>>>(r_prev, r_out, g->contrib, g->out_deg, n, r_prev != r_out);
  DFPR_HIP(hipGetLastError());
  double *Ra = R0, *Rb = g->rn, *ca = g->contrib, *cb = g->contrib2;
  PullArgs a = make_args(g, p);
  int it = 0;
  double dR = 0.0;
  bool conv = false;
  bool ranks_out = false;
  if (use_fused(g)) {
    a.R = Ra;
    a.Rw = Rb;
    a.contrib = ca;
    a.cw = cb;
    FusedResult fr;
    DFPR_TRY(fused_run<kSync>(g, p, a, s, st, &fr, r_out));
    it = fr.iters;
    conv = fr.converged;
    dR = fr.last;
    st->vertex_updates += (int64_t)it * n;
    st->edges_pulled += (int64_t)it * g->m;
    st->pull_bytes += (double)it * (36.0 * n + 12.0 * (double)g->m);
    if (it & 1) std::swap(Ra, Rb);
    ranks_out = true;  // the loop ran to the end (converged or the cap) and wrote r_out
  }
  for (; !conv && it < p.max_iters; it++) {
    a.contrib = ca;
    a.R = Ra;
    a.Rw = Rb;
    a.cw = cb;
    DFPR_TRY((pull_parts<kSync, false>(g, a, s, st, true)));
    if (g->ngraphs > 1) DFPR_TRY(dr_finish(g, p, it, s));
    DFPR_TRY(finish_and_read(g, s, g->ngraphs > 1 ? nullptr : &p, it));
    dR = bits_to_double(g->ctl_host->dR);
    st->vertex_updates += n;
    st->edges_pulled += g->m;
    st->pull_bytes += 36.0 * n + 12.0 * (double)g->m;
    std::swap(Ra, Rb);
    std::swap(ca, cb);
    if (g->ctl_host->active == 0) {
      conv = true;
      it++;
      break;
    }
  }
  if (ranks_out) {
  } else if (g->perm) {
    k_scatter_ranks<<<gi, 256, 0, s>>>(Ra, g->inv, r_out, n);
  } else if (Ra != r_out) {
    DFPR_HIP(hipMemcpyAsync(r_out, Ra, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  // ranks now come from a full solve: pending batch marks are void
  if (g->pending_any) {
    k_fill_u8<<<gi, 256, 0, s>>>(g->pend_src, n, 0);
    k_fill_u8<<<gi, 256, 0, s>>>(g->flag_cur, n, 0);
    g->pending_any = false;
  }
  DFPR_HIP(hipStreamSynchronize(s));
  st->iterations = it;
  st->converged = conv ? 1 : 0;
  st->last_delta = dR;
  st->ever_affected = n;
  return DFPR_OK;
}

// dense pull over all vertices needs the cached all-vertex bins
static int ensure_all_bins(dfpr_graph* g, hipStream_t s) {
  if (g->all_bins_valid) return DFPR_OK;
  for (auto& pt : g->parts) {
    DFPR_TRY(bin_vertices(g, nullptr, g->all_bins + pt.lo, nullptr, s, pt.lo, pt.hi));
    DFPR_TRY(finish_and_read(g, s));
    std::copy(g->ctl_host->bin_end, g->ctl_host->bin_end + kBins, pt.bin_end);
    std::copy(g->ctl_host->bin_edges, g->ctl_host->bin_edges + kBins, pt.bin_edges);
  }
  g->all_bins_valid = true;
  g->all_chunks_valid = false;
  return DFPR_OK;
}

// One pull over every vertex: one launch per part.
template <int MODE, bool DENSE>
static int pull_parts(dfpr_graph* g, const PullArgs& a, hipStream_t s, dfpr_stats* st, bool count_bins) {
  for (size_t k = 0; k < g->parts.size(); k++) {
    const auto& pt = g->parts[k];
    DFPR_TRY((pull_all<MODE, DENSE>(g, a, g->all_bins + pt.lo, pt.bin_end, pt.bin_edges,
                                    g->all_chunk_pre + pt.lo + (int64_t)k, g->all_chunks_valid, s, st)));
    if (count_bins) add_bins(st, pt.bin_end, pt.bin_edges);
  }
  g->all_chunks_valid = true;
  return DFPR_OK;
}

// One dense iteration through the two-phase pull; the layout is rebuilt first
// when the graph changed since it was built (timed with the binning work).
template <int MODE>
static int tp_pull(dfpr_graph* g, const PullArgs& a, bool use_x, hipStream_t s, dfpr_stats* st) {
  TwoPhase& t = *g->tp;
  size_t tok;
  if (t.built != g->csr_version) {
    DFPR_TRY(g->pool.start(&tok));
    DFPR_TRY(tp_build(g, s));
    DFPR_TRY(g->pool.stop(kTBin, tok));
  }
  DFPR_TRY(g->pool.start(&tok));
  DFPR_TRY(tp_phases(g, a.contrib, use_x ? a.x_in : nullptr, s));
  k_tp_finish<MODE><<<(unsigned)((g->n + 255) / 256), 256, 0, s>>>(a, g->n, t.glo.as<uint64_t>(), t.ghi.as<uint64_t>(),
                                                                    t.gfl.as<uint32_t>(), t.split.as<uint8_t>());
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(g->pool.stop(kTPull1, tok));
  st->two_phase_passes++;
  return DFPR_OK;
}

// DF / DF-P.  Each iteration runs in one of two forms with the same result:
//  frontier: pull over the binned worklist of affected vertices (ranks in
//    place), commit their contributions and push-mark the out-rows of the
//    expanding vertices into the next flags, then bin those flags;
//  dense: pull over every vertex; a vertex is affected iff its own keep flag
//    is set or an in-neighbour expanded (read from the in-neighbours' expand
//    flags, so no marks are written); ranks and contributions ping-pong.
// The affected sets, the per-vertex sums (same bins, same order) and so the
// ranks are identical.  The forms differ in how the expansion of an iteration
// reaches the next one, and that is what the choice weighs: the frontier form
// pushes a mark along every out-edge of the expanding vertices (a scattered
// byte store each), the dense form makes every vertex it does not keep scan
// its in-neighbours' expand flags (a gathered byte each, |E| minus the
// in-edges of the affected set) and carries every vertex over (about one
// gathered edge's time per vertex).  An iteration runs dense when
//     |E| - (in-edges of the affected set) + |V| < w * (out-edges to mark),
// w = dense_switch: 0 never dense, infinity always; the default 1 prices a
// pushed mark like a scanned flag, which measurement on large R-MAT graphs
// supports.  The out-edges to mark are those of the last iteration's
// expanding vertices (counted in its pull), the best predictor of the next
// ones; before the first iteration, those of the initially marked vertices.
static bool prefer_dense(double w, int64_t m, int32_t n, int64_t aff_edges, int64_t mark_edges) {
  if (std::isinf(w)) return true;
  return (double)(m - aff_edges) + (double)n < w * (double)mark_edges;
}
template <int MODE>
static int run_frontier(dfpr_graph* g, const dfpr_params& p, const double* r_prev, double* r_out, hipStream_t s,
                        dfpr_stats* st) {
  const int32_t n = g->n;
  const int64_t m = g->m;
  const unsigned gi = grid_for(n, 256, 2048);
  k_reset_ctl<<<64, 256, 0, s>>>(g->ctl);
  const bool async = (p.flags & DFPR_FLAG_ASYNC) != 0;
  double* Ra = g->perm ? g->rint : r_out;  // current ranks, internal order
  double* Rb = g->rn;
  double* ca = g->contrib;
  double* cb = g->contrib2;
  if (g->perm)
    k_gather_ranks<<<gi, 256, 0, s>>>(r_prev, g->inv, Ra, ca, g->out_deg, n);
  else
    k_init_prev<<<gi, 256, 0, s>>>(r_prev, r_out, ca, g->out_deg, n, r_prev != r_out);
  // initial marking: out(u) of pending sources (+ deletion targets already in flag_cur)
  size_t tok;
  DFPR_TRY(g->pool.start(&tok));
  k_mark_pending<<<gi, 256, 0, s>>>(g->pend_src, n, g->out.off, g->out_deg, g->out.idx, g->flag_cur, g->big_list,
                                    &g->ctl->big_count, kPendBigRow);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(mark_big(g, g->flag_cur, s));
  DFPR_TRY(g->pool.stop(kTMark, tok));
  g->pending_any = false;
  if (use_fused(g)) {
    // every iteration in the dense form, all in one launch
    PullArgs a = make_args(g, p);
    a.R = Ra;
    a.Rw = async ? Ra : Rb;  // asynchronous: one rank and one contribution vector
    a.contrib = ca;
    a.cw = async ? ca : cb;
    a.stay_in = g->flag_cur;
    a.x_in = g->xflag;
    a.stay_out = g->flag_next;
    a.x_out = g->xflag2;
    a.ever = g->ever;
    a.use_x = 0;
    FusedResult fr;
    // the kernel's epilogue writes r_out, clears the flags and counts the
    // processed vertices; fused_run read the outcome back
    DFPR_TRY(fused_run<MODE>(g, p, a, s, st, &fr, r_out));
    const IterCtl* h = g->ctl_host;
    st->vertex_updates += h->dense_cnt;
    st->edges_pulled += h->dense_edges;
    st->pull_bytes += (double)fr.iters * (24.0 * n + 5.0 * (double)m) +
                      8.0 * (double)(h->dense_cnt + h->dense_carry) + 8.0 * (double)h->dense_edges;
    st->dense_iterations += fr.iters;
    st->iterations = fr.iters;
    st->converged = fr.converged ? 1 : 0;
    st->last_delta = fr.last;
    st->ever_affected = g->ctl_host->ever_count;
    return DFPR_OK;
  }
  DFPR_TRY(bin_vertices(g, g->flag_cur, g->worklist, g->ever, s));
  DFPR_TRY(finish_and_read(g, s));
  uint8_t *cur = g->flag_cur, *next = g->flag_next, *xa = g->xflag, *xb = g->xflag2;
  bool dense = false, use_x = false;
  int64_t front_edges = 0, front_cnt = 0;
  int64_t mark_edges = g->ctl_host->bin_out_edges;  // before the first pull: out-edges of the marked vertices
  {
    const int64_t* h = g->ctl_host->bin_edges;
    for (int k = 0; k < kBins; k++) front_edges += h[k];
    front_cnt = g->ctl_host->bin_end[kBins - 1];
  }
  PullArgs a = make_args(g, p);
  int it = 0;
  double dR = 0.0;
  bool conv = false;
  int carry = 0;  // stamp of the previous dense iteration (0: the vectors are not in step)
  const bool use_tp = g->tp && g->tp->on && g->ngraphs == 1 && !async;
  bool tp_ran = false;
  for (it = 0; it < p.max_iters; it++) {
    if (!dense && front_cnt > 0 && prefer_dense(p.dense_switch, m, n, front_edges, mark_edges)) {
      dense = true;  // the complete frontier is in `cur`; no expand flags to read
      use_x = false;
      carry = 0;     // the frontier form updated one vector in place
    }
    if (dense) {
      if (!use_tp) DFPR_TRY(ensure_all_bins(g, s));  // the gather pull's all-vertex bins
      a.contrib = ca;
      a.R = Ra;
      a.Rw = async ? Ra : Rb;
      a.cw = async ? ca : cb;
      a.cmut = nullptr;
      a.stay_in = cur;
      a.x_in = xa;
      a.stay_out = next;
      a.x_out = xb;
      a.ever = g->ever;
      a.use_x = use_x ? 1 : 0;
      a.stamp = dense_stamp(it);
      a.carry = async ? 0 : carry;
      const bool two = use_tp;
      tp_ran = tp_ran || two;
      if (two)
        DFPR_TRY(tp_pull<MODE>(g, a, use_x, s, st));
      else
        DFPR_TRY((pull_parts<MODE, true>(g, a, s, st, false)));
      carry = a.stamp;
      if (g->ngraphs > 1) DFPR_TRY(dr_finish(g, p, it, s));
      DFPR_TRY(finish_and_read(g, s, g->ngraphs > 1 ? nullptr : &p, it));
      const IterCtl* h = g->ctl_host;
      dR = bits_to_double(h->dR);
      st->vertex_updates += h->dense_cnt;
      st->edges_pulled += h->dense_edges;
      if (two)
        st->two_phase_bytes += 22.0 * (double)m + 65.0 * n + 8.0 * (double)(h->dense_cnt + h->dense_carry) +
                               4.0 * (double)g->tp->n1 * g->tp->nB;
      else
        st->pull_bytes += 24.0 * n + 8.0 * (double)(h->dense_cnt + h->dense_carry) + 5.0 * (double)m +
                          8.0 * (double)h->dense_edges;
      st->dense_iterations++;
      if (!async) {
        std::swap(Ra, Rb);
        std::swap(ca, cb);
      }
      std::swap(cur, next);  // cur = keep flags of the next iteration
      std::swap(xa, xb);     // xa = expand flags of this iteration
      use_x = true;
      // next frontier: the kept vertices (affected again for sure) plus the
      // out-neighbours of the expanding ones, whose in-degrees are estimated
      // by the mean; switch back to the frontier form when that is small (the
      // dense form scans every vertex's in-neighbour flags however few
      // vertices are affected)
      front_edges = std::min<int64_t>(
          m, h->dense_sedges + (int64_t)((double)h->dense_xedges * ((double)m / (double)n)));
      if (h->active == 0) {
        conv = true;
        it++;
        break;
      }
      // leave the dense form when pushing this iteration's marks costs less
      // than scanning the flags of the vertices the next one will not keep
      mark_edges = h->dense_xedges;
      if (!prefer_dense(p.dense_switch, m, n, front_edges, mark_edges)) {
        // back to the frontier form: mark out(v) of this iteration's expanders
        // into the keep flags (clears xa), then bin
        k_mark_pending<<<gi, 256, 0, s>>>(xa, n, g->out.off, g->out_deg, g->out.idx, cur, g->big_list, &g->ctl->big_count,
                                          kBigRow);
        DFPR_HIP(hipGetLastError());
        DFPR_TRY(mark_big(g, cur, s));
        k_fill_u8<<<gi, 256, 0, s>>>(next, n, 0);
        DFPR_TRY(bin_vertices(g, cur, g->worklist, g->ever, s));
        DFPR_TRY(finish_and_read(g, s));
        dense = false;
        front_edges = 0;
        for (int k = 0; k < kBins; k++) front_edges += g->ctl_host->bin_edges[k];
        front_cnt = g->ctl_host->bin_end[kBins - 1];
      }
      continue;
    }
    int64_t be[kBins], bedges[kBins];
    std::copy(g->ctl_host->bin_end, g->ctl_host->bin_end + kBins, be);
    std::copy(g->ctl_host->bin_edges, g->ctl_host->bin_edges + kBins, bedges);
    const int64_t cnt = front_cnt;
    st->vertex_updates += cnt;
    st->edges_pulled += front_edges;
    st->pull_bytes += 30.0 * cnt + 12.0 * (double)front_edges;
    add_bins(st, be, bedges);
    if (cnt == 0) {  // nothing affected: the L-inf change of this iteration is 0
      DFPR_TRY(dr_finish(g, p, it, s));  // retires every member still running
      dR = 0.0;
      conv = true;
      it++;
      break;
    }
    a.contrib = ca;
    a.cmut = async ? ca : nullptr;
    a.R = Ra;
    a.next = next;
    a.xflag = xa;
    DFPR_TRY(pull_all<MODE>(g, a, g->worklist, be, bedges, g->chunk_pre, false, s, st));
    DFPR_TRY(g->pool.start(&tok));
    k_commit_expand<<<grid_for(cnt, 256, 2048), 256, 0, s>>>(g->worklist, cnt, Ra, ca, g->out.off, g->out_deg, g->out.idx, cur,
                                                             next, xa, g->big_list, &g->ctl->big_count);
    DFPR_HIP(hipGetLastError());
    DFPR_TRY(mark_big(g, next, s));
    DFPR_TRY(g->pool.stop(kTCommit, tok));
    if (g->ngraphs > 1) DFPR_TRY(dr_finish(g, p, it, s));  // before binning: converged members drop out
    std::swap(cur, next);
    DFPR_TRY(bin_vertices(g, cur, g->worklist, g->ever, s));
    DFPR_TRY(finish_and_read(g, s, g->ngraphs > 1 ? nullptr : &p, it));
    dR = bits_to_double(g->ctl_host->dR);
    front_edges = 0;
    for (int k = 0; k < kBins; k++) front_edges += g->ctl_host->bin_edges[k];
    front_cnt = g->ctl_host->bin_end[kBins - 1];
    mark_edges = g->ctl_host->dense_xedges;  // out-edges this iteration's expanders marked
    if (g->ctl_host->active == 0) {
      conv = true;
      it++;
      break;
    }
  }
  if (g->perm)
    k_scatter_ranks<<<gi, 256, 0, s>>>(Ra, g->inv, r_out, n);
  else if (Ra != r_out)
    DFPR_HIP(hipMemcpyAsync(r_out, Ra, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
  // leave every flag array clear for the next batch (converged members of a
  // batch may leave flags in both keep arrays)
  {
    const bool dense_used = st->dense_iterations > 0;
    uint8_t* nx = (g->ngraphs > 1 || dense_used) ? next : nullptr;
    k_clear_flags<<<grid_for(n / 16 + 1, 256, 65536), 256, 0, s>>>(
        cur, nx, dense_used ? xa : nullptr, dense_used ? xb : nullptr, g->ngraphs > 1 ? nullptr : g->ever, n,
        &g->ctl->acc_slots[0][0]);
  }
  if (g->ngraphs > 1)
    k_count_ever_members<<<grid_for((n + 63) / 64, 256, 2048), 256, 0, s>>>(g->ever, n, g->gidv, g->g_ever);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(finish_and_read(g, s));
  g->flag_cur = cur;
  g->flag_next = next;
  g->xflag = xa;
  g->xflag2 = xb;
  if (tp_ran) {  // phase one flags contributions outside [0, 2^31)
    int32_t bad = 0;
    DFPR_HIP(hipMemcpyAsync(&bad, g->tp->bad.p, sizeof(bad), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    if (bad) {
      DFPR_HIP(hipMemsetAsync(g->tp->bad.p, 0, sizeof(bad), s));
      set_error("two-phase pull: a contribution outside [0, 2^31) (ranks must be non-negative and below 2^31)");
      return DFPR_EINVAL;
    }
  }
  st->iterations = it;
  st->converged = conv ? 1 : 0;
  st->last_delta = dR;
  st->ever_affected = g->ctl_host->ever_count;
  return DFPR_OK;
}

// Pinned host mirror of the per-member results.
struct MemberHost {
  double* dr;
  int64_t* ever;
  int32_t* iters;
  uint8_t* done;
};
static MemberHost member_host(dfpr_graph* g) {
  const size_t G = (size_t)g->ngraphs;
  char* b = static_cast<char*>(g->g_host);
  MemberHost h;
  h.dr = reinterpret_cast<double*>(b);
  h.ever = reinterpret_cast<int64_t*>(b + 8 * G);
  h.iters = reinterpret_cast<int32_t*>(b + 32 * G);  // g_eff's mirror sits at 16 G
  h.done = reinterpret_cast<uint8_t*>(b + 36 * G);
  return h;
}

int update_ranks(dfpr_graph* g, dfpr_mode mode, const dfpr_params& p, const double* r_prev, double* r_out,
                 hipStream_t s, dfpr_stats* st_out, dfpr_stats* per_member) {
  dfpr_stats st{};
  EventPool& ep = g->pool;
  ep.reset(g->timing || (p.flags & DFPR_FLAG_TIMING) != 0, s);
  size_t tok;
  DFPR_TRY(ep.start(&tok));
  k_member_reset<<<grid_for((int64_t)g->ngraphs * g->gsub, 256, 64), 256, 0, s>>>(
      g->ngraphs, g->gsub, g->gslots, g->done, g->g_dr, g->g_iters, g->g_ever);
  DFPR_HIP(hipGetLastError());
  int rc;
  switch (mode) {
    case DFPR_STATIC: rc = run_sync(g, true, p, r_prev, r_out, s, &st); break;
    case DFPR_ND: rc = run_sync(g, false, p, r_prev, r_out, s, &st); break;
    case DFPR_DF: rc = run_frontier<kDF>(g, p, r_prev, r_out, s, &st); break;
    default: rc = run_frontier<kDFP>(g, p, r_prev, r_out, s, &st); break;
  }
  if (rc != DFPR_OK) return rc;
  if (ep.on) {
    DFPR_TRY(ep.stop(kTTotal, tok));
    DFPR_HIP(hipStreamSynchronize(s));
    double ms[kTNum] = {0};
    int cnt[kTNum] = {0};
    DFPR_TRY(ep.collect(ms, cnt));
    st.ms_total = ms[kTTotal];
    st.ms_pull = ms[kTPull0];
    st.ms_two_phase = ms[kTPull1];
    st.ms_commit = ms[kTCommit];
    st.ms_bin = ms[kTBin];
    st.ms_mark = ms[kTMark];
  }
  if (g->ngraphs > 1) {
    // batch: iteration counts, convergence and changes are per member; the
    // totals report the slowest member and the sum of processed vertices
    const size_t G = (size_t)g->ngraphs;
    const MemberHost h = member_host(g);
    DFPR_HIP(hipMemcpyAsync(h.dr, g->g_dr, G * sizeof(double), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(h.ever, g->g_ever, G * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(h.iters, g->g_iters, G * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(h.done, g->done, G, hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    const bool sync_mode = mode == DFPR_STATIC || mode == DFPR_ND;
    int64_t ever = 0;
    double worst = 0.0;
    int32_t conv = 1;
    for (size_t k = 0; k < G; k++) {
      const int64_t nkk = g->vbase[k + 1] - g->vbase[k];
      const int64_t ek = sync_mode ? nkk : h.ever[k];
      ever += ek;
      worst = std::max(worst, h.dr[k]);
      conv &= h.done[k] ? 1 : 0;
      if (per_member) {
        dfpr_stats m{};
        m.iterations = h.iters[k];
        m.converged = h.done[k] ? 1 : 0;
        m.last_delta = h.dr[k];
        m.ever_affected = ek;
        per_member[k] = m;
      }
    }
    st.ever_affected = ever;
    st.converged = conv;
    st.last_delta = worst;
  }
  if (st_out) *st_out = st;
  return DFPR_OK;
}

// ---- autotuner: coordinate descent over the five bin thresholds, each
// candidate timed on Static iterations (pull kernel only, HIP events).
static int time_pull(dfpr_graph* g, double* r, hipStream_t s, double* ms) {
  dfpr_params p;
  p.alpha = 0.85;
  p.tol = 1e-300;  // run the full iteration count
  p.frontier_tol = p.prune_tol = 1e-6;
  p.dense_switch = 0.4;
  p.max_iters = 4;
  p.flags = DFPR_FLAG_TIMING;
  p.criterion = DFPR_CRIT_RELATIVE;
  p.reserved = 0;
  // pending marks must survive: run_sync clears them only if pending_any.
  // Candidates are timed on the path the graph's updates take (the single
  // launch, where its limit admits the graph).
  const bool pend = g->pending_any;
  g->pending_any = false;
  // the minimum over repeats (at least 3, until 4 ms have been timed): one
  // short launch on a small graph is too noisy to rank candidates 3 % apart
  double best = 0.0, timed = 0.0;
  int rc = DFPR_OK;
  for (int rep = 0; rep < 32 && rc == DFPR_OK && (rep < 3 || timed < 4.0); rep++) {
    dfpr_stats st{};
    rc = update_ranks(g, DFPR_STATIC, p, nullptr, r, s, &st);
    const double t = st.pull_launches ? st.ms_pull / st.pull_launches : 0.0;
    best = rep == 0 ? t : std::min(best, t);
    timed += st.ms_pull;
  }
  g->pending_any = pend;
  if (rc != DFPR_OK) return rc;
  *ms = best;
  return DFPR_OK;
}

// Rows of more than `t` in-edges: the tuner's stand-in for a frontier that
// keeps a graph's hubs (on hub-heavy graphs a DF-P frontier is mostly these
// rows plus short ones, and its pull is set by how the long rows are split).
__global__ void k_flag_long_rows(const int32_t* __restrict__ in_deg, int32_t n, int32_t t, uint8_t* flags) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    flags[v] = in_deg[v] > t ? 1 : 0;
}

// Pull launch over the flagged rows alone (Equation 1 into the scratch
// vectors): the minimum launch time over repeats, then the change slots
// folded and cleared as after any iteration.
static int time_pull_rows(dfpr_graph* g, double* r, const uint8_t* flags, hipStream_t s, double* ms) {
  DFPR_TRY(bin_vertices(g, flags, g->worklist, nullptr, s));
  DFPR_TRY(finish_and_read(g, s));
  int64_t be[kBins], bedges[kBins];
  std::copy(g->ctl_host->bin_end, g->ctl_host->bin_end + kBins, be);
  std::copy(g->ctl_host->bin_edges, g->ctl_host->bin_edges + kBins, bedges);
  *ms = 0.0;
  if (be[kBins - 1] == 0) return DFPR_OK;
  dfpr_params p;
  p.alpha = 0.85;
  p.tol = 1e-300;
  p.frontier_tol = p.prune_tol = 1e-6;
  p.dense_switch = 0.4;
  p.max_iters = 1;
  p.flags = 0;
  p.criterion = DFPR_CRIT_RELATIVE;
  p.reserved = 0;
  PullArgs a = make_args(g, p);
  a.R = r;
  a.Rw = g->rn;
  a.contrib = g->contrib;
  a.cw = g->contrib2;
  hipEvent_t e0, e1;
  DFPR_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DFPR_EHIP;
  }
  dfpr_stats st{};
  double best = 0.0, timed = 0.0;
  int rc = DFPR_OK;
  for (int rep = 0; rep < 32 && rc == DFPR_OK && (rep < 3 || timed < 2.0); rep++) {
    float t = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess) rc = DFPR_EHIP;
    if (rc == DFPR_OK) rc = pull_all<kSync, false>(g, a, g->worklist, be, bedges, g->chunk_pre, rep > 0, s, &st);
    if (rc == DFPR_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      rc = DFPR_EHIP;
    best = rep == 0 ? t : std::min(best, (double)t);
    timed += t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == DFPR_OK) rc = finish_and_read(g, s, &p, 0);
  *ms = best;
  return rc;
}

int autotune(dfpr_graph* g, hipStream_t s, int32_t* bounds_out, double* ms_out) {
  double* r = nullptr;
  uint8_t* longf = nullptr;  // rows of more than 128 in-edges (plain graphs)
  if (hipMalloc((void**)&r, (size_t)g->n * sizeof(double)) != hipSuccess ||
      (g->ngraphs == 1 && hipMalloc((void**)&longf, (size_t)g->n) != hipSuccess)) {
    (void)hipGetLastError();
    if (r) (void)hipFree(r);
    set_error("autotune: device allocation failed");
    return DFPR_ENOMEM;
  }
  if (longf) {
    k_flag_long_rows<<<grid_for(g->n, 256, 65536), 256, 0, s>>>(g->in_deg, g->n, 128, longf);
    if (hipGetLastError() != hipSuccess) {
      (void)hipFree(r);
      (void)hipFree(longf);
      return DFPR_EHIP;
    }
  }
  static const int32_t cand[5][6] = {{2, 4, 8, 16, 0, 0},
                                     {8, 16, 32, 64, 0, 0},
                                     {32, 64, 128, 256, 512, 0},
                                     {256, 512, 1024, 2048, 4096, 8192},
                                     {4096, 8192, 16384, 32768, 131072, 1 << 20}};
  int32_t best[5];
  std::copy(g->bounds, g->bounds + 5, best);
  double best_ms = 0.0, best_static = 0.0, last_static = 0.0;
  int rc = DFPR_OK;
  auto eval = [&](const int32_t* b, double* ms) {
    const int32_t keep[5] = {g->bounds[0], g->bounds[1], g->bounds[2], g->bounds[3], g->bounds[4]};
    std::copy(b, b + 5, g->bounds);
    g->all_bins_valid = false;
    int e = time_pull(g, r, s, ms);  // first call rebuilds the bins
    if (e == DFPR_OK) e = time_pull(g, r, s, ms);
    // plain graphs: plus the pull over the long rows alone, which the
    // all-vertex pull hides (its other rows keep the device busy while a
    // workgroup walks a long row) and a hub-heavy frontier does not
    double ml = 0.0;
    if (e == DFPR_OK && longf) e = time_pull_rows(g, r, longf, s, &ml);
    last_static = *ms;
    *ms += ml;
    std::copy(keep, keep + 5, g->bounds);
    g->all_bins_valid = false;
    return e;
  };
  rc = eval(best, &best_ms);
  best_static = last_static;
  for (int pass = 0; pass < 2 && rc == DFPR_OK; pass++) {
    for (int k = 4; k >= 0 && rc == DFPR_OK; k--) {
      for (int c = 0; c < 6 && rc == DFPR_OK; c++) {
        const int32_t v = cand[k][c];
        if (v == 0 || v == best[k]) continue;
        int32_t b[5];
        std::copy(best, best + 5, b);
        b[k] = v;
        bool ok = b[0] >= 1;
        for (int i = 1; i < 5; i++) ok = ok && b[i] >= b[i - 1];
        if (!ok) continue;
        double ms = 0.0;
        rc = eval(b, &ms);
        // a change must win by 3 %: timing noise alone does not move the thresholds
        if (rc == DFPR_OK && ms < 0.97 * best_ms) {
          best_ms = ms;
          best_static = last_static;
          std::copy(b, b + 5, best);
        }
      }
    }
  }
  (void)hipFree(r);
  if (longf) (void)hipFree(longf);
  if (rc != DFPR_OK) return rc;
  std::copy(best, best + 5, g->bounds);
  g->all_bins_valid = false;
  if (bounds_out) std::copy(best, best + 5, bounds_out);
  if (ms_out) *ms_out = best_static;
  return DFPR_OK;
}

}  // namespace dfpr
