// Rank engine: Static, Naive-dynamic, Dynamic Frontier and Dynamic Frontier
// with Pruning (Algorithm 1; Equations 1 and 2), pull-based (Section 4.4),
// iterated synchronously: every read of iteration i sees the ranks of
// iteration i, prunes and marks take effect in iteration i+1.
//
// Per iteration:
//   bin      affected flags -> worklist split by in-degree (lane / wave / chunk)
//   pull     c = sum of contrib[u] over in(v); the Equation 1 or 2 rank; the
//            L-inf change reduced per workgroup into one 64-bit atomicMax
//   commit   contrib[v] = R[v]/|out(v)| for the processed vertices (DF, DF-P)
//            and marking of out(v) for vertices whose relative change > tau_f
// Static and ND process every vertex and ping-pong two rank/contribution
// buffers instead of committing.
#include <algorithm>

#include "prim.hpp"

namespace dfpr {

enum : int { kSync = 0, kDF = 2, kDFP = 3 };  // kSync = Static and ND (Equation 1, no flags)

struct PullArgs {
  const int32_t* __restrict__ in_off;
  const int32_t* __restrict__ in_idx;
  const int32_t* __restrict__ out_off;
  const double* __restrict__ contrib;
  double* R;       // ranks of this iteration (DF/DF-P: written in place)
  double* Rw;      // Static/ND: ranks of the next iteration
  double* cw;      // Static/ND: contributions of the next iteration
  uint8_t* next;   // DF/DF-P: affected in the next iteration
  uint8_t* xflag;  // DF/DF-P: expands
  unsigned long long* dR;
  double alpha, C0, tf, tp;
};

// Equation 1 (DF, Static, ND) or Equation 2 (DF-P) for vertex v from its
// in-neighbour sum c; returns |r - R[v]|.  Same operation order as the
// algorithm states it; the library is built without FMA contraction.
template <int MODE>
__device__ __forceinline__ double vertex_finish(const PullArgs& a, int32_t v, double c) {
  const double d = (double)(a.out_off[v + 1] - a.out_off[v]);
  const double Rv = a.R[v];
  double r;
  if (MODE == kDFP)
    r = (1.0 / (1.0 - a.alpha / d)) * (a.C0 + a.alpha * (c - Rv / d));
  else
    r = a.C0 + a.alpha * c;
  const double dr = fabs(r - Rv);
  if (MODE == kSync) {
    a.Rw[v] = r;
    a.cw[v] = r / d;
  } else {
    a.R[v] = r;
    const double rel = dr / fmax(r, Rv);
    if (!(MODE == kDFP && rel <= a.tp)) a.next[v] = 1;  // prune (DF-P) or keep
    if (rel > a.tf) a.xflag[v] = 1;                      // expand
  }
  return dr;
}

// Workgroup max of non-negative doubles, then one atomicMax on the bit
// pattern (monotone for non-negative IEEE doubles).
__device__ __forceinline__ void block_max_commit(double x, unsigned long long* dR) {
  __shared__ double sh[1024 / kWave];
  x = wave_max(x);
  if (lane_id() == 0) sh[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); w++) m = fmax(m, sh[w]);
    if (m > 0.0) atomicMax(dR, (unsigned long long)__double_as_longlong(m));
  }
}

// ---- lane bin: one vertex per lane, left fold in ascending source order
template <int MODE>
__global__ void __launch_bounds__(256) k_pull_lane(PullArgs a, const int32_t* __restrict__ wl, int64_t lo,
                                                   int64_t hi) {
  double mx = 0.0;
  for (int64_t k = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < hi;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = wl[k];
    const int32_t s = a.in_off[v], e = a.in_off[v + 1];
    double c = 0.0;
    for (int32_t p = s; p < e; p++) c = c + a.contrib[a.in_idx[p]];
    mx = fmax(mx, vertex_finish<MODE>(a, v, c));
  }
  block_max_commit(mx, a.dR);
}

// ---- wave bin: one vertex per wavefront; per-lane strided sums + butterfly
template <int MODE>
__global__ void __launch_bounds__(256) k_pull_wave(PullArgs a, const int32_t* __restrict__ wl, int64_t lo,
                                                   int64_t hi) {
  const int lane = lane_id();
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
  double mx = 0.0;
  for (int64_t k = lo + blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; k < hi; k += nw) {
    const int32_t v = wl[k];
    const int32_t s = a.in_off[v], e = a.in_off[v + 1];
    double part = 0.0;
    for (int32_t p = s + lane; p < e; p += kWave) part += a.contrib[a.in_idx[p]];
    const double c = wave_sum(part);
    if (lane == 0) mx = fmax(mx, vertex_finish<MODE>(a, v, c));
  }
  block_max_commit(mx, a.dR);
}

// ---- chunk bin: rows split into kPullChunk-edge work items over workgroups;
// partial sums land in `partial`, combined in chunk order by k_pull_chunk_finish.
struct LoadChunks {
  const int32_t* wl;
  const int32_t* in_off;
  int64_t lo;
  __device__ int64_t operator()(int64_t i) const {
    const int32_t v = wl[lo + i];
    return ((int64_t)(in_off[v + 1] - in_off[v]) + kPullChunk - 1) / kPullChunk;
  }
};
struct StoreI64r {
  int64_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = v; }
};

__device__ __forceinline__ int64_t upper_bound_i64(const int64_t* a, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_pull_chunk(PullArgs a, const int32_t* __restrict__ wl, int64_t lo,
                                                    int64_t nv, const int64_t* __restrict__ chunk_pre,
                                                    double* partial) {
  __shared__ double sh[256 / kWave];
  const int64_t total = chunk_pre[nv];
  for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
    const int64_t j = upper_bound_i64(chunk_pre, 0, nv + 1, q) - 1;
    const int32_t v = wl[lo + j];
    const int32_t s = a.in_off[v] + (int32_t)((q - chunk_pre[j]) * kPullChunk);
    const int32_t e = min(s + kPullChunk, a.in_off[v + 1]);
    double part = 0.0;
    for (int32_t p = s + (int32_t)threadIdx.x; p < e; p += (int32_t)blockDim.x) part += a.contrib[a.in_idx[p]];
    part = wave_sum(part);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < 256 / kWave; w++) t += sh[w];
      partial[q] = t;
    }
    __syncthreads();
  }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_pull_chunk_finish(PullArgs a, const int32_t* __restrict__ wl, int64_t lo,
                                                           int64_t nv, const int64_t* __restrict__ chunk_pre,
                                                           const double* __restrict__ partial) {
  double mx = 0.0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nv; j += (int64_t)gridDim.x * blockDim.x) {
    double c = 0.0;
    for (int64_t q = chunk_pre[j]; q < chunk_pre[j + 1]; q++) c += partial[q];
    mx = fmax(mx, vertex_finish<MODE>(a, wl[lo + j], c));
  }
  block_max_commit(mx, a.dR);
}

// ---- marking of out-rows.  Short rows by their lane, medium rows by the
// whole wavefront, rows longer than kBigRow appended to big_list for the
// chunked pass.  Used by the initial marking and by the expansion.
__device__ __forceinline__ void mark_out_rows(bool want, int32_t v, int32_t os, int32_t oe,
                                              const int32_t* __restrict__ out_idx, uint8_t* flags,
                                              int32_t* big_list, int64_t* big_count) {
  const int32_t d = oe - os;
  if (want && d <= 16)
    for (int32_t p = os; p < oe; p++) flags[out_idx[p]] = 1;
  uint64_t mask = __ballot(want && d > 16 && d <= kBigRow);
  while (mask) {
    const int l = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    const int32_t s = __shfl(os, l, kWave), e = __shfl(oe, l, kWave);
    for (int32_t p = s + lane_id(); p < e; p += kWave) flags[out_idx[p]] = 1;
  }
  if (want && d > kBigRow) {
    const int64_t pos = (int64_t)atomicAdd((unsigned long long*)big_count, 1ull);
    big_list[pos] = v;
  }
}

// Initial marking (Algorithm 1): for every pending source u mark out(u) in
// G^t; the targets of effective deletions (the rest of out(u) in G^{t-1})
// were already set in `flags` when the batch was applied.
__global__ void __launch_bounds__(256) k_mark_pending(uint8_t* pend_src, int32_t n, const int32_t* __restrict__ out_off,
                                                      const int32_t* __restrict__ out_idx, uint8_t* flags,
                                                      int32_t* big_list, int64_t* big_count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < n; base += stride) {
    const int64_t u = base + lane_id();
    bool want = false;
    int32_t os = 0, oe = 0;
    if (u < n && pend_src[u]) {
      pend_src[u] = 0;
      want = true;
      os = out_off[u];
      oe = out_off[u + 1];
    }
    mark_out_rows(want, (int32_t)u, os, oe, out_idx, flags, big_list, big_count);
  }
}

// Commit (Jacobi reading): contrib[v] = R[v]/|out(v)| for the processed
// vertices, clear their current flag, and expand out(v) where flagged.
__global__ void __launch_bounds__(256) k_commit_expand(const int32_t* __restrict__ wl, int64_t cnt, const double* R,
                                                       double* contrib, const int32_t* __restrict__ out_off,
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
      oe = out_off[v + 1];
      contrib[v] = R[v] / (double)(oe - os);
      cur[v] = 0;
      if (xflag[v]) {
        xflag[v] = 0;
        want = true;
      }
    }
    mark_out_rows(want, v, os, oe, out_idx, next, big_list, big_count);
  }
}

// Chunk prefix of the big out-row list (one workgroup; the list is short).
__global__ void __launch_bounds__(1024) k_big_scan(const int32_t* big_list, const int64_t* big_count,
                                                   const int32_t* out_off, int64_t* big_pre) {
  __shared__ int64_t sh[1024 / kWave + 1];
  const int64_t nb = *big_count;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = min(lo + per, nb);
  int64_t local = 0;
  for (int64_t i = lo; i < hi; i++) {
    const int32_t v = big_list[i];
    local += ((int64_t)(out_off[v + 1] - out_off[v]) + kMarkChunk - 1) / kMarkChunk;
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(local, sh, &tot);
  for (int64_t i = lo; i < hi; i++) {
    big_pre[i] = run;
    const int32_t v = big_list[i];
    run += ((int64_t)(out_off[v + 1] - out_off[v]) + kMarkChunk - 1) / kMarkChunk;
  }
  if (threadIdx.x == 0) big_pre[nb] = tot;
}

__global__ void __launch_bounds__(256) k_big_mark(const int32_t* big_list, const int64_t* big_count,
                                                  const int64_t* big_pre, const int32_t* __restrict__ out_off,
                                                  const int32_t* __restrict__ out_idx, uint8_t* flags) {
  const int64_t nb = *big_count;
  const int64_t total = big_pre[nb];
  for (int64_t q = blockIdx.x; q < total; q += gridDim.x) {
    const int64_t j = upper_bound_i64(big_pre, 0, nb + 1, q) - 1;
    const int32_t v = big_list[j];
    const int32_t s = out_off[v] + (int32_t)((q - big_pre[j]) * kMarkChunk);
    const int32_t e = min(s + kMarkChunk, out_off[v + 1]);
    for (int32_t p = s + (int32_t)threadIdx.x; p < e; p += (int32_t)blockDim.x) flags[out_idx[p]] = 1;
  }
}

// ---- binning: affected vertices (flags == nullptr: all) -> worklist in
// ascending vertex order within each bin; bins laid out back to back.
constexpr int kBinItems = 8;
constexpr int kBinTile = 256 * kBinItems;
constexpr int kBinShift = 20;  // three 20-bit counters packed in one int64

__device__ __forceinline__ int bin_of(int32_t deg, int32_t t1, int32_t t2) { return deg <= t1 ? 0 : (deg <= t2 ? 1 : 2); }

__global__ void __launch_bounds__(256) k_bin_count(const uint8_t* flags, const int32_t* __restrict__ in_off, int32_t n,
                                                   int32_t t1, int32_t t2, int64_t* blk, int64_t nb,
                                                   int64_t* bin_edges) {
  __shared__ int64_t sh[256 / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinItems;
  int64_t packed = 0, e0 = 0, e1 = 0, e2 = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; j++) {
    const int64_t v = base + j;
    if (v < n && (flags == nullptr || flags[v])) {
      const int32_t deg = in_off[v + 1] - in_off[v];
      const int b = bin_of(deg, t1, t2);
      packed += (int64_t)1 << (kBinShift * b);
      if (b == 0) e0 += deg; else if (b == 1) e1 += deg; else e2 += deg;
    }
  }
  int64_t tot;
  block_exclusive_scan(packed, sh, &tot);
  if (threadIdx.x == 0) {
    const int64_t m = ((int64_t)1 << kBinShift) - 1;
    blk[0 * nb + blockIdx.x] = tot & m;
    blk[1 * nb + blockIdx.x] = (tot >> kBinShift) & m;
    blk[2 * nb + blockIdx.x] = (tot >> (2 * kBinShift)) & m;
  }
  e0 = wave_sum_i64(e0);
  e1 = wave_sum_i64(e1);
  e2 = wave_sum_i64(e2);
  if (lane_id() == 0) {
    if (e0) atomicAdd((unsigned long long*)&bin_edges[0], (unsigned long long)e0);
    if (e1) atomicAdd((unsigned long long*)&bin_edges[1], (unsigned long long)e1);
    if (e2) atomicAdd((unsigned long long*)&bin_edges[2], (unsigned long long)e2);
  }
}

__global__ void __launch_bounds__(256) k_bin_scatter(const uint8_t* flags, const int32_t* __restrict__ in_off,
                                                     int32_t n, int32_t t1, int32_t t2, const int64_t* offs,
                                                     int64_t nb, int32_t* wl, uint8_t* ever, int64_t* bin_end) {
  __shared__ int64_t sh[256 / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kBinTile + (int64_t)threadIdx.x * kBinItems;
  uint8_t bins[kBinItems];
  int64_t packed = 0;
#pragma unroll
  for (int j = 0; j < kBinItems; j++) {
    const int64_t v = base + j;
    bins[j] = 3;
    if (v < n && (flags == nullptr || flags[v])) {
      const int b = bin_of(in_off[v + 1] - in_off[v], t1, t2);
      bins[j] = (uint8_t)b;
      packed += (int64_t)1 << (kBinShift * b);
    }
  }
  int64_t tot;
  const int64_t pre = block_exclusive_scan(packed, sh, &tot);
  const int64_t m = ((int64_t)1 << kBinShift) - 1;
  int64_t pos[3] = {offs[0 * nb + blockIdx.x] + (pre & m), offs[1 * nb + blockIdx.x] + ((pre >> kBinShift) & m),
                    offs[2 * nb + blockIdx.x] + ((pre >> (2 * kBinShift)) & m)};
#pragma unroll
  for (int j = 0; j < kBinItems; j++) {
    if (bins[j] < 3) {
      const int32_t v = (int32_t)(base + j);
      wl[pos[bins[j]]++] = v;
      if (ever) ever[v] = 1;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bin_end[0] = offs[nb];
    bin_end[1] = offs[2 * nb];
    bin_end[2] = offs[3 * nb];
  }
}

// ---- small helpers
__global__ void k_init_static(double* R, double* contrib, const int32_t* __restrict__ out_off, int32_t n) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const double r = 1.0 / (double)n;
    R[v] = r;
    contrib[v] = r / (double)(out_off[v + 1] - out_off[v]);
  }
}
__global__ void k_init_prev(const double* r_prev, double* R, double* contrib, const int32_t* __restrict__ out_off,
                            int32_t n, int copy) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const double r = r_prev[v];
    if (copy) R[v] = r;
    contrib[v] = r / (double)(out_off[v + 1] - out_off[v]);
  }
}
// Reset the per-iteration counters; slot = the dR slot the next pull uses.
__global__ void k_iter_reset(IterCtl* c, int slot) {
  c->dR[slot] = 0ull;
  c->bin_edges[0] = c->bin_edges[1] = c->bin_edges[2] = 0;
  c->big_count = 0;
}
__global__ void k_reset_all(IterCtl* c) {
  c->dR[0] = c->dR[1] = 0ull;
  c->bin_edges[0] = c->bin_edges[1] = c->bin_edges[2] = 0;
  c->big_count = 0;
  c->ever_count = 0;
}
__global__ void __launch_bounds__(256) k_count_clear_ever(uint8_t* ever, int32_t n, int64_t* count) {
  int64_t c = 0;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (ever[v]) {
      c++;
      ever[v] = 0;
    }
  }
  c = wave_sum_i64(c);
  if (lane_id() == 0 && c) atomicAdd((unsigned long long*)count, (unsigned long long)c);
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

static int bin_vertices(dfpr_graph* g, const uint8_t* flags, int32_t* wl, uint8_t* ever, hipStream_t s) {
  const int32_t n = g->n;
  size_t tok;
  DFPR_TRY(g->pool.start(&tok));
  const int64_t nb = ((int64_t)n + kBinTile - 1) / kBinTile;
  k_bin_count<<<(unsigned)nb, 256, 0, s>>>(flags, g->in.off, n, g->t_thread, g->t_wave, g->bin_blk, nb,
                                           g->ctl->bin_edges);
  DFPR_TRY(scan_i64(g->bin_blk, g->bin_blk, 3 * nb, g->scan_tmp, s));
  k_bin_scatter<<<(unsigned)nb, 256, 0, s>>>(flags, g->in.off, n, g->t_thread, g->t_wave, g->bin_blk, nb, wl, ever,
                                             g->ctl->bin_end);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(g->pool.stop(kTBin, tok));
  return DFPR_OK;
}

static int readback(dfpr_graph* g, hipStream_t s) {
  DFPR_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(IterCtl), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  return DFPR_OK;
}

// Chunked marking of the rows collected in big_list.
static int mark_big(dfpr_graph* g, uint8_t* flags, hipStream_t s) {
  k_big_scan<<<1, 1024, 0, s>>>(g->big_list, &g->ctl->big_count, g->out.off, g->big_pre);
  k_big_mark<<<512, 256, 0, s>>>(g->big_list, &g->ctl->big_count, g->big_pre, g->out.off, g->out.idx, flags);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

// Launch the pull kernels of one iteration over worklist `wl` with bins
// [0,e0) [e0,e1) [e1,e2); per-bin timing when t->on.
template <int MODE>
static int pull_all(dfpr_graph* g, const PullArgs& a, const int32_t* wl, const int64_t* be, const int64_t* bedges,
                    hipStream_t s) {
  const int64_t n0 = be[0], n1 = be[1] - be[0], n2 = be[2] - be[1];
  EventPool& ep = g->pool;
  size_t tok;
  if (n0 > 0) {
    DFPR_TRY(ep.start(&tok));
    k_pull_lane<MODE><<<grid_for(n0, 256, 1u << 16), 256, 0, s>>>(a, wl, 0, be[0]);
    DFPR_HIP(hipGetLastError());
    DFPR_TRY(ep.stop(kTPull0, tok));
  }
  if (n1 > 0) {
    DFPR_TRY(ep.start(&tok));
    k_pull_wave<MODE><<<grid_for(n1, 4, 1u << 16), 256, 0, s>>>(a, wl, be[0], be[1]);
    DFPR_HIP(hipGetLastError());
    DFPR_TRY(ep.stop(kTPull1, tok));
  }
  if (n2 > 0) {
    DFPR_TRY(ep.start(&tok));
    DFPR_TRY(scan_generic(LoadChunks{wl, g->in.off, be[1]}, StoreI64r{g->chunk_pre}, n2, g->scan_tmp, s));
    const int64_t max_chunks = bedges[2] / kPullChunk + n2;
    k_pull_chunk<<<grid_for(max_chunks, 1, 1u << 16), 256, 0, s>>>(a, wl, be[1], n2, g->chunk_pre, g->partial);
    k_pull_chunk_finish<MODE><<<grid_for(n2, 256, 4096), 256, 0, s>>>(a, wl, be[1], n2, g->chunk_pre, g->partial);
    DFPR_HIP(hipGetLastError());
    DFPR_TRY(ep.stop(kTPull2, tok));
  }
  return DFPR_OK;
}

static void add_bins(dfpr_stats* st, const int64_t* be, const int64_t* bedges) {
  st->bin_vertices[0] += be[0];
  st->bin_vertices[1] += be[1] - be[0];
  st->bin_vertices[2] += be[2] - be[1];
  for (int k = 0; k < 3; k++) st->bin_edges[k] += bedges[k];
}

static int run_sync(dfpr_graph* g, bool cold, const dfpr_params& p, const double* r_prev, double* r_out,
                    hipStream_t s, dfpr_stats* st) {
  const int32_t n = g->n;
  if (!g->all_bins_valid) {
    k_reset_all<<<1, 1, 0, s>>>(g->ctl);
    DFPR_TRY(bin_vertices(g, nullptr, g->all_bins, nullptr, s));
    DFPR_TRY(readback(g, s));
    std::copy(g->ctl_host->bin_end, g->ctl_host->bin_end + 3, g->all_bin_end);
    std::copy(g->ctl_host->bin_edges, g->ctl_host->bin_edges + 3, g->all_bin_edges);
    g->all_bins_valid = true;
  }
  const unsigned gi = grid_for(n, 256, 1u << 16);
  if (cold)
    k_init_static<<<gi, 256, 0, s>>>(r_out, g->contrib, g->out.off, n);
  else
    k_init_prev<<<gi, 256, 0, s>>>(r_prev, r_out, g->contrib, g->out.off, n, r_prev != r_out);
  k_reset_all<<<1, 1, 0, s>>>(g->ctl);
  DFPR_HIP(hipGetLastError());
  double *Ra = r_out, *Rb = g->rn, *ca = g->contrib, *cb = g->contrib2;
  PullArgs a{g->in.off, g->in.idx, g->out.off, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
             p.alpha, (1.0 - p.alpha) / (double)n, p.frontier_tol, p.prune_tol};
  int it = 0;
  double dR = 0.0;
  bool conv = false;
  for (it = 0; it < p.max_iters; it++) {
    const int slot = it & 1;
    a.contrib = ca;
    a.R = Ra;
    a.Rw = Rb;
    a.cw = cb;
    a.dR = &g->ctl->dR[slot];
    DFPR_TRY(pull_all<kSync>(g, a, g->all_bins, g->all_bin_end, g->all_bin_edges, s));
    k_iter_reset<<<1, 1, 0, s>>>(g->ctl, slot ^ 1);
    DFPR_TRY(readback(g, s));
    dR = bits_to_double(g->ctl_host->dR[slot]);
    st->vertex_updates += n;
    st->edges_pulled += g->m;
    add_bins(st, g->all_bin_end, g->all_bin_edges);
    std::swap(Ra, Rb);
    std::swap(ca, cb);
    if (dR <= p.tol) {
      conv = true;
      it++;
      break;
    }
  }
  if (Ra != r_out) DFPR_HIP(hipMemcpyAsync(r_out, Ra, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
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

template <int MODE>
static int run_frontier(dfpr_graph* g, const dfpr_params& p, const double* r_prev, double* r_out, hipStream_t s,
                        dfpr_stats* st) {
  const int32_t n = g->n;
  const unsigned gi = grid_for(n, 256, 1u << 16);
  k_init_prev<<<gi, 256, 0, s>>>(r_prev, r_out, g->contrib, g->out.off, n, r_prev != r_out);
  k_reset_all<<<1, 1, 0, s>>>(g->ctl);
  // initial marking: out(u) of pending sources (+ deletion targets already in flag_cur)
  size_t tok;
  DFPR_TRY(g->pool.start(&tok));
  k_mark_pending<<<gi, 256, 0, s>>>(g->pend_src, n, g->out.off, g->out.idx, g->flag_cur, g->big_list,
                                    &g->ctl->big_count);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(mark_big(g, g->flag_cur, s));
  DFPR_TRY(g->pool.stop(kTMark, tok));
  g->pending_any = false;
  k_iter_reset<<<1, 1, 0, s>>>(g->ctl, 0);
  DFPR_TRY(bin_vertices(g, g->flag_cur, g->worklist, g->ever, s));
  DFPR_TRY(readback(g, s));
  uint8_t *cur = g->flag_cur, *next = g->flag_next;
  PullArgs a{g->in.off, g->in.idx, g->out.off, g->contrib, r_out, nullptr, nullptr, nullptr, g->xflag, nullptr,
             p.alpha, (1.0 - p.alpha) / (double)n, p.frontier_tol, p.prune_tol};
  int it = 0;
  double dR = 0.0;
  bool conv = false;
  for (it = 0; it < p.max_iters; it++) {
    const int slot = it & 1;
    int64_t be[3], bedges[3];
    std::copy(g->ctl_host->bin_end, g->ctl_host->bin_end + 3, be);
    std::copy(g->ctl_host->bin_edges, g->ctl_host->bin_edges + 3, bedges);
    const int64_t cnt = be[2];
    st->vertex_updates += cnt;
    st->edges_pulled += bedges[0] + bedges[1] + bedges[2];
    add_bins(st, be, bedges);
    if (cnt == 0) {  // nothing affected: the L-inf change of this iteration is 0
      dR = 0.0;
      conv = dR <= p.tol;
      it++;
      break;
    }
    a.next = next;
    a.dR = &g->ctl->dR[slot];
    DFPR_TRY(pull_all<MODE>(g, a, g->worklist, be, bedges, s));
    DFPR_TRY(g->pool.start(&tok));
    k_commit_expand<<<grid_for(cnt, 256, 1u << 16), 256, 0, s>>>(g->worklist, cnt, r_out, g->contrib, g->out.off,
                                                                 g->out.idx, cur, next, g->xflag, g->big_list,
                                                                 &g->ctl->big_count);
    DFPR_HIP(hipGetLastError());
    DFPR_TRY(mark_big(g, next, s));
    DFPR_TRY(g->pool.stop(kTCommit, tok));
    std::swap(cur, next);
    k_iter_reset<<<1, 1, 0, s>>>(g->ctl, slot ^ 1);
    DFPR_TRY(bin_vertices(g, cur, g->worklist, g->ever, s));
    DFPR_TRY(readback(g, s));
    dR = bits_to_double(g->ctl_host->dR[slot]);
    if (dR <= p.tol) {
      conv = true;
      it++;
      break;
    }
  }
  // leave both flag arrays clear for the next batch
  k_fill_u8<<<gi, 256, 0, s>>>(cur, n, 0);
  k_count_clear_ever<<<gi, 256, 0, s>>>(g->ever, n, &g->ctl->ever_count);
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(readback(g, s));
  // both arrays are zero again; which one is called "current" does not matter
  g->flag_cur = cur;
  g->flag_next = next;
  st->iterations = it;
  st->converged = conv ? 1 : 0;
  st->last_delta = dR;
  st->ever_affected = g->ctl_host->ever_count;
  return DFPR_OK;
}

int update_ranks(dfpr_graph* g, dfpr_mode mode, const dfpr_params& p, const double* r_prev, double* r_out,
                 hipStream_t s, dfpr_stats* st_out) {
  dfpr_stats st{};
  EventPool& ep = g->pool;
  ep.reset(g->timing || (p.flags & DFPR_FLAG_TIMING) != 0, s);
  size_t tok;
  DFPR_TRY(ep.start(&tok));
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
    for (int k = 0; k < 3; k++) {
      st.ms_pull[k] = ms[kTPull0 + k];
      st.pull_launches[k] = cnt[kTPull0 + k];
    }
    st.ms_commit = ms[kTCommit];
    st.ms_bin = ms[kTBin];
    st.ms_mark = ms[kTMark];
  }
  if (st_out) *st_out = st;
  return DFPR_OK;
}

}  // namespace dfpr
