// Two-phase pull for the dense form of DF / DF-P (an optional replacement of
// the gather pull; dfpr_set_two_phase).
//
// The in-neighbour sums of Equations 1 and 2 are formed without gathering
// contributions from random addresses.  Phase one walks the edges grouped by
// source block (8192 sources, whose contributions sit in LDS) and writes each
// edge's contribution into a value array ordered by destination bucket (4096
// destinations); phase two streams every bucket once and adds its values
// into LDS accumulators.  Global memory is touched in streams and in the
// contiguous runs of each (source block, bucket) pair; the random accesses
// are in LDS.
//
// Sums are formed exactly: each contribution is taken on a grid of 2^-96
// (exactly, for contributions of at least 2^-44) as a 128-bit integer and the
// integers are added, so the sum does not depend on the order of the
// additions; the total is rounded to FP64 once.  A bucket split over several
// workgroups is combined with 64-bit atomics whose returned old value
// carries into the high word.  Contributions must lie in [0, 2^31) and each
// vertex's sum below 2^32 (ranks of a probability vector always do); a
// contribution outside the range is reported.
//
// Layout (rebuilt from the in-CSR whenever the graph changed):
//   pair (S, b): the edges from source block S into destination bucket b;
//   p1   [m] source-major order (S, b, any): b << 13 | source slot in S
//   dstl [m] bucket-major order (b, S, any): destination slot in b
//   the k-th edge of pair (S, b) sits at tabS[S][b] + k in p1 and at
//   tabB[b][S] + k in dstl (and val): delta[S][b] = tabB[b][S] - tabS[S][b].
#include "prim.hpp"

namespace dfpr {

// ---- layout build: one workgroup per item (a slot range of one bucket's
// rows in the in-CSR); row of a slot by binary search over the bucket's
// offsets in LDS
constexpr int kTpBuildThreads = 512;

__device__ __forceinline__ int tp_row_of(const int32_t* roff, int nrows, int32_t e) {
  int lo = 0, hi = nrows;  // roff[lo] <= e < roff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (roff[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

struct TpBuildShared {
  int32_t roff[kTpDst + 1];
  int32_t rdeg[kTpDst];
  int32_t hist[kTpMaxS];
};

// Lanes whose keys equal the first remaining lane's key are combined when at
// least kTpRun of them do (a long row's run: its sources share a block, its
// entries one destination), so a hub's run costs one LDS atomic instead of
// 64 serialised ones.  Loops that call these keep every lane active (uniform
// trip counts, a `valid` predicate instead of an exit).
constexpr int kTpRun = 16;

// hist[key] += 1 for every valid lane; returns each lane's value before its
// increment (a slot number; runs take consecutive slots).
__device__ __forceinline__ int32_t tp_hist_take(int32_t* hist, int key, bool valid) {
  const int lane = lane_id();
  int32_t slot = 0;
  uint64_t act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int kl = __shfl(key, leader, kWave);
    const uint64_t mk = __ballot(valid && key == kl);
    if (__popcll(mk) < kTpRun) break;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&hist[kl], (int32_t)__popcll(mk));
    base = __shfl(base, leader, kWave);
    if ((mk >> lane) & 1) {
      slot = base + (int32_t)__popcll(mk & ((1ull << lane) - 1));
      valid = false;
    }
    act &= ~mk;
  }
  if (valid) slot = atomicAdd(&hist[key], 1);
  return slot;
}

__device__ __forceinline__ void tp_load_rows(TpBuildShared& sh, const int32_t* off, const int32_t* deg, int32_t n,
                                             int b, int nS, int* nrows_out) {
  const int32_t r0 = b * kTpDst;
  const int nrows = min(kTpDst, n - r0);
  for (int t = threadIdx.x; t <= nrows; t += blockDim.x) sh.roff[t] = off[r0 + t];
  for (int t = threadIdx.x; t < nrows; t += blockDim.x) sh.rdeg[t] = deg[r0 + t];
  for (int t = threadIdx.x; t < nS; t += blockDim.x) sh.hist[t] = 0;
  *nrows_out = nrows;
  __syncthreads();
}

// The slot's row and source block, or valid = false for a free slot / past the end.
__device__ __forceinline__ bool tp_slot(const TpBuildShared& sh, const int32_t* idx, int nrows, int32_t e, int32_t hi,
                                        int* r_out, int32_t* u_out) {
  if (e >= hi) return false;
  const int r = tp_row_of(sh.roff, nrows, e);
  if (e >= sh.roff[r] + sh.rdeg[r]) return false;
  *r_out = r;
  *u_out = idx[e];
  return true;
}

__device__ __forceinline__ void tp_count_item(TpBuildShared& sh, const int32_t* idx, int nrows, int32_t lo, int32_t hi) {
  for (int32_t base = lo; base < hi; base += kTpBuildThreads) {
    int r = 0;
    int32_t u = 0;
    const bool valid = tp_slot(sh, idx, nrows, base + (int32_t)threadIdx.x, hi, &r, &u);
    (void)tp_hist_take(sh.hist, u >> kTpSrcBits, valid);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kTpBuildThreads) k_tp_count(const int32_t* __restrict__ off,
                                                              const int32_t* __restrict__ deg,
                                                              const int32_t* __restrict__ idx, int32_t n, int nS,
                                                              const int32_t* __restrict__ items, int32_t* cnt) {
  __shared__ TpBuildShared sh;
  const int b = items[3 * blockIdx.x];
  int nrows;
  tp_load_rows(sh, off, deg, n, b, nS, &nrows);
  tp_count_item(sh, idx, nrows, items[3 * blockIdx.x + 1], items[3 * blockIdx.x + 2]);
  for (int t = threadIdx.x; t < nS; t += blockDim.x)
    if (sh.hist[t]) atomicAdd(&cnt[(int64_t)b * nS + t], sh.hist[t]);
}

// Each item reserves its share of every pair it feeds (one atomic per pair),
// then places its edges inside the share; which slot an edge gets does not
// matter to the sums.  hist[S] then runs over the share's positions in the
// bucket-major order; the source-major position is that minus delta[S][b].
__global__ void __launch_bounds__(kTpBuildThreads) k_tp_fill(const int32_t* __restrict__ off,
                                                             const int32_t* __restrict__ deg,
                                                             const int32_t* __restrict__ idx, int32_t n, int nS,
                                                             int nB, const int32_t* __restrict__ items,
                                                             int32_t* cursor, const int64_t* __restrict__ tabB,
                                                             const int32_t* __restrict__ delta,
                                                             uint32_t* __restrict__ p1, uint16_t* __restrict__ dstl) {
  __shared__ TpBuildShared sh;
  __shared__ int32_t dl[kTpMaxS];
  const int b = items[3 * blockIdx.x];
  const int32_t lo = items[3 * blockIdx.x + 1], hi = items[3 * blockIdx.x + 2];
  int nrows;
  tp_load_rows(sh, off, deg, n, b, nS, &nrows);
  tp_count_item(sh, idx, nrows, lo, hi);
  for (int t = threadIdx.x; t < nS; t += blockDim.x) {
    const int32_t c = sh.hist[t];
    if (c) {
      sh.hist[t] = (int32_t)tabB[(int64_t)b * nS + t] + atomicAdd(&cursor[(int64_t)b * nS + t], c);
      dl[t] = delta[(int64_t)t * nB + b];
    }
  }
  __syncthreads();
  for (int32_t base = lo; base < hi; base += kTpBuildThreads) {
    int r = 0;
    int32_t u = 0;
    const bool valid = tp_slot(sh, idx, nrows, base + (int32_t)threadIdx.x, hi, &r, &u);
    const int S = u >> kTpSrcBits;
    const int32_t q2 = tp_hist_take(sh.hist, S, valid);
    if (valid) {
      p1[q2 - dl[S]] = ((uint32_t)b << kTpSrcBits) | (uint32_t)(u & (kTpSrc - 1));
      dstl[q2] = (uint16_t)r;
    }
  }
}

struct TpLoadCnt {  // pair counts in [b][S] order
  const int32_t* c;
  __device__ int64_t operator()(int64_t i) const { return c[i]; }
};
struct TpLoadCntT {  // the same counts read in [S][b] order
  const int32_t* c;
  int64_t nB, nS;
  __device__ int64_t operator()(int64_t i) const { return c[(i % nB) * nS + i / nB]; }
};
struct TpStore {
  int64_t* o;
  __device__ void operator()(int64_t i, int64_t v) const { o[i] = v; }
};

__global__ void k_tp_delta(const int64_t* __restrict__ tabB, const int64_t* __restrict__ tabS, int64_t nS, int64_t nB,
                           int32_t* __restrict__ delta) {
  const int64_t np = nS * nB;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t S = i / nB, b = i % nB;
    delta[i] = (int32_t)(tabB[b * nS + S] - tabS[i]);
  }
}

// starts[0..nS]: first p1 entry of each source block (starts[nS] = m);
// starts[nS+1 .. nS+1+nB]: first value of each bucket (the last = m)
__global__ void k_tp_starts(const int64_t* __restrict__ tabB, const int64_t* __restrict__ tabS, int nS, int nB,
                            int64_t* __restrict__ starts) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= nS + nB + 1; i += gridDim.x * blockDim.x)
    starts[i] = i <= nS ? tabS[(int64_t)i * nB] : tabB[(int64_t)(i - nS - 1) * nS];
}

// out[b] = first in-CSR slot of bucket b's rows, b = 0..nB (out[nB] = off[n])
__global__ void k_tp_row_starts(const int32_t* __restrict__ off, int32_t n, int nB, int64_t* __restrict__ out) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nB; b += gridDim.x * blockDim.x)
    out[b] = off[min((int64_t)b * kTpDst, (int64_t)n)];
}

// ---- phase one: contributions into bucket order
// MAXB: bucket count the LDS table holds (4096 keeps two workgroups per CU)
template <int MAXB>
__global__ void __launch_bounds__(512) k_tp_scatter(const double* __restrict__ contrib,
                                                    const uint8_t* __restrict__ xflag, int32_t n,
                                                    const int32_t* __restrict__ items,
                                                    const uint32_t* __restrict__ p1,
                                                    const int32_t* __restrict__ delta, int nB,
                                                    uint64_t* __restrict__ val, int32_t* bad) {
  __shared__ uint64_t lc[kTpSrc];  // the block's contributions (bit 63: expands)
  __shared__ int32_t ld[MAXB];     // delta of each of the block's pairs
  const int S = items[3 * blockIdx.x];
  const int32_t lo = items[3 * blockIdx.x + 1], hi = items[3 * blockIdx.x + 2];
  const int32_t v0 = S * kTpSrc;
  int badc = 0;
  for (int t = threadIdx.x; t < kTpSrc; t += blockDim.x) {
    const int32_t v = v0 + t;
    uint64_t bits = 0;
    if (v < n) {
      const double c = contrib[v];
      badc |= !(c >= 0.0 && c < 0x1p31);
      bits = (uint64_t)__double_as_longlong(c) & ~(1ull << 63);
      if (xflag && xflag[v]) bits |= 1ull << 63;
    }
    lc[t] = bits;
  }
  if (badc) atomicOr(bad, 1);
  const int32_t* dS = delta + (int64_t)S * nB;
  for (int t = threadIdx.x; t < nB; t += blockDim.x) ld[t] = dS[t];
  __syncthreads();
  int32_t e = lo + (int32_t)threadIdx.x;
  for (; e + 3 * 512 < hi; e += 4 * 512) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; j++) w[j] = __builtin_nontemporal_load(p1 + e + j * 512);
#pragma unroll
    for (int j = 0; j < 4; j++) val[e + j * 512 + ld[w[j] >> kTpSrcBits]] = lc[w[j] & (kTpSrc - 1)];
  }
  for (; e < hi; e += 512) {
    const uint32_t w = __builtin_nontemporal_load(p1 + e);
    val[e + ld[w >> kTpSrcBits]] = lc[w & (kTpSrc - 1)];
  }
}

// ---- phase two: bucket streams into 128-bit LDS accumulators
__device__ __forceinline__ void wave_sum128(uint64_t& lo, uint64_t& hi) {
#pragma unroll
  for (int o = kWave / 2; o >= 1; o >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, o, kWave), h2 = __shfl_xor(hi, o, kWave);
    const uint64_t sl = lo + l2;
    hi = hi + h2 + (uint64_t)(sl < lo);
    lo = sl;
  }
}

__device__ __forceinline__ void lds_add128(unsigned long long* lo, unsigned long long* hi, int d, uint64_t xl,
                                           uint64_t xh) {
  const unsigned long long old = atomicAdd(&lo[d], (unsigned long long)xl);
  atomicAdd(&hi[d], (unsigned long long)(xh + (uint64_t)(old + xl < old)));
}

// One value per lane (valid lanes only); runs of one destination (a hub's
// in-row) are summed across the wave first.
__device__ __forceinline__ void tp_accum_lane(unsigned long long* lo, unsigned long long* hi, uint32_t* fl, int d,
                                              uint64_t bits, bool valid) {
  const int lane = lane_id();
  const Fix128 x = fix128(bits & ~(1ull << 63));
  const bool xf = (bits >> 63) != 0;
  uint64_t act = __ballot(valid);
  while (act) {
    const int leader = __ffsll((long long)act) - 1;
    const int dlead = __shfl(d, leader, kWave);
    const uint64_t mk = __ballot(valid && d == dlead);
    if (__popcll(mk) < kTpRun) break;
    const bool in = (mk >> lane) & 1;
    uint64_t l = in ? x.lo : 0, h = in ? x.hi : 0;
    wave_sum128(l, h);
    const bool anyx = (__ballot(in && xf) != 0);
    if (lane == leader) {
      lds_add128(lo, hi, dlead, l, h);
      if (anyx) atomicOr(&fl[dlead >> 5], 1u << (dlead & 31));
    }
    if (in) valid = false;
    act &= ~mk;
  }
  if (valid) {
    lds_add128(lo, hi, d, x.lo, x.hi);
    if (xf) atomicOr(&fl[d >> 5], 1u << (d & 31));
  }
}

__global__ void __launch_bounds__(512) k_tp_accum(const int32_t* __restrict__ items, const uint16_t* __restrict__ dstl,
                                                  const uint64_t* __restrict__ val, uint64_t* glo, uint64_t* ghi,
                                                  uint32_t* gfl) {
  __shared__ unsigned long long lo[kTpDst], hi[kTpDst];
  __shared__ uint32_t fl[kTpDst / 32];
  const int b = items[4 * blockIdx.x];
  const int32_t e0 = items[4 * blockIdx.x + 1], e1 = items[4 * blockIdx.x + 2];
  const bool split = items[4 * blockIdx.x + 3] != 0;
  for (int t = threadIdx.x; t < kTpDst; t += blockDim.x) lo[t] = hi[t] = 0ull;
  for (int t = threadIdx.x; t < kTpDst / 32; t += blockDim.x) fl[t] = 0u;
  __syncthreads();
  // every lane runs the same number of rounds (the wave-wide combining above
  // needs all lanes); four loads in flight per lane
  for (int32_t base = e0; base < e1; base += 4 * 512) {
    uint16_t d[4];
    uint64_t v[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int32_t e = base + j * 512 + (int32_t)threadIdx.x;
      d[j] = e < e1 ? __builtin_nontemporal_load(dstl + e) : (uint16_t)0;
      v[j] = e < e1 ? __builtin_nontemporal_load(val + e) : 0ull;
    }
#pragma unroll
    for (int j = 0; j < 4; j++) tp_accum_lane(lo, hi, fl, d[j], v[j], base + j * 512 + (int32_t)threadIdx.x < e1);
  }
  __syncthreads();
  const int64_t gb = (int64_t)b * kTpDst;
  for (int t = threadIdx.x; t < kTpDst; t += blockDim.x) {
    const unsigned long long l = lo[t], h = hi[t];
    if (!split) {
      glo[gb + t] = l;
      ghi[gb + t] = h;
    } else if (l | h) {
      const unsigned long long old = atomicAdd((unsigned long long*)&glo[gb + t], l);
      atomicAdd((unsigned long long*)&ghi[gb + t], h + (unsigned long long)(old + l < old));
    }
  }
  for (int t = threadIdx.x; t < kTpDst / 32; t += blockDim.x) {
    if (!split) gfl[gb / 32 + t] = fl[t];
    else if (fl[t]) atomicOr(&gfl[gb / 32 + t], fl[t]);
  }
}

// ---- host side
bool tp_supported(const dfpr_graph* g, const char** why) {
  if (g->ngraphs > 1) {
    *why = "the two-phase pull serves plain graphs, not batch handles";
    return false;
  }
  if ((int64_t)g->n > (int64_t)kTpMaxB * kTpDst) {
    *why = "the two-phase pull handles at most 2^25 vertices";
    return false;
  }
  return true;
}

static int up(const void* host, void* dev, size_t bytes, hipStream_t s) {
  DFPR_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s));
  DFPR_HIP(hipStreamSynchronize(s));  // the host vector dies with the caller
  return DFPR_OK;
}

int tp_build(dfpr_graph* g, hipStream_t s) {
  TwoPhase& t = *g->tp;
  const int32_t n = g->n;
  const int64_t m = g->m;
  const int nS = (n + kTpSrc - 1) / kTpSrc, nB = (n + kTpDst - 1) / kTpDst;
  const int64_t np = (int64_t)nS * nB;
  t.nS = nS;
  t.nB = nB;
  DFPR_TRY(t.p1.ensure((size_t)std::max<int64_t>(m, 1) * 4));
  DFPR_TRY(t.dstl.ensure((size_t)std::max<int64_t>(m, 1) * 2));
  DFPR_TRY(t.val.ensure((size_t)std::max<int64_t>(m, 1) * 8));
  DFPR_TRY(t.cnt.ensure((size_t)np * 4));
  DFPR_TRY(t.tabB.ensure((size_t)(np + 1) * 8));
  DFPR_TRY(t.tabS.ensure((size_t)(np + 1) * 8));
  DFPR_TRY(t.delta.ensure((size_t)np * 4));
  DFPR_TRY(t.tmp.ensure(scan_tmp_elems(np + 1) * 8));
  DFPR_TRY(t.glo.ensure((size_t)nB * kTpDst * 8));
  DFPR_TRY(t.ghi.ensure((size_t)nB * kTpDst * 8));
  DFPR_TRY(t.gfl.ensure((size_t)nB * kTpDst / 8));
  DFPR_TRY(t.split.ensure((size_t)nB));
  DFPR_TRY(t.starts.ensure((size_t)(nS + 2 * nB + 3) * 8));  // either table below
  DFPR_TRY(t.bad.ensure(4));
  // build items: the in-CSR slot range of each bucket's rows, in pieces
  std::vector<int64_t> st(std::max(nS + nB + 2, nB + 1));
  k_tp_row_starts<<<grid_for(nB + 1, 256, 1024), 256, 0, s>>>(g->in.off, n, nB, t.starts.as<int64_t>());
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipMemcpyAsync(st.data(), t.starts.as<int64_t>(), (size_t)(nB + 1) * 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> bi;
  for (int b = 0; b < nB; b++) {
    const int64_t lo = st[b], hi = st[b + 1];
    for (int64_t x = lo; x < hi; x += kTpItemBuild) {
      bi.push_back(b);
      bi.push_back((int32_t)x);
      bi.push_back((int32_t)std::min<int64_t>(hi, x + kTpItemBuild));
    }
  }
  const int nbi = (int)(bi.size() / 3);
  DFPR_TRY(t.bitems.ensure(std::max<size_t>(bi.size(), 1) * 4));
  if (nbi) DFPR_TRY(up(bi.data(), t.bitems.p, bi.size() * 4, s));
  DFPR_HIP(hipMemsetAsync(t.cnt.p, 0, (size_t)np * 4, s));
  if (nbi)
    k_tp_count<<<nbi, kTpBuildThreads, 0, s>>>(g->in.off, g->in_deg, g->in.idx, n, nS, t.bitems.as<int32_t>(),
                                               t.cnt.as<int32_t>());
  DFPR_HIP(hipGetLastError());
  DFPR_TRY(scan_generic(TpLoadCnt{t.cnt.as<int32_t>()}, TpStore{t.tabB.as<int64_t>()}, np, t.tmp.as<int64_t>(), s));
  DFPR_TRY(scan_generic(TpLoadCntT{t.cnt.as<int32_t>(), nB, nS}, TpStore{t.tabS.as<int64_t>()}, np,
                        t.tmp.as<int64_t>(), s));
  k_tp_delta<<<grid_for(np, 256, 65536), 256, 0, s>>>(t.tabB.as<int64_t>(), t.tabS.as<int64_t>(), nS, nB,
                                                      t.delta.as<int32_t>());
  DFPR_HIP(hipMemsetAsync(t.cnt.p, 0, (size_t)np * 4, s));
  if (nbi)
    k_tp_fill<<<nbi, kTpBuildThreads, 0, s>>>(g->in.off, g->in_deg, g->in.idx, n, nS, nB, t.bitems.as<int32_t>(),
                                              t.cnt.as<int32_t>(), t.tabB.as<int64_t>(), t.delta.as<int32_t>(),
                                              t.p1.as<uint32_t>(), t.dstl.as<uint16_t>());
  k_tp_starts<<<grid_for(nS + nB + 2, 256, 1024), 256, 0, s>>>(t.tabB.as<int64_t>(), t.tabS.as<int64_t>(), nS, nB,
                                                               t.starts.as<int64_t>());
  DFPR_HIP(hipGetLastError());
  st.assign(nS + nB + 2, 0);
  DFPR_HIP(hipMemcpyAsync(st.data(), t.starts.as<int64_t>(), st.size() * 8, hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  if (st[nS] != m || st[nS + 1 + nB] != m) {
    set_error("internal inconsistency in the two-phase layout (%lld, %lld edges, expected %lld)",
              (long long)st[nS], (long long)st[nS + 1 + nB], (long long)m);
    return DFPR_EHIP;
  }
  // phase items: pieces of each source block (phase one) and of each bucket
  // (phase two; every bucket has one, so an empty bucket writes its zeros)
  std::vector<int32_t> i1, i2;
  std::vector<uint8_t> sp(nB, 0);
  for (int S = 0; S < nS; S++)
    for (int64_t x = st[S]; x < st[S + 1]; x += kTpItem1) {
      i1.push_back(S);
      i1.push_back((int32_t)x);
      i1.push_back((int32_t)std::min<int64_t>(st[S + 1], x + kTpItem1));
    }
  for (int b = 0; b < nB; b++) {
    const int64_t lo = st[nS + 1 + b], hi = st[nS + 2 + b];
    sp[b] = hi - lo > kTpItem2;
    int64_t x = lo;
    do {
      i2.push_back(b);
      i2.push_back((int32_t)x);
      i2.push_back((int32_t)std::min<int64_t>(hi, x + kTpItem2));
      i2.push_back(sp[b]);
      x += kTpItem2;
    } while (x < hi);
  }
  t.n1 = (int)(i1.size() / 3);
  t.n2 = (int)(i2.size() / 4);
  DFPR_TRY(t.items1.ensure(std::max<size_t>(i1.size(), 1) * 4));
  DFPR_TRY(t.items2.ensure(i2.size() * 4));
  if (t.n1) DFPR_TRY(up(i1.data(), t.items1.p, i1.size() * 4, s));
  DFPR_TRY(up(i2.data(), t.items2.p, i2.size() * 4, s));
  DFPR_TRY(up(sp.data(), t.split.p, sp.size(), s));
  // split buckets add into the accumulators: start them at zero (the finish
  // kernel clears them again after reading)
  DFPR_HIP(hipMemsetAsync(t.glo.p, 0, (size_t)nB * kTpDst * 8, s));
  DFPR_HIP(hipMemsetAsync(t.ghi.p, 0, (size_t)nB * kTpDst * 8, s));
  DFPR_HIP(hipMemsetAsync(t.gfl.p, 0, (size_t)nB * kTpDst / 8, s));
  DFPR_HIP(hipMemsetAsync(t.bad.p, 0, 4, s));
  t.m = m;
  t.built = g->csr_version;
  return DFPR_OK;
}

int tp_phases(dfpr_graph* g, const double* contrib, const uint8_t* xflag, hipStream_t s) {
  TwoPhase& t = *g->tp;
  if (t.n1 && t.nB <= kTpMaxB / 2)
    k_tp_scatter<kTpMaxB / 2><<<t.n1, 512, 0, s>>>(contrib, xflag, g->n, t.items1.as<int32_t>(), t.p1.as<uint32_t>(),
                                                  t.delta.as<int32_t>(), t.nB, t.val.as<uint64_t>(),
                                                  t.bad.as<int32_t>());
  else if (t.n1)
    k_tp_scatter<kTpMaxB><<<t.n1, 512, 0, s>>>(contrib, xflag, g->n, t.items1.as<int32_t>(), t.p1.as<uint32_t>(),
                                              t.delta.as<int32_t>(), t.nB, t.val.as<uint64_t>(), t.bad.as<int32_t>());
  k_tp_accum<<<t.n2, 512, 0, s>>>(t.items2.as<int32_t>(), t.dstl.as<uint16_t>(), t.val.as<uint64_t>(),
                                  t.glo.as<uint64_t>(), t.ghi.as<uint64_t>(), t.gfl.as<uint32_t>());
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

TwoPhase::~TwoPhase() {
  for (DevBuf* b : {&p1, &dstl, &val, &cnt, &tabB, &tabS, &delta, &tmp, &glo, &ghi, &gfl, &split, &starts, &bad,
                    &bitems, &items1, &items2})
    b->release();
}

}  // namespace dfpr
