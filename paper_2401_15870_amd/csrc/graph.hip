// Device graph store: canonical in- and out-CSR, creation, export and batch
// application (Section 3.2 batch semantics; self-loop on every vertex as in
// Sections 3.1 and 5.1.3).
//
// Batch keys pack an edge as (row << (b+1)) | (col << 1) | tag with b bits
// per id and tag 1 = insertion, 0 = deletion, so one radix sort orders a batch
// by row, then column, with deletions of a pair before its insertion.
#include <algorithm>
#include <cstdarg>
#include <cstdio>

#include <type_traits>

#include "prim.hpp"

namespace dfpr {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char* last_error() { return g_err; }
void clear_error() { g_err[0] = 0; }

int DevBuf::ensure(size_t want) {
  if (want <= bytes) return DFPR_OK;
  release();
  if (heap) {
    const size_t nb = (want + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign;
    p = heap->alloc(nb);
    if (!p) {
      set_error("scratch heap exhausted: %zu bytes wanted", nb);
      return DFPR_ENOMEM;
    }
    bytes = nb;
    return DFPR_OK;
  }
  size_t nb = want + want / 4 + 4096;
  hipError_t e = hipMalloc(&p, nb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    bytes = 0;
    set_error("device allocation of %zu bytes failed: %s", nb, hipGetErrorString(e));
    return DFPR_ENOMEM;
  }
  bytes = nb;
  return DFPR_OK;
}
void DevBuf::release() {
  if (p && heap) heap->free(p);
  else if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

template <class T>
static int dalloc(T** p, size_t count) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("device allocation of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    return DFPR_ENOMEM;
  }
  return DFPR_OK;
}
template <class T>
static void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// ------------------------------------------------------------------ kernels
constexpr uint64_t kBadKey = ~0ull;

// ---- internal numbering by decreasing in-degree (ties by caller id)
// Validates the ids and counts the in-degree of every target.  A hub can be
// the target of a large share of all pairs, so the wavefront first sorts its
// 64 targets (bitonic network over the lanes) and each run of equal targets
// adds its length with one atomic: a hub costs one atomic per wavefront
// instead of one per pair.
__global__ void __launch_bounds__(256) k_validate_count(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                                                        int32_t* deg, int64_t* err) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < m; base += stride) {
    const int64_t i = base + lane;
    int32_t v = INT32_MAX;  // lanes past the end and invalid pairs sort last and count nothing
    if (i < m) {
      const int32_t u = src[i], w = dst[i];
      if (u < 0 || u >= n || w < 0 || w >= n)
        atomicOr((unsigned long long*)err, 1ull);
      else
        v = w;
    }
    if (!deg) continue;
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int32_t y = __shfl_xor(v, j, kWave);
        const bool up = (lane & k) == 0;
        const bool lower = (lane & j) == 0;
        v = (lower == up) ? min(v, y) : max(v, y);
      }
    }
    const int32_t prev = __shfl_up(v, 1, kWave);
    const bool head = lane == 0 || prev != v;
    const unsigned long long heads = __ballot(head);
    if (head && v != INT32_MAX) {
      const unsigned long long above = lane == kWave - 1 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
      const int next = above ? __ffsll((long long)above) - 1 : kWave;
      atomicAdd(&deg[v], next - lane);
    }
  }
}
// Sort key of the internal numbering: member, then decreasing in-degree
// (capped at 2^24-1), then caller id; members keep their contiguous vertex
// ranges.
__global__ void k_degree_keys(const int32_t* deg, const int32_t* gidv, int32_t n, int b, uint64_t* keys) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t d = (uint64_t)min(deg[v], 0xFFFFFF);
    const uint64_t gk = gidv ? (uint64_t)gidv[v] : 0ull;
    keys[v] = (gk << (24 + b)) | ((0xFFFFFFull - d) << b) | (uint64_t)v;
  }
}
// Member of every vertex from the member vertex bases (binary search).
__global__ void k_member_ids(const int64_t* vbase, int32_t count, int32_t n, int32_t* gidv) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = count;  // largest k with vbase[k] <= v
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if (vbase[mid] <= v) lo = mid; else hi = mid;
    }
    gidv[v] = lo;
  }
}
// Per-member effective insertion / deletion counts of a batch (keys sorted by
// row, so a wavefront is nearly always inside one member).
__global__ void k_member_eff(const uint64_t* eff, const int64_t* count, int b, const int32_t* gidv, int64_t* g_eff) {
  const int64_t T = *count;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~(kWave - 1)); base < T; base += stride) {
    const int64_t i = base + lane_id();
    const bool ok = i < T;
    const uint64_t k = ok ? eff[i] : 0ull;
    const int32_t gk = ok ? gidv[(int32_t)(k >> (b + 1))] : -1;
    const int is_ins = ok ? (int)(k & 1ull) : 0;
    const int32_t g0 = __shfl(gk, 0, kWave);
    const bool same = __ballot(ok && gk != g0) == 0ull;
    if (same) {
      const int64_t ni = wave_sum_i64(is_ins), nd = wave_sum_i64(ok ? 1 - is_ins : 0);
      if (lane_id() == 0 && g0 >= 0) {
        if (ni) atomicAdd((unsigned long long*)&g_eff[2 * g0], (unsigned long long)ni);
        if (nd) atomicAdd((unsigned long long*)&g_eff[2 * g0 + 1], (unsigned long long)nd);
      }
    } else if (ok) {
      atomicAdd((unsigned long long*)&g_eff[2 * gk + (is_ins ? 0 : 1)], 1ull);
    }
  }
}
// Edge count of every member after a batch: the sum of its vertices' out-degrees
// (a workgroup per member).
__global__ void __launch_bounds__(256) k_member_m(const int32_t* out_deg, const int64_t* vbase, int32_t G,
                                                  int64_t* m_out) {
  __shared__ int64_t sh[256 / kWave];
  for (int64_t k = blockIdx.x; k < G; k += gridDim.x) {
    int64_t t = 0;
    for (int64_t v = vbase[k] + threadIdx.x; v < vbase[k + 1]; v += blockDim.x) t += out_deg[v];
    t = wave_sum_i64(t);
    if (lane_id() == 0) sh[threadIdx.x / kWave] = t;
    __syncthreads();
    if (threadIdx.x == 0) m_out[k] = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
  }
}
// Degrees of a CSR without slack: deg[v] = off[v+1] - off[v].
__global__ void k_deg_from_off(const int32_t* off, int32_t n, int32_t* deg) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    deg[v] = off[v + 1] - off[v];
}
// Degrees after an accepted batch: every effective insertion (u, v) adds one to
// |out(u)| and |in(v)|, every effective deletion takes one off.  One atomic per
// row: the first entry of each row's run in the (u, v) order (out-degrees)
// and in the (v, u) order (in-degrees) adds the run's insertions minus its
// deletions (pre_*: prefix counts of the deletions), so a hub that many
// entries touch is not one hot address.  Nothing changes when the batch was
// rejected (err set).
__global__ void k_update_degrees(const uint64_t* eff_out, const uint64_t* eff_in, const int64_t* count,
                                 const int64_t* pre_out, const int64_t* pre_in, int b, const int64_t* err,
                                 int32_t* out_deg, int32_t* in_deg) {
  if (*err) return;
  const int64_t t = *count;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * t; i += (int64_t)gridDim.x * blockDim.x) {
    const bool in_side = i >= t;
    const int64_t e = in_side ? i - t : i;
    const uint64_t* eff = in_side ? eff_in : eff_out;
    const int64_t* pre = in_side ? pre_in : pre_out;
    const int64_t r = (int64_t)(eff[e] >> (b + 1));
    if (e > 0 && (int64_t)(eff[e - 1] >> (b + 1)) == r) continue;
    const int64_t end = lower_bound_u64(eff, e + 1, t, (uint64_t)(r + 1) << (b + 1));
    const int32_t net = (int32_t)((end - e) - 2 * (pre[end] - pre[e]));
    if (net) atomicAdd(&(in_side ? in_deg : out_deg)[r], net);
  }
}
// ---- rows with free slots
// Row v of a CSR with slack keeps its deg[v] neighbours, ascending, at
// off[v] .. off[v] + deg[v] and the pad id n (above every real id) in its
// remaining slots up to off[v + 1].  Pads sort after every real id, so a row
// searched or copied as a whole stays ordered and the full rebuild carries
// them along as ordinary entries.

// Row lengths of a layout with `slack` free slots per row.
struct LoadPadded {
  const int32_t* deg;
  int32_t slack;
  __device__ int64_t operator()(int64_t v) const { return (int64_t)deg[v] + slack; }
};
struct StoreOff {
  int32_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = (int32_t)v; }
};

// Largest i in [lo, hi) with a[i] <= x, given a[lo] <= x < a[hi] and `a`
// ascending; called by a whole wavefront (64 probes per round).
template <class T>
__device__ int64_t wave_last_le(const T* a, int64_t lo, int64_t hi, int64_t x) {
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + kWave - 1) / kWave;
    const int64_t p = lo + (int64_t)lane_id() * step;
    const uint64_t le = __ballot(p < hi && (int64_t)a[p] <= x);  // a prefix of the lanes, lane 0 included
    lo += (int64_t)(63 - __builtin_clzll(le)) * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// Copy every row's neighbours to its place in a new layout (offsets noff,
// `total` slots) and pad the rest of the new row; rows flagged in `skip` are
// left to the merge below.  Each workgroup writes a tile of consecutive new
// slots: its first wavefront finds the rows the tile covers, their offsets
// and degrees go to LDS, and every slot looks its row up there.  Every row
// holds at least one slot (its self-loop), so a tile covers at most
// kRelayTile rows.
constexpr int kRelayTile = 2048;
__global__ void __launch_bounds__(256) k_relayout(const int32_t* __restrict__ ooff, const int32_t* __restrict__ oidx,
                                                  const int32_t* __restrict__ deg, const int32_t* __restrict__ noff,
                                                  int32_t* __restrict__ nidx, int32_t n, int64_t total, int32_t pad,
                                                  const uint8_t* __restrict__ skip) {
  __shared__ int32_t s_noff[kRelayTile + 1];
  __shared__ int32_t s_src[kRelayTile];
  __shared__ int32_t s_deg[kRelayTile];
  __shared__ int64_t s_rows[2];
  for (int64_t q0 = (int64_t)blockIdx.x * kRelayTile; q0 < total; q0 += (int64_t)gridDim.x * kRelayTile) {
    const int64_t q1 = min(q0 + (int64_t)kRelayTile, total);
    if (threadIdx.x < kWave) {
      const int64_t r0 = wave_last_le(noff, 0, n, q0);
      const int64_t r1 = wave_last_le(noff, r0, min((int64_t)n, r0 + kRelayTile), q1 - 1);
      if (threadIdx.x == 0) {
        s_rows[0] = r0;
        s_rows[1] = min(r1 - r0 + 1, (int64_t)kRelayTile);
      }
    }
    __syncthreads();
    const int64_t r0 = s_rows[0];
    const int32_t nr = (int32_t)s_rows[1];
    for (int32_t i = threadIdx.x; i <= nr; i += blockDim.x) s_noff[i] = noff[r0 + i];
    for (int32_t i = threadIdx.x; i < nr; i += blockDim.x) {
      s_src[i] = (skip && skip[r0 + i]) ? -1 : ooff[r0 + i];
      s_deg[i] = deg[r0 + i];
    }
    __syncthreads();
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
      int32_t lo = 0, hi = nr - 1;  // the row of slot q: last i with s_noff[i] <= q
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (s_noff[mid] <= q) lo = mid; else hi = mid - 1;
      }
      const int32_t src = s_src[lo];
      if (src < 0) continue;
      const int32_t j = (int32_t)(q - s_noff[lo]);
      nidx[q] = j < s_deg[lo] ? oidx[src + j] : pad;
    }
    __syncthreads();
  }
}

// Row-local apply, first pass over a sorted effective batch (one entry per
// pair; delpre = prefix count of its deletions): list each touched row (the
// index of its first entry), flag it, and count the rows whose free slots
// cannot take their net insertions.
__global__ void k_local_rows(const uint64_t* __restrict__ eff, const int64_t* count,
                             const int64_t* __restrict__ delpre, int b, const int32_t* __restrict__ off,
                             const int32_t* __restrict__ deg, int64_t* heads, int64_t* nheads, int64_t* no_room,
                             uint8_t* touched) {
  const int64_t t = *count;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < t; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = (int64_t)(eff[e] >> (b + 1));
    if (e > 0 && (int64_t)(eff[e - 1] >> (b + 1)) == r) continue;
    const int64_t end = lower_bound_u64(eff, e + 1, t, (uint64_t)(r + 1) << (b + 1));
    const int64_t dels = delpre[end] - delpre[e];
    const int64_t grow = (end - e) - 2 * dels;  // insertions minus deletions
    if (grow > (int64_t)off[r + 1] - off[r] - deg[r]) atomicAdd((unsigned long long*)no_room, 1ull);
    heads[atomicAdd((unsigned long long*)nheads, 1ull)] = e;
    touched[r] = 1;
  }
}

// Work items of the second pass: each touched row in chunks of kMergeChunk
// old neighbours (at least one item per row); prefix over the row list.
constexpr int64_t kMergeChunk = 4096;
struct LoadRowChunks {
  const int64_t* heads;
  const int64_t* nheads;
  const uint64_t* eff;
  int b;
  const int32_t* deg;  // old degrees
  __device__ int64_t operator()(int64_t q) const {
    if (q >= *nheads) return 0;
    const int64_t d = deg[eff[heads[q]] >> (b + 1)];
    return d > kMergeChunk ? (d + kMergeChunk - 1) / kMergeChunk : 1;
  }
};

// One work item of the second pass, located by the block's first wavefront.
struct MergeItem {
  int64_t h, end, dels, ins, r;
  int32_t d, lo, hi;  // old degree; the item's old neighbours [lo, hi)
  bool first;         // the row's first item (also places insertions and pads)
};
__device__ void merge_item(int64_t w, const int64_t* heads, int64_t nr, const int64_t* cpre, const uint64_t* eff,
                           int64_t t, const int64_t* delpre, int b, const int32_t* deg, int deg_new, MergeItem* it) {
  __shared__ int64_t s_q;
  __syncthreads();  // the previous item is done with s_q
  if (threadIdx.x < kWave) {
    const int64_t q = wave_last_le(cpre, 0, nr, w);
    if (threadIdx.x == 0) s_q = q;
  }
  __syncthreads();
  const int64_t q = s_q;
  it->h = heads[q];
  it->r = (int64_t)(eff[it->h] >> (b + 1));
  it->end = lower_bound_u64(eff, it->h + 1, t, (uint64_t)(it->r + 1) << (b + 1));
  it->dels = delpre[it->end] - delpre[it->h];
  it->ins = (it->end - it->h) - it->dels;
  it->d = deg_new ? (int32_t)(deg[it->r] - it->ins + it->dels) : deg[it->r];
  const int64_t c = w - cpre[q];
  it->lo = (int32_t)min(c * kMergeChunk, (int64_t)it->d);
  it->hi = (int32_t)min((c + 1) * kMergeChunk, (int64_t)it->d);
  it->first = c == 0;
}

// In place, first: the old neighbours of the touched rows go to `cp` at
// their own offsets (the merge then reads them there).
__global__ void __launch_bounds__(256) k_row_save(const int64_t* __restrict__ heads, const int64_t* nheads,
                                                  const int64_t* __restrict__ cpre, const uint64_t* __restrict__ eff,
                                                  const int64_t* count, const int64_t* __restrict__ delpre, int b,
                                                  const int32_t* __restrict__ deg, const int32_t* __restrict__ off,
                                                  const int32_t* __restrict__ idx, int32_t* __restrict__ cp) {
  const int64_t nr = *nheads, t = *count, items = cpre[nr];
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    MergeItem it;
    merge_item(w, heads, nr, cpre, eff, t, delpre, b, deg, 0, &it);
    const int32_t os = off[it.r];
    for (int32_t i = it.lo + threadIdx.x; i < it.hi; i += blockDim.x) cp[os + i] = idx[os + i];
  }
}

// Row-local apply, second pass: per work item, the old neighbours [lo, hi)
// of a touched row r (row r of soff/sidx) are merged with the row's entries
// (a deletion drops an old neighbour, an insertion adds one) into row r of
// doff/didx, ascending; the row's first item also places its insertions and
// pads the rest of the row.  The position of each result follows from
// counts: an old neighbour x moves by the insertions minus the deletions
// before it in the row's entries; an insertion y lands after the old
// neighbours below y, less the deletions and plus the insertions before it.
// `deg` holds the old degrees, or the new ones when deg_new.
__global__ void __launch_bounds__(256) k_row_merge(const int64_t* __restrict__ heads, const int64_t* nheads,
                                                   const int64_t* __restrict__ cpre, const uint64_t* __restrict__ eff,
                                                   const int64_t* count, const int64_t* __restrict__ delpre, int b,
                                                   const int32_t* __restrict__ deg, int deg_new,
                                                   const int32_t* __restrict__ soff, const int32_t* sidx,
                                                   const int32_t* __restrict__ doff, int32_t* didx, int32_t pad) {
  const uint64_t mask = (1ull << b) - 1;
  const int64_t nr = *nheads, t = *count, items = cpre[nr];
  for (int64_t w = blockIdx.x; w < items; w += gridDim.x) {
    MergeItem it;
    merge_item(w, heads, nr, cpre, eff, t, delpre, b, deg, deg_new, &it);
    const int32_t* old = sidx + soff[it.r];
    const int32_t ds = doff[it.r];
    const uint64_t rk = (uint64_t)it.r << (b + 1);
    for (int32_t i = it.lo + threadIdx.x; i < it.hi; i += blockDim.x) {
      const int32_t x = old[i];
      const uint64_t kx = rk | ((uint64_t)x << 1);  // the deletion key of (r, x)
      const int64_t e = lower_bound_u64(eff, it.h, it.end, kx);
      if (e < it.end && eff[e] == kx) continue;
      const int64_t dl = delpre[e] - delpre[it.h];
      didx[ds + i + (e - it.h) - 2 * dl] = x;
    }
    if (!it.first) continue;
    for (int64_t j = it.h + threadIdx.x; j < it.end; j += blockDim.x) {
      const uint64_t k = eff[j];
      if (!(k & 1ull)) continue;
      const int32_t y = (int32_t)((k >> 1) & mask);
      const int64_t dl = delpre[j] - delpre[it.h];
      didx[ds + lower_bound_i32(old, 0, it.d, y) + (j - it.h) - 2 * dl] = y;
    }
    const int32_t len = doff[it.r + 1] - ds;
    for (int32_t p = (int32_t)(it.d + it.ins - it.dels) + threadIdx.x; p < len; p += blockDim.x) didx[ds + p] = pad;
  }
}

__global__ void k_clear_touched(const int64_t* heads, const int64_t* nheads, const uint64_t* eff, int b,
                                uint8_t* touched) {
  const int64_t nr = *nheads;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nr; q += (int64_t)gridDim.x * blockDim.x)
    touched[eff[heads[q]] >> (b + 1)] = 0;
}

// Member-local batch ids -> union ids, with validation against the member size.
__global__ void k_offset_ids(const int32_t* a, const int32_t* b, int64_t cnt, int32_t nmem, int64_t base, int32_t* oa,
                             int32_t* ob, int64_t* err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = a[i], v = b[i];
    if (u < 0 || u >= nmem || v < 0 || v >= nmem) {
      atomicOr((unsigned long long*)err, 1ull);
      oa[i] = 0;
      ob[i] = 0;
    } else {
      oa[i] = (int32_t)(u + base);
      ob[i] = (int32_t)(v + base);
    }
  }

}
__global__ void k_perm_from_sorted(const uint64_t* keys, int32_t n, int b, int32_t* perm, int32_t* inv) {
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)(keys[i] & mask);
    inv[i] = v;
    perm[v] = (int32_t)i;
  }
}

// Edge keys (row << b | col) in internal ids plus one self-loop per vertex;
// ids were validated by k_validate_count.
__global__ void k_make_graph_keys(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int b,
                                  const int32_t* perm, uint64_t* keys) {
  const int64_t total = m + n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k;
    if (i < m) {
      int32_t u = src[i], v = dst[i];
      if (perm) {
        u = perm[u];
        v = perm[v];
      }
      k = ((uint64_t)u << b) | (uint64_t)v;
    } else {
      const uint64_t v = (uint64_t)(i - m);
      k = (v << b) | v;  // the self-loop of every vertex
    }
    keys[i] = k;
  }
}

__global__ void k_mark_unique(const uint64_t* keys, int64_t n, uint8_t* keep) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    keep[i] = (keys[i] != kBadKey) && (i == 0 || keys[i] != keys[i - 1]);
}

// Sorted unique (row << b | col) keys -> CSR (every row holds its self-loop,
// so every row start is written).
__global__ void k_csr_from_sorted(const uint64_t* keys, int64_t m, int b, int32_t n, int32_t* off, int32_t* idx) {
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    const uint64_t row = k >> b;
    idx[i] = (int32_t)(k & mask);
    if (i == 0 || (keys[i - 1] >> b) != row) off[row] = (int32_t)i;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) off[n] = (int32_t)m;
}

// Internal CSR -> (caller row << b | caller col) keys, one thread per row; the
// keys of row i go to pos[i] on (its neighbours only, not its free slots).
__global__ void k_external_keys(const int32_t* off, const int32_t* idx, const int32_t* deg, const int32_t* pos,
                                int32_t n, const int32_t* inv, int b, uint64_t* keys) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t r = (uint64_t)inv[i] << b;
    const int32_t s = off[i], q = pos[i], d = deg[i];
    for (int32_t j = 0; j < d; j++) keys[q + j] = r | (uint64_t)inv[idx[s + j]];
  }
}

__global__ void k_transpose_keys(const uint64_t* in, int64_t m, int b, uint64_t* out) {
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = in[i];
    out[i] = ((k & mask) << b) | (k >> b);
  }
}

// Batch keys; out-of-range ids raise err and produce kBadKey.
__global__ void k_make_batch_keys(const int32_t* del_src, const int32_t* del_dst, int64_t nd, const int32_t* ins_src,
                                  const int32_t* ins_dst, int64_t ni, int32_t n, int b, const int32_t* perm,
                                  uint64_t* keys, int64_t* err) {
  const int64_t total = nd + ni;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const bool ins = i >= nd;
    int32_t u = ins ? ins_src[i - nd] : del_src[i];
    int32_t v = ins ? ins_dst[i - nd] : del_dst[i];
    uint64_t k;
    if (u < 0 || u >= n || v < 0 || v >= n) {
      atomicOr((unsigned long long*)err, 1ull);
      k = kBadKey;
    } else {
      if (perm) {
        u = perm[u];
        v = perm[v];
      }
      k = ((uint64_t)u << (b + 1)) | ((uint64_t)v << 1) | (ins ? 1ull : 0ull);
    }
    keys[i] = k;
  }
}

// Classify each distinct pair of a sorted batch against the old out-CSR.
// The last key of a pair's run owns the pair: it is an insertion key iff the
// pair was inserted; the pair was deleted iff (pair << 1) is present.
//   effective insertion: inserted and not in E^{t-1}
//   effective deletion:  deleted, in E^{t-1}, and not inserted (insert wins)
// Effective pairs set row deltas, touched rows and the pending marks.  When
// the batch failed validation (bit 0 of *bad) nothing is effective and nothing
// is marked, so the graph's state is untouched and the host reports the error
// after the (then trivial) rebuild.
__global__ void k_classify(const uint64_t* keys, int64_t nk, int b, const int32_t* ooff, const int32_t* oidx,
                           uint8_t* keep, int32_t* delta_out, int32_t* delta_in, uint8_t* touched_out,
                           uint8_t* touched_in, uint8_t* pend_src, uint8_t* pend_tgt, int64_t* counters,
                           const int32_t* gidv, int64_t* g_self, const int64_t* bad) {
  const uint64_t mask = (1ull << b) - 1;
  const bool invalid = (*bad & 1) != 0;
  int64_t n_ins = 0, n_del = 0, n_self = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nk; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    uint8_t kp = 0;
    const uint64_t pair = k >> 1;
    const bool owner = !invalid && (k != kBadKey) && (i + 1 == nk || (keys[i + 1] >> 1) != pair);
    if (owner) {
      const bool has_ins = k & 1ull;
      const int64_t q = lower_bound_u64(keys, 0, i + 1, pair << 1);
      const bool has_del = keys[q] == (pair << 1);
      const int32_t u = (int32_t)(pair >> b);
      const int32_t v = (int32_t)(pair & mask);
      if (u == v) {
        if (has_del) {
          n_self++;
          if (gidv) atomicAdd((unsigned long long*)&g_self[gidv[u]], 1ull);  // batch: per member
        }
      } else {
        const int32_t s = ooff[u], e = ooff[u + 1];
        const int32_t p = lower_bound_i32(oidx, s, e, v);
        const bool exists = p < e && oidx[p] == v;
        const bool eff_ins = has_ins && !exists;
        const bool eff_del = has_del && exists && !has_ins;
        if (eff_ins || eff_del) {
          if (delta_out) {  // row deltas and touched rows: read by the rebuild for many entries only
            const int32_t d = eff_ins ? 1 : -1;
            atomicAdd(&delta_out[u], d);
            atomicAdd(&delta_in[v], d);
            touched_out[u] = 1;
            touched_in[v] = 1;
          }
          pend_src[u] = 1;
          if (eff_del) pend_tgt[v] = 1;
          kp = 1;
          if (eff_ins) n_ins++; else n_del++;
        }
      }
    }
    keep[i] = kp;
  }
  n_ins = wave_sum_i64(n_ins);
  n_del = wave_sum_i64(n_del);
  n_self = wave_sum_i64(n_self);
  if (lane_id() == 0) {
    if (n_ins) atomicAdd((unsigned long long*)&counters[0], (unsigned long long)n_ins);
    if (n_del) atomicAdd((unsigned long long*)&counters[1], (unsigned long long)n_del);
    if (n_self) atomicAdd((unsigned long long*)&counters[2], (unsigned long long)n_self);
  }
}

// Effective list in out-order (row = u) -> in-order keys (row = v); entries
// past *count become kBadKey so a sort over nk keys leaves them at the end.
__global__ void k_in_order_keys(const uint64_t* eff, const int64_t* count, int64_t nk, int b, uint64_t* out) {
  const uint64_t mask = (1ull << b) - 1;
  const int64_t t = *count;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nk; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < t) {
      const uint64_t k = eff[i];
      const uint64_t u = k >> (b + 1), v = (k >> 1) & mask;
      out[i] = (v << (b + 1)) | (u << 1) | (k & 1ull);
    } else {
      out[i] = kBadKey;
    }
  }
}

struct LoadIsDel {
  const uint64_t* eff;
  const int64_t* count;
  __device__ int64_t operator()(int64_t i) const { return (i < *count && !(eff[i] & 1ull)) ? 1 : 0; }
};
struct StoreI64b {
  int64_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = v; }
};

// Rebuild of one CSR for a batch with many effective entries (few entries take
// the run-by-run copy further below).  Rows are taken in groups of 64 (one per
// lane).  A group without touched rows keeps its rows and only shifts them,
// and the shift (new offset - old offset) stays the same up to the next
// touched group, so k_shift_copy moves each run of untouched groups as one
// contiguous copy.  k_rebuild handles the touched groups: their old edges are
// cut into pieces of at most `piece` edges (piece_pre = prefix of the piece
// counts per group, zero for untouched groups) and each wavefront takes one
// piece, so a long row is spread over many wavefronts.  In a touched row an
// old element x lands at j - #del(<x) + #ins(<x) (counts by binary search over
// the row's sorted effective entries, delpre = prefix count of deletions in
// that list); deleted elements are dropped.  Insertions are placed by
// k_place_inserts.

// True iff a row of group g (rows g*64 .. g*64+63, clipped to n) is touched.
__device__ __forceinline__ bool group_touched(const uint8_t* touched, int64_t g, int32_t n) {
  const int64_t r0 = g * kWave;
  if (r0 + kWave <= n) {
    const uint64_t* t8 = reinterpret_cast<const uint64_t*>(touched + r0);  // 64-byte aligned
    uint64_t any = 0;
#pragma unroll
    for (int i = 0; i < kWave / 8; i++) any |= t8[i];
    return any != 0;
  }
  bool any = false;
  for (int64_t r = r0; r < n; r++) any |= touched[r] != 0;
  return any;
}

struct LoadPieces {
  const int32_t* ooff;
  const uint8_t* touched;  // 64-byte aligned, n entries
  int32_t n;
  int32_t piece;
  __device__ int64_t operator()(int64_t g) const {
    const int32_t r0 = (int32_t)(g * kWave);
    const int32_t r1 = (int32_t)min((int64_t)r0 + kWave, (int64_t)n);
    if (!group_touched(touched, g, n)) return 0;
    const int64_t len = (int64_t)ooff[r1] - ooff[r0];
    return len > piece ? (len + piece - 1) / piece : 1;
  }
};
struct StorePieces {
  int64_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = v; }
};

__device__ __forceinline__ int64_t upper_bound_pre(const int64_t* a, int64_t lo, int64_t hi, int64_t x) {
  while (lo < hi) {
    int64_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// largest lane j with st[j] <= e (st non-decreasing across lanes, st[0] <= e)
__device__ __forceinline__ int lane_seg(int32_t st, int32_t e) {
  int lo = 0, hi = kWave;
#pragma unroll
  for (int i = 0; i < 6; i++) {
    const int mid = (lo + hi) >> 1;
    if (__shfl(st, mid, kWave) <= e) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x = min(x, (int64_t)__shfl_xor(x, o, kWave));
  return x;
}
__device__ __forceinline__ int64_t wave_max_i64(int64_t x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, (int64_t)__shfl_xor(x, o, kWave));
  return x;
}

// Each workgroup takes `chunk` entries of the new index array and fills those
// that belong to untouched groups.  Its waves find runs of untouched groups 64
// groups at a time (lane l looks at group g + l) and copy each run with its
// shift.  mnew = noff[n] is read on the device; the grid covers an upper bound.
constexpr int kCopyBlock = 256;

__global__ void __launch_bounds__(kCopyBlock) k_shift_copy(const int32_t* __restrict__ ooff,
                                                           const int32_t* __restrict__ oidx,
                                                           const int32_t* __restrict__ noff,
                                                           int32_t* __restrict__ nidx, const uint8_t* touched,
                                                           int32_t n, int32_t chunk, int64_t* err) {
  const int64_t mnew = noff[n];
  const int64_t groups = ((int64_t)n + kWave - 1) / kWave;
  const int lane = lane_id();
  for (int64_t q0 = (int64_t)blockIdx.x * chunk; q0 < mnew; q0 += (int64_t)gridDim.x * chunk) {
    const int64_t q1 = min(q0 + (int64_t)chunk, mnew);
    // the row holding q0: the last row that starts at or before it
    int64_t lo = 0, hi = (int64_t)n - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if ((int64_t)noff[mid] <= q0) lo = mid; else hi = mid - 1;
    }
    int64_t g = lo / kWave;
    int64_t q = q0;
    while (q < q1 && g < groups) {
      const int64_t gl = g + lane;
      const bool tl = gl < groups && group_touched(touched, gl, n);
      const uint64_t tm = __ballot(tl);  // bit l: group g + l is touched
      if (tm & 1ull) {  // touched groups are left to k_rebuild
        const int run = (~tm == 0ull) ? kWave : __builtin_ctzll(~tm);
        g = min(g + run, groups);
        q = max(q, (int64_t)noff[min(g * kWave, (int64_t)n)]);
        continue;
      }
      const int run = tm == 0ull ? kWave : __builtin_ctzll(tm);
      const int64_t tg = min(g + run, groups);
      const int32_t ra = (int32_t)(g * kWave), rb = (int32_t)min(tg * kWave, (int64_t)n);
      const int64_t shift = (int64_t)noff[ra] - ooff[ra];
      if ((int64_t)noff[rb] - ooff[rb] != shift) {  // offsets disagree: refuse to write
        if (threadIdx.x == 0) atomicOr((unsigned long long*)err, 2ull);
        break;
      }
      const int64_t end = min((int64_t)noff[rb], q1);
      int64_t p = q + threadIdx.x;
      for (; p + 7 * kCopyBlock < end; p += 8 * kCopyBlock) {
        int32_t x[8];
#pragma unroll
        for (int k = 0; k < 8; k++) x[k] = __builtin_nontemporal_load(oidx + (p + k * kCopyBlock - shift));
#pragma unroll
        for (int k = 0; k < 8; k++) nidx[p + k * kCopyBlock] = x[k];
      }
      for (; p < end; p += kCopyBlock) nidx[p] = __builtin_nontemporal_load(oidx + (p - shift));
      q = end;
      g = tg;
    }
  }
}

// Few effective entries: the old index array cut at the entries is a list of
// runs, each moved by one shift.  With the entries in (row, column) order,
// opos[e] is entry e's position in the old array (a deleted element's own
// position, an insertion's insertion point), non-decreasing in e.  Before
// entry e the old elements have moved by S_e = #ins(<e) - #del(<e) =
// e - 2 * delpre[e]; entry e cuts the new array at dcut(e) = opos[e] + S_e
// (where an insertion lands), and the run after it starts at dcut(e) + ins(e)
// with shift S_{e+1}.  opos comes from a binary search of the entry's column
// in its old row (k_run_offsets).
__device__ __forceinline__ int64_t run_cut(const int64_t* opos, const int64_t* delpre, int64_t e) {
  return opos[e] + e - 2 * delpre[e];
}
__device__ __forceinline__ int64_t run_begin(const uint64_t* eff, const int64_t* opos, const int64_t* delpre,
                                             int64_t e) {
  return e < 0 ? 0 : run_cut(opos, delpre, e) + (int64_t)(eff[e] & 1ull);
}

// Each workgroup fills `chunk` entries of the new index array: the runs that
// cover them and the insertions that land between the runs.  The runs and
// the insertion slots tile the new array in entry order; the workgroup that
// takes position 0 checks that the tiling ends inside the new array.
// m_new (optional) receives the new edge count of `m_off`.
__global__ void __launch_bounds__(kCopyBlock) k_run_copy(const int32_t* __restrict__ oidx,
                                                         int32_t* __restrict__ nidx, const uint64_t* eff,
                                                         const int64_t* delpre, const int64_t* opos,
                                                         const int64_t* count, int b, const int32_t* noff, int32_t n,
                                                         int64_t m_old, int32_t chunk, int64_t* err,
                                                         const int32_t* m_off, int64_t* m_new) {
  const uint64_t mask = (1ull << b) - 1;
  const int64_t mnew = noff[n];
  const int64_t T = *count;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (m_new) *m_new = m_off[n];
    if (T > 0 && run_begin(eff, opos, delpre, T - 1) > mnew) atomicOr((unsigned long long*)err, 2ull);
  }
  for (int64_t q0 = (int64_t)blockIdx.x * chunk; q0 < mnew; q0 += (int64_t)gridDim.x * chunk) {
    const int64_t q1 = min(q0 + (int64_t)chunk, mnew);
    // the run holding q0: the last e in [-1, T) whose run begins at or before q0
    int64_t lo = -1, hi = T - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (run_begin(eff, opos, delpre, mid) <= q0) lo = mid; else hi = mid - 1;
    }
    int64_t e = lo;
    int64_t q = q0;
    while (q < q1) {
      const int64_t start = run_begin(eff, opos, delpre, e);
      const int64_t end = e + 1 < T ? run_cut(opos, delpre, e + 1) : mnew;
      const int64_t shift = e < 0 ? 0 : (e + 1) - 2 * delpre[e + 1];
      const int64_t a = max(q, start), z = min(end, q1);
      if (a < z) {
        if (a - shift < 0 || z - shift > m_old) {  // runs disagree with the array: refuse to write
          if (threadIdx.x == 0) atomicOr((unsigned long long*)err, 2ull);
          break;
        }
        int64_t p = a + threadIdx.x;
        for (; p + 7 * kCopyBlock < z; p += 8 * kCopyBlock) {
          int32_t x[8];
#pragma unroll
          for (int k = 0; k < 8; k++) x[k] = __builtin_nontemporal_load(oidx + (p + k * kCopyBlock - shift));
#pragma unroll
          for (int k = 0; k < 8; k++) nidx[p + k * kCopyBlock] = x[k];
        }
        for (; p < z; p += kCopyBlock) nidx[p] = __builtin_nontemporal_load(oidx + (p - shift));
      }
      if (e + 1 >= T) break;
      // entry e+1 cuts at `end`; an insertion lands there
      const uint64_t k = eff[e + 1];
      if ((k & 1ull) && end >= q0 && end < q1 && threadIdx.x == 0) nidx[end] = (int32_t)((k >> 1) & mask);
      q = max(z, run_begin(eff, opos, delpre, e + 1));
      e++;
    }
  }
}

// The same copy when the entries cut the old array into short runs (under
// kShortRun elements on average): wavefront w takes run w - 1 (run e holds the
// old elements between entries e and e + 1), copies it with its shift and
// writes entry e + 1's insertion behind it, so the runs go in parallel with
// no search for a chunk's first run and no run-after-run walk.  A run longer
// than `piece` elements (runs can be very uneven: entries that cluster leave
// one long run) is cut into pieces listed in `pieces` (run + 1 above bit 20,
// piece number below), which k_run_copy_pieces then copies a workgroup each.
constexpr int64_t kShortRun = 4096;
constexpr int kPieceBits = 20;
__global__ void __launch_bounds__(256) k_run_copy_waves(const int32_t* __restrict__ oidx, int32_t* __restrict__ nidx,
                                                        const uint64_t* eff, const int64_t* delpre,
                                                        const int64_t* opos, const int64_t* count, int b,
                                                        const int32_t* noff, int32_t n, int64_t m_old, int64_t* err,
                                                        const int32_t* m_off, int64_t* m_new, int64_t piece,
                                                        int64_t* pieces, int64_t piece_cap, int64_t* npieces) {
  const uint64_t mask = (1ull << b) - 1;
  const int64_t mnew = noff[n];
  const int64_t T = *count;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (m_new) *m_new = m_off[n];
    if (T > 0 && run_begin(eff, opos, delpre, T - 1) > mnew) atomicOr((unsigned long long*)err, 2ull);
  }
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int lane = lane_id();
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave - 1; e < T; e += waves) {
    const int64_t start = run_begin(eff, opos, delpre, e);
    const int64_t end = e + 1 < T ? run_cut(opos, delpre, e + 1) : mnew;
    const int64_t shift = e < 0 ? 0 : (e + 1) - 2 * delpre[e + 1];
    if (start < end) {
      if (start - shift < 0 || end - shift > m_old || end > mnew) {  // runs disagree with the array: refuse to write
        if (lane == 0) atomicOr((unsigned long long*)err, 2ull);
        continue;
      }
      if (end - start <= piece) {
        int64_t p = start + lane;
        for (; p + 3 * kWave < end; p += 4 * kWave) {
          int32_t x[4];
#pragma unroll
          for (int k = 0; k < 4; k++) x[k] = __builtin_nontemporal_load(oidx + (p + k * kWave - shift));
#pragma unroll
          for (int k = 0; k < 4; k++) nidx[p + k * kWave] = x[k];
        }
        for (; p < end; p += kWave) nidx[p] = __builtin_nontemporal_load(oidx + (p - shift));
      } else {
        const int64_t np = (end - start + piece - 1) / piece;
        int64_t base = 0;
        if (lane == 0) base = (int64_t)atomicAdd((unsigned long long*)npieces, (unsigned long long)np);
        base = __shfl(base, 0, kWave);
        if (base + np > piece_cap) {  // the piece size is chosen so that the list holds every piece
          if (lane == 0) atomicOr((unsigned long long*)err, 2ull);
        } else {
          for (int64_t j = lane; j < np; j += kWave) pieces[base + j] = ((e + 1) << kPieceBits) | j;
        }
      }
    }
    if (e + 1 < T && lane == 0) {
      const uint64_t k = eff[e + 1];
      if (k & 1ull) {
        if (end < 0 || end >= mnew) atomicOr((unsigned long long*)err, 2ull);
        else nidx[end] = (int32_t)((k >> 1) & mask);
      }
    }
  }
}

// The pieces of the long runs listed by k_run_copy_waves, a workgroup each.
__global__ void __launch_bounds__(256) k_run_copy_pieces(const int32_t* __restrict__ oidx,
                                                         int32_t* __restrict__ nidx, const uint64_t* eff,
                                                         const int64_t* delpre, const int64_t* opos,
                                                         const int64_t* count, const int32_t* noff, int32_t n,
                                                         int64_t piece, const int64_t* pieces,
                                                         const int64_t* npieces) {
  const int64_t mnew = noff[n];
  const int64_t T = *count, total = *npieces;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int64_t it = pieces[w];
    const int64_t e = (it >> kPieceBits) - 1, j = it & ((1ll << kPieceBits) - 1);
    const int64_t start = run_begin(eff, opos, delpre, e);
    const int64_t end = e + 1 < T ? run_cut(opos, delpre, e + 1) : mnew;
    const int64_t shift = e < 0 ? 0 : (e + 1) - 2 * delpre[e + 1];
    const int64_t a = start + j * piece, z = min(a + piece, end);
    int64_t p = a + threadIdx.x;
    for (; p + 3 * 256 < z; p += 4 * 256) {
      int32_t x[4];
#pragma unroll
      for (int k = 0; k < 4; k++) x[k] = __builtin_nontemporal_load(oidx + (p + k * 256 - shift));
#pragma unroll
      for (int k = 0; k < 4; k++) nidx[p + k * 256] = x[k];
    }
    for (; p < z; p += 256) nidx[p] = __builtin_nontemporal_load(oidx + (p - shift));
  }
}

// Few effective entries: the new row offsets are the old ones plus the shift
// S(r) = #ins - #del over the entries of the rows before r (e - 2*delpre[e]
// for the first entry e of row r or later, as in the run copy).  Each
// workgroup takes `rows` of the n+1 offsets (256 to 4096, so that large graphs
// get a few thousand workgroups and small ones one offset per thread) and
// finds the chunk's entries once; a row's search then covers only those.
static int32_t run_offset_rows(int32_t n) {
  int32_t rows = 256;
  while (rows < 4096 && ((int64_t)n + 1) / rows > 4096) rows <<= 1;
  return rows;
}
// The same launch computes the entries' old positions opos: workgroups
// [0, off_blocks) take the offsets, the others the entries.
__global__ void __launch_bounds__(256) k_run_offsets(const int32_t* __restrict__ ooff, int32_t* __restrict__ noff,
                                                     const int32_t* __restrict__ oidx, int64_t* opos,
                                                     const uint64_t* eff, const int64_t* delpre, const int64_t* count,
                                                     int b, int32_t n, int32_t rows, int32_t off_blocks) {
  const int64_t T = *count;
  if ((int)blockIdx.x >= off_blocks) {
    const uint64_t mask = (1ull << b) - 1;
    const int64_t stride = (int64_t)(gridDim.x - off_blocks) * blockDim.x;
    for (int64_t e = (blockIdx.x - off_blocks) * (int64_t)blockDim.x + threadIdx.x; e < T; e += stride) {
      const uint64_t k = eff[e];
      const int32_t r = (int32_t)(k >> (b + 1));
      const int32_t x = (int32_t)((k >> 1) & mask);
      opos[e] = lower_bound_i32(oidx, ooff[r], ooff[r + 1], x);
    }
    return;
  }
  // the chunk's entries (rows and shifts) staged in LDS when they fit
  constexpr int kStage = 512;
  __shared__ int32_t st_row[kStage];
  __shared__ int64_t st_shift[kStage + 1];
  for (int64_t r0 = blockIdx.x * (int64_t)rows; r0 <= n; r0 += (int64_t)off_blocks * rows) {
    const int64_t r1 = min(r0 + rows, (int64_t)n + 1);
    const int64_t e0 = lower_bound_u64(eff, 0, T, (uint64_t)r0 << (b + 1));
    const int64_t e1 = lower_bound_u64(eff, e0, T, (uint64_t)r1 << (b + 1));
    const int cnt = (int)min(e1 - e0, (int64_t)kStage + 1);
    if (cnt <= kStage) {  // the same in every thread
      __syncthreads();    // the previous chunk's readers are done
      for (int k = threadIdx.x; k <= cnt; k += blockDim.x) {
        if (k < cnt) st_row[k] = (int32_t)(eff[e0 + k] >> (b + 1));
        st_shift[k] = (e0 + k) - 2 * delpre[e0 + k];
      }
      __syncthreads();
      for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        int lo = 0, hi = cnt;  // first staged entry of row r or later
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (st_row[mid] < r) lo = mid + 1; else hi = mid;
        }
        noff[r] = (int32_t)((int64_t)ooff[r] + st_shift[lo]);
      }
    } else {
      for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const int64_t e = lower_bound_u64(eff, e0, e1, (uint64_t)r << (b + 1));
        noff[r] = (int32_t)((int64_t)ooff[r] + e - 2 * delpre[e]);
      }
    }
  }
}

// Touched groups.  When the group's effective entries fit in one wavefront
// (at most 63), lane k holds entry k and the deletion prefix count at k, and
// each element's counts come from a search over the lanes instead of global
// memory; otherwise the element searches its row's entries in memory.  Four
// rounds of 64 elements are loaded before any is placed.
__global__ void __launch_bounds__(256) k_rebuild(const int32_t* __restrict__ ooff, const int32_t* __restrict__ oidx,
                                                 const int32_t* __restrict__ noff, int32_t* __restrict__ nidx,
                                                 const uint8_t* touched, const uint64_t* eff, const int64_t* delpre,
                                                 const int64_t* count, int b, int32_t n, const int64_t* piece_pre,
                                                 int32_t piece, int64_t* err) {
  constexpr int kRounds = 4;
  const int lane = lane_id();
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int64_t groups = ((int64_t)n + kWave - 1) / kWave;
  const int64_t total = piece_pre[groups];
  const int64_t T = *count;
  for (int64_t q = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; q < total; q += waves) {
    const int64_t g = upper_bound_pre(piece_pre, 0, groups + 1, q) - 1;
    const int64_t k = q - piece_pre[g];
    const int32_t r0 = (int32_t)(g * kWave);
    const int32_t rend = (int32_t)min((int64_t)r0 + kWave, (int64_t)n);
    const int32_t r = r0 + lane;
    const bool valid = r < rend;
    const bool t = valid ? touched[r] != 0 : false;
    const int32_t s1 = ooff[rend];
    const int32_t a = ooff[r0] + (int32_t)(k * piece);
    const int32_t bnd = (int32_t)min((int64_t)a + piece, (int64_t)s1);
    // per-lane row data of the group (lane l holds row r0 + l)
    const int32_t os = valid ? ooff[r] : INT32_MAX;
    const int32_t base = valid ? noff[r] : 0;
    const int32_t lim = valid ? noff[r + 1] : 0;
    int64_t lo = 0, hi = 0, dlo = 0;
    if (t) {
      const uint64_t rk = (uint64_t)r << (b + 1);
      lo = lower_bound_u64(eff, 0, T, rk);
      hi = lower_bound_u64(eff, lo, T, rk + (1ull << (b + 1)));
      dlo = delpre[lo];
    }
    const int64_t glo = wave_min_i64(t ? lo : INT64_MAX);
    const int64_t ghi = wave_max_i64(t ? hi : (int64_t)-1);
    if (ghi < glo) {  // counted as touched but no touched row: refuse to write
      if (lane == 0) atomicOr((unsigned long long*)err, 2ull);
      continue;
    }
    const int64_t kg = ghi - glo;
    const bool win = kg < kWave;
    uint64_t wkey = ~0ull;  // padding sorts after every key
    int64_t wdp = 0;
    if (win) {
      if (lane < kg) wkey = eff[glo + lane];
      if (lane <= kg) wdp = delpre[glo + lane];
    }
    for (int32_t p0 = a; p0 < bnd; p0 += kRounds * kWave) {
      int32_t xs[kRounds];
#pragma unroll
      for (int u = 0; u < kRounds; u++) {
        const int32_t p = p0 + u * kWave + lane;
        xs[u] = p < bnd ? oidx[p] : 0;
      }
#pragma unroll
      for (int u = 0; u < kRounds; u++) {
        if (p0 + u * kWave >= bnd) break;  // the same for every lane
        const int32_t p = p0 + u * kWave + lane;
        const bool ok = p < bnd;
        const int j = lane_seg(os, ok ? p : p0 + u * kWave);
        const int32_t r_os = __shfl(os, j, kWave), r_base = __shfl(base, j, kWave), r_lim = __shfl(lim, j, kWave);
        const bool r_t = __shfl((int)t, j, kWave) != 0;
        const int64_t r_lo = __shfl(lo, j, kWave), r_hi = __shfl(hi, j, kWave), r_dlo = __shfl(dlo, j, kWave);
        const int32_t x = xs[u];
        const int32_t jj = p - r_os;
        const uint64_t xk = ((uint64_t)(r0 + j) << (b + 1)) | ((uint64_t)x << 1);
        int64_t pos = (int64_t)r_base + jj;
        bool drop = !ok;
        if (win) {
          // c = number of window entries below xk (every lane takes part)
          int c = 0;
#pragma unroll
          for (int st = kWave / 2; st >= 1; st >>= 1)
            if (__shfl(wkey, c + st - 1, kWave) < xk) c += st;
          const uint64_t at = __shfl(wkey, min(c, kWave - 1), kWave);
          const int64_t dp = __shfl(wdp, min(c, kWave - 1), kWave);
          if (r_t) {
            if (c < kg && at == xk) drop = true;  // deleted
            const int64_t qq = glo + c;
            const int64_t dels = dp - r_dlo;
            pos = (int64_t)r_base + jj - dels + ((qq - r_lo) - dels);
          }
        } else if (ok && r_t) {
          const int64_t qq = lower_bound_u64(eff, r_lo, r_hi, xk);
          if (qq < r_hi && eff[qq] == xk) drop = true;  // deleted
          const int64_t dels = delpre[qq] - r_dlo;
          pos = (int64_t)r_base + jj - dels + ((qq - r_lo) - dels);
        }
        if (drop) continue;
        if (pos < r_base || pos >= r_lim) {
          atomicOr((unsigned long long*)err, 2ull);
          continue;
        }
        nidx[pos] = x;
      }
    }
  }
}

// Insertions: an inserted y of row r lands at k + #old(<y) - #del(<y), k its
// index among the row's insertions.
__global__ void k_place_inserts(const int32_t* __restrict__ ooff, const int32_t* __restrict__ oidx,
                                const int32_t* __restrict__ noff, int32_t* __restrict__ nidx, const uint64_t* eff,
                                const int64_t* delpre, const int64_t* count, int b, int64_t* err) {
  const int64_t T = *count;
  const uint64_t mask = (1ull << b) - 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < T; e += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = eff[e];
    if (!(k & 1ull)) continue;
    const int32_t r = (int32_t)(k >> (b + 1));
    const int32_t y = (int32_t)((k >> 1) & mask);
    const int64_t lo = lower_bound_u64(eff, 0, e, (uint64_t)r << (b + 1));
    const int64_t dels = delpre[e] - delpre[lo];
    const int64_t kins = (e - lo) - dels;
    const int32_t os = ooff[r], oe = ooff[r + 1];
    const int32_t oless = lower_bound_i32(oidx, os, oe, y) - os;
    const int64_t pos = (int64_t)noff[r] + kins + oless - dels;
    if (pos < noff[r] || pos >= noff[r + 1]) {
      atomicOr((unsigned long long*)err, 2ull);
      continue;
    }
    nidx[pos] = y;
  }
}

__global__ void k_clear_rows(const uint64_t* eff, const int64_t* count, int b, int32_t* delta_out, int32_t* delta_in,
                             uint8_t* touched_out, uint8_t* touched_in) {
  const uint64_t mask = (1ull << b) - 1;
  const int64_t t = *count;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < t; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = eff[i];
    const int32_t u = (int32_t)(k >> (b + 1)), v = (int32_t)((k >> 1) & mask);
    delta_out[u] = 0;
    touched_out[u] = 0;
    delta_in[v] = 0;
    touched_in[v] = 0;
  }
}

__global__ void k_finish_apply(const int32_t* noff, int32_t n, int64_t* counters) { counters[5] = noff[n]; }

// ------------------------------------------------------------------ host
// Chunk partial sums of the pull's chunked bin: at most one chunk per vertex
// plus one per kPullChunk edges of the capacity.
// Chunk partial sums of the long-row bin: at most |bin| + its edges / chunk per
// pull; the single-launch loop gives every part its own range (one spare entry
// per part, parts are at least kPartVertices vertices apart but for the last).
static int64_t partial_entries(int32_t n, int64_t cap) {
  return (int64_t)n + 1 + cap / kPullChunk + (int64_t)n / kPartVertices + 2;
}

// Carve the scratch arrays from `base` (nullptr: only measure).  The arrays
// that must start at zero come first, so one clear covers them; returns the
// block size and, in *zero_bytes, the size of that prefix.
static size_t carve_scratch(dfpr_graph* g, char* base, size_t* zero_bytes) {
  const size_t n = (size_t)g->n;
  size_t off = 0;
  auto take = [&](auto*& ptr, size_t count) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    off = (off + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign;
    if (base) ptr = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
  };
  // zero-initialised prefix
  take(g->ctl, 1);
  take(g->flag_cur, n);
  take(g->flag_next, n);
  take(g->xflag, n);
  take(g->xflag2, n);
  take(g->ever, n);
  take(g->pend_src, n);
  take(g->touched_out, n);
  take(g->touched_in, n);
  take(g->delta_out, n);
  take(g->delta_in, n);
  take(g->arrive, n);
  if (zero_bytes) *zero_bytes = off;
  // contents defined before use
  take(g->contrib, n);
  take(g->contrib2, n);
  take(g->rn, n);
  if (g->perm) take(g->rint, n);
  take(g->worklist, n);
  take(g->all_bins, n);
  const size_t nbins = (n + 2047) / 2048;
  take(g->bin_blk, kBins * nbins + 2);
  take(g->chunk_pre, n + 1);
  take(g->piece_pre, n / kWave + 2);
  take(g->all_chunk_pre, n + std::max<size_t>(g->parts.size(), 1) + 1);
  take(g->big_list, n);
  take(g->big_pre, n + 1);
  g->scan_tmp_n = scan_tmp_elems((int64_t)n + 1);
  take(g->scan_tmp, g->scan_tmp_n);
  return (off + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign;
}

size_t scratch_size(const dfpr_graph* g) {
  dfpr_graph probe_fields;  // carve writes only pointer and size fields
  probe_fields.n = g->n;
  probe_fields.perm = g->perm;
  probe_fields.parts = g->parts;
  const size_t b = carve_scratch(&probe_fields, nullptr, nullptr);
  probe_fields.perm = nullptr;
  return b;
}

int attach_scratch(dfpr_graph* g, void* block, size_t bytes, hipStream_t s) {
  size_t zero = 0;
  if (carve_scratch(g, nullptr, &zero) > bytes) {
    set_error("scratch block too small");
    return DFPR_EINVAL;
  }
  carve_scratch(g, static_cast<char*>(block), &zero);
  g->scratch = block;
  g->scratch_bytes = bytes;
  DFPR_HIP(hipMemsetAsync(block, 0, zero, s));
  g->all_bins_valid = false;
  g->all_chunks_valid = false;
  g->pending_any = false;
  return DFPR_OK;
}

void detach_scratch(dfpr_graph* g) {
  g->ctl = nullptr;
  g->flag_cur = g->flag_next = g->xflag = g->xflag2 = g->ever = g->pend_src = nullptr;
  g->touched_out = g->touched_in = nullptr;
  g->delta_out = g->delta_in = g->arrive = nullptr;
  g->contrib = g->contrib2 = g->rn = g->rint = nullptr;
  g->worklist = g->all_bins = g->big_list = nullptr;
  g->bin_blk = g->chunk_pre = g->piece_pre = g->all_chunk_pre = g->big_pre = g->scan_tmp = nullptr;
  g->scratch = nullptr;
  g->scratch_bytes = 0;
  g->all_bins_valid = false;
  g->all_chunks_valid = false;
  g->pending_any = false;
}

size_t apply_buffer_bytes(int64_t nk, bool host_input) {
  auto r = [](size_t x) { return (x + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign; };
  size_t t = 0;
  t += 2 * r(nk * sizeof(uint64_t));                                              // keys_a, keys_b
  t += r(nk * sizeof(uint64_t) + nk);                                             // keys_c + keep bytes
  t += r((radix_hist_elems(nk) + std::max(radix_scan_tmp_elems(nk), scan_tmp_elems(nk + 1))) * sizeof(int64_t) +
         64);                                                                     // sort_hist
  t += r(3 * (nk + 1) * sizeof(int64_t));                                         // eff_pre
  t += r(2 * (nk + 1) * sizeof(int64_t));                                         // row_work
  if (host_input) t += r(2 * nk * sizeof(int32_t));                               // batch_in
  return t + 8 * Heap::kAlign;
}

// Per-handle state kept for the handle's life: control mirror, member tables
// and the chunk partial sums (sized by the edge capacity).
static int alloc_fixed_state(dfpr_graph* g) {
  g->partial_n = partial_entries(g->n, g->cap);
  DFPR_TRY(dalloc(&g->partial, (size_t)g->partial_n));
  DFPR_TRY(dalloc(&g->partial_x, (size_t)g->partial_n));
  DFPR_HIP(hipHostMalloc((void**)&g->ctl_host, sizeof(IterCtl), hipHostMallocDefault));
  const size_t G = (size_t)g->ngraphs;
  DFPR_TRY(dalloc(&g->nk, G));
  DFPR_TRY(dalloc(&g->done, G));
  g->gsub = G == 1 ? kSlots : kGSub;
  DFPR_TRY(dalloc(&g->gslots, G * g->gsub * kSlotStride));
  DFPR_TRY(dalloc(&g->g_dr, G));
  DFPR_TRY(dalloc(&g->g_iters, G));
  DFPR_TRY(dalloc(&g->g_ever, G));
  DFPR_TRY(dalloc(&g->g_eff, 4 * G));  // ins/del pairs, edges after, ignored self-loop deletions
  DFPR_HIP(hipHostMalloc(&g->g_host, G * (8 + 4 + 8 + 16 + 1) + 64, hipHostMallocDefault));
  DFPR_HIP(hipMemset(g->gslots, 0, G * g->gsub * kSlotStride * sizeof(unsigned long long)));
  DFPR_HIP(hipMemset(g->done, 0, G));
  std::vector<int32_t> nkh(G);
  for (size_t k = 0; k < G; k++) nkh[k] = (int32_t)(g->vbase[k + 1] - g->vbase[k]);
  DFPR_HIP(hipMemcpy(g->nk, nkh.data(), G * sizeof(int32_t), hipMemcpyHostToDevice));
  return DFPR_OK;
}

// A plain handle owns its scratch block for its whole life.
static int alloc_rank_scratch(dfpr_graph* g) {
  DFPR_TRY(alloc_fixed_state(g));
  const size_t bytes = scratch_size(g);
  void* block = nullptr;
  if (hipMalloc(&block, bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of %zu scratch bytes failed", bytes);
    return DFPR_ENOMEM;
  }
  g->scratch_owned = true;
  DFPR_TRY(attach_scratch(g, block, bytes, nullptr));
  DFPR_HIP(hipDeviceSynchronize());
  return DFPR_OK;
}

static int alloc_csr(Csr* c, int32_t n, int64_t cap) {
  DFPR_TRY(dalloc(&c->off, (size_t)n + 1));
  DFPR_TRY(dalloc(&c->idx, (size_t)cap));
  return DFPR_OK;
}
static void free_csr(Csr* c) {
  dfree(c->off);
  dfree(c->idx);
}

size_t csr_pair_bytes(int32_t n, int64_t cap) {
  auto r = [](size_t x) { return (x + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign; };
  return 2 * (r(((size_t)n + 1) * sizeof(int32_t)) + r((size_t)std::max<int64_t>(cap, 1) * sizeof(int32_t)));
}
void carve_csr_pair(void* block, int32_t n, int64_t cap, Csr* out, Csr* in) {
  auto r = [](size_t x) { return (x + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign; };
  const size_t bo = r(((size_t)n + 1) * sizeof(int32_t)), bi = r((size_t)std::max<int64_t>(cap, 1) * sizeof(int32_t));
  char* p = static_cast<char*>(block);
  out->off = reinterpret_cast<int32_t*>(p);
  out->idx = reinterpret_cast<int32_t*>(p + bo);
  in->off = reinterpret_cast<int32_t*>(p + bo + bi);
  in->idx = reinterpret_cast<int32_t*>(p + 2 * bo + bi);
}

int move_csrs_to_heap(dfpr_graph* g, Heap* heap, hipStream_t s) {
  void* block = heap->alloc(csr_pair_bytes(g->n, g->cap));
  if (!block) {
    set_error("the server heap cannot hold the graph's CSRs (%zu bytes)", csr_pair_bytes(g->n, g->cap));
    return DFPR_ENOMEM;
  }
  Csr out, in;
  carve_csr_pair(block, g->n, g->cap, &out, &in);
  const size_t ob = ((size_t)g->n + 1) * sizeof(int32_t), eb = (size_t)g->slots * sizeof(int32_t);
  if (hipMemcpyAsync(out.off, g->out.off, ob, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipMemcpyAsync(in.off, g->in.off, ob, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      (eb && hipMemcpyAsync(out.idx, g->out.idx, eb, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
      (eb && hipMemcpyAsync(in.idx, g->in.idx, eb, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess) {
    heap->free(block);
    set_error("copy of the graph's CSRs into the server heap failed");
    return DFPR_EHIP;
  }
  free_csr(&g->out);
  free_csr(&g->in);
  free_csr(&g->out2);
  free_csr(&g->in2);
  g->out = out;
  g->in = in;
  g->csr_heap = heap;
  g->csr_block = block;
  return DFPR_OK;
}

int graph_destroy(dfpr_graph* g) {
  if (!g) return DFPR_OK;
  (void)hipDeviceSynchronize();
  if (g->csr_heap) {  // served: one heap block; the rebuild targets belong to requests
    g->csr_heap->free(g->csr_block);
    g->csr_block = nullptr;
    g->out = g->in = g->out2 = g->in2 = Csr();
  }
  free_csr(&g->out);
  free_csr(&g->in);
  free_csr(&g->out2);
  free_csr(&g->in2);
  if (g->scratch_owned && g->scratch) (void)hipFree(g->scratch);
  detach_scratch(g);
  dfree(g->partial);
  dfree(g->partial_x);
  dfree(g->perm);
  dfree(g->inv);
  if (g->ctl_host) (void)hipHostFree(g->ctl_host);
  g->ctl_host = nullptr;
  dfree(g->gidv);
  dfree(g->vbase_d);
  dfree(g->nk);
  dfree(g->done);
  dfree(g->gslots);
  dfree(g->g_dr);
  dfree(g->g_iters);
  dfree(g->g_ever);
  dfree(g->g_eff);
  if (g->g_host) (void)hipHostFree(g->g_host);
  g->g_host = nullptr;
  if (g->fused_parts) (void)hipFree(g->fused_parts);
  g->fused_parts = nullptr;
  dfree(g->out_deg);
  dfree(g->in_deg);
  if (g->fused_parts_host) (void)hipHostFree(g->fused_parts_host);
  g->fused_parts_host = nullptr;
  delete g->tp;
  g->tp = nullptr;
  g->keys_a.release();
  g->keys_b.release();
  g->keys_c.release();
  g->sort_hist.release();
  g->eff_pre.release();
  g->batch_in.release();
  g->keys_in.release();
  g->row_work.release();
  g->pool.destroy();
  delete g;
  return DFPR_OK;
}

// Temporary device buffers of one create call.
struct CreateTmp {
  int32_t* coo = nullptr;
  uint64_t *ka = nullptr, *kb = nullptr;
  uint8_t* keep = nullptr;
  int64_t *pre = nullptr, *hist = nullptr, *tmp = nullptr, *cnt = nullptr;
  ~CreateTmp() {
    dfree(coo);
    dfree(ka);
    dfree(kb);
    dfree(keep);
    dfree(pre);
    dfree(hist);
    dfree(tmp);
    dfree(cnt);
  }
};

static int build_csr_from_keys(uint64_t** ka, uint64_t** kb, int64_t m, int b, int32_t n, Csr* c, int64_t* hist,
                               int64_t* tmp, hipStream_t s) {
  DFPR_TRY(radix_sort(ka, kb, m, 2 * b, hist, tmp, s));
  k_csr_from_sorted<<<grid_for(m, 256, 65536), 256, 0, s>>>(*ka, m, b, n, c->off, c->idx);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

int graph_create(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, dfpr_where where,
                 int64_t edge_capacity, int32_t flags, hipStream_t s, dfpr_graph** out,
                 const std::vector<int64_t>* members) {
  *out = nullptr;
  const int64_t total = m + n;
  if (total > INT32_MAX) {
    set_error("graph too large for int32 CSR offsets: %lld pairs", (long long)total);
    return DFPR_EINVAL;
  }
  dfpr_graph* g = new (std::nothrow) dfpr_graph();
  if (!g) {
    set_error("host allocation failed");
    return DFPR_ENOMEM;
  }
  DFPR_HIP(hipGetDevice(&g->device));
  g->n = n;
  g->id_bits = bits_for(n);
  if (members) {
    g->vbase = *members;
    g->ngraphs = (int32_t)members->size() - 1;
  } else {
    g->vbase = {0, (int64_t)n};
    g->ngraphs = 1;
  }
  const int b = g->id_bits;
  const int gbits = g->ngraphs > 1 ? bits_for(g->ngraphs) : 0;
  if (gbits + 24 + b > 64) {
    delete g;
    set_error("too many member graphs for the sort key");
    return DFPR_EINVAL;
  }
  const bool relabel = (flags & DFPR_CREATE_KEEP_IDS) == 0;
  int rc = DFPR_OK;
  {
    CreateTmp t;
    const int32_t *dsrc = src, *ddst = dst;
    auto fail = [&](int code) {
      graph_destroy(g);
      return code;
    };
    if (m > 0 && where == DFPR_HOST) {
      if ((rc = dalloc(&t.coo, (size_t)(2 * m))) != DFPR_OK) return fail(rc);
      if (hipMemcpyAsync(t.coo, src, m * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(t.coo + m, dst, m * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("edge upload failed");
        return fail(DFPR_EHIP);
      }
      dsrc = t.coo;
      ddst = t.coo + m;
    }
    const int64_t kmax = std::max<int64_t>(total, n);
    if ((rc = dalloc(&t.ka, kmax)) || (rc = dalloc(&t.kb, kmax)) || (rc = dalloc(&t.keep, total)) ||
        (rc = dalloc(&t.pre, total + 1)) || (rc = dalloc(&t.hist, radix_hist_elems(kmax))) ||
        (rc = dalloc(&t.tmp, std::max(radix_scan_tmp_elems(kmax), scan_tmp_elems(total + 1)))) ||
        (rc = dalloc(&t.cnt, 2)))
      return fail(rc);
    int32_t* deg = nullptr;
    if (relabel) {
      if ((rc = dalloc(&g->perm, n)) || (rc = dalloc(&g->inv, n))) return fail(rc);
      deg = reinterpret_cast<int32_t*>(t.kb);  // the second key buffer is free until the sort
      if (hipMemsetAsync(deg, 0, (size_t)n * sizeof(int32_t), s) != hipSuccess) return fail(DFPR_EHIP);
    }
    if (hipMemsetAsync(t.cnt, 0, 2 * sizeof(int64_t), s) != hipSuccess) return fail(DFPR_EHIP);
    if (m > 0) k_validate_count<<<grid_for(m, 256, 65536), 256, 0, s>>>(dsrc, ddst, m, n, deg, t.cnt);
    int64_t err = 0;
    if (hipMemcpyAsync(&err, t.cnt, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("edge validation failed");
      return fail(DFPR_EHIP);
    }
    if (err) {
      set_error("vertex id outside [0, %d)", n);
      return fail(DFPR_ERANGE);
    }
    if (g->ngraphs > 1) {
      if ((rc = dalloc(&g->gidv, n)) || (rc = dalloc(&g->vbase_d, g->vbase.size()))) return fail(rc);
      if (hipMemcpy(g->vbase_d, g->vbase.data(), g->vbase.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
          hipSuccess)
        return fail(DFPR_EHIP);
      k_member_ids<<<grid_for(n, 256, 65536), 256, 0, s>>>(g->vbase_d, g->ngraphs, n, g->gidv);
    }
    // parts of the all-vertex pull: whole members, about kPartVertices vertices each
    g->parts.clear();
    {
      dfpr_graph::Part pt;
      pt.lo = 0;
      for (int32_t k = 0; k < g->ngraphs; k++) {
        const int64_t hi = g->vbase[k + 1];
        if (hi - pt.lo >= kPartVertices || k + 1 == g->ngraphs) {
          pt.hi = hi;
          g->parts.push_back(pt);
          pt = dfpr_graph::Part();
          pt.lo = hi;
        }
      }
    }
    if (relabel) {
      // order vertices by member, then decreasing in-degree (ties by id)
      k_degree_keys<<<grid_for(n, 256, 65536), 256, 0, s>>>(deg, g->gidv, n, b, t.ka);
      if ((rc = radix_sort(&t.ka, &t.kb, n, gbits + 24 + b, t.hist, t.tmp, s))) return fail(rc);
      k_perm_from_sorted<<<grid_for(n, 256, 65536), 256, 0, s>>>(t.ka, n, b, g->perm, g->inv);
    }
    k_make_graph_keys<<<grid_for(total, 256, 65536), 256, 0, s>>>(dsrc, ddst, m, n, b, g->perm, t.ka);
    if ((rc = radix_sort(&t.ka, &t.kb, total, 2 * b, t.hist, t.tmp, s))) return fail(rc);
    k_mark_unique<<<grid_for(total, 256, 65536), 256, 0, s>>>(t.ka, total, t.keep);
    if ((rc = compact_keys(t.ka, t.keep, t.kb, total, t.cnt + 1, t.pre, t.tmp, s))) return fail(rc);
    int64_t mu = 0;
    if (hipMemcpyAsync(&mu, t.cnt + 1, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error("unique count readback failed");
      return fail(DFPR_EHIP);
    }
    g->m = g->slots = mu;
    int64_t cap = edge_capacity > 0 ? edge_capacity : mu + mu / 8 + 1024;
    cap = std::max<int64_t>(cap, mu);
    cap = std::min<int64_t>(cap, INT32_MAX);
    g->cap = cap;
    if ((rc = alloc_csr(&g->out, n, cap)) || (rc = alloc_csr(&g->in, n, cap)) || (rc = alloc_csr(&g->out2, n, cap)) ||
        (rc = alloc_csr(&g->in2, n, cap)))
      return fail(rc);
    // out-CSR straight from the unique sorted keys (already row-major by source)
    k_csr_from_sorted<<<grid_for(mu, 256, 65536), 256, 0, s>>>(t.kb, mu, b, n, g->out.off, g->out.idx);
    // in-CSR: transpose the keys and sort again
    k_transpose_keys<<<grid_for(mu, 256, 65536), 256, 0, s>>>(t.kb, mu, b, t.ka);
    if ((rc = build_csr_from_keys(&t.ka, &t.kb, mu, b, n, &g->in, t.hist, t.tmp, s))) return fail(rc);
    if ((rc = dalloc(&g->out_deg, n)) || (rc = dalloc(&g->in_deg, n))) return fail(rc);
    k_deg_from_off<<<grid_for(n, 256, 65536), 256, 0, s>>>(g->out.off, n, g->out_deg);
    k_deg_from_off<<<grid_for(n, 256, 65536), 256, 0, s>>>(g->in.off, n, g->in_deg);
    if ((rc = alloc_rank_scratch(g))) return fail(rc);
    if (hipStreamSynchronize(s) != hipSuccess) {
      set_error("graph creation failed on the device");
      return fail(DFPR_EHIP);
    }
  }
  *out = g;
  return DFPR_OK;
}

int graph_export(const dfpr_graph* g, int in_csr, int32_t* off, int32_t* idx, dfpr_where where, hipStream_t s) {
  const Csr& c = in_csr ? g->in : g->out;
  const int32_t* deg = in_csr ? g->in_deg : g->out_deg;
  const hipMemcpyKind kind = where == DFPR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  const bool padded = g->slots != g->m;  // some row has free slots
  if (!g->perm && !padded) {
    DFPR_HIP(hipMemcpyAsync(off, c.off, ((size_t)g->n + 1) * sizeof(int32_t), kind, s));
    if (g->m > 0) DFPR_HIP(hipMemcpyAsync(idx, c.idx, (size_t)g->m * sizeof(int32_t), kind, s));
    DFPR_HIP(hipStreamSynchronize(s));
    return DFPR_OK;
  }
  const int32_t n = g->n;
  const int64_t m = g->m;
  const int b = g->id_bits;
  CreateTmp t;
  Csr outc;
  int rc;
  int32_t* doff = off;
  int32_t* didx = idx;
  if (where == DFPR_HOST) {
    if ((rc = dalloc(&t.coo, (size_t)(n + 1 + m)))) return rc;
    doff = t.coo;
    didx = t.coo + n + 1;
  }
  // rows without their free slots: offsets from the degrees
  const int32_t* pos = c.off;
  if (padded) {
    if ((rc = dalloc(&t.pre, scan_tmp_elems(n)))) return rc;
    DFPR_TRY(scan_generic(LoadPadded{deg, 0}, StoreOff{doff}, n, t.pre, s));
    pos = doff;
  }
  if (!g->perm) {
    k_relayout<<<grid_for(m, kRelayTile, 65536), 256, 0, s>>>(c.off, c.idx, deg, doff, didx, n, m, n, nullptr);
    DFPR_HIP(hipGetLastError());
  } else {
    // caller numbering: map both ends of every edge back and sort again
    if ((rc = dalloc(&t.ka, m)) || (rc = dalloc(&t.kb, m)) || (rc = dalloc(&t.hist, radix_hist_elems(m))) ||
        (rc = dalloc(&t.tmp, radix_scan_tmp_elems(m))))
      return rc;
    k_external_keys<<<grid_for(n, 256, 65536), 256, 0, s>>>(c.off, c.idx, deg, pos, n, g->inv, b, t.ka);
    DFPR_HIP(hipGetLastError());
    outc.off = doff;
    outc.idx = didx;
    DFPR_TRY(build_csr_from_keys(&t.ka, &t.kb, m, b, n, &outc, t.hist, t.tmp, s));
    outc.off = outc.idx = nullptr;
  }
  if (where == DFPR_HOST) {
    DFPR_HIP(hipMemcpyAsync(off, doff, ((size_t)n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (m > 0) DFPR_HIP(hipMemcpyAsync(idx, didx, (size_t)m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  DFPR_HIP(hipStreamSynchronize(s));
  return DFPR_OK;
}

// Index-array slots an apply of `ni` insertions may need: a rebuild adds at
// most ni entries; a re-layout gives every row its free slots again.
int64_t slots_bound(const dfpr_graph* g, int64_t ni) {
  return std::max(g->slots, g->slack > 0 ? g->m + (int64_t)g->n * g->slack : (int64_t)0) + ni;
}

// Grow the edge capacity of all four index arrays to at least `want`.
int ensure_partials(dfpr_graph* g, int64_t cap) {
  const int64_t pn = partial_entries(g->n, cap);
  if (pn > g->partial_n) {
    dfree(g->partial);
    dfree(g->partial_x);
    DFPR_TRY(dalloc(&g->partial, (size_t)pn));
    DFPR_TRY(dalloc(&g->partial_x, (size_t)pn));
    g->partial_n = pn;
  }
  return DFPR_OK;
}

static int grow_capacity(dfpr_graph* g, int64_t want, hipStream_t s) {
  if (g->csr_heap) {  // a served graph's rebuild targets, sized by the server, hold the batch
    set_error("internal: a served graph's capacity is raised by its request");
    return DFPR_EHIP;
  }
  int64_t cap = std::min<int64_t>(std::max<int64_t>(want + want / 4, g->cap), INT32_MAX);
  DFPR_HIP(hipStreamSynchronize(s));
  for (Csr* c : {&g->out, &g->in, &g->out2, &g->in2}) {
    int32_t* p = nullptr;
    DFPR_TRY(dalloc(&p, (size_t)cap));
    if (c == &g->out || c == &g->in)
      DFPR_HIP(hipMemcpyAsync(p, c->idx, (size_t)g->slots * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    DFPR_HIP(hipStreamSynchronize(s));
    dfree(c->idx);
    c->idx = p;
  }
  g->cap = cap;
  return ensure_partials(g, cap);
}

// One CSR.  Few effective entries (at most one per 256 edges): runs between
// the entries.  Otherwise: runs of untouched groups, pieces of the touched
// groups, then the insertions.  Copy chunks and pieces get smaller on small
// graphs so that the work still spreads over many wavefronts.
// Few entries: opos was filled by k_run_offsets; m_new (optional) receives
// the new edge count of `m_off` (run path only).
static int rebuild_csr(dfpr_graph* g, const Csr& o, const Csr& nw, const uint8_t* touched, const uint64_t* eff,
                       const int64_t* delpre, int64_t* opos, const int64_t* cnt, int64_t nk, int64_t ni,
                       int64_t* err, const int32_t* m_off, int64_t* m_new, hipStream_t s) {
  const int32_t n = g->n;
  const int64_t groups = ((int64_t)n + kWave - 1) / kWave;
  int32_t chunk = 1024;
  while (chunk < 16384 && (int64_t)chunk * 2048 < g->slots) chunk <<= 1;
  const int64_t m_bound = g->slots + ni;  // the new slot count is at most this
  if (nk * 256 <= g->slots) {  // the same test as the offsets in graph_apply
    // many short runs (a workgroup would walk dozens of them one after the
    // other): one wavefront per run, and the long runs' pieces after them.
    // The piece list uses the group-rebuild scratch (idle on this path); the
    // piece size keeps every piece in it (long runs are at most m_bound/piece,
    // their pieces at most twice that).
    if (g->slots < (int64_t)kShortRun * nk) {
      const int64_t cap = (int64_t)n / kWave + 2;
      const int64_t piece = std::max<int64_t>(kShortRun, (2 * m_bound + cap - 1) / cap);
      int64_t* npieces = g->ctl->n_local + 5;
      DFPR_HIP(hipMemsetAsync(npieces, 0, sizeof(int64_t), s));
      k_run_copy_waves<<<grid_for(nk + 1, 256 / kWave, 1u << 16), 256, 0, s>>>(
          o.idx, nw.idx, eff, delpre, opos, cnt, g->id_bits, nw.off, n, g->slots, err, m_off, m_new, piece,
          g->piece_pre, cap, npieces);
      k_run_copy_pieces<<<grid_for(2 * m_bound / piece + 1, 1, 8192), 256, 0, s>>>(
          o.idx, nw.idx, eff, delpre, opos, cnt, nw.off, n, piece, g->piece_pre, npieces);
      DFPR_HIP(hipGetLastError());
      return DFPR_OK;
    }
    k_run_copy<<<grid_for(m_bound, chunk, 1u << 16), kCopyBlock, 0, s>>>(o.idx, nw.idx, eff, delpre, opos, cnt,
                                                                       g->id_bits, nw.off, n, g->slots, chunk, err,
                                                                       m_off, m_new);
    DFPR_HIP(hipGetLastError());
    return DFPR_OK;
  }
  int32_t piece = 256;
  while (piece < 4096 && (int64_t)piece * 65536 < g->slots) piece <<= 1;
  DFPR_TRY(scan_generic(LoadPieces{o.off, touched, n, piece}, StorePieces{g->piece_pre}, groups, g->scan_tmp, s));
  k_shift_copy<<<grid_for(m_bound, chunk, 1u << 16), kCopyBlock, 0, s>>>(o.off, o.idx, nw.off, nw.idx, touched, n,
                                                                       chunk, err);
  const int64_t est = std::min(groups, nk) + g->slots / piece + 1;  // upper bound on the piece count
  k_rebuild<<<grid_for(est, 4, 4096), 256, 0, s>>>(o.off, o.idx, nw.off, nw.idx, touched, eff, delpre, cnt,
                                                   g->id_bits, n, g->piece_pre, piece, err);
  k_place_inserts<<<grid_for(nk, 256, 4096), 256, 0, s>>>(o.off, o.idx, nw.off, nw.idx, eff, delpre, cnt, g->id_bits,
                                                          err);
  DFPR_HIP(hipGetLastError());
  return DFPR_OK;
}

// Lay both CSRs out again with `slack` free slots after every row (0: none).
int graph_set_row_slack(dfpr_graph* g, int32_t slack, hipStream_t s) {
  if (slack < 0 || slack > kMaxRowSlack) {
    set_error("row slack %d outside [0, %d]", slack, kMaxRowSlack);
    return DFPR_EINVAL;
  }
  if (g->csr_heap) {
    set_error("the row layout of a served graph is fixed when it is added");
    return DFPR_EINVAL;
  }
  const int32_t n = g->n;
  const int64_t want = g->m + (int64_t)n * slack;
  if (want > INT32_MAX) {
    set_error("%lld slots exceed int32 edge offsets", (long long)want);
    return DFPR_EINVAL;
  }
  if (want + want / 8 > g->cap) DFPR_TRY(grow_capacity(g, want, s));  // room for insertions, as at create
  // the general rebuild packs every row entry, pads included, into a batch
  // key with id_bits per column: the pad id n must fit, or its key would read
  // as the first key of the next row
  if (slack > 0) g->id_bits = std::max(g->id_bits, bits_for((int64_t)n + 1));
  const unsigned gr = grid_for(want, kRelayTile, 65536);
  DFPR_TRY(scan_generic(LoadPadded{g->out_deg, slack}, StoreOff{g->out2.off}, n, g->scan_tmp, s));
  k_relayout<<<gr, 256, 0, s>>>(g->out.off, g->out.idx, g->out_deg, g->out2.off, g->out2.idx, n, want, n, nullptr);
  DFPR_TRY(scan_generic(LoadPadded{g->in_deg, slack}, StoreOff{g->in2.off}, n, g->scan_tmp, s));
  k_relayout<<<gr, 256, 0, s>>>(g->in.off, g->in.idx, g->in_deg, g->in2.off, g->in2.idx, n, want, n, nullptr);
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipStreamSynchronize(s));
  std::swap(g->out, g->out2);
  std::swap(g->in, g->in2);
  g->slots = want;
  g->slack = slack;
  g->all_bins_valid = false;
  g->csr_version++;
  return DFPR_OK;
}

int graph_apply(dfpr_graph* g, int64_t nd, const int32_t* del_src, const int32_t* del_dst, int64_t ni,
                const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where, hipStream_t s,
                dfpr_batch_info* info) {
  const int64_t nk = nd + ni;
  const int32_t n = g->n;
  const int b = g->id_bits;
  if (info) {
    *info = dfpr_batch_info{};
    info->ins_in = ni;
    info->del_in = nd;
    info->m_after = g->m;
  }
  if (nk == 0) return DFPR_OK;
  const int64_t need = slots_bound(g, ni);
  if (need > INT32_MAX) {
    set_error("batch would exceed int32 edge offsets");
    return DFPR_EINVAL;
  }
  if (need > g->cap) DFPR_TRY(grow_capacity(g, need, s));

  // ---- scratch
  DFPR_TRY(g->keys_a.ensure(nk * sizeof(uint64_t)));
  DFPR_TRY(g->keys_b.ensure(nk * sizeof(uint64_t)));
  DFPR_TRY(g->keys_c.ensure(nk * sizeof(uint64_t) + nk));  // in-order keys + keep bytes
  DFPR_TRY(g->sort_hist.ensure((radix_hist_elems(nk) + std::max(radix_scan_tmp_elems(nk), scan_tmp_elems(nk + 1))) *
                               sizeof(int64_t)));
  DFPR_TRY(g->eff_pre.ensure(3 * (nk + 1) * sizeof(int64_t)));  // deletion prefixes (out, in), opos
  uint64_t* ka = g->keys_a.as<uint64_t>();
  uint64_t* kb = g->keys_b.as<uint64_t>();
  uint64_t* kc = g->keys_c.as<uint64_t>();
  uint8_t* keep = reinterpret_cast<uint8_t*>(kc + nk);
  int64_t* hist = g->sort_hist.as<int64_t>();
  int64_t* tmp = hist + radix_hist_elems(nk);
  int64_t* pre_out = g->eff_pre.as<int64_t>();
  int64_t* pre_in = pre_out + (nk + 1);
  int64_t* opos = pre_in + (nk + 1);
  int64_t* counters = g->ctl->n_apply;

  const int32_t *ds = del_src, *dd = del_dst, *is = ins_src, *id = ins_dst;
  if (where == DFPR_HOST) {
    DFPR_TRY(g->batch_in.ensure(2 * nk * sizeof(int32_t)));
    int32_t* bi = g->batch_in.as<int32_t>();
    if (nd) {
      DFPR_HIP(hipMemcpyAsync(bi, del_src, nd * sizeof(int32_t), hipMemcpyHostToDevice, s));
      DFPR_HIP(hipMemcpyAsync(bi + nd, del_dst, nd * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    if (ni) {
      DFPR_HIP(hipMemcpyAsync(bi + 2 * nd, ins_src, ni * sizeof(int32_t), hipMemcpyHostToDevice, s));
      DFPR_HIP(hipMemcpyAsync(bi + 2 * nd + ni, ins_dst, ni * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    ds = bi;
    dd = bi + nd;
    is = bi + 2 * nd;
    id = bi + 2 * nd + ni;
  }

  EventPool& ep = g->pool;
  ep.reset(g->timing, s);
  size_t t_total, tok;
  DFPR_TRY(ep.start(&t_total));
  // ---- keys + validation.  An id out of range sets bit 0 of counters[4];
  // the classification then marks nothing, the rebuild targets are not
  // swapped in, and the error is reported after the one sync at the end, so
  // a rejected batch leaves the graph and its pending marks as they were.
  DFPR_HIP(hipMemsetAsync(counters, 0, 6 * sizeof(int64_t), s));
  k_make_batch_keys<<<grid_for(nk, 256, 65536), 256, 0, s>>>(ds, dd, nd, is, id, ni, n, b, g->perm, ka,
                                                              counters + 4);
  DFPR_HIP(hipGetLastError());

  // ---- sort by (u, v, tag) and classify against the old out-CSR
  DFPR_TRY(ep.start(&tok));
  DFPR_TRY(radix_sort(&ka, &kb, nk, 2 * b + 1, hist, tmp, s));
  DFPR_TRY(ep.stop(kTSort, tok));
  int64_t* g_self = g->ngraphs > 1 ? g->g_eff + 3 * (size_t)g->ngraphs : nullptr;
  if (g_self) DFPR_HIP(hipMemsetAsync(g_self, 0, (size_t)g->ngraphs * sizeof(int64_t), s));
  // few effective entries (at most one per 256 edges): the rebuild copies run
  // by run and needs no per-row deltas or touched flags
  const bool few = nk * 256 <= g->slots;
  k_classify<<<grid_for(nk, 256, 65536), 256, 0, s>>>(
      ka, nk, b, g->out.off, g->out.idx, keep, few ? nullptr : g->delta_out, few ? nullptr : g->delta_in,
      few ? nullptr : g->touched_out, few ? nullptr : g->touched_in, g->pend_src, g->flag_cur, counters, g->gidv,
      g_self, counters + 4);
  DFPR_HIP(hipGetLastError());
  // effective entries, sorted by (u, v): count lands in counters[3]
  DFPR_TRY(compact_keys(ka, keep, kb, nk, counters + 3, pre_out, tmp, s));
  uint64_t* eff_out = kb;
  const int64_t* cnt = counters + 3;
  if (g->ngraphs > 1) {
    DFPR_HIP(hipMemsetAsync(g->g_eff, 0, 2 * (size_t)g->ngraphs * sizeof(int64_t), s));
    k_member_eff<<<grid_for(nk, 256, 4096), 256, 0, s>>>(eff_out, cnt, b, g->gidv, g->g_eff);
  }
  DFPR_TRY(scan_generic(LoadIsDel{eff_out, cnt}, StoreI64b{pre_out}, nk, tmp, s));

  // ---- in-side entries: the same entries ordered by (v, u)
  k_in_order_keys<<<grid_for(nk, 256, 65536), 256, 0, s>>>(eff_out, cnt, nk, b, ka);
  uint64_t* eff_in = ka;
  uint64_t* alt = kc;
  DFPR_TRY(ep.start(&tok));
  // the entries arrive in (u, v) order and each pair is one entry, so a
  // stable sort on the v field alone gives (v, u) order
  DFPR_TRY(radix_sort(&eff_in, &alt, nk, 2 * b + 1, hist, tmp, s, b + 1));
  DFPR_TRY(ep.stop(kTSort, tok));
  DFPR_TRY(scan_generic(LoadIsDel{eff_in, cnt}, StoreI64b{pre_in}, nk, tmp, s));

  // Three ways to write the new CSRs:
  //   row-local (rows with free slots, few entries, every touched row has
  //     room): merge each touched row in place, offsets unchanged;
  //   re-laid out (rows with free slots, few entries, some row without room):
  //     every row moves to a new layout with fresh free slots, the touched
  //     rows merged on the way;
  //   rebuilt (otherwise): the run-by-run or group rebuild below, which
  //     carries free slots along as ordinary entries.
  enum { kRebuilt, kRowLocal, kRelaid } path = kRebuilt;
  const int64_t* h = g->ctl_host->n_apply;
  int64_t* nl = g->ctl->n_local;
  int64_t* heads_out = opos;  // the run-by-run rebuild's positions are not needed on these paths
  int64_t* heads_in = reinterpret_cast<int64_t*>(alt);  // free once the in-side sort is done
  int64_t* cpre_out = g->row_work.as<int64_t>();  // merge work-item prefixes (rows_out + 1, rows_in + 1)
  int64_t* cpre_in = cpre_out + (nk + 1);
  if (few && g->slack > 0) {
    DFPR_TRY(g->row_work.ensure(2 * (nk + 1) * sizeof(int64_t)));
    cpre_out = g->row_work.as<int64_t>();
    cpre_in = cpre_out + (nk + 1);
    DFPR_HIP(hipMemsetAsync(nl, 0, 3 * sizeof(int64_t), s));
    const unsigned gk = grid_for(nk, 256, 65536);
    k_local_rows<<<gk, 256, 0, s>>>(eff_out, cnt, pre_out, b, g->out.off, g->out_deg, heads_out, nl, nl + 2,
                                    g->touched_out);
    k_local_rows<<<gk, 256, 0, s>>>(eff_in, cnt, pre_in, b, g->in.off, g->in_deg, heads_in, nl + 1, nl + 2,
                                    g->touched_in);
    DFPR_HIP(hipGetLastError());
    DFPR_TRY(scan_generic(LoadRowChunks{heads_out, nl, eff_out, b, g->out_deg}, StoreI64b{cpre_out}, nk, tmp, s));
    DFPR_TRY(scan_generic(LoadRowChunks{heads_in, nl + 1, eff_in, b, g->in_deg}, StoreI64b{cpre_in}, nk, tmp, s));
    DFPR_HIP(hipMemcpyAsync(g->ctl_host->n_apply, counters, 6 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(g->ctl_host->n_local, nl, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(g->ctl_host->n_local + 3, cpre_out + nk, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipMemcpyAsync(g->ctl_host->n_local + 4, cpre_in + nk, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    DFPR_HIP(hipStreamSynchronize(s));
    if (h[4] & 1) {  // nothing was touched: a rejected batch has no effective entries
      set_error("vertex id outside [0, %d) in batch", n);
      return DFPR_ERANGE;
    }
    path = g->ctl_host->n_local[2] == 0 ? kRowLocal : kRelaid;
  }
  const int64_t rows_out = g->ctl_host->n_local[0], rows_in = g->ctl_host->n_local[1];
  const int32_t pad = n;
  const unsigned g_out = grid_for(g->ctl_host->n_local[3], 1, 16384);  // one workgroup per work item
  const unsigned g_in = grid_for(g->ctl_host->n_local[4], 1, 16384);
  if (path == kRowLocal) {
    // the old neighbours of the touched rows are saved to the idle rebuild
    // targets, then merged back into their rows
    DFPR_TRY(ep.start(&tok));
    k_row_save<<<g_out, 256, 0, s>>>(heads_out, nl, cpre_out, eff_out, cnt, pre_out, b, g->out_deg, g->out.off,
                                     g->out.idx, g->out2.idx);
    k_row_merge<<<g_out, 256, 0, s>>>(heads_out, nl, cpre_out, eff_out, cnt, pre_out, b, g->out_deg, 0, g->out.off,
                                      g->out2.idx, g->out.off, g->out.idx, pad);
    DFPR_TRY(ep.stop(kTRebuildOut, tok));
    DFPR_TRY(ep.start(&tok));
    k_row_save<<<g_in, 256, 0, s>>>(heads_in, nl + 1, cpre_in, eff_in, cnt, pre_in, b, g->in_deg, g->in.off,
                                    g->in.idx, g->in2.idx);
    k_row_merge<<<g_in, 256, 0, s>>>(heads_in, nl + 1, cpre_in, eff_in, cnt, pre_in, b, g->in_deg, 0, g->in.off,
                                     g->in2.idx, g->in.off, g->in.idx, pad);
    DFPR_TRY(ep.stop(kTRebuildIn, tok));
    k_update_degrees<<<grid_for(2 * nk, 256, 65536), 256, 0, s>>>(eff_out, eff_in, cnt, pre_out, pre_in, b,
                                                                    counters + 4, g->out_deg, g->in_deg);
  } else if (path == kRelaid) {
    // new degrees first: they size the new rows (untouched rows keep theirs)
    k_update_degrees<<<grid_for(2 * nk, 256, 65536), 256, 0, s>>>(eff_out, eff_in, cnt, pre_out, pre_in, b,
                                                                    counters + 4, g->out_deg, g->in_deg);
    const int64_t total = g->m + h[0] - h[1] + (int64_t)n * g->slack;
    const unsigned gr = grid_for(total, kRelayTile, 65536);
    DFPR_TRY(ep.start(&tok));
    DFPR_TRY(scan_generic(LoadPadded{g->out_deg, g->slack}, StoreOff{g->out2.off}, n, g->scan_tmp, s));
    k_relayout<<<gr, 256, 0, s>>>(g->out.off, g->out.idx, g->out_deg, g->out2.off, g->out2.idx, n, total, pad,
                                  g->touched_out);
    k_row_merge<<<g_out, 256, 0, s>>>(heads_out, nl, cpre_out, eff_out, cnt, pre_out, b, g->out_deg, 1, g->out.off,
                                      g->out.idx, g->out2.off, g->out2.idx, pad);
    DFPR_TRY(ep.stop(kTRebuildOut, tok));
    DFPR_TRY(ep.start(&tok));
    DFPR_TRY(scan_generic(LoadPadded{g->in_deg, g->slack}, StoreOff{g->in2.off}, n, g->scan_tmp, s));
    k_relayout<<<gr, 256, 0, s>>>(g->in.off, g->in.idx, g->in_deg, g->in2.off, g->in2.idx, n, total, pad,
                                  g->touched_in);
    k_row_merge<<<g_in, 256, 0, s>>>(heads_in, nl + 1, cpre_in, eff_in, cnt, pre_in, b, g->in_deg, 1, g->in.off,
                                     g->in.idx, g->in2.off, g->in2.idx, pad);
    DFPR_TRY(ep.stop(kTRebuildIn, tok));
    k_finish_apply<<<1, 1, 0, s>>>(g->out2.off, n, counters);
  } else {
    // ---- out-CSR (few effective entries: offsets shifted run by run, as the
    // index arrays are copied; otherwise a scan of the row-length deltas)
    const int32_t off_rows = run_offset_rows(n);
    const unsigned off_blocks = grid_for((int64_t)n + 1, off_rows, 65536);
    const unsigned pos_blocks = grid_for(nk, 256, 4096);
    if (few)
      k_run_offsets<<<off_blocks + pos_blocks, 256, 0, s>>>(g->out.off, g->out2.off, g->out.idx, opos, eff_out,
                                                            pre_out, cnt, b, n, off_rows, (int32_t)off_blocks);
    else
      DFPR_TRY(scan_row_offsets(g->out.off, g->delta_out, g->out2.off, n, g->scan_tmp, s));
    DFPR_TRY(ep.start(&tok));
    DFPR_TRY(rebuild_csr(g, g->out, g->out2, g->touched_out, eff_out, pre_out, opos, cnt, nk, ni, counters + 4,
                         nullptr, nullptr, s));
    DFPR_TRY(ep.stop(kTRebuildOut, tok));

    // ---- in-CSR
    if (few)
      k_run_offsets<<<off_blocks + pos_blocks, 256, 0, s>>>(g->in.off, g->in2.off, g->in.idx, opos, eff_in, pre_in,
                                                            cnt, b, n, off_rows, (int32_t)off_blocks);
    else
      DFPR_TRY(scan_row_offsets(g->in.off, g->delta_in, g->in2.off, n, g->scan_tmp, s));
    DFPR_TRY(ep.start(&tok));
    // (few entries: the in-side copy also records the new slot count)
    DFPR_TRY(rebuild_csr(g, g->in, g->in2, g->touched_in, eff_in, pre_in, opos, cnt, nk, ni, counters + 4,
                         g->out2.off, counters + 5, s));
    DFPR_TRY(ep.stop(kTRebuildIn, tok));
    if (!few) {
      k_clear_rows<<<grid_for(nk, 256, 65536), 256, 0, s>>>(eff_out, cnt, b, g->delta_out, g->delta_in,
                                                            g->touched_out, g->touched_in);
      k_finish_apply<<<1, 1, 0, s>>>(g->out2.off, n, counters);
    }
    k_update_degrees<<<grid_for(2 * nk, 256, 65536), 256, 0, s>>>(eff_out, eff_in, cnt, pre_out, pre_in, b,
                                                                    counters + 4, g->out_deg, g->in_deg);
  }
  if (path != kRebuilt) {
    k_clear_touched<<<grid_for(rows_out, 256, 4096), 256, 0, s>>>(heads_out, nl, eff_out, b, g->touched_out);
    k_clear_touched<<<grid_for(rows_in, 256, 4096), 256, 0, s>>>(heads_in, nl + 1, eff_in, b, g->touched_in);
  }
  DFPR_HIP(hipGetLastError());
  DFPR_HIP(hipMemcpyAsync(g->ctl_host->n_apply, counters, 6 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DFPR_TRY(ep.stop(kTTotal, t_total));
  DFPR_HIP(hipStreamSynchronize(s));

  if (h[4] & 1) {
    set_error("vertex id outside [0, %d) in batch", n);
    return DFPR_ERANGE;
  }
  const int64_t m_new = g->m + h[0] - h[1];
  // slot count of the new CSRs (row-local: unchanged; re-laid out: the new
  // degrees plus the free slots; rebuilt: the old count plus the net change)
  const int64_t slots_new = path == kRowLocal ? g->slots
                            : path == kRelaid ? m_new + (int64_t)n * g->slack
                                              : g->slots + h[0] - h[1];
  if (h[4] != 0 || (path != kRowLocal && h[5] != slots_new)) {
    set_error("internal inconsistency in the CSR rebuild (flag %lld, slots %lld -> %lld, expected %lld)",
              (long long)h[4], (long long)g->slots, (long long)h[5], (long long)slots_new);
    return DFPR_EHIP;
  }
  if (path != kRowLocal) {
    std::swap(g->out, g->out2);
    std::swap(g->in, g->in2);
  }
  g->m = m_new;
  g->slots = slots_new;
  g->all_bins_valid = false;
  g->csr_version++;
  if (h[3] > 0) g->pending_any = true;
  if (info) {
    info->ins_effective = h[0];
    info->del_effective = h[1];
    info->self_loop_dels_ignored = h[2];
    info->m_after = g->m;
    info->row_local = path == kRowLocal ? 1 : 0;
  }
  if (ep.on) {
    double ms[kTNum] = {0};
    int c[kTNum] = {0};
    DFPR_TRY(ep.collect(ms, c));
    if (info) {
      info->ms_total = ms[kTTotal];
      info->ms_sort = ms[kTSort];
      info->ms_rebuild[0] = ms[kTRebuildOut];
      info->ms_rebuild[1] = ms[kTRebuildIn];
    }
  }
  return DFPR_OK;
}

}  // namespace dfpr

namespace dfpr {

// ---- allocation-free apply.  The sort and staging buffers of one apply live
// in a fixed device array instead of the handle's growable buffers.  In host
// code `noalloc_scratch` names a host-side stand-in, never the device memory:
// its device address is looked up once per device (hipGetSymbolAddress with
// that device current) and only that address reaches kernels.  Every call on
// a device uses the same array; a per-device lock, held until the call's work
// has finished on its stream, serialises the calls of this process.
constexpr size_t kNoallocBytes = (size_t)40 << 20;
__device__ __align__(256) unsigned char noalloc_scratch[kNoallocBytes];

namespace {
constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu[kNoallocDevices];
void* g_noalloc_ptr[kNoallocDevices] = {};  // device address of noalloc_scratch per device
}  // namespace

int graph_apply_noalloc(dfpr_graph* g, int64_t nd, const int32_t* del_src, const int32_t* del_dst, int64_t ni,
                        const int32_t* ins_src, const int32_t* ins_dst, dfpr_where where, hipStream_t s,
                        dfpr_batch_info* info) {
  const int64_t nk = nd + ni;
  if (nk > DFPR_NOALLOC_MAX_PAIRS) {
    set_error("allocation-free apply: %lld batch pairs exceed the limit of %d", (long long)nk, DFPR_NOALLOC_MAX_PAIRS);
    return DFPR_EINVAL;
  }
  if (slots_bound(g, ni) > g->cap) {
    set_error("allocation-free apply: %lld insertions could exceed the edge capacity (%lld slots of %lld)",
              (long long)ni, (long long)g->slots, (long long)g->cap);
    return DFPR_ENOMEM;
  }
  const int dev = g->device;
  if (dev < 0 || dev >= kNoallocDevices) {
    set_error("allocation-free apply: device %d not supported", dev);
    return DFPR_EINVAL;
  }
  auto r = [](size_t x) { return (x + Heap::kAlign - 1) / Heap::kAlign * Heap::kAlign; };
  const size_t n8 = (size_t)nk * sizeof(uint64_t);
  const size_t b_keys_c = r(n8 + (size_t)nk);
  const size_t b_hist =
      r((radix_hist_elems(nk) + std::max(radix_scan_tmp_elems(nk), scan_tmp_elems(nk + 1))) * sizeof(int64_t));
  const size_t b_pre = r(3 * (size_t)(nk + 1) * sizeof(int64_t));
  const size_t b_in = where == DFPR_HOST ? r(2 * (size_t)nk * sizeof(int32_t)) : 0;
  const size_t b_work = g->slack > 0 ? r(2 * (size_t)(nk + 1) * sizeof(int64_t)) : 0;
  const size_t need = 2 * r(n8) + b_keys_c + b_hist + b_pre + b_in + b_work;
  if (need > kNoallocBytes) {
    set_error("allocation-free apply: %zu scratch bytes needed, %zu available", need, kNoallocBytes);
    return DFPR_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    DFPR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)));
    g_noalloc_ptr[dev] = ptr;
  }
  char* base = static_cast<char*>(g_noalloc_ptr[dev]);
  // views over the array, sized as the apply's ensure() calls ask, so none of
  // them allocates; the handle's own buffers are put back afterwards
  DevBuf* bufs[7] = {&g->keys_a, &g->keys_b, &g->keys_c, &g->sort_hist, &g->eff_pre, &g->batch_in, &g->row_work};
  const size_t sizes[7] = {r(n8), r(n8), b_keys_c, b_hist, b_pre, b_in, b_work};
  DevBuf saved[7];
  size_t off = 0;
  for (int i = 0; i < 7; i++) {
    saved[i] = *bufs[i];
    bufs[i]->p = sizes[i] ? base + off : nullptr;
    bufs[i]->bytes = sizes[i];
    bufs[i]->heap = nullptr;
    off += sizes[i];
  }
  const bool timing = g->timing;
  g->timing = false;  // no event creation on this path
  const int rc = graph_apply(g, nd, del_src, del_dst, ni, ins_src, ins_dst, where, s, info);
  (void)hipStreamSynchronize(s);  // the array is free for the next call only once this one's work is done
  g->timing = timing;
  for (int i = 0; i < 7; i++) *bufs[i] = saved[i];
  return rc;
}

// ---- batches of graphs: one disjoint union, member ids local to each member
int batch_create(int32_t count, const int32_t* n, const int64_t* m, const int32_t* const* src,
                 const int32_t* const* dst, dfpr_where where, int32_t flags, hipStream_t s, dfpr_graph** out) {
  std::vector<int64_t> vb(count + 1, 0);
  int64_t mt = 0;
  for (int32_t k = 0; k < count; k++) {
    vb[k + 1] = vb[k] + n[k];
    mt += m[k];
  }
  if (vb[count] > INT32_MAX || mt + vb[count] > INT32_MAX) {
    set_error("batch too large for int32 ids and offsets");
    return DFPR_EINVAL;
  }
  int32_t* coo = nullptr;
  int64_t* err = nullptr;
  int rc;
  if ((rc = dalloc(&coo, (size_t)(2 * mt))) || (rc = dalloc(&err, 1))) {
    dfree(coo);
    return rc;
  }
  DFPR_HIP(hipMemsetAsync(err, 0, sizeof(int64_t), s));
  // member arrays -> union arrays (device), ids shifted by the member base
  int32_t* tmp = nullptr;
  int64_t off = 0;
  for (int32_t k = 0; k < count && rc == DFPR_OK; k++) {
    if (m[k] == 0) continue;
    const int32_t *ps = src[k], *pd = dst[k];
    if (where == DFPR_HOST) {
      dfree(tmp);
      if ((rc = dalloc(&tmp, (size_t)(2 * m[k])))) break;
      if (hipMemcpyAsync(tmp, src[k], m[k] * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
          hipMemcpyAsync(tmp + m[k], dst[k], m[k] * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess) {
        rc = DFPR_EHIP;
        break;
      }
      ps = tmp;
      pd = tmp + m[k];
    }
    k_offset_ids<<<grid_for(m[k], 256, 65536), 256, 0, s>>>(ps, pd, m[k], n[k], vb[k], coo + off, coo + mt + off, err);
    if (where == DFPR_HOST && hipStreamSynchronize(s) != hipSuccess) rc = DFPR_EHIP;
    off += m[k];
  }
  int64_t herr = 0;
  if (rc == DFPR_OK && (hipMemcpyAsync(&herr, err, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
    rc = DFPR_EHIP;
  dfree(tmp);
  dfree(err);
  if (rc == DFPR_OK && herr) {
    set_error("vertex id outside its member graph");
    rc = DFPR_ERANGE;
  }
  if (rc == DFPR_OK)
    rc = graph_create((int32_t)vb[count], mt, coo, coo + mt, DFPR_DEVICE, 0, flags, s, out, &vb);
  if (rc == DFPR_OK) (*out)->fused_limit = kFusedBatchEdges;
  dfree(coo);
  return rc;
}

int batch_apply(dfpr_graph* g, const int64_t* n_del, const int32_t* const* del_src, const int32_t* const* del_dst,
                const int64_t* n_ins, const int32_t* const* ins_src, const int32_t* const* ins_dst, dfpr_where where,
                hipStream_t s, dfpr_batch_info* info) {
  const int32_t G = g->ngraphs;
  int64_t nd = 0, ni = 0;
  for (int32_t k = 0; k < G; k++) {
    nd += n_del[k];
    ni += n_ins[k];
  }
  const int64_t nk = nd + ni;
  DFPR_TRY(g->batch_in.ensure((size_t)(2 * nk + 2) * sizeof(int32_t) + 16));
  int32_t* bi = g->batch_in.as<int32_t>();
  int32_t *ds = bi, *dd = bi + nd, *is = bi + 2 * nd, *id = bi + 2 * nd + ni;
  int64_t* err = reinterpret_cast<int64_t*>(bi + 2 * nk + ((2 * nk) & 1));
  DFPR_HIP(hipMemsetAsync(err, 0, sizeof(int64_t), s));
  DevBuf stage;
  int64_t od = 0, oi = 0;
  for (int32_t k = 0; k < G; k++) {
    const int32_t nmem = (int32_t)(g->vbase[k + 1] - g->vbase[k]);
    for (int pass = 0; pass < 2; pass++) {
      const int64_t c = pass ? n_ins[k] : n_del[k];
      if (c == 0) continue;
      const int32_t* a = pass ? ins_src[k] : del_src[k];
      const int32_t* b = pass ? ins_dst[k] : del_dst[k];
      if (where == DFPR_HOST) {
        DFPR_TRY(stage.ensure((size_t)(2 * c) * sizeof(int32_t)));
        int32_t* st = stage.as<int32_t>();
        DFPR_HIP(hipMemcpyAsync(st, a, c * sizeof(int32_t), hipMemcpyHostToDevice, s));
        DFPR_HIP(hipMemcpyAsync(st + c, b, c * sizeof(int32_t), hipMemcpyHostToDevice, s));
        a = st;
        b = st + c;
      }
      int32_t* oa = pass ? is + oi : ds + od;
      int32_t* ob = pass ? id + oi : dd + od;
      k_offset_ids<<<grid_for(c, 256, 65536), 256, 0, s>>>(a, b, c, nmem, g->vbase[k], oa, ob, err);
      DFPR_HIP(hipGetLastError());
      if (where == DFPR_HOST) DFPR_HIP(hipStreamSynchronize(s));
      if (pass) oi += c; else od += c;
    }
  }
  int64_t herr = 0;
  DFPR_HIP(hipMemcpyAsync(&herr, err, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DFPR_HIP(hipStreamSynchronize(s));
  stage.release();
  if (herr) {
    set_error("vertex id outside its member graph in batch");
    return DFPR_ERANGE;
  }
  // the union ids live in batch_in; graph_apply reads DEVICE input in place
  // (and returns early on an empty batch: clear the per-member counts here)
  if (G > 1) DFPR_HIP(hipMemsetAsync(g->g_eff, 0, 4 * (size_t)G * sizeof(int64_t), s));
  dfpr_batch_info total{};
  DFPR_TRY(graph_apply(g, nd, ds, dd, ni, is, id, DFPR_DEVICE, s, &total));
  if (info) {
    // per member: effective counts (set by the apply), edges after, ignored self-loop deletions
    std::vector<int64_t> eff(4 * (size_t)G, 0);
    if (G > 1) {
      k_member_m<<<(unsigned)std::min<int64_t>(G, 1024), 256, 0, s>>>(g->out_deg, g->vbase_d, G, g->g_eff + 2 * (size_t)G);
      DFPR_HIP(hipGetLastError());
      DFPR_HIP(hipMemcpyAsync(eff.data(), g->g_eff, eff.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      DFPR_HIP(hipStreamSynchronize(s));
    } else {
      eff[0] = total.ins_effective;
      eff[1] = total.del_effective;
      eff[2] = total.m_after;
      eff[3] = total.self_loop_dels_ignored;
    }
    for (int32_t k = 0; k < G; k++) {
      info[k] = dfpr_batch_info{};
      info[k].ins_in = n_ins[k];
      info[k].del_in = n_del[k];
      info[k].ins_effective = eff[2 * k];
      info[k].del_effective = eff[2 * k + 1];
      info[k].m_after = eff[2 * (size_t)G + k];
      info[k].self_loop_dels_ignored = eff[3 * (size_t)G + k];
      info[k].ms_total = total.ms_total;  // timings are of the whole batch
      info[k].ms_sort = total.ms_sort;
      info[k].ms_rebuild[0] = total.ms_rebuild[0];
      info[k].ms_rebuild[1] = total.ms_rebuild[1];
      info[k].row_local = total.row_local;  // the arena's rows take one path together
    }
  }
  return DFPR_OK;
}

}  // namespace dfpr
