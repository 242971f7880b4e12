// Device-wide primitives: exclusive scans, LSD radix sort, stable compaction.
#include "prim.hpp"

namespace dfpr {

__global__ void __launch_bounds__(1024) k_scan_block_sums(int64_t* sums, int64_t nb) {
  __shared__ int64_t sh[1024 / kWave + 1];
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  int64_t local = 0;
  for (int64_t i = lo; i < hi; i++) local += sums[i];
  int64_t tot;
  int64_t run = block_exclusive_scan(local, sh, &tot);
  for (int64_t i = lo; i < hi; i++) {
    int64_t t = sums[i];
    sums[i] = run;
    run += t;
  }
  if (threadIdx.x == 0) sums[nb] = tot;
}

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 2; }

struct LoadI64 {
  const int64_t* a;
  __device__ int64_t operator()(int64_t i) const { return a[i]; }
};
struct StoreI64 {
  int64_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = v; }
};

int scan_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* tmp, hipStream_t s) {
  return scan_generic(LoadI64{in}, StoreI64{out}, n, tmp, s);
}

struct LoadRowLen {
  const int32_t* off;
  const int32_t* delta;
  __device__ int64_t operator()(int64_t u) const {
    return (int64_t)(off[u + 1] - off[u]) + (int64_t)delta[u];
  }
};
struct StoreI32 {
  int32_t* a;
  __device__ void operator()(int64_t i, int64_t v) const { a[i] = (int32_t)v; }
};

int scan_row_offsets(const int32_t* base_off, const int32_t* delta, int32_t* out, int32_t n,
                     int64_t* tmp, hipStream_t s) {
  return scan_generic(LoadRowLen{base_off, delta}, StoreI32{out}, n, tmp, s);
}

// ------------------------------------------------------------------ radix sort
// 8-bit digits, 256 threads per block, 16 keys per thread.  Keys of a tile
// are visited in rounds j = 0..15 where round j holds positions
// tile + j*256 + t, so (round, thread) order is input order and the ranking
// below is stable.
constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixBlock * kRadixItems;

// Stable rank of this thread's digit among the valid keys of the current
// round, offset by running[digit] (counts of earlier rounds); updates running.
__device__ __forceinline__ int block_rank_round(uint32_t digit, bool valid, int* wave_cnt, int* running) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; b++) {
    const bool bit = (digit >> b) & 1u;
    const uint64_t bal = __ballot(valid && bit);
    peers &= bit ? bal : ~bal;
  }
  const int rank_in_wave = __popcll(peers & ((1ull << lane) - 1ull));
  const int leader = __ffsll((long long)peers) - 1;
  if (valid && lane == leader) wave_cnt[w * 256 + digit] = __popcll(peers);
  __syncthreads();
  int pos = 0;
  if (valid) {
    int before = running[digit];
    for (int w2 = 0; w2 < w; w2++) before += wave_cnt[w2 * 256 + digit];
    pos = before + rank_in_wave;
  }
  __syncthreads();
  {
    const int d = threadIdx.x;  // kRadixBlock == 256 digits
    int tot = 0;
#pragma unroll
    for (int w2 = 0; w2 < kRadixBlock / kWave; w2++) {
      tot += wave_cnt[w2 * 256 + d];
      wave_cnt[w2 * 256 + d] = 0;
    }
    running[d] += tot;
  }
  __syncthreads();
  return pos;
}

__global__ void __launch_bounds__(kRadixBlock) k_radix_hist(const uint64_t* keys, int64_t n, int shift,
                                                            int64_t* hist, int64_t nb) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll 4
  for (int j = 0; j < kRadixItems; j++) {
    int64_t i = base + j * kRadixBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(kRadixBlock) k_radix_scatter(const uint64_t* keys, uint64_t* out, int64_t n,
                                                               int shift, const int64_t* offs, int64_t nb) {
  __shared__ int wave_cnt[(kRadixBlock / kWave) * 256];
  __shared__ int running[256];
  __shared__ int64_t gbase[256];
  for (int i = threadIdx.x; i < (kRadixBlock / kWave) * 256; i += kRadixBlock) wave_cnt[i] = 0;
  running[threadIdx.x] = 0;
  gbase[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int j = 0; j < kRadixItems; j++) {
    const int64_t i = base + j * kRadixBlock + threadIdx.x;
    const bool valid = i < n;
    const uint64_t k = valid ? keys[i] : 0;
    const uint32_t digit = (uint32_t)((k >> shift) & 255u);
    const int pos = block_rank_round(digit, valid, wave_cnt, running);
    if (valid) out[gbase[digit] + pos] = k;
  }
}

// Scatter for up to kFusedScanBlocks tiles: each block derives its digit
// offsets from the raw per-tile counts itself (thread d sums digit d over the
// tiles, then one block scan over the digits), so a pass needs no separate
// scan of the counts.
constexpr int64_t kFusedScanBlocks = 32;
__global__ void __launch_bounds__(kRadixBlock) k_radix_scatter_own(const uint64_t* keys, uint64_t* out, int64_t n,
                                                                   int shift, const int64_t* hist, int64_t nb) {
  __shared__ int wave_cnt[(kRadixBlock / kWave) * 256];
  __shared__ int running[256];
  __shared__ int64_t gbase[256];
  __shared__ int64_t scan_sh[kRadixBlock / kWave + 1];
  for (int i = threadIdx.x; i < (kRadixBlock / kWave) * 256; i += kRadixBlock) wave_cnt[i] = 0;
  running[threadIdx.x] = 0;
  {
    const int64_t* row = hist + (int64_t)threadIdx.x * nb;  // digit threadIdx.x over the tiles
    int64_t before = 0, total = 0;
    for (int64_t b = 0; b < nb; b++) {
      const int64_t c = row[b];
      if (b < blockIdx.x) before += c;
      total += c;
    }
    int64_t all;
    gbase[threadIdx.x] = block_exclusive_scan(total, scan_sh, &all) + before;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int j = 0; j < kRadixItems; j++) {
    const int64_t i = base + j * kRadixBlock + threadIdx.x;
    const bool valid = i < n;
    const uint64_t k = valid ? keys[i] : 0;
    const uint32_t digit = (uint32_t)((k >> shift) & 255u);
    const int pos = block_rank_round(digit, valid, wave_cnt, running);
    if (valid) out[gbase[digit] + pos] = k;
  }
}

// Whole sort inside one block for n <= kSmallSort keys.
constexpr int kSmallSort = 2048;
__global__ void __launch_bounds__(kRadixBlock) k_radix_small(uint64_t* keys, int64_t n, int lo_bit, int bits) {
  __shared__ uint64_t buf[2][kSmallSort];
  __shared__ int wave_cnt[(kRadixBlock / kWave) * 256];
  __shared__ int running[256];
  __shared__ int cnt[256];
  __shared__ int64_t scan_sh[kRadixBlock / kWave + 1];
  for (int i = threadIdx.x; i < kSmallSort; i += kRadixBlock) buf[0][i] = (i < n) ? keys[i] : 0;
  for (int i = threadIdx.x; i < (kRadixBlock / kWave) * 256; i += kRadixBlock) wave_cnt[i] = 0;
  const int rounds = (int)((n + kRadixBlock - 1) / kRadixBlock);  // only the rounds that hold keys
  int src = 0;
  for (int shift = lo_bit; shift < bits; shift += 8) {
    cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kRadixBlock) atomicAdd(&cnt[(buf[src][i] >> shift) & 255u], 1);
    __syncthreads();
    int64_t tot;
    running[threadIdx.x] = (int)block_exclusive_scan(cnt[threadIdx.x], scan_sh, &tot);  // one digit per thread
    __syncthreads();
    for (int j = 0; j < rounds; j++) {
      const int i = j * kRadixBlock + threadIdx.x;
      const bool valid = i < n;
      const uint64_t k = buf[src][i];
      const uint32_t digit = (uint32_t)((k >> shift) & 255u);
      const int pos = block_rank_round(digit, valid, wave_cnt, running);
      if (valid) buf[src ^ 1][pos] = k;
    }
    __syncthreads();
    src ^= 1;
  }
  for (int i = threadIdx.x; i < n; i += kRadixBlock) keys[i] = buf[src][i];
}

size_t radix_hist_elems(int64_t n) {
  int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  return (size_t)(256 * nb + 1);
}
size_t radix_scan_tmp_elems(int64_t n) { return scan_tmp_elems((int64_t)radix_hist_elems(n)); }

int radix_sort(uint64_t** keys, uint64_t** alt, int64_t n, int bits, int64_t* hist, int64_t* scan_tmp,
               hipStream_t s, int lo_bit) {
  if (n <= 1) return DFPR_OK;
  if (n <= kSmallSort) {
    k_radix_small<<<1, kRadixBlock, 0, s>>>(*keys, n, lo_bit, bits);
    return hipGetLastError() == hipSuccess ? DFPR_OK : DFPR_EHIP;
  }
  const int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  for (int shift = lo_bit; shift < bits; shift += 8) {
    k_radix_hist<<<(unsigned)nb, kRadixBlock, 0, s>>>(*keys, n, shift, hist, nb);
    if (nb <= kFusedScanBlocks) {
      k_radix_scatter_own<<<(unsigned)nb, kRadixBlock, 0, s>>>(*keys, *alt, n, shift, hist, nb);
    } else {
      DFPR_TRY(scan_i64(hist, hist, 256 * nb, scan_tmp, s));
      k_radix_scatter<<<(unsigned)nb, kRadixBlock, 0, s>>>(*keys, *alt, n, shift, hist, nb);
    }
    uint64_t* t = *keys;
    *keys = *alt;
    *alt = t;
  }
  return hipGetLastError() == hipSuccess ? DFPR_OK : DFPR_EHIP;
}

// ------------------------------------------------------------------ compaction
struct LoadKeep {
  const uint8_t* keep;
  __device__ int64_t operator()(int64_t i) const { return keep[i] ? 1 : 0; }
};

__global__ void k_compact_scatter(const uint64_t* in, const uint8_t* keep, const int64_t* pre, uint64_t* out,
                                  int64_t n, int64_t* count_dev) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (keep[i]) out[pre[i]] = in[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) *count_dev = pre[n];
}

int compact_keys(const uint64_t* in, const uint8_t* keep, uint64_t* out, int64_t n, int64_t* count_dev,
                 int64_t* tmp_pre, int64_t* tmp, hipStream_t s) {
  DFPR_TRY(scan_generic(LoadKeep{keep}, StoreI64{tmp_pre}, n, tmp, s));
  k_compact_scatter<<<grid_for(n, 256, 65536), 256, 0, s>>>(in, keep, tmp_pre, out, n, count_dev);
  return hipGetLastError() == hipSuccess ? DFPR_OK : DFPR_EHIP;
}

}  // namespace dfpr
