// Scan primitives shared by the graph and rank kernels (templated on the
// element producer and consumer so the scans fuse their load and store work).
#pragma once

#include "dfpr_impl.hpp"

namespace dfpr {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;  // 2048

// Block-wide exclusive scan of one int64 per thread; returns the exclusive
// prefix and writes the block total to *total (all threads).
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t x, int64_t* sh /*[kScanBlock/64 + 1]*/,
                                                        int64_t* total) {
  const int lane = lane_id();
  const int w = threadIdx.x / kWave;
  int64_t incl = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int64_t y = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += y;
  }
  if (lane == kWave - 1) sh[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
      int64_t t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[blockDim.x / kWave] = run;
  }
  __syncthreads();
  int64_t r = sh[w] + incl - x;
  *total = sh[blockDim.x / kWave];
  __syncthreads();
  return r;
}

template <class Load>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(Load ld, int64_t n, int64_t* block_sums) {
  __shared__ int64_t sh[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + j * kScanBlock + threadIdx.x;
    if (i < n) s += ld(i);
  }
  int64_t tot;
  block_exclusive_scan(s, sh, &tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// In-place exclusive scan of nb block sums by one block of 1024 threads;
// sums[nb] receives the grand total.
__global__ void __launch_bounds__(1024) k_scan_block_sums(int64_t* sums, int64_t nb);

template <class Load, class Store>
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(Load ld, Store st, int64_t n,
                                                           const int64_t* block_sums) {
  __shared__ int64_t tile[kScanTile];
  __shared__ int64_t sh[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + j * kScanBlock + threadIdx.x;
    tile[j * kScanBlock + threadIdx.x] = (i < n) ? ld(i) : 0;
  }
  __syncthreads();
  int64_t v[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    v[j] = run;
    run += tile[threadIdx.x * kScanItems + j];
  }
  int64_t tot;
  int64_t pre = block_exclusive_scan(run, sh, &tot) + block_sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanItems; j++) {
    int64_t i = base + threadIdx.x * kScanItems + j;
    if (i < n) st(i, pre + v[j]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st(n, block_sums[gridDim.x]);
}

template <class Store>
__global__ void k_scan_empty(Store st) { st(0, 0); }

// The whole scan in one workgroup of B threads (small batches, short bin
// tables): one launch instead of three.  With B = 1024 a tile holds 8192
// elements, so every input scan_generic sends here is one tile.
template <class Load, class Store, int B = kScanBlock>
__global__ void __launch_bounds__(B) k_scan_one_tile(Load ld, Store st, int64_t n) {
  constexpr int kTile = B * kScanItems;
  __shared__ int64_t tile[kTile];
  __shared__ int64_t sh[B / kWave + 1];
  int64_t carry = 0;  // total of the tiles before
  for (int64_t base = 0; base < n; base += kTile) {
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
      const int64_t i = base + j * B + threadIdx.x;
      tile[j * B + threadIdx.x] = (i < n) ? ld(i) : 0;
    }
    __syncthreads();
    int64_t v[kScanItems];
    int64_t run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
      v[j] = run;
      run += tile[threadIdx.x * kScanItems + j];
    }
    int64_t tot;
    const int64_t pre = block_exclusive_scan(run, sh, &tot);  // ends with a barrier: the tile is free again
#pragma unroll
    for (int j = 0; j < kScanItems; j++) {
      const int64_t i = base + threadIdx.x * kScanItems + j;
      if (i < n) st(i, carry + pre + v[j]);
    }
    carry += tot;
  }
  if (threadIdx.x == 0) st(n, carry);
}

// Exclusive scan of ld(0..n) into st(0..n) (st(n, total) included).  Up to
// kScanFewTiles tiles of 2048: one workgroup of 1024 threads (one launch
// instead of three).
constexpr int64_t kScanFewTiles = 4;
template <class Load, class Store>
int scan_generic(Load ld, Store st, int64_t n, int64_t* tmp, hipStream_t s) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 0) {  // empty input: only the total, 0
    k_scan_empty<<<1, 1, 0, s>>>(st);
    return hipGetLastError() == hipSuccess ? DFPR_OK : DFPR_EHIP;
  }
  if (nb <= kScanFewTiles) {
    k_scan_one_tile<Load, Store, 1024><<<1, 1024, 0, s>>>(ld, st, n);
    return hipGetLastError() == hipSuccess ? DFPR_OK : DFPR_EHIP;
  }
  k_scan_reduce<<<(unsigned)nb, kScanBlock, 0, s>>>(ld, n, tmp);
  k_scan_block_sums<<<1, 1024, 0, s>>>(tmp, nb);
  k_scan_apply<<<(unsigned)nb, kScanBlock, 0, s>>>(ld, st, n, tmp);
  return hipGetLastError() == hipSuccess ? DFPR_OK : DFPR_EHIP;
}

}  // namespace dfpr
