// Exclusive scan of 64-bit counts and order-preserving selection of flagged
// keys, for the breadth-first exploration's split levels (successor offsets
// per frontier state; the keys a find-or-put reported new, in batch order).
//
// Both run in three passes over `grid` blocks, block b owning one contiguous
// chunk of the input: (1) each block totals its chunk; (2) one block scans
// the totals; (3) each block walks its chunk in tiles of 256 items, a wave
// ranking its 64 items with a ballot (selection) or a shuffle scan (counts),
// the four waves of a tile combined through LDS, and writes each item at its
// block's offset plus the running tile offset.  The inputs are read twice and
// the outputs written once, all coalesced.
#include "ht_device.h"

namespace ht {

namespace {

constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ void chunk_of(uint64_t n, uint64_t& lo, uint64_t& hi) {
  const uint64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  lo = (uint64_t)blockIdx.x * chunk;
  hi = lo + chunk;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
}

// Sum of `v` over the block (every thread gets it).
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v, unsigned long long* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) lds[w] = v;
  __syncthreads();
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) s += lds[i];
  __syncthreads();
  return s;
}

// Inclusive prefix sum of `v` over the wave (64-bit values).
__device__ __forceinline__ unsigned long long wave_inclusive(unsigned long long v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const unsigned long long o = shfl64(v, lane >= off ? lane - off : lane);
    if (lane >= off) v += o;
  }
  return v;
}

// Pass 1 of the scan: per-block totals of the counts.
__global__ __launch_bounds__(kBlock) void scan_totals_kernel(const unsigned long long* __restrict__ in, uint64_t n,
                                                             unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long lds[kWavesPerBlock];
  uint64_t lo, hi;
  chunk_of(n, lo, hi);
  unsigned long long s = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) s += in[i];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) totals[blockIdx.x] = s;
}

// Pass 1 of the selection: per-block number of flagged items (flag != 0).
__global__ __launch_bounds__(kBlock) void select_totals_kernel(const uint8_t* __restrict__ flags, uint64_t n,
                                                               unsigned long long* __restrict__ totals) {
  __shared__ unsigned long long lds[kWavesPerBlock];
  uint64_t lo, hi;
  chunk_of(n, lo, hi);
  unsigned long long s = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) s += flags[i] != 0 ? 1u : 0u;
  s = block_sum(s, lds);
  if (threadIdx.x == 0) totals[blockIdx.x] = s;
}

// Pass 2: exclusive scan of the nb block totals in place by one block; the
// grand total goes to totals[nb] and, when given, to *grand.
__global__ __launch_bounds__(kBlock) void scan_block_totals_kernel(unsigned long long* __restrict__ totals,
                                                                   uint32_t nb, unsigned long long* grand) {
  __shared__ unsigned long long lds[kWavesPerBlock];
  const uint32_t per = (nb + kBlock - 1) / kBlock;     // consecutive totals per thread
  const uint32_t a = threadIdx.x * per;
  const uint32_t b = a + per < nb ? a + per : nb;
  unsigned long long mine = 0;
  for (uint32_t i = a; i < b; ++i) mine += totals[i];
  // exclusive prefix of `mine` over the block
  const unsigned long long incl = wave_inclusive(mine);
  const int w = threadIdx.x / kWave;
  if (lane_id() == kWave - 1) lds[w] = incl;
  __syncthreads();
  unsigned long long base = 0, all = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) {
    if (i < w) base += lds[i];
    all += lds[i];
  }
  unsigned long long run = base + incl - mine;
  for (uint32_t i = a; i < b; ++i) {
    const unsigned long long v = totals[i];
    totals[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) {
    totals[nb] = all;
    if (grand) *grand = all;
  }
}

// Pass 3 of the scan: out[i] = sum of in[0..i).
__global__ __launch_bounds__(kBlock) void scan_write_kernel(const unsigned long long* __restrict__ in, uint64_t n,
                                                            const unsigned long long* __restrict__ offs,
                                                            unsigned long long* __restrict__ out) {
  __shared__ unsigned long long lds[kWavesPerBlock];
  uint64_t lo, hi;
  chunk_of(n, lo, hi);
  unsigned long long run = offs[blockIdx.x];
  const int w = threadIdx.x / kWave;
  for (uint64_t t0 = lo; t0 < hi; t0 += kBlock) {
    const uint64_t i = t0 + threadIdx.x;
    const unsigned long long v = i < hi ? in[i] : 0;
    const unsigned long long incl = wave_inclusive(v);
    if (lane_id() == kWave - 1) lds[w] = incl;
    __syncthreads();
    unsigned long long base = 0, tile = 0;
#pragma unroll
    for (int q = 0; q < kWavesPerBlock; ++q) {
      if (q < w) base += lds[q];
      tile += lds[q];
    }
    if (i < hi) out[i] = run + base + incl - v;
    run += tile;
    __syncthreads();
  }
}

// Pass 3 of the selection: the flagged items of the block's chunk, in order,
// from its offset on.
__global__ __launch_bounds__(kBlock) void select_write_kernel(const uint64_t* __restrict__ in,
                                                              const uint8_t* __restrict__ flags, uint64_t n,
                                                              const unsigned long long* __restrict__ offs,
                                                              uint64_t* __restrict__ out) {
  __shared__ uint32_t lds[kWavesPerBlock];
  uint64_t lo, hi;
  chunk_of(n, lo, hi);
  unsigned long long run = offs[blockIdx.x];
  const int w = threadIdx.x / kWave;
  for (uint64_t t0 = lo; t0 < hi; t0 += kBlock) {
    const uint64_t i = t0 + threadIdx.x;
    const bool f = i < hi && flags[i] != 0;
    const uint64_t m = ballot(f);
    if (lane_id() == 0) lds[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t base = 0, tile = 0;
#pragma unroll
    for (int q = 0; q < kWavesPerBlock; ++q) {
      if (q < w) base += lds[q];
      tile += lds[q];
    }
    if (f) out[run + base + lanes_below(m)] = in[i];
    run += tile;
    __syncthreads();
  }
}

}  // namespace

// Exclusive scan of n counts: out[i] = in[0] + ... + in[i-1]; the total goes
// to *total (device).  `work` holds grid + 1 words.
hipError_t scan_exclusive(const unsigned long long* in, unsigned long long* out, uint64_t n,
                          unsigned long long* total, unsigned long long* work, uint32_t grid, hipStream_t s) {
  // n == 0 still runs the passes, so that *total is written (0)
  hipLaunchKernelGGL(scan_totals_kernel, dim3(grid), dim3(kBlock), 0, s, in, n, work);
  hipLaunchKernelGGL(scan_block_totals_kernel, dim3(1), dim3(kBlock), 0, s, work, grid, total);
  hipLaunchKernelGGL(scan_write_kernel, dim3(grid), dim3(kBlock), 0, s, in, n, work, out);
  return hipGetLastError();
}

// out = the in[i] with flags[i] != 0, in index order; their number goes to
// *count (device).  `work` holds grid + 1 words.
hipError_t select_flagged(const uint64_t* in, const uint8_t* flags, uint64_t n, uint64_t* out,
                          unsigned long long* count, unsigned long long* work, uint32_t grid, hipStream_t s) {
  // n == 0 still runs the passes, so that *count is written (0)
  hipLaunchKernelGGL(select_totals_kernel, dim3(grid), dim3(kBlock), 0, s, flags, n, work);
  hipLaunchKernelGGL(scan_block_totals_kernel, dim3(1), dim3(kBlock), 0, s, work, grid, count);
  hipLaunchKernelGGL(select_write_kernel, dim3(grid), dim3(kBlock), 0, s, in, flags, n, work, out);
  return hipGetLastError();
}

}  // namespace ht
