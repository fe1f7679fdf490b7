// Table maintenance kernels (fill, dump) and memory-system probe kernels used
// to measure the random-access roofline (streaming copy, random line gather,
// random 64-bit compare-and-swap).
#include "ht_device.h"

namespace ht {

// n words of value v from p: 16-byte stores over the 16-byte aligned pairs,
// 8-byte stores for a leading and a trailing odd word.
__global__ __launch_bounds__(kBlock) void fill_kernel(uint64_t* __restrict__ p, uint64_t n, uint64_t v) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint64_t first = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t head = (reinterpret_cast<uintptr_t>(p) & 15) ? 1 : 0;   // p is 8-byte aligned
  const uint64_t pairs = (n - (head < n ? head : n)) / 2;
  ulonglong2* q = reinterpret_cast<ulonglong2*>(p + head);
  const ulonglong2 vv = make_ulonglong2(v, v);
  for (uint64_t i = first; i < pairs; i += stride) q[i] = vv;
  if (first == 0) {
    if (head && n) p[0] = v;
    if (head + 2 * pairs < n) p[n - 1] = v;
  }
}

__global__ void zero_words_kernel(uint32_t* __restrict__ p, uint64_t nwords) {
  for (uint64_t i = threadIdx.x; i < nwords; i += blockDim.x) p[i] = 0u;
}

// Compact the non-empty words of src[0..n) into dst; *count is the running
// position (one atomic per wave).  Words past `cap` are counted, not written.
__global__ __launch_bounds__(kBlock) void compact_kernel(const uint64_t* __restrict__ src, uint64_t n,
                                                         uint64_t* __restrict__ dst, uint64_t cap,
                                                         unsigned long long* count) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const int lane = lane_id();
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); base < n; base += stride) {
    const uint64_t i = base + lane;
    const uint64_t v = i < n ? src[i] : kEmpty;
    const bool keep = v != kEmpty;
    const uint64_t m = ballot(keep);
    if (!m) continue;
    unsigned long long b = 0;
    if (lane == 0) b = add_agent(count, (unsigned long long)__popcll(m));
    b = shfl64(b, 0);
    if (keep) {
      const uint64_t pos = b + lanes_below(m);
      if (pos < cap) dst[pos] = v;
    }
  }
}

// A fill writes each 16-byte pair once with a thread per pair, up to 2^17
// blocks (then a few pairs per thread).  Clearing a 0.69 GB table: 0.110 ms
// (6.2 TB/s) against 0.164 ms for 8-byte stores from a persistent grid of 8
// blocks per compute unit, 0.130 ms for 8-byte stores from 2^17 blocks.
hipError_t fill_words(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t need = (n / 2 + kBlock - 1) / kBlock + 1;
  const uint32_t g = (uint32_t)(need < (1u << 17) ? need : (1u << 17));
  hipLaunchKernelGGL(fill_kernel, dim3(g), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t zero_words(uint32_t* p, uint64_t nwords, hipStream_t s) {
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(kBlock), 0, s, p, nwords);
  return hipGetLastError();
}

hipError_t compact_words(const uint64_t* src, uint64_t n, uint64_t* dst, uint64_t cap,
                         unsigned long long* count, uint32_t grid, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t need = (n + kBlock - 1) / kBlock;
  const uint32_t g = (uint32_t)(need < grid ? need : grid);
  hipLaunchKernelGGL(compact_kernel, dim3(g), dim3(kBlock), 0, s, src, n, dst, cap, count);
  return hipGetLastError();
}

// ---- probes ------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void probe_copy_kernel(const ulonglong2* __restrict__ src,
                                                            ulonglong2* __restrict__ dst, uint64_t n2) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += stride) dst[i] = src[i];
}

// Random gather: each access reads one aligned `LINE`-byte line, split over
// LINE/16 lanes (16 bytes each); a wave serves 64*16/LINE lines per step.
template <int LINE>
__global__ __launch_bounds__(kBlock) void probe_gather_kernel(const uint64_t* __restrict__ a, uint64_t nlines,
                                                              uint64_t naccess, uint64_t seed,
                                                              uint64_t* __restrict__ sink) {
  constexpr int LPL = LINE / 16;                  // lanes per line
  constexpr int PER_WAVE = kWave / LPL;
  const int lane = lane_id();
  const int sub = lane % LPL;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  uint64_t acc = 0;
  for (uint64_t base = wave * PER_WAVE; base < naccess; base += nwaves * PER_WAVE) {
    const uint64_t id = base + lane / LPL;
    if (id < naccess) {
      const uint64_t line = mulhi64(mix64(id ^ seed), nlines);
      const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(a + line * (LINE / 8) + 2 * sub);
      acc ^= v.x ^ v.y;
    }
  }
  if (acc == 0x5eed5eed5eed5eedull) sink[0] = acc;   // keeps the loads live
}

__global__ __launch_bounds__(kBlock) void probe_gather8_kernel(const uint64_t* __restrict__ a, uint64_t nwords,
                                                               uint64_t naccess, uint64_t seed,
                                                               uint64_t* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint64_t acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < naccess; i += stride)
    acc ^= a[mulhi64(mix64(i ^ seed), nwords)];
  if (acc == 0x5eed5eed5eed5eedull) sink[0] = acc;
}

__global__ __launch_bounds__(kBlock) void probe_cas_kernel(uint64_t* __restrict__ a, uint64_t nwords,
                                                           uint64_t naccess, uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < naccess; i += stride) {
    const uint64_t h = mix64(i ^ seed);
    cas64(&a[mulhi64(h, nwords)], kEmpty, h);
  }
}

// Mixed probe: the memory pattern of a find-or-put kernel without the table
// logic.  One lane per item: read the item's 8-byte key (coalesced), make
// `lines` random 8-byte reads (whole lines at the memory) at addresses mixed
// from the key, then with probability `cas` one random 64-bit
// compare-and-swap (empty -> key) whose address depends on the words read --
// in a line of its own, or (SAME_LINE) in the line of the first read, as a
// table kernel compare-and-swaps into the bucket or slot it has just read --
// and write a 1-byte flag (coalesced).  Fractional counts are met per item
// by a keyed draw: lines_q / 256 reads on average, cas_q / 256 CAS.
template <bool SAME_LINE>
__global__ __launch_bounds__(kBlock) void probe_mix_kernel(const uint64_t* __restrict__ keys,
                                                           uint8_t* __restrict__ out, uint64_t nitems,
                                                           uint64_t* __restrict__ a, uint64_t nwords,
                                                           uint32_t lines_q, uint32_t cas_q, uint64_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nitems; i += stride) {
    const uint64_t k = keys[i];
    const uint64_t r = mix64(k ^ seed ^ 0x243f6a8885a308d3ull);
    const uint32_t nl = (lines_q >> 8) + (((uint32_t)r & 255u) < (lines_q & 255u) ? 1u : 0u);
    uint64_t acc = 0, first = 0;
    for (uint32_t l = 0; l < nl; ++l) {
      const uint64_t w = mulhi64(mix64(k ^ seed ^ (0x9e3779b97f4a7c15ull * (l + 1))), nwords);
      if (l == 0) first = w;
      acc ^= a[w];
    }
    uint8_t f = (uint8_t)(acc & 1);
    if (((uint32_t)(r >> 8) & 255u) < cas_q) {
      uint64_t w;
      if (SAME_LINE && nl > 0) {
        // a word of the first line read, chosen after the read completes
        w = (first & ~15ull) + ((mix64(k ^ (acc & 0x100)) >> 60) & 15ull);
        if (w >= nwords) w = first;
      } else {
        w = mulhi64(mix64(k ^ seed ^ (acc & 0x100)), nwords);   // issued after the reads complete
      }
      f = cas64(&a[w], kEmpty, k) == kEmpty ? 1 : 0;
    }
    out[i] = f;
  }
}

hipError_t probe_mix(const uint64_t* keys, uint8_t* out, uint64_t nitems, uint64_t* a, uint64_t nwords,
                     uint32_t lines_q, uint32_t cas_q, bool same_line, uint64_t seed, uint32_t grid, hipStream_t s) {
  const uint64_t need = (nitems + kBlock - 1) / kBlock;
  const uint32_t g = (uint32_t)(need < grid ? need : grid);
  if (same_line)
    hipLaunchKernelGGL(probe_mix_kernel<true>, dim3(g), dim3(kBlock), 0, s, keys, out, nitems, a, nwords, lines_q,
                       cas_q, seed);
  else
    hipLaunchKernelGGL(probe_mix_kernel<false>, dim3(g), dim3(kBlock), 0, s, keys, out, nitems, a, nwords, lines_q,
                       cas_q, seed);
  return hipGetLastError();
}

hipError_t probe_copy(const uint64_t* src, uint64_t* dst, uint64_t n, uint32_t grid, hipStream_t s) {
  const uint64_t n2 = n / 2;
  hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(kBlock), 0, s,
                     reinterpret_cast<const ulonglong2*>(src), reinterpret_cast<ulonglong2*>(dst), n2);
  return hipGetLastError();
}

hipError_t probe_gather(const uint64_t* a, uint64_t nwords, uint64_t naccess, uint32_t line_bytes,
                        uint64_t seed, uint64_t* sink, uint32_t grid, hipStream_t s) {
  switch (line_bytes) {
    case 8:
      hipLaunchKernelGGL(probe_gather8_kernel, dim3(grid), dim3(kBlock), 0, s, a, nwords, naccess, seed, sink);
      break;
    case 64:
      hipLaunchKernelGGL((probe_gather_kernel<64>), dim3(grid), dim3(kBlock), 0, s, a, nwords / 8, naccess,
                         seed, sink);
      break;
    case 128:
      hipLaunchKernelGGL((probe_gather_kernel<128>), dim3(grid), dim3(kBlock), 0, s, a, nwords / 16, naccess,
                         seed, sink);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t probe_cas(uint64_t* a, uint64_t nwords, uint64_t naccess, uint64_t seed, uint32_t grid,
                     hipStream_t s) {
  hipLaunchKernelGGL(probe_cas_kernel, dim3(grid), dim3(kBlock), 0, s, a, nwords, naccess, seed);
  return hipGetLastError();
}

}  // namespace ht
