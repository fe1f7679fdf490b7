// Host launchers of the Cuckoo-table kernels (device code: cuckoo_dev.h).
#include "cuckoo_dev.h"

namespace ht {

// ---- host launchers --------------------------------------------------------

#define HT_R_DISPATCH(CALL)       \
  switch (R) {                    \
    case 1: CALL(1); break;       \
    case 2: CALL(2); break;       \
    case 4: CALL(4); break;       \
    default: return hipErrorInvalidValue; \
  }

hipError_t cuckoo_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid,
                        uint32_t R, bool scripted, hipStream_t st) {
  if (scripted) {
    hipLaunchKernelGGL((cuckoo_query_kernel<1, true>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out);
  } else {
#define HT_Q(RR) hipLaunchKernelGGL((cuckoo_query_kernel<RR, false>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out)
    HT_R_DISPATCH(HT_Q)
#undef HT_Q
  }
  return hipGetLastError();
}

// Kernel 1 of find-or-put: probe and place.
hipError_t cuckoo_probe(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                        const CuckooScratch& s, uint32_t grid, uint32_t R, bool scripted, bool paper_order,
                        hipStream_t st) {
  if (scripted && paper_order) {
    hipLaunchKernelGGL((cuckoo_probe_kernel<1, true, true>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out, s);
  } else if (scripted) {
    hipLaunchKernelGGL((cuckoo_probe_kernel<1, true, false>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out, s);
  } else if (paper_order) {
#define HT_P(RR) \
  hipLaunchKernelGGL((cuckoo_probe_kernel<RR, false, true>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out, s)
    HT_R_DISPATCH(HT_P)
#undef HT_P
  } else {
#define HT_P(RR) \
  hipLaunchKernelGGL((cuckoo_probe_kernel<RR, false, false>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out, s)
    HT_R_DISPATCH(HT_P)
#undef HT_P
  }
  return hipGetLastError();
}

// The paper's single-pass insertion (ablation; see cuckoo_dev.h).
hipError_t cuckoo_single_pass(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid,
                              bool scripted, hipStream_t st) {
  if (scripted)
    hipLaunchKernelGGL((cuckoo_single_pass_kernel<true>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out);
  else
    hipLaunchKernelGGL((cuckoo_single_pass_kernel<false>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out);
  return hipGetLastError();
}

// Kernel 2: deduplicate the listed keys and run their eviction chains.
// `grid`: the probe kernel's blocks; the evict kernel runs one wave per
// `pack` of its waves' regions.
hipError_t cuckoo_evict(const DevTable& t, uint64_t n, uint8_t* out, const CuckooScratch& s, uint32_t grid,
                        uint32_t pack, bool scripted, hipStream_t st) {
  if (pack < 1 || pack > kMaxPack) return hipErrorInvalidValue;
  const uint64_t nregions = (uint64_t)grid * (kBlock / kWave);
  const uint64_t waves = (nregions + pack - 1) / pack;
  const uint32_t g = (uint32_t)((waves + kBlock / kWave - 1) / (kBlock / kWave));
  const bool look = (t.flags & kFlagLookahead) != 0;
  if (scripted && look)
    hipLaunchKernelGGL((cuckoo_evict_kernel<true, true>), dim3(g), dim3(kBlock), t.lds, st, t, n, out, s, nregions,
                       pack);
  else if (scripted)
    hipLaunchKernelGGL((cuckoo_evict_kernel<true, false>), dim3(g), dim3(kBlock), t.lds, st, t, n, out, s, nregions,
                       pack);
  else if (look)
    hipLaunchKernelGGL((cuckoo_evict_kernel<false, true>), dim3(g), dim3(kBlock), t.lds, st, t, n, out, s, nregions,
                       pack);
  else
    hipLaunchKernelGGL((cuckoo_evict_kernel<false, false>), dim3(g), dim3(kBlock), t.lds, st, t, n, out, s, nregions,
                       pack);
  return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void cuckoo_scrub_kernel(uint64_t n, CuckooScratch s) {
  cuckoo_scrub_region(n, s, ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave);
}

// Kernel 3: clear the scratch-set slots kernel 2 took.
hipError_t cuckoo_scrub(uint64_t n, const CuckooScratch& s, uint32_t grid, hipStream_t st) {
  hipLaunchKernelGGL(cuckoo_scrub_kernel, dim3(grid), dim3(kBlock), 0, st, n, s);
  return hipGetLastError();
}

}  // namespace ht
