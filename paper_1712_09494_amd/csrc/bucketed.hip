// Host launchers of the bucketed-table kernels (device code: bucketed_dev.h).
#include "bucketed_dev.h"

namespace ht {

// ---- host launchers --------------------------------------------------------

// Find-or-put lane groups of B / 4 lanes, each lane holding four slots (two
// 16-byte loads).  Against two slots per lane (B / 2 lanes, one load), on the
// 2^20-key batches of a 2^26-key fill at LF 0.7: B = 8 3.47 against 3.86 ms,
// B = 16 3.64 against 4.80, B = 32 5.24 against 8.09, B = 64 8.75 against
// 14.1 (one key per group, 8 blocks per compute unit; the two-slot times at
// their best settings).
template <int B, int R>
static hipError_t launch_fop(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid,
                             bool coherent, bool scripted, hipStream_t s) {
  if (scripted)
    hipLaunchKernelGGL((bucketed_fop_kernel<B, 4, 1, true, true>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n,
                       out);
  else if (coherent)
    hipLaunchKernelGGL((bucketed_fop_kernel<B, 4, R, false, true>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n,
                       out);
  else
    hipLaunchKernelGGL((bucketed_fop_kernel<B, 4, R, false, false>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n,
                       out);
  return hipGetLastError();
}

template <int B, int R>
static hipError_t launch_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid,
                               bool scripted, hipStream_t s) {
  if (scripted)
    hipLaunchKernelGGL((bucketed_query_kernel<B, 1, true>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n, out);
  else
    hipLaunchKernelGGL((bucketed_query_kernel<B, R, false>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n, out);
  return hipGetLastError();
}

// Keys one wave serves per loop turn (lane groups of B / spl lanes).
uint64_t bucketed_keys_per_wave(uint32_t B, uint32_t R, uint32_t spl) { return (64 * spl / B) * R; }

#define HT_BUCKET_DISPATCH(CALL)                                   \
  switch (t.bucket_slots * 16 + R) {                               \
    case 8 * 16 + 1: return CALL(8, 1);                            \
    case 8 * 16 + 2: return CALL(8, 2);                            \
    case 8 * 16 + 4: return CALL(8, 4);                            \
    case 16 * 16 + 1: return CALL(16, 1);                          \
    case 16 * 16 + 2: return CALL(16, 2);                          \
    case 16 * 16 + 4: return CALL(16, 4);                          \
    case 32 * 16 + 1: return CALL(32, 1);                          \
    case 32 * 16 + 2: return CALL(32, 2);                          \
    case 32 * 16 + 4: return CALL(32, 4);                          \
    case 64 * 16 + 1: return CALL(64, 1);                          \
    case 64 * 16 + 2: return CALL(64, 2);                          \
    case 64 * 16 + 4: return CALL(64, 4);                          \
    default: return hipErrorInvalidValue;                          \
  }

hipError_t bucketed_find_or_put(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                                uint32_t grid, uint32_t R, bool coherent, bool scripted, hipStream_t s) {
#define HT_FOP(BB, RR) launch_fop<BB, RR>(t, keys, n, out, grid, coherent, scripted, s)
  HT_BUCKET_DISPATCH(HT_FOP)
#undef HT_FOP
}

hipError_t bucketed_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid,
                          uint32_t R, bool scripted, hipStream_t s) {
#define HT_QRY(BB, RR) launch_query<BB, RR>(t, keys, n, out, grid, scripted, s)
  HT_BUCKET_DISPATCH(HT_QRY)
#undef HT_QRY
}

// One lane per key (HT_FLAG_BUCKETED_ONE_LANE).
hipError_t bucketed_lane_find_or_put(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                                     uint32_t grid, bool scripted, hipStream_t s) {
  if (scripted)
    hipLaunchKernelGGL((bucketed_lane_fop_kernel<true>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n, out);
  else
    hipLaunchKernelGGL((bucketed_lane_fop_kernel<false>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n, out);
  return hipGetLastError();
}

hipError_t bucketed_lane_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid,
                               bool scripted, hipStream_t s) {
  if (scripted)
    hipLaunchKernelGGL((bucketed_lane_query_kernel<true>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n, out);
  else
    hipLaunchKernelGGL((bucketed_lane_query_kernel<false>), dim3(grid), dim3(kBlock), t.lds, s, t, keys, n, out);
  return hipGetLastError();
}

}  // namespace ht

