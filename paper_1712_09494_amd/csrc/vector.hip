// Host launchers of the state-vector kernels (device code: vector_dev.h).
#include "vector_dev.h"

namespace ht {

#define HT_W_DISPATCH(CALL)             \
  switch (W) {                          \
    case 2: CALL(2); break;             \
    case 4: CALL(4); break;             \
    default: return hipErrorInvalidValue; \
  }

hipError_t vec_evict(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, const CuckooScratch& s,
                      uint32_t grid, uint32_t W, hipStream_t st) {
#define HT_L(WW) hipLaunchKernelGGL((vec_evict_kernel<WW>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out, s)
  HT_W_DISPATCH(HT_L)
#undef HT_L
  return hipGetLastError();
}

hipError_t vec_find_or_claim(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                             const CuckooScratch& s, uint32_t grid, uint32_t W, hipStream_t st) {
#define HT_L(WW) \
  hipLaunchKernelGGL((vec_find_or_claim_kernel<WW>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out, s)
  HT_W_DISPATCH(HT_L)
#undef HT_L
  return hipGetLastError();
}

hipError_t vec_commit(const DevTable& t, const uint64_t* keys, uint64_t n, const CuckooScratch& s, uint32_t grid,
                      uint32_t W, hipStream_t st) {
#define HT_L(WW) hipLaunchKernelGGL((vec_commit_kernel<WW>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, s)
  HT_W_DISPATCH(HT_L)
#undef HT_L
  return hipGetLastError();
}

hipError_t vec_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t grid, uint32_t W,
                     hipStream_t st) {
#define HT_L(WW) hipLaunchKernelGGL((vec_query_kernel<WW>), dim3(grid), dim3(kBlock), t.lds, st, t, keys, n, out)
  HT_W_DISPATCH(HT_L)
#undef HT_L
  return hipGetLastError();
}

hipError_t vec_dump(const uint64_t* handles, uint64_t nh, const uint64_t* arena, uint64_t* dst, uint64_t cap,
                    unsigned long long* count, uint32_t grid, uint32_t W, hipStream_t st) {
  if (nh == 0) return hipSuccess;
  const uint64_t need = (nh + kBlock - 1) / kBlock;
  const uint32_t g = (uint32_t)(need < grid ? need : grid);
#define HT_L(WW) \
  hipLaunchKernelGGL((vec_dump_kernel<WW>), dim3(g), dim3(kBlock), 0, st, handles, nh, arena, dst, cap, count)
  HT_W_DISPATCH(HT_L)
#undef HT_L
  return hipGetLastError();
}

}  // namespace ht
