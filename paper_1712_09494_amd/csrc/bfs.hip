// Breadth-first state-space exploration on the GPU with the hash table as the
// visited set (the use the tables are built for: GPUexplore keeps its
// explored states in one, Sec. 3.2).  Each level: the successors of the
// frontier are generated on the device, find-or-put into the table as one
// batch, and the states reported new (in batch order) become the next
// frontier.
//
// Model: P = 16 processes with 16 local states each, packed 4 bits per
// process into one 64-bit word; each local state has up to 4 local
// transitions; 4 synchronising actions each move two processes p, q at once
// (at most one edge per local state for each).  Successor order of one state:
// for p = 0..15 each local target in list order, then for each synchronising
// action the (p-edge, q-edge) pair when both exist.
//
// Successors are written in two passes (count per state, exclusive scan of
// the counts, write at the scanned offsets), so each state's successors sit
// contiguously in frontier order.  Scan and flagged selection use hipCUB.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "runtime.h"

using namespace ht;
using namespace ht_rt;

namespace {

struct BfsModelDev {
  uint8_t lcnt[16][16];
  uint8_t ltgt[16][16][4];
  uint8_t sp[4], sq[4];
  int8_t pe[4][16], qe[4][16];   // -1: no edge
};

__device__ __forceinline__ uint32_t local_of(uint64_t st, uint32_t p) { return (uint32_t)(st >> (4 * p)) & 15u; }

__global__ __launch_bounds__(kBlock) void bfs_count_kernel(BfsModelDev m, const uint64_t* __restrict__ f, uint64_t nf,
                                                           unsigned long long* __restrict__ cnt) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nf; i += stride) {
    const uint64_t st = f[i];
    uint32_t c = 0;
#pragma unroll
    for (uint32_t p = 0; p < 16; ++p) c += m.lcnt[p][local_of(st, p)];
#pragma unroll
    for (uint32_t a = 0; a < 4; ++a)
      c += (m.pe[a][local_of(st, m.sp[a])] >= 0 && m.qe[a][local_of(st, m.sq[a])] >= 0) ? 1u : 0u;
    cnt[i] = c;
  }
}

__global__ __launch_bounds__(kBlock) void bfs_write_kernel(BfsModelDev m, const uint64_t* __restrict__ f, uint64_t nf,
                                                           const unsigned long long* __restrict__ off,
                                                           uint64_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nf; i += stride) {
    const uint64_t st = f[i];
    uint64_t o = off[i];
    for (uint32_t p = 0; p < 16; ++p) {
      const uint32_t s = local_of(st, p);
      const uint64_t cleared = st & ~(15ull << (4 * p));
      for (uint32_t k = 0; k < m.lcnt[p][s]; ++k) out[o++] = cleared | ((uint64_t)m.ltgt[p][s][k] << (4 * p));
    }
    for (uint32_t a = 0; a < 4; ++a) {
      const uint32_t p = m.sp[a], q = m.sq[a];
      const int tp = m.pe[a][local_of(st, p)], tq = m.qe[a][local_of(st, q)];
      if (tp >= 0 && tq >= 0) {
        const uint64_t cleared = st & ~(15ull << (4 * p)) & ~(15ull << (4 * q));
        out[o++] = cleared | ((uint64_t)tp << (4 * p)) | ((uint64_t)tq << (4 * q));
      }
    }
  }
}

// Device buffer that only grows.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return HT_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, need);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(HT_ENOMEM, "hipMalloc in breadth-first exploration failed");
    }
    bytes = need;
    return HT_OK;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

extern "C" int ht_bfs_explore(ht_table* t, const ht_bfs_model* model, uint64_t initial, uint32_t levels,
                              uint64_t* batch_sizes, uint64_t* new_counts, double* fop_ms, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!model) return fail(HT_EINVAL, "model is NULL");
  if (t->cfg.key_words > 1) return fail(HT_EINVAL, "the exploration packs states into single-word keys");
  BfsModelDev m;
  static_assert(sizeof(BfsModelDev) == sizeof(ht_bfs_model), "model layout");
  std::memcpy(&m, model, sizeof(m));
  for (int a = 0; a < 4; ++a)
    if (m.sp[a] > 15 || m.sq[a] > 15) return fail(HT_EINVAL, "synchronising action names a process above 15");
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q)
      if (m.lcnt[p][q] > 4) return fail(HT_EINVAL, "more than 4 local transitions");
  Buf frontier, next, batch, flags, counts, offsets, tmp, nsel;
  const uint32_t grid = max_blocks(t);
  rc = frontier.ensure(8);
  if (!rc) rc = nsel.ensure(16);
  if (rc) return rc;
  HT_HIP(hipMemcpyAsync(frontier.p, &initial, 8, hipMemcpyHostToDevice, s));
  rc = do_find_or_put(t, static_cast<uint64_t*>(frontier.p), 1, nullptr, s);
  if (rc) return rc;
  uint64_t nf = 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HT_HIP(hipEventCreate(&e0));
  HT_HIP(hipEventCreate(&e1));
  for (uint32_t L = 0; L < levels && nf; ++L) {
    rc = counts.ensure(nf * 8);
    if (!rc) rc = offsets.ensure(nf * 8);
    if (rc) break;
    auto* cnt = static_cast<unsigned long long*>(counts.p);
    auto* off = static_cast<unsigned long long*>(offsets.p);
    auto* fr = static_cast<const uint64_t*>(frontier.p);
    const uint32_t g1 = (uint32_t)std::min<uint64_t>((nf + kBlock - 1) / kBlock, grid);
    hipLaunchKernelGGL(bfs_count_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, cnt);
    HT_HIP(hipGetLastError());
    size_t tb = 0;
    HT_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)nf, s));
    rc = tmp.ensure(std::max<size_t>(tb, 256));
    if (rc) break;
    HT_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tb, cnt, off, (int)nf, s));
    unsigned long long last[2] = {0, 0};
    HT_HIP(hipMemcpyAsync(&last[0], off + nf - 1, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipMemcpyAsync(&last[1], cnt + nf - 1, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipStreamSynchronize(s));
    const uint64_t nb = last[0] + last[1];
    if (batch_sizes) batch_sizes[L] = nb;
    if (nb >= (1ull << 31)) {
      rc = fail(HT_EINVAL, "a level's batch exceeds 2^31 keys");
      break;
    }
    rc = batch.ensure(std::max<uint64_t>(nb, 1) * 8);
    if (!rc) rc = flags.ensure(std::max<uint64_t>(nb, 1));
    if (!rc) rc = next.ensure(std::max<uint64_t>(nb, 1) * 8);
    if (rc) break;
    auto* bt = static_cast<uint64_t*>(batch.p);
    hipLaunchKernelGGL(bfs_write_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, off, bt);
    HT_HIP(hipGetLastError());
    auto* fl = static_cast<uint8_t*>(flags.p);
    rc = reserve_scratch(t, nb);   // Cuckoo scratch for this batch, outside the timed region
    if (rc) break;
    HT_HIP(hipEventRecord(e0, s));
    rc = do_find_or_put(t, bt, nb, fl, s);
    if (rc) break;
    HT_HIP(hipEventRecord(e1, s));
    auto* ns = static_cast<unsigned long long*>(nsel.p);
    HT_HIP(hipcub::DeviceSelect::Flagged(nullptr, tb, bt, fl, static_cast<uint64_t*>(next.p), ns, (int)nb, s));
    rc = tmp.ensure(std::max<size_t>(tb, 256));
    if (rc) break;
    HT_HIP(hipcub::DeviceSelect::Flagged(tmp.p, tb, bt, fl, static_cast<uint64_t*>(next.p), ns, (int)nb, s));
    unsigned long long nnew = 0;
    HT_HIP(hipMemcpyAsync(&nnew, ns, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    HT_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (fop_ms) fop_ms[L] = ms;
    if (new_counts) new_counts[L] = nnew;
    std::swap(frontier.p, next.p);
    std::swap(frontier.bytes, next.bytes);
    nf = nnew;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  return rc;
}
