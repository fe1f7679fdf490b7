// Breadth-first state-space exploration on the GPU with the hash table as the
// visited set (the use the tables are built for: GPUexplore keeps its
// explored states in one, Sec. 3.2).  Each level: the successors of the
// frontier are generated on the device and find-or-put into the table, and
// the states reported new become the next frontier.
//
// Model: P = 16 processes with 16 local states each, packed 4 bits per
// process into one 64-bit word; each local state has up to 4 local
// transitions; 4 synchronising actions each move two processes p, q at once
// (at most one edge per local state for each).  Successor order of one state:
// for p = 0..15 each local target in list order, then for each synchronising
// action the (p-edge, q-edge) pair when both exist; at most 68 successors.
//
// Split levels (the batch interface of Sec. 5): successors are written in
// two passes (count per state, exclusive scan of the counts, write at the
// scanned offsets), so each state's successors sit contiguously in frontier
// order; the batch is find-or-put as one call and the keys flagged new are
// selected.  Scan and flagged selection use hipCUB.
//
// Fused levels (bucketed tables; successor generation and hash table access
// in one kernel, as GPUexplore does, Sec. 3.2 and 7): a lane takes a frontier
// state, generates its successors in registers in the same order, and
// find-or-puts each with the one-lane bucket probe, recording in a 68-bit
// mask which of them were new and counting them; after an exclusive scan of
// the counts a second pass regenerates the successors and writes the new ones
// at the scanned offsets.  The successor batch is never stored: a level moves
// the frontier, the masks and the new states instead of writing the batch,
// reading it for the find-or-put and again for the selection.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "bucketed_dev.h"
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

// Successors of `st` in model order; visit(succ) is called for each.
template <class F>
__device__ __forceinline__ void for_each_successor(const BfsModelDev& m, uint64_t st, F&& visit) {
  for (uint32_t p = 0; p < 16; ++p) {
    const uint32_t s = local_of(st, p);
    const uint64_t cleared = st & ~(15ull << (4 * p));
    for (uint32_t k = 0; k < m.lcnt[p][s]; ++k) visit(cleared | ((uint64_t)m.ltgt[p][s][k] << (4 * p)));
  }
  for (uint32_t a = 0; a < 4; ++a) {
    const uint32_t p = m.sp[a], q = m.sq[a];
    const int tp = m.pe[a][local_of(st, p)], tq = m.qe[a][local_of(st, q)];
    if (tp >= 0 && tq >= 0) {
      const uint64_t cleared = st & ~(15ull << (4 * p)) & ~(15ull << (4 * q));
      visit(cleared | ((uint64_t)tp << (4 * p)) | ((uint64_t)tq << (4 * q)));
    }
  }
}

// Split pass: every successor, written at the state's scanned offset.
__global__ __launch_bounds__(kBlock) void bfs_write_kernel(BfsModelDev m, const uint64_t* __restrict__ f, uint64_t nf,
                                                           const unsigned long long* __restrict__ off,
                                                           uint64_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nf; i += stride) {
    uint64_t o = off[i];
    for_each_successor(m, f[i], [&](uint64_t succ) { out[o++] = succ; });
  }
}

// Fused pass: find-or-put of every successor of the frontier; per state the
// mask of new successors (bit k = successor k; two words) and their count;
// the number of successors generated is added to *generated.
__global__ __launch_bounds__(kBlock) void bfs_fused_kernel(BfsModelDev m, DevTable t, const uint64_t* __restrict__ f,
                                                           uint64_t nf, unsigned long long* __restrict__ cnt,
                                                           uint64_t* __restrict__ mask,
                                                           unsigned long long* __restrict__ generated) {
  const uint64_t first = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  unsigned long long placed = 0, gen = 0;
  for (uint64_t i = first; i < nf; i += stride) {
    uint64_t m0 = 0, m1 = 0;
    uint32_t k = 0, nnew = 0;
    for_each_successor(m, f[i], [&](uint64_t succ) {
      const uint32_t r = lane_find_or_put<false>(t, succ);
      if (r) {                     // 1 = stored, 2 = kept on the overflow list: new either way
        if (k < 64) m0 |= 1ull << k;
        else m1 |= 1ull << (k - 64);
        ++nnew;
      }
      placed += r == 1;
      ++k;
    });
    cnt[i] = nnew;
    mask[2 * i] = m0;
    mask[2 * i + 1] = m1;
    gen += k;
  }
  wave_count(t.ctr->size, placed, (uint32_t)(first / kWave));
  const unsigned long long g = wave_sum(gen);
  if (lane_id() == 0 && g) add_agent(generated, g);
}

// Second fused pass: the successors marked new, written at the scanned offsets.
__global__ __launch_bounds__(kBlock) void bfs_fused_write_kernel(BfsModelDev m, const uint64_t* __restrict__ f,
                                                                 uint64_t nf, const uint64_t* __restrict__ mask,
                                                                 const unsigned long long* __restrict__ off,
                                                                 uint64_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < nf; i += stride) {
    const uint64_t m0 = mask[2 * i], m1 = mask[2 * i + 1];
    if (!(m0 | m1)) continue;
    uint64_t o = off[i];
    uint32_t k = 0;
    for_each_successor(m, f[i], [&](uint64_t succ) {
      if ((k < 64 ? (m0 >> k) : (m1 >> (k - 64))) & 1) out[o++] = succ;
      ++k;
    });
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

// Events of one exploration, destroyed on every return path.
struct Events {
  hipEvent_t e[6] = {};
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

}  // namespace

// Device time between two recorded events, in ms.
static double span_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? (double)ms : 0.0;
}

extern "C" int ht_bfs_explore_ex(ht_table* t, const ht_bfs_model* model, uint64_t initial, uint32_t levels,
                                 uint32_t mode, uint64_t* batch_sizes, uint64_t* new_counts, double* fop_ms,
                                 double* level_ms, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!model) return fail(HT_EINVAL, "model is NULL");
  if (t->cfg.key_words > 1) return fail(HT_EINVAL, "the exploration packs states into single-word keys");
  if (mode != HT_BFS_SPLIT && mode != HT_BFS_FUSED) return fail(HT_EINVAL, "unknown exploration mode");
  const bool fused = mode == HT_BFS_FUSED;
  if (fused && t->cfg.kind != HT_BUCKETED) return fail(HT_EINVAL, "fused levels need a bucketed table");
  if (fused && is_scripted(t)) return fail(HT_EINVAL, "fused levels do not take scripted-hash tables");
  BfsModelDev m;
  static_assert(sizeof(BfsModelDev) == sizeof(ht_bfs_model), "model layout");
  std::memcpy(&m, model, sizeof(m));
  for (int a = 0; a < 4; ++a)
    if (m.sp[a] > 15 || m.sq[a] > 15) return fail(HT_EINVAL, "synchronising action names a process above 15");
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q)
      if (m.lcnt[p][q] > 4) return fail(HT_EINVAL, "more than 4 local transitions");
  Buf frontier, next, batch, flags, counts, offsets, tmp, nsel, masks;
  const uint32_t grid = max_blocks(t);
  rc = frontier.ensure(8);
  if (!rc) rc = nsel.ensure(16);
  if (rc) return rc;
  HT_HIP(hipMemcpyAsync(frontier.p, &initial, 8, hipMemcpyHostToDevice, s));
  rc = do_find_or_put(t, static_cast<uint64_t*>(frontier.p), 1, nullptr, s);
  if (rc) return rc;
  const DevTable dt = launch_view(t);
  uint64_t nf = 1;
  // ev[0..1]: first span of a level; ev[2..3]: second span (a host round trip
  // between them reads sizes); ev[4]: end of the find-or-put (or fused pass);
  // ev[5]: start of the find-or-put
  Events evs;
  hipEvent_t* ev = evs.e;
  for (int i = 0; i < 6; ++i) HT_HIP(hipEventCreate(&ev[i]));
  for (uint32_t L = 0; L < levels && nf && rc == HT_OK; ++L) {
    rc = counts.ensure(nf * 8);
    if (!rc) rc = offsets.ensure(nf * 8);
    if (!rc && fused) rc = masks.ensure(nf * 16);
    if (rc) break;
    auto* cnt = static_cast<unsigned long long*>(counts.p);
    auto* off = static_cast<unsigned long long*>(offsets.p);
    auto* fr = static_cast<const uint64_t*>(frontier.p);
    auto* ns = static_cast<unsigned long long*>(nsel.p);
    const uint32_t g1 = (uint32_t)std::min<uint64_t>((nf + kBlock - 1) / kBlock, grid);
    size_t tb = 0;
    HT_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, off, (int)nf, s));
    rc = tmp.ensure(std::max<size_t>(tb, 256));
    if (rc) break;
    if (fused) HT_HIP(hipMemsetAsync(ns, 0, 8, s));
    HT_HIP(hipEventRecord(ev[0], s));
    if (fused) {
      hipLaunchKernelGGL(bfs_fused_kernel, dim3(g1), dim3(kBlock), 0, s, m, dt, fr, nf, cnt,
                         static_cast<uint64_t*>(masks.p), ns);
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[4], s));
    } else {
      hipLaunchKernelGGL(bfs_count_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, cnt);
      HT_HIP(hipGetLastError());
    }
    HT_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tb, cnt, off, (int)nf, s));
    HT_HIP(hipEventRecord(ev[1], s));
    unsigned long long last[3] = {0, 0, 0};
    HT_HIP(hipMemcpyAsync(&last[0], off + nf - 1, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipMemcpyAsync(&last[1], cnt + nf - 1, 8, hipMemcpyDeviceToHost, s));
    if (fused) HT_HIP(hipMemcpyAsync(&last[2], ns, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipStreamSynchronize(s));
    const uint64_t total = last[0] + last[1];   // split: successors; fused: new states
    const uint64_t nb = fused ? last[2] : total;
    if (batch_sizes) batch_sizes[L] = nb;
    if ((fused ? total : nb) >= (1ull << 31)) {   // the next scan counts in int
      rc = fail(HT_EINVAL, fused ? "a level's new states exceed 2^31" : "a level's batch exceeds 2^31 keys");
      break;
    }
    uint64_t nnew = 0;
    if (fused) {
      nnew = total;
      rc = next.ensure(std::max<uint64_t>(nnew, 1) * 8);
      if (rc) break;
      HT_HIP(hipEventRecord(ev[2], s));
      hipLaunchKernelGGL(bfs_fused_write_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf,
                         static_cast<const uint64_t*>(masks.p), off, static_cast<uint64_t*>(next.p));
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[3], s));
      HT_HIP(hipStreamSynchronize(s));
      if (fop_ms) fop_ms[L] = span_ms(ev[0], ev[4]);
    } else {
      rc = batch.ensure(std::max<uint64_t>(nb, 1) * 8);
      if (!rc) rc = flags.ensure(std::max<uint64_t>(nb, 1));
      if (!rc) rc = next.ensure(std::max<uint64_t>(nb, 1) * 8);
      if (!rc) rc = reserve_scratch(t, nb);   // Cuckoo scratch for this batch, outside the timed spans
      if (rc) break;
      auto* bt = static_cast<uint64_t*>(batch.p);
      auto* fl = static_cast<uint8_t*>(flags.p);
      size_t tbs = 0;
      HT_HIP(hipcub::DeviceSelect::Flagged(nullptr, tbs, bt, fl, static_cast<uint64_t*>(next.p), ns, (int)nb, s));
      rc = tmp.ensure(std::max<size_t>(tbs, 256));
      if (rc) break;
      HT_HIP(hipEventRecord(ev[2], s));
      hipLaunchKernelGGL(bfs_write_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, off, bt);
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[5], s));
      rc = do_find_or_put(t, bt, nb, fl, s);
      if (rc) break;
      HT_HIP(hipEventRecord(ev[4], s));
      HT_HIP(hipcub::DeviceSelect::Flagged(tmp.p, tbs, bt, fl, static_cast<uint64_t*>(next.p), ns, (int)nb, s));
      HT_HIP(hipEventRecord(ev[3], s));
      unsigned long long nsv = 0;
      HT_HIP(hipMemcpyAsync(&nsv, ns, 8, hipMemcpyDeviceToHost, s));
      HT_HIP(hipStreamSynchronize(s));
      nnew = nsv;
      if (fop_ms) fop_ms[L] = span_ms(ev[5], ev[4]);
    }
    if (level_ms) level_ms[L] = span_ms(ev[0], ev[1]) + span_ms(ev[2], ev[3]);
    if (new_counts) new_counts[L] = nnew;
    std::swap(frontier.p, next.p);
    std::swap(frontier.bytes, next.bytes);
    nf = nnew;
  }
  (void)hipStreamSynchronize(s);
  return rc;
}

extern "C" int ht_bfs_explore(ht_table* t, const ht_bfs_model* model, uint64_t initial, uint32_t levels,
                              uint64_t* batch_sizes, uint64_t* new_counts, double* fop_ms, hipStream_t s) {
  return ht_bfs_explore_ex(t, model, initial, levels, HT_BFS_SPLIT, batch_sizes, new_counts, fop_ms, nullptr, s);
}
