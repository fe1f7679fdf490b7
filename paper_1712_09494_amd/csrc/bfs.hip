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
// selected in batch order.  Scan and selection are the three-pass kernels of
// compact.hip.
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
#include <algorithm>
#include <cstring>
#include <vector>

#include "bucketed_dev.h"
#include "cuckoo_dev.h"
#include "runtime.h"

namespace ht {
hipError_t zero_words(uint32_t*, uint64_t, hipStream_t);
hipError_t scan_exclusive(const unsigned long long*, unsigned long long*, uint64_t, unsigned long long*,
                          unsigned long long*, uint32_t, hipStream_t);
hipError_t select_flagged(const uint64_t*, const uint8_t*, uint64_t, uint64_t*, unsigned long long*,
                          unsigned long long*, uint32_t, hipStream_t);
}  // namespace ht

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

// Writing a level's successors (all of them, or those a mask marks) at the
// states' scanned offsets, staged through LDS so that the stores coalesce:
// a block takes a tile of kBlock consecutive states, whose outputs form one
// contiguous range; each thread places its state's successors that fall in
// the current window of kWriteWin positions, then the block copies the
// window out in consecutive words.  A thread per state storing its own
// successors one after another wrote 8-byte words to 64 unrelated places per
// instruction: 7.7 ms for the 5.7 GB batch of the 7-level workload's last
// level.
constexpr uint32_t kWriteWin = 2048;

template <bool MASKED>
__device__ __forceinline__ void write_tiles(const BfsModelDev& m, const uint64_t* __restrict__ f, uint64_t nf,
                                            const unsigned long long* __restrict__ cnt,
                                            const unsigned long long* __restrict__ off,
                                            const uint64_t* __restrict__ mask, uint64_t* __restrict__ out) {
  __shared__ uint64_t win[kWriteWin];
  const uint32_t tid = threadIdx.x;
  for (uint64_t i0 = (uint64_t)blockIdx.x * kBlock; i0 < nf; i0 += (uint64_t)gridDim.x * kBlock) {
    const uint64_t last = (i0 + kBlock < nf ? i0 + kBlock : nf) - 1;
    const uint64_t base = off[i0];
    const uint64_t end = off[last] + cnt[last];
    const uint64_t i = i0 + tid;
    const bool live = i < nf;
    const uint64_t st = live ? f[i] : 0ull;
    const uint64_t mine = live ? off[i] : 0ull;
    const uint64_t myend = live ? mine + cnt[i] : 0ull;
    const uint64_t m0 = MASKED && live ? mask[2 * i] : ~0ull;
    const uint64_t m1 = MASKED && live ? mask[2 * i + 1] : ~0ull;
    for (uint64_t w = base; w < end; w += kWriteWin) {
      if (live && mine < w + kWriteWin && myend > w) {
        uint64_t o = mine;
        uint32_t k = 0;
        for_each_successor(m, st, [&](uint64_t succ) {
          const bool take = !MASKED || (((k < 64 ? (m0 >> k) : (m1 >> (k - 64))) & 1ull) != 0);
          ++k;
          if (take) {
            if (o >= w && o < w + kWriteWin) win[o - w] = succ;
            ++o;
          }
        });
      }
      __syncthreads();
      const uint64_t nw = end - w < kWriteWin ? end - w : kWriteWin;
      for (uint32_t j = tid; j < nw; j += kBlock) out[w + j] = win[j];
      __syncthreads();
    }
  }
}

// Split pass: every successor, written at the state's scanned offset (cnt:
// successors per state, off: their exclusive scan).
__global__ __launch_bounds__(kBlock) void bfs_write_kernel(BfsModelDev m, const uint64_t* __restrict__ f, uint64_t nf,
                                                           const unsigned long long* __restrict__ cnt,
                                                           const unsigned long long* __restrict__ off,
                                                           uint64_t* __restrict__ out) {
  write_tiles<false>(m, f, nf, cnt, off, nullptr, out);
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

// Second fused pass: the successors marked new, written at the scanned
// offsets (cnt: new successors per state, off: their exclusive scan).
__global__ __launch_bounds__(kBlock) void bfs_fused_write_kernel(BfsModelDev m, const uint64_t* __restrict__ f,
                                                                 uint64_t nf, const uint64_t* __restrict__ mask,
                                                                 const unsigned long long* __restrict__ cnt,
                                                                 const unsigned long long* __restrict__ off,
                                                                 uint64_t* __restrict__ out) {
  write_tiles<true>(m, f, nf, cnt, off, mask, out);
}

// Successors of one state, one per call, in model order (the same order as
// for_each_successor); lets a wave step through its lanes' successors
// together, so wave-wide votes stay converged.
struct SuccIter {
  uint64_t st;
  uint32_t p = 0, kk = 0, a = 0;
  __device__ __forceinline__ bool next(const BfsModelDev& m, uint64_t& succ) {
    while (p < 16) {
      const uint32_t s = local_of(st, p);
      if (kk < m.lcnt[p][s]) {
        succ = (st & ~(15ull << (4 * p))) | ((uint64_t)m.ltgt[p][s][kk] << (4 * p));
        ++kk;
        return true;
      }
      ++p;
      kk = 0;
    }
    while (a < 4) {
      const uint32_t pp = m.sp[a], q = m.sq[a];
      const int tp = m.pe[a][local_of(st, pp)], tq = m.qe[a][local_of(st, q)];
      ++a;
      if (tp >= 0 && tq >= 0) {
        succ = (st & ~(15ull << (4 * pp)) & ~(15ull << (4 * q))) | ((uint64_t)tp << (4 * pp)) |
               ((uint64_t)tq << (4 * q));
        return true;
      }
    }
    return false;
  }
};

constexpr uint32_t kListed = 2;   // every candidate taken: listed for the evict pass

// Probe and place of one key per lane (called by every lane of the wave; act
// false for lanes without a key), as the single-table Cuckoo probe kernel
// does it: h_1, h_2, ... are read in turn, the key found ends the search, an
// empty candidate is compare-and-swapped at once (keys whose slot indices
// coincide read all c first and then try the empty ones in order).  Returns
// 1 placed, 0 found (or another copy placed it), kListed when every candidate
// is taken.
__device__ __forceinline__ uint32_t cuckoo_probe_key(const DevTable& t, uint64_t k, bool act, uint32_t sc,
                                                     uint32_t oc) {
  uint32_t res = 0;
  bool pend = act && k != kEmpty;
  if (act && k == kEmpty) res = sentinel_put(t);
  if (pend && (sc | oc) && stash_query(t, k, sc, oc)) pend = false;
  const bool dist = pend && hashes_distinct<false>(t, k);
  uint32_t em = 0;
  for (uint32_t j = 0; j < t.nhash && ballot(pend); ++j) {
    uint64_t idx = 0, v = 0;
    if (pend) {
      idx = hidx<false>(t, k, j);
      v = t.slots[idx];
    }
    bool cas = false;
    if (pend) {
      if (v == k) pend = false;
      else if (v == kEmpty) {
        if (dist) cas = true;
        else em |= 1u << j;
      }
    }
    if (cas) {
      const uint64_t old = cas64(&t.slots[idx], kEmpty, k);
      if (old == kEmpty) res = 1;
      if (old == kEmpty || old == k) pend = false;
    }
  }
  while (ballot(pend && em)) {
    if (pend && em) {
      const uint32_t j = (uint32_t)__builtin_ctz(em);
      em &= em - 1;
      const uint64_t old = cas64(&t.slots[hidx<false>(t, k, j)], kEmpty, k);
      if (old == kEmpty) res = 1;
      if (old == kEmpty || old == k) pend = false;
    }
  }
  return pend ? kListed : res;
}

// Fused Cuckoo pass 1: a wave takes groups of 64 frontier states, one per
// lane, and steps through their successors together; each successor is probed
// and placed as above, new ones marked in the state's mask and counted, and
// those with every candidate taken listed as (key, state << 7 | successor
// number) in the group's region of the scratch list, which starts at the
// group's first successor offset (a group never lists more keys than it has
// successors).
__global__ __launch_bounds__(kBlock) void bfs_cuckoo_probe_kernel(BfsModelDev m, DevTable t,
                                                                  const uint64_t* __restrict__ f, uint64_t nf,
                                                                  const unsigned long long* __restrict__ soff,
                                                                  CuckooScratch s, uint32_t* __restrict__ gcnt,
                                                                  unsigned long long* __restrict__ cnt,
                                                                  uint64_t* __restrict__ mask) {
  const int lane = lane_id();
  const uint64_t wave =
      __builtin_amdgcn_readfirstlane((uint32_t)(((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave));
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  const uint64_t ngroups = (nf + kWave - 1) / kWave;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  unsigned long long placed = 0;
  for (uint64_t g = wave; g < ngroups; g += nwaves) {
    const uint64_t i = g * kWave + lane;
    const bool live = i < nf;
    SuccIter it{live ? f[i] : 0ull};
    const uint64_t begin = soff[g * kWave];
    uint64_t m0 = 0, m1 = 0;
    uint32_t k = 0, nnew = 0, nlist = 0;
    for (;;) {
      uint64_t succ = 0;
      const bool has = live && it.next(m, succ);
      if (!ballot(has)) break;
      const uint32_t r = cuckoo_probe_key(t, succ, has, sc, oc);
      if (has && r == 1) {
        if (k < 64) m0 |= 1ull << k;
        else m1 |= 1ull << (k - 64);
        ++nnew;
        ++placed;
      }
      const bool l = has && r == kListed;
      const uint64_t mm = ballot(l);
      if (l) {
        const uint64_t slot = begin + nlist + lanes_below(mm);
        s.wkey[slot] = succ;
        s.wmeta[slot] = (i << 7) | k;
      }
      nlist += (uint32_t)__popcll(mm);
      k += has ? 1u : 0u;
    }
    if (live) {
      cnt[i] = nnew;
      mask[2 * i] = m0;
      mask[2 * i + 1] = m1;
    }
    if (lane == 0) gcnt[g] = nlist;
  }
  wave_count(t.ctr->size, placed, (uint32_t)wave);
}

// Fused Cuckoo pass 2: the listed keys, deduplicated in the scratch set; each
// winner marks its successor new in the state's mask and count and runs the
// eviction chain from h_1 (then the stash), as the single-table evict kernel
// does.  The scratch-set slot a winner took replaces its list entry's meta.
__global__ __launch_bounds__(kBlock) void bfs_cuckoo_evict_kernel(DevTable t, uint64_t nf,
                                                                  const unsigned long long* __restrict__ soff,
                                                                  CuckooScratch s, const uint32_t* __restrict__ gcnt,
                                                                  unsigned long long* __restrict__ cnt,
                                                                  uint64_t* __restrict__ mask) {
  const int lane = lane_id();
  const uint64_t wave =
      __builtin_amdgcn_readfirstlane((uint32_t)(((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave));
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  const uint64_t ngroups = (nf + kWave - 1) / kWave;
  unsigned long long nnew = 0, nevict = 0;
  for (uint64_t g = wave; g < ngroups; g += nwaves) {
    const uint64_t begin = soff[g * kWave];
    const uint32_t c = gcnt[g];
    for (uint32_t e = lane; e < c; e += kWave) {
      const uint64_t k = s.wkey[begin + e];
      const uint64_t meta = s.wmeta[begin + e];
      uint64_t p = mix64(k ^ s.dset_seed) & s.dset_mask;
      bool winner = false;
      for (;;) {
        const uint64_t old = cas64(&s.dset[p], kEmpty, k);
        if (old == kEmpty) {
          winner = true;
          break;
        }
        if (old == k) break;
        p = (p + 1) & s.dset_mask;
      }
      s.wmeta[begin + e] = winner ? p : ~0ull;
      if (!winner) continue;
      const uint64_t i = meta >> 7;
      const uint32_t kb = (uint32_t)(meta & 127);
      __hip_atomic_fetch_or(&mask[2 * i + (kb >> 6)], 1ull << (kb & 63), __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&cnt[i], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      uint64_t y = k;
      uint32_t steps = 0;
      const uint64_t h1 = hidx<false>(t, y, 0);
      const bool placed = (t.flags & kFlagLookahead) ? cuckoo_chain<false, true>(t, y, h1, nevict, steps)
                                                      : cuckoo_chain<false, false>(t, y, h1, nevict, steps);
      if (!placed) stash_put(t, y);
      ++nnew;
    }
  }
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
  wave_count(t.ctr->evictions, nevict, (uint32_t)wave);
}

// Fused Cuckoo pass 3: empty the scratch-set slots the evict pass took.
__global__ __launch_bounds__(kBlock) void bfs_cuckoo_scrub_kernel(uint64_t nf,
                                                                  const unsigned long long* __restrict__ soff,
                                                                  CuckooScratch s, const uint32_t* __restrict__ gcnt) {
  const int lane = lane_id();
  const uint64_t wave =
      __builtin_amdgcn_readfirstlane((uint32_t)(((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave));
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  const uint64_t ngroups = (nf + kWave - 1) / kWave;
  for (uint64_t g = wave; g < ngroups; g += nwaves) {
    const uint64_t begin = soff[g * kWave];
    const uint32_t c = gcnt[g];
    for (uint32_t e = lane; e < c; e += kWave) {
      const uint64_t p = s.wmeta[begin + e];
      if (p != ~0ull) s.dset[p] = kEmpty;
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

// Events of one exploration, destroyed on every return path.
struct Events {
  hipEvent_t e[8] = {};
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
  const bool ck = fused && t->cfg.kind == HT_CUCKOO;   // fused Cuckoo levels: count and scan first
  if (fused && is_scripted(t)) return fail(HT_EINVAL, "fused levels do not take scripted-hash tables");
  BfsModelDev m;
  static_assert(sizeof(BfsModelDev) == sizeof(ht_bfs_model), "model layout");
  std::memcpy(&m, model, sizeof(m));
  for (int a = 0; a < 4; ++a)
    if (m.sp[a] > 15 || m.sq[a] > 15) return fail(HT_EINVAL, "synchronising action names a process above 15");
  for (int p = 0; p < 16; ++p)
    for (int q = 0; q < 16; ++q)
      if (m.lcnt[p][q] > 4) return fail(HT_EINVAL, "more than 4 local transitions");
  Buf frontier, next, batch, flags, counts, offsets, tmp, nsel, masks, gcounts, noffsets;
  const uint32_t grid = max_blocks(t);
  rc = frontier.ensure(8);
  if (!rc) rc = nsel.ensure(16);
  if (!rc) rc = tmp.ensure((grid + 1) * 8ull);   // block totals of the scans and the selection
  if (rc) return rc;
  auto* wk = static_cast<unsigned long long*>(tmp.p);
  HT_HIP(hipMemcpyAsync(frontier.p, &initial, 8, hipMemcpyHostToDevice, s));
  rc = do_find_or_put(t, static_cast<uint64_t*>(frontier.p), 1, nullptr, s);
  if (rc) return rc;
  const DevTable dt = launch_view(t);
  uint64_t nf = 1;
  // A level runs as up to three spans of device work with a host round trip
  // between them (reading sizes, growing buffers): ev[0..1], ev[2..3],
  // ev[4..5]; ev[6..7] bracket the find-or-put (or the fused passes).
  Events evs;
  hipEvent_t* ev = evs.e;
  for (int i = 0; i < 8; ++i) HT_HIP(hipEventCreate(&ev[i]));
  for (uint32_t L = 0; L < levels && nf && rc == HT_OK; ++L) {
    rc = counts.ensure(nf * 8);
    if (!rc) rc = offsets.ensure(nf * 8);
    if (!rc && fused) rc = masks.ensure(nf * 16);
    if (!rc && ck) rc = noffsets.ensure(nf * 8);
    if (!rc && ck) rc = gcounts.ensure((nf + kWave - 1) / kWave * 4);
    if (rc) break;
    auto* cnt = static_cast<unsigned long long*>(counts.p);
    auto* off = static_cast<unsigned long long*>(offsets.p);
    auto* fr = static_cast<const uint64_t*>(frontier.p);
    auto* ns = static_cast<unsigned long long*>(nsel.p);
    auto* mk = static_cast<uint64_t*>(masks.p);
    const uint32_t g1 = (uint32_t)std::min<uint64_t>((nf + kBlock - 1) / kBlock, grid);
    if (fused && !ck) HT_HIP(zero_words(reinterpret_cast<uint32_t*>(ns), 2, s));
    double lms = 0.0;
    // span 1: successor counts (split, fused Cuckoo) or the fused bucketed pass, then a scan
    HT_HIP(hipEventRecord(ev[0], s));
    if (fused && !ck) {
      HT_HIP(hipEventRecord(ev[6], s));
      // the grid of the one-lane find-or-put kernels (7-level workload: 22.3-23.1 ms
      // for the fused levels at 8 blocks per compute unit, 19.3 at 6)
      const uint32_t gf = (uint32_t)std::min<uint64_t>((nf + kBlock - 1) / kBlock, atomic_grid_blocks(t));
      hipLaunchKernelGGL(bfs_fused_kernel, dim3(gf), dim3(kBlock), 0, s, m, dt, fr, nf, cnt, mk, ns);
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[7], s));
    } else {
      hipLaunchKernelGGL(bfs_count_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, cnt);
      HT_HIP(hipGetLastError());
    }
    HT_HIP(scan_exclusive(cnt, off, nf, ns + 1, wk, grid, s));
    HT_HIP(hipEventRecord(ev[1], s));
    unsigned long long last[3] = {0, 0, 0};
    HT_HIP(hipMemcpyAsync(&last[0], off + nf - 1, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipMemcpyAsync(&last[1], cnt + nf - 1, 8, hipMemcpyDeviceToHost, s));
    if (fused && !ck) HT_HIP(hipMemcpyAsync(&last[2], ns, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipStreamSynchronize(s));
    lms += span_ms(ev[0], ev[1]);
    const uint64_t total = last[0] + last[1];   // fused bucketed: new states; otherwise successors
    const uint64_t nb = (fused && !ck) ? last[2] : total;
    if (batch_sizes) batch_sizes[L] = nb;
    uint64_t nnew = 0;
    if (fused && !ck) {
      nnew = total;
    } else if (ck) {
      // span 2: fused probe and placement, evict, scrub, scan of the new counts
      rc = reserve_scratch(t, nb);   // lists and scratch set for this level, outside the timed spans
      if (rc) break;
      const CuckooScratch sc = scratch_view(t, nb);
      auto* gc = static_cast<uint32_t*>(gcounts.p);
      auto* noff = static_cast<unsigned long long*>(noffsets.p);
      const uint64_t ngroups = (nf + kWave - 1) / kWave;
      // the probe grid of the single-table Cuckoo find-or-put (fused levels of
      // the 7-level workload: 36.3-38.6 ms at 8 blocks per compute unit, 32.9
      // at 6)
      const uint32_t g2 = (uint32_t)std::min<uint64_t>((ngroups + 3) / 4, atomic_grid_blocks(t));
      HT_HIP(hipEventRecord(ev[2], s));
      HT_HIP(hipEventRecord(ev[6], s));
      hipLaunchKernelGGL(bfs_cuckoo_probe_kernel, dim3(g2), dim3(kBlock), 0, s, m, dt, fr, nf, off, sc, gc, cnt, mk);
      HT_HIP(hipGetLastError());
      hipLaunchKernelGGL(bfs_cuckoo_evict_kernel, dim3(g2), dim3(kBlock), 0, s, dt, nf, off, sc, gc, cnt, mk);
      HT_HIP(hipGetLastError());
      hipLaunchKernelGGL(bfs_cuckoo_scrub_kernel, dim3(g2), dim3(kBlock), 0, s, nf, off, sc, gc);
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[7], s));
      HT_HIP(scan_exclusive(cnt, noff, nf, ns + 1, wk, grid, s));
      HT_HIP(hipEventRecord(ev[3], s));
      unsigned long long lastn[2] = {0, 0};
      HT_HIP(hipMemcpyAsync(&lastn[0], noff + nf - 1, 8, hipMemcpyDeviceToHost, s));
      HT_HIP(hipMemcpyAsync(&lastn[1], cnt + nf - 1, 8, hipMemcpyDeviceToHost, s));
      HT_HIP(hipStreamSynchronize(s));
      lms += span_ms(ev[2], ev[3]);
      nnew = lastn[0] + lastn[1];
    }
    if (fused) {
      // last span: the new states written at their scanned offsets
      rc = next.ensure(std::max<uint64_t>(nnew, 1) * 8);
      if (rc) break;
      const unsigned long long* woff = ck ? static_cast<const unsigned long long*>(noffsets.p) : off;
      HT_HIP(hipEventRecord(ev[4], s));
      hipLaunchKernelGGL(bfs_fused_write_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, mk, cnt, woff,
                         static_cast<uint64_t*>(next.p));
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[5], s));
      HT_HIP(hipStreamSynchronize(s));
      lms += span_ms(ev[4], ev[5]);
      if (fop_ms) fop_ms[L] = span_ms(ev[6], ev[7]);
    } else {
      rc = batch.ensure(std::max<uint64_t>(nb, 1) * 8);
      if (!rc) rc = flags.ensure(std::max<uint64_t>(nb, 1));
      if (!rc) rc = next.ensure(std::max<uint64_t>(nb, 1) * 8);
      if (!rc) rc = reserve_scratch(t, nb);   // Cuckoo scratch for this batch, outside the timed spans
      if (rc) break;
      auto* bt = static_cast<uint64_t*>(batch.p);
      auto* fl = static_cast<uint8_t*>(flags.p);
      // span 2: write the batch, find-or-put it, select the new keys
      HT_HIP(hipEventRecord(ev[2], s));
      hipLaunchKernelGGL(bfs_write_kernel, dim3(g1), dim3(kBlock), 0, s, m, fr, nf, cnt, off, bt);
      HT_HIP(hipGetLastError());
      HT_HIP(hipEventRecord(ev[6], s));
      rc = do_find_or_put(t, bt, nb, fl, s);
      if (rc) break;
      HT_HIP(hipEventRecord(ev[7], s));
      HT_HIP(select_flagged(bt, fl, nb, static_cast<uint64_t*>(next.p), ns, wk, grid, s));
      HT_HIP(hipEventRecord(ev[3], s));
      unsigned long long nsv = 0;
      HT_HIP(hipMemcpyAsync(&nsv, ns, 8, hipMemcpyDeviceToHost, s));
      HT_HIP(hipStreamSynchronize(s));
      lms += span_ms(ev[2], ev[3]);
      nnew = nsv;
      if (fop_ms) fop_ms[L] = span_ms(ev[6], ev[7]);
    }
    if (level_ms) level_ms[L] = lms;
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
