// Parallel Cuckoo table: query, probe/deduplicate and insert kernels.
//
// Paper Sec. 4.1 / Fig. 2: c hash functions into one slot array; a key is
// looked up in at most c slots; an insertion writes the key into h_1(k) and,
// if that slot held k', evicts k' and re-inserts it with the hash function
// after the one that placed it, repeating until an empty slot is found or the
// eviction bound is hit; a key left over goes to a small stash.  One lane
// handles one key (the Alcantara et al. layout the paper describes).
//
// Duplicates (Sec. 5.1.1): the paper lets an inserter stop when it evicts its
// own key.  That does not cover a key that is in flight -- evicted by one
// lane and not yet re-placed -- while another lane looks it up, misses it and
// inserts a second copy.  Here find-or-put is split in two kernels so that no
// lookup overlaps an eviction:
//   1. probe: every key is looked up (read-only on the table); keys that miss
//      are deduplicated by compare-and-swap into a scratch set, whose winner
//      alone will insert the key and reports "new";
//   2. insert: the winners -- distinct and absent -- run the eviction chain.
//      Exchanges conserve keys, so every key is in exactly one slot or held
//      by exactly one lane, and no copy can appear.
// Winners are written to a per-wave region of the scratch lists (no global
// counter); the insert kernel walks the same regions.  Each winner clears its
// scratch-set slot again, so the set is empty for the next call without a
// fill pass.
#include "ht_device.h"

namespace ht {

// Look k up in its c slots; returns true on a hit.  `empty_mask` gets bit j
// when slot h_j(k) was seen empty.
template <bool SCRIPTED>
__device__ __forceinline__ bool cuckoo_lookup(const DevTable& t, uint64_t k, uint32_t& empty_mask) {
  empty_mask = 0;
  for (uint32_t j = 0; j < t.nhash; ++j) {
    const uint64_t v = t.slots[hidx<SCRIPTED>(t, k, j)];
    if (v == k) return true;
    if (v == kEmpty) empty_mask |= 1u << j;
  }
  return false;
}

template <bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void cuckoo_query_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint64_t k = keys[i];
    bool hit;
    if (k == kEmpty) {
      hit = t.ctr->sentinel != 0;
    } else {
      uint32_t em;
      hit = cuckoo_lookup<SCRIPTED>(t, k, em);
      if (!hit && (sc | oc)) hit = stash_query(t, k, sc, oc);
    }
    out[i] = hit ? 1 : 0;
  }
}

// Phase 1: lookup + deduplication.  Wave w owns keys [w*per_wave, ...).
template <bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void cuckoo_probe_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out,
                                                               CuckooScratch s) {
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t begin = wave * s.per_wave;
  uint64_t end = begin + s.per_wave;
  if (end > n) end = n;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  uint32_t nwin = 0;
  unsigned long long nsent = 0;
  for (uint64_t base = begin; base < end; base += kWave) {
    const uint64_t i = base + lane;
    const bool active = i < end;
    const uint64_t k = active ? keys[i] : 0;
    uint32_t res = 0;
    bool winner = false;
    uint64_t meta = 0;
    // the all-ones key: one lane per wave competes for the flag word
    const uint64_t sent = ballot(active && k == kEmpty);
    if (sent && lane == (int)__builtin_ctzll(sent)) {
      res = sentinel_put(t);
      nsent += res;
    }
    if (active && k != kEmpty) {
      uint32_t em;
      bool hit = cuckoo_lookup<SCRIPTED>(t, k, em);
      if (!hit && (sc | oc)) hit = stash_query(t, k, sc, oc);
      if (!hit) {
        uint64_t p = mix64(k ^ s.dset_seed) & s.dset_mask;
        for (;;) {
          const uint64_t old = cas64(&s.dset[p], kEmpty, k);
          if (old == kEmpty) {
            winner = true;
            res = 1;
            meta = p | ((uint64_t)em << 48);
            break;
          }
          if (old == k) break;            // another copy won
          p = (p + 1) & s.dset_mask;
        }
      }
    }
    if (active && out) out[i] = (uint8_t)res;
    const uint64_t wm = ballot(winner);
    if (winner) {
      const uint64_t slot = begin + nwin + lanes_below(wm);
      s.wkey[slot] = k;
      s.wmeta[slot] = meta;
    }
    nwin += (uint32_t)__popcll(wm);
  }
  if (lane == 0 && begin < n) s.wcnt[wave] = nwin;
  wave_count(t.ctr->size, nsent, (uint32_t)wave);
}

// Eviction chain of Sec. 4.1 for key x starting at slot index `slot` (which
// is h_j0(x)).  Returns true when the chain ended on an empty slot; on false
// `x` holds the key left without a slot.
template <bool SCRIPTED>
__device__ __forceinline__ bool cuckoo_chain(const DevTable& t, uint64_t& x, uint64_t slot,
                                             unsigned long long& nevict) {
  const uint32_t c = t.nhash;
  for (uint32_t step = 0;; ++step) {
    const uint64_t old = exch64(&t.slots[slot], x);
    if (old == kEmpty) return true;
    x = old;
    ++nevict;
    if (step + 1 >= t.max_chain) return false;   // the max_chain-th evicted key goes to the stash
    // The hash function that placed x here is the last j with h_j(x) == slot;
    // continue with the next one (cyclically), skipping ones that map here.
    uint64_t h[kMaxHash];
    int a = -1;
    for (uint32_t j = 0; j < c; ++j) {
      h[j] = hidx<SCRIPTED>(t, x, j);
      if (h[j] == slot) a = (int)j;
    }
    uint32_t nj = (uint32_t)(a + 1) % c;
    uint32_t tries = 0;
    while (h[nj] == slot && tries < c) {
      nj = (nj + 1) % c;
      ++tries;
    }
    if (h[nj] == slot) return false;   // no other slot for x
    slot = h[nj];
  }
}

// Phase 2: winners insert.  Wave w walks the winners of its own region.
template <bool SCRIPTED, bool PAPER_ORDER>
__global__ __launch_bounds__(kBlock) void cuckoo_insert_kernel(DevTable t, uint64_t n, CuckooScratch s) {
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? s.wcnt[wave] : 0u;
  unsigned long long nevict = 0, nnew = 0;
  for (uint32_t e = lane; e < cnt; e += kWave) {
    uint64_t x = s.wkey[begin + e];
    const uint64_t meta = s.wmeta[begin + e];
    bool placed = false;
    if constexpr (!PAPER_ORDER) {
      uint32_t em = (uint32_t)(meta >> 48);
      while (em && !placed) {
        const uint32_t j = (uint32_t)__builtin_ctz(em);
        em &= em - 1;
        placed = cas64(&t.slots[hidx<SCRIPTED>(t, x, j)], kEmpty, x) == kEmpty;
      }
    }
    if (!placed) placed = cuckoo_chain<SCRIPTED>(t, x, hidx<SCRIPTED>(t, x, 0), nevict);
    if (!placed) stash_put(t, x);     // x may be another key than the winner's
    ++nnew;
    store_coherent(&s.dset[meta & ((1ull << 48) - 1)], kEmpty);
  }
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
  wave_count(t.ctr->evictions, nevict, (uint32_t)wave);
}

// ---- host launchers --------------------------------------------------------

hipError_t cuckoo_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                        uint32_t grid, bool scripted, hipStream_t st) {
  if (scripted)
    hipLaunchKernelGGL((cuckoo_query_kernel<true>), dim3(grid), dim3(kBlock), 0, st, t, keys, n, out);
  else
    hipLaunchKernelGGL((cuckoo_query_kernel<false>), dim3(grid), dim3(kBlock), 0, st, t, keys, n, out);
  return hipGetLastError();
}

hipError_t cuckoo_probe(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                        const CuckooScratch& s, uint32_t grid, bool scripted, hipStream_t st) {
  if (scripted)
    hipLaunchKernelGGL((cuckoo_probe_kernel<true>), dim3(grid), dim3(kBlock), 0, st, t, keys, n, out, s);
  else
    hipLaunchKernelGGL((cuckoo_probe_kernel<false>), dim3(grid), dim3(kBlock), 0, st, t, keys, n, out, s);
  return hipGetLastError();
}

hipError_t cuckoo_insert(const DevTable& t, uint64_t n, const CuckooScratch& s, uint32_t grid, bool scripted,
                         bool paper_order, hipStream_t st) {
  if (scripted) {
    if (paper_order)
      hipLaunchKernelGGL((cuckoo_insert_kernel<true, true>), dim3(grid), dim3(kBlock), 0, st, t, n, s);
    else
      hipLaunchKernelGGL((cuckoo_insert_kernel<true, false>), dim3(grid), dim3(kBlock), 0, st, t, n, s);
  } else {
    if (paper_order)
      hipLaunchKernelGGL((cuckoo_insert_kernel<false, true>), dim3(grid), dim3(kBlock), 0, st, t, n, s);
    else
      hipLaunchKernelGGL((cuckoo_insert_kernel<false, false>), dim3(grid), dim3(kBlock), 0, st, t, n, s);
  }
  return hipGetLastError();
}

}  // namespace ht
