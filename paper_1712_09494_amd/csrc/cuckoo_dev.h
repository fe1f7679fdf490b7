// Parallel Cuckoo table: query kernel and the four find-or-put phases.
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
// inserts a second copy.  Here find-or-put runs in four kernels so that no
// lookup or duplicate check overlaps an eviction:
//   1. probe: every key is looked up (read-only on the table); hits report 0;
//      misses are listed with the mask of candidate slots h_j(k) seen empty.
//   2. place: every miss compare-and-swaps itself into its candidate slots,
//      in mask order.  No key moves in this phase and slots only go from
//      empty to a key, so all copies of a key walk the same slots and meet:
//      the first copy to reach an empty candidate wins and reports 1, the
//      others find it there and report 0.  Misses that find every candidate
//      taken are listed again.
//   3. evict: the keys left over are deduplicated by compare-and-swap into a
//      scratch set (one winner per key) and the winners run the eviction
//      chain of Sec. 4.1.  Exchanges conserve keys, so every key is in exactly
//      one slot or held by exactly one lane.
//   4. scrub: the winners' scratch-set slots are emptied again.
// With the paper's insertion order (HT_FLAG_CUCKOO_PAPER_ORDER) phase 2 is
// skipped and every miss goes through the scratch set and the chain, which
// starts by exchanging the key into h_1.
// Lists are kept in per-wave regions of the scratch arrays (no global
// counter); later phases walk the same regions and compact in place.  Only
// the slots phase 3 used are cleared, so the set is empty for the next call
// without a fill pass.
#pragma once
#include "ht_device.h"

namespace ht {

// Look up R keys per lane in their c slots, probing h_1, h_2, ... with an
// early exit on a hit; the loads of the R keys for one j are issued together.
// hit[r] is set on a hit; empty_mask[r] gets bit j when slot h_j was empty.
template <int R, bool SCRIPTED>
__device__ __forceinline__ void cuckoo_lookup(const DevTable& t, const uint64_t (&k)[R], const bool (&live)[R],
                                              bool (&hit)[R], uint32_t (&empty_mask)[R]) {
  bool go[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    hit[r] = false;
    empty_mask[r] = 0;
    go[r] = live[r];
  }
  for (uint32_t j = 0; j < t.nhash; ++j) {
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = go[r] ? t.slots[hidx<SCRIPTED>(t, k[r], j)] : kEmpty;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (go[r]) {
        if (v[r] == k[r]) {
          hit[r] = true;
          go[r] = false;
        } else if (v[r] == kEmpty) {
          empty_mask[r] |= 1u << j;
        }
      }
    }
  }
}

template <int R, bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void cuckoo_query_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out) {
  const uint64_t per = (uint64_t)kBlock * R;
  const uint64_t stride = (uint64_t)gridDim.x * per;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  for (uint64_t base = (uint64_t)blockIdx.x * per + threadIdx.x; base < n; base += stride) {
    uint64_t k[R];
    bool live[R], hit[R];
    uint32_t em[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * kBlock;
      k[r] = i < n ? keys[i] : kEmpty;
      live[r] = i < n && k[r] != kEmpty;
    }
    cuckoo_lookup<R, SCRIPTED>(t, k, live, hit, em);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * kBlock;
      if (i < n) {
        bool h = hit[r];
        if (k[r] == kEmpty) h = t.ctr->sentinel != 0;
        else if (!h && (sc | oc)) h = stash_query(t, k[r], sc, oc);
        out[i] = h ? 1 : 0;
      }
    }
  }
}

// Phase 1: lookup.  Wave w owns keys [w*per_wave, ...); a loop turn covers
// 64*R keys, lane l taking base + r*64 + l.  Misses go to the wave's region
// as (key, index | empty-candidate mask << 48).
template <int R, bool SCRIPTED>
__device__ __forceinline__ unsigned long long cuckoo_probe_region(const DevTable& t, const uint64_t* __restrict__ keys,
                                                                  uint64_t n, uint8_t* __restrict__ out,
                                                                  const CuckooScratch& s, uint64_t wave) {
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  uint64_t end = begin + s.per_wave;
  if (end > n) end = n;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  uint32_t nmiss = 0;
  unsigned long long nsent = 0;
  for (uint64_t base = begin; base < end; base += (uint64_t)kWave * R) {
    uint64_t k[R];
    bool act[R], live[R], hit[R];
    uint32_t em[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * kWave + lane;
      act[r] = i < end;
      k[r] = act[r] ? keys[i] : 0;
      live[r] = act[r] && k[r] != kEmpty;
    }
    cuckoo_lookup<R, SCRIPTED>(t, k, live, hit, em);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * kWave + lane;
      uint32_t res = 0;
      // the all-ones key: one lane per wave competes for the flag word
      const uint64_t sent = ballot(act[r] && k[r] == kEmpty);
      if (sent && lane == (int)__builtin_ctzll(sent)) {
        res = sentinel_put(t);
        nsent += res;
      }
      if (live[r] && !hit[r] && (sc | oc)) hit[r] = stash_query(t, k[r], sc, oc);
      const bool miss = live[r] && !hit[r];
      if (act[r] && !miss && out) out[i] = (uint8_t)res;
      const uint64_t mm = ballot(miss);
      if (miss) {
        const uint64_t slot = begin + nmiss + lanes_below(mm);
        s.wkey[slot] = k[r];
        s.wmeta[slot] = i | ((uint64_t)em[r] << 48);
      }
      nmiss += (uint32_t)__popcll(mm);
    }
  }
  if (lane == 0 && begin < n) s.wcnt[wave] = nmiss;
  return nsent;
}

template <int R, bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void cuckoo_probe_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out,
                                                               CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  wave_count(t.ctr->size, cuckoo_probe_region<R, SCRIPTED>(t, keys, n, out, s, wave), (uint32_t)wave);
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

constexpr uint64_t kIdxMask = (1ull << 40) - 1;

// Phase 2: place.  Wave w walks the misses of its region, R per lane per
// turn, compare-and-swapping each into its empty candidates (all R issued
// together).  Keys that find every candidate taken are compacted to the
// front of the region for phase 3.
template <int R, bool SCRIPTED>
__device__ __forceinline__ unsigned long long cuckoo_place_region(const DevTable& t, uint64_t n,
                                                                  uint8_t* __restrict__ out, const CuckooScratch& s,
                                                                  uint64_t wave) {
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? s.wcnt[wave] : 0u;
  unsigned long long nnew = 0;
  uint32_t nleft = 0;
  for (uint32_t e0 = 0; e0 < cnt; e0 += kWave * R) {
    uint64_t x[R], meta[R];
    bool live[R], done[R];
    uint32_t em[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t e = e0 + r * kWave + lane;
      live[r] = e < cnt;
      x[r] = live[r] ? s.wkey[begin + e] : 0;
      meta[r] = live[r] ? s.wmeta[begin + e] : 0;
      done[r] = !live[r];
      em[r] = (uint32_t)(meta[r] >> 48);
    }
    for (;;) {
      bool any = false;
#pragma unroll
      for (int r = 0; r < R; ++r) any |= !done[r] && em[r];
      if (!any) break;
      uint64_t old[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        old[r] = 0;
        if (!done[r] && em[r]) {
          const uint32_t j = (uint32_t)__builtin_ctz(em[r]);
          em[r] &= em[r] - 1;
          old[r] = cas64(&t.slots[hidx<SCRIPTED>(t, x[r], j)], kEmpty, x[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!done[r] && (old[r] == kEmpty || old[r] == x[r])) {
          const uint32_t res = old[r] == kEmpty ? 1u : 0u;   // placed, or another copy was
          nnew += res;
          if (out) out[meta[r] & kIdxMask] = (uint8_t)res;
          done[r] = true;
        }
      }
    }
    // every candidate taken: keep for the eviction phase (in-place compaction)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool left = !done[r];
      const uint64_t lm = ballot(left);
      if (left) {
        const uint64_t slot = begin + nleft + lanes_below(lm);
        s.wkey[slot] = x[r];
        s.wmeta[slot] = meta[r];
      }
      nleft += (uint32_t)__popcll(lm);
    }
  }
  if (lane == 0 && begin < n) s.ccnt[wave] = nleft;
  return nnew;
}

template <int R, bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void cuckoo_place_kernel(DevTable t, uint64_t n, uint8_t* __restrict__ out,
                                                               CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  wave_count(t.ctr->size, cuckoo_place_region<R, SCRIPTED>(t, n, out, s, wave), (uint32_t)wave);
}

// Phase 3: evict.  The keys left by phase 2 (or, in paper order, every
// miss) are deduplicated in the scratch set; each winner reports 1 and runs
// the eviction chain from h_1.
template <bool SCRIPTED, bool PAPER_ORDER>
__device__ __forceinline__ void cuckoo_evict_region(const DevTable& t, uint64_t n, uint8_t* __restrict__ out,
                                                    const CuckooScratch& s, uint64_t wave,
                                                    unsigned long long& nnew, unsigned long long& nevict) {
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? (PAPER_ORDER ? s.wcnt[wave] : s.ccnt[wave]) : 0u;
  for (uint32_t e = lane; e < cnt; e += kWave) {
    const uint64_t k = s.wkey[begin + e];
    const uint64_t meta = s.wmeta[begin + e];
    uint64_t p = mix64(k ^ s.dset_seed) & s.dset_mask;
    bool winner = false;
    for (;;) {
      const uint64_t old = cas64(&s.dset[p], kEmpty, k);
      if (old == kEmpty) { winner = true; break; }
      if (old == k) break;               // another copy won
      p = (p + 1) & s.dset_mask;
    }
    if (out) out[meta & kIdxMask] = winner ? 1 : 0;
    // remember the scratch-set slot for phase 4 (~0: nothing to clear)
    s.wmeta[begin + e] = winner ? p : ~0ull;
    if (!winner) continue;
    uint64_t y = k;
    if (!cuckoo_chain<SCRIPTED>(t, y, hidx<SCRIPTED>(t, y, 0), nevict))
      stash_put(t, y);                   // y may be another key than the winner's
    ++nnew;
  }
}

template <bool SCRIPTED, bool PAPER_ORDER>
__global__ __launch_bounds__(kBlock) void cuckoo_evict_kernel(DevTable t, uint64_t n, uint8_t* __restrict__ out,
                                                               CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  unsigned long long nnew = 0, nevict = 0;
  cuckoo_evict_region<SCRIPTED, PAPER_ORDER>(t, n, out, s, wave, nnew, nevict);
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
  wave_count(t.ctr->evictions, nevict, (uint32_t)wave);
}

// Phase 4: empty the scratch-set slots the winners of phase 3 took.  It runs
// after phase 3 has finished, so no copy of a key can find its slot empty and
// win a second time.
template <bool PAPER_ORDER>
__device__ __forceinline__ void cuckoo_scrub_region(uint64_t n, const CuckooScratch& s, uint64_t wave) {
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? (PAPER_ORDER ? s.wcnt[wave] : s.ccnt[wave]) : 0u;
  for (uint32_t e = lane; e < cnt; e += kWave) {
    const uint64_t p = s.wmeta[begin + e];
    if (p != ~0ull) s.dset[p] = kEmpty;
  }
}

template <bool PAPER_ORDER>
__global__ __launch_bounds__(kBlock) void cuckoo_scrub_kernel(uint64_t n, CuckooScratch s) {
  cuckoo_scrub_region<PAPER_ORDER>(n, s, ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave);
}

}  // namespace ht
