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
// inserts a second copy.  Here find-or-put runs in three kernels so that no
// lookup or duplicate check overlaps an eviction:
//   1. probe and place: every key is looked up in its c slots; a key that
//      misses compare-and-swaps itself into the candidate slots it saw
//      empty, in order h_1, h_2, ...  No key moves in this kernel and slots
//      only go from empty to a key, so a later probe sees a subset of an
//      earlier probe's empty slots and all copies of a key meet: the first
//      copy to reach an empty candidate wins and reports 1, the others find
//      it there (probe hit or compare-and-swap result) and report 0.  Keys
//      that find every candidate taken are listed.
//   2. evict: the listed keys are deduplicated by compare-and-swap into a
//      scratch set (one winner per key) and the winners run the eviction
//      chain of Sec. 4.1.  Exchanges conserve keys, so every key is in
//      exactly one slot or held by exactly one lane.
//   3. scrub: the winners' scratch-set slots are emptied again.
// With the paper's insertion order (HT_FLAG_CUCKOO_PAPER_ORDER) kernel 1
// places nothing and lists every miss; its chain starts by exchanging the
// key into h_1.
// Lists are kept in per-wave regions of the scratch arrays (no global
// counter); later kernels walk the same regions.  Only the scratch-set slots
// the evict kernel used are cleared, so the set is empty for the next call
// without a fill pass.
#pragma once
#include "ht_device.h"

namespace ht {

// Early exit on an empty slot.  Slots are never emptied (a key leaves a slot
// only when an exchange puts another key there), a key is placed at h_j only
// after h_1..h_{j-1} were seen taken, and a key evicted from h_j moves on to
// h_{j+1} (or back to h_1).  So while a key's c slot indices are pairwise
// distinct, a key stored at h_j has h_1..h_{j-1} all taken, and a lookup may
// stop at the first empty slot of h_1, h_2, ...  A key with coinciding slot
// indices can skip a slot when it is evicted (the next hash after the last
// index that maps to its slot), so such keys always read all c slots.
template <bool SCRIPTED>
__device__ __forceinline__ bool hashes_distinct(const DevTable& t, uint64_t k) {
  bool d = true;
  for (uint32_t a = 0; a + 1 < t.nhash; ++a) {
    const uint64_t ha = hidx<SCRIPTED>(t, k, a);
    for (uint32_t b = a + 1; b < t.nhash; ++b) d &= hidx<SCRIPTED>(t, k, b) != ha;
  }
  return d;
}

template <int R>
__device__ __forceinline__ bool any_lane(const bool (&f)[R]) {
  bool a = false;
#pragma unroll
  for (int r = 0; r < R; ++r) a |= f[r];
  return ballot(a) != 0;
}

// Look up R keys per lane in their c slots, probing h_1, h_2, ... and
// stopping on a hit or (distinct indices) on an empty slot; the loads of the
// R keys for one j are issued together.
template <int R, bool SCRIPTED>
__device__ __forceinline__ void cuckoo_lookup(const DevTable& t, const uint64_t (&k)[R], const bool (&live)[R],
                                              bool (&hit)[R]) {
  bool go[R], dist[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    hit[r] = false;
    go[r] = live[r];
    dist[r] = live[r] && hashes_distinct<SCRIPTED>(t, k[r]);
  }
  for (uint32_t j = 0; j < t.nhash && any_lane(go); ++j) {
    uint64_t v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = go[r] ? t.slots[hidx<SCRIPTED>(t, k[r], j)] : kEmpty;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (go[r]) {
        if (v[r] == k[r]) {
          hit[r] = true;
          go[r] = false;
        } else if (v[r] == kEmpty && dist[r]) {
          go[r] = false;
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
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * kBlock;
      k[r] = i < n ? keys[i] : kEmpty;
      live[r] = i < n && k[r] != kEmpty;
    }
    cuckoo_lookup<R, SCRIPTED>(t, k, live, hit);
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

constexpr uint64_t kIdxMask = (1ull << 40) - 1;

// Kernel 1: probe and place.  Wave w owns keys [w*per_wave, ...); a loop
// turn covers 64*R keys, lane l taking base + r*64 + l.  For j = 1..c each
// pending key reads h_j: its own key there ends the search (found); an empty
// slot is compare-and-swapped at once (placed, or found if another copy got
// there first, or taken by another key: go on with h_{j+1}).  Keys whose
// slot indices coincide read all c slots first and then try the empty ones
// in order.  Keys with every candidate taken go to the wave's region as
// (key, index).  In paper order nothing is placed: the first empty slot (or
// the end of the probe) lists the key.
template <int R, bool SCRIPTED, bool PAPER_ORDER>
__device__ __forceinline__ unsigned long long cuckoo_probe_region(const DevTable& t, const uint64_t* __restrict__ keys,
                                                                  uint64_t n, uint8_t* __restrict__ out,
                                                                  const CuckooScratch& s, uint64_t wave) {
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  uint64_t end = begin + s.per_wave;
  if (end > n) end = n;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  uint32_t nlist = 0;
  unsigned long long nnew = 0;
  for (uint64_t base = begin; base < end; base += (uint64_t)kWave * R) {
    uint64_t k[R];
    bool act[R], pend[R], dist[R], lst[R];
    uint32_t em[R];
    // the flag of each resolved key, stored once after the turn (1 << 8: none)
    uint32_t fl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * kWave + lane;
      act[r] = i < end;
      k[r] = act[r] ? keys[i] : 0;
      pend[r] = act[r] && k[r] != kEmpty;
      dist[r] = pend[r] && hashes_distinct<SCRIPTED>(t, k[r]);
      lst[r] = false;
      em[r] = 0;
      fl[r] = 1u << 8;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // the all-ones key: one lane per wave competes for the flag word
      const uint64_t sent = ballot(act[r] && k[r] == kEmpty);
      if (act[r] && k[r] == kEmpty) {
        uint32_t res = 0;
        if (lane == (int)__builtin_ctzll(sent)) {
          res = sentinel_put(t);
          nnew += res;
        }
        fl[r] = res;
      }
      // keys in the stash or the overflow list are found before any placement
      if (pend[r] && (sc | oc) && stash_query(t, k[r], sc, oc)) {
        fl[r] = 0;
        pend[r] = false;
      }
    }
    for (uint32_t j = 0; j < t.nhash && any_lane(pend); ++j) {
      uint64_t idx[R], v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        idx[r] = pend[r] ? hidx<SCRIPTED>(t, k[r], j) : 0;
        v[r] = pend[r] ? t.slots[idx[r]] : 0;
      }
      bool cas[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cas[r] = false;
        if (!pend[r]) continue;
        if (v[r] == k[r]) {
          fl[r] = 0;
          pend[r] = false;
        } else if (v[r] == kEmpty) {
          if (!dist[r]) {
            em[r] |= 1u << j;
          } else if (PAPER_ORDER) {
            lst[r] = true;
            pend[r] = false;
          } else {
            cas[r] = true;
          }
        }
      }
      if (PAPER_ORDER) continue;
      uint64_t old[R];
#pragma unroll
      for (int r = 0; r < R; ++r) old[r] = cas[r] ? cas64(&t.slots[idx[r]], kEmpty, k[r]) : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (cas[r] && (old[r] == kEmpty || old[r] == k[r])) {
          const uint32_t res = old[r] == kEmpty ? 1u : 0u;   // placed, or another copy was
          nnew += res;
          fl[r] = res;
          pend[r] = false;
        }
      }
    }
    // keys with coinciding slot indices: try the empty candidates in order
    if (!PAPER_ORDER) {
      for (;;) {
        bool go[R];
#pragma unroll
        for (int r = 0; r < R; ++r) go[r] = pend[r] && em[r];
        if (!any_lane(go)) break;
        uint64_t old[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          old[r] = 0;
          if (go[r]) {
            const uint32_t j = (uint32_t)__builtin_ctz(em[r]);
            em[r] &= em[r] - 1;
            old[r] = cas64(&t.slots[hidx<SCRIPTED>(t, k[r], j)], kEmpty, k[r]);
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (go[r] && (old[r] == kEmpty || old[r] == k[r])) {
            const uint32_t res = old[r] == kEmpty ? 1u : 0u;
            nnew += res;
            fl[r] = res;
            pend[r] = false;
          }
        }
      }
    }
    if (out) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (fl[r] < (1u << 8)) out[base + (uint64_t)r * kWave + lane] = (uint8_t)fl[r];
    }
    // every candidate taken (or, in paper order, not found): list for the evict kernel
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool l = pend[r] || lst[r];
      const uint64_t mm = ballot(l);
      if (l) {
        const uint64_t slot = begin + nlist + lanes_below(mm);
        s.wkey[slot] = k[r];
        s.wmeta[slot] = base + (uint64_t)r * kWave + lane;
      }
      nlist += (uint32_t)__popcll(mm);
    }
  }
  if (lane == 0 && begin < n) s.wcnt[wave] = nlist;
  return nnew;
}

// Empty the set slots the previous call's winners took (deferred scrub).  It
// runs in the probe kernel, which never touches the set, and the kernel
// boundary orders it before this call's evict kernel.  Wave w takes the
// record of the previous call's wave w (and of waves w + nwaves, ... when
// that call had more); `regions`, `cnt0` and `p0` (this wave's count and
// each lane's first entry) were loaded when the kernel started, so only the
// stores remain here.
__device__ __forceinline__ void cuckoo_scrub_deferred(const CuckooScratch& s, uint64_t wave, uint64_t nwaves,
                                                      uint64_t regions, uint32_t cnt0, uint64_t p0) {
  const int lane = lane_id();
  if (wave < regions) {
    if ((uint32_t)lane < cnt0 && p0 != ~0ull) s.dset[p0] = kEmpty;
    for (uint32_t e = lane + kWave; e < cnt0; e += kWave) {
      const uint64_t p = s.dirty[wave * s.dirty_stride + e];
      if (p != ~0ull) s.dset[p] = kEmpty;
    }
  }
  for (uint64_t r = wave + nwaves; r < regions; r += nwaves) {
    const uint32_t cnt = s.dirty_cnt[r];
    for (uint32_t e = lane; e < cnt; e += kWave) {
      const uint64_t p = s.dirty[r * s.dirty_stride + e];
      if (p != ~0ull) s.dset[p] = kEmpty;
    }
  }
}

template <int R, bool SCRIPTED, bool PAPER_ORDER>
__global__ __launch_bounds__(kBlock) void cuckoo_probe_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out,
                                                               CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  // the deferred scrub's loads go out with the first keys' loads
  uint64_t regions = 0, p0 = ~0ull;
  uint32_t cnt0 = 0;
  if (s.dirty) {
    // a vector load (the pointer in vector registers), so that nothing waits
    // for it before the probe starts
    const uint64_t* desc = s.dirty_desc;
    asm volatile("" : "+v"(desc));
    regions = *(const __attribute__((address_space(1))) uint64_t*)desc;
    cnt0 = s.dirty_cnt[wave];
    p0 = s.dirty[wave * s.dirty_stride + lane_id()];
  }
  wave_count(t.ctr->size, cuckoo_probe_region<R, SCRIPTED, PAPER_ORDER>(t, keys, n, out, s, wave), (uint32_t)wave);
  if (s.dirty) cuckoo_scrub_deferred(s, wave, nwaves, regions, cnt0, p0);
}

// Eviction chain of Sec. 4.1 for key x starting at slot index `slot` (which
// is h_j0(x)).  Returns true when the chain ended on an empty slot; on false
// `x` holds the key left without a slot.  `steps` counts the exchanges.
//
// With the lookahead flag (kFlagLookahead), a key y evicted from h_a(y)
// first reads its later candidates h_{a+1}(y), ..., h_c(y) (one load each,
// issued together) and compare-and-swaps itself into the lowest-numbered one
// it saw empty; only when none is empty (or every such compare-and-swap
// loses) does the chain go on by exchange into the next candidate.  Placing
// y at h_j this way keeps the early-exit invariant of the lookups: h_1..h_a
// are taken (y sat at h_a, which the evicting key now holds) and
// h_{a+1}..h_{j-1} were seen taken, and slots never empty again.
template <bool SCRIPTED, bool LOOK>
__device__ __forceinline__ bool cuckoo_chain(const DevTable& t, uint64_t& x, uint64_t slot,
                                             unsigned long long& nevict, uint32_t& steps) {
  const uint32_t c = t.nhash;
  for (uint32_t step = 0;; ++step) {
    const uint64_t old = exch64(&t.slots[slot], x);
    ++steps;
    if (old == kEmpty) return true;
    x = old;
    ++nevict;
    if (step + 1 >= t.max_chain) return false;   // the max_chain-th evicted key goes to the stash
    if constexpr (LOOK) {
      uint64_t h[kMaxHash];
      int a = -1;
      for (uint32_t j = 0; j < c; ++j) {
        h[j] = hidx<SCRIPTED>(t, x, j);
        if (h[j] == slot) a = (int)j;
      }
      if (a + 1 < (int)c) {
        uint64_t v[kMaxHash];
        for (uint32_t j = (uint32_t)(a + 1); j < c; ++j) v[j] = h[j] != slot ? t.slots[h[j]] : 0;
        for (uint32_t j = (uint32_t)(a + 1); j < c; ++j) {
          if (h[j] != slot && v[j] == kEmpty && cas64(&t.slots[h[j]], kEmpty, x) == kEmpty) return true;
        }
      }
    }
    // The hash function that placed x here is the last j with h_j(x) == slot
    // (a); x continues with h_{a+1}, which maps elsewhere by the choice of a,
    // or, after h_c (or when none maps here), with the first h_j that maps
    // elsewhere.  One pass over j, keeping no per-j values, so the kernel
    // stays within 64 vector registers.
    int a = -1;
    bool after = false, have_first = false;
    uint64_t hnext = 0, hfirst = 0;
    for (uint32_t j = 0; j < c; ++j) {
      const uint64_t hj = hidx<SCRIPTED>(t, x, j);
      if (hj == slot) {
        a = (int)j;
        after = true;
      } else {
        if (after) {
          hnext = hj;
          after = false;
        }
        if (!have_first) {
          hfirst = hj;
          have_first = true;
        }
      }
    }
    if (a >= 0 && a + 1 < (int)c) {
      slot = hnext;
    } else if (have_first) {
      slot = hfirst;
    } else {
      return false;   // no other slot for x
    }
  }
}

// Chain-length histogram (measurement flag): one atomic per chain on one of
// kSpread copies.
__device__ __forceinline__ void chain_record(const DevTable& t, uint32_t steps, bool placed, uint64_t wave) {
  if (!(t.flags & kFlagChainStats)) return;
  const uint32_t bin = placed ? (steps < (uint32_t)kChainBins ? steps : (uint32_t)kChainBins - 1) : 0u;
  add_agent(&t.ctr->chain_hist[(wave % kSpread) * kChainBins + bin], 1ull);
}

// Kernel 2: evict.  The keys kernel 1 listed are deduplicated in the
// scratch set; each winner reports 1 and runs the eviction chain from h_1.
// A wave serves the lists of `m` consecutive regions r0 .. r0+m-1 (m <=
// kMaxPack) as one list, so its lanes stay busy when each region listed
// fewer keys than a wave has lanes.
constexpr uint32_t kMaxPack = 8;

template <bool SCRIPTED, bool LOOK>
__device__ __forceinline__ void cuckoo_evict_regions(const DevTable& t, uint64_t n, uint8_t* __restrict__ out,
                                                     const CuckooScratch& s, uint64_t r0, uint32_t m,
                                                     unsigned long long& nnew, unsigned long long& nevict) {
  const int lane = lane_id();
  uint32_t cnt[kMaxPack];
  uint32_t total = 0;
#pragma unroll
  for (uint32_t q = 0; q < kMaxPack; ++q) {
    cnt[q] = q < m && (r0 + q) * s.per_wave < n ? s.wcnt[r0 + q] : 0u;
    total += cnt[q];
  }
  for (uint32_t e = lane; e < total; e += kWave) {
    // region q with cnt[0] + ... + cnt[q-1] <= e < ... + cnt[q], entry `off` of it
    uint32_t q = 0, off = e, acc = 0;
#pragma unroll
    for (uint32_t u = 0; u + 1 < kMaxPack; ++u) {
      acc += cnt[u];
      if (e >= acc) {
        q = u + 1;
        off = e - acc;
      }
    }
    const uint64_t r = r0 + q;
    const uint64_t begin = r * s.per_wave;
    const uint64_t k = s.wkey[begin + off];
    const uint64_t meta = s.wmeta[begin + off];
    uint64_t p = mix64(k ^ s.dset_seed) & s.dset_mask;
    bool winner = false;
    for (;;) {
      const uint64_t old = cas64(&s.dset[p], kEmpty, k);
      if (old == kEmpty) { winner = true; break; }
      if (old == k) break;               // another copy won
      p = (p + 1) & s.dset_mask;
    }
    if (out) out[meta & kIdxMask] = winner ? 1 : 0;
    // remember the scratch-set slot for the scrub (~0: nothing to clear)
    if (s.dirty) s.dirty[r * s.dirty_stride + off] = winner ? p : ~0ull;
    else s.wmeta[begin + off] = winner ? p : ~0ull;
    if (!winner) continue;
    uint64_t y = k;
    uint32_t steps = 0;
    const bool placed = cuckoo_chain<SCRIPTED, LOOK>(t, y, hidx<SCRIPTED>(t, y, 0), nevict, steps);
    if (!placed) stash_put(t, y);        // y may be another key than the winner's
    chain_record(t, steps, placed, r);
    ++nnew;
  }
  if (s.dirty && lane == 0) {
#pragma unroll
    for (uint32_t q = 0; q < kMaxPack; ++q)
      if (q < m) s.dirty_cnt[r0 + q] = cnt[q];
  }
}

template <bool SCRIPTED, bool LOOK>
__device__ __forceinline__ void cuckoo_evict_region(const DevTable& t, uint64_t n, uint8_t* __restrict__ out,
                                                    const CuckooScratch& s, uint64_t wave,
                                                    unsigned long long& nnew, unsigned long long& nevict) {
  cuckoo_evict_regions<SCRIPTED, LOOK>(t, n, out, s, wave, 1, nnew, nevict);
}

// `nregions`: the probe kernel's waves; wave w takes regions w*pack ...
template <bool SCRIPTED, bool LOOK>
__global__ __launch_bounds__(kBlock) void cuckoo_evict_kernel(DevTable t, uint64_t n, uint8_t* __restrict__ out,
                                                               CuckooScratch s, uint64_t nregions, uint32_t pack) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  unsigned long long nnew = 0, nevict = 0;
  if (s.dirty && wave == 0 && lane_id() == 0) s.dirty_desc[0] = nregions;
  const uint64_t r0 = wave * pack;
  if (r0 < nregions) {
    const uint32_t m = (uint32_t)(nregions - r0 < pack ? nregions - r0 : pack);
    cuckoo_evict_regions<SCRIPTED, LOOK>(t, n, out, s, r0, m, nnew, nevict);
  }
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
  wave_count(t.ctr->evictions, nevict, (uint32_t)wave);
}

// Single pass (HT_FLAG_CUCKOO_SINGLE_PASS), the insertion as Sec. 4.1 and
// Sec. 5.1.1 give it, kept to measure what the three kernels above prevent:
// one lane per key looks the key up in its c slots (and the stash), and on a
// miss exchanges it into h_1 and follows the eviction chain; a lane that
// evicts a copy of the key it is carrying stops there.  A lookup that runs
// while another lane holds a copy of its key in flight misses it, so a key
// can end up stored twice (a duplicate store) and reported new more than
// once.  Exact for batches without repeated keys.
template <bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void cuckoo_single_pass_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                                     uint64_t n, uint8_t* __restrict__ out) {
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  const uint32_t c = t.nhash;
  unsigned long long nnew = 0, nevict = 0;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint64_t first = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  for (uint64_t base = first - (first & (kWave - 1)); base < n; base += stride) {
    const uint64_t i = base + lane_id();
    if (i >= n) continue;
    const uint64_t k = keys[i];
    uint32_t res = 0;
    if (k == kEmpty) {
      res = sentinel_put(t);
    } else {
      bool hit = false;
      for (uint32_t j = 0; j < c && !hit; ++j) hit = t.slots[hidx<SCRIPTED>(t, k, j)] == k;
      if (!hit && (sc | oc)) hit = stash_query(t, k, sc, oc);
      if (!hit) {
        res = 1;
        uint64_t x = k;
        uint64_t slot = hidx<SCRIPTED>(t, k, 0);
        for (uint32_t step = 0;; ++step) {
          const uint64_t old = exch64(&t.slots[slot], x);
          if (old == kEmpty) break;
          if (old == x) {                  // evicted a copy of the key it carries: stop
            if (x == k) res = 0;
            break;
          }
          x = old;
          ++nevict;
          uint64_t h[kMaxHash];
          int a = -1;
          for (uint32_t j = 0; j < c; ++j) {
            h[j] = hidx<SCRIPTED>(t, x, j);
            if (h[j] == slot) a = (int)j;
          }
          uint32_t nj = (uint32_t)(a + 1) % c;
          for (uint32_t tries = 0; h[nj] == slot && tries < c; ++tries) nj = (nj + 1) % c;
          if (step + 1 >= t.max_chain || h[nj] == slot) {
            stash_put(t, x);
            break;
          }
          slot = h[nj];
        }
      }
    }
    nnew += res;
    if (out) out[i] = (uint8_t)res;
  }
  wave_count(t.ctr->size, nnew, (uint32_t)(first / kWave));
  wave_count(t.ctr->evictions, nevict, (uint32_t)(first / kWave));
}

// Kernel 3 (calls without the deferred scrub): empty the scratch-set slots
// the winners of kernel 2 took.  It runs after kernel 2 has finished, so no
// copy of a key can find its slot empty and win a second time.
__device__ __forceinline__ void cuckoo_scrub_region(uint64_t n, const CuckooScratch& s, uint64_t wave) {
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? s.wcnt[wave] : 0u;
  for (uint32_t e = lane; e < cnt; e += kWave) {
    const uint64_t p = s.wmeta[begin + e];
    if (p != ~0ull) s.dset[p] = kEmpty;
  }
}

}  // namespace ht
