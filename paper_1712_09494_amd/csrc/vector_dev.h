// Keys that are state vectors of W 64-bit words (W = 2 or 4).  GPUexplore
// keeps each state as a vector of words in its bucketed table (Sec. 3.2,
// Sec. 4.2); the Cuckoo table of Sec. 4.1 moves keys with single-word
// exchanges, which a multi-word key cannot use directly.
//
// Layout.  Every member vector is written once into the table's arena (W
// words per entry, append-only).  Table slots, stash and overflow list hold
// 64-bit handles: the top 30 bits of the vector's hash H and a 34-bit arena
// index.  Bucket and slot positions are functions of those 30 hash bits, so
// a handle carries everything an eviction chain needs and a chain never reads
// the arena.  A handle is never all ones (arena indices stay below 2^34 - 1),
// so the empty marker needs no special key.
//
// Find-or-put, with no kernel reading a vector another lane is still writing
// and no lane waiting for another:
//   1. find or claim, one walk per vector: along its bucket sequence (then
//      stash, then overflow set) or, in a Cuckoo table, the stash and
//      overflow set and then its candidate slots h_1..h_c.  A stored handle
//      with the vector's hash bits is compared with the arena words (equal:
//      present, report 0); an empty slot gets a placeholder -- the hash bits
//      and the batch index -- by compare-and-swap.  Copies of a vector walk
//      the same slots in the same order, so a second copy meets the first
//      one's placeholder and compares the two batch rows (complete before the
//      kernel starts): equal means it reports 0.  No handle is committed and
//      no exchange runs in this kernel, so placeholders stay where they were
//      put.  One atomic per new vector; claims are listed per wave region;
//   2. commit: each claimed slot takes an arena entry (one counter atomic per
//      wave), gets the vector's words written there and its placeholder
//      replaced by the final handle;
// and for Cuckoo tables, the vectors that found every candidate taken:
//   3. evict: deduplicated in the scratch set by batch index (equal vectors
//      compared word by word in the batch); each winner reports 1, takes an
//      arena entry, writes its words and runs the exchange chain of Sec. 4.1
//      from h_1 with its handle (then stash, overflow set);
//   4. scrub the scratch set (the single-word Cuckoo scrub kernel).
// The stash and the overflow list of a vector table are open-addressed sets
// of handles, probed from positions given by the hash bits.
// Lookups stop early by the same rules as the single-word tables: a bucket
// with an empty slot ends the bucket sequence (slots fill as a prefix and are
// never emptied), and a Cuckoo lookup stops at an empty candidate when the
// handle's c slot indices are distinct.
#pragma once
#include "cuckoo_dev.h"

namespace ht {

constexpr uint64_t kArenaMask = (1ull << kArenaBits) - 1;
// Arena indices stay below 2^33; bit 33 of a handle marks a placeholder whose
// low 33 bits are a batch index (find-or-claim kernel, replaced in commit).
constexpr uint64_t kPlaceBit = 1ull << 33;
constexpr uint64_t kBatchMask = kPlaceBit - 1;

// Hash of a vector: the words folded through mix64 in order, seeded per table.
template <int W>
__device__ __forceinline__ uint64_t vec_hash(const uint64_t (&v)[W], uint64_t seed) {
  uint64_t h = mix64(v[0] ^ seed);
#pragma unroll
  for (int j = 1; j < W; ++j) h = mix64(h ^ mix64(v[j] + 0x9e3779b97f4a7c15ull * (uint64_t)j));
  return h;
}

__device__ __forceinline__ uint64_t handle_hb(uint64_t hd) { return hd >> kArenaBits; }
__device__ __forceinline__ uint64_t handle_idx(uint64_t hd) { return hd & kArenaMask; }

// W words from a 16-byte aligned address.
template <int W>
__device__ __forceinline__ void load_vec(const uint64_t* p, uint64_t (&v)[W]) {
#pragma unroll
  for (int j = 0; j < W; j += 2) {
    const ulonglong2 x = *reinterpret_cast<const ulonglong2*>(p + j);
    v[j] = x.x;
    v[j + 1] = x.y;
  }
}

template <int W>
__device__ __forceinline__ bool vec_eq(const uint64_t (&a)[W], const uint64_t (&b)[W]) {
  bool e = true;
#pragma unroll
  for (int j = 0; j < W; ++j) e &= a[j] == b[j];
  return e;
}

// Handle hd holds vector v: hash bits first, then the arena words.  Empty
// slots and placeholders hold no arena entry.
template <int W>
__device__ __forceinline__ bool vec_holds(const DevTable& t, uint64_t hd, uint64_t hb, const uint64_t (&v)[W]) {
  if (hd == kEmpty || (hd & kPlaceBit) || handle_hb(hd) != hb) return false;
  uint64_t a[W];
  load_vec<W>(t.arena + handle_idx(hd) * W, a);
  return vec_eq<W>(a, v);
}

// q-th bucket of the bucket sequence: h_1..h_c, then the walk of consecutive
// buckets after h_c (wrapping at the end of the table), given the (q-1)-th.
__device__ __forceinline__ uint64_t vec_bucket(const DevTable& t, uint64_t hb, uint32_t q, uint64_t prev) {
  if (q < t.nhash) return hidx<false>(t, hb, q);
  return prev + 1 == t.nrange ? 0 : prev + 1;
}

template <int W>
__device__ bool vec_lookup_bucketed(const DevTable& t, uint64_t hb, const uint64_t (&v)[W]) {
  const uint32_t B = t.bucket_slots;
  const uint32_t steps = t.nhash + t.walk;
  uint64_t b = 0;
  for (uint32_t q = 0; q < steps; ++q) {
    b = vec_bucket(t, hb, q, b);
    const uint64_t* bk = t.slots + b * B;
    for (uint32_t c0 = 0; c0 < B; c0 += 8) {
      uint64_t x[8];
      load8(bk + c0, x);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (x[k] == kEmpty) return false;       // prefix: the rest of the sequence is unused
        if (vec_holds<W>(t, x[k], hb, v)) return true;
      }
    }
  }
  return false;
}

template <int W>
__device__ bool vec_lookup_cuckoo(const DevTable& t, uint64_t hb, const uint64_t (&v)[W]) {
  const bool dist = hashes_distinct<false>(t, hb);
  for (uint32_t j = 0; j < t.nhash; ++j) {
    const uint64_t hd = t.slots[hidx<false>(t, hb, j)];
    if (hd == kEmpty) {
      if (dist) return false;
      continue;
    }
    if (vec_holds<W>(t, hd, hb, v)) return true;
  }
  return false;
}

// Start of the overflow set's probe sequence (linear probing, any length).
__device__ __forceinline__ uint32_t overflow_start(const DevTable& t, uint64_t hb) {
  return (uint32_t)mulhi64(mix64(hb ^ t.stash_seed ^ 0x5851f42d4c957f2dull), t.overflow_slots);
}

// Stash and overflow set: probe from the hash bits' position until an empty slot.
template <int W>
__device__ bool vec_stash_query(const DevTable& t, uint64_t hb, const uint64_t (&v)[W], uint32_t sc,
                                uint32_t oc) {
  if (sc) {
    const uint32_t S = t.stash_slots;
    uint32_t p = stash_start(t, hb);
    for (uint32_t i = 0; i < S; ++i) {
      const uint64_t hd = t.stash[p];
      if (hd == kEmpty) break;
      if (vec_holds<W>(t, hd, hb, v)) return true;
      p = (p + 1) & (S - 1);
    }
  }
  if (oc) {
    const uint32_t m = t.overflow_slots;
    uint32_t p = overflow_start(t, hb);
    for (uint32_t i = 0; i < m; ++i) {
      const uint64_t hd = t.overflow[p];
      if (hd == kEmpty) break;
      if (vec_holds<W>(t, hd, hb, v)) return true;
      p = p + 1 == m ? 0 : p + 1;
    }
  }
  return false;
}

template <int W>
__device__ __forceinline__ bool vec_find(const DevTable& t, uint64_t hb, const uint64_t (&v)[W], uint32_t sc,
                                         uint32_t oc) {
  const bool f = t.kind == HT_KIND_BUCKETED ? vec_lookup_bucketed<W>(t, hb, v) : vec_lookup_cuckoo<W>(t, hb, v);
  return f || ((sc | oc) && vec_stash_query<W>(t, hb, v, sc, oc));
}

// Place a handle of a vector known to be absent (no comparison needed).
__device__ inline void vec_stash_put(const DevTable& t, uint64_t hd) {
  const uint32_t S = t.stash_slots;
  uint32_t p = stash_start(t, handle_hb(hd));
  for (uint32_t i = 0; i < S; ++i) {
    if (cas64(&t.stash[p], kEmpty, hd) == kEmpty) {
      add_agent(&t.ctr->stash_count, 1u);
      return;
    }
    p = (p + 1) & (S - 1);
  }
  const uint32_t m = t.overflow_slots;
  p = overflow_start(t, handle_hb(hd));
  for (uint32_t i = 0; i < m; ++i) {
    if (cas64(&t.overflow[p], kEmpty, hd) == kEmpty) {
      add_agent(&t.ctr->overflow_count, 1u);
      return;
    }
    p = p + 1 == m ? 0 : p + 1;
  }
  add_agent(&t.ctr->lost, 1u);
}

__device__ inline void vec_place_cuckoo(const DevTable& t, uint64_t hd, unsigned long long& nevict) {
  const uint32_t c = t.nhash;
  for (uint32_t j = 0; j < c; ++j) {
    uint64_t* p = &t.slots[hidx<false>(t, handle_hb(hd), j)];
    if (*p == kEmpty && cas64(p, kEmpty, hd) == kEmpty) return;
  }
  // every candidate taken: the exchange chain of Sec. 4.1 from h_1
  uint64_t x = hd;
  uint64_t slot = hidx<false>(t, handle_hb(x), 0);
  for (uint32_t step = 0;; ++step) {
    const uint64_t old = exch64(&t.slots[slot], x);
    if (old == kEmpty) return;
    x = old;
    ++nevict;
    if (step + 1 >= t.max_chain) break;
    // next hash after the last one that maps x here, skipping ones that also do
    uint64_t h[kMaxHash];
    int a = -1;
    for (uint32_t j = 0; j < c; ++j) {
      h[j] = hidx<false>(t, handle_hb(x), j);
      if (h[j] == slot) a = (int)j;
    }
    uint32_t nj = (uint32_t)(a + 1) % c;
    for (uint32_t tries = 0; h[nj] == slot && tries < c; ++tries) nj = (nj + 1) % c;
    if (h[nj] == slot) break;
    slot = h[nj];
  }
  vec_stash_put(t, x);
}

// Arena entries for the lanes with `want` set: one counter atomic per wave
// and range.  A wave starts at its own range and moves on while a range is
// full, so every entry of every range is handed out.  ~0 when all are taken.
__device__ inline uint64_t arena_take(const DevTable& t, bool want, uint64_t wave) {
  uint64_t idx = ~0ull;
  for (uint32_t a = 0; a < (uint32_t)kSpread; ++a) {
    const uint64_t wm = ballot(want);
    if (!wm) break;
    const uint32_t rg = (uint32_t)((wave + a) % kSpread);
    unsigned long long first = 0;
    if (lane_id() == 0) first = add_agent(&t.ctr->arena_next[rg * kLineWords], (unsigned long long)__popcll(wm));
    first = shfl64(first, 0);
    const uint64_t avail = first < t.arena_cap ? t.arena_cap - first : 0;
    const uint64_t rank = lanes_below(wm);
    if (want && rank < avail) {
      idx = (uint64_t)rg * t.arena_cap + first + rank;
      want = false;
    }
  }
  return idx;
}

// List entry of a vector whose Cuckoo candidates were all taken at claim
// time: it goes to the evict kernel.
constexpr uint64_t kLeftover = ~1ull;

// Kernel 3 (Cuckoo): the leftover vectors are deduplicated in the scratch
// set by batch index (equal vectors compared word by word in the batch);
// each winner reports 1, takes an arena entry, writes its words and runs the
// exchange chain of Sec. 4.1 from h_1 with its handle.  Every list entry's
// meta word becomes its scratch-set slot (or ~0) for the scrub kernel.
template <int W>
__global__ __launch_bounds__(kBlock) void vec_evict_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                            uint64_t n, uint8_t* __restrict__ out,
                                                            CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? s.wcnt[wave] : 0u;
  unsigned long long nnew = 0, nevict = 0;
  for (uint32_t e0 = 0; e0 < cnt; e0 += kWave) {
    const uint32_t e = e0 + (uint32_t)lane;
    bool winner = false;
    uint64_t hb = 0;
    uint64_t v[W];
#pragma unroll
    for (int j = 0; j < W; ++j) v[j] = 0;
    if (e < cnt) {
      uint64_t p = ~0ull;
      if (s.wkey[begin + e] == kLeftover) {
        const uint64_t m = s.wmeta[begin + e];
        const uint64_t i = m & kBatchMask;
        hb = m >> 33;
        load_vec<W>(keys + i * W, v);
        p = mix64(hb ^ s.dset_seed) & s.dset_mask;
        for (;;) {
          const uint64_t old = cas64(&s.dset[p], kEmpty, i);
          if (old == kEmpty) {
            winner = true;
            break;
          }
          if (old < n) {                   // the set holds indices of this batch only
            uint64_t u[W];
            load_vec<W>(keys + old * W, u);
            if (vec_eq<W>(u, v)) break;    // an equal vector of the batch won
          }
          p = (p + 1) & s.dset_mask;
        }
        if (out) out[i] = winner ? 1 : 0;
        if (!winner) p = ~0ull;
      }
      s.wmeta[begin + e] = p;
    }
    if (!ballot(winner)) continue;
    const uint64_t idx = arena_take(t, winner, wave);
    if (winner) {
      ++nnew;
      if (idx == ~0ull) {
        add_agent(&t.ctr->lost, 1u);     // only after more members than slots + stash + overflow
      } else {
#pragma unroll
        for (int j = 0; j < W; j += 2)
          *reinterpret_cast<ulonglong2*>(t.arena + idx * W + j) = make_ulonglong2(v[j], v[j + 1]);
        vec_place_cuckoo(t, (hb << kArenaBits) | idx, nevict);
      }
    }
  }
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
  wave_count(t.ctr->evictions, nevict, (uint32_t)wave);
}

// One slot of a claim walk, given the value read there: 1 = the placeholder
// is now here, 2 = an equal vector of the batch holds this slot, 0 = go on.
template <int W>
__device__ __forceinline__ int vec_claim_seen(uint64_t* p, uint64_t hd, uint64_t ph, uint64_t hb,
                                              const uint64_t (&v)[W], const uint64_t* __restrict__ keys,
                                              uint64_t n) {
  if (hd == kEmpty) {
    hd = cas64(p, kEmpty, ph);
    if (hd == kEmpty) return 1;
  }
  if ((hd & kPlaceBit) && hd != kEmpty && handle_hb(hd) == hb) {
    const uint64_t j = hd & kBatchMask;
    if (j < n) {
      uint64_t u[W];
      load_vec<W>(keys + j * W, u);
      if (vec_eq<W>(u, v)) return 2;
    }
  }
  return 0;
}

// One slot of a bucketed walk that both looks up and claims: a member stored
// by an earlier call (a committed handle) that holds the vector gives 3;
// otherwise as vec_claim_seen.  No handle is committed while this runs (the
// commit kernel comes after), so a failed compare-and-swap only ever returns
// a placeholder.
template <int W>
__device__ __forceinline__ int vec_find_or_claim_seen(const DevTable& t, uint64_t* p, uint64_t hd, uint64_t ph,
                                                      uint64_t hb, const uint64_t (&v)[W],
                                                      const uint64_t* __restrict__ keys, uint64_t n) {
  if (hd != kEmpty && !(hd & kPlaceBit)) return vec_holds<W>(t, hd, hb, v) ? 3 : 0;
  return vec_claim_seen<W>(p, hd, ph, hb, v, keys, n);
}

// Kernel 1: lookup and claim in one walk.  Bucketed: slots
// fill as a prefix of each vector's bucket sequence, then the stash, then
// the overflow set, and none is ever emptied, so the walk meets a stored copy
// of the vector before the first empty slot it could claim.  Cuckoo: the
// stash and overflow set are looked up first (a chain that ends there can
// leave the vector's other candidates empty); then the candidates h_1..h_c
// in order, a stored copy never lying past an empty candidate when the c
// indices are distinct (else all c are looked up before any claim); a vector
// with every candidate taken is left for the evict kernel.  Either way one
// walk per vector answers "present" or claims a free location, and copies
// within the batch meet at one placeholder.  Claimed locations (and Cuckoo
// leftovers, as kLeftover) are listed per wave region as (location, hash
// bits << 33 | batch index) for the commit and evict kernels.
template <int W>
__global__ __launch_bounds__(kBlock) void vec_find_or_claim_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                                    uint64_t n, uint8_t* __restrict__ out,
                                                                    CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int lane = lane_id();
  const uint64_t begin = wave * s.per_wave;
  uint64_t end = begin + s.per_wave;
  if (end > n) end = n;
  const uint32_t B = t.bucket_slots;
  const uint32_t steps = t.nhash + t.walk;
  const uint64_t nslots = t.nrange * B;
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  uint32_t nlist = 0;
  unsigned long long nnew = 0;
  for (uint64_t base = begin; base < end; base += kWave) {
    const uint64_t i = base + lane;
    bool claimed = false, leftover = false;
    uint64_t loc = ~0ull, hb = 0;
    if (i < end && t.kind == HT_KIND_CUCKOO) {
      uint64_t v[W];
      load_vec<W>(keys + i * W, v);
      hb = vec_hash<W>(v, t.vseed) >> kArenaBits;
      const uint64_t ph = (hb << kArenaBits) | kPlaceBit | i;
      int st = (sc | oc) && vec_stash_query<W>(t, hb, v, sc, oc) ? 3 : 0;
      if (!st && !hashes_distinct<false>(t, hb)) {
        for (uint32_t j = 0; j < t.nhash && !st; ++j) {
          const uint64_t hd = t.slots[hidx<false>(t, hb, j)];
          if (hd != kEmpty && !(hd & kPlaceBit) && vec_holds<W>(t, hd, hb, v)) st = 3;
        }
      }
      for (uint32_t j = 0; j < t.nhash && !st; ++j) {
        const uint64_t sl = hidx<false>(t, hb, j);
        st = vec_find_or_claim_seen<W>(t, t.slots + sl, t.slots[sl], ph, hb, v, keys, n);
        if (st == 1) loc = sl;
      }
      claimed = st == 1;
      leftover = st == 0;                        // every candidate taken: the evict kernel decides
      nnew += claimed ? 1u : 0u;
      if (out && !leftover) out[i] = claimed ? 1 : 0;
    } else if (i < end) {
      uint64_t v[W];
      load_vec<W>(keys + i * W, v);
      hb = vec_hash<W>(v, t.vseed) >> kArenaBits;
      const uint64_t ph = (hb << kArenaBits) | kPlaceBit | i;
      int st = 0;
      uint64_t b = 0;
      for (uint32_t q = 0; q < steps && !st; ++q) {
        b = vec_bucket(t, hb, q, b);
        for (uint32_t c0 = 0; c0 < B && !st; c0 += 8) {
          uint64_t x[8];
          load8(t.slots + b * B + c0, x);
          for (uint32_t k = 0; k < 8 && !st; ++k) {
            st = vec_find_or_claim_seen<W>(t, t.slots + b * B + c0 + k, x[k], ph, hb, v, keys, n);
            if (st == 1) loc = b * B + c0 + k;
          }
        }
      }
      if (!st) {
        const uint32_t S = t.stash_slots;
        uint32_t p = stash_start(t, hb);
        for (uint32_t k = 0; k < S && !st; ++k) {
          st = vec_find_or_claim_seen<W>(t, t.stash + p, t.stash[p], ph, hb, v, keys, n);
          if (st == 1) {
            loc = nslots + p;
            add_agent(&t.ctr->stash_count, 1u);
          }
          p = (p + 1) & (S - 1);
        }
      }
      if (!st) {
        const uint32_t m = t.overflow_slots;
        uint32_t p = overflow_start(t, hb);
        for (uint32_t k = 0; k < m && !st; ++k) {
          st = vec_find_or_claim_seen<W>(t, t.overflow + p, t.overflow[p], ph, hb, v, keys, n);
          if (st == 1) {
            loc = nslots + t.stash_slots + p;
            add_agent(&t.ctr->overflow_count, 1u);
          }
          p = p + 1 == m ? 0 : p + 1;
        }
      }
      if (!st) add_agent(&t.ctr->lost, 1u);
      claimed = st == 1;
      nnew += claimed ? 1u : 0u;
      if (out) out[i] = claimed ? 1 : 0;
    }
    const bool listed = claimed || leftover;
    const uint64_t mm = ballot(listed);
    if (listed) {
      const uint64_t slot = begin + nlist + lanes_below(mm);
      s.wkey[slot] = claimed ? loc : kLeftover;
      s.wmeta[slot] = (hb << 33) | i;
    }
    nlist += (uint32_t)__popcll(mm);
  }
  if (lane == 0 && begin < n) s.wcnt[wave] = nlist;
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
}

__device__ __forceinline__ uint64_t* vec_location(const DevTable& t, uint64_t loc) {
  const uint64_t nslots = t.nrange * t.bucket_slots;
  if (loc < nslots) return t.slots + loc;
  loc -= nslots;
  if (loc < t.stash_slots) return t.stash + loc;
  return t.overflow + (loc - t.stash_slots);
}

// Kernel 2: the claimed slots get arena entries, the vectors' words and
// their final handles.
template <int W>
__global__ __launch_bounds__(kBlock) void vec_commit_kernel(DevTable t, const uint64_t* __restrict__ keys, uint64_t n,
                                                             CuckooScratch s) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t begin = wave * s.per_wave;
  const uint32_t cnt = begin < n ? s.wcnt[wave] : 0u;
  for (uint32_t e0 = 0; e0 < cnt; e0 += kWave) {
    const uint32_t e = e0 + (uint32_t)lane_id();
    const uint64_t loc = e < cnt ? s.wkey[begin + e] : ~0ull;
    const bool have = loc != ~0ull && loc != kLeftover;
    if (!ballot(have)) continue;
    const uint64_t idx = arena_take(t, have, wave);
    if (!have) continue;
    if (idx == ~0ull) {
      add_agent(&t.ctr->lost, 1u);               // cannot happen: every claimed location has an entry
      continue;
    }
    const uint64_t m = s.wmeta[begin + e];
    const uint64_t i = m & kBatchMask;
    uint64_t v[W];
    load_vec<W>(keys + i * W, v);
#pragma unroll
    for (int j = 0; j < W; j += 2)
      *reinterpret_cast<ulonglong2*>(t.arena + idx * W + j) = make_ulonglong2(v[j], v[j + 1]);
    store_coherent(vec_location(t, loc), ((m >> 33) << kArenaBits) | idx);
  }
}

template <int W>
__global__ __launch_bounds__(kBlock) void vec_query_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                            uint64_t n, uint8_t* __restrict__ out) {
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    uint64_t v[W];
    load_vec<W>(keys + i * W, v);
    const uint64_t H = vec_hash<W>(v, t.vseed);
    out[i] = vec_find<W>(t, H >> kArenaBits, v, sc, oc) ? 1 : 0;
  }
}

// Members: the arena entries named by the handles in `handles[0, nh)`.
template <int W>
__global__ __launch_bounds__(kBlock) void vec_dump_kernel(const uint64_t* __restrict__ handles, uint64_t nh,
                                                           const uint64_t* __restrict__ arena,
                                                           uint64_t* __restrict__ dst, uint64_t cap,
                                                           unsigned long long* count) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const int lane = lane_id();
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock + (threadIdx.x & ~63u); base < nh; base += stride) {
    const uint64_t i = base + lane;
    const uint64_t hd = i < nh ? handles[i] : kEmpty;
    const bool keep = hd != kEmpty && !(hd & kPlaceBit);
    const uint64_t m = ballot(keep);
    if (!m) continue;
    unsigned long long b = 0;
    if (lane == 0) b = add_agent(count, (unsigned long long)__popcll(m));
    b = shfl64(b, 0);
    if (keep) {
      const uint64_t pos = b + lanes_below(m);
      if (pos < cap) {
#pragma unroll
        for (int j = 0; j < W; ++j) dst[pos * W + j] = arena[handle_idx(hd) * W + j];
      }
    }
  }
}

}  // namespace ht
