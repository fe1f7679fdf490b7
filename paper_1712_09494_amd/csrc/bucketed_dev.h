// Bucketed (GPUexplore-style) table: find-or-put and query kernels.
//
// Paper Sec. 4.2 / Fig. 4: a key is hashed with h_1 to a bucket; the whole
// bucket is read cooperatively, one slot share per lane; the lanes vote
// whether the key is already there and which slots are free; a free slot is
// written atomically; a lost race moves on to the next free slot; a full
// bucket moves on to h_2, ...; when all c buckets are full the table is full.
// Sec. 5.1.2 reduces the element to one word per key, as here.
//
// wave64 layout: a bucket of B 64-bit slots is read by a group of L lanes.
// Find-or-put: L = B/4, each lane loading four slots with two 16-byte loads,
// so one wave serves 256/B keys per step (B = 8: 32 keys).  Lane-group query:
// L = B/2, one 16-byte load per lane.  Votes are 64-bit ballots cut to the
// group's L bits; the compare-and-swap is issued by the lane that owns
// the chosen slot and its result is broadcast to the group.  Each group keeps
// R keys in flight: every loop turn first issues the bucket loads of all R
// keys, then evaluates them, then issues all their compare-and-swaps, then
// resolves them, so the memory latencies of the R keys overlap.
//
// Placement protocol for one-word keys: a group always writes the lowest
// slot that it sees empty.  Slots change only from empty to a key, so
// occupied slots of a bucket form a prefix, a bucket seen full stays full,
// and two inserters of the same key walk the same buckets and meet at the
// same slot.  A stale empty slot is fixed by the compare-and-swap result (the
// group patches its copy and moves on), so no reload is needed.  A query may
// stop at the first bucket that is not full.
//
// Probe sequence: the buckets of h_1..h_c, then (unless the table keeps the
// paper's "full after c buckets" rule) up to `walk` consecutive buckets after
// h_c's bucket, then the stash.  The sequence depends only on the key, so the
// invariants above hold along it.  With c = 3 and B = 16 the c buckets alone
// reject about 0.7% of keys at load factor 0.9; the walk takes them.
#pragma once
#include "ht_device.h"

namespace ht {

template <int B>
struct BucketGeo {
  static constexpr int L = B / 2;                                  // lanes per key
  static constexpr int G = kWave / L;                              // key groups per wave
  static constexpr uint64_t GMASK = (L >= 64) ? ~0ull : ((1ull << L) - 1);
};

__device__ __forceinline__ uint64_t group_bits(bool p, int g0, uint64_t gmask) {
  return (ballot(p) >> g0) & gmask;
}

// Geometry of a bucket of B slots; B is a compile-time constant, or 0 to take
// it from the table at run time (one code path for every width).
template <int B>
__device__ __forceinline__ uint32_t bucket_width(const DevTable& t) {
  return B ? (uint32_t)B : t.bucket_slots;
}

__device__ __forceinline__ uint64_t lanes_mask(uint32_t L) { return L >= 64 ? ~0ull : ((1ull << L) - 1); }

// Bucket number of position j of key k's probe sequence; `prev` is the bucket
// of position j-1.
template <bool SCRIPTED>
__device__ __forceinline__ uint64_t probe_bucket(const DevTable& t, uint64_t k, uint32_t j, uint64_t prev) {
  if (j < t.nhash) return hidx<SCRIPTED>(t, k, j);
  return prev + 1 == t.nrange ? 0 : prev + 1;
}

// Find-or-put of R keys per lane group.  Called by all 64 lanes of a wave;
// k[r] and active[r] are uniform within a group.  res[r] gets 0/1/2 (ht.h).
// A group has L = B / SPL lanes, each holding SPL consecutive slots of the
// bucket (SPL = 2: one 16-byte load per lane; SPL = 4: two).
template <int B, int SPL, int R, bool SCRIPTED, bool COHERENT>
__device__ __forceinline__ void bucket_find_or_put(const DevTable& t, const uint64_t (&k)[R],
                                                   const bool (&active)[R], uint32_t (&res)[R]) {
  static_assert(SPL == 2 || SPL == 4, "slots per lane");
  const uint32_t Bw = bucket_width<B>(t);
  const int L = (int)(Bw / SPL);
  const uint64_t gm = lanes_mask((uint32_t)L);
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int g0 = lane - gl;                 // first lane of the group
  const uint32_t nseq = t.nhash + t.walk;   // probe sequence length
  bool done[R], need[R];
  uint32_t j[R];
  uint64_t b[R], v[R][SPL];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    res[r] = 0;
    done[r] = !active[r];
    need[r] = true;
    j[r] = 0;
    b[r] = 0;
#pragma unroll
    for (int q = 0; q < SPL; ++q) v[r][q] = kEmpty;
    if (active[r] && k[r] == kEmpty) {     // all-ones key: flag word
      uint32_t won = 0;
      if (gl == 0) won = sentinel_put(t);
      res[r] = shfl32(won, g0);
      done[r] = true;
    }
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) any |= !done[r];
    if (!ballot(any)) break;
    // 1. issue the bucket loads
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!done[r] && need[r]) {
        b[r] = probe_bucket<SCRIPTED>(t, k[r], j[r], b[r]);
        const uint64_t* p = t.slots + b[r] * (uint64_t)Bw + SPL * gl;
#pragma unroll
        for (int q = 0; q < SPL; q += 2) load_pair<COHERENT>(p + q, v[r][q], v[r][q + 1]);
        need[r] = false;
      }
    }
    // 2. vote: present / full / lowest empty slot (lowest lane with an empty
    //    slot, then its lowest empty slot)
    int tgt[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      tgt[r] = -1;
      if (!done[r]) {
        bool has = false;
#pragma unroll
        for (int q = 0; q < SPL; ++q) has |= v[r][q] == k[r];
        if (group_bits(has, g0, gm)) {
          res[r] = 0;
          done[r] = true;
        } else {
          uint64_t e[SPL];
          uint64_t ea = 0;
#pragma unroll
          for (int q = 0; q < SPL; ++q) {
            e[q] = group_bits(v[r][q] == kEmpty, g0, gm);
            ea |= e[q];
          }
          if (ea == 0) {
            if (++j[r] < nseq) {
              need[r] = true;            // bucket full: next bucket of the sequence
            } else {
              uint32_t s = 0;
              if (gl == 0) s = stash_put(t, k[r]);
              res[r] = shfl32(s, g0);
              done[r] = true;
            }
          } else {
            const int lf = __builtin_ctzll(ea);
            int q0 = SPL - 1;
#pragma unroll
            for (int q = SPL - 2; q >= 0; --q) q0 = ((e[q] >> lf) & 1ull) ? q : q0;
            tgt[r] = SPL * lf + q0;
          }
        }
      }
    }
    // 3. issue the compare-and-swaps (lane owning the chosen slot)
    uint64_t old[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      old[r] = 0;
      if (tgt[r] >= 0 && gl == tgt[r] / SPL)
        old[r] = cas64(t.slots + b[r] * (uint64_t)Bw + tgt[r], kEmpty, k[r]);
    }
    // 4. resolve: won, found, or patch the stale copy and retry
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (tgt[r] >= 0) {
        const int owner = tgt[r] / SPL;
        const uint64_t o = shfl64(old[r], g0 + owner);
        if (o == kEmpty) {
          res[r] = 1;
          done[r] = true;
        } else if (o == k[r]) {
          res[r] = 0;
          done[r] = true;
        } else if (gl == owner) {
          const int qq = tgt[r] % SPL;
#pragma unroll
          for (int q = 0; q < SPL; ++q) v[r][q] = q == qq ? o : v[r][q];
        }
      }
    }
  }
}

// Query of R keys per lane group (read-only; runs after all writers).
template <int B, int R, bool SCRIPTED>
__device__ __forceinline__ void bucket_query(const DevTable& t, const uint64_t (&k)[R], const bool (&active)[R],
                                             uint32_t stash_count, uint32_t overflow_count, uint32_t (&res)[R]) {
  const uint32_t Bw = bucket_width<B>(t);
  const int L = (int)(Bw / 2);
  const uint64_t gm = lanes_mask((uint32_t)L);
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int g0 = lane - gl;
  const uint32_t nseq = t.nhash + t.walk;
  bool done[R];
  uint32_t j[R];
  uint64_t b[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    res[r] = 0;
    done[r] = !active[r];
    j[r] = 0;
    b[r] = 0;
    if (active[r] && k[r] == kEmpty) {
      res[r] = t.ctr->sentinel ? 1u : 0u;
      done[r] = true;
    }
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int r = 0; r < R; ++r) any |= !done[r];
    if (!ballot(any)) break;
    uint64_t v0[R], v1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v0[r] = v1[r] = kEmpty;
      if (!done[r]) {
        b[r] = probe_bucket<SCRIPTED>(t, k[r], j[r], b[r]);
        load_pair<false>(t.slots + b[r] * (uint64_t)Bw + 2 * gl, v0[r], v1[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!done[r]) {
        const uint64_t eq = group_bits((v0[r] == k[r]) | (v1[r] == k[r]), g0, gm);
        const uint64_t em = group_bits((v0[r] == kEmpty) | (v1[r] == kEmpty), g0, gm);
        if (eq) {
          res[r] = 1;
          done[r] = true;
        } else if (em) {
          res[r] = 0;            // first non-full bucket: the key would be here
          done[r] = true;
        } else if (++j[r] >= nseq) {
          uint32_t s = 0;
          if (gl == 0) s = stash_query(t, k[r], stash_count, overflow_count) ? 1u : 0u;
          res[r] = shfl32(s, g0);
          done[r] = true;
        }
      }
    }
  }
}

// One wave, one turn: find-or-put of keys base .. base + G*R (clipped at
// end); group g handles keys base + r*G + g (consecutive groups read
// consecutive keys).  Returns (in group leaders) the number of new keys.
template <int B, int SPL, int R, bool SCRIPTED, bool COHERENT>
__device__ __forceinline__ unsigned long long bucketed_fop_turn(const DevTable& t, const uint64_t* __restrict__ keys,
                                                                uint64_t base, uint64_t end,
                                                                uint8_t* __restrict__ out) {
  const uint32_t L = bucket_width<B>(t) / SPL;
  const uint32_t G = kWave / L;
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int grp = lane / L;
  uint64_t k[R];
  bool act[R];
  uint32_t res[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint64_t i = base + (uint64_t)r * G + grp;
    act[r] = i < end;
    k[r] = act[r] ? keys[i] : 0;
  }
  bucket_find_or_put<B, SPL, R, SCRIPTED, COHERENT>(t, k, act, res);
  unsigned long long nnew = 0;
  if (gl == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (act[r]) {
        if (out) out[base + (uint64_t)r * G + grp] = (uint8_t)res[r];
        nnew += (res[r] == 1);
      }
    }
  }
  return nnew;
}

// Grid-stride find-or-put: wave w takes turns w, w + nwaves, ...
template <int B, int SPL, int R, bool SCRIPTED, bool COHERENT>
__global__ __launch_bounds__(kBlock) void bucketed_fop_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out) {
  constexpr uint64_t PER = (uint64_t)(kWave / (B / SPL)) * R;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  unsigned long long nnew = 0;
  for (uint64_t base = wave * PER; base < n; base += nwaves * PER)
    nnew += bucketed_fop_turn<B, SPL, R, SCRIPTED, COHERENT>(t, keys, base, n, out);
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
}

template <int B, int R, bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void bucketed_query_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                                 uint64_t n, uint8_t* __restrict__ out) {
  using Geo = BucketGeo<B>;
  constexpr uint64_t PER = (uint64_t)Geo::G * R;
  const int lane = lane_id();
  const int gl = lane & (Geo::L - 1);
  const int grp = lane / Geo::L;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  for (uint64_t base = wave * PER; base < n; base += nwaves * PER) {
    uint64_t k[R];
    bool act[R];
    uint32_t res[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + (uint64_t)r * Geo::G + grp;
      act[r] = i < n;
      k[r] = act[r] ? keys[i] : 0;
    }
    bucket_query<B, R, SCRIPTED>(t, k, act, sc, oc, res);
    if (gl == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        if (act[r]) out[base + (uint64_t)r * Geo::G + grp] = (uint8_t)res[r];
    }
  }
}

// ---- one lane per key (HT_FLAG_BUCKETED_ONE_LANE) ---------------------------
// The same table and probe sequence, but each lane probes whole buckets for
// its own key: eight slots per step (four independent 16-byte loads), then
// the first empty slot is compare-and-swapped.  Copies of a key read the same
// slots in the same order, so they meet at one slot exactly as with a lane
// group.  A wave serves 64 keys per turn instead of 128/B: less work issued
// per key, which pays where hits dominate and the table sits in cache.

template <bool SCRIPTED>
__device__ __forceinline__ uint32_t lane_find_or_put(const DevTable& t, uint64_t k) {
  if (k == kEmpty) return sentinel_put(t);
  const uint32_t B = t.bucket_slots;
  const uint32_t nseq = t.nhash + t.walk;
  uint64_t b = 0;
  for (uint32_t j = 0; j < nseq; ++j) {
    b = probe_bucket<SCRIPTED>(t, k, j, b);
    uint64_t* bk = t.slots + b * B;
    for (uint32_t c0 = 0; c0 < B; c0 += 8) {
      uint64_t x[8];
      load8(bk + c0, x);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        uint64_t v = x[q];
        if (v == kEmpty) v = cas64(bk + c0 + q, kEmpty, k);
        if (v == kEmpty) return 1;     // placed
        if (v == k) return 0;          // present (or another copy won this slot)
      }
    }
  }
  return stash_put(t, k);              // every bucket of the sequence full
}

template <bool SCRIPTED>
__device__ __forceinline__ uint32_t lane_query(const DevTable& t, uint64_t k, uint32_t sc, uint32_t oc) {
  if (k == kEmpty) return t.ctr->sentinel ? 1u : 0u;
  const uint32_t B = t.bucket_slots;
  const uint32_t nseq = t.nhash + t.walk;
  uint64_t b = 0;
  for (uint32_t j = 0; j < nseq; ++j) {
    b = probe_bucket<SCRIPTED>(t, k, j, b);
    const uint64_t* bk = t.slots + b * B;
    for (uint32_t c0 = 0; c0 < B; c0 += 8) {
      uint64_t x[8];
      load8(bk + c0, x);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (x[q] == k) return 1;
        if (x[q] == kEmpty) return 0;  // slots fill as a prefix and a full sequence precedes the stash
      }
    }
  }
  return (sc | oc) && stash_query(t, k, sc, oc) ? 1u : 0u;
}

template <bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void bucketed_lane_fop_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                                    uint64_t n, uint8_t* __restrict__ out) {
  const uint64_t first = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  unsigned long long nnew = 0;
  for (uint64_t i = first; i < n; i += stride) {
    const uint32_t res = lane_find_or_put<SCRIPTED>(t, keys[i]);
    if (out) out[i] = (uint8_t)res;
    nnew += res == 1;
  }
  wave_count(t.ctr->size, nnew, (uint32_t)(first / kWave));
}

template <bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void bucketed_lane_query_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                                      uint64_t n, uint8_t* __restrict__ out) {
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    out[i] = (uint8_t)lane_query<SCRIPTED>(t, keys[i], sc, oc);
}

}  // namespace ht
