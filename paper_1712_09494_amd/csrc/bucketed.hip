// Bucketed (GPUexplore-style) table: find-or-put and query kernels.
//
// Paper Sec. 4.2 / Fig. 4: a key is hashed with h_1 to a bucket; the whole
// bucket is read cooperatively, one slot share per lane; the lanes vote
// whether the key is already there and which slots are free; a free slot is
// written atomically; a lost race moves on to the next free slot; a full
// bucket moves on to h_2, ...; when all c buckets are full the table is full.
// Sec. 5.1.2 reduces the element to one word per key, as here.
//
// wave64 layout: a bucket of B 64-bit slots is read by a group of L = B/2
// lanes, each loading 16 bytes, so one wave serves 128/B keys per step
// (B = 16: a 128-byte line, 8 keys per wave).  Votes are 64-bit ballots cut
// to the group's L bits; the compare-and-swap is issued by the lane that owns
// the chosen slot and its result is broadcast to the group.
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
#include "ht_device.h"

namespace ht {

template <int B>
struct BucketGeo {
  static constexpr int L = B / 2;                                  // lanes per key
  static constexpr int G = kWave / L;                              // keys per wave step
  static constexpr uint64_t GMASK = (L >= 64) ? ~0ull : ((1ull << L) - 1);
};

// Find-or-put of one key per lane group.  Called by all 64 lanes of a wave;
// `k` and `active` are uniform within a group.  Returns 0/1/2 (see ht.h).
template <int B, bool SCRIPTED, bool COHERENT>
__device__ __forceinline__ uint32_t bucket_find_or_put(const DevTable& t, uint64_t k, bool active) {
  using Geo = BucketGeo<B>;
  constexpr int L = Geo::L;
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int g0 = lane - gl;                 // first lane of the group
  uint32_t res = 0;
  bool done = !active;
  if (active && k == kEmpty) {
    uint32_t won = 0;
    if (gl == 0) won = sentinel_put(t);
    res = shfl32(won, g0);
    done = true;
  }
  uint32_t j = 0;                           // position in the probe sequence
  uint64_t b = 0;                           // current bucket
  uint64_t v0 = kEmpty, v1 = kEmpty;
  uint64_t* bp = nullptr;
  bool need_load = true;
  while (ballot(!done)) {
    if (!done) {
      if (need_load) {
        b = j < t.nhash ? hidx<SCRIPTED>(t, k, j) : (b + 1 == t.nrange ? 0 : b + 1);
        bp = t.slots + b * (uint64_t)B;
        load_pair<COHERENT>(bp + 2 * gl, v0, v1);
        need_load = false;
      }
      const uint64_t eq = (ballot((v0 == k) | (v1 == k)) >> g0) & Geo::GMASK;
      if (eq) {
        res = 0;
        done = true;
      } else {
        const uint64_t e0 = (ballot(v0 == kEmpty) >> g0) & Geo::GMASK;
        const uint64_t e1 = (ballot(v1 == kEmpty) >> g0) & Geo::GMASK;
        const uint64_t ea = e0 | e1;
        if (ea == 0) {
          // bucket full: next bucket of the sequence, or the stash after it
          if (++j < t.nhash + t.walk) {
            need_load = true;
          } else {
            uint32_t r = 0;
            if (gl == 0) r = stash_put(t, k);
            res = shfl32(r, g0);
            done = true;
          }
        } else {
          const int lf = __builtin_ctzll(ea);
          const int which = ((e0 >> lf) & 1ull) ? 0 : 1;
          uint64_t old = 0;
          if (gl == lf) old = cas64(bp + 2 * lf + which, kEmpty, k);
          old = shfl64(old, g0 + lf);
          if (old == kEmpty) {
            res = 1;
            done = true;
          } else if (old == k) {
            res = 0;
            done = true;
          } else if (gl == lf) {
            if (which == 0) v0 = old; else v1 = old;   // patch the stale copy
          }
        }
      }
    }
  }
  return res;
}

// Query of one key per lane group (read-only; runs after all writers).
template <int B, bool SCRIPTED>
__device__ __forceinline__ uint32_t bucket_query(const DevTable& t, uint64_t k, bool active,
                                                 uint32_t stash_count, uint32_t overflow_count) {
  using Geo = BucketGeo<B>;
  constexpr int L = Geo::L;
  const int lane = lane_id();
  const int gl = lane & (L - 1);
  const int g0 = lane - gl;
  uint32_t res = 0;
  bool done = !active;
  if (active && k == kEmpty) {
    res = t.ctr->sentinel ? 1u : 0u;
    done = true;
  }
  uint32_t j = 0;
  uint64_t b = 0;
  while (ballot(!done)) {
    if (!done) {
      b = j < t.nhash ? hidx<SCRIPTED>(t, k, j) : (b + 1 == t.nrange ? 0 : b + 1);
      uint64_t v0, v1;
      load_pair<false>(t.slots + b * (uint64_t)B + 2 * gl, v0, v1);
      const uint64_t eq = (ballot((v0 == k) | (v1 == k)) >> g0) & Geo::GMASK;
      const uint64_t em = (ballot((v0 == kEmpty) | (v1 == kEmpty)) >> g0) & Geo::GMASK;
      if (eq) {
        res = 1;
        done = true;
      } else if (em) {
        res = 0;            // first non-full bucket: the key would be here
        done = true;
      } else if (++j >= t.nhash + t.walk) {
        uint32_t r = 0;
        if (gl == 0) r = stash_query(t, k, stash_count, overflow_count) ? 1u : 0u;
        res = shfl32(r, g0);
        done = true;
      }
    }
  }
  return res;
}

// Grid-stride find-or-put over n keys: each wave takes G keys per step.
template <int B, bool SCRIPTED, bool COHERENT>
__global__ __launch_bounds__(kBlock) void bucketed_fop_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                               uint64_t n, uint8_t* __restrict__ out) {
  using Geo = BucketGeo<B>;
  const int lane = lane_id();
  const int gl = lane & (Geo::L - 1);
  const int grp = lane / Geo::L;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  unsigned long long nnew = 0;
  for (uint64_t base = wave * Geo::G; base < n; base += nwaves * Geo::G) {
    const uint64_t i = base + grp;
    const bool active = i < n;
    const uint64_t k = active ? keys[i] : 0;
    const uint32_t r = bucket_find_or_put<B, SCRIPTED, COHERENT>(t, k, active);
    if (active && gl == 0) {
      if (out) out[i] = (uint8_t)r;
      nnew += (r == 1);
    }
  }
  wave_count(t.ctr->size, nnew, (uint32_t)wave);
}

template <int B, bool SCRIPTED>
__global__ __launch_bounds__(kBlock) void bucketed_query_kernel(DevTable t, const uint64_t* __restrict__ keys,
                                                                 uint64_t n, uint8_t* __restrict__ out) {
  using Geo = BucketGeo<B>;
  const int lane = lane_id();
  const int gl = lane & (Geo::L - 1);
  const int grp = lane / Geo::L;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  const uint32_t sc = t.ctr->stash_count;
  const uint32_t oc = t.ctr->overflow_count;
  for (uint64_t base = wave * Geo::G; base < n; base += nwaves * Geo::G) {
    const uint64_t i = base + grp;
    const bool active = i < n;
    const uint64_t k = active ? keys[i] : 0;
    const uint32_t r = bucket_query<B, SCRIPTED>(t, k, active, sc, oc);
    if (active && gl == 0) out[i] = (uint8_t)r;
  }
}

// ---- host launchers --------------------------------------------------------

template <int B, bool S>
static hipError_t launch_fop_b(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                               uint32_t grid, bool coherent, hipStream_t s) {
  if (coherent)
    hipLaunchKernelGGL((bucketed_fop_kernel<B, S, true>), dim3(grid), dim3(kBlock), 0, s, t, keys, n, out);
  else
    hipLaunchKernelGGL((bucketed_fop_kernel<B, S, false>), dim3(grid), dim3(kBlock), 0, s, t, keys, n, out);
  return hipGetLastError();
}

template <int B, bool S>
static hipError_t launch_query_b(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                                 uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((bucketed_query_kernel<B, S>), dim3(grid), dim3(kBlock), 0, s, t, keys, n, out);
  return hipGetLastError();
}

uint64_t bucketed_keys_per_wave(uint32_t B) { return 128 / B; }

hipError_t bucketed_find_or_put(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                                uint32_t grid, bool coherent, bool scripted, hipStream_t s) {
  switch (t.bucket_slots) {
    case 8:  return scripted ? launch_fop_b<8, true>(t, keys, n, out, grid, coherent, s)
                             : launch_fop_b<8, false>(t, keys, n, out, grid, coherent, s);
    case 16: return scripted ? launch_fop_b<16, true>(t, keys, n, out, grid, coherent, s)
                             : launch_fop_b<16, false>(t, keys, n, out, grid, coherent, s);
    case 32: return scripted ? launch_fop_b<32, true>(t, keys, n, out, grid, coherent, s)
                             : launch_fop_b<32, false>(t, keys, n, out, grid, coherent, s);
    case 64: return scripted ? launch_fop_b<64, true>(t, keys, n, out, grid, coherent, s)
                             : launch_fop_b<64, false>(t, keys, n, out, grid, coherent, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t bucketed_query(const DevTable& t, const uint64_t* keys, uint64_t n, uint8_t* out,
                          uint32_t grid, bool scripted, hipStream_t s) {
  switch (t.bucket_slots) {
    case 8:  return scripted ? launch_query_b<8, true>(t, keys, n, out, grid, s)
                             : launch_query_b<8, false>(t, keys, n, out, grid, s);
    case 16: return scripted ? launch_query_b<16, true>(t, keys, n, out, grid, s)
                             : launch_query_b<16, false>(t, keys, n, out, grid, s);
    case 32: return scripted ? launch_query_b<32, true>(t, keys, n, out, grid, s)
                             : launch_query_b<32, false>(t, keys, n, out, grid, s);
    case 64: return scripted ? launch_query_b<64, true>(t, keys, n, out, grid, s)
                             : launch_query_b<64, false>(t, keys, n, out, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ht
