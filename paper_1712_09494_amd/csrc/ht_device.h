// Device-side building blocks shared by the bucketed and Cuckoo kernels:
// the hash family, the table descriptor passed to kernels, wave64 helpers and
// agent-scope 64-bit atomics.  gfx950 (CDNA4) only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ht {

// Empty-slot marker.  The key with this value is stored in a per-table flag
// word instead of a slot.
constexpr uint64_t kEmpty = ~0ull;

// Table kinds (same values as HT_BUCKETED / HT_CUCKOO of the C ABI).
constexpr uint32_t HT_KIND_BUCKETED = 1;
constexpr uint32_t HT_KIND_CUCKOO = 2;

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr int kSpread = 16;          // hot counters are spread over 16 lines
constexpr int kLineWords = 16;       // 128-byte line = 16 words
constexpr int kMaxHash = 8;
constexpr int kArenaBits = 34;       // vector tables: arena index bits of a handle
constexpr int kChainBins = 64;       // eviction-chain histogram bins

// Table flags the kernels read (same values as the HT_FLAG_* of the C ABI).
constexpr uint32_t kFlagChainStats = 1u << 6;
constexpr uint32_t kFlagLookahead = 1u << 7;
constexpr uint32_t kFlagGroupQuery = 1u << 8;

// Hash family: h_j(k) = floor(mix64(k ^ s_j) * range / 2^64).
// mix64 is the splitmix64 finalizer (Steele, Lea & Flood 2014), a bijection
// on 64-bit words; the range reduction is the multiply-high map (Lemire
// 2019), so range need not be a power of two.  The constants s_j come from a
// splitmix64 stream of the table seed (the paper's "hash constants",
// Sec. 4.1 and Sec. 5); a rebuild draws new ones.
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// Counters kept in device memory.  Each spread counter occupies its own
// 128-byte line; readers sum the kSpread copies.
struct Counters {
  unsigned long long size[kSpread * kLineWords];       // keys stored in slots/stash
  unsigned long long evictions[kSpread * kLineWords];  // cuckoo evictions
  unsigned int sentinel;        // 1 when the all-ones key is a member
  unsigned int stash_count;     // keys in the stash
  unsigned int overflow_count;  // appends to the overflow list (may exceed its length)
  unsigned int lost;            // appends that found the overflow list full
  unsigned int pad[28];
  // vector tables: entries taken in each of the kSpread arena ranges (may
  // exceed the range size; the excess was never handed out)
  unsigned long long arena_next[kSpread * kLineWords];
  // Cuckoo eviction chains by number of exchanges (bin 0: chains that ended
  // in the stash; 1..kChainBins-1: exchanges, the last bin also counting
  // longer ones); kSpread copies, filled only under the chain-stats flag
  unsigned long long chain_hist[kSpread * kChainBins];
};

// Scripted hash row (test mode): key and its c hash values.
struct ScriptRow {
  uint64_t key;
  uint64_t h[kMaxHash];
};

// Table descriptor, passed by value to kernels.
struct DevTable {
  uint64_t* slots;          // nrange * bucket_slots words (bucketed) or nrange (cuckoo)
  uint64_t* stash;          // stash_slots words, open addressing
  uint64_t* overflow;       // overflow_slots words, append-only
  Counters* ctr;
  const ScriptRow* script;  // scripted hashes (test mode) or nullptr
  uint64_t nrange;          // range of h_j: bucket count or slot count
  uint64_t seed[kMaxHash];  // hash constants s_0..s_{c-1}
  uint64_t stash_seed;
  uint32_t nhash;
  uint32_t bucket_slots;
  uint32_t stash_slots;     // power of two
  uint32_t overflow_slots;
  uint32_t max_chain;
  uint32_t nscript;
  uint32_t flags;
  uint32_t kind;
  uint32_t walk;            // bucketed: extra consecutive buckets after h_c
  uint32_t lds;             // host side: dynamic LDS bytes per block at launch (ablation)
  uint64_t* arena;          // vector tables: member vectors, key_words words each
  uint64_t arena_cap;       // arena entries per range (kSpread ranges)
  uint64_t vseed;           // vector tables: seed of the vector hash
  uint32_t key_words;       // words per key (1: single-word keys)
  uint32_t pad_;
};

// Scratch of the Cuckoo find-or-put (owned by the table).
struct CuckooScratch {
  uint64_t* dset;        // deduplication set, dset_mask + 1 words, all empty when an evict kernel starts
  uint64_t dset_mask;
  uint64_t dset_seed;
  uint64_t* wkey;        // listed keys, per-wave regions
  uint64_t* wmeta;       // key index (scratch-set slot once the evict kernel has run)
  uint32_t* wcnt;        // listed keys per wave
  uint64_t per_wave;     // keys (and list room) per wave
  // Deferred scrub (single-table calls; NULL elsewhere): the evict kernel
  // records the set slots its winners took here instead of in wmeta, and the
  // next call's probe kernel empties them, so no third kernel runs.
  uint64_t* dirty;       // set slot per listed key (~0: none); wave w's at w * dirty_stride
  uint32_t* dirty_cnt;   // entries per wave
  uint64_t* dirty_desc;  // [0] = waves of the call that wrote them
  uint64_t dirty_stride; // entries per wave (>= per_wave)
};

template <bool SCRIPTED>
__device__ __forceinline__ uint64_t hidx(const DevTable& t, uint64_t k, uint32_t j) {
  if constexpr (SCRIPTED) {
    for (uint32_t r = 0; r < t.nscript; ++r)
      if (t.script[r].key == k) return t.script[r].h[j];
    return 0;
  } else {
    return mulhi64(mix64(k ^ t.seed[j]), t.nrange);
  }
}

// ---- wave64 helpers -------------------------------------------------------

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Value of `v` in lane `src` (per-lane source; backed by ds_bpermute).
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  const int addr = src << 2;
  uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v);
  uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t shfl32(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = shfl64(v, lane_id() ^ off);
    v += o;
  }
  return v;
}

// ---- agent-scope atomics on device memory --------------------------------

__device__ __forceinline__ uint64_t cas64(uint64_t* p, uint64_t expected, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return expected;   // value found at *p
}

__device__ __forceinline__ uint64_t exch64(uint64_t* p, uint64_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t load_coherent(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_coherent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T add_agent(T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two adjacent 64-bit words (16-byte aligned): two agent-scope atomic 8-byte
// loads (COHERENT) or one ordinary 16-byte load.  On gfx950 the agent scope
// adds no cache-control bits to a relaxed load, so the two differ only in
// load width; correctness never rests on a load being fresh (a stale empty
// slot is caught by the compare-and-swap result).
template <bool COHERENT>
__device__ __forceinline__ void load_pair(const uint64_t* p, uint64_t& a, uint64_t& b) {
  if constexpr (COHERENT) {
    a = load_coherent(p);
    b = load_coherent(p + 1);
  } else {
    const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(p);
    a = v.x;
    b = v.y;
  }
}

// Eight consecutive slots (64-byte aligned: bucket widths are multiples of
// 8 slots), four independent 16-byte loads in flight together.
__device__ __forceinline__ void load8(const uint64_t* p, uint64_t (&x)[8]) {
#pragma unroll
  for (int k = 0; k < 8; k += 2) {
    const ulonglong2 y = *reinterpret_cast<const ulonglong2*>(p + k);
    x[k] = y.x;
    x[k + 1] = y.y;
  }
}

// ---- stash and overflow list ---------------------------------------------
// The stash (Sec. 4.1, after Alcantara et al.) holds keys that could not be
// placed; it is open-addressed with linear probing so that a lookup costs one
// line in the common case.  When it is full the key is appended to the
// overflow list, which keeps it a member until the table is rebuilt.

__device__ __forceinline__ uint32_t stash_start(const DevTable& t, uint64_t k) {
  return (uint32_t)(mix64(k ^ t.stash_seed) & (uint64_t)(t.stash_slots - 1));
}

__device__ __forceinline__ bool overflow_contains(const DevTable& t, uint64_t k) {
  uint32_t n = t.ctr->overflow_count;
  if (n > t.overflow_slots) n = t.overflow_slots;
  for (uint32_t i = 0; i < n; ++i)
    if (t.overflow[i] == k) return true;
  return false;
}

// Insert `k` into the stash or, when the stash is full, the overflow list.
// Returns 1 when stored as a new member in the stash, 0 when already present,
// 2 when appended to the overflow list.  Single-lane operation.
__device__ inline uint32_t stash_put(const DevTable& t, uint64_t k) {
  const uint32_t S = t.stash_slots;
  uint32_t p = stash_start(t, k);
  for (uint32_t i = 0; i < S; ++i) {
    const uint64_t old = cas64(&t.stash[p], kEmpty, k);
    if (old == kEmpty) {
      add_agent(&t.ctr->stash_count, 1u);
      return 1;
    }
    if (old == k) return 0;
    p = (p + 1) & (S - 1);
  }
  if (t.ctr->overflow_count && overflow_contains(t, k)) return 0;
  const uint32_t pos = add_agent(&t.ctr->overflow_count, 1u);
  if (pos < t.overflow_slots) {
    store_coherent(&t.overflow[pos], k);
  } else {
    add_agent(&t.ctr->lost, 1u);
  }
  return 2;
}

// Membership in stash or overflow list (read-only phases; single lane).
__device__ inline bool stash_query(const DevTable& t, uint64_t k, uint32_t stash_count,
                                   uint32_t overflow_count) {
  if (stash_count) {
    const uint32_t S = t.stash_slots;
    uint32_t p = stash_start(t, k);
    for (uint32_t i = 0; i < S; ++i) {
      const uint64_t v = t.stash[p];
      if (v == k) return true;
      if (v == kEmpty) break;
      p = (p + 1) & (S - 1);
    }
  }
  if (overflow_count) {
    uint32_t n = overflow_count < t.overflow_slots ? overflow_count : t.overflow_slots;
    for (uint32_t i = 0; i < n; ++i)
      if (t.overflow[i] == k) return true;
  }
  return false;
}

// Sentinel key (all ones): membership is a flag word set by compare-and-swap,
// so exactly one caller sees it absent.
__device__ __forceinline__ uint32_t sentinel_put(const DevTable& t) {
  unsigned int expected = 0u;
  const bool won = __hip_atomic_compare_exchange_strong(&t.ctr->sentinel, &expected, 1u,
                                                        __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
  return won ? 1u : 0u;
}

// Add per-lane counts to a spread counter: one atomic per wave.
__device__ __forceinline__ void wave_count(unsigned long long* spread, unsigned long long v,
                                           uint32_t salt) {
  const unsigned long long s = wave_sum(v);
  if (lane_id() == 0 && s) add_agent(&spread[(salt % kSpread) * kLineWords], s);
}

}  // namespace ht
