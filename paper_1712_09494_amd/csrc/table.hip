// Host runtime and C ABI: table storage, hash constants, launch shapes,
// scratch management, dump/rebuild and the argument checks of every entry
// point declared in include/ht.h.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "multi.h"
#include "runtime.h"

namespace ht {
// kernels (bucketed.hip, cuckoo.hip, util.hip, multi.hip)
hipError_t bucketed_find_or_put(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, uint32_t, bool,
                                bool, hipStream_t);
hipError_t bucketed_query(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, uint32_t, bool,
                          hipStream_t);
uint64_t bucketed_keys_per_wave(uint32_t B, uint32_t R, uint32_t spl);
// slots each lane of a find-or-put lane group holds (bucketed.hip)
constexpr uint32_t kFopSlotsPerLane = 4;
hipError_t bucketed_lane_find_or_put(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, bool,
                                     hipStream_t);
hipError_t bucketed_lane_query(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, bool, hipStream_t);
hipError_t cuckoo_query(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, uint32_t, bool,
                        hipStream_t);
hipError_t cuckoo_probe(const DevTable&, const uint64_t*, uint64_t, uint8_t*, const CuckooScratch&, uint32_t,
                        uint32_t, bool, bool, hipStream_t);
hipError_t cuckoo_evict(const DevTable&, uint64_t, uint8_t*, const CuckooScratch&, uint32_t, uint32_t, bool,
                        hipStream_t);
hipError_t cuckoo_single_pass(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, bool, hipStream_t);
hipError_t cuckoo_scrub(uint64_t, const CuckooScratch&, uint32_t, hipStream_t);
hipError_t vec_evict(const DevTable&, const uint64_t*, uint64_t, uint8_t*, const CuckooScratch&, uint32_t,
                      uint32_t, hipStream_t);
hipError_t vec_find_or_claim(const DevTable&, const uint64_t*, uint64_t, uint8_t*, const CuckooScratch&, uint32_t,
                             uint32_t, hipStream_t);
hipError_t vec_commit(const DevTable&, const uint64_t*, uint64_t, const CuckooScratch&, uint32_t, uint32_t,
                      hipStream_t);
hipError_t vec_query(const DevTable&, const uint64_t*, uint64_t, uint8_t*, uint32_t, uint32_t, hipStream_t);
hipError_t vec_dump(const uint64_t*, uint64_t, const uint64_t*, uint64_t*, uint64_t, unsigned long long*, uint32_t,
                    uint32_t, hipStream_t);
hipError_t fill_words(uint64_t*, uint64_t, uint64_t, hipStream_t);
hipError_t zero_words(uint32_t*, uint64_t, hipStream_t);
hipError_t compact_words(const uint64_t*, uint64_t, uint64_t*, uint64_t, unsigned long long*, uint32_t,
                         hipStream_t);
hipError_t probe_copy(const uint64_t*, uint64_t*, uint64_t, uint32_t, hipStream_t);
hipError_t probe_gather(const uint64_t*, uint64_t, uint64_t, uint32_t, uint64_t, uint64_t*, uint32_t,
                        hipStream_t);
hipError_t probe_cas(uint64_t*, uint64_t, uint64_t, uint64_t, uint32_t, hipStream_t);
hipError_t probe_mix(const uint64_t*, uint8_t*, uint64_t, uint64_t*, uint64_t, uint32_t, uint32_t, bool, uint64_t,
                     uint32_t, hipStream_t);
}  // namespace ht

using namespace ht;
using namespace ht_rt;

namespace ht_rt {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return HT_EHIP;
}


// Compute units of the current device (cached per device id).
uint32_t device_cus(int dev) {
  static std::mutex mu;
  static std::vector<uint32_t> cache;
  std::lock_guard<std::mutex> lk(mu);
  if (dev < 0) dev = 0;
  if ((size_t)dev >= cache.size()) cache.resize(dev + 1, 0);
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    cache[dev] = (uint32_t)cus;
  }
  return cache[dev];
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint32_t ceil_log2(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x && l < 63) ++l;
  return l;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- kernel timing (measurement aid) ---------------------------------------
// When enabled, each library kernel launch is bracketed by two HIP events
// recorded on the launch stream; ht_timing_report resolves them.
struct PendingTiming {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<PendingTiming> g_pending;
std::map<std::string, std::pair<uint64_t, double>> g_acc;   // name -> (launches, total ms)

// Set while the allocation-free call runs: its launches create no events.
thread_local bool g_quiet = false;

struct KernelTimer {
  PendingTiming p{};
  bool on = false;
  hipStream_t s;
  KernelTimer(const char* name, hipStream_t st) : s(st) {
    if (g_quiet) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return;
    p.name = name;
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return;
    on = hipEventRecord(p.a, s) == hipSuccess;
  }
  ~KernelTimer() {
    if (!on) return;
    if (hipEventRecord(p.b, s) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back(p);
  }
};

void resolve_timings() {
  std::lock_guard<std::mutex> lk(g_tmu);
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& e = g_acc[p.name];
      e.first += 1;
      e.second += ms;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}

}  // namespace ht_rt


struct ht_multi_plan {
  struct VecJob {             // a state-vector table: its own kernels, after the merged launches
    ht_table* t;
    const uint64_t* keys;
    uint64_t n;
    uint8_t* out;
  };
  std::vector<ht_table*> tables;
  MultiPlanDev dev;           // bucketed persistent launch + Cuckoo phase launches
  std::vector<VecJob> vec;
  uint32_t grid = 0;
};

namespace ht_rt {

uint32_t max_blocks(const ht_table* t) { return t->cus * 8; }

// Grid of the one-lane-per-key kernels that mix random reads with
// compare-and-swaps (the Cuckoo probe phases, the state-vector kernels, the
// one-lane bucketed find-or-put and fused BFS levels): 6
// blocks (24 waves) per compute unit, which keeps fewer requests queued at
// the memory than the full 8.  Measured on the 2^20-key batches of a
// 2^26-key fill at c = 4 (probe kernel, average per launch): 73.9 us at 8
// blocks per unit, 67.7 at 7, 66.6 at 6, 70.2 at 5, 67.5 at 4; 2^24 state
// vectors in batches of 2^20: 5-7% faster at 6 than at 8 for both designs
// and W = 2, 4.  The bucketed lane-group kernel is fastest at 8 (two slots
// per lane: fill 3.88 ms at 8, 4.05 at 7, 4.33 at 6; four slots per lane at
// B = 64: 8.75 at 8, 10.3 at 6), and so is the many-table bucketed fill (256
// tables: 5.73 ms at 8, 5.92 at 6).
uint32_t atomic_grid_blocks(const ht_table* t) { return t->cus * 6; }

bool is_scripted(const ht_table* t) { return (t->cfg.flags & HT_FLAG_SCRIPTED_HASH) != 0; }

void draw_constants(ht_table* t) {
  for (uint32_t j = 0; j < kMaxHash; ++j) t->dev.seed[j] = t->rng.next();
  t->dev.stash_seed = t->rng.next();
  t->dset_seed = t->rng.next();
  t->dev.vseed = t->rng.next();
}

int free_storage(ht_table* t) {
  if (t->storage) {
    (void)hipFree(t->storage);
    t->storage = nullptr;
  }
  return HT_OK;
}

// Allocate slots/stash/overflow/counters for t->nslots and clear them.
int alloc_storage(ht_table* t) {
  const size_t slot_bytes = align_up(t->nslots * 8, 256);
  const size_t stash_bytes = align_up((size_t)t->dev.stash_slots * 8, 256);
  const size_t ovf_bytes = align_up((size_t)t->dev.overflow_slots * 8, 256);
  const size_t ctr_bytes = align_up(sizeof(Counters), 256);
  const size_t misc_bytes = 256;
  const uint32_t W = t->cfg.key_words;
  // vector arena: kSpread ranges that together hold every possible member
  const uint64_t members = t->nslots + t->dev.stash_slots + t->dev.overflow_slots;
  t->dev.arena_cap = W > 1 ? (members + kSpread - 1) / kSpread : 0;
  const size_t arena_bytes = align_up(t->dev.arena_cap * kSpread * W * 8, 256);
  const size_t total = slot_bytes + stash_bytes + ovf_bytes + ctr_bytes + misc_bytes + arena_bytes;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, total);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HT_ENOMEM, std::string("hipMalloc of table storage failed: ") + hipGetErrorString(e));
  }
  char* c = static_cast<char*>(p);
  t->storage = p;
  t->dev.slots = reinterpret_cast<uint64_t*>(c);
  t->dev.stash = reinterpret_cast<uint64_t*>(c + slot_bytes);
  t->dev.overflow = reinterpret_cast<uint64_t*>(c + slot_bytes + stash_bytes);
  t->dev.ctr = reinterpret_cast<Counters*>(c + slot_bytes + stash_bytes + ovf_bytes);
  t->misc = reinterpret_cast<unsigned long long*>(c + slot_bytes + stash_bytes + ovf_bytes + ctr_bytes);
  t->dev.arena = W > 1 ? reinterpret_cast<uint64_t*>(c + slot_bytes + stash_bytes + ovf_bytes + ctr_bytes +
                                                     misc_bytes)
                       : nullptr;
  return HT_OK;
}

int clear_async(ht_table* t, hipStream_t s) {
  KernelTimer kt("clear", s);
  HT_HIP(fill_words(t->dev.slots, t->nslots, kEmpty, s));
  HT_HIP(fill_words(t->dev.stash, t->dev.stash_slots, kEmpty, s));
  HT_HIP(fill_words(t->dev.overflow, t->dev.overflow_slots, kEmpty, s));
  HT_HIP(zero_words(reinterpret_cast<uint32_t*>(t->dev.ctr), sizeof(Counters) / 4, s));
  return HT_OK;
}

int free_scratch(ht_table* t) {
  if (t->dset) (void)hipFree(t->dset);
  t->dset = nullptr;
  t->wkey = nullptr;
  t->wmeta = nullptr;
  t->wcnt = nullptr;
  t->dset_defer = nullptr;
  t->dirty = nullptr;
  t->dirty_cnt = nullptr;
  t->dirty_desc = nullptr;
  t->dirty_stride = 0;
  t->scratch_n = 0;
  t->dset_slots = 0;
  return HT_OK;
}

// Find-or-put scratch (Cuckoo and vector tables) for batches up to n keys (one allocation).
int reserve_scratch(ht_table* t, uint64_t n) {
  if (t->cfg.kind != HT_CUCKOO && t->cfg.key_words <= 1) return HT_OK;
  if (n <= t->scratch_n && t->dset) return HT_OK;
  if (n < 1024) n = 1024;
  HT_HIP(hipDeviceSynchronize());
  free_scratch(t);
  // the deduplication set serves Cuckoo tables only (bucketed vector tables
  // deduplicate in their slots); keep a token one otherwise
  const uint64_t ds = t->cfg.kind == HT_CUCKOO ? pow2_at_least(2 * n) : 64;
  const uint64_t nw = (uint64_t)max_blocks(t) * (kBlock / kWave);
  const size_t b_dset = align_up(ds * 8, 256);
  const size_t b_k = align_up(n * 8, 256);
  const size_t b_c = align_up(nw * 4, 256);   // wcnt
  // single-word Cuckoo tables: a second set, the slot record (a fixed
  // stride per wave, at least the keys per wave of any probe launch: 64 * R
  // <= 256 below its full grid, n / waves at it) and its count per wave for
  // the deferred scrub, and a word with the record's wave count
  const bool defer = t->cfg.kind == HT_CUCKOO && t->cfg.key_words <= 1;
  const uint64_t pw = (uint64_t)atomic_grid_blocks(t) * (kBlock / kWave);
  const uint64_t stride = std::max<uint64_t>(256, (n + pw - 1) / pw);
  const size_t b_rec = align_up(nw * stride * 8, 256);
  const size_t b_defer = defer ? b_dset + b_rec + b_c + 256 : 0;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, b_dset + 2 * b_k + b_c + b_defer);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HT_ENOMEM, std::string("hipMalloc of find-or-put scratch failed: ") + hipGetErrorString(e));
  }
  char* c = static_cast<char*>(p);
  t->dset = reinterpret_cast<uint64_t*>(c);
  t->wkey = reinterpret_cast<uint64_t*>(c + b_dset);
  t->wmeta = reinterpret_cast<uint64_t*>(c + b_dset + b_k);
  t->wcnt = reinterpret_cast<uint32_t*>(c + b_dset + 2 * b_k);
  if (defer) {
    char* d = c + b_dset + 2 * b_k + b_c;
    t->dset_defer = reinterpret_cast<uint64_t*>(d);
    t->dirty = reinterpret_cast<uint64_t*>(d + b_dset);
    t->dirty_cnt = reinterpret_cast<uint32_t*>(d + b_dset + b_rec);
    t->dirty_desc = reinterpret_cast<uint64_t*>(d + b_dset + b_rec + b_c);
    t->dirty_stride = stride;
  }
  t->dset_slots = ds;
  t->scratch_n = n;
  HT_HIP(fill_words(t->dset, ds, kEmpty, nullptr));
  if (defer) {
    HT_HIP(fill_words(t->dset_defer, ds, kEmpty, nullptr));
    HT_HIP(zero_words(reinterpret_cast<uint32_t*>(t->dirty_desc), 4, nullptr));   // no record yet
  }
  HT_HIP(hipDeviceSynchronize());
  return HT_OK;
}

int validate_config(const ht_config* c) {
  if (!c) return fail(HT_EINVAL, "config is NULL");
  if (c->kind != HT_BUCKETED && c->kind != HT_CUCKOO) return fail(HT_EINVAL, "kind must be HT_BUCKETED or HT_CUCKOO");
  if (c->nhash < 1 || c->nhash > kMaxHash) return fail(HT_EINVAL, "nhash must be in 1..8");
  if (c->capacity == 0) return fail(HT_EINVAL, "capacity must be > 0");
  if (c->capacity > (1ull << 40)) return fail(HT_EINVAL, "capacity above 2^40 slots");
  if (c->kind == HT_BUCKETED) {
    const uint32_t b = c->bucket_slots;
    if (b != 0 && b != 8 && b != 16 && b != 32 && b != 64)
      return fail(HT_EINVAL, "bucket_slots must be 8, 16, 32 or 64");
  }
  if (c->stash_slots && (c->stash_slots & (c->stash_slots - 1)))
    return fail(HT_EINVAL, "stash_slots must be a power of two");
  if (c->stash_slots > 65536) return fail(HT_EINVAL, "stash_slots above 65536");
  if (c->keys_per_group != 0 && c->keys_per_group != 1 && c->keys_per_group != 2 && c->keys_per_group != 4)
    return fail(HT_EINVAL, "keys_per_group must be 0, 1, 2 or 4");
  if (c->flags & ~(uint32_t)(HT_FLAG_CUCKOO_PAPER_ORDER | HT_FLAG_BUCKETED_ATOMIC_LOADS | HT_FLAG_SCRIPTED_HASH |
                             HT_FLAG_BUCKETED_PAPER_FULL | HT_FLAG_CUCKOO_SINGLE_PASS |
                             HT_FLAG_BUCKETED_ONE_LANE | HT_FLAG_CHAIN_STATS | HT_FLAG_CUCKOO_LOOKAHEAD |
                             HT_FLAG_BUCKETED_GROUP_QUERY))
    return fail(HT_EINVAL, "unknown flag bits");
  if ((c->flags & HT_FLAG_CUCKOO_LOOKAHEAD) && (c->flags & HT_FLAG_CUCKOO_PAPER_ORDER))
    return fail(HT_EINVAL, "the lookahead flag changes the paper-order insertion; use one of them");
  if ((c->flags & HT_FLAG_BUCKETED_ONE_LANE) && (c->kind != HT_BUCKETED || c->key_words > 1))
    return fail(HT_EINVAL, "the one-lane flag is for bucketed tables of single-word keys");
  if ((c->flags & HT_FLAG_CUCKOO_SINGLE_PASS) && (c->kind != HT_CUCKOO || c->key_words > 1))
    return fail(HT_EINVAL, "the single-pass flag is for Cuckoo tables of single-word keys");
  if (c->key_words != 0 && c->key_words != 1 && c->key_words != 2 && c->key_words != 4)
    return fail(HT_EINVAL, "key_words must be 0, 1, 2 or 4");
  if (c->reserved) return fail(HT_EINVAL, "reserved must be 0");
  if (c->key_words > 1) {
    if (c->flags & HT_FLAG_SCRIPTED_HASH) return fail(HT_EINVAL, "scripted hashes need single-word keys");
    if (c->capacity + 65536ull + (c->overflow_slots ? c->overflow_slots : 65536u) + 64 >= (1ull << (kArenaBits - 1)))
      return fail(HT_EINVAL, "vector table capacity above 2^33 entries");
  }
  if (c->lds_bytes) {
    int dev = 0, lim = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lim = 65536;
    if (c->lds_bytes > (uint32_t)lim) return fail(HT_EINVAL, "lds_bytes above the device's LDS per block");
  }
  return HT_OK;
}

// Geometry and defaults from a validated config.
void setup_geometry(ht_table* t) {
  ht_config& c = t->cfg;
  if (c.kind == HT_BUCKETED) {
    if (!c.bucket_slots) c.bucket_slots = 16;
    const uint64_t nb = (c.capacity + c.bucket_slots - 1) / c.bucket_slots;
    t->dev.nrange = nb;
    t->nslots = nb * c.bucket_slots;
  } else {
    c.bucket_slots = 1;
    const uint64_t ns = (c.capacity + 15) / 16 * 16;
    t->dev.nrange = ns;
    t->nslots = ns;
  }
  if (!c.stash_slots) c.stash_slots = 1024;
  if (!c.overflow_slots) c.overflow_slots = 65536;
  if (!c.max_chain) c.max_chain = 8 * std::max<uint32_t>(1, ceil_log2(t->nslots));
  // one key per lane group or lane: measured best for Cuckoo (2^26-key fill
  // at LF 0.7, c = 4: 5.88 ms at 1 key per lane, 5.96 at 2, 6.20 at 4) and,
  // with four slots per lane, for every bucket width (B = 16 3.64 ms at 1 key
  // per group against 4.13 at 2; B = 32 5.24 against 5.84)
  if (!c.keys_per_group) c.keys_per_group = 1;
  t->dev.nhash = c.nhash;
  t->dev.bucket_slots = c.bucket_slots;
  t->dev.stash_slots = c.stash_slots;
  t->dev.overflow_slots = c.overflow_slots;
  t->dev.max_chain = c.max_chain;
  t->dev.flags = c.flags;
  t->dev.kind = c.kind;
  if (!c.bucket_walk) c.bucket_walk = 64;
  t->dev.walk = (c.kind == HT_BUCKETED && !(c.flags & HT_FLAG_BUCKETED_PAPER_FULL)) ? c.bucket_walk : 0;
  t->dev.lds = c.lds_bytes;
  if (!c.key_words) c.key_words = 1;
  t->dev.key_words = c.key_words;
}

int check_table(const ht_table* t) {
  if (!t) return fail(HT_EINVAL, "table is NULL");
  if (!t->storage) return fail(HT_EINVAL, "table has no storage");
  return HT_OK;
}

int read_counters(ht_table* t, Counters* h, hipStream_t s) {
  HT_HIP(hipMemcpyAsync(h, t->dev.ctr, sizeof(Counters), hipMemcpyDeviceToHost, s));
  HT_HIP(hipStreamSynchronize(s));
  return HT_OK;
}

uint64_t spread_sum(const unsigned long long* a) {
  uint64_t s = 0;
  for (int i = 0; i < kSpread; ++i) s += a[i * kLineWords];
  return s;
}

// Distinct keys on the overflow list (host copy, sorted, unique).
int overflow_keys(ht_table* t, const Counters& h, std::vector<uint64_t>& out, hipStream_t s) {
  out.clear();
  const uint32_t n = std::min(h.overflow_count, t->dev.overflow_slots);
  if (!n) return HT_OK;
  out.resize(n);
  HT_HIP(hipMemcpyAsync(out.data(), t->dev.overflow, n * 8ull, hipMemcpyDeviceToHost, s));
  HT_HIP(hipStreamSynchronize(s));
  std::sort(out.begin(), out.end());
  out.erase(std::unique(out.begin(), out.end()), out.end());
  if (!out.empty() && out.back() == kEmpty) out.pop_back();   // not-yet-written entries
  return HT_OK;
}

DevTable launch_view(const ht_table* t) {
  DevTable d = t->dev;
  d.script = t->script;
  d.nscript = t->nscript;
  return d;
}

// Scratch of a Cuckoo call with n keys (per_wave left for the caller).
CuckooScratch scratch_view(const ht_table* t, uint64_t n) {
  CuckooScratch sc{};
  sc.dset = t->dset;
  sc.dset_mask = std::min<uint64_t>(pow2_at_least(std::max<uint64_t>(2 * n, 64)), t->dset_slots) - 1;
  sc.dset_seed = t->dset_seed;
  sc.wkey = t->wkey;
  sc.wmeta = t->wmeta;
  sc.wcnt = t->wcnt;
  return sc;
}

// Launch shape of the one-lane-per-key kernels: blocks and keys per wave.
static void lane_grid(const ht_table* t, uint64_t n, uint32_t keys_per_lane, uint64_t& blocks, uint64_t& per_wave) {
  const uint64_t waves_needed = (n + (uint64_t)kWave * keys_per_lane - 1) / ((uint64_t)kWave * keys_per_lane);
  blocks = std::min<uint64_t>((waves_needed + 3) / 4, atomic_grid_blocks(t));
  const uint64_t nwaves = blocks * 4;
  per_wave = (n + nwaves - 1) / nwaves;
}

static int vec_find_or_put(ht_table* t, const uint64_t* keys, uint64_t n, uint8_t* out, hipStream_t s) {
  int rc = reserve_scratch(t, n);
  if (rc != HT_OK) return rc;
  const DevTable d = launch_view(t);
  uint64_t blocks = 0;
  CuckooScratch sc = scratch_view(t, n);
  lane_grid(t, n, 1, blocks, sc.per_wave);
  const uint32_t W = t->cfg.key_words;
  // one walk looks up and claims, then the commit
  {
    KernelTimer kt("vec_find_or_claim", s);
    HT_HIP(vec_find_or_claim(d, keys, n, out, sc, (uint32_t)blocks, W, s));
  }
  {
    KernelTimer kt("vec_commit", s);
    HT_HIP(vec_commit(d, keys, n, sc, (uint32_t)blocks, W, s));
  }
  if (t->cfg.kind == HT_BUCKETED) return HT_OK;
  // Cuckoo: vectors whose candidates were all taken run the eviction chain
  {
    KernelTimer kt("vec_evict", s);
    HT_HIP(vec_evict(d, keys, n, out, sc, (uint32_t)blocks, W, s));
  }
  {
    KernelTimer kt("vec_scrub", s);
    HT_HIP(cuckoo_scrub(n, sc, (uint32_t)blocks, s));
  }
  return HT_OK;
}

// Regions of the probe kernel whose listed keys one wave of the evict kernel
// serves as one list.  Near the end of a fill a region lists about half as
// many keys as a wave has lanes.  With a probe grid of 8 blocks per compute
// unit, two per wave cut the evict kernel of the 2^20-key batches of a
// 2^26-key fill from 33.7 to 29.7 us on average (c = 4; three: 30.5, four:
// 31.0, eight: 35.0); with the probe grid of 6 blocks per unit, one and two
// per wave give the same fill time (5.92 ms; three: 6.02, four: 6.07).
constexpr uint32_t kEvictPack = 2;

int do_find_or_put(ht_table* t, const uint64_t* keys, uint64_t n, uint8_t* out, hipStream_t s,
                   const CuckooScratch* fixed) {
  if (t->cfg.key_words > 1) {
    if (fixed) return fail(HT_EINVAL, "state-vector tables take no caller scratch");
    return vec_find_or_put(t, keys, n, out, s);
  }
  const DevTable d = launch_view(t);
  const bool scripted = is_scripted(t);
  const uint32_t R = t->cfg.keys_per_group;
  if (t->cfg.kind == HT_BUCKETED && (t->cfg.flags & HT_FLAG_BUCKETED_ONE_LANE)) {
    // W2 fill: 4.08 ms at 8 blocks per compute unit, 3.72 at 6, 3.90 at 4
    const uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, atomic_grid_blocks(t));
    KernelTimer kt("bucketed_lane_fop", s);
    HT_HIP(bucketed_lane_find_or_put(d, keys, n, out, (uint32_t)blocks, scripted, s));
    return HT_OK;
  }
  if (t->cfg.kind == HT_BUCKETED) {
    const uint64_t g = bucketed_keys_per_wave(t->cfg.bucket_slots, R, kFopSlotsPerLane);
    const uint64_t waves = (n + g - 1) / g;
    const uint64_t blocks = std::min<uint64_t>((waves + 3) / 4, max_blocks(t));
    KernelTimer kt("bucketed_fop", s);
    HT_HIP(bucketed_find_or_put(d, keys, n, out, (uint32_t)blocks, R,
                                (t->cfg.flags & HT_FLAG_BUCKETED_ATOMIC_LOADS) != 0, scripted, s));
    return HT_OK;
  }
  if (t->cfg.flags & HT_FLAG_CUCKOO_SINGLE_PASS) {
    const uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, max_blocks(t));
    KernelTimer kt("cuckoo_single_pass", s);
    HT_HIP(cuckoo_single_pass(d, keys, n, out, (uint32_t)blocks, scripted, s));
    return HT_OK;
  }
  CuckooScratch sc{};
  if (fixed) {
    sc = *fixed;                  // scratch the caller provides (the allocation-free call)
  } else {
    int rc = reserve_scratch(t, n);
    if (rc != HT_OK) return rc;
    sc = scratch_view(t, n);
    // deferred scrub: this path's own set, emptied by the next call's probe
    // kernel; the record describes the slots this call's winners take
    sc.dset = t->dset_defer;
    sc.dirty = t->dirty;
    sc.dirty_cnt = t->dirty_cnt;
    sc.dirty_desc = t->dirty_desc;
    sc.dirty_stride = t->dirty_stride;
  }
  const uint64_t waves_needed = (n + (uint64_t)kWave * R - 1) / ((uint64_t)kWave * R);
  const uint64_t blocks = std::min<uint64_t>((waves_needed + 3) / 4, atomic_grid_blocks(t));
  const uint64_t nwaves = blocks * 4;
  sc.per_wave = (n + nwaves - 1) / nwaves;
  if (sc.dirty && sc.per_wave > sc.dirty_stride) {
    // a record too narrow for this launch (not reached: the stride is sized
    // for the largest batch the scratch serves): the shared set and the scrub
    // kernel instead, leaving the record for the next call
    sc.dset = t->dset;
    sc.dirty = nullptr;
    sc.dirty_cnt = nullptr;
    sc.dirty_desc = nullptr;
  }
  const bool paper = (t->cfg.flags & HT_FLAG_CUCKOO_PAPER_ORDER) != 0;
  {
    KernelTimer kt("cuckoo_probe", s);
    HT_HIP(cuckoo_probe(d, keys, n, out, sc, (uint32_t)blocks, R, scripted, paper, s));
  }
  {
    KernelTimer kt("cuckoo_evict", s);
    HT_HIP(cuckoo_evict(d, n, out, sc, (uint32_t)blocks, kEvictPack, scripted, s));
  }
  if (!sc.dirty) {
    KernelTimer kt("cuckoo_scrub", s);
    HT_HIP(cuckoo_scrub(n, sc, (uint32_t)blocks, s));
  }
  return HT_OK;
}

int do_query(ht_table* t, const uint64_t* keys, uint64_t n, uint8_t* out, hipStream_t s) {
  const DevTable d = launch_view(t);
  if (t->cfg.key_words > 1) {
    const uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, max_blocks(t));
    KernelTimer kt("vec_query", s);
    HT_HIP(vec_query(d, keys, n, out, (uint32_t)blocks, t->cfg.key_words, s));
    return HT_OK;
  }
  const bool scripted = is_scripted(t);
  const uint32_t R = t->cfg.keys_per_group;
  // bucketed: one lane per key unless the table asks for the lane groups of
  // Sec. 4.2 (same answers; one lane per key is faster at every bucket width)
  if (t->cfg.kind == HT_BUCKETED &&
      ((t->cfg.flags & HT_FLAG_BUCKETED_ONE_LANE) || !(t->cfg.flags & HT_FLAG_BUCKETED_GROUP_QUERY))) {
    const uint64_t blocks = std::min<uint64_t>((n + kBlock - 1) / kBlock, max_blocks(t));
    KernelTimer kt("bucketed_lane_query", s);
    HT_HIP(bucketed_lane_query(d, keys, n, out, (uint32_t)blocks, scripted, s));
    return HT_OK;
  }
  if (t->cfg.kind == HT_BUCKETED) {
    // a query issues no atomics, so a second key in flight per group pays off
    // even where find-or-put prefers one (measured: +11-14% at B = 8 and 16)
    const uint32_t Rq = R < 2 ? 2 : R;
    const uint64_t g = bucketed_keys_per_wave(t->cfg.bucket_slots, Rq, 2);
    const uint64_t waves = (n + g - 1) / g;
    const uint64_t blocks = std::min<uint64_t>((waves + 3) / 4, max_blocks(t));
    KernelTimer kt("bucketed_query", s);
    HT_HIP(bucketed_query(d, keys, n, out, (uint32_t)blocks, Rq, scripted, s));
  } else {
    const uint64_t per = (uint64_t)kBlock * R;
    const uint64_t blocks = std::min<uint64_t>((n + per - 1) / per, max_blocks(t));
    KernelTimer kt("cuckoo_query", s);
    HT_HIP(cuckoo_query(d, keys, n, out, (uint32_t)blocks, R, scripted, s));
  }
  return HT_OK;
}

// All members to a device buffer (allocated here, caller frees); returns count.
int dump_members(ht_table* t, uint64_t** d_buf, uint64_t* count, hipStream_t s) {
  Counters h;
  int rc = read_counters(t, &h, s);
  if (rc) return rc;
  std::vector<uint64_t> ovf;
  rc = overflow_keys(t, h, ovf, s);
  if (rc) return rc;
  const uint64_t upper = spread_sum(h.size) + ovf.size() + 1;
  uint64_t* buf = nullptr;
  hipError_t e = hipMalloc(&buf, std::max<uint64_t>(upper, 1) * 8 * t->cfg.key_words);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HT_ENOMEM, "hipMalloc of dump buffer failed");
  }
  uint64_t n = 0;
  rc = ht_dump(t, buf, upper, &n, s);
  if (rc) {
    (void)hipFree(buf);
    return rc;
  }
  *d_buf = buf;
  *count = std::min(n, upper);
  return HT_OK;
}

}  // namespace ht_rt

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

void ht_config_default(ht_config* cfg, uint32_t kind) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->kind = kind;
  cfg->nhash = 3;
  cfg->bucket_slots = kind == HT_BUCKETED ? 16 : 0;
  cfg->keys_per_group = 0;
  cfg->stash_slots = 1024;
  cfg->overflow_slots = 65536;
  cfg->bucket_walk = kind == HT_BUCKETED ? 64 : 0;
}

int ht_create(const ht_config* cfg, ht_table** out) {
  if (!out) return fail(HT_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_config(cfg);
  if (rc) return rc;
  ht_table* t = new ht_table();
  t->cfg = *cfg;
  t->user_cfg = *cfg;
  (void)hipGetDevice(&t->device);
  t->cus = device_cus(t->device);
  setup_geometry(t);
  t->rng.s = cfg->seed ^ 0x6a09e667f3bcc909ull;
  draw_constants(t);
  rc = alloc_storage(t);
  if (rc) {
    delete t;
    return rc;
  }
  rc = clear_async(t, nullptr);
  if (!rc && cfg->max_batch) rc = reserve_scratch(t, cfg->max_batch);
  if (!rc) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_fail(e, "hipDeviceSynchronize");
  }
  if (rc) {
    free_scratch(t);
    free_storage(t);
    delete t;
    return rc;
  }
  *out = t;
  return HT_OK;
}

int ht_create_simple(uint32_t kind, uint64_t capacity, uint32_t nhash, ht_table** out) {
  ht_config c;
  ht_config_default(&c, kind);
  c.capacity = capacity;
  c.nhash = nhash;
  return ht_create(&c, out);
}

int ht_destroy(ht_table* t) {
  if (!t) return fail(HT_EINVAL, "table is NULL");
  (void)hipDeviceSynchronize();
  free_scratch(t);
  free_storage(t);
  if (t->script) (void)hipFree(t->script);
  delete t;
  return HT_OK;
}

int ht_find_or_put(ht_table* t, const uint64_t* d_keys, uint64_t n, uint8_t* d_out_is_new, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (n == 0) return HT_OK;
  if (!d_keys) return fail(HT_EINVAL, "keys is NULL");
  if (n >= (1ull << 40)) return fail(HT_EINVAL, "batch above 2^40 keys");
  if (t->cfg.key_words > 1 && (reinterpret_cast<uintptr_t>(d_keys) & 15))
    return fail(HT_EINVAL, "vector keys must be 16-byte aligned");
  if (t->cfg.key_words > 1 && n >= (1ull << (kArenaBits - 1)))
    return fail(HT_EINVAL, "vector batch above 2^33 keys");
  return do_find_or_put(t, d_keys, n, d_out_is_new, s);
}

int ht_insert(ht_table* t, const uint64_t* d_keys, uint64_t n, uint8_t* d_out_is_new, hipStream_t s) {
  return ht_find_or_put(t, d_keys, n, d_out_is_new, s);
}

int ht_query(ht_table* t, const uint64_t* d_keys, uint64_t n, uint8_t* d_out_found, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (n == 0) return HT_OK;
  if (!d_keys || !d_out_found) return fail(HT_EINVAL, "keys or out is NULL");
  if (t->cfg.key_words > 1 && (reinterpret_cast<uintptr_t>(d_keys) & 15))
    return fail(HT_EINVAL, "vector keys must be 16-byte aligned");
  return do_query(t, d_keys, n, d_out_found, s);
}

int ht_multi_plan_create(ht_table* const* t, const uint64_t* const* d_keys, const uint64_t* n,
                         uint8_t* const* d_out_is_new, uint32_t ntables, ht_multi_plan** out) {
  if (!out) return fail(HT_EINVAL, "out is NULL");
  *out = nullptr;
  if (ntables && (!t || !d_keys || !n || !d_out_is_new)) return fail(HT_EINVAL, "NULL argument array");
  if (ntables > (1u << 23)) return fail(HT_EINVAL, "too many tables in one plan");
  std::vector<MultiSpec> specs;
  std::vector<MultiCuckooSpec> cuckoo;
  std::vector<ht_multi_plan::VecJob> vec;
  std::vector<ht_table*> seen;
  for (uint32_t i = 0; i < ntables; ++i) {
    int rc = check_table(t[i]);
    if (rc) return rc;
    if (std::find(seen.begin(), seen.end(), t[i]) != seen.end())
      return fail(HT_EINVAL, "a table appears twice in one multi-table call");
    seen.push_back(t[i]);
    if (n[i] && !d_keys[i]) return fail(HT_EINVAL, "keys is NULL");
    if (n[i] >= (1ull << 40)) return fail(HT_EINVAL, "batch above 2^40 keys");
    if (is_scripted(t[i])) return fail(HT_EINVAL, "scripted-hash tables are not supported by the multi-table call");
    if (t[i]->cfg.key_words > 1) {
      if (n[i] && (reinterpret_cast<uintptr_t>(d_keys[i]) & 15))
        return fail(HT_EINVAL, "vector keys must be 16-byte aligned");
      if (n[i] >= (1ull << (kArenaBits - 1))) return fail(HT_EINVAL, "vector batch of 2^33 keys or more");
      rc = reserve_scratch(t[i], n[i]);     // so that launches allocate nothing
      if (rc) return rc;
      if (n[i]) vec.push_back(ht_multi_plan::VecJob{t[i], d_keys[i], n[i], d_out_is_new[i]});
      continue;
    }
    if (t[i]->cfg.kind == HT_CUCKOO) {
      rc = reserve_scratch(t[i], n[i]);     // so that launches allocate nothing
      if (rc) return rc;
      if (n[i]) {
        MultiCuckooSpec cs{};
        cs.t = launch_view(t[i]);
        cs.s = scratch_view(t[i], n[i]);
        cs.keys = d_keys[i];
        cs.out = d_out_is_new[i];
        cs.n = n[i];
        cs.max_regions = (uint64_t)max_blocks(t[i]) * (kBlock / kWave);
        cs.paper = (t[i]->cfg.flags & HT_FLAG_CUCKOO_PAPER_ORDER) != 0;
        cuckoo.push_back(cs);
      }
      continue;
    }
    MultiSpec sp{};
    sp.t = launch_view(t[i]);
    sp.keys = d_keys[i];
    sp.out = d_out_is_new[i];
    sp.n = n[i];
    specs.push_back(sp);
  }
  ht_multi_plan* p = new ht_multi_plan();
  p->tables = seen;
  p->vec = vec;
  int dev = 0;
  (void)hipGetDevice(&dev);
  p->grid = device_cus(dev) * 8;
  hipError_t e = multi_plan_build(specs, cuckoo, p->grid, p->dev);
  if (e != hipSuccess) {
    multi_plan_free(p->dev);
    delete p;
    return hip_fail(e, "multi_plan_build");
  }
  *out = p;
  return HT_OK;
}

int ht_multi_plan_launch(ht_multi_plan* p, hipStream_t s) {
  if (!p) return fail(HT_EINVAL, "plan is NULL");
  if (p->dev.nitems) {
    KernelTimer kt("multi_fill", s);
    HT_HIP(multi_plan_launch(p->dev, s));
  }
  if (p->dev.ncitems) {
    static const char* const names[3] = {"multi_cuckoo_probe", "multi_cuckoo_evict", "multi_cuckoo_scrub"};
    for (int ph = 0; ph < 3; ++ph) {
      KernelTimer kt(names[ph], s);
      HT_HIP(multi_cuckoo_launch(p->dev, ph, s));
    }
  }
  // vector tables: scratch reserved at creation, so these only launch kernels
  for (const auto& j : p->vec) {
    int rc = do_find_or_put(j.t, j.keys, j.n, j.out, s);
    if (rc) return rc;
  }
  return HT_OK;
}

int ht_multi_plan_status(ht_multi_plan* p, hipStream_t s) {
  if (!p) return fail(HT_EINVAL, "plan is NULL");
  HT_HIP(hipStreamSynchronize(s));
  return HT_OK;
}

int ht_multi_plan_destroy(ht_multi_plan* p) {
  if (!p) return fail(HT_EINVAL, "plan is NULL");
  (void)hipDeviceSynchronize();
  multi_plan_free(p->dev);
  delete p;
  return HT_OK;
}

int ht_find_or_put_multi(ht_table* const* t, const uint64_t* const* d_keys, const uint64_t* n,
                         uint8_t* const* d_out_is_new, uint32_t ntables, hipStream_t s) {
  if (ntables == 0) return HT_OK;
  ht_multi_plan* p = nullptr;
  int rc = ht_multi_plan_create(t, d_keys, n, d_out_is_new, ntables, &p);
  if (rc) return rc;
  rc = ht_multi_plan_launch(p, s);
  if (!rc) rc = ht_multi_plan_status(p, s);
  ht_multi_plan_destroy(p);
  return rc;
}

int ht_query_multi(ht_table* const* t, const uint64_t* const* d_keys, const uint64_t* n,
                   uint8_t* const* d_out_found, uint32_t ntables, hipStream_t s) {
  if (ntables == 0) return HT_OK;
  if (!t || !d_keys || !n || !d_out_found) return fail(HT_EINVAL, "NULL argument array");
  if (ntables > (1u << 23)) return fail(HT_EINVAL, "too many tables in one call");
  std::vector<MultiQuerySpec> qs;
  for (uint32_t i = 0; i < ntables; ++i) {
    int rc = check_table(t[i]);
    if (rc) return rc;
    if (n[i] && (!d_keys[i] || !d_out_found[i])) return fail(HT_EINVAL, "keys or flags is NULL");
    if (n[i] >= (1ull << 40)) return fail(HT_EINVAL, "batch above 2^40 keys");
    if (is_scripted(t[i])) return fail(HT_EINVAL, "scripted-hash tables are not supported by the multi-table call");
    if (t[i]->cfg.key_words > 1 && n[i] && (reinterpret_cast<uintptr_t>(d_keys[i]) & 15))
      return fail(HT_EINVAL, "vector keys must be 16-byte aligned");
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint32_t grid = device_cus(dev) * 8;
  for (uint32_t i = 0; i < ntables; ++i) {
    if (!n[i]) continue;
    MultiQuerySpec q{};
    q.t = launch_view(t[i]);
    q.keys = d_keys[i];
    q.out = d_out_found[i];
    q.n = n[i];
    q.cuckoo = t[i]->cfg.kind == HT_CUCKOO;
    if (t[i]->cfg.key_words > 1 || multi_query_alone(q, grid)) {   // vector tables: their own kernel
      int rc = do_query(t[i], d_keys[i], n[i], d_out_found[i], s);
      if (rc) return rc;
    } else {
      qs.push_back(q);
    }
  }
  {
    KernelTimer kt("multi_query", s);
    HT_HIP(multi_query_once(qs.data(), (uint32_t)qs.size(), grid, s));
  }
  HT_HIP(hipStreamSynchronize(s));
  return HT_OK;
}

int ht_sync_status(ht_table* t, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  Counters h;
  rc = read_counters(t, &h, s);
  if (rc) return rc;
  if (h.overflow_count || h.lost) return fail(HT_EFULL, "keys on the overflow list; rebuild the table");
  return HT_OK;
}

int ht_size(ht_table* t, uint64_t* out_n, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!out_n) return fail(HT_EINVAL, "out_n is NULL");
  Counters h;
  rc = read_counters(t, &h, s);
  if (rc) return rc;
  uint64_t n = spread_sum(h.size);
  if (t->cfg.kind == HT_BUCKETED && t->cfg.key_words == 1 && h.overflow_count) {
    std::vector<uint64_t> ovf;
    rc = overflow_keys(t, h, ovf, s);
    if (rc) return rc;
    n += ovf.size();
  }
  *out_n = n;
  return HT_OK;
}

int ht_dump(ht_table* t, uint64_t* d_out, uint64_t cap, uint64_t* out_n, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!out_n) return fail(HT_EINVAL, "out_n is NULL");
  if (!d_out && cap) return fail(HT_EINVAL, "d_out is NULL");
  HT_HIP(zero_words(reinterpret_cast<uint32_t*>(t->misc), 2, s));
  const uint32_t g = max_blocks(t);
  if (t->cfg.key_words > 1) {
    // members are the arena entries named by the handles in slots, stash and overflow list
    Counters h;
    rc = read_counters(t, &h, s);
    if (rc) return rc;
    const uint32_t W = t->cfg.key_words;
    HT_HIP(vec_dump(t->dev.slots, t->nslots, t->dev.arena, d_out, cap, t->misc, g, W, s));
    HT_HIP(vec_dump(t->dev.stash, t->dev.stash_slots, t->dev.arena, d_out, cap, t->misc, g, W, s));
    if (h.overflow_count)    // an open-addressed set for vector tables
      HT_HIP(vec_dump(t->dev.overflow, t->dev.overflow_slots, t->dev.arena, d_out, cap, t->misc, g, W, s));
    unsigned long long nv = 0;
    HT_HIP(hipMemcpyAsync(&nv, t->misc, 8, hipMemcpyDeviceToHost, s));
    HT_HIP(hipStreamSynchronize(s));
    *out_n = nv;
    return HT_OK;
  }
  HT_HIP(compact_words(t->dev.slots, t->nslots, d_out, cap, t->misc, g, s));
  HT_HIP(compact_words(t->dev.stash, t->dev.stash_slots, d_out, cap, t->misc, g, s));
  Counters h;
  rc = read_counters(t, &h, s);
  if (rc) return rc;
  unsigned long long n = 0;
  HT_HIP(hipMemcpyAsync(&n, t->misc, 8, hipMemcpyDeviceToHost, s));
  HT_HIP(hipStreamSynchronize(s));
  std::vector<uint64_t> extra;
  rc = overflow_keys(t, h, extra, s);
  if (rc) return rc;
  if (h.sentinel) extra.push_back(kEmpty);
  if (n < cap && !extra.empty()) {
    const uint64_t m = std::min<uint64_t>(extra.size(), cap - n);
    HT_HIP(hipMemcpyAsync(d_out + n, extra.data(), m * 8, hipMemcpyHostToDevice, s));
    HT_HIP(hipStreamSynchronize(s));
  }
  *out_n = n + extra.size();
  return HT_OK;
}

int ht_dump_raw(ht_table* t, uint64_t* d_slots, uint64_t cap, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  const uint64_t need = t->nslots + t->dev.stash_slots;
  if (!d_slots || cap < need) return fail(HT_EINVAL, "d_slots NULL or smaller than slots + stash");
  HT_HIP(hipMemcpyAsync(d_slots, t->dev.slots, t->nslots * 8, hipMemcpyDeviceToDevice, s));
  HT_HIP(hipMemcpyAsync(d_slots + t->nslots, t->dev.stash, (size_t)t->dev.stash_slots * 8,
                        hipMemcpyDeviceToDevice, s));
  return HT_OK;
}

int ht_clear(ht_table* t, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  return clear_async(t, s);
}

int ht_rebuild(ht_table* t, uint64_t new_capacity, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (new_capacity > (1ull << 40)) return fail(HT_EINVAL, "capacity above 2^40 slots");
  if (t->cfg.key_words > 1 && new_capacity &&
      new_capacity + t->dev.stash_slots + t->dev.overflow_slots + 64 >= (1ull << (kArenaBits - 1)))
    return fail(HT_EINVAL, "vector table capacity above 2^33 entries");
  // every member (slots, stash, overflow list, the all-ones key) to a device buffer
  uint64_t* buf = nullptr;
  uint64_t n = 0;
  rc = dump_members(t, &buf, &n, s);
  if (rc) return rc;
  HT_HIP(hipStreamSynchronize(s));
  // The old storage stays untouched until the members are all placed in the
  // new one: allocate first, and on any failure put the old table back.
  const ht_config old_cfg = t->cfg, old_user = t->user_cfg;
  const uint64_t old_nslots = t->nslots;
  const DevTable old_dev = t->dev;
  void* const old_storage = t->storage;
  unsigned long long* const old_misc = t->misc;
  auto restore = [&]() {
    t->cfg = old_cfg;
    t->user_cfg = old_user;
    t->nslots = old_nslots;
    t->dev = old_dev;
    t->storage = old_storage;
    t->misc = old_misc;
  };
  if (new_capacity) {
    t->cfg = t->user_cfg;
    t->cfg.capacity = new_capacity;
    t->user_cfg.capacity = new_capacity;
    setup_geometry(t);
  }
  t->storage = nullptr;
  rc = alloc_storage(t);
  if (rc) {
    restore();
    (void)hipFree(buf);
    return rc;
  }
  for (int attempt = 0; attempt < 8; ++attempt) {
    draw_constants(t);          // the hash constants live in t->dev, so a restore keeps the old ones
    rc = clear_async(t, s);
    if (!rc && n) rc = do_find_or_put(t, buf, n, nullptr, s);
    if (rc) break;
    Counters h;
    rc = read_counters(t, &h, s);
    if (rc) break;
    if (!h.overflow_count && !h.lost) break;
    rc = fail(HT_EFULL, "rebuild could not place every key in slots and stash; the table is unchanged "
                        "(grow it)");
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (rc) {
    (void)hipFree(t->storage);
    restore();
    return rc;
  }
  (void)hipFree(old_storage);
  return HT_OK;
}

int ht_stats(ht_table* t, ht_stats_t* out, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!out) return fail(HT_EINVAL, "out is NULL");
  Counters h;
  rc = read_counters(t, &h, s);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  uint64_t n = 0;
  rc = ht_size(t, &n, s);
  if (rc) return rc;
  out->size = n;
  out->capacity = t->nslots;
  out->stash_count = h.stash_count;
  out->overflow_count = h.overflow_count;
  out->lost = h.lost;
  out->evictions = spread_sum(h.evictions);
  out->nbuckets = t->dev.nrange;
  out->kind = t->cfg.kind;
  out->nhash = t->cfg.nhash;
  out->bucket_slots = t->cfg.bucket_slots;
  out->stash_slots = t->dev.stash_slots;
  out->seed = t->dev.seed[0];
  return HT_OK;
}

int ht_hash_index(const ht_table* t, uint64_t key, uint32_t j, uint64_t* out_index) {
  if (!t || !out_index) return fail(HT_EINVAL, "NULL argument");
  if (j >= t->cfg.nhash) return fail(HT_EINVAL, "j >= nhash");
  if (t->cfg.flags & HT_FLAG_SCRIPTED_HASH) return fail(HT_EINVAL, "scripted table");
  *out_index = mulhi64(mix64(key ^ t->dev.seed[j]), t->dev.nrange);
  return HT_OK;
}

int ht_set_scripted_hash(ht_table* t, const uint64_t* keys, const uint64_t* h_index, uint32_t nkeys) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!(t->cfg.flags & HT_FLAG_SCRIPTED_HASH)) return fail(HT_EINVAL, "table not created with HT_FLAG_SCRIPTED_HASH");
  if (nkeys && (!keys || !h_index)) return fail(HT_EINVAL, "NULL argument");
  if (nkeys > 4096) return fail(HT_EINVAL, "at most 4096 scripted keys");
  std::vector<ScriptRow> rows(nkeys);
  for (uint32_t r = 0; r < nkeys; ++r) {
    rows[r].key = keys[r];
    for (uint32_t j = 0; j < kMaxHash; ++j) {
      const uint64_t v = j < t->cfg.nhash ? h_index[(size_t)r * t->cfg.nhash + j] : 0;
      if (v >= t->dev.nrange) return fail(HT_EINVAL, "scripted hash value out of range");
      rows[r].h[j] = v;
    }
  }
  HT_HIP(hipDeviceSynchronize());
  if (t->script) (void)hipFree(t->script);
  t->script = nullptr;
  t->nscript = 0;
  if (nkeys) {
    HT_HIP(hipMalloc(&t->script, sizeof(ScriptRow) * nkeys));
    HT_HIP(hipMemcpy(t->script, rows.data(), sizeof(ScriptRow) * nkeys, hipMemcpyHostToDevice));
  }
  t->nscript = nkeys;
  return HT_OK;
}

int ht_chain_histogram(ht_table* t, uint64_t* out, hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (!out) return fail(HT_EINVAL, "out is NULL");
  Counters h;
  rc = read_counters(t, &h, s);
  if (rc) return rc;
  for (int b = 0; b < kChainBins; ++b) {
    uint64_t v = 0;
    for (int i = 0; i < kSpread; ++i) v += h.chain_hist[i * kChainBins + b];
    out[b] = v;
  }
  return HT_OK;
}

int ht_reserve(ht_table* t, uint64_t max_batch) {
  int rc = check_table(t);
  if (rc) return rc;
  return reserve_scratch(t, max_batch);
}

const char* ht_strerror(int code) {
  switch (code) {
    case HT_OK: return "ok";
    case HT_EINVAL: return "invalid argument";
    case HT_ENOMEM: return "out of device memory";
    case HT_EFULL: return "table full: keys on the overflow list";
    case HT_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* ht_last_error(void) { return g_err.c_str(); }

int ht_timing_enable(int on) {
  resolve_timings();
  std::lock_guard<std::mutex> lk(g_tmu);
  g_acc.clear();
  g_timing = on != 0;
  return HT_OK;
}

int ht_timing_report(char* buf, uint64_t len) {
  if (!buf || len == 0) return fail(HT_EINVAL, "buffer is NULL or empty");
  resolve_timings();
  std::string js = "{";
  {
    std::lock_guard<std::mutex> lk(g_tmu);
    bool first = true;
    for (auto& kv : g_acc) {
      char item[256];
      std::snprintf(item, sizeof(item), "%s\"%s\": [%llu, %.6f]", first ? "" : ", ", kv.first.c_str(),
                    (unsigned long long)kv.second.first, kv.second.second);
      js += item;
      first = false;
    }
  }
  js += "}";
  if (js.size() + 1 > len) return fail(HT_EINVAL, "buffer too small");
  std::memcpy(buf, js.c_str(), js.size() + 1);
  return HT_OK;
}

int ht_probe_copy(const uint64_t* d_src, uint64_t* d_dst, uint64_t n, hipStream_t s) {
  if (n == 0) return HT_OK;
  if (!d_src || !d_dst) return fail(HT_EINVAL, "NULL pointer");
  int dev = 0;
  (void)hipGetDevice(&dev);
  HT_HIP(probe_copy(d_src, d_dst, n, device_cus(dev) * 8, s));
  return HT_OK;
}

int ht_probe_gather(const uint64_t* d_array, uint64_t n_words, uint64_t n_access, uint32_t line_bytes,
                    uint64_t seed, uint64_t* d_sink, hipStream_t s) {
  if (n_access == 0) return HT_OK;
  if (!d_array || !d_sink) return fail(HT_EINVAL, "NULL pointer");
  if (line_bytes != 8 && line_bytes != 64 && line_bytes != 128) return fail(HT_EINVAL, "line_bytes must be 8, 64 or 128");
  if (n_words < line_bytes / 8) return fail(HT_EINVAL, "array smaller than one line");
  int dev = 0;
  (void)hipGetDevice(&dev);
  HT_HIP(probe_gather(d_array, n_words, n_access, line_bytes, seed, d_sink, device_cus(dev) * 8, s));
  return HT_OK;
}

int ht_probe_cas(uint64_t* d_array, uint64_t n_words, uint64_t n_access, uint64_t seed, hipStream_t s) {
  if (n_access == 0) return HT_OK;
  if (!d_array || n_words == 0) return fail(HT_EINVAL, "NULL or empty array");
  int dev = 0;
  (void)hipGetDevice(&dev);
  HT_HIP(probe_cas(d_array, n_words, n_access, seed, device_cus(dev) * 8, s));
  return HT_OK;
}

int ht_probe_mix(const uint64_t* d_keys, uint8_t* d_out, uint64_t n_items, uint64_t* d_array, uint64_t n_words,
                 double lines_per_item, double cas_per_item, uint32_t same_line, uint64_t seed, hipStream_t s) {
  if (n_items == 0) return HT_OK;
  if (!d_keys || !d_out || !d_array || n_words == 0) return fail(HT_EINVAL, "NULL pointer or empty array");
  if (!(lines_per_item >= 0.0 && lines_per_item <= 64.0)) return fail(HT_EINVAL, "lines_per_item outside 0..64");
  if (!(cas_per_item >= 0.0 && cas_per_item <= 1.0)) return fail(HT_EINVAL, "cas_per_item outside 0..1");
  const uint32_t lq = (uint32_t)(lines_per_item * 256.0 + 0.5);
  const uint32_t cq = (uint32_t)(cas_per_item * 256.0 + 0.5);
  int dev = 0;
  (void)hipGetDevice(&dev);
  KernelTimer kt("probe_mix", s);
  HT_HIP(probe_mix(d_keys, d_out, n_items, d_array, n_words, lq, cq, same_line != 0, seed, device_cus(dev) * 8, s));
  return HT_OK;
}

}  // extern "C"
