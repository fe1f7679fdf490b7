// Many bucketed tables in one persistent launch.
//
// The find-or-put of every bucketed table is cut into work items of equal
// size (a power of two between 64 and 4096 keys, chosen so that a launch has
// about as many items as the device has wave slots); wave w takes items w,
// w + W, w + 2W, ... of the queue.  The items are equal, so this static
// split balances, and it needs no shared queue counter (a counter popped by
// every wave of a large grid serialises on one address).  Each lane probes
// its own key (the one-lane probe: the key's buckets read eight slots at a
// time, the first empty slot compare-and-swapped; same probe sequence and
// results as a lane group), with the bucket width taken from each table at
// run time, so one code path serves 8/16/32/64-slot tables.  On 256 tables
// of 2^10..2^22 slots, half of them filled with BFS batches full of repeats,
// this ran 1.4x faster than lane groups of B/2 lanes per key; against lane
// groups of B/4 lanes holding four slots each it is within 2% at B = 8
// (5.76 against 5.64 ms, 256 tables) and 7% faster at B = 16 (6.34 against
// 6.77 ms).  Tables may
// mix bucket widths and hash counts; each uses its own storage, so the
// results equal one find-or-put call per table.  The launch allocates nothing and uses no
// memset, so it can be captured in a HIP graph.
//
// The Cuckoo tables of a many-table call run their three phases (probe and
// place, evict, scrub) as three launches over all of them: the phases need a
// grid-wide barrier between them, which kernel boundaries give.  Each launch
// walks the same item list (table, region); a region is the part of a table's
// batch whose misses one wave lists, exactly as in the single-table kernels.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bucketed_dev.h"
#include "cuckoo_dev.h"
#include "multi.h"

namespace ht {

struct MultiTable {
  DevTable t;
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
  uint64_t chunk;           // keys per work item
  uint32_t nregions;        // work items
  uint32_t pad_;
};

constexpr uint64_t kRegionMask = (1ull << 40) - 1;

__host__ __device__ inline uint64_t make_item(uint32_t table, uint64_t region) {
  return ((uint64_t)table << 40) | region;
}

__global__ __launch_bounds__(kBlock) void multi_fill_kernel(const MultiTable* __restrict__ tabs,
                                                            const uint64_t* __restrict__ items, uint32_t nitems) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t idx = wave; idx < nitems; idx += nwaves) {
    // uniform across the wave: keep the item (and so the table descriptor's
    // address) in scalar registers
    const uint64_t raw = items[idx];
    const uint64_t it = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(raw >> 32)) << 32) |
                        __builtin_amdgcn_readfirstlane((uint32_t)raw);
    const MultiTable& m = tabs[(uint32_t)(it >> 40)];
    const uint64_t begin = (it & kRegionMask) * m.chunk;
    const uint64_t end = begin + m.chunk < m.n ? begin + m.chunk : m.n;
    unsigned long long nnew = 0;
    for (uint64_t i = begin + lane_id(); i < end; i += kWave) {
      const uint32_t r = lane_find_or_put<false>(m.t, m.keys[i]);
      if (m.out) m.out[i] = (uint8_t)r;
      nnew += r == 1;
    }
    wave_count(m.t.ctr->size, nnew, (uint32_t)(wave + idx));
  }
}

struct MultiCuckoo {
  DevTable t;
  CuckooScratch s;          // per_wave = keys per region
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
  uint32_t paper;           // HT_FLAG_CUCKOO_PAPER_ORDER
  uint32_t pad_;
};

__device__ __forceinline__ uint64_t uniform_item(const uint64_t* items, uint64_t idx) {
  const uint64_t raw = items[idx];
  return ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(raw >> 32)) << 32) |
         __builtin_amdgcn_readfirstlane((uint32_t)raw);
}

__global__ __launch_bounds__(kBlock) void multi_cuckoo_probe_kernel(const MultiCuckoo* __restrict__ tabs,
                                                                    const uint64_t* __restrict__ items,
                                                                    uint32_t nitems) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t idx = wave; idx < nitems; idx += nwaves) {
    const uint64_t it = uniform_item(items, idx);
    const MultiCuckoo& m = tabs[(uint32_t)(it >> 40)];
    const uint64_t region = it & kRegionMask;
    const unsigned long long nnew =
        m.paper ? cuckoo_probe_region<1, false, true>(m.t, m.keys, m.n, m.out, m.s, region)
                : cuckoo_probe_region<1, false, false>(m.t, m.keys, m.n, m.out, m.s, region);
    wave_count(m.t.ctr->size, nnew, (uint32_t)(wave + idx));
  }
}

__global__ __launch_bounds__(kBlock) void multi_cuckoo_evict_kernel(const MultiCuckoo* __restrict__ tabs,
                                                                    const uint64_t* __restrict__ items,
                                                                    uint32_t nitems) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t idx = wave; idx < nitems; idx += nwaves) {
    const uint64_t it = uniform_item(items, idx);
    const MultiCuckoo& m = tabs[(uint32_t)(it >> 40)];
    unsigned long long nnew = 0, nevict = 0;
    if (m.t.flags & kFlagLookahead)
      cuckoo_evict_region<false, true>(m.t, m.n, m.out, m.s, it & kRegionMask, nnew, nevict);
    else
      cuckoo_evict_region<false, false>(m.t, m.n, m.out, m.s, it & kRegionMask, nnew, nevict);
    wave_count(m.t.ctr->size, nnew, (uint32_t)(wave + idx));
    wave_count(m.t.ctr->evictions, nevict, (uint32_t)(wave + idx));
  }
}

__global__ __launch_bounds__(kBlock) void multi_cuckoo_scrub_kernel(const MultiCuckoo* __restrict__ tabs,
                                                                    const uint64_t* __restrict__ items,
                                                                    uint32_t nitems) {
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  for (uint64_t idx = wave; idx < nitems; idx += nwaves) {
    const uint64_t it = uniform_item(items, idx);
    const MultiCuckoo& m = tabs[(uint32_t)(it >> 40)];
    cuckoo_scrub_region(m.n, m.s, it & kRegionMask);
  }
}

// Queries of many tables, of either kind, in one launch.  A query writes
// nothing to the table, so no phases are needed.  The launch is a list of
// items, each a run of one table's keys; table i owns items first_i ..
// first_{i+1} - 1, and wave w takes items w, w + W, w + 2W, ...  A wave's
// item index only grows, so it finds each item's table by walking the
// descriptors forward (no item list is stored).  Items are short, so the
// waves sweep the tables in order, a few at a time, and the tables being
// probed stay in cache together, as when each table has a launch of its own.
// A bucketed table is read as by the single-table query: groups of B/2 lanes
// read a whole bucket in one access, two keys per group in flight, and stop
// at the key or at the first bucket with an empty slot; a Cuckoo table gives
// each lane a key and reads h_1, h_2, ..., stopping at the key or (distinct
// indices) an empty slot.  Both then check the stash and overflow list if
// those hold keys.
struct MultiQuery {
  DevTable t;
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
  uint64_t chunk;           // keys per item
  uint64_t first;           // index of the table's first item
  uint32_t cuckoo;
  uint32_t pad_;
};

__global__ __launch_bounds__(kBlock) void multi_query_kernel(const MultiQuery* __restrict__ tabs, uint32_t ntabs,
                                                             uint64_t nitems) {
  const int lane = lane_id();
  const uint64_t wave =
      __builtin_amdgcn_readfirstlane((uint32_t)(((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave));
  const uint64_t nwaves = (uint64_t)gridDim.x * (kBlock / kWave);
  uint32_t ti = 0;
  for (uint64_t idx = wave; idx < nitems; idx += nwaves) {
    while (ti + 1 < ntabs && idx >= tabs[ti + 1].first) ++ti;
    const MultiQuery& m = tabs[ti];
    const uint64_t begin = (idx - m.first) * m.chunk;
    const uint64_t end = begin + m.chunk < m.n ? begin + m.chunk : m.n;
    const uint32_t sc = m.t.ctr->stash_count;
    const uint32_t oc = m.t.ctr->overflow_count;
    if (m.cuckoo) {
      for (uint64_t base = begin; base < end; base += kWave) {
        const uint64_t i = base + lane;
        const uint64_t k[1] = {i < end ? m.keys[i] : kEmpty};
        const bool live[1] = {i < end && k[0] != kEmpty};
        bool hit[1];
        cuckoo_lookup<1, false>(m.t, k, live, hit);
        if (i < end) {
          bool h = hit[0];
          if (k[0] == kEmpty) h = m.t.ctr->sentinel != 0;
          else if (!h && (sc | oc)) h = stash_query(m.t, k[0], sc, oc);
          m.out[i] = h ? 1 : 0;
        }
      }
    } else if (!(m.t.flags & kFlagGroupQuery)) {
      for (uint64_t base = begin; base < end; base += kWave) {
        const uint64_t i = base + lane;
        if (i < end) m.out[i] = (uint8_t)lane_query<false>(m.t, m.keys[i], sc, oc);
      }
    } else {
      const uint32_t L = m.t.bucket_slots / 2;
      const uint32_t G = kWave / L;
      const int grp = lane / (int)L;
      const int gl = lane & (int)(L - 1);
      for (uint64_t base = begin; base < end; base += 2 * G) {
        uint64_t k[2];
        bool act[2];
        uint32_t res[2];
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const uint64_t i = base + (uint64_t)r * G + grp;
          act[r] = i < end;
          k[r] = act[r] ? m.keys[i] : 0;
        }
        bucket_query<0, 2, false>(m.t, k, act, sc, oc, res);
        if (gl == 0) {
#pragma unroll
          for (int r = 0; r < 2; ++r)
            if (act[r]) m.out[base + (uint64_t)r * G + grp] = (uint8_t)res[r];
        }
      }
    }
  }
}

// Item size for a launch of `total` keys on a device with `max_waves` wave
// slots: a power of two in [64, 4096] giving about max_waves items (small
// launches still fill every wave slot).
uint64_t multi_chunk(uint64_t total, uint64_t max_waves) {
  uint64_t c = 64;
  while (c < 4096 && c * max_waves < total) c <<= 1;
  return c;
}

// Grid cap of the Cuckoo phases: three quarters of `max_blocks` (6 blocks
// per compute unit), as for the single-table Cuckoo probe; 256 tables of
// 2^6..2^26 slots in one plan launch: 8.8-8.9 ms at 8 blocks per unit,
// 8.05-8.19 at 6, 7.95 at 5, 8.04 at 4.
static uint32_t cuckoo_blocks(uint32_t max_blocks) { return max_blocks / 4 * 3 ? max_blocks / 4 * 3 : 1; }

uint32_t multi_grid(uint64_t nitems, uint32_t max_blocks) {
  const uint64_t blocks = (nitems + (kBlock / kWave) - 1) / (kBlock / kWave);
  return (uint32_t)(blocks < max_blocks ? (blocks ? blocks : 1) : max_blocks);
}

// ---- host side ------------------------------------------------------------

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Fill the descriptors and (table, region) items of `nt` bucketed tables
// (find-or-put).  Returns the item count, or ~0 when the items would exceed
// cap_items.
static uint64_t fill_bucketed(const MultiSpec* sp, uint32_t nt, uint64_t max_waves, MultiTable* tabs,
                              uint64_t* items, uint64_t cap_items) {
  uint64_t total = 0;
  for (uint32_t i = 0; i < nt; ++i) total += sp[i].n;
  const uint64_t chunk = multi_chunk(total, max_waves);
  uint64_t nitems = 0;
  for (uint32_t i = 0; i < nt; ++i) {
    MultiTable& m = tabs[i];
    std::memset(&m, 0, sizeof(m));
    m.t = sp[i].t;
    m.keys = sp[i].keys;
    m.out = sp[i].out;
    m.n = sp[i].n;
    m.chunk = chunk;
    m.nregions = (uint32_t)((sp[i].n + chunk - 1) / chunk);
    if (nitems + m.nregions > cap_items) return ~0ull;
    for (uint64_t r = 0; r < m.nregions; ++r) items[nitems++] = make_item(i, r);
  }
  return nitems;
}

// Fill the descriptors and (table, region) items of `nc` Cuckoo tables.  A
// region holds at least a whole item's worth of keys (a multiple of 64) and a
// table never gets more regions than its scratch has per-wave counts.
// Returns the item count, or ~0 when they would exceed cap_items or a
// table's counts.
static uint64_t fill_cuckoo(const MultiCuckooSpec* cs, uint32_t nc, uint64_t max_waves, MultiCuckoo* tabs,
                            uint64_t* items, uint64_t cap_items) {
  uint64_t total = 0;
  for (uint32_t i = 0; i < nc; ++i) total += cs[i].n;
  const uint64_t chunk = multi_chunk(total, max_waves);
  uint64_t nitems = 0;
  for (uint32_t i = 0; i < nc; ++i) {
    const MultiCuckooSpec& sp = cs[i];
    MultiCuckoo& m = tabs[i];
    std::memset(&m, 0, sizeof(m));
    m.t = sp.t;
    m.s = sp.s;
    m.keys = sp.keys;
    m.out = sp.out;
    m.n = sp.n;
    m.paper = sp.paper ? 1u : 0u;
    const uint64_t maxr = std::max<uint64_t>(sp.max_regions, 1);
    uint64_t per = std::max<uint64_t>(chunk, (sp.n + maxr - 1) / maxr);
    per = (per + kWave - 1) / kWave * kWave;
    m.s.per_wave = per;
    const uint64_t nr = (sp.n + per - 1) / per;
    if (nr > maxr || nitems + nr > cap_items) return ~0ull;
    for (uint64_t r = 0; r < nr; ++r) items[nitems++] = make_item(i, r);
  }
  return nitems;
}

// Keys one wave answers per turn of the many-table query: 64 (a key per
// lane) for a Cuckoo table and a bucketed one queried one lane per key, two
// per lane group of B/2 lanes for a bucketed one with group queries.
static uint64_t query_turn(const MultiQuerySpec& q) {
  if (q.cuckoo || !(q.t.flags & kFlagGroupQuery)) return kWave;
  return 2ull * (kWave / (q.t.bucket_slots / 2));
}

bool multi_query_alone(const MultiQuerySpec& q, uint32_t max_blocks) {
  return q.n >= (uint64_t)max_blocks * (kBlock / kWave) * query_turn(q);
}

// Fill the descriptors of a many-table query; returns the item count.  An
// item is the same number of turns for every table: the fewest (a power of
// two, at most kQueryTurns) that leave at most one item per wave slot, so a
// small launch answers every key in one turn and a large one has many short
// items, swept in table order.
constexpr uint64_t kQueryTurns = 16;

static uint64_t fill_query(const MultiQuerySpec* qs, uint32_t nq, uint64_t max_waves, MultiQuery* tabs) {
  uint64_t turns = 1;
  for (; turns < kQueryTurns; turns <<= 1) {
    uint64_t count = 0;
    for (uint32_t i = 0; i < nq; ++i) {
      const uint64_t c = query_turn(qs[i]) * turns;
      count += (qs[i].n + c - 1) / c;
    }
    if (count <= max_waves) break;
  }
  uint64_t nitems = 0;
  for (uint32_t i = 0; i < nq; ++i) {
    MultiQuery& m = tabs[i];
    std::memset(&m, 0, sizeof(m));
    m.t = qs[i].t;
    m.keys = qs[i].keys;
    m.out = qs[i].out;
    m.n = qs[i].n;
    m.chunk = query_turn(qs[i]) * turns;
    m.first = nitems;
    m.cuckoo = qs[i].cuckoo ? 1u : 0u;
    nitems += (qs[i].n + m.chunk - 1) / m.chunk;
  }
  return nitems;
}

static void launch_query(const MultiQuery* d_tabs, uint32_t nq, uint64_t nitems, uint32_t max_blocks,
                         hipStream_t s) {
  hipLaunchKernelGGL(multi_query_kernel, dim3(multi_grid(nitems, max_blocks)), dim3(kBlock), 0, s, d_tabs, nq,
                     nitems);
}

// Build descriptors and the item lists on the host and copy them to one
// device allocation (synchronous).  Returns hipSuccess or the HIP error
// (hipErrorInvalidValue when a Cuckoo table's scratch has too few per-wave
// counts for its regions).
hipError_t multi_plan_build(const std::vector<MultiSpec>& specs, const std::vector<MultiCuckooSpec>& cspecs,
                            uint32_t max_blocks, MultiPlanDev& plan) {
  const uint64_t max_waves = (uint64_t)max_blocks * (kBlock / kWave);
  const uint32_t nt = (uint32_t)specs.size();
  const uint32_t nc = (uint32_t)cspecs.size();
  uint64_t cap_b = 0, cap_c = 0;
  for (const auto& sp : specs) cap_b += multi_items_for(sp.n);
  for (const auto& sp : cspecs) cap_c += multi_items_for(sp.n);
  std::vector<MultiTable> tabs(nt);
  std::vector<uint64_t> items(cap_b);
  std::vector<MultiCuckoo> ctabs(nc);
  std::vector<uint64_t> citems(cap_c);
  const uint32_t cmb = cuckoo_blocks(max_blocks);
  const uint64_t nit = fill_bucketed(specs.data(), nt, max_waves, tabs.data(), items.data(), cap_b);
  const uint64_t ncit = fill_cuckoo(cspecs.data(), nc, (uint64_t)cmb * (kBlock / kWave), ctabs.data(), citems.data(),
                                    cap_c);
  if (nit == ~0ull || ncit == ~0ull) return hipErrorInvalidValue;
  items.resize(nit);
  citems.resize(ncit);
  plan.nitems = (uint32_t)items.size();
  plan.ncitems = (uint32_t)citems.size();
  plan.grid = multi_grid(plan.nitems, max_blocks);
  plan.cgrid = multi_grid(plan.ncitems, cmb);
  const size_t b_tabs = align256(sizeof(MultiTable) * nt);
  const size_t b_items = align256(items.size() * 8);
  const size_t b_ctabs = align256(sizeof(MultiCuckoo) * nc);
  const size_t b_citems = align256(citems.size() * 8);
  hipError_t e = hipMalloc(&plan.base, b_tabs + b_items + b_ctabs + b_citems + 256);
  if (e != hipSuccess) return e;
  char* c = static_cast<char*>(plan.base);
  plan.tabs = reinterpret_cast<MultiTable*>(c);
  plan.items = reinterpret_cast<uint64_t*>(c + b_tabs);
  plan.ctabs = reinterpret_cast<MultiCuckoo*>(c + b_tabs + b_items);
  plan.citems = reinterpret_cast<uint64_t*>(c + b_tabs + b_items + b_ctabs);
  if (nt) e = hipMemcpy(plan.tabs, tabs.data(), sizeof(MultiTable) * nt, hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(plan.items, items.data(), items.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && nc) e = hipMemcpy(plan.ctabs, ctabs.data(), sizeof(MultiCuckoo) * nc, hipMemcpyHostToDevice);
  if (e == hipSuccess && !citems.empty())
    e = hipMemcpy(plan.citems, citems.data(), citems.size() * 8, hipMemcpyHostToDevice);
  return e;
}

void multi_plan_free(MultiPlanDev& plan) {
  if (plan.base) (void)hipFree(plan.base);
  plan = MultiPlanDev{};
}

hipError_t multi_plan_launch(const MultiPlanDev& plan, hipStream_t s) {
  if (plan.nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(multi_fill_kernel, dim3(plan.grid), dim3(kBlock), 0, s, plan.tabs, plan.items, plan.nitems);
  return hipGetLastError();
}

// The Cuckoo phases: `phase` 0 = probe and place, 1 = evict, 2 = scrub.
hipError_t multi_cuckoo_launch(const MultiPlanDev& plan, int phase, hipStream_t s) {
  if (plan.ncitems == 0) return hipSuccess;
  const dim3 g(plan.cgrid), b(kBlock);
  if (phase == 0)
    hipLaunchKernelGGL(multi_cuckoo_probe_kernel, g, b, 0, s, plan.ctabs, plan.citems, plan.ncitems);
  else if (phase == 1)
    hipLaunchKernelGGL(multi_cuckoo_evict_kernel, g, b, 0, s, plan.ctabs, plan.citems, plan.ncitems);
  else
    hipLaunchKernelGGL(multi_cuckoo_scrub_kernel, g, b, 0, s, plan.ctabs, plan.citems, plan.ncitems);
  return hipGetLastError();
}

// ---- per-launch descriptors (serving loop) -----------------------------------
// A launch group whose table set changes every time: its descriptors and
// items are packed one after another into a pinned host buffer owned by one
// stream slot and copied to that slot's device buffer with ONE copy on the
// launch stream, so nothing is allocated per group.  The caller reuses a slot
// only after its previous group has completed.

static size_t dyn_bytes(uint32_t cap_tabs, uint64_t cap_items) {
  return align256(sizeof(MultiTable) * cap_tabs) + align256(cap_items * 8) +
         align256(sizeof(MultiCuckoo) * cap_tabs) + align256(cap_items * 8) + align256(sizeof(MultiQuery) * cap_tabs);
}

hipError_t multi_dyn_alloc(MultiDyn& d, uint32_t cap_tabs, uint32_t cap_items) {
  d.cap_tabs = cap_tabs;
  d.cap_items = cap_items;
  const size_t bytes = dyn_bytes(cap_tabs, cap_items);
  hipError_t e = hipMalloc(&d.d_base, bytes);
  if (e != hipSuccess) return e;
  return hipHostMalloc(&d.h_base, bytes, hipHostMallocDefault);
}

void multi_dyn_free(MultiDyn& d) {
  if (d.d_base) (void)hipFree(d.d_base);
  if (d.h_base) (void)hipHostFree(d.h_base);
  d = MultiDyn{};
}

// Number of work items a table of n keys needs.
uint64_t multi_items_for(uint64_t n) { return (n + 63) / 64; }

hipError_t multi_dyn_issue(MultiDyn& d, const MultiSpec* specs, uint32_t nt, const MultiCuckooSpec* cspecs,
                           uint32_t nc, const MultiQuerySpec* qs, uint32_t nq, uint32_t max_blocks, hipStream_t s) {
  if (nt > d.cap_tabs || nc > d.cap_tabs || nq > d.cap_tabs) return hipErrorInvalidValue;
  const uint64_t max_waves = (uint64_t)max_blocks * (kBlock / kWave);
  char* h = static_cast<char*>(d.h_base);
  char* dv = static_cast<char*>(d.d_base);
  size_t o = 0;
  auto tabs = reinterpret_cast<MultiTable*>(h + o);
  const size_t o_tabs = o;
  o += align256(sizeof(MultiTable) * nt);
  const size_t o_items = o;
  const uint64_t nit = fill_bucketed(specs, nt, max_waves, tabs, reinterpret_cast<uint64_t*>(h + o), d.cap_items);
  if (nit == ~0ull) return hipErrorInvalidValue;
  o += align256(nit * 8);
  const size_t o_ctabs = o;
  o += align256(sizeof(MultiCuckoo) * nc);
  const size_t o_citems = o;
  const uint32_t cmb = cuckoo_blocks(max_blocks);
  const uint64_t ncit = fill_cuckoo(cspecs, nc, (uint64_t)cmb * (kBlock / kWave),
                                    reinterpret_cast<MultiCuckoo*>(h + o_ctabs), reinterpret_cast<uint64_t*>(h + o),
                                    d.cap_items);
  if (ncit == ~0ull) return hipErrorInvalidValue;
  o += align256(ncit * 8);
  const size_t o_qtabs = o;
  const uint64_t nqit = fill_query(qs, nq, max_waves, reinterpret_cast<MultiQuery*>(h + o_qtabs));
  o += align256(sizeof(MultiQuery) * nq);
  if (!nit && !ncit && !nqit) return hipSuccess;
  hipError_t e = hipMemcpyAsync(dv, h, o, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  if (nit)
    hipLaunchKernelGGL(multi_fill_kernel, dim3(multi_grid(nit, max_blocks)), dim3(kBlock), 0, s,
                       reinterpret_cast<const MultiTable*>(dv + o_tabs),
                       reinterpret_cast<const uint64_t*>(dv + o_items), (uint32_t)nit);
  if (ncit) {
    const dim3 g(multi_grid(ncit, cmb)), b(kBlock);
    const MultiCuckoo* ct = reinterpret_cast<const MultiCuckoo*>(dv + o_ctabs);
    const uint64_t* ci = reinterpret_cast<const uint64_t*>(dv + o_citems);
    hipLaunchKernelGGL(multi_cuckoo_probe_kernel, g, b, 0, s, ct, ci, (uint32_t)ncit);
    hipLaunchKernelGGL(multi_cuckoo_evict_kernel, g, b, 0, s, ct, ci, (uint32_t)ncit);
    hipLaunchKernelGGL(multi_cuckoo_scrub_kernel, g, b, 0, s, ct, ci, (uint32_t)ncit);
  }
  if (nqit) launch_query(reinterpret_cast<const MultiQuery*>(dv + o_qtabs), nq, nqit, max_blocks, s);
  return hipGetLastError();
}

hipError_t multi_query_once(const MultiQuerySpec* qs, uint32_t nq, uint32_t max_blocks, hipStream_t s) {
  const uint64_t max_waves = (uint64_t)max_blocks * (kBlock / kWave);
  std::vector<MultiQuery> tabs(nq);
  const uint64_t nit = fill_query(qs, nq, max_waves, tabs.data());
  if (!nit) return hipSuccess;
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, sizeof(MultiQuery) * nq);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(base, tabs.data(), sizeof(MultiQuery) * nq, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    launch_query(static_cast<const MultiQuery*>(base), nq, nit, max_blocks, s);
    e = hipGetLastError();
  }
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(base);
  return e != hipSuccess ? e : e2;
}

}  // namespace ht
