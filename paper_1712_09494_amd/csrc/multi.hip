// Many bucketed tables in one persistent launch.
//
// The find-or-put of every bucketed table is cut into work items of equal
// size (a power of two between 64 and 4096 keys, chosen so that a launch has
// about as many items as the device has wave slots); wave w takes items w,
// w + W, w + 2W, ... of the queue.  The items are equal, so this static
// split balances, and it needs no shared queue counter (a counter popped by
// every wave of a large grid serialises on one address).  Each wave runs the
// same wave-level bucket probe as the single-table kernel, with the bucket
// width taken from each table at run time (one code path for 8/16/32/64
// slots, one key per lane group in flight, so the kernel keeps the
// occupancy of the single-table kernels).  Tables may mix bucket widths and
// hash counts; each uses its own storage, so the results equal one
// find-or-put call per table.  The launch allocates nothing and uses no
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
    const unsigned long long nnew = bucketed_fop_range<0, 1, false, true>(m.t, m.keys, begin, end, m.out);
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
    cuckoo_evict_region<false>(m.t, m.n, m.out, m.s, it & kRegionMask, nnew, nevict);
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

// Item size for a launch of `total` keys on a device with `max_waves` wave
// slots: a power of two in [64, 4096] giving about max_waves items (small
// launches still fill every wave slot).
uint64_t multi_chunk(uint64_t total, uint64_t max_waves) {
  uint64_t c = 64;
  while (c < 4096 && c * max_waves < total) c <<= 1;
  return c;
}

uint32_t multi_grid(uint64_t nitems, uint32_t max_blocks) {
  const uint64_t blocks = (nitems + (kBlock / kWave) - 1) / (kBlock / kWave);
  return (uint32_t)(blocks < max_blocks ? (blocks ? blocks : 1) : max_blocks);
}

// ---- host side ------------------------------------------------------------

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

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Build descriptors and the item lists on the host and copy them to one
// device allocation (synchronous).  Returns hipSuccess or the HIP error
// (hipErrorInvalidValue when a Cuckoo table's scratch has too few per-wave
// counts for its regions).
hipError_t multi_plan_build(const std::vector<MultiSpec>& specs, const std::vector<MultiCuckooSpec>& cspecs,
                            uint32_t max_blocks, MultiPlanDev& plan) {
  const uint64_t max_waves = (uint64_t)max_blocks * (kBlock / kWave);
  const uint32_t nt = (uint32_t)specs.size();
  std::vector<MultiTable> tabs(nt);
  std::vector<uint64_t> items;
  uint64_t total = 0;
  for (const auto& sp : specs) total += sp.n;
  const uint64_t chunk = multi_chunk(total, max_waves);
  for (uint32_t i = 0; i < nt; ++i) {
    const MultiSpec& sp = specs[i];
    MultiTable& m = tabs[i];
    std::memset(&m, 0, sizeof(m));
    m.t = sp.t;
    m.keys = sp.keys;
    m.out = sp.out;
    m.n = sp.n;
    m.chunk = chunk;
    m.nregions = sp.n ? (uint32_t)((sp.n + m.chunk - 1) / m.chunk) : 0;
    for (uint64_t r = 0; r < m.nregions; ++r) items.push_back(make_item(i, r));
  }
  const uint32_t nc = (uint32_t)cspecs.size();
  std::vector<MultiCuckoo> ctabs(nc);
  uint64_t cap_c = 0;
  for (const auto& sp : cspecs) cap_c += multi_items_for(sp.n);
  std::vector<uint64_t> citems(cap_c);
  const uint64_t ncit = fill_cuckoo(cspecs.data(), nc, max_waves, ctabs.data(), citems.data(), cap_c);
  if (ncit == ~0ull) return hipErrorInvalidValue;
  citems.resize(ncit);
  plan.nitems = (uint32_t)items.size();
  plan.ncitems = (uint32_t)citems.size();
  plan.grid = multi_grid(plan.nitems, max_blocks);
  plan.cgrid = multi_grid(plan.ncitems, max_blocks);
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
// A launch whose table set changes every time: descriptors and items are
// written into pinned host buffers owned by one stream slot and copied to
// that slot's device buffers on the launch stream, so nothing is allocated
// per launch.  The caller reuses a slot only after its previous launch has
// completed.

hipError_t multi_dyn_alloc(MultiDyn& d, uint32_t cap_tabs, uint32_t cap_items) {
  d.cap_tabs = cap_tabs;
  d.cap_items = cap_items;
  const size_t b_tabs = align256(sizeof(MultiTable) * cap_tabs);
  const size_t b_items = align256((size_t)cap_items * 8);
  const size_t b_ctabs = align256(sizeof(MultiCuckoo) * cap_tabs);
  const size_t bytes = b_tabs + 2 * b_items + b_ctabs;
  hipError_t e = hipMalloc(&d.d_base, bytes);
  if (e != hipSuccess) return e;
  e = hipHostMalloc(&d.h_base, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  char* c = static_cast<char*>(d.d_base);
  char* h = static_cast<char*>(d.h_base);
  d.d_tabs = reinterpret_cast<MultiTable*>(c);
  d.h_tabs = reinterpret_cast<MultiTable*>(h);
  d.d_items = reinterpret_cast<uint64_t*>(c + b_tabs);
  d.h_items = reinterpret_cast<uint64_t*>(h + b_tabs);
  d.d_ctabs = reinterpret_cast<MultiCuckoo*>(c + b_tabs + b_items);
  d.h_ctabs = reinterpret_cast<MultiCuckoo*>(h + b_tabs + b_items);
  d.d_citems = reinterpret_cast<uint64_t*>(c + b_tabs + b_items + b_ctabs);
  d.h_citems = reinterpret_cast<uint64_t*>(h + b_tabs + b_items + b_ctabs);
  return hipSuccess;
}

void multi_dyn_free(MultiDyn& d) {
  if (d.d_base) (void)hipFree(d.d_base);
  if (d.h_base) (void)hipHostFree(d.h_base);
  d = MultiDyn{};
}

// Number of work items a table of n keys needs.
uint64_t multi_items_for(uint64_t n) { return (n + 63) / 64; }

hipError_t multi_dyn_launch(MultiDyn& d, const MultiSpec* specs, uint32_t nt, const MultiCuckooSpec* cspecs,
                            uint32_t nc, uint32_t max_blocks, hipStream_t s) {
  if (nt > d.cap_tabs || nc > d.cap_tabs) return hipErrorInvalidValue;
  const uint64_t max_waves = (uint64_t)max_blocks * (kBlock / kWave);
  uint64_t total = 0;
  for (uint32_t i = 0; i < nt; ++i) total += specs[i].n;
  const uint64_t chunk = multi_chunk(total, max_waves);
  uint32_t nitems = 0;
  for (uint32_t i = 0; i < nt; ++i) {
    MultiTable& m = d.h_tabs[i];
    std::memset(&m, 0, sizeof(m));
    m.t = specs[i].t;
    m.keys = specs[i].keys;
    m.out = specs[i].out;
    m.n = specs[i].n;
    m.chunk = chunk;
    m.nregions = (uint32_t)((specs[i].n + chunk - 1) / chunk);
    if (nitems + m.nregions > d.cap_items) return hipErrorInvalidValue;
    for (uint64_t r = 0; r < m.nregions; ++r) d.h_items[nitems++] = make_item(i, r);
  }
  const uint64_t ncit = fill_cuckoo(cspecs, nc, max_waves, d.h_ctabs, d.h_citems, d.cap_items);
  if (ncit == ~0ull) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (nitems) {
    e = hipMemcpyAsync(d.d_tabs, d.h_tabs, sizeof(MultiTable) * nt, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d.d_items, d.h_items, (size_t)nitems * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(multi_fill_kernel, dim3(multi_grid(nitems, max_blocks)), dim3(kBlock), 0, s, d.d_tabs,
                       d.d_items, nitems);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ncit) {
    e = hipMemcpyAsync(d.d_ctabs, d.h_ctabs, sizeof(MultiCuckoo) * nc, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d.d_citems, d.h_citems, (size_t)ncit * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const dim3 g(multi_grid(ncit, max_blocks)), b(kBlock);
    hipLaunchKernelGGL(multi_cuckoo_probe_kernel, g, b, 0, s, d.d_ctabs, d.d_citems, (uint32_t)ncit);
    hipLaunchKernelGGL(multi_cuckoo_evict_kernel, g, b, 0, s, d.d_ctabs, d.d_citems, (uint32_t)ncit);
    hipLaunchKernelGGL(multi_cuckoo_scrub_kernel, g, b, 0, s, d.d_ctabs, d.d_citems, (uint32_t)ncit);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace ht
