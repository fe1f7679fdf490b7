// Many bucketed tables in one persistent launch.
//
// The find-or-put of every bucketed table is cut into work items of equal
// size (a power of two between 256 and 4096 keys, chosen so that a launch has
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
// Cuckoo tables of a many-table call run their four phase kernels per table
// after this kernel, in the same stream order (see the host runtime): their
// phases need a grid-wide barrier between them, which kernel boundaries give.
#include <cstring>
#include <vector>

#include "bucketed_dev.h"
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

// Item size for a launch of `total` keys on a device with `max_waves` wave
// slots: a power of two in [256, 4096] giving about max_waves items.
uint64_t multi_chunk(uint64_t total, uint64_t max_waves) {
  uint64_t c = 256;
  while (c < 4096 && c * max_waves < total) c <<= 1;
  return c;
}

uint32_t multi_grid(uint64_t nitems, uint32_t max_blocks) {
  const uint64_t blocks = (nitems + (kBlock / kWave) - 1) / (kBlock / kWave);
  return (uint32_t)(blocks < max_blocks ? (blocks ? blocks : 1) : max_blocks);
}

// ---- host side ------------------------------------------------------------

struct MultiPlanDev {
  MultiTable* tabs = nullptr;
  uint64_t* items = nullptr;
  unsigned int* ctl = nullptr;
  void* base = nullptr;
  uint32_t nitems = 0;
  uint32_t nctl = 0;
  uint32_t grid = 0;
};

// Build descriptors and the item queue on the host and copy them to one
// device allocation (synchronous).  Returns hipSuccess or the HIP error.
hipError_t multi_plan_build(const std::vector<MultiSpec>& specs, uint32_t max_blocks, MultiPlanDev& plan) {
  const uint32_t nt = (uint32_t)specs.size();
  std::vector<MultiTable> tabs(nt);
  std::vector<uint64_t> items;
  uint64_t total = 0;
  for (const auto& sp : specs) total += sp.n;
  const uint64_t chunk = multi_chunk(total, (uint64_t)max_blocks * (kBlock / kWave));
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
  plan.nitems = (uint32_t)items.size();
  plan.grid = multi_grid(plan.nitems, max_blocks);
  plan.nctl = 0;
  const size_t b_tabs = (sizeof(MultiTable) * nt + 255) / 256 * 256;
  const size_t b_items = (items.size() * 8 + 255) / 256 * 256;
  const size_t b_ctl = 256;
  hipError_t e = hipMalloc(&plan.base, b_tabs + b_items + b_ctl);
  if (e != hipSuccess) return e;
  char* c = static_cast<char*>(plan.base);
  plan.tabs = reinterpret_cast<MultiTable*>(c);
  plan.items = reinterpret_cast<uint64_t*>(c + b_tabs);
  plan.ctl = reinterpret_cast<unsigned int*>(c + b_tabs + b_items);
  if (nt) e = hipMemcpy(plan.tabs, tabs.data(), sizeof(MultiTable) * nt, hipMemcpyHostToDevice);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpy(plan.items, items.data(), items.size() * 8, hipMemcpyHostToDevice);
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

// ---- per-launch descriptors (serving loop) -----------------------------------
// A launch whose table set changes every time: descriptors and items are
// written into pinned host buffers owned by one stream slot and copied to
// that slot's device buffers on the launch stream, so nothing is allocated
// per launch.  The caller reuses a slot only after its previous launch has
// completed.

hipError_t multi_dyn_alloc(MultiDyn& d, uint32_t cap_tabs, uint32_t cap_items) {
  d.cap_tabs = cap_tabs;
  d.cap_items = cap_items;
  const size_t b_tabs = (sizeof(MultiTable) * cap_tabs + 255) / 256 * 256;
  const size_t b_items = ((size_t)cap_items * 8 + 255) / 256 * 256;
  hipError_t e = hipMalloc(&d.d_base, b_tabs + b_items + 256);
  if (e != hipSuccess) return e;
  e = hipHostMalloc(&d.h_base, b_tabs + b_items, hipHostMallocDefault);
  if (e != hipSuccess) return e;
  char* c = static_cast<char*>(d.d_base);
  d.d_tabs = reinterpret_cast<MultiTable*>(c);
  d.d_items = reinterpret_cast<uint64_t*>(c + b_tabs);
  d.d_ctl = reinterpret_cast<unsigned int*>(c + b_tabs + b_items);
  char* h = static_cast<char*>(d.h_base);
  d.h_tabs = reinterpret_cast<MultiTable*>(h);
  d.h_items = reinterpret_cast<uint64_t*>(h + b_tabs);
  return hipSuccess;
}

void multi_dyn_free(MultiDyn& d) {
  if (d.d_base) (void)hipFree(d.d_base);
  if (d.h_base) (void)hipHostFree(d.h_base);
  d = MultiDyn{};
}

// Number of work items a table of n keys needs.
uint64_t multi_items_for(uint64_t n) { return (n + 255) / 256; }

hipError_t multi_dyn_launch(MultiDyn& d, const MultiSpec* specs, uint32_t nt, uint32_t max_blocks, hipStream_t s) {
  if (nt > d.cap_tabs) return hipErrorInvalidValue;
  uint64_t total = 0;
  for (uint32_t i = 0; i < nt; ++i) total += specs[i].n;
  const uint64_t chunk = multi_chunk(total, (uint64_t)max_blocks * (kBlock / kWave));
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
  if (nitems == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(d.d_tabs, d.h_tabs, sizeof(MultiTable) * nt, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d.d_items, d.h_items, (size_t)nitems * 8, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(multi_fill_kernel, dim3(multi_grid(nitems, max_blocks)), dim3(kBlock), 0, s, d.d_tabs,
                     d.d_items, nitems);
  return hipGetLastError();
}

}  // namespace ht
