// Many bucketed tables in one persistent launch.
//
// The find-or-put of every bucketed table is cut into work items of 4096
// keys; resident waves take items in queue order through one atomic counter
// and run the same wave-level bucket probe as the single-table kernel, with
// the bucket width taken from each table at run time (one code path for
// 8/16/32/64 slots, one key per lane group in flight, so the kernel keeps
// the occupancy of the single-table kernels).  Items never wait on each
// other, so the queue drains as fast as the waves work.  Tables may mix
// bucket widths and hash counts; each uses its own storage, so the results
// equal one find-or-put call per table.  The launch allocates nothing and
// uses no memset, so it can be captured in a HIP graph.
//
// Cuckoo tables of a many-table call run their four phase kernels per table
// after this kernel, in the same stream order (see the host runtime): their
// phases need a grid-wide barrier between them, which kernel boundaries give.
#include <cstring>
#include <vector>

#include "bucketed_dev.h"

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

// ctl[0]: queue head
__global__ void multi_reset_kernel(unsigned int* ctl, uint32_t nwords) {
  for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) ctl[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void multi_fill_kernel(const MultiTable* __restrict__ tabs,
                                                            const uint64_t* __restrict__ items, uint32_t nitems,
                                                            unsigned int* ctl) {
  const int lane = lane_id();
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  for (;;) {
    unsigned int idx = 0;
    if (lane == 0) idx = add_agent(&ctl[0], 1u);
    idx = __builtin_amdgcn_readfirstlane(idx);
    if (idx >= nitems) break;
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

// ---- host side ------------------------------------------------------------

struct MultiSpec {
  DevTable t;
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
};

struct MultiPlanDev {
  MultiTable* tabs = nullptr;
  uint64_t* items = nullptr;
  unsigned int* ctl = nullptr;
  void* base = nullptr;
  uint32_t nitems = 0;
  uint32_t nctl = 0;
};

// Build descriptors and the item queue on the host and copy them to one
// device allocation (synchronous).  Returns hipSuccess or the HIP error.
hipError_t multi_plan_build(const std::vector<MultiSpec>& specs, MultiPlanDev& plan) {
  const uint32_t nt = (uint32_t)specs.size();
  std::vector<MultiTable> tabs(nt);
  std::vector<uint64_t> items;
  for (uint32_t i = 0; i < nt; ++i) {
    const MultiSpec& sp = specs[i];
    MultiTable& m = tabs[i];
    std::memset(&m, 0, sizeof(m));
    m.t = sp.t;
    m.keys = sp.keys;
    m.out = sp.out;
    m.n = sp.n;
    m.chunk = 4096;
    m.nregions = sp.n ? (uint32_t)((sp.n + m.chunk - 1) / m.chunk) : 0;
    for (uint64_t r = 0; r < m.nregions; ++r) items.push_back(make_item(i, r));
  }
  plan.nitems = (uint32_t)items.size();
  plan.nctl = 2;
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

hipError_t multi_plan_launch(const MultiPlanDev& plan, uint32_t grid, hipStream_t s) {
  if (plan.nitems == 0) return hipSuccess;
  hipLaunchKernelGGL(multi_reset_kernel, dim3(1), dim3(kBlock), 0, s, plan.ctl, plan.nctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(multi_fill_kernel, dim3(grid), dim3(kBlock), 0, s, plan.tabs, plan.items, plan.nitems,
                     plan.ctl);
  return hipGetLastError();
}

}  // namespace ht
