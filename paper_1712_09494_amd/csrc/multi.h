// Many-table launches: shared declarations (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ht_device.h"

namespace ht {

struct MultiTable;

// One table of a many-table launch.
struct MultiSpec {
  DevTable t;
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
};

// One Cuckoo table of a many-table launch.  `s` is the table's scratch view
// (per_wave is set by the plan); max_regions is the number of per-wave
// counts the scratch holds.
struct MultiCuckooSpec {
  DevTable t;
  CuckooScratch s;
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
  uint64_t max_regions;
  bool paper;
};

// Per-stream-slot descriptor buffers for launches whose table set changes
// every time (pinned host staging + device copy; nothing allocated per launch).
struct MultiCuckoo;

struct MultiDyn {
  MultiTable* d_tabs = nullptr;
  uint64_t* d_items = nullptr;
  MultiTable* h_tabs = nullptr;
  uint64_t* h_items = nullptr;
  MultiCuckoo* d_ctabs = nullptr;
  uint64_t* d_citems = nullptr;
  MultiCuckoo* h_ctabs = nullptr;
  uint64_t* h_citems = nullptr;
  void* d_base = nullptr;
  void* h_base = nullptr;
  uint32_t cap_tabs = 0, cap_items = 0;   // per kind
};

// A prepared many-table launch: descriptors and item lists in one device
// allocation.
struct MultiPlanDev {
  MultiTable* tabs = nullptr;       // bucketed tables
  uint64_t* items = nullptr;
  MultiCuckoo* ctabs = nullptr;     // Cuckoo tables
  uint64_t* citems = nullptr;
  void* base = nullptr;
  uint32_t nitems = 0, ncitems = 0;
  uint32_t grid = 0, cgrid = 0;
};

hipError_t multi_plan_build(const std::vector<MultiSpec>& specs, const std::vector<MultiCuckooSpec>& cspecs,
                            uint32_t max_blocks, MultiPlanDev& plan);
void multi_plan_free(MultiPlanDev& plan);
hipError_t multi_plan_launch(const MultiPlanDev& plan, hipStream_t s);
hipError_t multi_cuckoo_launch(const MultiPlanDev& plan, int phase, hipStream_t s);

hipError_t multi_dyn_alloc(MultiDyn& d, uint32_t cap_tabs, uint32_t cap_items);
void multi_dyn_free(MultiDyn& d);
uint64_t multi_items_for(uint64_t n);
// Bucketed tables in one persistent launch, then the three Cuckoo phase
// launches over the Cuckoo tables; all on stream s.
hipError_t multi_dyn_launch(MultiDyn& d, const MultiSpec* specs, uint32_t nt, const MultiCuckooSpec* cspecs,
                            uint32_t nc, uint32_t max_blocks, hipStream_t s);

}  // namespace ht
