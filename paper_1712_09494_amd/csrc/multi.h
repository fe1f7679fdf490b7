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

// One table of a many-table query (either kind).
struct MultiQuerySpec {
  DevTable t;
  const uint64_t* keys;
  uint8_t* out;
  uint64_t n;
  bool cuckoo;
};

// Per-stream-slot descriptor buffers for launches whose table set changes
// every time (pinned host staging + device copy; nothing allocated per launch).
struct MultiCuckoo;
struct MultiQuery;

struct MultiDyn {
  void* d_base = nullptr;
  void* h_base = nullptr;
  uint32_t cap_tabs = 0;     // tables per kind
  uint32_t cap_items = 0;    // find-or-put items per kind
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
// One launch group on stream s: one copy of every descriptor, then the
// bucketed find-or-puts in one persistent launch, the three Cuckoo phase
// launches, and the queries of every table (either kind) in one launch.
hipError_t multi_dyn_issue(MultiDyn& d, const MultiSpec* specs, uint32_t nt, const MultiCuckooSpec* cspecs,
                           uint32_t nc, const MultiQuerySpec* qs, uint32_t nq, uint32_t max_blocks, hipStream_t s);
// True when a query batch alone gives every wave slot of a max_blocks grid
// a turn: such a batch is better served by the single-table query, which
// keeps its table's probes together in cache (measured on 256 tables of
// 2^6..2^26 slots: merged large batches ran 10-20% slower than one launch
// per table), while smaller batches gain from sharing one launch.
bool multi_query_alone(const MultiQuerySpec& q, uint32_t max_blocks);
// Queries of nq tables in one launch, allocating the descriptors and
// synchronising s (one-off calls).
hipError_t multi_query_once(const MultiQuerySpec* qs, uint32_t nq, uint32_t max_blocks, hipStream_t s);

}  // namespace ht
