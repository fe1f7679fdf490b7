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

// Per-stream-slot descriptor buffers for launches whose table set changes
// every time (pinned host staging + device copy; nothing allocated per launch).
struct MultiDyn {
  MultiTable* d_tabs = nullptr;
  uint64_t* d_items = nullptr;
  unsigned int* d_ctl = nullptr;
  MultiTable* h_tabs = nullptr;
  uint64_t* h_items = nullptr;
  void* d_base = nullptr;
  void* h_base = nullptr;
  uint32_t cap_tabs = 0, cap_items = 0;
};

hipError_t multi_dyn_alloc(MultiDyn& d, uint32_t cap_tabs, uint32_t cap_items);
void multi_dyn_free(MultiDyn& d);
uint64_t multi_items_for(uint64_t n);
hipError_t multi_dyn_launch(MultiDyn& d, const MultiSpec* specs, uint32_t nt, uint32_t max_blocks, hipStream_t s);

}  // namespace ht
