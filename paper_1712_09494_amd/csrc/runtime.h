// Host runtime internals shared by the C ABI (table.hip) and the serving
// engine (server.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ht_device.h"
#include "../../include/ht.h"

namespace ht_rt {

struct SplitMix {
  uint64_t s;
  uint64_t next() {
    s += 0x9e3779b97f4a7c15ull;
    return ht::mix64(s);
  }
};

}  // namespace ht_rt

struct ht_table {
  ht_config cfg;             // effective configuration (defaults filled in)
  ht_config user_cfg;        // as passed to ht_create
  int device = 0;
  uint32_t cus = 256;
  uint64_t nslots = 0;       // total slot words
  ht::DevTable dev{};
  ht_rt::SplitMix rng{0};
  void* storage = nullptr;   // slots | stash | overflow | counters | misc
  unsigned long long* misc = nullptr;
  // cuckoo scratch
  uint64_t scratch_n = 0;
  uint64_t dset_slots = 0;
  uint64_t dset_seed = 0;
  uint64_t* dset = nullptr;
  uint64_t* wkey = nullptr;
  uint64_t* wmeta = nullptr;
  uint32_t* wcnt = nullptr;
  // deferred scrub of the single-table Cuckoo find-or-put: its own set and
  // the record of the slots the last such call took (no other path uses them)
  uint64_t* dset_defer = nullptr;
  uint64_t* dirty = nullptr;
  uint32_t* dirty_cnt = nullptr;
  uint64_t* dirty_desc = nullptr;
  uint64_t dirty_stride = 0;
  // scripted hashes
  ht::ScriptRow* script = nullptr;
  uint32_t nscript = 0;
};

#define HT_HIP(call)                                           \
  do {                                                         \
    hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return ht_rt::hip_fail(e_, #call);   \
  } while (0)

namespace ht_rt {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
uint32_t device_cus(int dev);
uint32_t max_blocks(const ht_table* t);
uint32_t atomic_grid_blocks(const ht_table* t);
bool is_scripted(const ht_table* t);
int check_table(const ht_table* t);
int reserve_scratch(ht_table* t, uint64_t n);
ht::DevTable launch_view(const ht_table* t);
ht::CuckooScratch scratch_view(const ht_table* t, uint64_t n);   // per_wave left for the caller
// `fixed`: scratch provided by the caller (Cuckoo tables of single-word keys;
// per_wave is set here), instead of the table's own.
int do_find_or_put(ht_table* t, const uint64_t* keys, uint64_t n, uint8_t* out, hipStream_t s,
                   const ht::CuckooScratch* fixed = nullptr);
uint64_t pow2_at_least(uint64_t x);
extern thread_local bool g_quiet;   // set: launches create no timing events
int do_query(ht_table* t, const uint64_t* keys, uint64_t n, uint8_t* out, hipStream_t s);

}  // namespace ht_rt
