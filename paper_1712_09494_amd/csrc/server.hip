// Serving engine: replays a trace of find-or-put and query requests against
// resident tables with continuous batching.
//
// Requests carry pinned host keys and flags and an arrival time.  One host
// loop releases requests at their arrival times, retires finished launch
// groups (event polling), and admits pending requests into launch groups on
// free stream slots:
//   - per-table FIFO: a request is admitted only when no earlier request of
//     its table is pending or in flight, so each table sees its requests in
//     arrival order and every result equals the one the request gets alone
//     in that order;
//   - memory admission: each request above the small size needs device
//     staging for its keys and flags (9 bytes per key, 256-byte aligned
//     pieces) from a budget set at creation (by default a quarter of the free
//     device memory, at most 4 GiB); a request that does not fit waits, and
//     so do later requests of its table;
//   - merging: a group takes up to `merge` admissible requests of distinct
//     tables and up to `group_keys` keys (so small requests are not held
//     behind large ones); its find-or-puts run as many-table launches (one
//     for the bucketed tables, three phase launches for the Cuckoo tables),
//     its queries as one many-table query launch (a query large enough to
//     fill the device alone gets its own launch), all on the group's stream
//     between the host-to-device copies and the device-to-host copies;
//     requests on state-vector tables run their tables' own kernels inside
//     the group (the many-table launches take single-word keys);
//   - small requests: their keys are packed into the slot's pinned area and
//     sent with one copy, their flags returned with one (see kSmallKeyBytes);
//   - overlap: groups on different stream slots run concurrently.
// The sequential baseline runs one request at a time, waiting for each.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "multi.h"
#include "runtime.h"

using namespace ht;
using namespace ht_rt;

namespace {

// First-fit allocator over one device staging buffer.
class StagingPool {
 public:
  int init(uint64_t bytes) {
    bytes = bytes / 256 * 256;
    hipError_t e = hipMalloc(&base_, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(HT_ENOMEM, "hipMalloc of serving staging failed");
    }
    size_ = bytes;
    free_.assign(1, {0, bytes});
    return HT_OK;
  }
  // Every block free again (a run starts with nothing in flight).
  void reset() {
    free_.assign(1, {0, size_});
    used_ = 0;
  }
  void release_all() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }
  // offset of a block of `bytes` (multiple of 256), or ~0 when it does not fit
  uint64_t alloc(uint64_t bytes) {
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].second >= bytes) {
        const uint64_t off = free_[i].first;
        free_[i].first += bytes;
        free_[i].second -= bytes;
        if (!free_[i].second) free_.erase(free_.begin() + i);
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return off;
      }
    }
    return ~0ull;
  }
  void free(uint64_t off, uint64_t bytes) {
    used_ -= bytes;
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (uint64_t)0));
    it = free_.insert(it, {off, bytes});
    // coalesce with neighbours
    if (it + 1 != free_.end() && it->first + it->second == (it + 1)->first) {
      it->second += (it + 1)->second;
      free_.erase(it + 1);
    }
    if (it != free_.begin() && (it - 1)->first + (it - 1)->second == it->first) {
      (it - 1)->second += it->second;
      free_.erase(it);
    }
  }
  char* ptr(uint64_t off) const { return static_cast<char*>(base_) + off; }
  uint64_t size() const { return size_; }
  uint64_t peak() const { return peak_; }

 private:
  void* base_ = nullptr;
  uint64_t size_ = 0, used_ = 0, peak_ = 0;
  std::vector<std::pair<uint64_t, uint64_t>> free_;
};

// Small requests (keys of at most kSmallKeyBytes) skip the staging pool:
// each slot keeps a fixed device area and a pinned host area of the same
// layout -- up to kSmallKeysCap bytes of keys, then kSmallFlagsCap bytes of
// flags -- and a group's small requests are packed there by the host, so
// their keys go in with one copy and their flags come back with one.  A
// pinned copy costs about 10 us however small, while packing costs the
// host's memory copy (about 10 GB/s), so packing pays below about 100 KiB;
// 64 KiB measured best (served backlog 47-51 K req/s against 42-45 K at
// 256 KiB and 37-41 K unpacked).  The caps hold a whole group of them (at
// most 16 requests).
constexpr uint64_t kSmallKeyBytes = 64 << 10;
constexpr uint64_t kSmallKeysCap = 16 * kSmallKeyBytes;
constexpr uint64_t kSmallFlagsCap = 16 * (kSmallKeyBytes / 8);
constexpr uint64_t kSmallTag = 1ull << 63;   // offset of a request packed in its slot's small area

// Staging of one request: its keys (w words each) and its flags, each in
// 256-byte pieces (so vector keys keep the 16-byte alignment they need).
uint64_t key_bytes(uint64_t n, uint32_t w) { return (n * 8 * w + 255) / 256 * 256; }
uint64_t stage_bytes(uint64_t n, uint32_t w) { return key_bytes(n, w) + (n + 255) / 256 * 256; }

}  // namespace

struct ht_server {
  std::vector<ht_table*> tables;
  ht_server_config cfg{};
  StagingPool pool;
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    MultiDyn dyn;
    std::vector<uint32_t> reqs;          // requests of the group in flight
    std::vector<uint64_t> offs;          // their staging offsets (kSmallTag | key offset: small area)
    std::vector<uint64_t> foffs;         // small requests: flag offset in the small area
    char* d_small = nullptr;             // small area: kSmallKeysCap bytes of keys, then flags
    char* h_small = nullptr;             // its pinned host twin
    uint64_t small_keys = 0, small_flags = 0;   // bytes of each part in use
    bool busy = false;
  };
  std::vector<Slot> slots;
  uint32_t grid = 0;
};

extern "C" {

void ht_server_config_default(ht_server_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->slots = 16;
  cfg->merge = 16;
  cfg->group_keys = 1ull << 19;
}

int ht_server_create(ht_table* const* tables, uint32_t ntables, const ht_server_config* cfg, ht_server** out) {
  if (!out) return fail(HT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tables || ntables == 0) return fail(HT_EINVAL, "no tables");
  for (uint32_t i = 0; i < ntables; ++i) {
    int rc = check_table(tables[i]);
    if (rc) return rc;
    if (is_scripted(tables[i])) return fail(HT_EINVAL, "scripted-hash tables cannot be served");
  }
  ht_server_config c;
  ht_server_config_default(&c);
  if (cfg) c = *cfg;
  if (c.slots == 0) c.slots = 16;
  if (c.merge == 0) c.merge = 16;
  if (c.group_keys == 0) c.group_keys = 1ull << 19;
  if (c.slots > 16) return fail(HT_EINVAL, "at most 16 stream slots");
  if (c.sequential) {
    c.slots = 1;
    c.merge = 1;
  }
  if (c.staging_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 1ull << 32;
    c.staging_bytes = std::min<uint64_t>(fr / 4, 4ull << 30);
  }
  ht_server* s = new ht_server();
  s->tables.assign(tables, tables + ntables);
  s->cfg = c;
  int rc = s->pool.init(c.staging_bytes);
  if (rc) {
    delete s;
    return rc;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  s->grid = device_cus(dev) * 8;
  s->slots.resize(c.slots);
  for (auto& sl : s->slots) {
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sl.d_small), kSmallKeysCap + kSmallFlagsCap);
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void**>(&sl.h_small), kSmallKeysCap + kSmallFlagsCap, hipHostMallocDefault);
    if (e != hipSuccess) {
      ht_server_destroy(s);
      return hip_fail(e, "serving stream/event creation");
    }
  }
  *out = s;
  return HT_OK;
}

int ht_server_destroy(ht_server* s) {
  if (!s) return fail(HT_EINVAL, "server is NULL");
  (void)hipDeviceSynchronize();
  for (auto& sl : s->slots) {
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.d_small) (void)hipFree(sl.d_small);
    if (sl.h_small) (void)hipHostFree(sl.h_small);
    multi_dyn_free(sl.dyn);
  }
  s->pool.release_all();
  delete s;
  return HT_OK;
}

int ht_server_run(ht_server* s, ht_request* reqs, uint32_t nreq, ht_server_stats* stats) {
  if (!s) return fail(HT_EINVAL, "server is NULL");
  if (nreq && !reqs) return fail(HT_EINVAL, "requests is NULL");
  const uint32_t nt = (uint32_t)s->tables.size();
  uint64_t max_n = 0, max_stage = 0, total_keys = 0;
  std::vector<uint64_t> need(nt, 0);
  for (uint32_t i = 0; i < nreq; ++i) {
    const ht_request& r = reqs[i];
    if (r.table >= nt) return fail(HT_EINVAL, "request names a table the server does not hold");
    if (r.op != HT_OP_FIND_OR_PUT && r.op != HT_OP_QUERY) return fail(HT_EINVAL, "bad request op");
    if (r.n && (!r.h_keys || !r.h_out)) return fail(HT_EINVAL, "request with NULL keys or flags");
    if (s->tables[r.table]->cfg.key_words > 1 && r.n >= (1ull << (kArenaBits - 1)))
      return fail(HT_EINVAL, "vector request of 2^33 keys or more");
    max_n = std::max(max_n, r.n);
    max_stage = std::max(max_stage, stage_bytes(r.n, s->tables[r.table]->cfg.key_words));
    total_keys += r.n;
    if (r.op == HT_OP_FIND_OR_PUT) need[r.table] = std::max(need[r.table], r.n);
  }
  if (max_stage > s->pool.size()) return fail(HT_ENOMEM, "a request needs more staging than the server's budget");
  // a run starts with nothing in flight, also after an earlier run stopped on an error
  {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  }
  s->pool.reset();
  for (auto& sl : s->slots) {
    sl.reqs.clear();
    sl.offs.clear();
    sl.busy = false;
  }
  // everything that allocates happens before the clock starts
  for (uint32_t t = 0; t < nt; ++t)
    if ((s->tables[t]->cfg.kind == HT_CUCKOO || s->tables[t]->cfg.key_words > 1) && need[t]) {
      int rc = reserve_scratch(s->tables[t], need[t]);
      if (rc) return rc;
    }
  const uint32_t cap_items = (uint32_t)(s->cfg.merge * multi_items_for(std::max<uint64_t>(max_n, 1)));
  for (auto& sl : s->slots) {
    if (sl.dyn.cap_tabs < s->cfg.merge || sl.dyn.cap_items < cap_items) {
      multi_dyn_free(sl.dyn);
      hipError_t e = multi_dyn_alloc(sl.dyn, s->cfg.merge, cap_items);
      if (e != hipSuccess) return hip_fail(e, "serving descriptor buffers");
    }
  }
  {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  }

  std::vector<uint32_t> order(nreq);
  for (uint32_t i = 0; i < nreq; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return reqs[a].arrival_s < reqs[b].arrival_s; });
  std::deque<uint32_t> pending;
  std::vector<char> busy(nt, 0), blocked(nt, 0), in_group(nt, 0);
  uint32_t released = 0, completed = 0, groups = 0, merged = 0, throttled = 0, max_inflight = 0;
  const auto t0 = std::chrono::steady_clock::now();
  auto now_s = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  };
  std::vector<MultiSpec> specs;
  std::vector<MultiCuckooSpec> cspecs;
  std::vector<MultiQuerySpec> qspecs;
  specs.reserve(s->cfg.merge);
  cspecs.reserve(s->cfg.merge);
  int err = HT_OK;

  while (completed < nreq && err == HT_OK) {
    bool progress = false;
    double now = now_s();
    while (released < nreq && reqs[order[released]].arrival_s <= now) {
      pending.push_back(order[released++]);
      progress = true;
    }
    // retire finished groups
    for (auto& sl : s->slots) {
      if (!sl.busy) continue;
      hipError_t q = s->cfg.sequential ? hipEventSynchronize(sl.done) : hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        err = hip_fail(q, "serving completion event");
        break;
      }
      now = now_s();
      for (size_t k = 0; k < sl.reqs.size(); ++k) {
        ht_request& r = reqs[sl.reqs[k]];
        if (r.n && (sl.offs[k] & kSmallTag))
          std::memcpy(r.h_out, sl.h_small + kSmallKeysCap + sl.foffs[k], r.n);
        else if (r.n)
          s->pool.free(sl.offs[k], stage_bytes(r.n, s->tables[r.table]->cfg.key_words));
        r.done_s = now_s();
        busy[r.table] = 0;
        ++completed;
      }
      sl.reqs.clear();
      sl.offs.clear();
      sl.foffs.clear();
      sl.small_keys = sl.small_flags = 0;
      sl.busy = false;
      progress = true;
    }
    if (err) break;
    // admit pending requests into groups on free slots
    uint32_t inflight = 0;
    for (auto& sl : s->slots) inflight += sl.busy;
    for (uint32_t si = 0; si < s->slots.size() && !pending.empty(); ++si) {
      auto& sl = s->slots[si];
      if (sl.busy) continue;
      std::fill(blocked.begin(), blocked.end(), 0);
      std::fill(in_group.begin(), in_group.end(), 0);
      uint64_t group_n = 0;
      for (auto it = pending.begin(); it != pending.end() && sl.reqs.size() < s->cfg.merge;) {
        const uint32_t idx = *it;
        const uint32_t t = reqs[idx].table;
        if (!sl.reqs.empty() && group_n + reqs[idx].n > s->cfg.group_keys) {
          blocked[t] = 1;               // would overfill the group; keep order
          ++it;
          continue;
        }
        if (busy[t] || blocked[t] || in_group[t]) {
          blocked[t] = 1;               // keep this table's requests in arrival order
          ++it;
          continue;
        }
        const uint32_t w = s->tables[t]->cfg.key_words;
        const uint64_t kb = key_bytes(reqs[idx].n, w), fb = (reqs[idx].n + 255) / 256 * 256;
        uint64_t off = 0, foff = ~0ull;
        if (reqs[idx].n && kb <= kSmallKeyBytes && sl.small_keys + kb <= kSmallKeysCap &&
            sl.small_flags + fb <= kSmallFlagsCap) {
          off = kSmallTag | sl.small_keys;          // packed in the slot's small area
          foff = sl.small_flags;
          sl.small_keys += kb;
          sl.small_flags += fb;
        } else {
          const uint64_t sb = stage_bytes(reqs[idx].n, w);
          off = sb ? s->pool.alloc(sb) : 0;
          if (off == ~0ull) {
            ++throttled;
            blocked[t] = 1;
            ++it;
            continue;
          }
        }
        sl.reqs.push_back(idx);
        sl.offs.push_back(off);
        sl.foffs.push_back(foff);
        group_n += reqs[idx].n;
        in_group[t] = 1;
        busy[t] = 1;
        reqs[idx].admit_s = now_s();
        reqs[idx].slot = si;
        reqs[idx].group = groups;
        it = pending.erase(it);
      }
      if (sl.reqs.empty()) break;       // nothing admissible now
      // issue: keys in, kernels, flags out, completion event
      hipStream_t st = sl.stream;
      specs.clear();
      cspecs.clear();
      qspecs.clear();
      // where request k's keys and flags sit on the device
      auto dkeys = [&](size_t k) -> uint64_t* {
        const uint64_t o = sl.offs[k];
        return reinterpret_cast<uint64_t*>((o & kSmallTag) ? sl.d_small + (o & ~kSmallTag) : s->pool.ptr(o));
      };
      auto dflags = [&](size_t k) -> uint8_t* {
        const uint64_t o = sl.offs[k];
        const ht_request& r = reqs[sl.reqs[k]];
        if (o & kSmallTag) return reinterpret_cast<uint8_t*>(sl.d_small + kSmallKeysCap + sl.foffs[k]);
        return reinterpret_cast<uint8_t*>(s->pool.ptr(o) + key_bytes(r.n, s->tables[r.table]->cfg.key_words));
      };
      for (size_t k = 0; k < sl.reqs.size() && err == HT_OK; ++k) {
        const ht_request& r = reqs[sl.reqs[k]];
        if (!r.n) continue;
        const uint64_t bytes = r.n * 8 * s->tables[r.table]->cfg.key_words;
        if (sl.offs[k] & kSmallTag) {
          std::memcpy(sl.h_small + (sl.offs[k] & ~kSmallTag), r.h_keys, bytes);   // packed, sent below
          continue;
        }
        hipError_t e = hipMemcpyAsync(dkeys(k), r.h_keys, bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) err = hip_fail(e, "serving key copy");
      }
      if (err == HT_OK && sl.small_keys) {
        hipError_t e = hipMemcpyAsync(sl.d_small, sl.h_small, sl.small_keys, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) err = hip_fail(e, "serving key copy");
      }
      for (size_t k = 0; k < sl.reqs.size() && err == HT_OK; ++k) {
        const ht_request& r = reqs[sl.reqs[k]];
        if (!r.n) continue;
        ht_table* tb = s->tables[r.table];
        uint64_t* dk = dkeys(k);
        uint8_t* dflag = dflags(k);
        if (tb->cfg.key_words > 1) {
          // vector tables: their own kernels (the many-table launches take single-word keys)
          err = r.op == HT_OP_FIND_OR_PUT ? do_find_or_put(tb, dk, r.n, dflag, st) : do_query(tb, dk, r.n, dflag, st);
        } else if (r.op == HT_OP_FIND_OR_PUT && tb->cfg.kind == HT_BUCKETED && s->cfg.merge > 1) {
          specs.push_back(MultiSpec{launch_view(tb), dk, dflag, r.n});
        } else if (r.op == HT_OP_FIND_OR_PUT && s->cfg.merge > 1) {
          MultiCuckooSpec cs{};
          cs.t = launch_view(tb);
          cs.s = scratch_view(tb, r.n);
          cs.keys = dk;
          cs.out = dflag;
          cs.n = r.n;
          cs.max_regions = (uint64_t)max_blocks(tb) * (kBlock / kWave);
          cs.paper = (tb->cfg.flags & HT_FLAG_CUCKOO_PAPER_ORDER) != 0;
          cspecs.push_back(cs);
        } else if (r.op == HT_OP_FIND_OR_PUT) {
          err = do_find_or_put(tb, dk, r.n, dflag, st);
        } else {
          const MultiQuerySpec q{launch_view(tb), dk, dflag, r.n, tb->cfg.kind == HT_CUCKOO};
          if (s->cfg.merge > 1 && !multi_query_alone(q, s->grid))
            qspecs.push_back(q);
          else
            err = do_query(tb, dk, r.n, dflag, st);
        }
      }
      if (err == HT_OK && !(specs.empty() && cspecs.empty() && qspecs.empty())) {
        hipError_t e = multi_dyn_issue(sl.dyn, specs.data(), (uint32_t)specs.size(), cspecs.data(),
                                       (uint32_t)cspecs.size(), qspecs.data(), (uint32_t)qspecs.size(), s->grid, st);
        if (e != hipSuccess) err = hip_fail(e, "serving many-table launch");
        ++merged;
      }
      for (size_t k = 0; k < sl.reqs.size() && err == HT_OK; ++k) {
        const ht_request& r = reqs[sl.reqs[k]];
        if (!r.n || (sl.offs[k] & kSmallTag)) continue;
        hipError_t e = hipMemcpyAsync(r.h_out, dflags(k), r.n, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) err = hip_fail(e, "serving flag copy");
      }
      if (err == HT_OK && sl.small_flags) {   // unpacked into the requests' flags when the group retires
        hipError_t e = hipMemcpyAsync(sl.h_small + kSmallKeysCap, sl.d_small + kSmallKeysCap, sl.small_flags,
                                      hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) err = hip_fail(e, "serving flag copy");
      }
      if (err == HT_OK) {
        hipError_t e = hipEventRecord(sl.done, st);
        if (e != hipSuccess) err = hip_fail(e, "serving event record");
      }
      sl.busy = true;
      ++groups;
      ++inflight;
      max_inflight = std::max(max_inflight, inflight);
      progress = true;
    }
    if (!progress) {
      // idle: nothing finished, nothing admissible; wait a little
      if (released < nreq && pending.empty() && reqs[order[released]].arrival_s - now_s() > 200e-6)
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  }
  const double wall = now_s();
  if (err == HT_OK) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) err = hip_fail(e, "hipDeviceSynchronize");
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->wall_s = wall;
    stats->keys = total_keys;
    stats->groups = groups;
    stats->merged_launches = merged;
    stats->max_inflight_groups = max_inflight;
    stats->throttled = throttled;
    stats->peak_staging = s->pool.peak();
    stats->staging_bytes = s->pool.size();
  }
  return err;
}

}  // extern "C"
