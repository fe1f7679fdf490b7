// The allocation-free find-or-put: the same kernels as ht_find_or_put, with
// the Cuckoo insertion's scratch (deduplication set, listed keys and their
// indices, per-wave list counts) in a file-scope device array instead of
// table-owned memory that grows on demand.  For callers that cannot
// allocate.  Every call on one device shares that device's array.
#include <mutex>

#include "runtime.h"

namespace ht {
hipError_t fill_words(uint64_t*, uint64_t, uint64_t, hipStream_t);
}  // namespace ht

using namespace ht;
using namespace ht_rt;

namespace {

constexpr uint64_t kNoAllocMaxKeys = 1ull << 18;            // largest batch
constexpr uint64_t kDsetWords = 2 * kNoAllocMaxKeys;        // deduplication set: a power of two >= 2n
constexpr uint64_t kWcntWords = 8192;                       // room for 16384 per-wave counts (4 bytes each)
constexpr uint64_t kScratchWords = kDsetWords + 2 * kNoAllocMaxKeys + kWcntWords;   // 8.06 MiB
constexpr int kMaxDevices = 64;

std::mutex g_mu;
uint64_t* g_ptr[kMaxDevices] = {};                          // device address of `scratch`, per device

}  // namespace

// In host code this name is a host-side stand-in; kernels get the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint64_t scratch[kScratchWords];

namespace {

// Device address of this device's `scratch` (looked up once per device,
// with that device current).
int scratch_address(int dev, uint64_t** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    uint64_t* p = nullptr;
    hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return HT_OK;
}

struct QuietLaunches {              // no timing events while the call launches
  QuietLaunches() { g_quiet = true; }
  ~QuietLaunches() { g_quiet = false; }
};

}  // namespace

extern "C" int ht_find_or_put_noalloc(ht_table* t, const uint64_t* d_keys, uint64_t n, uint8_t* d_out_is_new,
                                      hipStream_t s) {
  int rc = check_table(t);
  if (rc) return rc;
  if (n == 0) return HT_OK;
  if (!d_keys) return fail(HT_EINVAL, "keys is NULL");
  if (n > kNoAllocMaxKeys) return fail(HT_EINVAL, "batch above 262144 keys, the limit of the static scratch");
  if (t->cfg.key_words > 1) return fail(HT_EINVAL, "the allocation-free call serves tables of single-word keys");
  int dev = -1;
  HT_HIP(hipGetDevice(&dev));
  if (dev != t->device) return fail(HT_EINVAL, "the table's device must be the current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(HT_EINVAL, "device index above 63");
  QuietLaunches quiet;
  // bucketed tables and the single-pass Cuckoo ablation use no scratch at all
  if (t->cfg.kind == HT_BUCKETED || (t->cfg.flags & HT_FLAG_CUCKOO_SINGLE_PASS))
    return do_find_or_put(t, d_keys, n, d_out_is_new, s);
  if ((uint64_t)max_blocks(t) * (kBlock / kWave) > 2 * kWcntWords)
    return fail(HT_EINVAL, "device has more wave slots than the static scratch counts");
  uint64_t* base = nullptr;
  rc = scratch_address(dev, &base);
  if (rc) return rc;
  CuckooScratch sc{};
  sc.dset = base;
  sc.dset_mask = pow2_at_least(std::max<uint64_t>(2 * n, 64)) - 1;
  sc.dset_seed = t->dset_seed;
  sc.wkey = base + kDsetWords;
  sc.wmeta = sc.wkey + kNoAllocMaxKeys;
  sc.wcnt = reinterpret_cast<uint32_t*>(sc.wmeta + kNoAllocMaxKeys);
  // The deduplication set must start empty; the array keeps what the last
  // call on this device left, so the part this call uses is filled first (a
  // fill kernel: no memset node when the caller captures a graph).  The lists
  // and counts are written before they are read.
  HT_HIP(fill_words(sc.dset, sc.dset_mask + 1, kEmpty, s));
  return do_find_or_put(t, d_keys, n, d_out_is_new, s, &sc);
}
