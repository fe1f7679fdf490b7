/* A plain C program using the library through include/ht.h only: device
 * buffers from the HIP runtime API, tables created, filled, queried and
 * sized, results checked here.  Exit status 0 when every check passes. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ht.h"

#define N 100000u

static int check(int rc, const char* what) {
  if (rc != HT_OK) {
    fprintf(stderr, "%s: %s (%s)\n", what, ht_strerror(rc), ht_last_error());
    return 1;
  }
  return 0;
}

static int run(uint32_t kind) {
  uint64_t* h_keys = (uint64_t*)malloc(2 * N * sizeof(uint64_t));
  uint8_t* h_flags = (uint8_t*)malloc(2 * N);
  if (!h_keys || !h_flags) return 1;
  for (uint64_t i = 0; i < N; ++i) {           /* N distinct keys, each twice */
    h_keys[i] = i * 0x9E3779B97F4A7C15ull + 17;
    h_keys[N + i] = h_keys[i];
  }
  uint64_t* d_keys = NULL;
  uint8_t* d_flags = NULL;
  if (hipMalloc((void**)&d_keys, 2 * N * sizeof(uint64_t)) != hipSuccess) return 1;
  if (hipMalloc((void**)&d_flags, 2 * N) != hipSuccess) return 1;
  if (hipMemcpy(d_keys, h_keys, 2 * N * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) return 1;

  ht_table* t = NULL;
  int bad = check(ht_create_simple(kind, 2 * N, 3, &t), "ht_create_simple");
  bad |= check(ht_find_or_put(t, d_keys, 2 * N, d_flags, NULL), "ht_find_or_put");
  if (hipMemcpy(h_flags, d_flags, 2 * N, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  uint64_t news = 0;
  for (uint64_t i = 0; i < 2 * N; ++i) news += h_flags[i];
  for (uint64_t i = 0; i < N; ++i)              /* exactly one of the two copies is new */
    if (h_flags[i] + h_flags[N + i] != 1) bad = 1;
  bad |= check(ht_query(t, d_keys, N, d_flags, NULL), "ht_query");
  if (hipMemcpy(h_flags, d_flags, N, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  for (uint64_t i = 0; i < N; ++i)
    if (h_flags[i] != 1) bad = 1;
  uint64_t size = 0;
  bad |= check(ht_size(t, &size, NULL), "ht_size");
  bad |= check(ht_sync_status(t, NULL), "ht_sync_status");
  if (news != N || size != N) bad = 1;
  printf("kind %u: new %llu size %llu %s\n", kind, (unsigned long long)news, (unsigned long long)size,
         bad ? "FAIL" : "ok");
  bad |= check(ht_destroy(t), "ht_destroy");
  hipFree(d_keys);
  hipFree(d_flags);
  free(h_keys);
  free(h_flags);
  return bad;
}

int main(void) {
  int bad = run(HT_BUCKETED);
  bad |= run(HT_CUCKOO);
  return bad ? 1 : 0;
}
