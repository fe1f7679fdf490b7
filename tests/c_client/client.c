/* A plain C program using the library through include/ht.h only: device
 * buffers from the HIP runtime API, tables created, filled, queried and
 * sized, many tables filled and queried at once (one-shot and through a
 * plan), and a small state space explored in split and fused levels;
 * results checked here.  Exit status 0 when every check passes. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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

/* Two tables of each kind: table j gets keys j*M .. j*M + M-1, each twice,
 * in one many-table call, then again through a plan (all present by then);
 * the many-table query finds every key of its own table and none of the next
 * table's. */
#define M 30000u
#define NT 4u

static int many(void) {
  uint64_t* h_keys = (uint64_t*)malloc(NT * 2 * M * sizeof(uint64_t));
  uint8_t* h_flags = (uint8_t*)malloc(NT * 2 * M);
  if (!h_keys || !h_flags) return 1;
  for (uint64_t j = 0; j < NT; ++j)
    for (uint64_t i = 0; i < M; ++i) {
      const uint64_t k = (j * M + i) * 0xD1B54A32D192ED03ull + 5;
      h_keys[j * 2 * M + i] = k;
      h_keys[j * 2 * M + M + i] = k;
    }
  uint64_t* d_keys = NULL;
  uint8_t* d_flags = NULL;
  if (hipMalloc((void**)&d_keys, NT * 2 * M * sizeof(uint64_t)) != hipSuccess) return 1;
  if (hipMalloc((void**)&d_flags, NT * 2 * M) != hipSuccess) return 1;
  if (hipMemcpy(d_keys, h_keys, NT * 2 * M * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) return 1;
  ht_table* t[NT];
  const uint64_t* keys[NT];
  const uint64_t* other[NT];
  uint64_t n[NT], half[NT];
  uint8_t* flags[NT];
  int bad = 0;
  for (uint32_t j = 0; j < NT; ++j) {
    bad |= check(ht_create_simple(j % 2 ? HT_CUCKOO : HT_BUCKETED, 4 * M, 3, &t[j]), "ht_create_simple");
    keys[j] = d_keys + (uint64_t)j * 2 * M;
    other[j] = d_keys + (uint64_t)((j + 1) % NT) * 2 * M;
    n[j] = 2 * M;
    half[j] = M;
    flags[j] = d_flags + (uint64_t)j * 2 * M;
  }
  if (bad) return 1;
  bad |= check(ht_find_or_put_multi(t, keys, n, flags, NT, NULL), "ht_find_or_put_multi");
  if (hipMemcpy(h_flags, d_flags, NT * 2 * M, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  for (uint64_t j = 0; j < NT; ++j)
    for (uint64_t i = 0; i < M; ++i)
      if (h_flags[j * 2 * M + i] + h_flags[j * 2 * M + M + i] != 1) bad = 1;
  ht_multi_plan* p = NULL;
  bad |= check(ht_multi_plan_create(t, keys, n, flags, NT, &p), "ht_multi_plan_create");
  if (!p) return 1;
  bad |= check(ht_multi_plan_launch(p, NULL), "ht_multi_plan_launch");
  bad |= check(ht_multi_plan_status(p, NULL), "ht_multi_plan_status");
  bad |= check(ht_multi_plan_destroy(p), "ht_multi_plan_destroy");
  if (hipMemcpy(h_flags, d_flags, NT * 2 * M, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  for (uint64_t i = 0; i < NT * 2 * M; ++i)
    if (h_flags[i] != 0) bad = 1;                /* every key already present */
  bad |= check(ht_query_multi(t, keys, half, flags, NT, NULL), "ht_query_multi (own keys)");
  if (hipMemcpy(h_flags, d_flags, NT * 2 * M, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  for (uint64_t j = 0; j < NT; ++j)
    for (uint64_t i = 0; i < M; ++i)
      if (h_flags[j * 2 * M + i] != 1) bad = 1;
  bad |= check(ht_query_multi(t, other, half, flags, NT, NULL), "ht_query_multi (other keys)");
  if (hipMemcpy(h_flags, d_flags, NT * 2 * M, hipMemcpyDeviceToHost) != hipSuccess) return 1;
  for (uint64_t j = 0; j < NT; ++j)
    for (uint64_t i = 0; i < M; ++i)
      if (h_flags[j * 2 * M + i] != 0) bad = 1;
  for (uint32_t j = 0; j < NT; ++j) {
    uint64_t size = 0;
    bad |= check(ht_size(t[j], &size, NULL), "ht_size");
    if (size != M) bad = 1;
    bad |= check(ht_destroy(t[j]), "ht_destroy");
  }
  printf("many tables: %s\n", bad ? "FAIL" : "ok");
  hipFree(d_keys);
  hipFree(d_flags);
  free(h_keys);
  free(h_flags);
  return bad;
}

/* Processes 0 and 1 each step around a cycle of 16 local states, the others
 * never move: the reachable states are the 16 x 16 torus, 256 of them, each
 * with two successors. */
static int explore(uint32_t kind, uint32_t mode) {
  ht_bfs_model m;
  memset(&m, 0, sizeof(m));
  for (int p = 0; p < 2; ++p)
    for (int s = 0; s < 16; ++s) {
      m.local_count[p][s] = 1;
      m.local_target[p][s][0] = (uint8_t)((s + 1) % 16);
    }
  for (int a = 0; a < 4; ++a) {
    m.sync_p[a] = 0;
    m.sync_q[a] = 1;
    for (int s = 0; s < 16; ++s) m.sync_p_edge[a][s] = m.sync_q_edge[a][s] = -1;
  }
  ht_table* t = NULL;
  int bad = check(ht_create_simple(kind, 1024, 3, &t), "ht_create_simple");
  if (bad) return 1;
  enum { L = 40 };
  uint64_t bs[L], nc[L];
  double fop[L], lv[L];
  memset(nc, 0, sizeof(nc));
  memset(bs, 0, sizeof(bs));
  bad |= check(ht_bfs_explore_ex(t, &m, 0, L, mode, bs, nc, fop, lv, NULL), "ht_bfs_explore_ex");
  uint64_t news = 0, succ = 0, size = 0;
  for (int i = 0; i < L; ++i) {
    news += nc[i];
    succ += bs[i];
  }
  bad |= check(ht_size(t, &size, NULL), "ht_size");
  if (news != 255 || size != 256 || succ != 2 * 256) bad = 1;
  printf("explore kind %u mode %u: states %llu %s\n", kind, mode, (unsigned long long)size, bad ? "FAIL" : "ok");
  bad |= check(ht_destroy(t), "ht_destroy");
  return bad;
}

int main(void) {
  int bad = run(HT_BUCKETED);
  bad |= run(HT_CUCKOO);
  bad |= many();
  bad |= explore(HT_BUCKETED, HT_BFS_SPLIT);
  bad |= explore(HT_BUCKETED, HT_BFS_FUSED);
  bad |= explore(HT_CUCKOO, HT_BFS_FUSED);
  return bad ? 1 : 0;
}
