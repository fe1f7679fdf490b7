/*
 * ht.h -- C ABI of the MI355X (gfx950) GPU hash tables for state-space
 * exploration: batched, lock-free find-or-put and query of 64-bit keys.
 *
 * Two table designs (Cassee & Wijs, "Analysing the Performance of GPU Hash
 * Tables for State Space Exploration"):
 *
 *   HT_BUCKETED  the bucketed GPUexplore table (Sec. 4.2, Fig. 4): a key is
 *                hashed with h_1..h_c to buckets of B slots; a group of lanes
 *                reads a whole bucket in one coalesced access, votes whether
 *                the key is present or which slots are free, and writes the
 *                key into a free slot atomically, retrying the next free slot
 *                on a lost race and the next hash function when the bucket is
 *                full.
 *   HT_CUCKOO    the parallel Cuckoo table (Sec. 4.1, Fig. 2): one lane per
 *                key, c hash functions into a slot array, insertion by atomic
 *                exchange with an eviction chain, and a stash for keys whose
 *                chain exceeds the bound.
 *
 * Semantics (Sec. 5): find_or_put applies "if present do nothing, otherwise
 * insert" to every key of a batch; the result is that of a set S applied in
 * index order, except that when one batch holds several copies of a key that
 * was absent, which copy reports "new" is unspecified (exactly one does).
 * Every 64-bit value is a legal key, including 0xFFFFFFFFFFFFFFFF.
 *
 * Conventions for every call taking a stream:
 *   - key, flag and output pointers are DEVICE pointers owned by the caller
 *     and must stay valid until the work queued on `stream` completes;
 *   - calls are asynchronous on `stream`; calls on one table must be ordered
 *     on one stream (or synchronised by the caller); different tables are
 *     independent;
 *   - the table owns only its own device storage (slots, stash, overflow list,
 *     counters and scratch);
 *   - n == 0 is a no-op returning HT_OK; a NULL pointer with n > 0 returns
 *     HT_EINVAL; nothing is launched when an argument is rejected;
 *   - a call never waits for the device unless it says "synchronises".
 *
 * Per-key output of find_or_put: 1 = the key was absent and is now stored,
 * 0 = the key was already present (or another copy in the batch reported 1),
 * 2 = the key was absent and could not be placed in its buckets nor the stash;
 * it is kept on the table's overflow list (still a member, found by query)
 * until ht_rebuild.  An overflowed key may report 2 more than once.  Only when
 * the overflow list is full as well is such a key not kept: it still reports
 * 2, is counted in ht_stats_t.lost, and is not a member; ht_sync_status
 * reports HT_EFULL in both cases (Sec. 4.1 and 4.2: the table is full and is
 * to be rebuilt with new hash constants).
 *
 * Entry points without a defining passage in the paper (memory management,
 * introspection, test and measurement aids) say "Infrastructure".
 */
#ifndef HT_H
#define HT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same declaration as the HIP runtime's stream handle. */
typedef struct ihipStream_t* hipStream_t;

typedef struct ht_table ht_table;

enum {
  HT_BUCKETED = 1,
  HT_CUCKOO = 2
};

enum {
  HT_OK = 0,
  HT_EINVAL = -1,   /* bad argument */
  HT_ENOMEM = -2,   /* device allocation failed */
  HT_EFULL = -3,    /* keys went to the overflow list, or were lost */
  HT_EHIP = -4      /* a HIP runtime call failed */
};

/* Configuration flags. */
enum {
  /* Cuckoo: place a new key by exchanging it into h_1 first, as the
   * Pagh-Rodler insertion of Sec. 4.1 describes.  Without the flag a new key
   * is first written (compare-and-swap) into a candidate slot that the probe
   * saw empty, and the eviction chain starts only when none is left. */
  HT_FLAG_CUCKOO_PAPER_ORDER = 1u << 0,
  /* Bucketed, lane groups: read each lane's four slots with four 8-byte
   * agent-scope atomic loads instead of two 16-byte loads.  Results are
   * identical (a stale empty slot is corrected by the compare-and-swap
   * result); the 16-byte loads touch a bucket with half the cache requests,
   * and are the default. */
  HT_FLAG_BUCKETED_ATOMIC_LOADS = 1u << 1,
  /* Test mode: h_j(key) is taken from a table installed with
   * ht_set_scripted_hash instead of the hash family. */
  HT_FLAG_SCRIPTED_HASH = 1u << 2,
  /* Bucketed: after the c buckets of h_1..h_c are full, go straight to the
   * stash, as the table of Sec. 4.2 declares itself full at that point.
   * Without the flag the probe first walks up to bucket_walk consecutive
   * buckets after h_c's bucket (same sequence for every inserter of a key). */
  HT_FLAG_BUCKETED_PAPER_FULL = 1u << 3,
  /* Cuckoo, ablation only: one kernel per find-or-put doing the lookup and
   * the eviction chain of Sec. 4.1 in the same pass, with the check of
   * Sec. 5.1.1 (a thread that evicts its own key stops).  Keys repeated in a
   * batch can then be stored twice and reported new more than once (a lookup
   * misses a copy that another thread holds in flight); exact only for
   * batches without repeated keys.  Not combinable with key_words > 1.  The
   * many-table call and the serving engine always use the exact three-phase
   * insertion. */
  HT_FLAG_CUCKOO_SINGLE_PASS = 1u << 4,
  /* Bucketed, single-word keys: probe with one lane per key (each lane reads
   * its buckets eight slots at a time and compare-and-swaps the first empty
   * slot) instead of a group of B/4 lanes sharing each bucket (Sec. 4.2).
   * Same table, probe sequence and results; a wave serves 64 keys per turn
   * instead of 256/B.  Faster where hits dominate (BFS keys, heavy
   * duplication).  The many-table launch always probes this way. */
  HT_FLAG_BUCKETED_ONE_LANE = 1u << 5,
  /* Measurement: record each Cuckoo eviction chain's number of exchanges in
   * a histogram read by ht_chain_histogram (one extra atomic per chain). */
  HT_FLAG_CHAIN_STATS = 1u << 6,
  /* Cuckoo: before each exchange of the eviction chain (Sec. 4.1), a key
   * evicted from h_a reads its candidates h_{a+1}..h_c and compare-and-swaps
   * itself into the lowest-numbered empty one; the chain goes on by exchange
   * only when none is empty.  Fewer exchanges, one more read per step.  Not
   * combinable with HT_FLAG_CUCKOO_PAPER_ORDER (which keeps the insertion of
   * Sec. 4.1 as written). */
  HT_FLAG_CUCKOO_LOOKAHEAD = 1u << 7,
  /* Bucketed: answer queries (single- and many-table) with groups of B/2
   * lanes sharing each bucket, the cooperative read of Sec. 4.2.  Without
   * the flag a query runs one lane per key, reading its buckets eight slots
   * at a time and stopping at the first empty slot: the same answers, since
   * a bucket's keys fill it as a prefix; on MI355X 7-27% faster at B = 8 and
   * about twice as fast at B = 32 and 64. */
  HT_FLAG_BUCKETED_GROUP_QUERY = 1u << 8
};

typedef struct {
  uint32_t kind;           /* HT_BUCKETED or HT_CUCKOO */
  uint32_t nhash;          /* c, number of hash functions, 1..8 */
  uint64_t capacity;       /* requested slots (> 0); bucketed rounds up to a
                              multiple of bucket_slots, cuckoo to a multiple of 16 */
  uint32_t bucket_slots;   /* bucketed: B in {8, 16, 32, 64}; 0 = 16 (one 128-byte
                              line of 64-bit keys).  Ignored by cuckoo */
  uint32_t keys_per_group; /* keys each lane group (bucketed) or lane (cuckoo)
                              keeps in flight: 1, 2 or 4; 0 = 1.  Bucketed
                              lane-group queries use at least 2 */
  uint32_t stash_slots;    /* stash size (power of two, <= 65536); 0 = 1024 */
  uint32_t max_chain;      /* cuckoo eviction bound; 0 = 8 * ceil(log2 capacity) */
  uint64_t seed;           /* seed of the hash constants */
  uint32_t flags;          /* HT_FLAG_* */
  uint32_t overflow_slots; /* overflow list length; 0 = 65536 */
  uint64_t max_batch;      /* scratch reserved for batches up to this size;
                              0 = grow on demand (the call then allocates) */
  uint32_t bucket_walk;    /* bucketed: consecutive buckets probed after h_c's
                              bucket before the stash; 0 = 64 */
  uint32_t lds_bytes;      /* ablation of the shared-memory setting of Sec. 6:
                              bytes of LDS allocated (and left unused) per
                              256-thread block of the single-table find-or-put
                              and query kernels, which lowers how many waves a
                              compute unit holds; 0 = none.  At most the
                              device's LDS per block (HT_EINVAL otherwise) */
  uint32_t key_words;      /* words per key: 1 (64-bit keys), 2 or 4 (state
                              vectors of 128 or 256 bits, the multi-word state
                              vectors of GPUexplore, Sec. 3.2 and 4.2); 0 = 1.
                              A vector table stores each member once in an
                              arena of (capacity + stash_slots + overflow_slots)
                              entries and keeps 64-bit handles in its slots;
                              capacity + stash + overflow below 2^33; batches
                              below 2^33 vectors; see ht_find_or_put for the
                              key layout */
  uint32_t reserved;       /* must be 0 */
} ht_config;

typedef struct {
  uint64_t size;           /* distinct keys stored (including stash, overflow) */
  uint64_t capacity;       /* actual slot count */
  uint64_t stash_count;    /* keys in the stash */
  uint64_t overflow_count; /* keys on the overflow list */
  uint64_t lost;           /* keys dropped because the overflow list was full */
  uint64_t evictions;      /* cuckoo: total evictions so far */
  uint64_t nbuckets;       /* bucketed: bucket count; cuckoo: slot count */
  uint32_t kind, nhash, bucket_slots, stash_slots;
  uint64_t seed;           /* current hash seed (changes on rebuild) */
} ht_stats_t;

/* Infrastructure.  Fills *cfg with the defaults for `kind` (capacity and
 * seed left 0). */
void ht_config_default(ht_config* cfg, uint32_t kind);

/* Create a table (Sec. 5: the table is allocated on the device and its hash
 * constants installed before the batch is processed).  Allocates device
 * memory on the current device, clears every slot to empty and synchronises.
 * *out receives the table; HT_EINVAL for a bad config, HT_ENOMEM when the
 * allocation fails. */
int ht_create(const ht_config* cfg, ht_table** out);

/* Infrastructure.  ht_create with defaults for everything but kind,
 * capacity and nhash. */
int ht_create_simple(uint32_t kind, uint64_t capacity, uint32_t nhash, ht_table** out);

/* Infrastructure.  Free the table's device memory (synchronises the device
 * first); HT_EINVAL for a NULL table. */
int ht_destroy(ht_table* t);

/* Find-or-put (Sec. 5; Sec. 4.1 insertion for cuckoo, Sec. 4.2 for bucketed).
 * d_keys: n keys (uint64, device); for a table with key_words W > 1, n
 * vectors of W words each, row-major (n * W words, 16-byte aligned; HT_EINVAL
 * otherwise).  d_out_is_new: n bytes (device), may be NULL when the flags are
 * not wanted.  Grows the table's scratch (allocating, synchronising) when n
 * exceeds what was reserved.  Cuckoo and state-vector calls on one table
 * must be ordered by the caller (one stream, or events between streams):
 * they share the table's scratch, and a Cuckoo call of single-word keys
 * leaves the deduplication slots its winners took for the next such call's
 * first kernel to empty (state kept on the device, so captured and replayed
 * calls stay exact). */
int ht_find_or_put(ht_table* t, const uint64_t* d_keys, uint64_t n,
                   uint8_t* d_out_is_new, hipStream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): ht_find_or_put that
 * allocates nothing.  Same results (Sec. 5 find-or-put) and the same probe
 * and evict kernels, followed by the scrub kernel that empties the
 * deduplication set before the call returns; the scratch of the Cuckoo
 * insertion (deduplication set, listed keys, per-wave
 * counts) is a static device array of 8.06 MiB held by each device the
 * library runs on until the process ends, instead of the table's own
 * scratch.  Limits: n <= 262144 keys (HT_EINVAL above), tables of
 * single-word keys only (HT_EINVAL for key_words > 1), and the table's device
 * must be the current device (HT_EINVAL otherwise).  Bucketed tables and
 * HT_FLAG_CUCKOO_SINGLE_PASS use no scratch.  Every call on one device shares
 * that device's array: calls that may overlap on one device (different
 * streams, different host threads, different tables) race and must be
 * ordered by the caller.  Creates no HIP events and calls no memset. */
int ht_find_or_put_noalloc(ht_table* t, const uint64_t* d_keys, uint64_t n,
                           uint8_t* d_out_is_new, hipStream_t stream);

/* Same as ht_find_or_put. */
int ht_insert(ht_table* t, const uint64_t* d_keys, uint64_t n,
              uint8_t* d_out_is_new, hipStream_t stream);

/* Query (Sec. 4.1: at most c slots; Sec. 4.2: at most c buckets).  Writes
 * d_out_found[i] = 1 if d_keys[i] is a member, else 0. */
int ht_query(ht_table* t, const uint64_t* d_keys, uint64_t n,
             uint8_t* d_out_found, hipStream_t stream);

/* Find-or-put into `ntables` tables at once (the find-or-insert benchmark
 * kernel of Sec. 5, applied to many tables).  t[i], d_keys[i], n[i],
 * d_out_is_new[i] are host arrays of per-table arguments (the key and flag
 * pointers themselves are device pointers; a flag pointer may be NULL).
 * Tables may mix kinds, bucket sizes, hash counts and key widths; each table
 * may appear at most once; scripted-hash tables are rejected.  All bucketed
 * tables of single-word keys are served by one persistent kernel; all Cuckoo
 * tables of single-word keys then run their three phases (probe and place,
 * evict, scrub) as three launches over all of them; state-vector tables
 * (key_words > 1: n[i] rows, 16-byte aligned) then run their own kernels,
 * all on the same stream.  Results equal one ht_find_or_put per table.
 * Builds a plan (allocating), launches it and synchronises `stream`. */
int ht_find_or_put_multi(ht_table* const* t, const uint64_t* const* d_keys,
                         const uint64_t* n, uint8_t* const* d_out_is_new,
                         uint32_t ntables, hipStream_t stream);

/* Query `ntables` tables at once (the lookups of Sec. 4.1 and 4.2, applied
 * to many tables): d_out_found[i][j] = 1 if d_keys[i][j] is a member of
 * t[i], else 0.  Arguments as for ht_find_or_put_multi (host arrays of
 * device pointers); flag pointers must not be NULL where n[i] > 0.  Tables
 * may mix kinds and repeat; scripted-hash tables are rejected.  Batches of
 * single-word keys too small to fill the device alone share one kernel
 * (bucketed tables read by lane groups, Cuckoo tables by one lane per key);
 * a batch that fills it alone, and every state-vector table (n[i] rows,
 * 16-byte aligned), runs the single-table query.  Results equal one
 * ht_query per table.  Allocates the descriptors and synchronises `stream`. */
int ht_query_multi(ht_table* const* t, const uint64_t* const* d_keys,
                   const uint64_t* n, uint8_t* const* d_out_found,
                   uint32_t ntables, hipStream_t stream);

typedef struct ht_multi_plan ht_multi_plan;

/* The find-or-insert of Sec. 5 for many tables, prepared once and launched
 * many times.  Prepare a many-table find-or-put: validates the arguments (as
 * ht_find_or_put_multi), reserves each Cuckoo and state-vector table's
 * scratch for its batch, and copies the tables' descriptors and work-item
 * lists to the device (allocates, synchronises).  The key and flag buffers
 * must stay valid for every launch of the plan. */
int ht_multi_plan_create(ht_table* const* t, const uint64_t* const* d_keys,
                         const uint64_t* n, uint8_t* const* d_out_is_new,
                         uint32_t ntables, ht_multi_plan** out);

/* The find-or-put of Sec. 5 (Sec. 4.1 and 4.2 insertion) of every table of
 * the plan.  Run the plan on `stream`: one persistent kernel for the bucketed tables,
 * then three phase kernels covering every Cuckoo table, then each
 * state-vector table's own kernels.
 * Allocates nothing, uses no memset and does not synchronise, so it may be
 * captured in a HIP graph and replayed.  Launches of one plan, and calls on
 * its tables, must be ordered on one stream. */
int ht_multi_plan_launch(ht_multi_plan* p, hipStream_t stream);

/* Infrastructure.  Synchronises `stream`; HT_EHIP if it reports an error,
 * else HT_OK; HT_EINVAL for a NULL plan. */
int ht_multi_plan_status(ht_multi_plan* p, hipStream_t stream);

/* Infrastructure.  Free the plan's device memory (synchronises the device);
 * HT_EINVAL for a NULL plan. */
int ht_multi_plan_destroy(ht_multi_plan* p);

/* The "table full" report (Sec. 4.1: a key left over after the eviction
 * chain and the stash means the table must be rebuilt with new hash
 * constants; Sec. 4.2: the bucketed table is considered full when all c
 * buckets of a key are full).  Synchronises `stream`; HT_EFULL if keys went
 * to the overflow list (or were lost, see above) since the table was created,
 * cleared or last rebuilt, else HT_OK. */
int ht_sync_status(ht_table* t, hipStream_t stream);

/* Rebuild (Sec. 4.1: when the stash overflows the table is rebuilt with new
 * hash constants): draws new constants, optionally grows to new_capacity
 * slots (0 = keep), and re-inserts every member (slots, stash, overflow list,
 * the all-ones key) into new storage.  The new storage is allocated before
 * the old is released, and the old table is kept until every member is
 * placed in slots or stash: up to 8 sets of constants are tried, and when
 * none places them all (HT_EFULL) or an allocation fails (HT_ENOMEM) the
 * table is left exactly as it was, every member kept.  Needs device memory
 * for the old and new storage at once.  HT_EINVAL for new_capacity above
 * 2^40 slots (2^33 entries for state-vector tables).  Synchronises. */
int ht_rebuild(ht_table* t, uint64_t new_capacity, hipStream_t stream);

/* The size of the set of inserted elements (Sec. 5: find-or-put stores each
 * distinct element once): *out_n = number of distinct keys stored (slots,
 * stash, overflow list).  HT_EINVAL for a NULL out_n.  Synchronises. */
int ht_size(ht_table* t, uint64_t* out_n, hipStream_t stream);

/* The set of inserted elements (Sec. 5): write every member once (any
 * order) to d_out (device, room for `cap` keys; a vector table writes rows of
 * key_words words); *out_n = member count (even when it exceeds cap, in which
 * case only cap keys are written).  HT_EINVAL for a NULL out_n, or a NULL
 * d_out with cap > 0.  Synchronises. */
int ht_dump(ht_table* t, uint64_t* d_out, uint64_t cap, uint64_t* out_n,
            hipStream_t stream);

/* Infrastructure (structural tests).  Copy the raw storage to d_slots
 * (device): the slot array (ht_stats_t capacity words) followed by the stash
 * (stash_slots words); empty slots hold 0xFFFFFFFFFFFFFFFF.  `cap` is the
 * room in words; HT_EINVAL when it is smaller than slots + stash.
 * Asynchronous on `stream`. */
int ht_dump_raw(ht_table* t, uint64_t* d_slots, uint64_t cap, hipStream_t stream);

/* Empty the table (Sec. 5: the table is initialised before each run of the
 * find-or-insert benchmark): every slot, the stash, the overflow list and the
 * counters are cleared; the hash constants are kept.  Asynchronous on
 * `stream`; HT_EINVAL for a NULL table. */
int ht_clear(ht_table* t, hipStream_t stream);

/* Infrastructure.  Counters and geometry.  HT_EINVAL for a NULL out.
 * Synchronises. */
int ht_stats(ht_table* t, ht_stats_t* out, hipStream_t stream);

/* Infrastructure (structural tests).  Host-side hash of the table: the
 * bucket index (bucketed) or slot index
 * (cuckoo) that h_j (0-based j < nhash) assigns to `key`.  For a vector table
 * `key` is a handle's hash bits (the handle shifted right by 34). */
int ht_hash_index(const ht_table* t, uint64_t key, uint32_t j, uint64_t* out_index);

/* Infrastructure.  Test mode (HT_FLAG_SCRIPTED_HASH), used to replay the
 * exchange sequence of Fig. 2: install `nkeys` scripted keys with
 * their hash values; h_index is nkeys*nhash host words (row per key, each
 * < bucket count or slot count).  Keys not in the script hash to index 0. */
int ht_set_scripted_hash(ht_table* t, const uint64_t* keys,
                         const uint64_t* h_index, uint32_t nkeys);

/* Infrastructure (measurement).  Eviction chains of the table's Cuckoo
 * find-or-puts since it was created or cleared, when it was created with
 * HT_FLAG_CHAIN_STATS (else all zeros): out[0] = chains that ended in the
 * stash (Sec. 4.1: after max_chain evictions), out[i] for 1 <= i < 63 =
 * chains of exactly i exchanges, out[63] = chains of 63 or more.  `out` is a
 * host array of 64 entries.  HT_EINVAL for a NULL table or out.
 * Synchronises `stream`. */
int ht_chain_histogram(ht_table* t, uint64_t* out, hipStream_t stream);

/* Infrastructure.  Reserve scratch for batches up to max_batch keys
 * (allocates, synchronises the device). */
int ht_reserve(ht_table* t, uint64_t max_batch);

/* Infrastructure.  Human-readable text of a status code (a static string;
 * "unknown status" for codes not listed above). */
const char* ht_strerror(int code);

/* Infrastructure.  Text of the last error raised on this thread (HIP error
 * string or argument check), "" if none. */
const char* ht_last_error(void);

/* ---- breadth-first exploration with a table as the visited set ---------- */

/* A synthetic concurrent model: 16 processes with 16 local states each, the
 * state vector packed 4 bits per process (process p in bits 4p..4p+3).
 * local_target[p][s][0 .. local_count[p][s]-1] are the local transitions of
 * process p in local state s (count <= 4); synchronising action a moves
 * processes sync_p[a] and sync_q[a] together, along their edges
 * sync_p_edge[a][s] / sync_q_edge[a][s] (-1: no edge from s). */
typedef struct {
  uint8_t local_count[16][16];
  uint8_t local_target[16][16][4];
  uint8_t sync_p[4], sync_q[4];
  int8_t sync_p_edge[4][16], sync_q_edge[4][16];
} ht_bfs_model;

/* Breadth-first exploration from `initial` for up to `levels` levels with
 * table `t` as the visited set (GPUexplore's use of the table, Sec. 3.2):
 * the initial state is find-or-put first; at each level the successors of
 * the frontier are generated on the device (per state: each process's local
 * transitions in order, then the synchronising actions), find-or-put as one
 * batch, and the states reported new become the next frontier, in batch
 * order.  Host arrays (may be NULL, else `levels` entries): batch_sizes[L]
 * successors generated, new_counts[L] states new at level L, fop_ms[L] the
 * find-or-put time (HIP events).  Allocates its buffers; synchronises. */
int ht_bfs_explore(ht_table* t, const ht_bfs_model* model, uint64_t initial, uint32_t levels,
                   uint64_t* batch_sizes, uint64_t* new_counts, double* fop_ms, hipStream_t stream);

enum {
  HT_BFS_SPLIT = 0,   /* generate the batch, find-or-put it, select the new keys */
  HT_BFS_FUSED = 1    /* generate and find-or-put without storing the batch */
};

/* ht_bfs_explore with the level's kernels chosen by `mode`.  HT_BFS_SPLIT is
 * ht_bfs_explore.  HT_BFS_FUSED joins successor generation and hash table
 * access, as GPUexplore does (Sec. 3.2 and 7): a lane takes a frontier state,
 * generates its successors in registers in the same order and find-or-puts
 * each, recording which were new; a last kernel writes the new ones, so the
 * successor batch is never stored.  Bucketed tables: one kernel, one lane per
 * key (the probe of HT_FLAG_BUCKETED_ONE_LANE).  Cuckoo tables: the exact
 * insertion's phases stay separate kernels (Sec. 4.1 with the deduplication
 * of the three-kernel insertion): successor counts and a scan place each
 * group of 64 states' list region, the fused pass probes and places every
 * successor and lists the ones whose candidates are all taken, then the
 * evict and scrub kernels run on those lists.  Not for tables with
 * HT_FLAG_SCRIPTED_HASH (HT_EINVAL).  Both modes give the same batch sizes,
 * new counts and visited set; within a level the next frontier holds the same
 * states (which copy of a repeated successor counts as new, and so its place,
 * may differ).  Extra host array (may be NULL): level_ms[L] the device time of
 * all of level L's kernels (split: count, scan, write, find-or-put, select;
 * fused: the passes above, scans and the write), without the host round trips
 * that read the level's sizes.  In fused mode fop_ms[L] is the time of the
 * fused find-or-put passes.  Allocates its buffers; synchronises. */
int ht_bfs_explore_ex(ht_table* t, const ht_bfs_model* model, uint64_t initial, uint32_t levels,
                      uint32_t mode, uint64_t* batch_sizes, uint64_t* new_counts, double* fop_ms,
                      double* level_ms, hipStream_t stream);

/* ---- serving: a request loop over resident tables ----------------------- */

enum {
  HT_OP_FIND_OR_PUT = 1,
  HT_OP_QUERY = 2
};

/* One request of a served trace.  Keys and flags are HOST buffers that must
 * be pinned (hipHostMalloc, or torch's pin_memory); the engine copies keys
 * in and flags out on its own streams.  arrival_s is the release time in
 * seconds after ht_server_run starts; the engine fills admit_s, done_s
 * (completion seen by the host, same clock), slot and group. */
typedef struct {
  uint32_t op;              /* HT_OP_FIND_OR_PUT or HT_OP_QUERY */
  uint32_t table;           /* index into the server's tables */
  const uint64_t* h_keys;   /* n keys; on a table with key_words > 1, n rows of key_words words */
  uint64_t n;
  uint8_t* h_out;           /* n flags: as ht_find_or_put / ht_query */
  double arrival_s;
  double admit_s;
  double done_s;
  uint32_t slot;
  uint32_t group;
} ht_request;

typedef struct {
  uint32_t slots;           /* launch groups in flight at once (streams), 1..16; 0 = 16 */
  uint32_t merge;           /* requests of distinct tables per launch group; 0 = 16 */
  uint64_t staging_bytes;   /* device staging budget for admission (9 bytes per key,
                               256-byte pieces); 0 = min(free device memory / 4, 4 GiB).
                               Requests of at most 64 KiB of keys do not use it: each
                               stream slot packs them into an area of its own (1 MiB of
                               keys and 128 KiB of flags, device and pinned host) */
  uint32_t sequential;      /* 1 = baseline: one request at a time, waiting for each */
  uint32_t reserved;
  uint64_t group_keys;      /* a group stops taking requests at this many keys
                               (its first request is always taken); 0 = 2^19 */
} ht_server_config;

typedef struct {
  double wall_s;            /* run start to the last completion */
  uint64_t keys;            /* keys in the trace */
  uint64_t peak_staging;    /* largest staging in use at once, bytes */
  uint64_t staging_bytes;   /* the budget */
  uint32_t groups;          /* launch groups issued */
  uint32_t merged_launches; /* groups that used many-table launches */
  uint32_t max_inflight_groups;
  uint32_t throttled;       /* admissions deferred for lack of staging */
} ht_server_stats;

typedef struct ht_server ht_server;

/* Infrastructure.  Fills *cfg with the defaults listed above (no-op for a
 * NULL cfg). */
void ht_server_config_default(ht_server_config* cfg);

/* Infrastructure (the serving engine has no counterpart in the paper; each
 * request it runs is the find-or-put of Sec. 5 or the query of Sec. 4.1 and
 * 4.2).  Serve `ntables` resident tables (the tables stay owned by the caller and
 * must outlive the server).  Allocates the staging budget, stream slots and
 * their events.  HT_EINVAL for scripted-hash tables or bad configs. */
int ht_server_create(ht_table* const* tables, uint32_t ntables, const ht_server_config* cfg,
                     ht_server** out);

/* Serve a trace of find-or-put (Sec. 5) and query (Sec. 4.1, 4.2) requests.
 * Replay `nreq` requests: each is released at its arrival time, admitted in
 * arrival order per table (FIFO) when its table is idle, a stream slot is
 * free and its staging fits, merged with admissible requests of other
 * tables into one launch group, and retired when the group's event
 * completes.  Each result equals the one the request gets when its table's
 * requests run one by one in arrival order.  Blocks until every request is
 * done; fills the per-request times and *stats (may be NULL).  Reserves
 * Cuckoo scratch for the largest request before starting the clock. */
int ht_server_run(ht_server* s, ht_request* reqs, uint32_t nreq, ht_server_stats* stats);

/* Infrastructure.  Free the server (synchronises the device); the tables are
 * untouched. */
int ht_server_destroy(ht_server* s);

/* ---- kernel timing (measurement aid) ------------------------------------ */

/* Infrastructure (measurement).  Enable (on != 0) or disable per-kernel
 * timing and reset the figures.  When
 * enabled, every kernel the library launches is bracketed by two HIP events
 * recorded on the stream it is launched on. */
int ht_timing_enable(int on);

/* Infrastructure (measurement).  JSON object {"kernel name": [launches,
 * total milliseconds], ...} of the
 * launches timed since ht_timing_enable; waits for their events.  HT_EINVAL
 * when buf is NULL or too small. */
int ht_timing_report(char* buf, uint64_t len);

/* ---- roofline probes: memory-system reference kernels ------------------- */

/* Infrastructure (measurement).  Streaming copy of n 64-bit words d_src ->
 * d_dst. */
int ht_probe_copy(const uint64_t* d_src, uint64_t* d_dst, uint64_t n, hipStream_t stream);

/* Infrastructure (measurement).  n_access random reads of `line_bytes`
 * (8, 64 or 128) from an array of
 * n_words 64-bit words; addresses come from a counter-based mixer seeded by
 * `seed`; the xor of the words read is stored to *d_sink. */
int ht_probe_gather(const uint64_t* d_array, uint64_t n_words, uint64_t n_access,
                    uint32_t line_bytes, uint64_t seed, uint64_t* d_sink,
                    hipStream_t stream);

/* Infrastructure (measurement).  n_access random 64-bit compare-and-swap
 * operations on d_array. */
int ht_probe_cas(uint64_t* d_array, uint64_t n_words, uint64_t n_access,
                 uint64_t seed, hipStream_t stream);

/* Infrastructure (measurement).  The memory pattern of a find-or-put
 * kernel, without the table logic: for each of n_items keys (device), read
 * the key, make `lines_per_item` random 8-byte reads (on average; each costs
 * a whole line at the memory) in d_array (n_words 64-bit words, device), then
 * with probability `cas_per_item` one 64-bit compare-and-swap (empty -> key)
 * there -- at a random word of its own line, or with same_line != 0 at a word
 * of the line the first read touched, as a table kernel compare-and-swaps
 * into the bucket or slot it has just read -- and write a 1-byte flag to
 * d_out.  Fractions are met per item by a keyed draw, in steps of 1/256.  Its
 * time against a table kernel's on the same keys, with the kernel's own read
 * and compare-and-swap counts, tells how close the kernel is to what the
 * memory system allows for that mix.  HT_EINVAL for NULL pointers, an empty
 * array, lines outside 0..64 or a probability outside 0..1. */
int ht_probe_mix(const uint64_t* d_keys, uint8_t* d_out, uint64_t n_items, uint64_t* d_array, uint64_t n_words,
                 double lines_per_item, double cas_per_item, uint32_t same_line, uint64_t seed,
                 hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HT_H */
