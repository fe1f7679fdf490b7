// CPU oracle in C++: the plain set definition of find-or-put and query.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite and the CPU-baseline leg of
// the benchmark load this library; the hash-table library never does, and
// this file includes nothing from it.
//
// What the method computes (paper Sec. 5, the find-or-insert benchmark): each
// element of a sequence is looked up in a set S; when present nothing
// happens, otherwise it is inserted.  Applied in index order:
//
//     find_or_put(keys):  is_new[i] = keys[i] not in S;  S = S u {keys[i]}
//     query(keys):        found[i]  = keys[i] in S
//
// Every 64-bit value is a legal key.  S is a std::unordered_set<uint64_t>.
//
// The partitioned form runs the same definition on T threads: thread p owns
// the keys whose partition number part(k) is p, keeps its own set, and walks
// the whole batch in index order applying the definition to its own keys
// only.  Every occurrence of a key is handled by one thread, in index order,
// so the flags are those of the sequential loop.  part() is a multiplicative
// hash written for this file only.
#include <cstdint>
#include <cstring>
#include <thread>
#include <unordered_set>
#include <vector>

namespace {

struct OracleSet {
  std::vector<std::unordered_set<uint64_t>> parts;   // one set, or one per thread
};

inline uint32_t part_of(uint64_t k, uint32_t nparts) {
  const uint64_t h = (k ^ (k >> 31)) * 0xD6E8FEB86659FD93ull;
  return (uint32_t)(((h >> 32) * (uint64_t)nparts) >> 32);
}

void fop_one(std::unordered_set<uint64_t>& s, const uint64_t* keys, uint64_t n, uint8_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    const bool fresh = s.insert(keys[i]).second;   // inserted <=> was absent
    if (out) out[i] = fresh ? 1 : 0;
  }
}

void fop_part(std::unordered_set<uint64_t>& s, uint32_t p, uint32_t nparts, const uint64_t* keys, uint64_t n,
              uint8_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    if (part_of(keys[i], nparts) != p) continue;
    const bool fresh = s.insert(keys[i]).second;
    if (out) out[i] = fresh ? 1 : 0;
  }
}

}  // namespace

extern "C" {

// A new empty set split into `nparts` partitions (1 = the plain sequential
// set), each with room reserved for `reserve / nparts` keys.
void* oracle_new(uint32_t nparts, uint64_t reserve) {
  if (nparts == 0) nparts = 1;
  OracleSet* o = new OracleSet();
  o->parts.resize(nparts);
  if (reserve)
    for (auto& s : o->parts) s.reserve(reserve / nparts + 1);
  return o;
}

void oracle_free(void* h) { delete static_cast<OracleSet*>(h); }

// find_or_put of keys[0..n) in index order; out (may be NULL) receives the
// flags.  With several partitions each runs on a thread of its own.
void oracle_find_or_put(void* h, const uint64_t* keys, uint64_t n, uint8_t* out) {
  OracleSet* o = static_cast<OracleSet*>(h);
  const uint32_t np = (uint32_t)o->parts.size();
  if (np == 1) {
    fop_one(o->parts[0], keys, n, out);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(np);
  for (uint32_t p = 0; p < np; ++p)
    th.emplace_back([o, p, np, keys, n, out] { fop_part(o->parts[p], p, np, keys, n, out); });
  for (auto& t : th) t.join();
}

void oracle_query(void* h, const uint64_t* keys, uint64_t n, uint8_t* out) {
  OracleSet* o = static_cast<OracleSet*>(h);
  const uint32_t np = (uint32_t)o->parts.size();
  for (uint64_t i = 0; i < n; ++i) {
    const auto& s = o->parts[np == 1 ? 0 : part_of(keys[i], np)];
    out[i] = s.count(keys[i]) ? 1 : 0;
  }
}

uint64_t oracle_size(void* h) {
  uint64_t n = 0;
  for (const auto& s : static_cast<OracleSet*>(h)->parts) n += s.size();
  return n;
}

// Write the members (any order) to out, at most cap; returns the member count.
uint64_t oracle_dump(void* h, uint64_t* out, uint64_t cap) {
  uint64_t i = 0;
  for (const auto& s : static_cast<OracleSet*>(h)->parts)
    for (uint64_t k : s) {
      if (i < cap) out[i] = k;
      ++i;
    }
  return i;
}

}  // extern "C"
