"""Comparators between the GPU tables and the CPU oracle (set semantics).

R1  query flags are bit-exact.
R2  find_or_put: within a call, for each distinct key, the number of
    occurrences reported new equals the oracle's (0 or 1); all flags are
    0 or 1.  Which duplicate reports new may differ.
R3  after the calls, the table's dump as a set equals the oracle's set, no key
    is stored twice and size equals the set size.
"""
import numpy as np


def as_u64(a):
    a = np.asarray(a)
    return a.view(np.uint64) if a.dtype == np.int64 else a.astype(np.uint64)


def check_flags_r2(keys, gpu, ora, what=""):
    keys = as_u64(keys)
    gpu = np.asarray(gpu, dtype=np.uint8)
    ora = np.asarray(ora, dtype=np.uint8)
    assert gpu.shape == keys.shape == ora.shape, what
    bad = np.flatnonzero(gpu > 1)
    assert bad.size == 0, f"{what}: flags outside {{0,1}} at {bad[:8]} (values {gpu[bad[:8]]})"
    g = np.sort(keys[gpu == 1])
    o = np.sort(keys[ora == 1])
    if g.size != o.size or not np.array_equal(g, o):
        gs, os_ = set(g.tolist()), set(o.tolist())
        dup = g.size - len(gs)
        raise AssertionError(
            f"{what}: new-key multisets differ: gpu {g.size} (dups {dup}) vs oracle {o.size}; "
            f"missing {list(os_ - gs)[:5]} extra {list(gs - os_)[:5]}")


def check_query_r1(gpu, ora, what=""):
    gpu = np.asarray(gpu, dtype=np.uint8)
    ora = np.asarray(ora, dtype=np.uint8)
    diff = np.flatnonzero(gpu != ora)
    assert diff.size == 0, f"{what}: {diff.size} query mismatches, first at {diff[:8]}"


def check_dump_r3(dump, oracle_keys, size, what=""):
    d = np.sort(as_u64(dump))
    o = np.sort(as_u64(oracle_keys))
    assert d.size == np.unique(d).size, f"{what}: a key is stored twice"
    assert d.size == o.size and np.array_equal(d, o), f"{what}: dump {d.size} vs oracle {o.size}"
    assert size == o.size, f"{what}: size {size} vs {o.size}"


def check_flags_r2_calls(keys, gpu, ora, bounds, what=""):
    """R2 for every call of a run of consecutive calls, exactly and in time
    linear in the keys.  ``ora`` are the oracle's flags for the same calls
    (the sequential set definition: for a run starting from an empty set,
    ``first_occurrence_flags`` of the whole sequence); ``bounds`` are the
    calls' start indices followed by the end.  Where the two flag arrays
    differ, the keys reported new only by the GPU and only by the oracle must
    be the same multiset within each call; where they agree there is nothing
    to compare.  So for every call and key the number of occurrences reported
    new is the oracle's (0 or 1)."""
    keys = as_u64(keys)
    gpu = np.asarray(gpu, dtype=np.uint8)
    ora = np.asarray(ora, dtype=np.uint8)
    assert gpu.shape == keys.shape == ora.shape, what
    bad = np.flatnonzero(gpu > 1)
    assert bad.size == 0, f"{what}: flags outside {{0,1}} at {bad[:8]} (values {gpu[bad[:8]]})"
    diff = np.flatnonzero(gpu != ora)
    g = diff[gpu[diff] == 1]
    o = diff[ora[diff] == 1]
    assert g.size == o.size, f"{what}: {g.size} keys new only on the GPU, {o.size} only in the oracle"
    if g.size == 0:
        return
    bounds = np.asarray(bounds, dtype=np.int64)
    call_g = np.searchsorted(bounds, g, side="right")
    call_o = np.searchsorted(bounds, o, side="right")
    gi = np.lexsort((call_g, keys[g]))
    oi = np.lexsort((call_o, keys[o]))
    assert np.array_equal(keys[g][gi], keys[o][oi]) and np.array_equal(call_g[gi], call_o[oi]), \
        f"{what}: keys reported new differ from the oracle's within a call"
