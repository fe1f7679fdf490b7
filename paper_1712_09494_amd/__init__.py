"""MI355X (gfx950) GPU hash tables for state-space exploration.

Batched, lock-free find-or-put and query of 64-bit keys in a bucketed
(GPUexplore-style) table and a parallel Cuckoo table, as compared by Cassee &
Wijs, "Analysing the Performance of GPU Hash Tables for State Space
Exploration".  The kernels are hand-written HIP in libht.so behind the C ABI
of include/ht.h; ``binding`` is the thin Python layer over it.
"""
from .binding import (  # noqa: F401
    EMPTY, HT_BUCKETED, HT_CUCKOO, HT_EFULL, HT_EHIP, HT_EINVAL, HT_ENOMEM, HT_OK,
    HT_FLAG_BUCKETED_ATOMIC_LOADS, HT_FLAG_CUCKOO_PAPER_ORDER, HT_FLAG_SCRIPTED_HASH,
    HT_FLAG_BUCKETED_PAPER_FULL, HT_FLAG_BUCKETED_ONE_LANE, HT_FLAG_BUCKETED_GROUP_QUERY, HT_FLAG_CHAIN_STATS,
    HT_FLAG_CUCKOO_LOOKAHEAD, HT_FLAG_CUCKOO_SINGLE_PASS,
    HtError, HtLibraryMissing, MultiPlan, Server, Table, find_or_put_multi, load, u64,
)
