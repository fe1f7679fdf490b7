"""Autotuner for table parameters.

For a table kind, capacity and load factor it measures find-or-put
throughput over a grid of bucket widths B (bucketed: 8/16/32/64) and hash
counts c (2..4, both designs), on a seeded random workload of the table's
shape, and keeps the fastest configuration that stores every key without
overflow.  Candidates are timed in the launch the many-table fill uses (a
plan over the one table: the persistent kernel for bucketed tables, the
three phase kernels for Cuckoo tables), so the choice is made on the kernel
that runs it.  That launch probes with one lane per key and sizes its work
items for the whole grid, so it has no keys-per-wave parameter: the
keys-per-group axis (R = 1/2/4) applies only to the single-table calls and is
swept there with ``single_table=True``.  Results are cached in a JSON file
keyed by (kind, floor(log2 capacity), load factor rounded to 0.1), so tables
of similar shape reuse one measurement.

The paper suggests smaller buckets than a warp as the next step for the
bucketed table (Sec. 7); the B axis of the grid is that experiment.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Optional

import numpy as np

from . import binding as b
from . import inputs

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gpuhash_tune.json")

GRID = {
    "bucketed": [dict(bucket_slots=B, nhash=c) for B in (8, 16, 32, 64) for c in (2, 3, 4)],
    "cuckoo": [dict(nhash=c) for c in (2, 3, 4)],
}

# single-table calls: the lane-group width and keys per group matter there
GRID_SINGLE = {
    "bucketed": [dict(bucket_slots=B, nhash=c, keys_per_group=R)
                 for B in (8, 16, 32, 64) for c in (2, 3, 4) for R in (1, 2, 4)],
    "cuckoo": [dict(nhash=c, keys_per_group=R) for c in (2, 3, 4) for R in (1, 2, 4)],
}

# fallback when a shape has not been measured: one 128-byte line per bucket, c = 3
DEFAULT = {"bucketed": dict(bucket_slots=16, nhash=3),
           "cuckoo": dict(nhash=3)}


def cache_key(kind: str, capacity: int, lf: float) -> str:
    return f"{kind}:{int(math.floor(math.log2(max(capacity, 1))))}:{round(lf, 1):.1f}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure(kind: str, capacity: int, lf: float, params: dict, keys_dev, reps: int = 3,
            batch: Optional[int] = None, single_table: bool = False) -> Optional[float]:
    """Mops/s of find-or-put of keys_dev into a fresh table, or None when the
    configuration cannot hold the keys (overflow).  Timed through a
    many-table plan over this one table (the launch of the batched fill), or
    with ``single_table`` through ht_find_or_put in batches of ``batch``."""
    import torch
    n = keys_dev.numel()
    batch = batch or n
    t = b.Table(kind, capacity=capacity, max_batch=batch, **params)
    out = torch.empty(n, dtype=torch.uint8, device=keys_dev.device)
    stream = torch.cuda.current_stream()
    plan = None if single_table else b.MultiPlan([t], [keys_dev], [out])
    best = None
    try:
        for _ in range(reps):
            t.clear()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if plan is not None:
                plan.launch()
            else:
                for s0 in range(0, n, batch):
                    t.find_or_put(keys_dev[s0:s0 + batch], out[s0:s0 + batch])
            e1.record(stream)
            torch.cuda.synchronize()
            if t.sync_status() != b.HT_OK:
                return None
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
    finally:
        if plan is not None:
            plan.close()
        t.close()
    return n / best / 1e3


def tune(kind: str, capacity: int, lf: float, grid: Optional[list] = None, reps: int = 3,
         dup_frac: float = 0.1, batch: Optional[int] = None, cache_path: Optional[str] = DEFAULT_CACHE,
         device: str = "cuda", verbose: bool = False, single_table: bool = False) -> dict:
    """Measure the grid for (kind, capacity, lf); return {"best": params, "mops": x, "results": [...]}.
    The best entry is also stored in the cache file (if cache_path is given)."""
    import torch
    n = max(1, int(round(lf * capacity / (1.0 - dup_frac)))) if dup_frac < 1 else int(lf * capacity)
    distinct = max(1, int(round(lf * capacity)))
    n = max(n, distinct)
    seq = inputs.random_sequence(n, distinct, seed=inputs.SEED_BASE + 3 + capacity)
    keys = torch.from_numpy(seq.view(np.int64)).to(device)
    results = []
    for params in (grid or (GRID_SINGLE if single_table else GRID)[kind]):
        t0 = time.time()
        mops = measure(kind, capacity, lf, params, keys, reps=reps, batch=batch, single_table=single_table)
        results.append({"params": params, "mops": mops})
        if verbose:
            print(f"[tune] {kind} cap={capacity} lf={lf} {params} -> {mops} ({time.time() - t0:.1f}s)",
                  flush=True)
    ok = [r for r in results if r["mops"] is not None]
    best = max(ok, key=lambda r: r["mops"]) if ok else {"params": DEFAULT[kind], "mops": None}
    res = {"best": best["params"], "mops": best["mops"], "results": results}
    if cache_path:
        cache = load_cache(cache_path)
        cache[cache_key(kind, capacity, lf)] = {"params": best["params"], "mops": best["mops"]}
        save_cache(cache, cache_path)
    return res


def pick(kind: str, capacity: int, lf: float, cache_path: Optional[str] = DEFAULT_CACHE) -> dict:
    """Cached best parameters for a table shape, else the defaults."""
    if cache_path:
        e = load_cache(cache_path).get(cache_key(kind, capacity, lf))
        if e:
            return dict(e["params"])
    return dict(DEFAULT[kind])
