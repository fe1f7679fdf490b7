"""Host-side logic without a GPU: the autotuner's grid, cache keys, cache file
round trip and pick; the bench's byte model and source hash."""
import json
import os
import sys

import pytest

from paper_1712_09494_amd import tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_grid_is_the_documented_sweep():
    bk = tune.GRID["bucketed"]
    assert len(bk) == 4 * 3 * 3
    assert {p["bucket_slots"] for p in bk} == {8, 16, 32, 64}
    assert {p["nhash"] for p in bk} == {2, 3, 4}
    assert {p["keys_per_group"] for p in bk} == {1, 2, 4}
    ck = tune.GRID["cuckoo"]
    assert len(ck) == 3 * 3 and all("bucket_slots" not in p for p in ck)


def test_cache_key_groups_similar_shapes():
    assert tune.cache_key("bucketed", 1 << 20, 0.6) == tune.cache_key("bucketed", (1 << 21) - 1, 0.61)
    assert tune.cache_key("bucketed", 1 << 20, 0.6) != tune.cache_key("bucketed", 1 << 21, 0.6)
    assert tune.cache_key("bucketed", 1 << 20, 0.6) != tune.cache_key("cuckoo", 1 << 20, 0.6)
    assert tune.cache_key("cuckoo", 1000, 0.74) != tune.cache_key("cuckoo", 1000, 0.76)
    assert tune.cache_key("cuckoo", 0, 0.5) == "cuckoo:0:0.5"


def test_cache_round_trip_and_pick(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    assert tune.pick("bucketed", 1 << 16, 0.6, cache_path=path) == tune.DEFAULT["bucketed"]
    entry = {"params": {"bucket_slots": 8, "nhash": 2, "keys_per_group": 1}, "mops": 123.0}
    tune.save_cache({tune.cache_key("bucketed", 1 << 16, 0.6): entry}, path)
    assert json.load(open(path))[tune.cache_key("bucketed", 1 << 16, 0.6)] == entry
    assert tune.pick("bucketed", (1 << 16) + 5, 0.6, cache_path=path) == entry["params"]
    assert tune.pick("bucketed", 1 << 18, 0.6, cache_path=path) == tune.DEFAULT["bucketed"]
    p = tune.pick("bucketed", 1 << 16, 0.6, cache_path=path)
    p["nhash"] = 9                                   # the caller's copy, not the cache
    assert tune.pick("bucketed", 1 << 16, 0.6, cache_path=path)["nhash"] == 2
    open(path, "w").write("not json")
    assert tune.load_cache(path) == {}


def test_bench_byte_model():
    sys.path.insert(0, ROOT)
    import bench
    n, d = 1 << 20, 943718
    # bucketed, B = 8: key + flag + one line per key, a half line per new key
    assert bench.kernel_bytes("bucketed_fop", n, d, 3, 8) == n * (9 + 128) + d * 64
    # B = 64: a bucket is four lines
    assert bench.kernel_bytes("bucketed_fop", n, d, 3, 64) == n * (9 + 4 * 128) + d * 64
    assert bench.kernel_bytes("cuckoo_probe", n, d, 3, 8) == n * (9 + 128) + d * 64
    assert bench.kernel_bytes("cuckoo_evict", n, d, 3, 8) is None
    h = bench.kernel_source_hash()
    assert len(h) == 64 and h == bench.kernel_source_hash()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus above 1 exits with status 2 and a
    message, before touching torch or the GPU."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
