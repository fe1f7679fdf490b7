"""Host-side logic without a GPU: the autotuner's grid, cache keys, cache file
round trip and pick; the bench's byte model and source hash."""
import json
import os
import sys

import pytest

from paper_1712_09494_amd import tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_grid_is_the_documented_sweep():
    """The many-table grid sweeps B and c for both designs (the launch it
    times has no keys-per-wave knob); the single-table grid adds R."""
    bk = tune.GRID["bucketed"]
    assert len(bk) == 4 * 3
    assert {p["bucket_slots"] for p in bk} == {8, 16, 32, 64}
    assert {p["nhash"] for p in bk} == {2, 3, 4}
    assert all("keys_per_group" not in p for p in bk)
    ck = tune.GRID["cuckoo"]
    assert [p["nhash"] for p in ck] == [2, 3, 4] and all("bucket_slots" not in p for p in ck)
    bs = tune.GRID_SINGLE["bucketed"]
    assert len(bs) == 4 * 3 * 3 and {p["keys_per_group"] for p in bs} == {1, 2, 4}
    assert len(tune.GRID_SINGLE["cuckoo"]) == 3 * 3


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
    # the probe kernel also empties the set slots of the previous call's winners
    assert (bench.kernel_model("cuckoo_probe", n, d, 3, 8, 0.5, scrubbed=1000)["bytes"]
            == bench.kernel_model("cuckoo_probe", n, d, 3, 8, 0.5)["bytes"] + 16 * 1000)
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


def _fake_result():
    """A result dict shaped like a full bench run (every section present)."""
    rl = {"bound": "hbm", "achieved": 4190.0, "peak": 8000.0, "unit": "GB/s", "frac": 0.52, "traffic": 268030000,
          "bytes_per_launch": 272900000, "avg_launch_ms": 0.0651, "keys_per_launch": 1 << 20,
          "model": {"lines_per_key": 1.51, "cas_per_key": 0.83, "model_vs_counter": 1.018},
          "mix": {"probe_ms": 0.06, "frac_of_mix": 0.92},
          "atomics": {"per_launch": 872461, "achieved_Gps": 13.4, "cas_probe_Gps": 18.6, "frac": 0.72},
          "random_lines": {"per_launch": 1500000, "achieved_Gps": 23.0, "line_probe_Gps": 52.8, "frac": 0.44}}
    served_design = {"sequential_backlog": {"requests_per_s": 17000.0, "latency_ms_p99": 230.0},
                     "served_backlog": {"requests_per_s": 45000.0, "latency_ms_p99": 90.0},
                     "poisson": [{"rho": r, "sequential": {"latency_ms_p99": 100.0 * r},
                                  "served": {"latency_ms_p99": 10.0 * r}} for r in (0.5, 0.8, 0.95)],
                     "admission": {"throttled": 120, "latency_ms_p99": 20.0, "requests_per_s": 30000.0}}
    sweep = []
    for design in ("bucketed", "cuckoo"):
        for lf in (0.5, 0.7, 0.9):
            for batch in (1 << 16, 1 << 20, 1 << 24):
                sweep.append({"design": design, "lf": lf, "batch": batch, "fop_mops": 12345.6,
                              "batch_ms_p50": 0.0612, "batch_ms_p99": 0.0734, "ok": True})
            for h in (0.0, 0.5, 1.0):
                sweep.append({"design": design, "lf": lf, "query_hit_rate": h, "query_mops": 30000.0, "ok": True})
    return {
        "value": 12000.0, "ms_per_step": 11.05, "steps": 20, "warmup": 5,
        "config": {"workload": "random-key scaling: 2^26 uniform 64-bit keys, 10% duplicates, find-or-put in "
                               "batches of 1048576 at load factor 0.7; bucketed (B=8, c=3) + cuckoo (c=3) per step",
                   "keys": 1 << 26, "distinct": 60397978, "batch": 1 << 20, "load_factor": 0.7,
                   "designs": ["bucketed", "cuckoo"]},
        "checks": {"bucketed": {"ok": True}, "cuckoo": {"ok": True}},
        "per_design": {k: {"mops": 16000.0, "batch_ms_p50": 0.061, "batch_ms_p99": 0.081, "ms_total": 4.2}
                       for k in ("bucketed", "cuckoo")},
        "paper_designs": {k: {"mops": 9000.0, "batch_ms_p50": 0.1, "batch_ms_p99": 0.2, "ms_total": 7.0,
                              "ok": True, "overflow_keys": 3700}
                          for k in ("cuckoo_paper_order", "bucketed_b16", "bucketed_b16_paper_full")},
        "per_kernel": {k: {"launches": 64, "avg_ms": 0.06, "total_ms": 3.9}
                       for k in ("bucketed_fop", "cuckoo_probe", "cuckoo_evict", "cuckoo_scrub", "clear")},
        "rooflines": {"cuckoo_probe": dict(rl), "bucketed_fop": dict(rl)},
        "roofline": dict(rl, kernel="cuckoo_probe"),
        "cuckoo_evict": {"avg_ms": 0.0369, "max_ms": 0.1295, "p99_ms": 0.12, "launches": 64, "evictions": 14800000,
                         "chains": {"bins": [2 ** i for i in range(16)], "counts": [123456] * 16, "mean": 2.7,
                                    "p99": 31, "max": 127}},
        "sweep": sweep,
        "w1": {"designs": {k: {"fop_mops": 15900.0, "query_mops": 36000.0, "frac_of_mix": 0.6}
                           for k in ("bucketed", "bucketed_group_query", "bucketed_one_lane", "cuckoo")}},
        "bfs": {"designs": {k: {"fop_mops": 32600.0, "level_mops": 13300.0}
                            for k in ("bucketed", "bucketed_one_lane", "bucketed_fused", "cuckoo", "cuckoo_fused",
                                      "bucketed_b16", "cuckoo_paper_order")}},
        "batched": {"designs": {k: {"plain_ms": 30.0, "graph_ms": 6.0, "speedup_graph_vs_plain": 5.0}
                                for k in ("bucketed", "cuckoo")}},
        "served": {"designs": {"bucketed": served_design, "cuckoo": served_design}},
        "cpu_baseline": {"value": 40.5, "unit": "Mops/s", "cores": 16, "kind": "oracle",
                         "sample": "the whole sequence (67108864 keys, 60397978 distinct) in batches of 1048576: "
                                   "C++ std::unordered_set oracle, hash-partitioned over per-thread sets",
                         "one_core": {"value": 2.5, "seconds": 27.0, "threads": 1, "new": 60397978},
                         "all_cores": {"value": 40.5, "seconds": 1.7, "threads": 16, "new": 60397978},
                         "host": {"cpu_model": "AMD EPYC 9575F 64-Core Processor", "nproc": 16, "cpu_count": 256}},
    }


def test_bench_headline_is_compact_and_complete():
    """The last stdout line of bench.py stays within 4 KB with every section
    present, and carries the fields the result contract names."""
    sys.path.insert(0, ROOT)
    import bench
    line = bench.headline(_fake_result())
    text = json.dumps(line)
    assert len(text) <= 4096, len(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in line, k
    assert line["config"]["workload"].startswith("random-key scaling")
    r = line["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel", "frac_of_mix", "atomics",
              "random_lines"):
        assert r[k] is not None, k
    c = line["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] == 16 and c["one_core"]["value"] and c["host"]["cpu_model"]
    assert line["cuckoo_over_bucketed"]["random"]["paper_cuckoo_over_bucketed"] == 1.0
    assert line["served"]["cuckoo"]["admission"]["throttled"] == 120
    # an empty result (sections skipped) still gives a line
    assert json.loads(json.dumps(bench.headline({"value": 1.0})))["value"] == 1.0


def test_bench_cuckoo_lines_model():
    """Lines read per key by the Cuckoo probe: one at an empty table, c when
    every slot is taken, and the W2 fill's average near the 1.48 lines per key
    the counters show (265 MB per 2^20-key launch)."""
    sys.path.insert(0, ROOT)
    import argparse
    import bench
    assert bench.cuckoo_lines(0.0, 3) == 1.0
    assert bench.cuckoo_lines(1.0, 3) == 3.0
    assert abs(bench.cuckoo_lines(0.5, 3) - 1.75) < 1e-12
    args = argparse.Namespace(n=1 << 26, batch=1 << 20, bucket_slots=8)
    d = 60397978
    cap = int(-(-d // 0.7))
    m = bench.fill_model("cuckoo_probe", args, d, cap, None)
    assert 1.45 < m["lines_per_key"] < 1.55
    b = bench.fill_model("bucketed_fop", args, d, cap, None)
    assert b["lines_per_key"] == 1.0 and abs(b["cas_per_key"] - d / args.n) < 1e-9
