"""GPU: breadth-first exploration with each table as the visited set.

Levels 0-4 are compared with the oracle's BFS (same batch multisets, same new
states); the full seven levels (a 715,127,564-key batch, 121,210,369 states)
are checked against tests/golden/bfs_calibration.json, written by the
oracle-only script beside it: every level's batch size and visited count,
and the visited set itself through its digest (count, sum and xor of two
mixes of every member)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle, set_digest  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "bfs_calibration.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


DESIGNS = [("bucketed", dict(bucket_slots=8)), ("bucketed", dict(bucket_slots=16)), ("cuckoo", dict()),
           ("cuckoo", dict(flags=b.HT_FLAG_CUCKOO_PAPER_ORDER))]


@pytest.mark.parametrize("kind,kw", DESIGNS)
def test_bfs_levels_match_oracle(kind, kw):
    model = inputs.BfsModel(1)
    o = Oracle([0])
    frontier = np.array([0], dtype=np.uint64)
    sizes, news = [], []
    for _ in range(5):
        batch = model.successors(frontier)
        f = o.find_or_put(batch)
        frontier = batch[f == 1]
        sizes.append(batch.size)
        news.append(int(f.sum()))
    with b.Table(kind, capacity=int(np.ceil(o.size / 0.7)), nhash=3, **kw) as t:
        r = t.bfs_explore(model, 5)
        assert r["batch_sizes"] == sizes
        assert r["new_counts"] == news
        d = np.sort(b.u64(t.dump()))
        assert np.array_equal(d, o.dump())
        assert t.size() == o.size


def check_visited_set(t, g):
    """The table's members equal the oracle's visited set after the last
    level (digest of the dump: count, sum and xor of two mixes)."""
    dump = b.u64(t.dump())
    assert set_digest(dump) == g["visited_digest"][-1]


# the bench's BFS configurations: bucketed B = 8, c = 3; Cuckoo c = 4 (and c = 3)
FULL = [("bucketed", dict(bucket_slots=8)), ("cuckoo", dict()), ("cuckoo", dict(nhash=4))]
# the bench's other split-level designs: one lane per key, the 128-byte bucket, the Sec. 4.1 order
FULL_SPLIT = FULL + [("bucketed", dict(bucket_slots=8, flags=b.HT_FLAG_BUCKETED_ONE_LANE)),
                     ("bucketed", dict(bucket_slots=16)),
                     ("cuckoo", dict(nhash=4, flags=b.HT_FLAG_CUCKOO_PAPER_ORDER))]


def table_args(kw):
    a = dict(nhash=3)
    a.update(kw)
    return a


@pytest.mark.parametrize("kind,kw", FULL_SPLIT)
def test_bfs_full_size_seed1(kind, kw):
    g = golden()["seed1"]
    visited = g["visited_after"]
    with b.Table(kind, capacity=int(np.ceil(visited[-1] / 0.7)), **table_args(kw)) as t:
        r = t.bfs_explore(inputs.BfsModel(1), 7)
        assert r["batch_sizes"] == g["batch_sizes"]
        assert r["new_counts"] == g["new_counts"]
        assert list(1 + np.cumsum(r["new_counts"])) == visited
        assert t.size() == visited[-1]
        assert t.sync_status() == b.HT_OK
        check_visited_set(t, g)


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", dict())])
def test_bfs_full_size_seed2(kind, kw):
    g = golden()["seed2"]
    with b.Table(kind, capacity=int(np.ceil(g["visited_after"][-1] / 0.7)), nhash=3, **kw) as t:
        r = t.bfs_explore(inputs.BfsModel(2), 7)
        assert r["batch_sizes"] == g["batch_sizes"]
        assert list(1 + np.cumsum(r["new_counts"])) == g["visited_after"]
        check_visited_set(t, g)


FUSED = [("bucketed", dict(bucket_slots=8)), ("bucketed", dict(bucket_slots=16)),
         ("bucketed", dict(bucket_slots=32, nhash=4)), ("bucketed", dict(bucket_slots=64, nhash=2)),
         ("bucketed", dict(bucket_slots=16, flags=b.HT_FLAG_BUCKETED_PAPER_FULL)),
         ("cuckoo", dict()), ("cuckoo", dict(nhash=4)), ("cuckoo", dict(nhash=2)),
         ("cuckoo", dict(flags=b.HT_FLAG_CUCKOO_PAPER_ORDER))]


def oracle_bfs(model, initial, levels):
    o = Oracle([initial])
    frontier = np.array([initial], dtype=np.uint64)
    sizes, news = [], []
    for _ in range(levels):
        batch = model.successors(frontier)
        f = o.find_or_put(batch)
        frontier = batch[f == 1]
        sizes.append(batch.size)
        news.append(int(f.sum()))
    return o, sizes, news


@pytest.mark.parametrize("kind,kw", FUSED)
def test_bfs_fused_levels_match_oracle(kind, kw):
    """Fused levels (successor generation joined with the find-or-put) give
    the oracle's batch sizes, new counts and visited set."""
    model = inputs.BfsModel(1)
    o, sizes, news = oracle_bfs(model, 0, 5)
    kw = dict(kw)
    kw.setdefault("nhash", 3)
    with b.Table(kind, capacity=int(np.ceil(o.size / 0.7)), **kw) as t:
        r = t.bfs_explore(model, 5, fused=True)
        assert r["batch_sizes"] == sizes
        assert r["new_counts"] == news
        assert all(x > 0 for x in r["level_ms"])
        assert np.array_equal(np.sort(b.u64(t.dump())), o.dump())
        assert t.size() == o.size


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", dict())])
def test_bfs_fused_from_all_ones_state(kind, kw):
    """The all-ones state (the table's empty marker) as the initial state:
    fused and split levels agree with the oracle."""
    model = inputs.BfsModel(2)
    init = int(b.EMPTY)
    o, sizes, news = oracle_bfs(model, init, 4)
    for fused in (False, True):
        with b.Table(kind, capacity=int(np.ceil(o.size / 0.7)), nhash=3, **kw) as t:
            r = t.bfs_explore(model, 4, initial=init, fused=fused)
            assert r["batch_sizes"] == sizes, fused
            assert r["new_counts"] == news, fused
            assert np.array_equal(np.sort(b.u64(t.dump())), o.dump()), fused
            assert t.query(torch.tensor([-1], dtype=torch.int64, device="cuda")).item() == 1


@pytest.mark.parametrize("kind,kw", FULL)
def test_bfs_fused_full_size_seed1(kind, kw):
    g = golden()["seed1"]
    visited = g["visited_after"]
    with b.Table(kind, capacity=int(np.ceil(visited[-1] / 0.7)), **table_args(kw)) as t:
        r = t.bfs_explore(inputs.BfsModel(1), 7, fused=True)
        assert r["batch_sizes"] == g["batch_sizes"]
        assert list(1 + np.cumsum(r["new_counts"])) == visited
        assert t.size() == visited[-1]
        assert t.sync_status() == b.HT_OK
        check_visited_set(t, g)


def test_bfs_split_level_times():
    """The mode-taking call in split mode equals the plain call and reports
    per-level device times that cover the find-or-put."""
    model = inputs.BfsModel(1)
    with b.Table("cuckoo", capacity=1 << 16, nhash=3) as t1, b.Table("cuckoo", capacity=1 << 16, nhash=3) as t2:
        r1 = t1.bfs_explore(model, 4)
        r2 = b.ht_bfs_explore_ex(t2.handle, model, 4, b.HT_BFS_SPLIT)
        assert r1["batch_sizes"] == r2["batch_sizes"] and r1["new_counts"] == r2["new_counts"]
        assert all(lv >= f > 0 for lv, f in zip(r2["level_ms"], r2["fop_ms"]))


def test_bfs_fused_rejects_other_tables():
    model = inputs.BfsModel(1)
    for kind in ("bucketed", "cuckoo"):
        with b.Table(kind, capacity=1024, flags=b.HT_FLAG_SCRIPTED_HASH) as t:
            with pytest.raises(b.HtError):
                t.bfs_explore(model, 2, fused=True)
    with b.Table("bucketed", capacity=1024) as t:
        with pytest.raises(b.HtError):
            b.ht_bfs_explore_ex(t.handle, model, 2, 7)
