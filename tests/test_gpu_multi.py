"""GPU: many tables filled in one persistent launch equal one call per table,
and the plan launch replays correctly from a captured HIP graph."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle, first_occurrence_flags  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_dump_r3, check_flags_r2  # noqa: E402

pytestmark = pytest.mark.gpu

KINDS = [
    ("bucketed", dict(bucket_slots=8)),
    ("bucketed", dict(bucket_slots=16)),
    ("bucketed", dict(bucket_slots=32, nhash=2)),
    ("bucketed", dict(bucket_slots=64, nhash=4)),
    ("cuckoo", dict()),
    ("cuckoo", dict(nhash=4)),
    ("cuckoo", dict(flags=b.HT_FLAG_CUCKOO_PAPER_ORDER)),
]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def make_set(seed, ntables, max_log=16, lf=0.6):
    rng = np.random.default_rng(seed)
    tables, keys, specs = [], [], []
    for i in range(ntables):
        kind, kw = KINDS[i % len(KINDS)]
        cap = int(round(2 ** rng.uniform(6, max_log)))
        distinct = max(1, int(lf * cap))
        n = distinct + int(rng.integers(0, distinct // 2 + 1))
        k = inputs.random_sequence(n, distinct, seed=seed * 1000 + i)
        if i % 5 == 0:
            k[:: 97] = b.EMPTY
        if i % 11 == 3:
            k = k[:0]                       # an empty batch
        kw = dict(kw)
        kw.setdefault("nhash", 3)
        tables.append(b.Table(kind, capacity=cap, **kw))
        keys.append(k)
        specs.append((kind, kw, cap))
    return tables, keys, specs


@pytest.mark.parametrize("seed,ntables", [(1, 7), (2, 40), (3, 256)])
def test_multi_equals_oracle(seed, ntables):
    tables, keys, _ = make_set(seed, ntables)
    outs = b.find_or_put_multi(tables, [dev(k) for k in keys])
    for i, t in enumerate(tables):
        f = outs[i].cpu().numpy()
        check_flags_r2(keys[i], f, first_occurrence_flags(keys[i]), f"table {i}")
        check_dump_r3(b.u64(t.dump()), np.unique(keys[i]), t.size(), f"table {i}")
        assert t.sync_status() == b.HT_OK
        t.close()


def test_multi_matches_single_calls():
    tables, keys, specs = make_set(4, 21)
    single = []
    for (kind, kw, cap), k in zip(specs, keys):
        with b.Table(kind, capacity=cap, **kw) as t:
            f = t.find_or_put(dev(k)).cpu().numpy() if k.size else np.zeros(0, np.uint8)
            single.append((f, np.sort(b.u64(t.dump()))))
    outs = b.find_or_put_multi(tables, [dev(k) for k in keys])
    for i, t in enumerate(tables):
        f = outs[i].cpu().numpy()
        # same new-key multiset and same stored set as the per-table call
        assert np.array_equal(np.sort(keys[i][f == 1]), np.sort(keys[i][single[i][0] == 1]))
        assert np.array_equal(np.sort(b.u64(t.dump())), single[i][1])
        t.close()


def test_plan_relaunch_and_graph_replay():
    tables, keys, _ = make_set(5, 24, max_log=14)
    kd = [dev(k) for k in keys]
    plan = b.MultiPlan(tables, kd)
    plan.launch()
    assert plan.status() == b.HT_OK
    for i, t in enumerate(tables):
        check_flags_r2(keys[i], plan.outs[i].cpu().numpy(), first_occurrence_flags(keys[i]), f"t{i}")
    # second launch on full tables: nothing is new
    plan.launch()
    assert plan.status() == b.HT_OK
    for i in range(len(tables)):
        assert int(plan.outs[i].sum()) == 0
    # capture the launch in a graph; replay it on cleared tables several times
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for t in tables:
            t.clear()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            plan.launch()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in tables:
            t.clear()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert plan.status() == b.HT_OK
        for i, t in enumerate(tables):
            check_flags_r2(keys[i], plan.outs[i].cpu().numpy(), first_occurrence_flags(keys[i]), f"rep{rep} t{i}")
            check_dump_r3(b.u64(t.dump()), np.unique(keys[i]), t.size(), f"rep{rep} t{i}")
    plan.close()
    for t in tables:
        t.close()


def test_multi_bfs_prefixes():
    """Tables filled from BFS successor streams (duplicates, structured keys)."""
    model = inputs.BfsModel(3)
    o = Oracle([0])
    frontier = np.array([0], dtype=np.uint64)
    stream = []
    for _ in range(4):
        batch = model.successors(frontier)
        frontier = batch[o.find_or_put(batch) == 1]
        stream.append(batch)
    seq = np.concatenate(stream)
    tables, keys = [], []
    for i, n in enumerate([100, 5000, 70000, seq.size]):
        k = seq[:n]
        d = np.unique(k).size
        kind, kw = KINDS[i % len(KINDS)]
        tables.append(b.Table(kind, capacity=int(d / 0.6) + 16, **kw))
        keys.append(k)
    outs = b.find_or_put_multi(tables, [dev(k) for k in keys])
    for i, t in enumerate(tables):
        check_flags_r2(keys[i], outs[i].cpu().numpy(), first_occurrence_flags(keys[i]), f"bfs t{i}")
        t.close()


def test_multi_large_cuckoo_table():
    """A Cuckoo table whose batch needs more keys per region than the item
    size (above 4096 keys x 8192 waves), beside small tables of both kinds."""
    n = (1 << 25) + 100003
    big = inputs.random_sequence(n, int(0.9 * n), seed=21)
    small = [inputs.random_sequence(3000, 2500, seed=22), inputs.random_sequence(70000, 60000, seed=23)]
    tables = [b.Table("cuckoo", capacity=int(0.9 * n / 0.6), nhash=3),
              b.Table("cuckoo", capacity=5000, nhash=4), b.Table("bucketed", capacity=120000, bucket_slots=8)]
    keys = [big] + small
    outs = b.find_or_put_multi(tables, [dev(k) for k in keys])
    for i, t in enumerate(tables):
        check_flags_r2(keys[i], outs[i].cpu().numpy(), first_occurrence_flags(keys[i]), f"t{i}")
        assert t.size() == np.unique(keys[i]).size
        assert t.sync_status() == b.HT_OK
        t.close()


def test_multi_rejects_bad_arguments():
    t = b.Table("bucketed", capacity=1024)
    k = dev(inputs.uniform_keys(10, seed=1))
    with pytest.raises(b.HtError):
        b.find_or_put_multi([t, t], [k, k])
    ts = b.Table("cuckoo", capacity=64, flags=b.HT_FLAG_SCRIPTED_HASH)
    with pytest.raises(b.HtError):
        b.find_or_put_multi([ts], [k])
    t.close()
    ts.close()


@pytest.mark.skip(reason="switched off: running the Cuckoo phases inside the persistent many-table kernel, "
                         "handed from wave to wave through per-table completion counters and fences, hung and "
                         "corrupted other tables' flags on MI355X; cause not established.  Cuckoo tables of a "
                         "many-table call now run as three phase launches (kernel boundaries as barriers).")
def test_cuckoo_phases_inside_persistent_kernel():
    pass
