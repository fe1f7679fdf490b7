"""GPU: the served request loop (continuous batching over resident tables).

Each result equals the one the request gets when its table's requests run
one by one in arrival order (per-table FIFO), and equals the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_flags_r2, check_query_r1  # noqa: E402

pytestmark = pytest.mark.gpu

SPECS = [("bucketed", dict(bucket_slots=8)), ("bucketed", dict(bucket_slots=16)), ("cuckoo", dict())]


def make_tables(ntables, cap):
    return [b.Table(SPECS[i % len(SPECS)][0], capacity=cap, **SPECS[i % len(SPECS)][1]) for i in range(ntables)]


def pinned(a):
    t = torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).pin_memory()
    assert t.is_pinned()
    return t


def alone(reqs, ntables, cap):
    """Each table's requests one by one, in arrival order, with plain calls."""
    tables = make_tables(ntables, cap)
    order = sorted(range(len(reqs)), key=lambda i: reqs[i][3])
    res = [None] * len(reqs)
    for i in order:
        op, t, keys, _ = reqs[i]
        if keys.size == 0:
            res[i] = np.zeros(0, np.uint8)
            continue
        k = torch.from_numpy(keys.view(np.int64)).cuda()
        out = tables[t].query(k) if op == "query" else tables[t].find_or_put(k)
        res[i] = out.cpu().numpy()
    dumps = [np.sort(b.u64(t.dump())) for t in tables]
    for t in tables:
        t.close()
    return res, dumps


def oracle_run(reqs, ntables):
    os_ = [Oracle() for _ in range(ntables)]
    order = sorted(range(len(reqs)), key=lambda i: reqs[i][3])
    res = [None] * len(reqs)
    for i in order:
        op, t, keys, _ = reqs[i]
        res[i] = os_[t].query(keys) if op == "query" else os_[t].find_or_put(keys)
    return res, os_


def compare(reqs, got, ref, what):
    for i, (op, t, keys, _) in enumerate(reqs):
        g = got[i]
        if op == "query":
            check_query_r1(g, ref[i], f"{what} req {i}")
        else:
            check_flags_r2(keys, g, ref[i], f"{what} req {i}")


@pytest.mark.parametrize("cfg", [dict(slots=4, merge=8), dict(slots=2, merge=1), dict(sequential=True),
                                 dict(slots=8, merge=16)])
@pytest.mark.parametrize("rate", [0.0, 20000.0])
def test_served_equals_alone_and_oracle(cfg, rate):
    ntables, cap = 7, 1 << 16
    reqs = inputs.served_trace(240, ntables, log_min=4, log_max=13, rate=rate, seed=11)
    tables = make_tables(ntables, cap)
    srv = b.Server(tables, **cfg)
    outs, admit, done, groups, st = srv.run([(op, t, pinned(k), a) for op, t, k, a in reqs])
    got = [o.numpy() for o in outs]
    assert (done >= admit).all() and (admit >= np.array([r[3] for r in reqs]) - 1e-9).all()
    ref, dumps = alone(reqs, ntables, cap)
    compare(reqs, got, ref, f"served vs alone {cfg}")
    ora, os_ = oracle_run(reqs, ntables)
    compare(reqs, got, ora, f"served vs oracle {cfg}")
    for t in range(ntables):
        d = np.sort(b.u64(tables[t].dump()))
        assert np.array_equal(d, dumps[t]) and np.array_equal(d, os_[t].dump())
    if not cfg.get("sequential") and cfg.get("merge", 16) > 1 and rate == 0.0:
        assert st["merged_launches"] > 0
    srv.close()
    for t in tables:
        t.close()


def test_served_admission_throttles_without_changing_results():
    """Requests above the small-request size (so they take staging from the
    budget) under a budget of two of the largest: admission waits, results
    do not change."""
    ntables, cap = 5, 1 << 20
    reqs = inputs.served_trace(60, ntables, log_min=13.2, log_max=16.5, seed=12)
    biggest = max(k.size for _, _, k, _ in reqs)
    budget = 2 * (((biggest * 8 + 255) // 256) * 256 + ((biggest + 255) // 256) * 256)
    tables = make_tables(ntables, cap)
    srv = b.Server(tables, slots=4, merge=8, staging_bytes=budget)
    outs, admit, done, groups, st = srv.run([(op, t, pinned(k), a) for op, t, k, a in reqs])
    assert st["throttled"] > 0 and st["peak_staging"] <= budget
    ora, _ = oracle_run(reqs, ntables)
    compare(reqs, [o.numpy() for o in outs], ora, "throttled")
    srv.close()
    for t in tables:
        t.close()


def test_served_rejects_bad_requests():
    t = b.Table("bucketed", capacity=1024)
    srv = b.Server([t])
    k = pinned(inputs.uniform_keys(10, seed=1))
    with pytest.raises(b.HtError):
        srv.run([("fop", 3, k, 0.0)])                  # no such table
    with pytest.raises(ValueError):
        srv.run([("fop", 0, torch.zeros(4, dtype=torch.int64), 0.0)])   # not pinned
    srv.close()
    t.close()


def _rows(a, w):
    a = np.ascontiguousarray(a).view(np.uint64).reshape(-1, w)
    return a.view(np.dtype((np.void, 8 * w))).reshape(-1)


def test_served_vector_tables_beside_single_word_ones():
    """State-vector tables (2 and 4 words, both designs) served beside
    single-word tables in merged groups: every request's result equals the
    oracle's in arrival order, and every table's stored set equals the
    oracle's."""
    from oracle import VecOracle
    specs = [("bucketed", dict(bucket_slots=8), 1), ("cuckoo", {}, 2), ("bucketed", dict(bucket_slots=16), 4),
             ("cuckoo", {}, 4), ("bucketed", dict(bucket_slots=8), 2), ("cuckoo", {}, 1)]
    tables = [b.Table(k, capacity=1 << 14, key_words=w, **kw) for k, kw, w in specs]
    rng = np.random.default_rng(21)
    pools = [inputs.vector_of_index(np.arange(6000), w, seed=40 + i, structured=bool(i % 2)) if w > 1
             else inputs.uniform_keys(6000, seed=40 + i) for i, (_, _, w) in enumerate(specs)]
    reqs = []
    for _ in range(150):
        t = int(rng.integers(0, len(specs)))
        keys = pools[t][rng.integers(0, len(pools[t]), int(rng.integers(0, 700)))]
        reqs.append(("query" if rng.random() < 0.4 else "fop", t, keys, 0.0))
    srv = b.Server(tables, slots=4, merge=8)
    outs, _, _, _, st = srv.run([(op, t, pinned(k), a) for op, t, k, a in reqs])
    assert st["merged_launches"] > 0
    oras = [VecOracle(w) if w > 1 else Oracle() for _, _, w in specs]
    for i, (op, t, keys, _) in enumerate(reqs):          # released together: arrival order is index order
        w = specs[t][2]
        got = outs[i].numpy()
        assert got.size == len(keys)
        if op == "query":
            check_query_r1(got, oras[t].query(keys), f"req {i}")
        elif w == 1:
            check_flags_r2(keys, got, oras[t].find_or_put(keys), f"req {i}")
        else:
            exp = oras[t].find_or_put(keys)
            assert set(np.unique(got).tolist()) <= {0, 1}, f"req {i}"
            v = _rows(keys, w)
            assert np.array_equal(np.sort(v[got == 1]), np.sort(v[exp == 1])), f"req {i}"
    for t, (_, _, w) in enumerate(specs):
        d = tables[t].dump().cpu().numpy()
        if w == 1:
            assert np.array_equal(np.sort(d.view(np.uint64)), oras[t].dump())
        else:
            assert np.array_equal(np.sort(_rows(d, w)), np.sort(_rows(oras[t].dump(), w)))
    srv.close()
    for t in tables:
        t.close()


def test_served_small_and_large_requests_in_one_group():
    """Small requests (packed into the slot's area, one copy each way) and
    large ones (their own staging and copies) mixed within groups, several
    groups deep: every result equals the oracle's."""
    ntables, cap = 6, 1 << 20
    reqs = inputs.served_trace(200, ntables, log_min=4, log_max=17, seed=13)
    assert any(k.size * 8 > (64 << 10) for _, _, k, _ in reqs) and any(k.size < 1024 for _, _, k, _ in reqs)
    tables = make_tables(ntables, cap)
    srv = b.Server(tables, slots=3, merge=16)
    outs, admit, done, groups, st = srv.run([(op, t, pinned(k), a) for op, t, k, a in reqs])
    ora, os_ = oracle_run(reqs, ntables)
    compare(reqs, [o.numpy() for o in outs], ora, "small and large")
    for t in range(ntables):
        assert np.array_equal(np.sort(b.u64(tables[t].dump())), os_[t].dump())
    srv.close()
    for t in tables:
        t.close()


def test_served_requests_at_the_packing_size():
    """Requests of exactly 64 KiB of keys (packed into the slot's area) and
    one key more (their own staging), single-word and 4-word vector tables,
    in the same groups: every result equals the oracle's."""
    from oracle import VecOracle
    tables = [b.Table("bucketed", capacity=1 << 17, bucket_slots=8), b.Table("cuckoo", capacity=1 << 17),
              b.Table("bucketed", capacity=1 << 16, key_words=4), b.Table("cuckoo", capacity=1 << 16, key_words=4)]
    words = [1, 1, 4, 4]
    oras = [Oracle(), Oracle(), VecOracle(4), VecOracle(4)]
    reqs = []
    for rnd in range(3):
        for t, w in enumerate(words):
            rows = (64 << 10) // (8 * w) + (rnd % 2)          # at the size, then one key above
            if w == 1:
                keys = inputs.random_sequence(rows, rows - rows // 5, seed=900 + 10 * rnd + t)
            else:
                keys = inputs.vector_sequence(rows, rows - rows // 5, w, seed=900 + 10 * rnd + t)
            reqs.append(("fop" if rnd < 2 else "query", t, keys, 0.0))
    srv = b.Server(tables, slots=2, merge=4)
    outs, _, _, _, st = srv.run([(op, t, pinned(k), a) for op, t, k, a in reqs])
    for i, (op, t, keys, _) in enumerate(reqs):
        got = outs[i].numpy()
        if op == "query":
            check_query_r1(got, oras[t].query(keys), f"req {i}")
        elif words[t] == 1:
            check_flags_r2(keys, got, oras[t].find_or_put(keys), f"req {i}")
        else:
            exp = oras[t].find_or_put(keys)
            v = _rows(keys, 4)
            assert np.array_equal(np.sort(v[got == 1]), np.sort(v[exp == 1])), f"req {i}"
    srv.close()
    for t in tables:
        t.close()
