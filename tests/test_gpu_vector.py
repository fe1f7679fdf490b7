"""GPU: tables whose keys are state vectors of 2 or 4 words.

Parity with the vector oracle (flags: the multiset of rows reported new;
queries bit-exact; dump: the member set with no row twice), through the
stash and overflow list, across calls, with duplicate storms and with
structured vectors that share most of their words."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import VecOracle, first_occurrence_flags_vec  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

DESIGNS = {
    "bkt8": dict(kind="bucketed", bucket_slots=8),
    "bkt16": dict(kind="bucketed", bucket_slots=16),
    "bkt8_paperfull": dict(kind="bucketed", bucket_slots=8, flags=b.HT_FLAG_BUCKETED_PAPER_FULL),
    "cuckoo": dict(kind="cuckoo"),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def rows(a, w):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64)).reshape(-1, w)
    return a.view(np.dtype((np.void, 8 * w))).reshape(-1)


def check_flags(keys, got, exp, w, what=""):
    got = np.asarray(got, dtype=np.uint8)
    assert set(np.unique(got).tolist()) <= {0, 1}, what
    g = np.sort(rows(keys, w)[got == 1])
    e = np.sort(rows(keys, w)[np.asarray(exp) == 1])
    assert g.size == e.size and (g == e).all(), f"{what}: new rows differ ({g.size} vs {e.size})"


def check_dump(t, o, w, what=""):
    d = t.dump().cpu().numpy().view(np.uint64).reshape(-1, w)
    dr = rows(d, w)
    assert np.unique(dr).size == dr.size, f"{what}: a row is stored twice"
    assert t.size() == o.size == dr.size, what
    assert (np.sort(dr) == np.sort(rows(o.dump(), w))).all(), what


def fop(t, keys):
    return t.find_or_put(dev(keys)).cpu().numpy() if len(keys) else np.zeros(0, np.uint8)


def query(t, keys):
    return t.query(dev(keys)).cpu().numpy()


@pytest.mark.parametrize("design", list(DESIGNS))
@pytest.mark.parametrize("w", [2, 4])
def test_vec_tiny_alphabets(design, w):
    """Short random sequences over a few vectors that share words, in a
    64-slot table, split into several calls."""
    M = (1 << 64) - 1
    base = [0, 1, 1 << 63, M]
    rng = np.random.default_rng(w * 7 + len(design))
    alpha = np.array([[base[(i >> (2 * j)) & 3] for j in range(w)] for i in range(4 ** w)], dtype=np.uint64)
    for trial in range(20):
        t = b.Table(capacity=64, nhash=int(rng.integers(1, 5)), key_words=w, **DESIGNS[design])
        o = VecOracle(w)
        for _ in range(3):
            seq = alpha[rng.integers(0, len(alpha), size=int(rng.integers(0, 40)))]
            check_flags(seq, fop(t, seq), o.find_or_put(seq), w, f"{design} w={w} trial {trial}")
        assert (query(t, alpha) == o.query(alpha)).all()
        check_dump(t, o, w, design)
        t.close()


@pytest.mark.parametrize("design", list(DESIGNS))
def test_vec_stash_overflow_rebuild(design):
    """A table far too small: vectors go to the stash and the overflow list,
    stay members, HT_EFULL is reported, and a rebuild restores the table."""
    w = 2
    kw = dict(DESIGNS[design])
    t = b.Table(capacity=64, nhash=1, stash_slots=16, overflow_slots=4096, key_words=w, **kw)
    keys = inputs.vector_sequence(700, 500, w, seed=3)
    o = VecOracle(w)
    check_flags(keys, fop(t, keys), o.find_or_put(keys), w, design)
    assert t.sync_status() == b.HT_EFULL
    st = t.stats()
    assert st["stash_count"] == 16 and st["overflow_count"] > 0 and st["lost"] == 0
    assert query(t, keys).all()
    check_dump(t, o, w, design)
    t.rebuild(new_capacity=1 << 14)
    assert t.sync_status() == b.HT_OK
    check_dump(t, o, w, design + " after rebuild")
    more = inputs.vector_sequence(3000, 2000, w, seed=4)
    check_flags(more, fop(t, more), o.find_or_put(more), w, design + " after rebuild")
    check_dump(t, o, w, design)
    t.close()


@pytest.mark.parametrize("design", ["bkt8", "bkt16", "cuckoo"])
@pytest.mark.parametrize("w", [2, 4])
@pytest.mark.parametrize("structured", [False, True])
def test_vec_2p20_batches(design, w, structured):
    """2^20 vectors with 10% duplicates at load factor 0.7 in batches of 2^16
    and 2^18 + 3, then queries at hit rate 0.5; both generators."""
    n, d = 1 << 20, int(0.9 * (1 << 20))
    seq = inputs.vector_sequence(n, d, w, seed=11 + w, structured=structured)
    t = b.Table(capacity=int(d / 0.7), nhash=3, key_words=w, **DESIGNS[design])
    o = VecOracle(w)
    flags = []
    for bs in (1 << 16, (1 << 18) + 3):
        t.clear()
        o = VecOracle(w)
        flags = []
        for s0 in range(0, n, bs):
            part = seq[s0:s0 + bs]
            flags.append(fop(t, part))
            o.find_or_put(part)
        f = np.concatenate(flags)
        check_flags(seq, f, first_occurrence_flags_vec(seq, w), w, f"{design} w={w} batch {bs}")
        assert t.size() == d and t.sync_status() == b.HT_OK
    present = inputs.vector_of_index(np.arange(0, d, 3), w, seed=11 + w, structured=structured)
    absent = inputs.vector_of_index(np.arange(d, d + present.shape[0]), w, seed=11 + w, structured=structured)
    q = np.concatenate([present, absent])
    got = query(t, q)
    assert got[: present.shape[0]].all() and not got[present.shape[0]:].any()
    check_dump(t, o, w, design)
    t.close()


@pytest.mark.parametrize("design", ["bkt8", "cuckoo"])
def test_vec_duplicate_storms(design):
    """One vector 2^18 times; 64 vectors differing only in their last word,
    each repeated 1000 times and interleaved; the all-ones vector."""
    w = 4
    t = b.Table(capacity=1 << 12, nhash=3, key_words=w, **DESIGNS[design])
    o = VecOracle(w)
    one = np.tile(np.array([[5, 6, 7, 8]], dtype=np.uint64), (1 << 18, 1))
    check_flags(one, fop(t, one), o.find_or_put(one), w, "one vector")
    near = np.tile(np.array([[5, 6, 7, 0]], dtype=np.uint64), (64 * 1000, 1))
    near[:, 3] = np.arange(64 * 1000, dtype=np.uint64) % 64
    check_flags(near, fop(t, near), o.find_or_put(near), w, "last word differs")
    ones = np.full((5000, w), (1 << 64) - 1, dtype=np.uint64)
    check_flags(ones, fop(t, ones), o.find_or_put(ones), w, "all ones")
    check_dump(t, o, w, design)
    assert t.size() == 65          # (5, 6, 7, 8) is also one of the 64 last-word variants
    t.close()


def test_vec_rejected_uses():
    t = b.Table("bucketed", capacity=1024, key_words=2)
    k = dev(inputs.vector_of_index(np.arange(8), 2, seed=1))
    with pytest.raises(b.HtError):                       # 8-byte aligned, not 16
        b.ht_find_or_put(t.handle, k.reshape(-1)[1:15], key_words=2)
    with pytest.raises(b.HtError):                       # a misaligned batch in a many-table call
        b.ht_find_or_put_multi([t.handle], [k.reshape(-1)[1:15]], key_words=[2])
    with pytest.raises(b.HtError):
        t.bfs_explore(inputs.BfsModel(1), 2)
    with pytest.raises(ValueError):
        t.find_or_put(k.reshape(-1)[:5])
    t.clear()
    assert t.size() == 0 and t.dump().shape[0] == 0
    t.close()


@pytest.mark.parametrize("kind", ["bucketed", "cuckoo"])
@pytest.mark.parametrize("w", [2, 4])
def test_vec_random_small_tables(kind, w):
    """Random small tables (64..1024 slots, c = 1..4, any bucket width), pools of
    vectors that share words, several batches with repeats: flags, queries and
    dump against the oracle, through spills into the stash and overflow set."""
    rng = np.random.default_rng(100 + w + (kind == "cuckoo"))
    for trial in range(10):
        cap = int(rng.choice([64, 128, 256, 1024]))
        kw = dict(bucket_slots=int(rng.choice([8, 16, 32, 64]))) if kind == "bucketed" else {}
        t = b.Table(kind, capacity=cap, nhash=int(rng.integers(1, 5)), stash_slots=32, overflow_slots=2048,
                    key_words=w, **kw)
        o = VecOracle(w)
        pool = inputs.vector_of_index(np.arange(int(rng.integers(8, 2 * cap))), w, seed=trial,
                                      structured=bool(trial % 2))
        for _ in range(4):
            part = pool[rng.integers(0, len(pool), size=int(rng.integers(0, 900)))]
            check_flags(part, fop(t, part), o.find_or_put(part), w, f"{kind} w={w} trial {trial} cap {cap}")
        extra = inputs.vector_of_index(np.arange(10 ** 6, 10 ** 6 + 50), w, seed=trial)
        q = np.concatenate([pool, extra])
        assert (query(t, q) == o.query(q)).all(), f"{kind} trial {trial}"
        check_dump(t, o, w, f"{kind} trial {trial}")
        t.close()


def test_vec_many_table_calls():
    """State-vector tables (2 and 4 words, both designs) in many-table calls
    beside single-word tables: the one-shot call, a plan launched from a
    captured HIP graph (replayed onto cleared tables) and the many-table query
    all equal the oracle."""
    from oracle import Oracle
    specs = [("bucketed", dict(bucket_slots=8), 2), ("cuckoo", {}, 4), ("bucketed", dict(bucket_slots=16), 1),
             ("cuckoo", {}, 2), ("bucketed", dict(bucket_slots=8), 4), ("cuckoo", {}, 1)]
    batches = []
    for i, (_, _, w) in enumerate(specs):
        n = 3000 + 777 * i
        if w == 1:
            batches.append(inputs.random_sequence(n, n * 2 // 3, seed=60 + i))
        else:
            batches.append(inputs.vector_sequence(n, n * 2 // 3, w, seed=60 + i, structured=bool(i % 2)))

    def make():
        return [b.Table(k, capacity=8192, key_words=w, **kw) for k, kw, w in specs]

    def oracles():
        return [VecOracle(w) if w > 1 else Oracle() for _, _, w in specs]

    def check(tables, outs, what):
        os_ = oracles()
        for i, (t, (_, _, w)) in enumerate(zip(tables, specs)):
            exp = os_[i].find_or_put(batches[i])
            got = outs[i].cpu().numpy()
            if w == 1:
                assert np.array_equal(np.sort(batches[i][got == 1]), np.sort(batches[i][exp == 1])), (what, i)
            else:
                check_flags(batches[i], got, exp, w, f"{what} table {i}")
            assert t.size() == os_[i].size, (what, i)
        return os_

    kd = [dev(x) for x in batches]
    tables = make()
    os_ = check(tables, b.find_or_put_multi(tables, kd), "one-shot call")
    queries = []
    for i, (_, _, w) in enumerate(specs):
        fresh = (inputs.uniform_keys(500, seed=80 + i) if w == 1
                 else inputs.vector_of_index(np.arange(10**6, 10**6 + 500), w, seed=60 + i))
        queries.append(np.concatenate([batches[i][:700], fresh]))
    found = b.query_multi(tables, [dev(q) for q in queries])
    for i in range(len(specs)):
        assert np.array_equal(found[i].cpu().numpy(), os_[i].query(queries[i])), i
    for t in tables:
        t.close()

    tables = make()
    outs = [torch.empty(len(x), dtype=torch.uint8, device="cuda") for x in batches]
    plan = b.MultiPlan(tables, kd, outs)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.launch()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in tables:
            t.clear()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(tables, outs, f"graph replay {rep}")
    del g
    plan.close()
    for t in tables:
        t.close()
