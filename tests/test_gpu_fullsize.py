"""GPU parity at the benchmark's full sizes, in its launch configurations.

Random-key scaling: 2^26 keys with 10% duplicates (60,397,978 distinct),
find-or-put in consecutive batches of 2^16, 2^20 and 2^24 keys into a
bucketed table (B = 8, c = 3) and a Cuckoo table (c = 3; c = 4 at load
factor 0.9, as the bench's sweep) sized for load factors 0.5, 0.7 and 0.9:
every configuration the bench times.  Every flag of every batch is checked
against the oracle (per call, exactly), the stored set in full (the dump's
digest against the oracle's set and every distinct key found by query), and
at the headline configuration 2^22 queries at hit rate 0.5 bit-exact.  Also
the state-vector case, the many-table case (one plan launch over 256 tables,
every table checked) and the served case (4,096 requests through the engine,
every request of every table checked)."""
import concurrent.futures as cf

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle, set_digest  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_flags_r2_calls, check_query_r1  # noqa: E402

pytestmark = pytest.mark.gpu


def _threads():
    import os
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 8


def oracle_flags_seq(seq):
    """oracle_flags on one thread (for callers that spread tables over threads)."""
    from oracle import c_oracle
    o = c_oracle.COracle(1, reserve=seq.size)
    f = o.find_or_put(seq)
    o.close()
    return f


def oracle_flags(seq):
    """The oracle's flags for a run of calls from an empty set (the C++ set
    oracle on hash-partitioned threads; the same flags as one sequential
    loop, and as first_occurrence_flags)."""
    from oracle import c_oracle
    o = c_oracle.COracle(_threads(), reserve=seq.size)
    f = o.find_or_put(seq)
    o.close()
    return f


@pytest.fixture(scope="module")
def w2():
    n = 1 << 26
    seq, d = inputs.scaling_workload(n=n, dup_frac=0.1, seed=inputs.SEED_BASE + 1)
    ora = oracle_flags(seq)
    members = seq[ora == 1]
    return {"seq": seq, "d": d, "ora": ora, "digest": set_digest(members),
            "keys": torch.from_numpy(seq.view(np.int64)).cuda(),
            "members": torch.from_numpy(members.view(np.int64)).cuda()}


# (batch, load factor, Cuckoo hash count): the sweep's configurations (c = 4 at
# load factor 0.9) and the headline step's (batches of 2^20, LF 0.7, c = 4)
W2_CONFIGS = [(batch, lf, 4 if lf > 0.85 else 3) for lf in (0.5, 0.7, 0.9)
              for batch in (1 << 16, 1 << 20, 1 << 24)] + [(1 << 20, 0.7, 4)]


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", {})])
@pytest.mark.parametrize("batch,lf,cuckoo_c", W2_CONFIGS)
def test_w2_full_size(w2, kind, kw, batch, lf, cuckoo_c):
    seq, d, n = w2["seq"], w2["d"], w2["seq"].size
    if kind == "bucketed" and cuckoo_c == 4 and lf < 0.85:
        pytest.skip("the bucketed table of this configuration is covered by the c = 3 case")
    print(f"W2 full size: {kind} batch {batch} load factor {lf} c {cuckoo_c}", flush=True)
    nhash = cuckoo_c if kind == "cuckoo" else 3
    keys = w2["keys"]
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t = b.Table(kind, capacity=int(np.ceil(d / lf)), nhash=nhash, max_batch=batch, **kw)
    for s0 in range(0, n, batch):
        t.find_or_put(keys[s0:s0 + batch], out[s0:s0 + batch])
    f = out.cpu().numpy()
    del out
    check_flags_r2_calls(seq, f, w2["ora"], list(range(0, n, batch)) + [n], f"{kind} batch {batch} lf {lf}")
    assert t.size() == d and t.sync_status() == b.HT_OK
    dump = b.u64(t.dump())
    assert set_digest(dump) == w2["digest"], f"{kind} batch {batch} lf {lf}: stored set"
    assert bool(t.query(w2["members"]).all())
    if batch == 1 << 20 and lf == 0.7 and nhash == 3 or (kind == "cuckoo" and nhash == 4 and lf == 0.7):
        q = inputs.query_sequence(1 << 22, d, 0.5, seed=inputs.SEED_BASE + 1)
        present = inputs.key_of_index(np.arange(d), inputs.SEED_BASE + 1)
        exp = Oracle(present).query(q)
        check_query_r1(t.query(torch.from_numpy(q.view(np.int64)).cuda()).cpu().numpy(), exp, f"{kind} queries")
    t.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", {})])
@pytest.mark.parametrize("w", [2, 4])
def test_vectors_full_size_bench_configuration(kind, kw, w):
    """The state-vector bench case: 2^24 vectors, 10% duplicates, batches of
    2^20 at load factor 0.7; every new flag and the stored set checked."""
    from oracle import first_occurrence_flags_vec
    n, batch = 1 << 24, 1 << 20
    d = int(0.9 * n)
    seq = inputs.vector_sequence(n, d, w, seed=inputs.SEED_BASE + 7 + w)
    keys = torch.from_numpy(seq.view(np.int64).reshape(-1)).cuda()
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t = b.Table(kind, capacity=int(np.ceil(d / 0.7)), nhash=3, key_words=w, max_batch=batch, **kw)
    for s0 in range(0, n, batch):
        t.find_or_put(keys[s0 * w:(s0 + batch) * w], out[s0:s0 + batch])
    f = out.cpu().numpy()
    rows = np.ascontiguousarray(seq).view(np.dtype((np.void, 8 * w))).reshape(-1)
    exp = first_occurrence_flags_vec(seq, w)
    # per batch: the rows reported new are the oracle's rows new in that batch
    for s0 in range(0, n, batch):
        g, o = f[s0:s0 + batch], exp[s0:s0 + batch]
        r = rows[s0:s0 + batch]
        assert (np.sort(r[g == 1]) == np.sort(r[o == 1])).all(), s0
    assert set(np.unique(f).tolist()) <= {0, 1}
    assert t.size() == d and t.sync_status() == b.HT_OK
    dump = t.dump().cpu().numpy().view(np.uint64).reshape(-1, w)
    drows = np.ascontiguousarray(dump).view(np.dtype((np.void, 8 * w))).reshape(-1)
    assert drows.size == d and (np.sort(drows) == np.sort(rows[exp == 1])).all()
    t.close()
    del keys, out
    torch.cuda.empty_cache()


# ---- many tables (256 tables of 2^10..2^22 slots, 198 M keys) ---------------------

@pytest.fixture(scope="module")
def w4():
    caps, keys, distinct = inputs.batched_workload()
    with cf.ThreadPoolExecutor(max_workers=_threads()) as ex:
        ora = list(ex.map(lambda k: oracle_flags_seq(k), keys))
    digests = [set_digest(k[o == 1]) for k, o in zip(keys, ora)]
    return caps, keys, distinct, ora, digests


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8, nhash=3)), ("cuckoo", dict(nhash=3))])
def test_w4_full_size_plan(w4, kind, kw):
    """The many-table case at full size in the launch the bench times (one
    plan launch over all 256 tables): every table's flags checked against
    the oracle call by call and its stored set against the oracle's set; the
    many-table query finds every key of every batch and answers fresh keys
    as the oracle does."""
    caps, keys, distinct, ora, digests = w4
    print(f"W4 full size: {kind}", flush=True)
    kd = [torch.from_numpy(k.view(np.int64)).cuda() for k in keys]
    outs = [torch.empty(k.numel(), dtype=torch.uint8, device="cuda") for k in kd]
    tables = [b.Table(kind, capacity=c, max_batch=k.size, **kw) for c, k in zip(caps, keys)]
    plan = b.MultiPlan(tables, kd, outs)
    plan.launch()
    assert plan.status() == b.HT_OK
    for t in range(len(caps)):
        check_flags_r2_calls(keys[t], outs[t].cpu().numpy(), ora[t], [0, keys[t].size], f"table {t}")
        assert tables[t].size() == distinct[t], t
        assert set_digest(b.u64(tables[t].dump())) == digests[t], f"table {t}: stored set"
    found = b.query_multi(tables, kd)
    for t in range(len(caps)):
        assert bool(found[t].all()), t
    fresh = [inputs.uniform_keys(4096, seed=inputs.SEED_BASE + 900 + t) for t in range(len(caps))]
    for t, q in enumerate(fresh):
        m = min(q[::3].size, keys[t].size)      # every third key a member, as far as the batch has keys
        q[: 3 * m: 3] = keys[t][:m]
    got = b.query_multi(tables, [torch.from_numpy(q.view(np.int64)).cuda() for q in fresh])
    for t, (q, g) in enumerate(zip(fresh, got)):
        check_query_r1(g.cpu().numpy(), Oracle(keys[t]).query(q), f"table {t} fresh queries")
    plan.close()
    for t in tables:
        t.close()


# ---- served (64 tables of 2^24 slots, 4,096 requests, 523 M keys) -------------------

@pytest.fixture(scope="module")
def w5():
    """The served trace and the oracle's answer to every request: each table's
    requests applied in arrival order (all released at once: index order) to
    that table's own C++ oracle set, tables on parallel threads."""
    from oracle import c_oracle
    stream = inputs.successor_stream(inputs.BfsModel(1), 1 << 23, start_states=(0, 0x123456789ABCDEF))
    base = inputs.served_trace(4096, 64, 8, 20, rate=0.0, seed=inputs.SEED_BASE + 5, stream=stream)
    by_table = {}
    for i, (_, t, _, _) in enumerate(base):
        by_table.setdefault(t, []).append(i)
    exp = [None] * len(base)
    digests = {}

    def replay(t):
        o = c_oracle.COracle(1)
        for i in by_table[t]:
            op, _, k, _ = base[i]
            exp[i] = o.query(k) if op == "query" else o.find_or_put(k)
        digests[t] = set_digest(o.dump())
        o.close()

    with cf.ThreadPoolExecutor(max_workers=_threads()) as ex:
        list(ex.map(replay, sorted(by_table)))
    return base, exp, digests


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", {})])
def test_w5_full_size_served(w5, kind, kw):
    """The served case at full size through the engine in the bench's
    configuration (16 stream slots, groups of up to 16 requests, every
    request released at once): every request of every table against the
    oracle replay in arrival order -- query flags bit-exact, find-or-put
    flags exact per request -- and every table's stored set against the
    oracle's."""
    base, exp, digests = w5
    print(f"W5 full size: {kind}", flush=True)
    keys = [torch.from_numpy(k.view(np.int64)).pin_memory() for _, _, k, _ in base]
    outs = [torch.empty(k.numel(), dtype=torch.uint8, pin_memory=True) for k in keys]
    tables = [b.Table(kind, capacity=1 << 24, nhash=3, **kw) for _ in range(64)]
    srv = b.Server(tables)
    _, _, _, _, st = srv.run([(op, t, keys[i], 0.0) for i, (op, t, _, _) in enumerate(base)], outs)
    srv.close()
    assert st["merged_launches"] > 0
    for i, (op, t, k, _) in enumerate(base):
        f = outs[i].numpy()
        if op == "query":
            check_query_r1(f, exp[i], f"table {t} request {i}")
        else:
            check_flags_r2_calls(k, f, exp[i], [0, k.size], f"table {t} request {i}")
    for t in sorted(digests):
        assert set_digest(b.u64(tables[t].dump())) == digests[t], f"table {t}: stored set"
    for t in tables:
        t.close()
