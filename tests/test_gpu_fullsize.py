"""GPU parity at the benchmark's full sizes, in its launch configurations.

Random-key scaling: 2^26 keys with 10% duplicates, find-or-put in
consecutive batches of 2^20 into a bucketed table (B = 8, c = 3) and a Cuckoo
table (c = 3) at load factor 0.7, batch after batch on the device.  Every
flag is checked (the multiset of keys reported new equals the oracle's), the
stored set is checked in full, and 2^22 queries at hit rate 0.5 are checked
bit-exact.  Also the state-vector case, the many-table case (one plan launch
over 256 tables) and the served case (4,096 requests through the engine)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import first_occurrence_flags  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_dump_r3, check_flags_r2, check_query_r1  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w2():
    n = 1 << 26
    seq, d = inputs.scaling_workload(n=n, dup_frac=0.1, seed=inputs.SEED_BASE + 1)
    return seq, d, first_occurrence_flags(seq), inputs.key_of_index(np.arange(d), inputs.SEED_BASE + 1)


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", {})])
def test_w2_full_size_bench_configuration(w2, kind, kw):
    seq, d, ora, present = w2
    n, batch = seq.size, 1 << 20
    keys = torch.from_numpy(seq.view(np.int64)).cuda()
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t = b.Table(kind, capacity=int(np.ceil(d / 0.7)), nhash=3, max_batch=batch, **kw)
    for s0 in range(0, n, batch):
        t.find_or_put(keys[s0:s0 + batch], out[s0:s0 + batch])
    f = out.cpu().numpy()
    del keys, out
    check_flags_r2(seq, f, ora, f"{kind} W2 full size")
    assert t.size() == d and t.sync_status() == b.HT_OK
    q = inputs.query_sequence(1 << 22, d, 0.5, seed=inputs.SEED_BASE + 1)
    check_query_r1(t.query(torch.from_numpy(q.view(np.int64)).cuda()).cpu().numpy(),
                   np.isin(q, present).astype(np.uint8), f"{kind} W2 queries")
    check_dump_r3(b.u64(t.dump()), present, t.size(), kind)
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
    assert (np.sort(rows[f == 1]) == np.sort(rows[exp == 1])).all()
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
    return inputs.batched_workload()


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8, nhash=3)), ("cuckoo", dict(nhash=3))])
def test_w4_full_size_plan(w4, kind, kw):
    """The many-table case at full size in the launch the bench times (one
    plan launch over all 256 tables): every table's size and new-flag count
    equal its distinct keys; 17 tables (every 16th and the largest) checked
    flag by flag and member by member against the oracle; the many-table
    query finds every key of every batch, and on the sampled tables answers
    fresh keys as the oracle does."""
    from oracle import Oracle
    caps, keys, distinct = w4
    kd = [torch.from_numpy(k.view(np.int64)).cuda() for k in keys]
    outs = [torch.empty(k.numel(), dtype=torch.uint8, device="cuda") for k in kd]
    tables = [b.Table(kind, capacity=c, max_batch=k.size, **kw) for c, k in zip(caps, keys)]
    plan = b.MultiPlan(tables, kd, outs)
    plan.launch()
    assert plan.status() == b.HT_OK
    sample = sorted(set(range(0, len(caps), 16)) | {int(np.argmax(caps))})
    for t in range(len(caps)):
        assert tables[t].size() == distinct[t], t
        assert int(outs[t].sum(dtype=torch.int64).item()) == distinct[t], t
        if t in sample:
            check_flags_r2(keys[t], outs[t].cpu().numpy(), first_occurrence_flags(keys[t]), f"table {t}")
            check_dump_r3(b.u64(tables[t].dump()), np.unique(keys[t]), tables[t].size(), f"table {t}")
    found = b.query_multi(tables, kd)
    for t in range(len(caps)):
        assert bool(found[t].all()), t
    fresh = [inputs.uniform_keys(4096, seed=inputs.SEED_BASE + 900 + t) for t in sample]
    for t, q in zip(sample, fresh):
        q[::3] = keys[t][: q[::3].size]
    got = b.query_multi([tables[t] for t in sample], [torch.from_numpy(q.view(np.int64)).cuda() for q in fresh])
    for t, q, g in zip(sample, fresh, got):
        check_query_r1(g.cpu().numpy(), Oracle(keys[t]).query(q), f"table {t} fresh queries")
    plan.close()
    for t in tables:
        t.close()


# ---- served (64 tables of 2^24 slots, 4,096 requests, 523 M keys) -------------------

@pytest.fixture(scope="module")
def w5():
    stream = inputs.successor_stream(inputs.BfsModel(1), 1 << 23, start_states=(0, 0x123456789ABCDEF))
    return inputs.served_trace(4096, 64, 8, 20, rate=0.0, seed=inputs.SEED_BASE + 5, stream=stream)


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", {})])
def test_w5_full_size_served(w5, kind, kw):
    """The served case at full size through the engine in the bench's
    configuration (16 stream slots, groups of up to 16 requests, every
    request released at once): the four tables with the most requests are
    replayed through the oracle in their arrival order; every query flag is
    bit-exact, every find-or-put exact in set semantics, and their stored sets
    equal the oracle's."""
    from oracle import Oracle
    base = w5
    keys = [torch.from_numpy(k.view(np.int64)).pin_memory() for _, _, k, _ in base]
    outs = [torch.empty(k.numel(), dtype=torch.uint8, pin_memory=True) for k in keys]
    tables = [b.Table(kind, capacity=1 << 24, nhash=3, **kw) for _ in range(64)]
    srv = b.Server(tables)
    _, _, _, _, st = srv.run([(op, t, keys[i], 0.0) for i, (op, t, _, _) in enumerate(base)], outs)
    srv.close()
    assert st["merged_launches"] > 0
    by_table = {}
    for i, (_, t, _, _) in enumerate(base):
        by_table.setdefault(t, []).append(i)
    for t in sorted(by_table, key=lambda x: -len(by_table[x]))[:4]:
        o = Oracle()
        for i in by_table[t]:                  # released together: arrival order is index order
            op, _, k, _ = base[i]
            f = outs[i].numpy()
            if op == "query":
                check_query_r1(f, o.query(k), f"table {t} request {i}")
            else:
                check_flags_r2(k, f, o.find_or_put(k), f"table {t} request {i}")
        check_dump_r3(b.u64(tables[t].dump()), o.dump(), tables[t].size(), f"table {t}")
    for t in tables:
        t.close()
