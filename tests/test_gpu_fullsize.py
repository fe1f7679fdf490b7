"""GPU parity at the benchmark's full size, in its launch configuration:
2^26 keys with 10% duplicates, find-or-put in consecutive batches of 2^20 into
a bucketed table (B = 8, c = 3) and a Cuckoo table (c = 3) at load factor 0.7,
batch after batch on the device.  Every flag is checked (the multiset of keys
reported new equals the oracle's), the stored set is checked in full, and
2^22 queries at hit rate 0.5 are checked bit-exact."""
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
