"""GPU: the allocation-free find-or-put (ht_find_or_put_noalloc) against
ht_find_or_put, through the C ABI: two calls in a row on the same tables, the
second smaller, each call's flags exact against the oracle (set semantics,
per call) for both entry points, and the two tables' stored sets equal to
each other and to the oracle's after each call; sizes above the static
scratch's limit and state-vector tables are rejected."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_dump_r3, check_flags_r2_calls  # noqa: E402

pytestmark = pytest.mark.gpu

MAX = 1 << 18


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


@pytest.mark.parametrize("kind,kw", [("cuckoo", {}), ("cuckoo", dict(flags=b.HT_FLAG_CUCKOO_PAPER_ORDER)),
                                     ("cuckoo", dict(nhash=4)), ("bucketed", dict(bucket_slots=8))])
def test_noalloc_matches_find_or_put(kind, kw):
    kw = dict(kw)
    nhash = kw.pop("nhash", 3)
    seq1 = inputs.random_sequence(MAX, 200000, seed=91)          # the largest batch, with repeats
    seq1[::4099] = np.uint64(b.EMPTY)                            # the all-ones key too
    seq2 = np.concatenate([seq1[:20000], inputs.uniform_keys(30000, seed=92)])   # smaller, half present
    rng = np.random.default_rng(3)
    seq2 = seq2[rng.permutation(seq2.size)]
    cap = int(300000 / 0.7)
    ref = b.Table(kind, capacity=cap, nhash=nhash, seed=5, **kw)
    na = b.Table(kind, capacity=cap, nhash=nhash, seed=5, **kw)
    o = Oracle()
    for i, seq in enumerate((seq1, seq2)):
        k = dev(seq)
        f_ref = ref.find_or_put(k).cpu().numpy()
        out = torch.full((seq.size,), 7, dtype=torch.uint8, device="cuda")
        b.ht_find_or_put_noalloc(na.handle, k, out)
        f_na = out.cpu().numpy()
        exp = o.find_or_put(seq)
        check_flags_r2_calls(seq, f_ref, exp, [0, seq.size], f"{kind} call {i} find_or_put")
        check_flags_r2_calls(seq, f_na, exp, [0, seq.size], f"{kind} call {i} noalloc")
        for t in (ref, na):
            assert t.sync_status() == b.HT_OK
            check_dump_r3(b.u64(t.dump()), o.dump(), t.size(), f"{kind} call {i}")
        q = np.concatenate([seq[:1000], inputs.key_of_index(np.arange(10 ** 7, 10 ** 7 + 1000), seed=93)])
        assert np.array_equal(na.query(dev(q)).cpu().numpy(), o.query(q))
    ref.close()
    na.close()


def test_noalloc_rejects_what_it_cannot_serve():
    with b.Table("cuckoo", capacity=1 << 20) as t:
        k = torch.zeros(MAX + 1, dtype=torch.int64, device="cuda")
        out = torch.zeros(MAX + 1, dtype=torch.uint8, device="cuda")
        with pytest.raises(b.HtError) as e:
            b.ht_find_or_put_noalloc(t.handle, k, out)
        assert e.value.code == b.HT_EINVAL
        assert t.size() == 0
        b.ht_find_or_put_noalloc(t.handle, k[:0], out[:0])       # n = 0: nothing to do
    with b.Table("cuckoo", capacity=1 << 12, key_words=2) as t:
        k = torch.zeros(64, dtype=torch.int64, device="cuda")
        with pytest.raises(b.HtError) as e:
            b.ht_find_or_put_noalloc(t.handle, k, torch.zeros(64, dtype=torch.uint8, device="cuda"))
        assert e.value.code == b.HT_EINVAL
