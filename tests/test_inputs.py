"""Seeded input generators (no GPU)."""
import numpy as np
import pytest

from paper_1712_09494_amd import inputs


def test_splitmix64_published_vector():
    # first outputs of splitmix64 seeded with 1234567 (reference C implementation)
    exp = [6457827717110365317, 3203168211198807973, 9817491932198370423,
           4593380528125082431, 16408922859458223821]
    r = inputs.SplitMix64(1234567)
    assert [r.next() for _ in range(5)] == exp
    assert inputs.splitmix64_stream(1234567, 5).tolist() == exp
    assert inputs.splitmix64_stream(1234567, 2, start=3).tolist() == exp[3:5]


def _fmix64_inverse(z):
    """Inverse of the MurmurHash3 finalizer (xorshift and odd-multiplier inverses)."""
    M = (1 << 64) - 1

    def unxorshift(v, s):
        x = v
        for _ in range(64 // s + 1):
            x = v ^ (x >> s)
        return x & M

    z = unxorshift(z, 33)
    z = (z * pow(0xC4CEB9FE1A85EC53, -1, 1 << 64)) & M
    z = unxorshift(z, 33)
    z = (z * pow(0xFF51AFD7ED558CCD, -1, 1 << 64)) & M
    return unxorshift(z, 33)


def test_fmix64_bijection():
    x = np.array([0, 1, 2, 12345, (1 << 64) - 1, 1 << 63], dtype=np.uint64)
    z = inputs.fmix64(x)
    assert [_fmix64_inverse(int(v)) for v in z] == x.tolist()
    keys = inputs.uniform_keys(1 << 18, seed=3)
    assert np.unique(keys).size == keys.size


@pytest.mark.parametrize("n", [1, 2, 3, 17, 1000, 4096, 65537])
def test_feistel_is_permutation(n):
    p = inputs.feistel_permutation(n, seed=99)
    assert p.size == n
    assert np.array_equal(np.sort(p), np.arange(n, dtype=np.uint64))


def test_uniform_below_range():
    r = inputs.splitmix64_stream(5, 100000)
    for m in (1, 3, 1000, 60397978, (1 << 32) - 1):
        v = inputs.uniform_below(r, m)
        assert int(v.max()) < m
    v = inputs.uniform_below(np.array([(1 << 64) - 1], dtype=np.uint64), 10)
    assert int(v[0]) == 9


def test_random_sequence_shape():
    seq = inputs.random_sequence(100000, 90000, seed=4)
    assert seq.size == 100000
    assert np.unique(seq).size == 90000
    # duplicates spread over the sequence (not all at the tail)
    _, first = np.unique(seq, return_index=True)
    later = np.setdiff1d(np.arange(seq.size), first)
    assert later.min() < 50000


def test_scaling_workload_counts_small():
    seq, d = inputs.scaling_workload(n=1 << 16, dup_frac=0.1, seed=8)
    assert d == round(0.9 * (1 << 16))
    assert np.unique(seq).size == d


@pytest.mark.parametrize("h", [0.0, 0.5, 1.0])
def test_query_sequence_hit_rate(h):
    n, d = 20000, 15000
    present = inputs.key_of_index(np.arange(d), seed=6)
    q = inputs.query_sequence(n, d, h, seed=6)
    hits = np.isin(q, present).sum()
    assert hits == round(h * n)


def test_small_workload():
    ins, q = inputs.small_workload(n=1 << 12)
    assert np.unique(ins).size == ins.size
    assert np.isin(q, ins).sum() == (1 << 11)


def test_bfs_vectorised_matches_reference():
    m = inputs.BfsModel(1)
    rng = np.random.default_rng(3)
    states = rng.integers(0, 1 << 63, size=300, dtype=np.int64).astype(np.uint64)
    states = np.concatenate([states, np.array([0, (1 << 64) - 1], dtype=np.uint64)])
    vec = m.successors(states, chunk=64)
    ref = [s for st in states.tolist() for s in m.successors_py(st)]
    assert vec.tolist() == ref


def test_bfs_model_shape():
    m = inputs.BfsModel(2)
    for p in range(16):
        for s in range(16):
            ts = m.local[p][s]
            assert 2 <= len(ts) <= 4 and s not in ts
    assert len(m.syncs) == 4
    for (p, q, pe, qe) in m.syncs:
        assert p != q


def test_served_trace_shape():
    reqs = inputs.served_trace(200, 9, log_min=4, log_max=10, rate=1000.0, seed=3)
    assert len(reqs) == 200
    arr = [a for _, _, _, a in reqs]
    assert arr == sorted(arr) and arr[0] > 0
    for op, t, k, a in reqs:
        assert op in ("fop", "query") and 0 <= t < 9
        assert 16 <= k.size < 1024 and k.dtype == np.uint64
    again = inputs.served_trace(200, 9, log_min=4, log_max=10, rate=1000.0, seed=3)
    assert all(np.array_equal(x[2], y[2]) and x[:2] == y[:2] for x, y in zip(reqs, again))
    ops = [op for op, *_ in reqs]
    assert 60 < ops.count("query") < 140


@pytest.mark.parametrize("structured", [False, True])
@pytest.mark.parametrize("w", [2, 4])
def test_vector_generators(w, structured):
    v = inputs.vector_of_index(np.arange(50000), w, seed=4, structured=structured)
    assert v.shape == (50000, w) and v.dtype == np.uint64
    assert np.unique(v, axis=0).shape[0] == 50000
    seq = inputs.vector_sequence(30000, 25000, w, seed=6, structured=structured)
    assert seq.shape == (30000, w)
    assert np.unique(seq, axis=0).shape[0] == 25000
    if structured:
        # most vectors share their later words with many others
        assert np.unique(v[:, -1]).size < 50000 // 10


def test_batched_workload_shape():
    """The many-table workload: 256 capacities in [2^10, 2^22], each table's
    batch holding exactly its stated number of distinct keys (random tables
    without repeats, BFS tables a stream prefix with repeats)."""
    caps, keys, distinct = inputs.batched_workload()
    assert len(caps) == len(keys) == len(distinct) == 256
    assert all(1 << 10 <= c <= 1 << 22 for c in caps)
    for t in list(range(0, 256, 17)) + [1, 3]:
        assert np.unique(keys[t]).size == distinct[t]
        assert distinct[t] <= max(1, int(0.6 * caps[t]))
        if t % 2 == 0:
            assert keys[t].size == distinct[t]
    assert sum(k.size for k in keys) > sum(distinct)     # the BFS prefixes repeat states
