"""Pins for the C++ set oracle and the set digest (no GPU).

The C++ oracle (oracle/set_oracle.cpp) is the set definition of find-or-put
(paper Sec. 5) over std::unordered_set, sequential or on hash-partitioned
threads.  It is pinned like the numpy oracle: exhaustive brute force on tiny
inputs against the quadratic list scan, the partitioned form against the
sequential one, and invariants on random inputs.  The digest used to compare
sets too large to store is pinned by its order independence and by the
changes it must detect."""
import itertools

import numpy as np
import pytest

from oracle import set_digest
from paper_1712_09494_amd import inputs

c_oracle = pytest.importorskip("oracle.c_oracle")


@pytest.fixture(scope="module", autouse=True)
def _built():
    c_oracle.build()


ALPHABET = [0, 1, 1 << 63, (1 << 64) - 1]


def scan_new(seq, prior=()):
    prior = list(prior)
    return [0 if (seq[i] in seq[:i] or seq[i] in prior) else 1 for i in range(len(seq))]


@pytest.mark.parametrize("parts", [1, 3])
def test_c_oracle_bruteforce(parts):
    """Every sequence of length <= 6 over 4 keys, split into two calls."""
    for n in range(7):
        for t in itertools.product(ALPHABET, repeat=n):
            seq = list(t)
            cut = n // 2
            o = c_oracle.COracle(parts)
            got = o.find_or_put(np.array(seq[:cut], dtype=np.uint64)).tolist() + \
                o.find_or_put(np.array(seq[cut:], dtype=np.uint64)).tolist()
            assert got == scan_new(seq), (seq, parts)
            assert o.size == len(set(seq))
            assert o.query(np.array(ALPHABET, dtype=np.uint64)).tolist() == [int(a in seq) for a in ALPHABET]
            assert sorted(o.dump().tolist()) == sorted(set(seq))
            o.close()


def test_c_oracle_partitioned_equals_sequential():
    rng = np.random.default_rng(3)
    seq = inputs.key_of_index(rng.integers(0, 50000, size=200000), seed=2)
    seq[::101] = np.uint64((1 << 64) - 1)
    ref = c_oracle.COracle(1)
    flags = [ref.find_or_put(p) for p in np.array_split(seq, 7)]
    for parts in (2, 5, 8):
        o = c_oracle.COracle(parts, reserve=60000)
        got = [o.find_or_put(p) for p in np.array_split(seq, 7)]
        for a, b in zip(got, flags):
            assert np.array_equal(a, b), parts
        assert o.size == ref.size == np.unique(seq).size
        assert np.array_equal(np.sort(o.dump()), np.unique(seq))
        q = inputs.key_of_index(np.arange(49000, 52000), seed=2)
        assert np.array_equal(o.query(q), np.isin(q, seq).astype(np.uint8))


def test_set_digest_order_free_and_sensitive():
    k = inputs.uniform_keys(100000, seed=4)
    d = set_digest(k)
    assert d == set_digest(k[::-1]) == set_digest(np.random.default_rng(1).permutation(k))
    assert d["count"] == k.size
    alt = k.copy()
    alt[5] ^= np.uint64(1)                    # one member changed by one bit
    assert set_digest(alt) != d
    assert set_digest(k[:-1]) != d            # one member dropped
    dup = k.copy()
    dup[7] = dup[8]                           # one member replaced by a copy of another
    assert set_digest(dup)["sum"] != d["sum"] and set_digest(dup)["xor"] != d["xor"]
    assert set_digest(np.zeros(0, dtype=np.uint64)) == {"count": 0, "sum": "0" * 16, "xor": "0" * 16}
