"""GPU structural checks: placement invariants read from the raw slot dump,
the paper's Fig. 2 Cuckoo example replayed with scripted hashes, and the
stash / overflow / rebuild path."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle, first_occurrence_flags  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_dump_r3, check_flags_r2  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
E = b.EMPTY


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def raw(t):
    return b.u64(t.dump_raw())


def positions(r):
    idx = np.flatnonzero(r != E)
    return dict(zip(r[idx].tolist(), idx.tolist()))


@pytest.mark.parametrize("B", [8, 16, 32, 64])
@pytest.mark.parametrize("lf", [0.5, 0.9])
@pytest.mark.parametrize("flags", [0, b.HT_FLAG_BUCKETED_ONE_LANE])
def test_bucketed_prefix_and_spill_order(B, lf, flags):
    """Occupied slots of each bucket form a prefix; a key found in h_j's bucket
    has the buckets of h_1..h_{j-1} full (Sec. 4.2 probe order); with lane
    groups and with one lane per key."""
    n = 20000
    t = b.Table("bucketed", capacity=int(n / lf), nhash=3, bucket_slots=B, flags=flags)
    keys = inputs.uniform_keys(n, seed=B)
    t.find_or_put(dev(keys))
    st = t.stats()
    nb = st["nbuckets"]
    r = raw(t)
    slots = r[: nb * B].reshape(nb, B)
    stash = r[nb * B:]
    occ = slots != E
    # prefix property: no empty slot before an occupied one
    first_empty = np.where((~occ).any(axis=1), (~occ).argmax(axis=1), B)
    assert (occ.sum(axis=1) == first_empty).all()
    full = occ.all(axis=1)
    where = {int(k): i for i, k in enumerate(slots.reshape(-1)) if k != E}
    walk = 64
    for k in keys[:3000].tolist():
        hs = [t.hash_index(k, j) for j in range(3)]
        seq = hs + [(hs[-1] + w) % nb for w in range(1, walk + 1)]
        if k in where:
            bk = where[k] // B
            j = seq.index(bk)
            assert all(full[seq[i]] for i in range(j)), (k, seq[:j + 1], j)
        else:
            assert k in set(stash.tolist())
            assert all(full[h] for h in seq)
    t.close()


@pytest.mark.parametrize("flags", [0, b.HT_FLAG_CUCKOO_PAPER_ORDER, b.HT_FLAG_CUCKOO_LOOKAHEAD])
def test_cuckoo_key_in_candidate_slot_or_stash(flags):
    n = 30000
    t = b.Table("cuckoo", capacity=int(n / 0.85), nhash=3, flags=flags)
    keys = inputs.uniform_keys(n, seed=77)
    t.find_or_put(dev(keys))
    st = t.stats()
    r = raw(t)
    slots = r[: st["capacity"]]
    stash = set(r[st["capacity"]:].tolist()) - {E}
    pos = {int(k): i for i, k in enumerate(slots.tolist()) if k != E}
    assert len(pos) + len(stash) == n
    for k in keys[:5000].tolist():
        hs = [t.hash_index(k, j) for j in range(3)]
        if k in pos:
            assert pos[k] in hs
            # the lookup stops at the first empty slot: every slot before the
            # key's own in h_1, h_2, ... must be taken (distinct indices)
            if len(set(hs)) == 3:
                j = hs.index(pos[k])
                assert all(slots[h] != E for h in hs[:j]), (k, hs, j)
        else:
            assert k in stash
    t.close()


@pytest.mark.parametrize("flags", [0, b.HT_FLAG_CUCKOO_PAPER_ORDER, b.HT_FLAG_CUCKOO_LOOKAHEAD])
def test_cuckoo_coinciding_indices_keep_full_lookup(flags):
    """A key with h_1 == h_3 (c = 4) evicted from that slot skips h_2 and moves
    to h_4 (next hash after the last index mapping to its slot, Sec. 4.1),
    leaving h_2 empty; find-or-put of it again must still find it."""
    y, x, f5, f6, f7 = 1001, 3000, 2005, 2006, 2007
    script = {y: [0, 1, 0, 2], f5: [5, 8, 9, 10], f6: [6, 11, 12, 13], f7: [7, 14, 15, 16],
              x: [0, 5, 6, 7]}
    t = b.Table("cuckoo", capacity=64, nhash=4, flags=flags | b.HT_FLAG_SCRIPTED_HASH)
    t.set_scripted_hash(script)

    def fop(ks):
        return b.u64(t.find_or_put(dev(np.array(ks, dtype=np.uint64))).to(torch.int64)).tolist()

    assert fop([y]) == [1]
    assert fop([f5, f6, f7]) == [1, 1, 1]
    assert fop([x]) == [1]
    r = raw(t)[:64]
    assert positions(r) == {x: 0, y: 2, f5: 5, f6: 6, f7: 7}
    assert r[1] == E
    assert fop([y, y, x]) == [0, 0, 0]
    assert b.u64(t.query(dev(np.array([y, x, 4242], dtype=np.uint64))).to(torch.int64)).tolist() == [1, 1, 0]
    assert t.size() == 5 and positions(raw(t)[:64]) == {x: 0, y: 2, f5: 5, f6: 6, f7: 7}
    t.close()


def test_paper_fig2_replay():
    """Sec. 4.1, Fig. 2: 18 evicts 26 from 26's h2 slot; 26 moves to its h3 slot."""
    with open(os.path.join(GOLDEN, "paper_fig2_cuckoo.json")) as f:
        g = json.load(f)
    t = b.Table("cuckoo", capacity=g["nslots"], nhash=g["nhash"],
                flags=b.HT_FLAG_CUCKOO_PAPER_ORDER | b.HT_FLAG_SCRIPTED_HASH)
    t.set_scripted_hash({int(k): v for k, v in g["hashes"].items()})

    def layout():
        r = raw(t)[: g["nslots"]]
        return {int(k): i for i, k in enumerate(r.tolist()) if k != E}

    for k in g["insert_order"]:
        if k == 18:
            assert layout() == {int(a): v for a, v in g["expected_before_18"].items()}
            ev0 = t.stats()["evictions"]
        f = b.u64(t.find_or_put(dev(np.array([k], dtype=np.uint64))).to(torch.int64))
        assert int(f[0]) == 1
    assert layout() == {int(a): v for a, v in g["expected_after_18"].items()}
    assert t.stats()["evictions"] - ev0 == g["expected_evictions_inserting_18"]
    t.close()


@pytest.mark.parametrize("kind,B", [("bucketed", 8), ("cuckoo", 0)])
def test_stash_overflow_and_rebuild(kind, B):
    """A table far too small: keys go to the stash, then the overflow list;
    no key is lost, queries still find them, and a rebuild restores the table."""
    kw = dict(bucket_slots=B, flags=b.HT_FLAG_BUCKETED_PAPER_FULL) if B else {}
    t = b.Table(kind, capacity=64, nhash=1, stash_slots=16, overflow_slots=4096, **kw)
    keys = inputs.uniform_keys(500, seed=3)
    keys = np.concatenate([keys, keys[:100]])           # duplicates too
    f = b.u64(t.find_or_put(dev(keys)).to(torch.int64)).astype(np.uint8)
    assert set(np.unique(f).tolist()) <= {0, 1, 2}
    assert t.sync_status() == b.HT_EFULL
    st = t.stats()
    assert st["stash_count"] == 16 and st["overflow_count"] > 0 and st["lost"] == 0
    q = b.u64(t.query(dev(keys)).to(torch.int64))
    assert q.all()
    assert t.size() == 500
    t.rebuild(new_capacity=1 << 16)
    assert t.sync_status() == b.HT_OK
    assert t.size() == 500
    assert b.u64(t.query(dev(keys)).to(torch.int64)).all()
    check_dump_r3(b.u64(t.dump()), np.unique(keys), t.size(), kind)
    o = Oracle(keys)
    more = inputs.uniform_keys(1000, seed=4)
    check_flags_r2(more, b.u64(t.find_or_put(dev(more)).to(torch.int64)).astype(np.uint8),
                   o.find_or_put(more), "after rebuild")
    t.close()


@pytest.mark.parametrize("kind,B", [("bucketed", 16), ("cuckoo", 0)])
def test_rebuild_that_fails_leaves_the_table_as_it_was(kind, B):
    """Sec. 4.1's rebuild may fail: a growth the device cannot allocate
    (hipMalloc returns an error) gives HT_ENOMEM, and a rebuild that cannot
    place every member in slots and stash gives HT_EFULL.  Either way the
    table keeps every member (overflow list included), its hash constants and
    its answers; a rebuild that can succeed afterwards does."""
    kw = dict(bucket_slots=B, flags=b.HT_FLAG_BUCKETED_PAPER_FULL) if B else {}
    t = b.Table(kind, capacity=64, nhash=1, stash_slots=16, overflow_slots=4096, **kw)
    keys = inputs.uniform_keys(500, seed=5)
    t.find_or_put(dev(keys))
    before = t.stats()
    dump0 = np.sort(b.u64(t.dump()))
    raw0 = b.u64(t.dump_raw())
    assert before["overflow_count"] > 0 and before["lost"] == 0 and t.size() == 500

    def unchanged(what):
        assert t.sync_status() == b.HT_EFULL, what
        st = t.stats()
        for k in ("size", "capacity", "stash_count", "overflow_count", "lost", "seed"):
            assert st[k] == before[k], (what, k)
        assert np.array_equal(np.sort(b.u64(t.dump())), dump0), what
        assert np.array_equal(b.u64(t.dump_raw()), raw0), what
        assert b.u64(t.query(dev(keys)).to(torch.int64)).all(), what
        absent = inputs.key_of_index(np.arange(10 ** 6, 10 ** 6 + 300), seed=5)   # indices never inserted
        assert not b.u64(t.query(dev(absent)).to(torch.int64)).any(), what

    with pytest.raises(b.HtError) as e:
        t.rebuild(new_capacity=1 << 39)          # 4 TiB of slots: the allocation fails
    assert e.value.code == b.HT_ENOMEM
    unchanged("after the failed growth")
    with pytest.raises(b.HtError) as e:
        t.rebuild()                              # 500 keys cannot fit 64 slots and 16 stash slots
    assert e.value.code == b.HT_EFULL
    unchanged("after the failed rebuild in place")
    with pytest.raises(b.HtError) as e:
        t.rebuild(new_capacity=(1 << 40) + 1)
    assert e.value.code == b.HT_EINVAL
    unchanged("after the rejected capacity")
    t.rebuild(new_capacity=1 << 16)            # c = 1: room for 500 keys with few collisions
    assert t.sync_status() == b.HT_OK and t.size() == 500
    check_dump_r3(b.u64(t.dump()), np.unique(keys), t.size(), kind)
    t.close()


@pytest.mark.parametrize("lf", [0.7, 0.85])
def test_chain_histogram_accounts_for_every_eviction(lf):
    """With the chain-stats flag every eviction chain of the plain Sec. 4.1
    chain is counted once: a chain placed after k exchanges evicted k - 1
    keys, one that reached the stash evicted max_chain, so the histogram sums
    to the table's eviction counter; with the lookahead flag the chains are
    counted too and the table stays exact."""
    n = 200000
    keys = inputs.uniform_keys(n, seed=31)
    for flags in (0, b.HT_FLAG_CUCKOO_LOOKAHEAD):
        t = b.Table("cuckoo", capacity=int(n / lf), nhash=3, max_chain=40, stash_slots=4096,
                    flags=flags | b.HT_FLAG_CHAIN_STATS)
        for s0 in range(0, n, 1 << 14):
            t.find_or_put(dev(keys[s0:s0 + (1 << 14)]))
        h = b.ht_chain_histogram(t.handle)
        st = t.stats()
        assert h["chains"] > 0 and h["counts"][0] == 0 and t.size() == n
        if flags == 0:
            assert h["counts"][63] == 0
            assert sum((i - 1) * c for i, c in enumerate(h["counts"]) if i) + 40 * h["stash"] == st["evictions"]
        t.clear()
        assert b.ht_chain_histogram(t.handle)["chains"] == 0
        t.close()
    with pytest.raises(b.HtError):
        b.Table("cuckoo", capacity=1024, flags=b.HT_FLAG_CUCKOO_LOOKAHEAD | b.HT_FLAG_CUCKOO_PAPER_ORDER)


def test_large_capacity_no_spill():
    """Very large capacity: every key lands in its first bucket / first slot."""
    keys = inputs.uniform_keys(4000, seed=12)
    t = b.Table("bucketed", capacity=1 << 22, nhash=3, bucket_slots=16)
    t.find_or_put(dev(keys))
    pos = positions(raw(t))
    assert all(pos[k] // 16 == t.hash_index(k, 0) for k in keys.tolist())
    t.close()
    t = b.Table("cuckoo", capacity=1 << 22, nhash=3)
    t.find_or_put(dev(keys))
    pos = positions(raw(t))
    hits0 = sum(pos[k] == t.hash_index(k, 0) for k in keys.tolist())
    assert hits0 >= 3990 and t.stats()["evictions"] == 0
    t.close()


def stored_entries(t):
    """Keys held in slots and stash, counted with repetition."""
    r = raw(t)
    return r[r != E]


@pytest.mark.parametrize("lf", [0.5, 0.8])
def test_cuckoo_single_pass_exact_without_repeats(lf):
    """The paper's single-pass insertion (ablation flag) is exact when no key
    repeats within a batch: every key new once, stored once."""
    n = 200000
    keys = inputs.uniform_keys(n, seed=31)
    t = b.Table("cuckoo", capacity=int(n / lf), nhash=3, flags=b.HT_FLAG_CUCKOO_SINGLE_PASS)
    o = Oracle()
    for part in np.array_split(keys, 4):
        check_flags_r2(part, b.u64(t.find_or_put(dev(part)).to(torch.int64)).astype(np.uint8),
                       o.find_or_put(part), f"single pass lf={lf}")
    s = stored_entries(t)
    assert s.size == np.unique(s).size == n
    again = b.u64(t.find_or_put(dev(keys)).to(torch.int64))
    assert not again.any()
    t.close()


def test_cuckoo_single_pass_with_repeats_keeps_every_key():
    """With repeated keys the single pass may store a key twice and report it
    new more than once, but never loses a key, and every distinct new key is
    reported new at least once.  The three-kernel insertion on the same input
    stores each key once."""
    n, d = 400000, 100000
    keys = inputs.random_sequence(n, d, seed=32)
    sp = b.Table("cuckoo", capacity=int(d / 0.8), nhash=3, flags=b.HT_FLAG_CUCKOO_SINGLE_PASS)
    ex = b.Table("cuckoo", capacity=int(d / 0.8), nhash=3)
    f = b.u64(sp.find_or_put(dev(keys)).to(torch.int64)).astype(np.uint8)
    assert set(np.unique(f).tolist()) <= {0, 1}
    assert b.u64(sp.query(dev(keys)).to(torch.int64)).all()
    new_keys = np.unique(keys[f == 1])
    assert new_keys.size == d
    s = stored_entries(sp)
    assert np.unique(s).size == d and s.size >= d
    fe = b.u64(ex.find_or_put(dev(keys)).to(torch.int64)).astype(np.uint8)
    check_flags_r2(keys, fe, first_occurrence_flags(keys), "three kernels")
    se = stored_entries(ex)
    assert se.size == np.unique(se).size == d
    sp.close()
    ex.close()
