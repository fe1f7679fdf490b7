"""GPU: the single-table Cuckoo find-or-put leaves the slots its winners took
in its deduplication set, with a record of them, and the next call's probe
kernel empties them (deferred scrub).  A key that finds a slot of the set
still taken by an earlier call would be reported as another copy and never
stored, so these cases refill cleared tables with the same keys: batch sizes
that change the per-wave layout between calls, the many-table and the
allocation-free calls (which use sets of their own) in between, and a
captured call replayed after eager calls that left records of their own.
Every call's flags equal the oracle's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_flags_r2  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def run_calls(t, seq, cuts, ora, what):
    bounds = [0] + list(np.cumsum(cuts))
    assert bounds[-1] == seq.size
    for i in range(len(cuts)):
        piece = seq[bounds[i]:bounds[i + 1]]
        if piece.size:
            got = t.find_or_put(dev(piece)).cpu().numpy()
            check_flags_r2(piece, got, ora.find_or_put(piece), f"{what} call {i} ({piece.size} keys)")


@pytest.mark.parametrize("nhash,lf", [(3, 0.85), (4, 0.9), (2, 0.45)])
def test_refill_with_the_same_keys(nhash, lf):
    d = 150000
    n = d + d // 4
    seq = inputs.random_sequence(n, d, seed=97 + nhash)
    t = b.Table("cuckoo", capacity=int(d / lf), nhash=nhash)
    cuts_a = [d // 3, 5, 63, 1, d // 2, 100003]
    cuts_a.append(n - sum(cuts_a))
    cuts_b = [n - 70000, 0, 4097, 65903]
    for rep, cuts in enumerate([cuts_a, cuts_b, cuts_a[::-1]]):
        t.clear()
        ora = Oracle()
        run_calls(t, seq, cuts, ora, f"nhash {nhash} refill {rep}")
        st = t.stats()
        assert st["size"] == d
        assert st["evictions"] > 0 or nhash == 2     # keys went through the evict kernel
    t.close()


def test_other_paths_in_between():
    d = 120000
    n = d + d // 5
    seq = inputs.random_sequence(n, d, seed=131)
    t = b.Table("cuckoo", capacity=int(d / 0.88), nhash=3)
    other = b.Table("cuckoo", capacity=1 << 16, nhash=3)
    other_keys = inputs.random_sequence(40000, 30000, seed=132)
    q = [0, 50000, 80000, 100000, n]
    for rep in range(2):
        t.clear()
        other.clear()
        ora, ora_other = Oracle(), Oracle()
        # single-table call: leaves its record
        run_calls(t, seq[q[0]:q[1]], [q[1] - q[0]], ora, f"rep {rep} single")
        # many-table call over this table and another one (their own set and scrub)
        outs = b.find_or_put_multi([t, other], [dev(seq[q[1]:q[2]]), dev(other_keys)])
        check_flags_r2(seq[q[1]:q[2]], outs[0].cpu().numpy(), ora.find_or_put(seq[q[1]:q[2]]), f"rep {rep} multi")
        check_flags_r2(other_keys, outs[1].cpu().numpy(), ora_other.find_or_put(other_keys), f"rep {rep} multi other")
        # allocation-free call (the static set)
        piece = seq[q[2]:q[3]]
        out = torch.empty(piece.size, dtype=torch.uint8, device="cuda")
        b.ht_find_or_put_noalloc(t.handle, dev(piece), out)
        check_flags_r2(piece, out.cpu().numpy(), ora.find_or_put(piece), f"rep {rep} noalloc")
        # single-table again, in two calls
        run_calls(t, seq[q[3]:q[4]], [7, q[4] - q[3] - 7], ora, f"rep {rep} single again")
        assert t.size() == d
    t.close()
    other.close()


def test_replay_after_eager_records():
    """A captured clear + find-or-put, replayed after eager calls on the same
    table whose winners include the captured batch's keys."""
    d = 100000
    seq_y = inputs.random_sequence(d + d // 4, d, seed=151)
    x = seq_y[: 60000].copy()
    batch = seq_y.size
    t = b.Table("cuckoo", capacity=int(d / 0.88), nhash=3, max_batch=batch)
    kx = dev(x)
    out = torch.zeros(x.size, dtype=torch.uint8, device="cuda")
    exp_x = Oracle().find_or_put(x)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        t.clear()
        t.find_or_put(kx, out)
    torch.cuda.synchronize()
    check_flags_r2(x, out.cpu().numpy(), exp_x, "eager before capture")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        t.clear()
        t.find_or_put(kx, out)
    torch.cuda.synchronize()
    for rep in range(3):
        # eager: the whole of y on a cleared table (its record names x's keys)
        t.clear()
        got_y = t.find_or_put(dev(seq_y)).cpu().numpy()
        check_flags_r2(seq_y, got_y, Oracle().find_or_put(seq_y), f"eager y {rep}")
        assert t.stats()["evictions"] > 0
        out.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check_flags_r2(x, out.cpu().numpy(), exp_x, f"replay {rep}")
        assert t.size() == np.unique(x).size
    t.close()
