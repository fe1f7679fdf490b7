"""GPU: the plain single-table calls (clear, then find-or-put batch by batch)
captured in a HIP graph and replayed several times, with eager work on the
same table between replays; every replay equals the oracle.  With scratch
reserved up front (max_batch) the calls allocate nothing and use fill
kernels instead of memsets, so they can be captured."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import first_occurrence_flags, first_occurrence_flags_vec  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_flags_r2  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "bucketed": dict(kind="bucketed", bucket_slots=8),
    "cuckoo": dict(kind="cuckoo"),
    "cuckoo_paper": dict(kind="cuckoo", flags=b.HT_FLAG_CUCKOO_PAPER_ORDER),
    "vec2_bucketed": dict(kind="bucketed", bucket_slots=8, key_words=2),
    "vec4_cuckoo": dict(kind="cuckoo", key_words=4),
}


@pytest.mark.parametrize("case", list(CASES))
def test_single_table_calls_in_a_graph(case):
    kw = dict(CASES[case])
    w = kw.get("key_words", 1)
    n, d, batch = 200000, 150000, 1 << 15
    if w == 1:
        seq = inputs.random_sequence(n, d, seed=41)
        exp = first_occurrence_flags(seq)
    else:
        seq = inputs.vector_sequence(n, d, w, seed=41)
        exp = first_occurrence_flags_vec(seq, w)
    keys = torch.from_numpy(np.ascontiguousarray(seq).view(np.int64).reshape(-1)).cuda()
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t = b.Table(capacity=int(d / 0.7), nhash=3, max_batch=batch, **kw)

    def work():
        t.clear()
        for s0 in range(0, n, batch):
            t.find_or_put(keys[s0 * w:min(n, s0 + batch) * w], out[s0:s0 + batch])

    def check(what):
        f = out.cpu().numpy()
        if w == 1:
            check_flags_r2(seq, f, exp, what)
        else:
            rows = np.ascontiguousarray(seq).view(np.dtype((np.void, 8 * w))).reshape(-1)
            assert (np.sort(rows[f == 1]) == np.sort(rows[exp == 1])).all(), what
        assert t.size() == d, what

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        work()                                  # eager on the capture stream first
    torch.cuda.synchronize()
    check("eager")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        work()
    torch.cuda.synchronize()
    probe = keys[: 1000 * w]
    for rep in range(3):
        out.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(f"replay {rep}")
        # eager work on the same table between replays
        assert t.query(probe).all()
        extra = t.find_or_put(probe)
        assert not extra.any()
    t.close()
