"""GPU: calls on different tables are independent, also when several host
threads drive them at once on streams of their own (the library keeps no
shared per-call state: its error text is per thread, its scratch per table)."""
import threading

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import Oracle  # noqa: E402
from paper_1712_09494_amd import binding as b  # noqa: E402
from paper_1712_09494_amd import inputs  # noqa: E402
from parity import check_flags_r2, check_query_r1  # noqa: E402

pytestmark = pytest.mark.gpu

SPECS = [("bucketed", dict(bucket_slots=8)), ("cuckoo", dict()), ("bucketed", dict(bucket_slots=16)),
         ("cuckoo", dict(nhash=4)), ("bucketed", dict(bucket_slots=8, flags=b.HT_FLAG_BUCKETED_ONE_LANE)),
         ("cuckoo", dict(flags=b.HT_FLAG_CUCKOO_PAPER_ORDER))]


def test_threads_on_their_own_tables_and_streams():
    nthreads, nbatch = len(SPECS), 12
    seqs = [inputs.random_sequence(nbatch * 20000, nbatch * 13000, seed=500 + i) for i in range(nthreads)]
    qs = [inputs.query_sequence(30000, nbatch * 13000, 0.5, seed=500 + i, query_seed=600 + i)
          for i in range(nthreads)]
    results = [None] * nthreads
    errors = []
    barrier = threading.Barrier(nthreads)

    def work(i):
        try:
            kind, kw = SPECS[i][0], dict(SPECS[i][1])
            s = torch.cuda.Stream()
            with torch.cuda.stream(s), b.Table(kind, capacity=nbatch * 13000 * 2, nhash=kw.pop("nhash", 3),
                                               **kw) as t:
                keys = torch.from_numpy(seqs[i].view(np.int64)).cuda()
                q = torch.from_numpy(qs[i].view(np.int64)).cuda()
                torch.cuda.current_stream().synchronize()
                barrier.wait()
                flags = []
                for j in range(nbatch):
                    flags.append(t.find_or_put(keys[j * 20000:(j + 1) * 20000], stream=s))
                    if j == nbatch // 2:
                        half = t.query(q, stream=s)
                found = t.query(q, stream=s)
                s.synchronize()
                results[i] = ([f.cpu().numpy() for f in flags], half.cpu().numpy(), found.cpu().numpy(), t.size())
        except Exception as e:          # reported on the main thread
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(nthreads)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for i in range(nthreads):
        flags, half, found, size = results[i]
        o = Oracle()
        for j in range(nbatch):
            part = seqs[i][j * 20000:(j + 1) * 20000]
            check_flags_r2(part, flags[j], o.find_or_put(part), f"thread {i} batch {j}")
            if j == nbatch // 2:
                check_query_r1(half, o.query(qs[i]), f"thread {i} mid-run queries")
        check_query_r1(found, o.query(qs[i]), f"thread {i} queries")
        assert size == o.size, i


@pytest.mark.parametrize("kind,kw", [("bucketed", dict(bucket_slots=8)), ("cuckoo", dict())])
@pytest.mark.parametrize("raw_handle", [False, True])
def test_stream_argument_without_entering_the_stream(kind, kw, raw_handle):
    """stream= given without making it current: the binding copies the
    numpy keys and allocates the flags on that stream, ordered with the
    kernels, while torch's current stream is busy with other work."""
    s = torch.cuda.Stream()
    arg = s.cuda_stream if raw_handle else s
    seq = inputs.random_sequence(8 * 50000, 300000, seed=77)
    q = inputs.query_sequence(40000, 300000, 0.5, seed=77, query_seed=78)
    big = torch.randn(4096, 4096, device="cuda")
    with b.Table(kind, capacity=1 << 20, nhash=3, **kw) as t:
        t.clear(stream=arg)
        o = Oracle()
        flags = []
        for j in range(8):
            big = big @ big * 1e-3                 # keeps torch's current stream busy
            flags.append(t.find_or_put(seq[j * 50000:(j + 1) * 50000], stream=arg))
        found = t.query(q, stream=arg)
        s.synchronize()
        for j in range(8):
            part = seq[j * 50000:(j + 1) * 50000]
            check_flags_r2(part, flags[j].cpu().numpy(), o.find_or_put(part), f"batch {j}")
        check_query_r1(found.cpu().numpy(), o.query(q), "queries")
        assert t.size(stream=arg) == o.size
    torch.cuda.synchronize()
