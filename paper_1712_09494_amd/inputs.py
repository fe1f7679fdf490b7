"""Seeded synthetic inputs for the find-or-put / query workloads.

This module only *produces* key sequences. It holds none of the hash-table
arithmetic (no table hash, no set membership): both the GPU path and the CPU
oracle consume what it returns, and neither is imported here.

Workloads (all keys are 64-bit):

* uniform keys  -- ``k_i = fmix64(i ^ seed)``; fmix64 is the MurmurHash3
  64-bit finalizer (Appleby), a bijection on 64-bit words, so distinct indices
  give distinct keys.  The table hash uses a different mixer, so keys and
  table positions are not correlated.
* random scaling sequence -- D distinct keys plus N-D copies of uniformly
  chosen present keys, the whole sequence shuffled by a keyed Feistel
  permutation (a bijection on [0, N), cycle-walked when N is not a power of 4).
* query sets -- a fixed fraction of hits drawn uniformly from the present
  keys, misses drawn from indices never inserted.
* BFS state vectors -- successors of a seeded synthetic concurrent model of
  16 processes with 16 local states each (4 bits per process packed in one
  64-bit word), standing in for the state-space exploration sequences of the
  paper's Sec. 5.2 (the recorded model-checker sequences themselves are not
  available).  The frontier of the next level is the set of *new* states of
  the current batch in first-occurrence order; computing it needs a set,
  which the caller supplies (the oracle in tests, the table on the GPU).

Random draws use the splitmix64 generator (Steele, Lea & Flood 2014):
state += 0x9e3779b97f4a7c15, output = finalizer(state).
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
SEED_BASE = 0x1712094940

_U = np.uint64


def _u(x: int) -> np.uint64:
    return np.uint64(x & M64)


# --------------------------------------------------------------------------
# scalar / vector mixers
# --------------------------------------------------------------------------

def fmix64(x: np.ndarray) -> np.ndarray:
    """MurmurHash3 fmix64 finalizer, vectorised over uint64 (wraps mod 2^64)."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> _U(33)
        z *= _u(0xFF51AFD7ED558CCD)
        z ^= z >> _U(33)
        z *= _u(0xC4CEB9FE1A85EC53)
        z ^= z >> _U(33)
    return z


def _sm_finalize(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _U(30))) * _u(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U(27))) * _u(0x94D049BB133111EB)
        z = z ^ (z >> _U(31))
    return z


def splitmix64_stream(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start..start+n-1 of the splitmix64 stream seeded with ``seed``."""
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        st = _u(seed) + i * _u(GOLDEN)
    return _sm_finalize(st)


class SplitMix64:
    """Sequential splitmix64 generator (used where the draw order matters)."""

    def __init__(self, seed: int):
        self.state = seed & M64

    def next(self) -> int:
        self.state = (self.state + GOLDEN) & M64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        return z ^ (z >> 31)


def uniform_below(r: np.ndarray, m: int) -> np.ndarray:
    """Map uniform 64-bit words to [0, m) by taking the high word of r*m."""
    r = np.asarray(r, dtype=np.uint64)
    hi32 = r >> _U(32)
    lo32 = r & _u(0xFFFFFFFF)
    m = int(m)
    if m < (1 << 32):
        # (r * m) >> 64 computed exactly with 32-bit limbs
        mm = _U(m)
        with np.errstate(over="ignore"):
            t = (lo32 * mm) >> _U(32)
            t = hi32 * mm + t
        return t >> _U(32)
    # general case via Python ints (rarely used, small arrays only)
    return np.array([(int(v) * m) >> 64 for v in r], dtype=np.uint64)


# --------------------------------------------------------------------------
# keyed Feistel permutation of [0, n)
# --------------------------------------------------------------------------

def feistel_permutation(n: int, seed: int, idx: np.ndarray | None = None) -> np.ndarray:
    """pi(idx) for a seeded pseudo-random bijection pi on [0, n).

    A balanced 4-round Feistel network on 2h bits (2^(2h) >= n) with
    cycle-walking back into [0, n); the round function is multiplicative
    hashing of the right half xor a round key.  Returns uint64 indices.
    """
    if n <= 1:
        m = (n if idx is None else len(idx))
        return np.zeros(m, dtype=np.uint64)
    bits = max(2, int(n - 1).bit_length())
    h = (bits + 1) // 2
    mask = _u((1 << h) - 1)
    keys = [int(k) for k in splitmix64_stream(seed ^ 0x5F3759DF, 4)]
    x = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64).copy()

    # round function: top h bits of (right ^ k_r) * odd multiplier
    mult = _u(0x9FB21C651E98DF25)
    top = _U(64 - h)

    def rounds(v):
        left = v >> _U(h)
        right = v & mask
        for k in keys:
            with np.errstate(over="ignore"):
                f = ((right ^ _u(k)) * mult) >> top
            left, right = right, left ^ f
        return (left << _U(h)) | right

    out = rounds(x)
    bad = out >= _U(n)
    while bad.any():
        out[bad] = rounds(out[bad])
        bad = out >= _U(n)
    return out


# --------------------------------------------------------------------------
# uniform-random workloads
# --------------------------------------------------------------------------

def uniform_keys(n: int, seed: int, start: int = 0) -> np.ndarray:
    """Distinct keys fmix64(i ^ seed) for i in [start, start + n)."""
    i = np.arange(start, start + n, dtype=np.uint64)
    return fmix64(i ^ _u(seed))


def key_of_index(idx: np.ndarray, seed: int) -> np.ndarray:
    return fmix64(np.asarray(idx, dtype=np.uint64) ^ _u(seed))


def random_sequence(n: int, distinct: int, seed: int) -> np.ndarray:
    """Sequence of n keys with exactly ``distinct`` distinct values.

    Indices 0..distinct-1 each appear once; the remaining n-distinct positions
    repeat indices drawn uniformly from [0, distinct); the index sequence is
    then shuffled by a keyed Feistel permutation and mapped to keys.
    """
    assert 0 < distinct <= n
    idx = np.empty(n, dtype=np.uint64)
    idx[:distinct] = np.arange(distinct, dtype=np.uint64)
    if n > distinct:
        r = splitmix64_stream(seed ^ 0xD1B54A32D192ED03, n - distinct)
        idx[distinct:] = uniform_below(r, distinct)
    perm = feistel_permutation(n, seed)
    return key_of_index(idx[perm], seed)


def vector_of_index(idx: np.ndarray, w: int, seed: int, structured: bool = False) -> np.ndarray:
    """(len(idx), w) state vectors, one per index, distinct for distinct indices.

    Random form: word j of vector i is fmix64(i ^ s_j) with per-word seeds.
    Structured form (like packed process states): the index's bits are spread
    over the words a few at a time and every word keeps many zero bits, so
    vectors share most of their words with many others.  Word 0 of the
    structured form carries the low 12 bits, word 1 the next 12, ..., and the
    last word the rest.
    """
    idx = np.asarray(idx, dtype=np.uint64)
    out = np.empty((idx.size, w), dtype=np.uint64)
    if structured:
        rest = idx.copy()
        for j in range(w):
            if j < w - 1:
                part = rest & np.uint64(0xFFF)
                rest = rest >> np.uint64(12)
            else:
                part = rest
            # 4 bits per process slot, 3 of them used: like local states packed in a word
            spread = np.zeros_like(part)
            for b in range(0, 12 if j < w - 1 else 48, 3):
                spread |= ((part >> np.uint64(b)) & np.uint64(7)) << np.uint64(4 * (b // 3))
            out[:, j] = spread ^ np.uint64((seed * 0x9E3779B97F4A7C15 + j) & 0xF0F0F0F0F0F0F0F0)
        return out
    for j in range(w):
        out[:, j] = fmix64(idx ^ _u(seed + 0x9E3779B97F4A7C15 * (j + 1)))
    return out


def vector_sequence(n: int, distinct: int, w: int, seed: int, structured: bool = False) -> np.ndarray:
    """(n, w) sequence of state vectors with exactly ``distinct`` distinct rows
    (same index recipe as random_sequence)."""
    assert 0 < distinct <= n
    idx = np.empty(n, dtype=np.uint64)
    idx[:distinct] = np.arange(distinct, dtype=np.uint64)
    if n > distinct:
        r = splitmix64_stream(seed ^ 0xD1B54A32D192ED03, n - distinct)
        idx[distinct:] = uniform_below(r, distinct)
    perm = feistel_permutation(n, seed)
    return vector_of_index(idx[perm], w, seed, structured)


def query_sequence(n: int, distinct: int, hit_rate: float, seed: int,
                   query_seed: int | None = None) -> np.ndarray:
    """n queries against the key set {key_of_index(i) : i < distinct}.

    round(hit_rate * n) hits are uniform over present indices, the rest are
    fresh indices >= distinct (absent); the result is shuffled.
    """
    qs = seed if query_seed is None else query_seed
    nh = int(round(hit_rate * n))
    idx = np.empty(n, dtype=np.uint64)
    if nh:
        r = splitmix64_stream(qs ^ 0x8CB92BA72F3D8DD7, nh)
        idx[:nh] = uniform_below(r, distinct)
    idx[nh:] = np.arange(distinct, distinct + (n - nh), dtype=np.uint64)
    perm = feistel_permutation(n, qs ^ 0x2545F4914F6CDD1D)
    return key_of_index(idx[perm], seed)


def small_workload(seed: int = SEED_BASE + 0, n: int = 1 << 20):
    """Plain-method small case: n distinct keys, then n queries, 50% present.

    Returns (insert_keys, query_keys).
    """
    ins = uniform_keys(n, seed)
    half = n // 2
    r = splitmix64_stream(seed ^ 0x94D049BB133111EB, half)
    hits = ins[uniform_below(r, n).astype(np.int64)]
    miss = uniform_keys(n - half, seed, start=n)
    q = np.concatenate([hits, miss])
    perm = feistel_permutation(n, seed ^ 0x7F4A7C15).astype(np.int64)
    return ins, q[perm]


def scaling_workload(n: int = 1 << 26, dup_frac: float = 0.1,
                     seed: int = SEED_BASE + 1):
    """Random-key scaling case: n keys with round((1-dup_frac) n) distinct."""
    d = int(round((1.0 - dup_frac) * n))
    return random_sequence(n, d, seed), d


# --------------------------------------------------------------------------
# synthetic concurrent model for BFS state vectors
# --------------------------------------------------------------------------

NPROC = 16
NLOCAL = 16
NSYNC = 4


class BfsModel:
    """Seeded 16-process model; successors of packed 64-bit state vectors.

    Draw order (splitmix64, one stream):
      for p in 0..15, s in 0..15: d = 2 + r%3 local transitions s -> t,
        t = r%16 redrawn while t == s;
      then 4 synchronising actions: p = r%16, q = r%16 redrawn while q == p;
        for s in 0..15: if r%4 == 0 add a p-edge s -> r%16;
                        if r%4 == 0 add a q-edge s -> r%16.
    Successor order of one state: for p = 0..15 each local target in list
    order, then for each synchronising action the product of the p-edges
    and q-edges of the current local states of p and q.
    """

    def __init__(self, seed: int = 1):
        r = SplitMix64(seed)
        self.local = [[None] * NLOCAL for _ in range(NPROC)]
        for p in range(NPROC):
            for s in range(NLOCAL):
                d = 2 + r.next() % 3
                ts = []
                for _ in range(d):
                    t = r.next() % NLOCAL
                    while t == s:
                        t = r.next() % NLOCAL
                    ts.append(t)
                self.local[p][s] = ts
        self.syncs = []
        for _ in range(NSYNC):
            p = r.next() % NPROC
            q = r.next() % NPROC
            while q == p:
                q = r.next() % NPROC
            pe = [[] for _ in range(NLOCAL)]
            qe = [[] for _ in range(NLOCAL)]
            for s in range(NLOCAL):
                if r.next() % 4 == 0:
                    pe[s].append(r.next() % NLOCAL)
                if r.next() % 4 == 0:
                    qe[s].append(r.next() % NLOCAL)
            self.syncs.append((p, q, pe, qe))
        # padded tables for vectorised expansion
        self.max_local = max(len(ts) for row in self.local for ts in row)
        self.tcnt = np.zeros((NPROC, NLOCAL), dtype=np.int64)
        self.ttab = np.zeros((NPROC, NLOCAL, self.max_local), dtype=np.uint64)
        for p in range(NPROC):
            for s in range(NLOCAL):
                ts = self.local[p][s]
                self.tcnt[p, s] = len(ts)
                self.ttab[p, s, :len(ts)] = ts
        self.max_sync = max(max(len(e) for e in pe) * max(len(e) for e in qe)
                            for (_, _, pe, qe) in self.syncs)
        self.width = NPROC * self.max_local + NSYNC * max(1, self.max_sync)

    initial_state = 0

    def successors_py(self, state: int) -> list[int]:
        """Reference expansion of one state (pure Python)."""
        ls = [(state >> (4 * p)) & 15 for p in range(NPROC)]
        out = []
        for p in range(NPROC):
            for t in self.local[p][ls[p]]:
                out.append((state & ~(15 << (4 * p)) & M64) | (t << (4 * p)))
        for (p, q, pe, qe) in self.syncs:
            for tp in pe[ls[p]]:
                for tq in qe[ls[q]]:
                    x = state & ~(15 << (4 * p)) & ~(15 << (4 * q)) & M64
                    out.append(x | (tp << (4 * p)) | (tq << (4 * q)))
        return out

    def successors(self, frontier: np.ndarray, chunk: int = 1 << 20) -> np.ndarray:
        """All successors of ``frontier`` (uint64), concatenated in order."""
        frontier = np.asarray(frontier, dtype=np.uint64)
        parts = []
        for c0 in range(0, len(frontier), chunk):
            parts.append(self._expand(frontier[c0:c0 + chunk]))
        if not parts:
            return np.zeros(0, dtype=np.uint64)
        return np.concatenate(parts)

    def _expand(self, f: np.ndarray) -> np.ndarray:
        nf = len(f)
        cols = []
        valid = []
        ls = [((f >> _U(4 * p)) & _U(15)).astype(np.int64) for p in range(NPROC)]
        for p in range(NPROC):
            cleared = f & ~_u(15 << (4 * p))
            cnt = self.tcnt[p][ls[p]]
            for ti in range(self.max_local):
                t = self.ttab[p, ls[p], ti]
                cols.append(cleared | (t << _U(4 * p)))
                valid.append(cnt > ti)
        for (p, q, pe, qe) in self.syncs:
            cleared = f & ~_u(15 << (4 * p)) & ~_u(15 << (4 * q))
            mp = max(len(e) for e in pe)
            mq = max(len(e) for e in qe)
            pcnt = np.array([len(e) for e in pe], dtype=np.int64)[ls[p]]
            qcnt = np.array([len(e) for e in qe], dtype=np.int64)[ls[q]]
            ptab = np.zeros((NLOCAL, max(mp, 1)), dtype=np.uint64)
            qtab = np.zeros((NLOCAL, max(mq, 1)), dtype=np.uint64)
            for s in range(NLOCAL):
                ptab[s, :len(pe[s])] = pe[s]
                qtab[s, :len(qe[s])] = qe[s]
            for a in range(mp):
                for b in range(mq):
                    cols.append(cleared | (ptab[ls[p], a] << _U(4 * p)) | (qtab[ls[q], b] << _U(4 * q)))
                    valid.append((pcnt > a) & (qcnt > b))
        m = np.stack(cols, axis=1)
        v = np.stack(valid, axis=1)
        return m[v]


# --------------------------------------------------------------------------
# served request traces
# --------------------------------------------------------------------------

def successor_stream(model: "BfsModel", min_keys: int, start_states=(0,)) -> np.ndarray:
    """Successor batches expanded level by level from `start_states` without
    removing duplicates (a state reached along several paths appears several
    times), concatenated until at least `min_keys` keys are produced."""
    out, total = [], 0
    for s0 in start_states:
        frontier = np.array([s0], dtype=np.uint64)
        while total < min_keys and frontier.size:
            batch = model.successors(frontier)
            out.append(batch)
            total += batch.size
            frontier = batch[: max(1, min_keys - total)]
        if total >= min_keys:
            break
    return np.concatenate(out) if out else np.zeros(0, dtype=np.uint64)


def batched_workload(ntables: int = 256, lf: float = 0.6):
    """Many-table workload: `ntables` capacities log-uniform in [2^10, 2^22)
    (splitmix64 stream of seed SEED_BASE + 3), each table with
    floor(lf * cap) distinct keys: even tables random keys (seed SEED_BASE +
    4 + t), odd tables a prefix of one synthetic BFS successor stream
    (16-process model, seed 1, levels 0-4, duplicates included) holding that
    many distinct keys (the stream holds 2,049,037 distinct states, which
    caps the largest BFS tables).  Returns (caps, keys, distinct counts)."""
    r = SplitMix64(SEED_BASE + 3)
    caps = []
    for _ in range(ntables):
        u = 10 + 12 * (r.next() / 2.0 ** 64)
        caps.append(int(round(2 ** u)))
    model = BfsModel(1)
    frontier = np.array([0], dtype=np.uint64)
    parts = []
    seen = np.array([0], dtype=np.uint64)
    for _ in range(5):
        batch = model.successors(frontier)
        parts.append(batch)
        u, first = np.unique(batch, return_index=True)
        new = ~np.isin(u, seen)
        frontier = batch[np.sort(first[new])]
        seen = np.union1d(seen, u[new])
    stream = np.concatenate(parts)
    _, first = np.unique(stream, return_index=True)
    first = np.sort(first)
    keys, distinct = [], []
    for t, cap in enumerate(caps):
        d = max(1, int(lf * cap))
        if t % 2 == 0:
            keys.append(uniform_keys(d, seed=SEED_BASE + 4 + t))
        else:
            d = min(d, first.size)
            keys.append(stream[: int(first[d - 1]) + 1])
        distinct.append(d)
    return caps, keys, distinct


def served_trace(nreq: int, ntables: int, log_min: float = 8, log_max: float = 20, rate: float = 0.0,
                 seed: int = SEED_BASE + 5, bfs_frac: float = 0.7, query_frac: float = 0.5,
                 stream: np.ndarray | None = None):
    """Requests for a served run: list of (op, table, keys, arrival_s).

    Sizes floor(2^U), U uniform in [log_min, log_max]; op is "query" with
    probability query_frac, else "fop"; table uniform; keys: the first
    round(bfs_frac * n) from the table's cursor into a shared successor
    stream (find-or-puts advance the cursor, queries read ahead of it without
    advancing), the rest fresh random keys.  Arrivals are a Poisson process
    of `rate` requests per second (all at 0 when rate is 0).
    """
    r = SplitMix64(seed)
    u01 = lambda: (r.next() >> 11) * (1.0 / (1 << 53))
    if stream is None:
        stream = successor_stream(BfsModel(1), 1 << 22, start_states=(0, 0x123456789ABCDEF))
    ns = max(1, stream.size)
    cursor = [(t * 1000003) % ns for t in range(ntables)]
    fresh = 0
    t_arr = 0.0
    reqs = []
    for i in range(nreq):
        n = int(2.0 ** (log_min + (log_max - log_min) * u01()))
        op = "query" if u01() < query_frac else "fop"
        t = int(u01() * ntables) % ntables
        nb = int(round(bfs_frac * n))
        idx = (cursor[t] + np.arange(nb, dtype=np.int64)) % ns
        bfs = stream[idx]
        if op == "fop":
            cursor[t] = (cursor[t] + nb) % ns
        rnd = uniform_keys(n - nb, seed ^ 0x5EED, start=fresh)
        fresh += n - nb
        keys = np.concatenate([bfs, rnd])
        if rate > 0:
            t_arr += -np.log(max(u01(), 1e-300)) / rate
        reqs.append((op, t, keys, t_arr))
    return reqs
