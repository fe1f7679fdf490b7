"""CPU oracle for batched find-or-put and query of 64-bit keys and state vectors.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module; the library path never
does, and this module imports nothing from the library.

What the method computes (paper Sec. 5, the find-or-insert benchmark): every
element of a sequence is looked up in a set; if it is present nothing happens,
otherwise it is inserted.  Both hash tables of Sec. 4 (the Cuckoo table of
Sec. 4.1 and the bucketed GPUexplore table of Sec. 4.2) reach exactly this
result -- they differ only in where a key is stored -- so the oracle is the
plain definition of a set over 64-bit words, applied in index order:

    find_or_put(keys):  is_new[i] = keys[i] not in S;  S = S | {keys[i]}
    query(keys):        found[i]  = keys[i] in S
    size = |S|,  dump = S

Every 64-bit value is a legal key (including the all-ones word that a table
may reserve internally as its empty marker).

State vectors of several words (GPUexplore stores a state as a vector of
words, Sec. 3.2 and 4.2) are keys in the same sense: two vectors are the same
key exactly when all their words are equal.  ``VecLoopOracle`` and
``VecOracle`` apply the same definition to keys given as rows of W words.

Two forms are given:

* ``LoopOracle`` -- the definition itself, a Python ``set`` and a loop over the
  keys in order.  For small inputs.
* ``Oracle`` -- the same definition over numpy arrays.  Within one call the
  i-th key is new exactly when it is absent from S and no earlier key of the
  call equals it, i.e. when i is the first occurrence of its value in the call
  and the value is not in S.  The first occurrences come from ``np.unique``
  (a sort) and membership in S from a binary search of S kept sorted.
"""
from __future__ import annotations

import numpy as np

U64 = np.uint64


class LoopOracle:
    """The set definition, literally: a Python set and a loop in index order."""

    def __init__(self):
        self.s: set[int] = set()

    def find_or_put(self, keys) -> list[int]:
        out = []
        for k in keys:
            k = int(k)
            if k in self.s:
                out.append(0)
            else:
                self.s.add(k)
                out.append(1)
        return out

    def query(self, keys) -> list[int]:
        return [1 if int(k) in self.s else 0 for k in keys]

    @property
    def size(self) -> int:
        return len(self.s)

    def dump(self) -> set[int]:
        return set(self.s)


def _as_u64(keys) -> np.ndarray:
    a = np.asarray(keys)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    return np.ascontiguousarray(a, dtype=np.uint64)


def _member(sorted_set: np.ndarray, keys: np.ndarray) -> np.ndarray:
    """Boolean array: keys[i] in sorted_set (binary search)."""
    if sorted_set.size == 0 or keys.size == 0:
        return np.zeros(keys.shape, dtype=bool)
    pos = np.searchsorted(sorted_set, keys)
    pos_c = np.minimum(pos, sorted_set.size - 1)
    return (pos < sorted_set.size) & (sorted_set[pos_c] == keys)


class Oracle:
    """The set definition over numpy arrays (state: sorted distinct keys)."""

    def __init__(self, initial=None):
        self.keys = np.zeros(0, dtype=U64)
        if initial is not None:
            self.keys = np.unique(_as_u64(initial))

    def find_or_put(self, keys) -> np.ndarray:
        """uint8 flags: 1 where keys[i] was new when its turn came, else 0."""
        k = _as_u64(keys)
        out = np.zeros(k.size, dtype=np.uint8)
        if k.size == 0:
            return out
        uniq, first = np.unique(k, return_index=True)
        absent = ~_member(self.keys, uniq)
        out[first[absent]] = 1
        if absent.any():
            self.keys = np.union1d(self.keys, uniq[absent])
        return out

    def query(self, keys) -> np.ndarray:
        """uint8 flags: 1 where keys[i] is in S."""
        k = _as_u64(keys)
        return _member(self.keys, k).astype(np.uint8)

    @property
    def size(self) -> int:
        return int(self.keys.size)

    def dump(self) -> np.ndarray:
        return self.keys.copy()


def _rows(keys, w: int) -> np.ndarray:
    a = np.asarray(keys)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    return np.ascontiguousarray(a, dtype=np.uint64).reshape(-1, w)


def _void(rows: np.ndarray) -> np.ndarray:
    """One opaque item per row: equal items exactly when all words are equal."""
    w = rows.shape[1]
    return np.ascontiguousarray(rows).view(np.dtype((np.void, 8 * w))).reshape(-1)


class VecLoopOracle:
    """The set definition over vectors of w words: a Python set of tuples."""

    def __init__(self, w: int):
        self.w = w
        self.s: set[tuple] = set()

    def find_or_put(self, keys) -> list[int]:
        out = []
        for row in _rows(keys, self.w).tolist():
            k = tuple(row)
            if k in self.s:
                out.append(0)
            else:
                self.s.add(k)
                out.append(1)
        return out

    def query(self, keys) -> list[int]:
        return [1 if tuple(row) in self.s else 0 for row in _rows(keys, self.w).tolist()]

    @property
    def size(self) -> int:
        return len(self.s)


class VecOracle:
    """The set definition over vectors of w words, with numpy: each row is
    one key; first occurrences within a call from ``np.unique`` over whole
    rows, membership by binary search of the sorted member rows."""

    def __init__(self, w: int, initial=None):
        self.w = w
        self.keys = _void(np.zeros((0, w), dtype=U64))
        if initial is not None:
            self.keys = np.unique(_void(_rows(initial, w)))

    def find_or_put(self, keys) -> np.ndarray:
        v = _void(_rows(keys, self.w))
        out = np.zeros(v.size, dtype=np.uint8)
        if v.size == 0:
            return out
        uniq, first = np.unique(v, return_index=True)
        absent = ~_member(self.keys, uniq)
        out[first[absent]] = 1
        if absent.any():
            self.keys = np.unique(np.concatenate([self.keys, uniq[absent]]))
        return out

    def query(self, keys) -> np.ndarray:
        return _member(self.keys, _void(_rows(keys, self.w))).astype(np.uint8)

    @property
    def size(self) -> int:
        return int(self.keys.size)

    def dump(self) -> np.ndarray:
        """Member vectors as an (n, w) array, rows in byte order."""
        return self.keys.view(U64).reshape(-1, self.w).copy()


def first_occurrence_flags(keys) -> np.ndarray:
    """find_or_put of the whole sequence into an empty set (uint8 flags).

    Applying a sequence batch by batch in order gives the same flags as
    applying it in one call, so this also answers a run of consecutive batches
    starting from an empty set.
    """
    k = _as_u64(keys)
    out = np.zeros(k.size, dtype=np.uint8)
    if k.size:
        _, first = np.unique(k, return_index=True)
        out[first] = 1
    return out


def first_occurrence_flags_vec(keys, w: int) -> np.ndarray:
    """first_occurrence_flags for keys given as rows of w words."""
    v = _void(_rows(keys, w))
    out = np.zeros(v.size, dtype=np.uint8)
    if v.size:
        _, first = np.unique(v, return_index=True)
        out[first] = 1
    return out


def set_digest(keys) -> dict:
    """Order-free fingerprint of a set of 64-bit keys, for comparing sets too
    large to store: the member count, and the sum (mod 2^64) and the xor of
    two multiply-xorshift mixes of every member.  Two sets with equal digests
    are equal with overwhelming probability.  ``keys`` must hold each member
    once (the count is the array length)."""
    k = _as_u64(keys).reshape(-1)
    with np.errstate(over="ignore"):
        a = k * U64(0x9E3779B97F4A7C15)
        a ^= a >> U64(29)
        a *= U64(0xBF58476D1CE4E5B9)
        a ^= a >> U64(32)
        b = (k ^ U64(0x5851F42D4C957F2D)) * U64(0xD6E8FEB86659FD93)
        b ^= b >> U64(31)
        b *= U64(0x94D049BB133111EB)
        b ^= b >> U64(29)
        s = int(np.sum(a, dtype=np.uint64)) if k.size else 0
        x = int(np.bitwise_xor.reduce(b)) if k.size else 0
    return {"count": int(k.size), "sum": f"{s:016x}", "xor": f"{x:016x}"}

