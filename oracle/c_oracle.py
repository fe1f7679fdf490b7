"""ctypes binding of the C++ set oracle (set_oracle.cpp -> liboracle.so).

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU
baseline).  The same set definition as ``set_oracle.Oracle``, as a
``std::unordered_set<uint64_t>`` walked in index order; ``parts > 1`` runs
it on that many threads over hash-partitioned sets, which gives the same
flags as the sequential loop (every occurrence of a key goes to one thread,
in index order).

    python -m oracle.c_oracle        # build liboracle.so with g++
"""
from __future__ import annotations

import ctypes as C
import os
import shutil
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "set_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with the host compiler (always recompiles)."""
    cxx = os.environ.get("CXX") or shutil.which("g++") or "g++"
    tmp = LIB + ".tmp"
    cmd = [cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-Wall", "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("building liboracle.so failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def load() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is not built; run `python -m oracle.c_oracle`")
        lib = C.CDLL(LIB)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        lib.oracle_new.restype = vp
        lib.oracle_new.argtypes = [u32, u64]
        lib.oracle_free.restype = None
        lib.oracle_free.argtypes = [vp]
        lib.oracle_find_or_put.restype = None
        lib.oracle_find_or_put.argtypes = [vp, vp, u64, vp]
        lib.oracle_query.restype = None
        lib.oracle_query.argtypes = [vp, vp, u64, vp]
        lib.oracle_size.restype = u64
        lib.oracle_size.argtypes = [vp]
        lib.oracle_dump.restype = u64
        lib.oracle_dump.argtypes = [vp, vp, u64]
        _lib = lib
    return _lib


def _keys(keys) -> np.ndarray:
    a = np.asarray(keys)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    return np.ascontiguousarray(a, dtype=np.uint64)


class COracle:
    """The set definition in C++; ``parts`` threads over hash-partitioned sets."""

    def __init__(self, parts: int = 1, reserve: int = 0):
        self.parts = max(1, int(parts))
        self.h = load().oracle_new(self.parts, int(reserve))

    def find_or_put(self, keys, out: np.ndarray | None = None, want_flags: bool = True) -> np.ndarray | None:
        """Flags (uint8) of keys in index order; written into ``out`` (a
        contiguous uint8 array of len(keys)) when given."""
        k = _keys(keys)
        if out is not None:
            if out.dtype != np.uint8 or out.size != k.size or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous uint8 array with one entry per key")
        elif want_flags:
            out = np.zeros(k.size, dtype=np.uint8)
        load().oracle_find_or_put(self.h, k.ctypes.data, k.size, None if out is None else out.ctypes.data)
        return out

    def query(self, keys) -> np.ndarray:
        k = _keys(keys)
        out = np.zeros(k.size, dtype=np.uint8)
        load().oracle_query(self.h, k.ctypes.data, k.size, out.ctypes.data)
        return out

    @property
    def size(self) -> int:
        return int(load().oracle_size(self.h))

    def dump(self) -> np.ndarray:
        n = self.size
        out = np.zeros(n, dtype=np.uint64)
        load().oracle_dump(self.h, out.ctypes.data, n)
        return out

    def close(self) -> None:
        if self.h:
            load().oracle_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


if __name__ == "__main__":
    print(build(verbose=True))
