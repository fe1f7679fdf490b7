"""Thin Python binding over the C ABI of libht.so (include/ht.h).

Argument marshalling only: every step of find-or-put and query runs in the
HIP kernels of libht.so.  Torch tensors supply device memory, and the stream
handle comes from ``torch.cuda.current_stream()`` unless one is given; a
given stream is made current while the call marshals its arguments, so key
copies, flag allocations and kernels are ordered on it.  The
functions ``ht_*`` mirror the C entry points one to one; ``Table`` wraps a
handle with the same calls.

If libht.so is missing the first call raises ``HtLibraryMissing`` -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libht.so")

HT_BUCKETED = 1
HT_CUCKOO = 2

HT_OK = 0
HT_EINVAL = -1
HT_ENOMEM = -2
HT_EFULL = -3
HT_EHIP = -4

HT_FLAG_CUCKOO_PAPER_ORDER = 1 << 0
HT_FLAG_BUCKETED_ATOMIC_LOADS = 1 << 1
HT_FLAG_SCRIPTED_HASH = 1 << 2
HT_FLAG_BUCKETED_PAPER_FULL = 1 << 3
HT_FLAG_CUCKOO_SINGLE_PASS = 1 << 4
HT_FLAG_BUCKETED_ONE_LANE = 1 << 5
HT_FLAG_CHAIN_STATS = 1 << 6
HT_FLAG_CUCKOO_LOOKAHEAD = 1 << 7
HT_FLAG_BUCKETED_GROUP_QUERY = 1 << 8

EMPTY = (1 << 64) - 1

KINDS = {"bucketed": HT_BUCKETED, "cuckoo": HT_CUCKOO}


class HtLibraryMissing(ImportError):
    pass


class HtError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code})" + (f": {detail}" if detail else ""))


class HtConfig(C.Structure):
    _fields_ = [
        ("kind", C.c_uint32),
        ("nhash", C.c_uint32),
        ("capacity", C.c_uint64),
        ("bucket_slots", C.c_uint32),
        ("keys_per_group", C.c_uint32),
        ("stash_slots", C.c_uint32),
        ("max_chain", C.c_uint32),
        ("seed", C.c_uint64),
        ("flags", C.c_uint32),
        ("overflow_slots", C.c_uint32),
        ("max_batch", C.c_uint64),
        ("bucket_walk", C.c_uint32),
        ("lds_bytes", C.c_uint32),
        ("key_words", C.c_uint32),
        ("reserved", C.c_uint32),
    ]


class HtRequest(C.Structure):
    _fields_ = [
        ("op", C.c_uint32),
        ("table", C.c_uint32),
        ("h_keys", C.c_void_p),
        ("n", C.c_uint64),
        ("h_out", C.c_void_p),
        ("arrival_s", C.c_double),
        ("admit_s", C.c_double),
        ("done_s", C.c_double),
        ("slot", C.c_uint32),
        ("group", C.c_uint32),
    ]


class HtServerConfig(C.Structure):
    _fields_ = [
        ("slots", C.c_uint32),
        ("merge", C.c_uint32),
        ("staging_bytes", C.c_uint64),
        ("sequential", C.c_uint32),
        ("reserved", C.c_uint32),
        ("group_keys", C.c_uint64),
    ]


class HtServerStats(C.Structure):
    _fields_ = [
        ("wall_s", C.c_double),
        ("keys", C.c_uint64),
        ("peak_staging", C.c_uint64),
        ("staging_bytes", C.c_uint64),
        ("groups", C.c_uint32),
        ("merged_launches", C.c_uint32),
        ("max_inflight_groups", C.c_uint32),
        ("throttled", C.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class HtBfsModel(C.Structure):
    _fields_ = [
        ("local_count", (C.c_uint8 * 16) * 16),
        ("local_target", ((C.c_uint8 * 4) * 16) * 16),
        ("sync_p", C.c_uint8 * 4),
        ("sync_q", C.c_uint8 * 4),
        ("sync_p_edge", (C.c_int8 * 16) * 4),
        ("sync_q_edge", (C.c_int8 * 16) * 4),
    ]


def pack_bfs_model(model) -> HtBfsModel:
    """ht_bfs_model from a model with .local[p][s] (target lists) and
    .syncs[a] = (p, q, p_edges[s], q_edges[s]) (at most one edge each)."""
    m = HtBfsModel()
    for p in range(16):
        for s in range(16):
            ts = model.local[p][s]
            if len(ts) > 4:
                raise ValueError("at most 4 local transitions")
            m.local_count[p][s] = len(ts)
            for k, t in enumerate(ts):
                m.local_target[p][s][k] = t
    if len(model.syncs) != 4:
        raise ValueError("exactly 4 synchronising actions")
    for a, (sp, sq, pe, qe) in enumerate(model.syncs):
        m.sync_p[a] = sp
        m.sync_q[a] = sq
        for s in range(16):
            if len(pe[s]) > 1 or len(qe[s]) > 1:
                raise ValueError("at most one synchronising edge per local state")
            m.sync_p_edge[a][s] = pe[s][0] if pe[s] else -1
            m.sync_q_edge[a][s] = qe[s][0] if qe[s] else -1
    return m


HT_BFS_SPLIT = 0
HT_BFS_FUSED = 1
HT_OP_FIND_OR_PUT = 1
HT_OP_QUERY = 2


class HtStats(C.Structure):
    _fields_ = [
        ("size", C.c_uint64),
        ("capacity", C.c_uint64),
        ("stash_count", C.c_uint64),
        ("overflow_count", C.c_uint64),
        ("lost", C.c_uint64),
        ("evictions", C.c_uint64),
        ("nbuckets", C.c_uint64),
        ("kind", C.c_uint32),
        ("nhash", C.c_uint32),
        ("bucket_slots", C.c_uint32),
        ("stash_slots", C.c_uint32),
        ("seed", C.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_vp = C.c_void_p
_u64 = C.c_uint64
_u32 = C.c_uint32
_PROTOS = {
    "ht_config_default": (None, [C.POINTER(HtConfig), _u32]),
    "ht_create": (C.c_int, [C.POINTER(HtConfig), C.POINTER(_vp)]),
    "ht_create_simple": (C.c_int, [_u32, _u64, _u32, C.POINTER(_vp)]),
    "ht_destroy": (C.c_int, [_vp]),
    "ht_find_or_put": (C.c_int, [_vp, _vp, _u64, _vp, _vp]),
    "ht_insert": (C.c_int, [_vp, _vp, _u64, _vp, _vp]),
    "ht_find_or_put_noalloc": (C.c_int, [_vp, _vp, _u64, _vp, _vp]),
    "ht_query": (C.c_int, [_vp, _vp, _u64, _vp, _vp]),
    "ht_find_or_put_multi": (C.c_int, [C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_u64), C.POINTER(_vp), _u32, _vp]),
    "ht_query_multi": (C.c_int, [C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_u64), C.POINTER(_vp), _u32, _vp]),
    "ht_multi_plan_create": (C.c_int, [C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_u64), C.POINTER(_vp), _u32,
                                       C.POINTER(_vp)]),
    "ht_multi_plan_launch": (C.c_int, [_vp, _vp]),
    "ht_multi_plan_status": (C.c_int, [_vp, _vp]),
    "ht_multi_plan_destroy": (C.c_int, [_vp]),
    "ht_sync_status": (C.c_int, [_vp, _vp]),
    "ht_rebuild": (C.c_int, [_vp, _u64, _vp]),
    "ht_size": (C.c_int, [_vp, C.POINTER(_u64), _vp]),
    "ht_dump": (C.c_int, [_vp, _vp, _u64, C.POINTER(_u64), _vp]),
    "ht_dump_raw": (C.c_int, [_vp, _vp, _u64, _vp]),
    "ht_clear": (C.c_int, [_vp, _vp]),
    "ht_stats": (C.c_int, [_vp, C.POINTER(HtStats), _vp]),
    "ht_hash_index": (C.c_int, [_vp, _u64, _u32, C.POINTER(_u64)]),
    "ht_set_scripted_hash": (C.c_int, [_vp, C.POINTER(_u64), C.POINTER(_u64), _u32]),
    "ht_reserve": (C.c_int, [_vp, _u64]),
    "ht_chain_histogram": (C.c_int, [_vp, C.POINTER(_u64), _vp]),
    "ht_strerror": (C.c_char_p, [C.c_int]),
    "ht_last_error": (C.c_char_p, []),
    "ht_bfs_explore": (C.c_int, [_vp, C.POINTER(HtBfsModel), _u64, _u32, C.POINTER(_u64), C.POINTER(_u64),
                                 C.POINTER(C.c_double), _vp]),
    "ht_bfs_explore_ex": (C.c_int, [_vp, C.POINTER(HtBfsModel), _u64, _u32, _u32, C.POINTER(_u64),
                                    C.POINTER(_u64), C.POINTER(C.c_double), C.POINTER(C.c_double), _vp]),
    "ht_server_config_default": (None, [C.POINTER(HtServerConfig)]),
    "ht_server_create": (C.c_int, [C.POINTER(_vp), _u32, C.POINTER(HtServerConfig), C.POINTER(_vp)]),
    "ht_server_run": (C.c_int, [_vp, C.POINTER(HtRequest), _u32, C.POINTER(HtServerStats)]),
    "ht_server_destroy": (C.c_int, [_vp]),
    "ht_timing_enable": (C.c_int, [C.c_int]),
    "ht_timing_report": (C.c_int, [C.c_char_p, _u64]),
    "ht_probe_copy": (C.c_int, [_vp, _vp, _u64, _vp]),
    "ht_probe_gather": (C.c_int, [_vp, _u64, _u64, _u32, _u64, _vp, _vp]),
    "ht_probe_cas": (C.c_int, [_vp, _u64, _u64, _u64, _vp]),
    "ht_probe_mix": (C.c_int, [_vp, _vp, _u64, _vp, _u64, C.c_double, C.c_double, _u32, _u64, _vp]),
}

EXPORTED = tuple(_PROTOS)

_lib: Optional[C.CDLL] = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libht.so (once) and declare the prototypes."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HtLibraryMissing(
            f"{path} is not built; run `python -m paper_1712_09494_amd.build` (hipcc, gfx950)")
    try:
        # load torch's HIP runtime first so that libht.so binds to the same one
        # (one runtime per process: torch's stream handles are then valid here)
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _strerror(code: int) -> str:
    try:
        return load().ht_strerror(code).decode()
    except Exception:
        return "error"


def _check(code: int, what: str) -> None:
    if code != HT_OK:
        detail = load().ht_last_error().decode()
        raise HtError(code, what, detail)


# ---- tensor marshalling -----------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _on_stream(stream):
    """Context in which torch's current stream is `stream` (a torch stream or
    a raw handle), so that the copies and allocations of the marshalling are
    ordered with the kernels launched there (and the caching allocator ties
    the temporaries to that stream); a no-op for None."""
    import contextlib
    torch = _torch()
    if stream is None:
        return contextlib.nullcontext()
    if isinstance(stream, int):
        stream = torch.cuda.ExternalStream(stream)
    return torch.cuda.stream(stream)


def _key_tensor(keys, device=None):
    """Device tensor of 64-bit keys (int64 view of uint64 bits)."""
    torch = _torch()
    if isinstance(keys, np.ndarray):
        a = np.ascontiguousarray(keys)
        if a.dtype == np.uint64:
            a = a.view(np.int64)
        elif a.dtype != np.int64:
            raise TypeError("keys must be uint64 or int64")
        return torch.from_numpy(a).to(device or "cuda")
    if not isinstance(keys, torch.Tensor):
        raise TypeError("keys must be a torch tensor or numpy array")
    if keys.dtype not in (torch.int64, torch.uint64):
        raise TypeError("keys must be int64 or uint64")
    if not keys.is_cuda:
        raise ValueError("keys must be on the GPU")
    if not keys.is_contiguous():
        keys = keys.contiguous()
    return keys


def _out_tensor(out, n, like):
    torch = _torch()
    if out is None:
        return torch.empty(n, dtype=torch.uint8, device=like.device)
    if out.dtype != torch.uint8 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
        raise ValueError("out must be a contiguous uint8 GPU tensor with room for every key")
    return out


# ---- C-named wrappers -----------------------------------------------------------

def ht_config_default(kind: int) -> HtConfig:
    c = HtConfig()
    load().ht_config_default(C.byref(c), kind)
    return c


def ht_create(cfg: HtConfig) -> int:
    h = _vp()
    _check(load().ht_create(C.byref(cfg), C.byref(h)), "ht_create")
    return h.value


def ht_create_simple(kind: int, capacity: int, nhash: int) -> int:
    h = _vp()
    _check(load().ht_create_simple(kind, capacity, nhash, C.byref(h)), "ht_create_simple")
    return h.value


def ht_destroy(h: int) -> None:
    _check(load().ht_destroy(h), "ht_destroy")


def _count(k, w: int) -> int:
    if k.numel() % w:
        raise ValueError(f"key tensor of {k.numel()} words is not a whole number of {w}-word keys")
    return k.numel() // w


def ht_find_or_put(h: int, keys, out=None, stream=None, key_words: int = 1):
    """keys: n 64-bit keys, or for a vector table n rows of key_words words
    (any shape with n * key_words elements, row-major).  With `stream`, the
    key copy, the flag allocation and the kernels all run on that stream."""
    with _on_stream(stream):
        k = _key_tensor(keys)
        n = _count(k, key_words)
        o = _out_tensor(out, n, k)
        _check(load().ht_find_or_put(h, k.data_ptr(), n, o.data_ptr(), _stream_handle(None)),
               "ht_find_or_put")
    return o


ht_insert = ht_find_or_put


def ht_find_or_put_noalloc(h: int, keys, out, stream=None):
    """The allocation-free find-or-put (at most 262144 single-word keys).
    ``keys`` and ``out`` must already be device tensors (int64/uint64 keys,
    uint8 flags with room for every key): nothing is copied or allocated."""
    torch = _torch()
    if not (isinstance(keys, torch.Tensor) and keys.is_cuda and keys.is_contiguous()
            and keys.dtype in (torch.int64, torch.uint64)):
        raise TypeError("keys must be a contiguous int64/uint64 GPU tensor")
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.is_contiguous() and out.dtype == torch.uint8
            and out.numel() >= keys.numel()):
        raise TypeError("out must be a contiguous uint8 GPU tensor with room for every key")
    _check(load().ht_find_or_put_noalloc(h, keys.data_ptr(), keys.numel(), out.data_ptr(), _stream_handle(stream)),
           "ht_find_or_put_noalloc")
    return out


def ht_query(h: int, keys, out=None, stream=None, key_words: int = 1):
    with _on_stream(stream):
        k = _key_tensor(keys)
        n = _count(k, key_words)
        o = _out_tensor(out, n, k)
        _check(load().ht_query(h, k.data_ptr(), n, o.data_ptr(), _stream_handle(None)), "ht_query")
    return o


def _multi_args(handles, keys_list, outs, key_words):
    """Marshal per-table arguments: keys as n rows of key_words[i] words."""
    n = len(handles)
    ks = [_key_tensor(k) for k in keys_list]
    if len(ks) != n:
        raise ValueError("one key tensor per table")
    ws = [1] * n if key_words is None else [int(w) for w in key_words]
    counts = [_count(ks[i], ws[i]) for i in range(n)]
    os_ = [_out_tensor(None if outs is None else outs[i], counts[i], ks[i]) for i in range(n)]
    th = (_vp * n)(*handles)
    kp = (_vp * n)(*[k.data_ptr() for k in ks])
    nn = (_u64 * n)(*counts)
    op = (_vp * n)(*[o.data_ptr() for o in os_])
    return ks, os_, th, kp, nn, op


def ht_find_or_put_multi(handles: Sequence[int], keys_list, outs=None, stream=None, key_words=None):
    with _on_stream(stream):
        ks, os_, th, kp, nn, op = _multi_args(handles, keys_list, outs, key_words)
        _check(load().ht_find_or_put_multi(th, kp, nn, op, len(handles), _stream_handle(None)),
               "ht_find_or_put_multi")
    return os_


def ht_query_multi(handles: Sequence[int], keys_list, outs=None, stream=None, key_words=None):
    with _on_stream(stream):
        ks, os_, th, kp, nn, op = _multi_args(handles, keys_list, outs, key_words)
        _check(load().ht_query_multi(th, kp, nn, op, len(handles), _stream_handle(None)), "ht_query_multi")
    return os_


class MultiPlan:
    """A prepared many-table find-or-put (ht_multi_plan_*).  The key and
    flag tensors are kept alive by the plan; launch() allocates nothing and
    may run inside torch.cuda.graph capture."""

    def __init__(self, tables, keys_list, outs=None):
        n = len(tables)
        self.tables = list(tables)
        self.keys, self.outs, th, kp, nn, op = _multi_args([t.handle for t in self.tables], keys_list, outs,
                                                           [t.key_words for t in self.tables])
        h = _vp()
        _check(load().ht_multi_plan_create(th, kp, nn, op, n, C.byref(h)), "ht_multi_plan_create")
        self.handle = h.value

    def launch(self, stream=None):
        _check(load().ht_multi_plan_launch(self.handle, _stream_handle(stream)), "ht_multi_plan_launch")

    def status(self, stream=None) -> int:
        return load().ht_multi_plan_status(self.handle, _stream_handle(stream))

    def close(self):
        if getattr(self, "handle", None):
            _check(load().ht_multi_plan_destroy(self.handle), "ht_multi_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ht_sync_status(h: int, stream=None) -> int:
    return load().ht_sync_status(h, _stream_handle(stream))


def ht_rebuild(h: int, new_capacity: int = 0, stream=None) -> None:
    _check(load().ht_rebuild(h, new_capacity, _stream_handle(stream)), "ht_rebuild")


def ht_size(h: int, stream=None) -> int:
    n = _u64()
    _check(load().ht_size(h, C.byref(n), _stream_handle(stream)), "ht_size")
    return n.value


def ht_stats(h: int, stream=None) -> dict:
    s = HtStats()
    _check(load().ht_stats(h, C.byref(s), _stream_handle(stream)), "ht_stats")
    return s.as_dict()


def ht_dump(h: int, stream=None, key_words: int = 1):
    """Members as an int64 GPU tensor (uint64 bits), any order; for a vector
    table an (n, key_words) tensor."""
    torch = _torch()
    with _on_stream(stream):
        n = ht_size(h)
        buf = torch.empty((max(n, 1), key_words), dtype=torch.int64, device="cuda")
        got = _u64()
        _check(load().ht_dump(h, buf.data_ptr(), buf.shape[0], C.byref(got), _stream_handle(None)), "ht_dump")
    buf = buf[: got.value]
    return buf.reshape(-1) if key_words == 1 else buf


def ht_dump_raw(h: int, stream=None):
    torch = _torch()
    with _on_stream(stream):
        st = ht_stats(h)
        cap = st["capacity"] + st["stash_slots"]
        buf = torch.empty(cap, dtype=torch.int64, device="cuda")
        _check(load().ht_dump_raw(h, buf.data_ptr(), cap, _stream_handle(None)), "ht_dump_raw")
    return buf


def ht_clear(h: int, stream=None) -> None:
    _check(load().ht_clear(h, _stream_handle(stream)), "ht_clear")


def ht_hash_index(h: int, key: int, j: int) -> int:
    out = _u64()
    _check(load().ht_hash_index(h, key & EMPTY, j, C.byref(out)), "ht_hash_index")
    return out.value


def ht_set_scripted_hash(h: int, script: dict, nhash: int) -> None:
    keys = list(script)
    n = len(keys)
    ka = (_u64 * max(n, 1))(*[k & EMPTY for k in keys])
    flat = [int(v) for k in keys for v in script[k]]
    if len(flat) != n * nhash:
        raise ValueError("each scripted key needs nhash values")
    ha = (_u64 * max(len(flat), 1))(*flat)
    _check(load().ht_set_scripted_hash(h, ka, ha, n), "ht_set_scripted_hash")


def ht_chain_histogram(h: int, stream=None) -> dict:
    """Eviction-chain histogram (tables created with HT_FLAG_CHAIN_STATS):
    {"stash": chains that ended in the stash, "counts": [chains of i
    exchanges for i = 0..63, the last counting 63 or more], "mean", "p99",
    "max": over chains that found a slot}."""
    a = (_u64 * 64)()
    _check(load().ht_chain_histogram(h, a, _stream_handle(stream)), "ht_chain_histogram")
    counts = [int(a[i]) for i in range(64)]
    stash, counts[0] = counts[0], 0
    total = sum(counts)
    mean = p99 = mx = None
    if total:
        mean = round(sum(i * c for i, c in enumerate(counts)) / total, 3)
        acc = 0
        for i, c in enumerate(counts):
            acc += c
            if p99 is None and acc >= 0.99 * total:
                p99 = i
        mx = max(i for i, c in enumerate(counts) if c)
    return {"stash": stash, "counts": counts, "chains": total, "mean": mean, "p99": p99, "max": mx}


def ht_reserve(h: int, max_batch: int) -> None:
    _check(load().ht_reserve(h, max_batch), "ht_reserve")


def ht_timing_enable(on: bool = True) -> None:
    _check(load().ht_timing_enable(1 if on else 0), "ht_timing_enable")


def ht_timing_report() -> dict:
    """{kernel: (launches, total_ms)} of the launches timed so far."""
    import json
    buf = C.create_string_buffer(1 << 16)
    _check(load().ht_timing_report(buf, len(buf)), "ht_timing_report")
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


def ht_probe_copy(src, dst, stream=None) -> None:
    _check(load().ht_probe_copy(src.data_ptr(), dst.data_ptr(), src.numel(), _stream_handle(stream)),
           "ht_probe_copy")


def ht_probe_gather(arr, n_access: int, line_bytes: int, seed: int, sink, stream=None) -> None:
    _check(load().ht_probe_gather(arr.data_ptr(), arr.numel(), n_access, line_bytes, seed & EMPTY,
                                  sink.data_ptr(), _stream_handle(stream)), "ht_probe_gather")


def ht_probe_cas(arr, n_access: int, seed: int, stream=None) -> None:
    _check(load().ht_probe_cas(arr.data_ptr(), arr.numel(), n_access, seed & EMPTY, _stream_handle(stream)),
           "ht_probe_cas")


def ht_probe_mix(keys, out, arr, lines_per_item: float, cas_per_item: float, seed: int, stream=None,
                 same_line: bool = False) -> None:
    _check(load().ht_probe_mix(keys.data_ptr(), out.data_ptr(), keys.numel(), arr.data_ptr(), arr.numel(),
                               float(lines_per_item), float(cas_per_item), 1 if same_line else 0, seed & EMPTY,
                               _stream_handle(stream)), "ht_probe_mix")


# ---- object wrapper --------------------------------------------------------------

class Table:
    """One GPU hash table (bucketed or cuckoo) behind the C ABI."""

    def __init__(self, kind: str = "bucketed", capacity: int = 1 << 20, nhash: int = 3,
                 bucket_slots: int = 16, stash_slots: int = 0, max_chain: int = 0, seed: int = 0,
                 flags: int = 0, overflow_slots: int = 0, max_batch: int = 0, keys_per_group: int = 0,
                 bucket_walk: int = 0, lds_bytes: int = 0, key_words: int = 1):
        self.kind = kind
        cfg = ht_config_default(KINDS[kind])
        cfg.capacity = int(capacity)
        cfg.nhash = int(nhash)
        cfg.bucket_slots = int(bucket_slots) if kind == "bucketed" else 0
        cfg.stash_slots = int(stash_slots)
        cfg.max_chain = int(max_chain)
        cfg.seed = int(seed) & EMPTY
        cfg.flags = int(flags)
        cfg.overflow_slots = int(overflow_slots)
        cfg.max_batch = int(max_batch)
        cfg.keys_per_group = int(keys_per_group)
        if bucket_walk:
            cfg.bucket_walk = int(bucket_walk)
        cfg.lds_bytes = int(lds_bytes)
        cfg.key_words = int(key_words)
        self.key_words = int(key_words)
        self.nhash = cfg.nhash
        self.handle = ht_create(cfg)

    def close(self) -> None:
        if getattr(self, "handle", None):
            ht_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def find_or_put(self, keys, out=None, stream=None):
        return ht_find_or_put(self.handle, keys, out, stream, self.key_words)

    insert = find_or_put

    def query(self, keys, out=None, stream=None):
        return ht_query(self.handle, keys, out, stream, self.key_words)

    def size(self, stream=None) -> int:
        return ht_size(self.handle, stream)

    def stats(self, stream=None) -> dict:
        return ht_stats(self.handle, stream)

    def dump(self, stream=None):
        return ht_dump(self.handle, stream, self.key_words)

    def dump_raw(self, stream=None):
        return ht_dump_raw(self.handle, stream)

    def clear(self, stream=None) -> None:
        ht_clear(self.handle, stream)

    def rebuild(self, new_capacity: int = 0, stream=None) -> None:
        ht_rebuild(self.handle, new_capacity, stream)

    def sync_status(self, stream=None) -> int:
        return ht_sync_status(self.handle, stream)

    def hash_index(self, key: int, j: int) -> int:
        return ht_hash_index(self.handle, key, j)

    def set_scripted_hash(self, script: dict) -> None:
        ht_set_scripted_hash(self.handle, script, self.nhash)

    def reserve(self, max_batch: int) -> None:
        ht_reserve(self.handle, max_batch)

    def bfs_explore(self, model, levels: int, initial: int = 0, stream=None, fused: bool = False) -> dict:
        if fused:
            return ht_bfs_explore_ex(self.handle, model, levels, HT_BFS_FUSED, initial, stream)
        return ht_bfs_explore(self.handle, model, levels, initial, stream)


def ht_bfs_explore(h: int, model, levels: int, initial: int = 0, stream=None) -> dict:
    """Breadth-first exploration on the GPU with table h as the visited set."""
    m = pack_bfs_model(model)
    bs = (_u64 * max(levels, 1))()
    nc = (_u64 * max(levels, 1))()
    ms = (C.c_double * max(levels, 1))()
    _check(load().ht_bfs_explore(h, C.byref(m), initial & EMPTY, levels, bs, nc, ms, _stream_handle(stream)),
           "ht_bfs_explore")
    done = [i for i in range(levels) if bs[i] or i == 0]
    return {"batch_sizes": [int(bs[i]) for i in range(levels)], "new_counts": [int(nc[i]) for i in range(levels)],
            "fop_ms": [float(ms[i]) for i in range(levels)], "levels": len(done)}


def ht_bfs_explore_ex(h: int, model, levels: int, mode: int = 0, initial: int = 0, stream=None) -> dict:
    """ht_bfs_explore with a mode (HT_BFS_SPLIT or HT_BFS_FUSED) and the
    device time of each whole level (level_ms)."""
    m = pack_bfs_model(model)
    bs = (_u64 * max(levels, 1))()
    nc = (_u64 * max(levels, 1))()
    ms = (C.c_double * max(levels, 1))()
    lv = (C.c_double * max(levels, 1))()
    _check(load().ht_bfs_explore_ex(h, C.byref(m), initial & EMPTY, levels, mode, bs, nc, ms, lv,
                                    _stream_handle(stream)), "ht_bfs_explore_ex")
    done = [i for i in range(levels) if bs[i] or i == 0]
    return {"batch_sizes": [int(bs[i]) for i in range(levels)], "new_counts": [int(nc[i]) for i in range(levels)],
            "fop_ms": [float(ms[i]) for i in range(levels)], "level_ms": [float(lv[i]) for i in range(levels)],
            "levels": len(done)}


class Server:
    """Request loop over resident tables (ht_server_*).

    run(reqs) takes a list of (op, table_index, keys, arrival_s) where keys is
    a pinned host tensor (int64/uint64; see torch's pin_memory); it returns a
    list of pinned host uint8 flag tensors, per-request admit/done times and
    the run statistics."""

    def __init__(self, tables, slots: int = 16, merge: int = 16, staging_bytes: int = 0,
                 sequential: bool = False, group_keys: int = 0):
        n = len(tables)
        self.tables = list(tables)
        cfg = HtServerConfig()
        load().ht_server_config_default(C.byref(cfg))
        cfg.slots = int(slots)
        cfg.merge = int(merge)
        cfg.staging_bytes = int(staging_bytes)
        cfg.sequential = 1 if sequential else 0
        cfg.group_keys = int(group_keys)
        th = (_vp * n)(*[t.handle for t in self.tables])
        h = _vp()
        _check(load().ht_server_create(th, n, C.byref(cfg), C.byref(h)), "ht_server_create")
        self.handle = h.value

    def run(self, reqs, outs=None):
        torch = _torch()
        n = len(reqs)
        arr = (HtRequest * max(n, 1))()
        keep = []
        outs = outs or [None] * n
        res = []
        for i, (op, table, keys, arrival) in enumerate(reqs):
            if keys.device.type != "cpu" or not keys.is_pinned():
                raise ValueError("request keys must be a pinned host tensor")
            # an index the server does not hold is rejected by the library
            w = self.tables[int(table)].key_words if 0 <= int(table) < len(self.tables) else 1
            if keys.numel() % w:
                raise ValueError(f"request {i}: keys are not whole rows of {w} words")
            nk = keys.numel() // w
            o = outs[i]
            if o is None:
                o = torch.empty(nk, dtype=torch.uint8, pin_memory=True)
            keep.append(keys)
            res.append(o)
            arr[i].op = HT_OP_QUERY if op == "query" else HT_OP_FIND_OR_PUT
            arr[i].table = int(table)
            arr[i].h_keys = keys.data_ptr() if nk else None
            arr[i].n = nk
            arr[i].h_out = o.data_ptr() if nk else None
            arr[i].arrival_s = float(arrival)
        st = HtServerStats()
        _check(load().ht_server_run(self.handle, arr, n, C.byref(st)), "ht_server_run")
        admit = np.array([arr[i].admit_s for i in range(n)])
        done = np.array([arr[i].done_s for i in range(n)])
        groups = np.array([arr[i].group for i in range(n)])
        return res, admit, done, groups, st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            _check(load().ht_server_destroy(self.handle), "ht_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def find_or_put_multi(tables: Iterable[Table], keys_list, outs=None, stream=None):
    tables = list(tables)
    return ht_find_or_put_multi([t.handle for t in tables], keys_list, outs, stream, [t.key_words for t in tables])


def query_multi(tables: Iterable[Table], keys_list, outs=None, stream=None):
    tables = list(tables)
    return ht_query_multi([t.handle for t in tables], keys_list, outs, stream, [t.key_words for t in tables])


def u64(t) -> np.ndarray:
    """GPU int64 tensor -> host uint64 array."""
    return t.cpu().numpy().view(np.uint64)
