"""C ABI of libht.so on the CPU host: the library loads, exports every entry
point include/ht.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1712_09494_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "ht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ht_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_expected_calls():
    names = header_functions()
    for must in ("ht_create", "ht_destroy", "ht_find_or_put", "ht_insert", "ht_query",
                 "ht_find_or_put_multi", "ht_sync_status", "ht_rebuild", "ht_size", "ht_dump",
                 "ht_dump_raw", "ht_clear", "ht_stats", "ht_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = b.load()
    for name in header_functions():
        assert hasattr(lib, name), name
    assert set(header_functions()) == set(b.EXPORTED)


def test_strerror_and_defaults():
    lib = b.load()
    for code in (b.HT_OK, b.HT_EINVAL, b.HT_ENOMEM, b.HT_EFULL, b.HT_EHIP):
        assert lib.ht_strerror(code)
    c = b.ht_config_default(b.HT_BUCKETED)
    assert (c.kind, c.nhash, c.bucket_slots, c.stash_slots) == (b.HT_BUCKETED, 3, 16, 1024)
    c = b.ht_config_default(b.HT_CUCKOO)
    assert (c.kind, c.nhash, c.bucket_slots) == (b.HT_CUCKOO, 3, 0)


@pytest.mark.parametrize("fn,args", [
    ("ht_find_or_put", (None, None, 5, None, None)),
    ("ht_query", (None, None, 5, None, None)),
    ("ht_size", (None, None, None)),
    ("ht_clear", (None, None)),
    ("ht_destroy", (None,)),
    ("ht_sync_status", (None, None)),
    ("ht_reserve", (None, 10)),
])
def test_null_table_rejected(fn, args):
    lib = b.load()
    assert getattr(lib, fn)(*args) == b.HT_EINVAL
    assert lib.ht_last_error()


def test_bad_configs_rejected_without_gpu():
    lib = b.load()
    h = C.c_void_p()
    bad = []
    c = b.ht_config_default(b.HT_BUCKETED); c.capacity = 0; bad.append(c)
    c = b.ht_config_default(b.HT_BUCKETED); c.capacity = 64; c.nhash = 0; bad.append(c)
    c = b.ht_config_default(b.HT_BUCKETED); c.capacity = 64; c.nhash = 9; bad.append(c)
    c = b.ht_config_default(b.HT_BUCKETED); c.capacity = 64; c.bucket_slots = 12; bad.append(c)
    c = b.ht_config_default(b.HT_CUCKOO); c.capacity = 64; c.stash_slots = 100; bad.append(c)
    c = b.ht_config_default(b.HT_CUCKOO); c.capacity = 64; c.flags = 1 << 9; bad.append(c)
    c = b.ht_config_default(7); c.capacity = 64; bad.append(c)
    c = b.ht_config_default(b.HT_BUCKETED); c.capacity = 64; c.lds_bytes = 1 << 30; bad.append(c)
    for c in bad:
        assert lib.ht_create(C.byref(c), C.byref(h)) == b.HT_EINVAL
        assert h.value is None
    assert lib.ht_find_or_put_multi(None, None, None, None, 3, None) == b.HT_EINVAL
    assert lib.ht_find_or_put_multi(None, None, None, None, 0, None) == b.HT_OK
    assert lib.ht_probe_gather(None, 0, 5, 64, 0, None, None) == b.HT_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    b2 = b.load  # the loader, pointed at a path with no library
    import importlib
    mod = importlib.import_module("paper_1712_09494_amd.binding")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(b.HtLibraryMissing):
            mod.load(str(tmp_path / "libht.so"))
    finally:
        mod._lib = saved
    assert b2 is mod.load


def test_bfs_model_packing():
    from paper_1712_09494_amd import inputs
    m = inputs.BfsModel(1)
    pm = b.pack_bfs_model(m)
    for p in range(16):
        for s in range(16):
            assert pm.local_count[p][s] == len(m.local[p][s])
            assert list(pm.local_target[p][s])[: len(m.local[p][s])] == m.local[p][s]
    for a, (sp, sq, pe, qe) in enumerate(m.syncs):
        assert (pm.sync_p[a], pm.sync_q[a]) == (sp, sq)
        assert [pm.sync_p_edge[a][s] for s in range(16)] == [x[0] if x else -1 for x in pe]
    lib = b.load()
    assert lib.ht_bfs_explore(None, C.byref(pm), 0, 3, None, None, None, None) == b.HT_EINVAL


def header_docs():
    """{function: the comment block right before its declaration}."""
    src = open(os.path.join(ROOT, "include", "ht.h")).read()
    out = {}
    for m in re.finditer(r"/\*((?:(?!\*/).)*)\*/\s*\n((?:[A-Za-z_][\w\s\*]*?\b(ht_[a-z_0-9]+)\s*\([^;]*;\s*\n?)+)",
                         src, flags=re.S):
        for name in re.findall(r"\b(ht_[a-z_0-9]+)\s*\(", m.group(2)):
            out.setdefault(name, m.group(1))
    return out


def test_every_entry_point_cites_its_passage_or_says_infrastructure():
    """Each declaration in ht.h follows a comment that cites the passage of
    the paper defining the operation (Sec. / Fig.), refers to the call it
    equals, or marks it as infrastructure."""
    docs = header_docs()
    names = header_functions()
    missing = [n for n in names if n not in docs]
    assert not missing, missing
    for n in names:
        d = docs[n]
        assert re.search(r"Sec\. \d|Fig\. \d|Infrastructure|Same as ht_", d), n
    # the calls whose defining passage the paper gives
    for n in ("ht_create", "ht_find_or_put", "ht_query", "ht_sync_status", "ht_rebuild", "ht_size", "ht_dump",
              "ht_clear", "ht_find_or_put_multi", "ht_bfs_explore"):
        assert re.search(r"Sec\. \d", docs[n]), n
    for n in ("ht_destroy", "ht_stats", "ht_dump_raw", "ht_strerror", "ht_create_simple", "ht_last_error"):
        assert "Infrastructure" in docs[n], n


def header_enum_values():
    """NAME -> value of every HT_* enumerator in include/ht.h (literals and 1u << n)."""
    src = open(os.path.join(ROOT, "include", "ht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    vals = {}
    for name, expr in re.findall(r"\b(HT_[A-Z0-9_]+)\s*=\s*([^,}\n]+)", src):
        expr = expr.strip()
        m = re.fullmatch(r"1u\s*<<\s*(\d+)", expr)
        if m:
            vals[name] = 1 << int(m.group(1))
        elif re.fullmatch(r"-?\d+", expr):
            vals[name] = int(expr)
    return vals


def test_binding_constants_match_header():
    """Every HT_* constant of the binding equals the header's enumerator, and
    every flag of the header has its constant in the binding."""
    vals = header_enum_values()
    flags = {k for k in vals if k.startswith("HT_FLAG_")}
    assert {"HT_FLAG_CUCKOO_PAPER_ORDER", "HT_FLAG_BUCKETED_GROUP_QUERY", "HT_FLAG_CUCKOO_LOOKAHEAD"} <= flags
    for name, v in vals.items():
        if hasattr(b, name):
            assert getattr(b, name) == v, name
    for name in flags:
        assert getattr(b, name) == vals[name], name
    # the flags are distinct bits
    bits = [vals[f] for f in flags]
    assert len(set(bits)) == len(bits) and all(x & (x - 1) == 0 for x in bits)


def test_device_flag_mirrors_match_header():
    """The device code tests some flags through its own constants; they must be
    the header's bits."""
    vals = header_enum_values()
    src = open(os.path.join(ROOT, "paper_1712_09494_amd", "csrc", "ht_device.h")).read()
    dev = {n: 1 << int(s) for n, s in re.findall(r"constexpr uint32_t (kFlag\w+) = 1u << (\d+);", src)}
    assert dev["kFlagChainStats"] == vals["HT_FLAG_CHAIN_STATS"]
    assert dev["kFlagLookahead"] == vals["HT_FLAG_CUCKOO_LOOKAHEAD"]
    assert dev["kFlagGroupQuery"] == vals["HT_FLAG_BUCKETED_GROUP_QUERY"]
