"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sortrace.h")


def _lib_path():
    from paper_1609_04471_amd import build, sortrace
    if not os.path.exists(sortrace.LIB_PATH):
        build.build()
    return sortrace.LIB_PATH


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sr_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_functions()
    for want in ("sr_sort_keys", "sr_sort_pairs", "sr_sort_segmented"):
        assert want in names


def test_library_exports_every_declared_symbol():
    out = subprocess.check_output(["nm", "-D", "--defined-only", _lib_path()]).decode()
    exported = set(re.findall(r"\bT (sr_[a-z_0-9]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    from paper_1609_04471_amd import sortrace
    assert set(sortrace.EXPORTS) == set(declared_functions())


@pytest.fixture(scope="module")
def lib():
    from paper_1609_04471_amd import sortrace
    return sortrace.load(_lib_path())


def test_host_side_validation(lib):
    vp = ctypes.c_void_p
    assert lib.sr_sort_keys(7, vp(0x1000), 10, None) == 1            # bad dtype
    assert lib.sr_sort_keys(0, None, 10, None) == 1                  # NULL keys
    assert lib.sr_sort_keys(0, vp(0x1002), 10, None) == 1            # misaligned int32
    assert lib.sr_sort_keys(1, vp(0x1004), 10, None) == 1            # misaligned uint64
    assert b"aligned" in lib.sr_last_error_message()
    assert lib.sr_sort_keys(0, None, 1, None) == 0                   # n <= 1: no-op
    assert lib.sr_sort_keys(0, None, 0, None) == 0
    assert lib.sr_sort_pairs(0, vp(0x1000), None, 10, None) == 1     # NULL payload
    assert lib.sr_sort_pairs(0, vp(0x1000), vp(0x2002), 10, None) == 1
    assert lib.sr_set_workspace(vp(0x1080), 1 << 20, None) == 1       # not 256-byte aligned
    assert b"aligned" in lib.sr_last_error_message()
    assert lib.sr_set_workspace(vp(0x1000), (1 << 20) - 256, None) == 1  # under 1 MiB
    assert lib.sr_set_option(b"no_such_option", 1) == 1
    assert lib.sr_set_option(b"force_path", 9) == 1
    assert lib.sr_set_option(b"profile", 0) == 0
    assert lib.sr_status_str(0) == b"ok"
    assert lib.sr_status_str(3) == b"out of memory"
    b = ctypes.c_size_t()
    assert lib.sr_workspace_bytes(0, 0, 1000, 0, ctypes.byref(b)) == 0 and b.value >= 4000
    assert lib.sr_workspace_bytes(5, 0, 1000, 0, ctypes.byref(b)) == 1
    from paper_1609_04471_amd import sortrace
    m = sortrace.SrPresortedness()
    assert lib.sr_measure_presortedness(0, vp(0x1000), 10, 2, ctypes.byref(m), None) == 1  # unknown flag
    assert lib.sr_measure_presortedness(0, vp(0x1000), 10, 0, None, None) == 1             # NULL output
    assert lib.sr_measure_presortedness(0, vp(0x1002), 10, 0, ctypes.byref(m), None) == 1  # misaligned
    assert lib.sr_measure_presortedness(0, None, 1, 1, ctypes.byref(m), None) == 0         # n <= 1
    assert (m.run, m.mono, m.inv, m.descents) == (1, 1, 0, 0)
    assert lib.sr_measure_presortedness(0, None, 0, 0, ctypes.byref(m), None) == 0
    assert (m.run, m.mono, m.inv) == (0, 0, -1)


@pytest.fixture
def keep_table(lib):
    """Restore the table the library had loaded after the test."""
    from paper_1609_04471_amd import sortrace
    saved = sortrace.tune_get()
    yield
    sortrace.tune_set(saved)


def test_tuning_table_validation(lib, keep_table):
    from paper_1609_04471_amd import sortrace
    sortrace.tune_set([])
    assert sortrace.tune_get() == []
    rows = [{"dtype": "uint64", "pairs": True, "min_n": 1 << 20, "partition": 1, "nontemporal": 0},
            {"dtype": "int32", "pairs": False, "min_n": 1 << 22, "tile_variant": 0, "partition": 1},
            {"dtype": "int32", "pairs": False, "min_n": 0, "tile_variant": 1, "merge_items": 16}]
    sortrace.tune_set(rows)
    got = sortrace.tune_get()
    assert [(r["dtype"], r["pairs"], r["min_n"]) for r in got] == \
        [("int32", False, 0), ("int32", False, 1 << 22), ("uint64", True, 1 << 20)]
    assert got[0]["merge_items"] == 16 and got[0]["partition"] == -1 and got[0]["nontemporal"] == -1
    assert got[2]["tile_variant"] == -1 and got[2]["merge_items"] == 0
    bad = [
        {"dtype": "int32", "min_n": -1},
        {"dtype": "int32", "min_n": 0, "tile_variant": 2},
        {"dtype": "int32", "min_n": 0, "merge_items": 12},
        {"dtype": "int32", "min_n": 0, "partition": 3},
        {"dtype": "int32", "min_n": 0, "nontemporal": -2},
        {"dtype": "int32", "min_n": 0, "fan_in": 3},
        {"dtype": "int32", "pairs": True, "min_n": 0, "fan_in": 4},   # pairs merge two-way
    ]
    for r in bad:
        with pytest.raises(sortrace.SortraceError) as ei:
            sortrace.tune_set([rows[0], r])
        assert ei.value.status == 1, r
        assert sortrace.tune_get() == got      # unchanged
    with pytest.raises(sortrace.SortraceError):
        sortrace.tune_set([rows[2], dict(rows[2], merge_items=8)])  # same (dtype, pairs, min_n)
    # segmented rows: their own kind (same min_n as a plain row is fine), only
    # tile_variant and merge_items
    seg = dict(rows[2], segmented=True, tile_variant=0, merge_items=8)
    sortrace.tune_set(rows + [seg])
    both = sortrace.tune_get()
    assert [(r["min_n"], r["segmented"]) for r in both if r["dtype"] == "int32"] == \
        [(0, False), (1 << 22, False), (0, True)]
    for r in (dict(seg, partition=1), dict(seg, nontemporal=0), dict(seg, fan_in=4)):
        with pytest.raises(sortrace.SortraceError):
            sortrace.tune_set([r])
    raw = (sortrace.SrTuneEntry * 1)()
    raw[0].tile_variant, raw[0].partition, raw[0].nontemporal, raw[0].segmented = -1, -1, -1, 2
    assert lib.sr_tune_set(raw, 1) == 1 and b"segmented" in lib.sr_last_error_message()
    four = dict(rows[1], fan_in=4)
    sortrace.tune_set([rows[0], four])
    assert [r["fan_in"] for r in sortrace.tune_get()] == [4, 0]   # int32 row first
    sortrace.tune_set(rows)
    e = (sortrace.SrTuneEntry * 1)()
    e[0].dtype = 9
    assert lib.sr_tune_set(e, 1) == 1 and b"dtype" in lib.sr_last_error_message()
    assert lib.sr_tune_set(None, 3) == 1
    assert lib.sr_tune_set(e, 1025) == 1
    cnt = ctypes.c_int64()
    assert lib.sr_tune_get(None, 0, ctypes.byref(cnt)) == 0 and cnt.value == 3
    assert lib.sr_tune_get(None, 0, None) == 1
    sortrace.tune_set([])
    assert sortrace.tune_get() == []
    assert lib.sr_set_option(b"merge_nontemporal", 2) == 1
    assert lib.sr_set_option(b"merge_nontemporal", -1) == 0
    assert lib.sr_set_option(b"merge_items", 12) == 1
    assert lib.sr_set_option(b"merge_items", 0) == 0
    assert lib.sr_set_option(b"partition_min_n", -2) == 1
    assert lib.sr_set_option(b"partition_min_n", -1) == 0


def test_autotune_host_logic(tmp_path, keep_table):
    import json
    from paper_1609_04471_amd import autotune, sortrace
    c = autotune.candidates("int32", False)
    # 2 tiles x (fused: 2 merge widths + persistent: 2 store kinds x 2 fan-ins)
    assert len(c) == 12 and len({json.dumps(x, sort_keys=True) for x in c}) == 12
    assert all(set(x) <= set(sortrace.TUNE_FIELDS) for x in c)
    assert autotune.candidates("uint64", False) == \
        [{"partition": 0}, {"partition": 1, "nontemporal": 0}, {"partition": 1, "nontemporal": 0, "fan_in": 4},
         {"partition": 1, "nontemporal": 1}, {"partition": 1, "nontemporal": 1, "fan_in": 4}]
    for dt, pairs in (("int32", True), ("float32", True), ("uint64", True)):
        c = autotune.candidates(dt, pairs)
        assert c == [{"partition": 0}, {"partition": 1, "nontemporal": 0}, {"partition": 1, "nontemporal": 1}]
    sizes = autotune.band_sizes("int32", False, 16, 20, 2)
    assert sizes == [1 << 16, 1 << 18, 1 << 20]
    assert autotune.band_starts(sizes) == [0, 1 << 17, 1 << 19]
    rows = [{"dtype": "int32", "pairs": False, "min_n": 0, "partition": 0, "merge_items": 8},
            {"dtype": "int32", "pairs": False, "min_n": 9, "partition": 0, "merge_items": 8},
            {"dtype": "int32", "pairs": False, "min_n": 99, "partition": 1, "nontemporal": 0},
            {"dtype": "int32", "pairs": True, "min_n": 0, "partition": 1, "nontemporal": 0}]
    assert [r["min_n"] for r in autotune.compress(rows)] == [0, 99, 0]
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"format": autotune.FORMAT, "rows": rows}))
    assert autotune.apply(str(p)) == autotune.validate(json.loads(p.read_text()))
    assert len(sortrace.tune_get()) == 4
    p.write_text(json.dumps({"format": "other", "rows": rows}))
    with pytest.raises(ValueError):
        autotune.apply(str(p))
    # the shipped table names only swept shapes
    for r in autotune.validate(json.load(open(sortrace.TUNE_TABLE))):
        shape = {k: v for k, v in r.items() if k in sortrace.TUNE_FIELDS}
        swept = autotune.seg_candidates(r["dtype"]) if r["segmented"] else autotune.candidates(r["dtype"], r["pairs"])
        assert shape in swept, r
