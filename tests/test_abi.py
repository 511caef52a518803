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
    assert lib.sr_set_option(b"no_such_option", 1) == 1
    assert lib.sr_set_option(b"force_path", 9) == 1
    assert lib.sr_set_option(b"profile", 0) == 0
    assert lib.sr_status_str(0) == b"ok"
    assert lib.sr_status_str(3) == b"out of memory"
    b = ctypes.c_size_t()
    assert lib.sr_workspace_bytes(0, 0, 1000, 0, ctypes.byref(b)) == 0 and b.value >= 4000
    assert lib.sr_workspace_bytes(5, 0, 1000, 0, ctypes.byref(b)) == 1
