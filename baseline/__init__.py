"""The paper's adaptive mergesort (Sort Race, Sec. 3: techniques (a), (b),
(e2), (f), (g)) as a plain C program with counted comparisons -- a CPU
comparison point for the GPU library.  It shares no code with the library or
with the test oracle; ``bench.py`` times it and reports its comparison counts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "paper_mergesort.c")
_LIB = os.path.join(_HERE, "libpaper_mergesort.so")
DTYPES = {"int32": 0, "uint64": 1, "float32": 2}
# Neither the minimum run length nor the number of wins that starts galloping
# is given by the paper (its Sec. 3 example shows galloping after three wins,
# as an illustration).  Taken here: runs of at least 8, galloping after 7 wins
# in a row (the starting threshold of timsort, the design Sec. 3 begins from).
MINRUN = 8
GALLOP_AFTER = 7


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.pm_sort.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_size_t,
                                ctypes.c_size_t, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64)]
        lib.pm_sort.restype = ctypes.c_int
        _lib = lib
    return _lib


def sort(keys: np.ndarray, payload: np.ndarray | None = None, minrun: int = MINRUN,
         gallop_after: int = GALLOP_AFTER):
    """Sorts a copy; returns (keys, comparisons) or, with a uint32 payload
    carried stably, ((keys, payload), comparisons)."""
    k = np.ascontiguousarray(keys)
    if k.dtype.name not in DTYPES:
        raise TypeError(k.dtype)
    n = k.size
    if payload is None:
        rec = k.copy()
        es = k.itemsize
    else:
        p = np.ascontiguousarray(payload, dtype=np.uint32)
        assert p.size == n
        es = k.itemsize + 4
        rec = np.empty((n, es), dtype=np.uint8)
        rec[:, :k.itemsize] = k.view(np.uint8).reshape(n, k.itemsize)
        rec[:, k.itemsize:] = p.view(np.uint8).reshape(n, 4)
    cnt = ctypes.c_uint64()
    rc = _load().pm_sort(DTYPES[k.dtype.name], rec.ctypes.data, n, es, minrun, gallop_after,
                         ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("paper mergesort rejected its arguments")
    if payload is None:
        return rec, int(cnt.value)
    ok = np.ascontiguousarray(rec[:, :k.itemsize]).view(k.dtype).reshape(n)
    op = np.ascontiguousarray(rec[:, k.itemsize:]).view(np.uint32).reshape(n)
    return (ok, op), int(cnt.value)
