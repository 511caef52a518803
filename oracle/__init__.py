"""CPU oracle for libsortrace -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
two share no code: the oracle is the plain C file ``sortrace_oracle.c``
(stable top-down mergesort, insertion sort, brute-force selection, the list
sort of the heavy items, and the presortedness measures Run/Inv/Mono of
Sec. 2 of the Sort Race paper), driven
here through ctypes on numpy arrays.

Every function takes a numpy array and returns a NEW sorted array (the input
is left untouched), so a test can hand the same bytes to the GPU and to the
oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sortrace_oracle.c")
_LIB = os.path.join(_HERE, "libsortrace_oracle.so")

DTYPES = {"int32": 0, "uint64": 1, "float32": 2}
_NP = {"int32": np.int32, "uint64": np.uint64, "float32": np.float32}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libsortrace_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared",
                               "-fPIC", _SRC, "-o", tmp, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        c_void_p, c_size_t, c_int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        for name in ("oracle_sort_keys",):
            getattr(lib, name).argtypes = [c_int, c_void_p, c_size_t]
            getattr(lib, name).restype = c_int
        for name in ("oracle_sort_pairs", "oracle_insertion_sort", "oracle_brute_sort"):
            getattr(lib, name).argtypes = [c_int, c_void_p, c_void_p, c_size_t]
            getattr(lib, name).restype = c_int
        lib.oracle_sort_segmented.argtypes = [c_int, c_void_p, c_void_p, c_void_p, c_size_t]
        lib.oracle_sort_segmented.restype = c_int
        lib.oracle_sort_lists.argtypes = [c_void_p, c_size_t, c_size_t]
        lib.oracle_sort_keys_parallel.argtypes = [c_int, c_void_p, c_size_t, c_int]
        lib.oracle_sort_keys_parallel.restype = c_int
        lib.oracle_sort_lists.restype = c_int
        for name in ("oracle_run", "oracle_ascents", "oracle_inv", "oracle_mono"):
            getattr(lib, name).argtypes = [c_int, c_void_p, c_size_t]
            getattr(lib, name).restype = ctypes.c_int64
        _lib = lib
    return _lib


def _dt(a: np.ndarray) -> int:
    name = a.dtype.name
    if name not in DTYPES:
        raise TypeError(f"oracle: unsupported dtype {name}")
    return DTYPES[name]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle: {what} rejected its arguments")


def sort_keys(keys: np.ndarray) -> np.ndarray:
    """Stable top-down mergesort of keys (the unique sorted permutation)."""
    out = np.ascontiguousarray(keys).copy()
    _check(_load().oracle_sort_keys(_dt(out), _ptr(out), out.size), "sort_keys")
    return out


def sort_keys_parallel(keys: np.ndarray, threads: int) -> np.ndarray:
    """The same mergesort on `threads` host threads (a power of two is used);
    for timing a CPU baseline only -- tests compare it with sort_keys."""
    out = np.ascontiguousarray(keys).copy()
    _check(_load().oracle_sort_keys_parallel(_dt(out), _ptr(out), out.size, int(threads)),
           "sort_keys_parallel")
    return out


def sort_pairs(keys: np.ndarray, payload: np.ndarray):
    """Stable mergesort of (key, uint32 payload) records; returns (keys, payload)."""
    k = np.ascontiguousarray(keys).copy()
    p = np.ascontiguousarray(payload, dtype=np.uint32).copy()
    assert k.size == p.size
    _check(_load().oracle_sort_pairs(_dt(k), _ptr(k), _ptr(p), k.size), "sort_pairs")
    return k, p


def sort_segmented(keys: np.ndarray, offsets: np.ndarray, payload: np.ndarray | None = None):
    """Each CSR segment [offsets[s], offsets[s+1]) sorted on its own."""
    k = np.ascontiguousarray(keys).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    _check(_load().oracle_sort_segmented(_dt(k), _ptr(k), _ptr(p), _ptr(off), off.size - 1),
           "sort_segmented")
    return k if p is None else (k, p)


def sort_lists(lists: np.ndarray) -> np.ndarray:
    """Stable mergesort of the rows of an (n, L) int32 array, compared word by
    word from the first (the heavy list items of Sec. 2)."""
    a = np.ascontiguousarray(lists, dtype=np.int32).copy()
    assert a.ndim == 2 and a.shape[1] >= 1
    _check(_load().oracle_sort_lists(_ptr(a), a.shape[0], a.shape[1]), "sort_lists")
    return a


def insertion_sort(keys: np.ndarray, payload: np.ndarray | None = None):
    """The paper's stable insertion sort (shift while strictly greater)."""
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    _check(_load().oracle_insertion_sort(_dt(k), _ptr(k), _ptr(p), k.size), "insertion_sort")
    return k if p is None else (k, p)


def brute_sort(keys: np.ndarray, payload: np.ndarray | None = None):
    """O(n^2) definition: output p takes the least remaining (key, index)."""
    k = np.ascontiguousarray(keys).copy()
    p = None if payload is None else np.ascontiguousarray(payload, dtype=np.uint32).copy()
    _check(_load().oracle_brute_sort(_dt(k), _ptr(k), _ptr(p), k.size), "brute_sort")
    return k if p is None else (k, p)


def run(keys: np.ndarray) -> int:
    """Run(A) = #descents + 1 (0 for an empty array)."""
    k = np.ascontiguousarray(keys)
    return int(_load().oracle_run(_dt(k), _ptr(k), k.size))


def ascents(keys: np.ndarray) -> int:
    k = np.ascontiguousarray(keys)
    return int(_load().oracle_ascents(_dt(k), _ptr(k), k.size))


def inv(keys: np.ndarray) -> int:
    """Inv(A): number of pairs i < j with a_i > a_j (O(n^2))."""
    k = np.ascontiguousarray(keys)
    return int(_load().oracle_inv(_dt(k), _ptr(k), k.size))


def mono(keys: np.ndarray) -> int:
    """Mono(A): least number of monotone contiguous pieces."""
    k = np.ascontiguousarray(keys)
    return int(_load().oracle_mono(_dt(k), _ptr(k), k.size))
