"""Thin ctypes binding of libsortrace.so (argument marshalling only).

Every sort runs in the HIP kernels of ``libsortrace.so``; this module only
passes device pointers, sizes and the torch stream handle through the C ABI
declared in ``include/sortrace.h``.  There is no fallback: if the library is
missing, ``load()`` raises.

Tensors must be CUDA (HIP) tensors, contiguous.  int32 and float32 tensors
map to SR_INT32 / SR_FLOAT32; uint64 keys are passed as torch.uint64 or as an
int64 tensor with ``dtype="uint64"`` (same bits).  Payloads are int32 or
uint32 tensors carrying uint32 values.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsortrace.so")
# Launch-shape table measured by the package's autotuner on gfx950; applied
# when the library loads unless SR_TUNE_TABLE names another file or "none".
TUNE_TABLE = os.path.join(_HERE, "tune_gfx950.json")

SR_INT32, SR_UINT64, SR_FLOAT32 = 0, 1, 2
DTYPES = {"int32": SR_INT32, "uint64": SR_UINT64, "float32": SR_FLOAT32}
PATHS = {-1: "trivial", 0: "sorted", 1: "reversed", 2: "outlier", 3: "general", 4: "runs", 5: "few", 6: "near"}
STATUS = {0: "SR_OK", 1: "SR_ERR_INVALID_ARGUMENT", 2: "SR_ERR_UNSUPPORTED",
          3: "SR_ERR_OUT_OF_MEMORY", 4: "SR_ERR_DEVICE", 5: "SR_ERR_INTERNAL"}

# Every symbol include/sortrace.h declares.
EXPORTS = ("sr_sort_keys", "sr_sort_pairs", "sr_sort_segmented", "sr_sort_batch", "sr_reserve",
           "sr_release_stream", "sr_measure", "sr_workspace_bytes", "sr_last_stats", "sr_status_str",
           "sr_last_error_message", "sr_set_option", "sr_profile_collect", "sr_copy_bandwidth_probe",
           "sr_server_create", "sr_server_submit", "sr_server_now", "sr_server_wait_idle",
           "sr_server_records", "sr_server_destroy", "sr_tune_set", "sr_tune_get",
           "sr_measure_presortedness", "sr_sort_lists", "sr_set_workspace", "sr_sort_keys_noalloc")
SR_MEASURE_INV = 1

# Fields of a tuning-table row (sr_tune_entry) and their "unset" values.
TUNE_FIELDS = ("tile_variant", "merge_items", "partition", "nontemporal", "fan_in")
TUNE_UNSET = {"tile_variant": -1, "merge_items": 0, "partition": -1, "nontemporal": -1, "fan_in": 0}


class SrStats(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("passes", ctypes.c_int32), ("n", ctypes.c_int64),
                ("descents", ctypes.c_int64), ("outliers", ctypes.c_int64),
                ("bytes_moved", ctypes.c_double), ("run_leaves", ctypes.c_int64),
                ("merge_passes", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SrServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("streams", ctypes.c_int),
                ("max_batch_requests", ctypes.c_int), ("max_batch_keys", ctypes.c_size_t)]


class SrRequestRecord(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("dtype", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("n", ctypes.c_int64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class SrTuneEntry(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("pairs", ctypes.c_int32), ("min_n", ctypes.c_int64),
                ("tile_variant", ctypes.c_int32), ("merge_items", ctypes.c_int32),
                ("partition", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("segmented", ctypes.c_int32), ("fan_in", ctypes.c_int32)]


class SrPresortedness(ctypes.Structure):
    _fields_ = [("descents", ctypes.c_int64), ("ascents", ctypes.c_int64), ("run", ctypes.c_int64),
                ("mono", ctypes.c_int64), ("inv", ctypes.c_int64)]


class SortraceError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} ({detail})")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libsortrace.so (torch first, so its HIP runtime is the one used)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the process's HIP runtime)
    if not os.path.exists(path):
        raise RuntimeError(f"libsortrace.so is not built ({path}); run "
                           "`python -m paper_1609_04471_amd.build`")
    lib = ctypes.CDLL(path)
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int64
    lib.sr_sort_keys.argtypes = [i32, vp, sz, vp]
    lib.sr_sort_keys_noalloc.argtypes = [i32, vp, sz, vp]
    lib.sr_sort_pairs.argtypes = [i32, vp, vp, sz, vp]
    lib.sr_sort_segmented.argtypes = [i32, vp, vp, sz, vp, sz, vp]
    lib.sr_measure.argtypes = [i32, vp, sz, ctypes.POINTER(ctypes.c_int64), vp]
    lib.sr_workspace_bytes.argtypes = [i32, i32, sz, sz, ctypes.POINTER(ctypes.c_size_t)]
    lib.sr_last_stats.argtypes = [vp, ctypes.POINTER(SrStats)]
    lib.sr_status_str.argtypes = [i32]
    lib.sr_status_str.restype = ctypes.c_char_p
    lib.sr_last_error_message.argtypes = []
    lib.sr_last_error_message.restype = ctypes.c_char_p
    lib.sr_set_option.argtypes = [ctypes.c_char_p, i64]
    lib.sr_profile_collect.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]
    lib.sr_copy_bandwidth_probe.argtypes = [vp, vp, sz, vp]
    lib.sr_sort_batch.argtypes = [i32, vp, vp, sz, sz, vp]
    lib.sr_reserve.argtypes = [i32, sz, sz, vp]
    lib.sr_release_stream.argtypes = [vp]
    lib.sr_set_workspace.argtypes = [vp, sz, vp]
    lib.sr_server_create.argtypes = [ctypes.POINTER(SrServerConfig), ctypes.POINTER(vp)]
    lib.sr_server_submit.argtypes = [vp, i32, vp, sz, ctypes.c_uint64, ctypes.c_double, vp]
    lib.sr_server_now.argtypes = [vp]
    lib.sr_server_wait_idle.argtypes = [vp, ctypes.c_double]
    lib.sr_server_records.argtypes = [vp, ctypes.POINTER(SrRequestRecord), sz, ctypes.POINTER(sz)]
    lib.sr_server_destroy.argtypes = [vp]
    lib.sr_sort_lists.argtypes = [vp, sz, ctypes.c_int32, vp]
    lib.sr_measure_presortedness.argtypes = [i32, vp, sz, ctypes.c_int32, ctypes.POINTER(SrPresortedness), vp]
    lib.sr_tune_set.argtypes = [ctypes.POINTER(SrTuneEntry), i64]
    lib.sr_tune_get.argtypes = [ctypes.POINTER(SrTuneEntry), i64, ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTS:
        if name not in ("sr_status_str", "sr_last_error_message"):
            getattr(lib, name).restype = i32
    lib.sr_server_now.restype = ctypes.c_double
    _lib = lib
    table = os.environ.get("SR_TUNE_TABLE")
    if table is None and os.path.exists(TUNE_TABLE):
        table = TUNE_TABLE
    if table and table != "none":
        from . import autotune
        autotune.apply(table)
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        msg = _lib.sr_last_error_message().decode(errors="replace")
        raise SortraceError(rc, what, msg)


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _key_dtype(t, dtype: str | None) -> int:
    import torch
    if dtype is not None:
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        want = {"int32": 4, "float32": 4, "uint64": 8}[dtype]
        if t.element_size() != want:
            raise ValueError(f"{dtype} keys need {want}-byte elements, got {t.dtype}")
        return DTYPES[dtype]
    if t.dtype == torch.int32:
        return SR_INT32
    if t.dtype == torch.float32:
        return SR_FLOAT32
    if t.dtype == getattr(torch, "uint64", None):
        return SR_UINT64
    raise ValueError(f"key dtype {t.dtype} needs an explicit dtype= (int32, uint64, float32)")


def _dev(t, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


def sort_keys(keys, dtype: str | None = None, stream=None):
    """Sort ``keys`` in place (ascending; float32 by totalOrder). Returns keys."""
    lib = load()
    dt = _key_dtype(keys, dtype)
    _check(lib.sr_sort_keys(dt, _dev(keys, "keys"), keys.numel(), _stream(stream)), "sr_sort_keys")
    return keys


def sort_keys_noalloc(keys, dtype: str | None = None, stream=None):
    """sort_keys through the allocation-free entry point (one fixed scratch
    array per device, shared by every call: order overlapping calls on one
    stream).  Returns keys."""
    lib = load()
    dt = _key_dtype(keys, dtype)
    _check(lib.sr_sort_keys_noalloc(dt, _dev(keys, "keys"), keys.numel(), _stream(stream)),
           "sr_sort_keys_noalloc")
    return keys


def sort_pairs(keys, payload, dtype: str | None = None, stream=None):
    """Stable in-place sort of (key, uint32 payload). Returns (keys, payload)."""
    lib = load()
    dt = _key_dtype(keys, dtype)
    if payload.numel() != keys.numel() or payload.element_size() != 4:
        raise ValueError("payload must hold one 4-byte value per key")
    _check(lib.sr_sort_pairs(dt, _dev(keys, "keys"), _dev(payload, "payload"), keys.numel(),
                             _stream(stream)), "sr_sort_pairs")
    return keys, payload


def sort_segmented(keys, offsets, payload=None, dtype: str | None = None, stream=None):
    """Sort every CSR segment [offsets[s], offsets[s+1]) of keys in place."""
    import torch
    lib = load()
    dt = _key_dtype(keys, dtype)
    if offsets.dtype != torch.int64:
        raise ValueError("offsets must be int64")
    pp = None
    if payload is not None:
        if payload.numel() != keys.numel() or payload.element_size() != 4:
            raise ValueError("payload must hold one 4-byte value per key")
        pp = _dev(payload, "payload")
    nseg = offsets.numel() - 1
    _check(lib.sr_sort_segmented(dt, _dev(keys, "keys"), pp, keys.numel(), _dev(offsets, "offsets"),
                                 max(nseg, 0), _stream(stream)), "sr_sort_segmented")
    return keys if payload is None else (keys, payload)


def measure(keys, dtype: str | None = None, stream=None):
    """(descents, ascents) of keys; Run(A) = descents + 1.  Synchronizes."""
    lib = load()
    out = (ctypes.c_int64 * 2)()
    _check(lib.sr_measure(_key_dtype(keys, dtype), _dev(keys, "keys"), keys.numel(), out,
                          _stream(stream)), "sr_measure")
    return int(out[0]), int(out[1])


def sort_lists(lists, stream=None):
    """Sort the rows of a 2-D int32 GPU tensor (n lists of `words` ints) in
    place, word by word from the first, stable.  Synchronizes."""
    import torch
    if lists.dim() != 2 or lists.dtype != torch.int32:
        raise ValueError("lists must be a 2-D int32 tensor")
    lib = load()
    _check(lib.sr_sort_lists(_dev(lists, "lists"), lists.shape[0], lists.shape[1], _stream(stream)),
           "sr_sort_lists")
    return lists


def presortedness(keys, dtype: str | None = None, inv: bool = False, stream=None) -> dict:
    """Run, Mono (and Inv when asked) of keys, with descents and ascents.
    inv is -1 unless asked for.  Synchronizes."""
    lib = load()
    out = SrPresortedness()
    _check(lib.sr_measure_presortedness(_key_dtype(keys, dtype), _dev(keys, "keys"), keys.numel(),
                                        SR_MEASURE_INV if inv else 0, ctypes.byref(out), _stream(stream)),
           "sr_measure_presortedness")
    return {f: int(getattr(out, f)) for f, _ in SrPresortedness._fields_}


def last_stats(stream=None) -> dict:
    """Path, passes and bytes of the last sort on the stream.  Synchronizes."""
    lib = load()
    s = SrStats()
    _check(lib.sr_last_stats(_stream(stream), ctypes.byref(s)), "sr_last_stats")
    return {"path": PATHS.get(s.path, s.path), "passes": s.passes, "n": s.n,
            "descents": s.descents, "outliers": s.outliers, "bytes_moved": s.bytes_moved,
            "run_leaves": s.run_leaves, "merge_passes": s.merge_passes}


def workspace_bytes(dtype: str, with_payload: bool, n: int, nseg: int = 0) -> int:
    lib = load()
    b = ctypes.c_size_t()
    _check(lib.sr_workspace_bytes(DTYPES[dtype], int(with_payload), n, nseg, ctypes.byref(b)),
           "sr_workspace_bytes")
    return b.value


def set_workspace(buf, stream=None) -> None:
    """Use the caller's device tensor `buf` (256-byte aligned, >= 1 MiB) as
    the data scratch of `stream`; None gives the scratch back to the
    library.  The tensor must outlive every call that uses it."""
    lib = load()
    if buf is None:
        _check(lib.sr_set_workspace(None, 0, _stream(stream)), "sr_set_workspace")
    else:
        _check(lib.sr_set_workspace(_dev(buf, "workspace"), buf.numel() * buf.element_size(),
                                    _stream(stream)), "sr_set_workspace")


def set_option(name: str, value: int) -> None:
    lib = load()
    _check(lib.sr_set_option(name.encode(), int(value)), "sr_set_option")


def tune_set(rows) -> None:
    """Replace the tuning table.  rows: dicts with dtype ("int32", "uint64",
    "float32"), pairs (bool), segmented (bool, default False), min_n and any of
    TUNE_FIELDS (missing = unset)."""
    lib = load()
    buf = (SrTuneEntry * max(1, len(rows)))()
    for i, r in enumerate(rows):
        e = buf[i]
        e.dtype = DTYPES[r["dtype"]]
        e.pairs = int(bool(r.get("pairs", False)))
        e.segmented = int(bool(r.get("segmented", False)))
        e.min_n = int(r.get("min_n", 0))
        for f in TUNE_FIELDS:
            setattr(e, f, int(r.get(f, TUNE_UNSET[f])))
    _check(lib.sr_tune_set(buf, len(rows)), "sr_tune_set")


def tune_get() -> list:
    """The tuning table as a list of dicts (sorted by dtype, pairs, segmented, min_n)."""
    lib = load()
    cnt = ctypes.c_int64()
    _check(lib.sr_tune_get(None, 0, ctypes.byref(cnt)), "sr_tune_get")
    buf = (SrTuneEntry * max(1, cnt.value))()
    _check(lib.sr_tune_get(buf, cnt.value, ctypes.byref(cnt)), "sr_tune_get")
    names = {v: k for k, v in DTYPES.items()}
    return [{"dtype": names[e.dtype], "pairs": bool(e.pairs), "segmented": bool(e.segmented), "min_n": e.min_n,
             **{f: getattr(e, f) for f in TUNE_FIELDS}} for e in buf[:cnt.value]]


def profile_collect(prefix: str = ""):
    """(launches, total_ms) of recorded kernels whose name starts with prefix."""
    lib = load()
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib.sr_profile_collect(prefix.encode(), ctypes.byref(n), ctypes.byref(ms)),
           "sr_profile_collect")
    return n.value, ms.value


def copy_probe(dst, src, stream=None) -> None:
    lib = load()
    nbytes = src.numel() * src.element_size()
    _check(lib.sr_copy_bandwidth_probe(_dev(dst, "dst"), _dev(src, "src"), nbytes, _stream(stream)),
           "sr_copy_bandwidth_probe")


def sort_batch(arrays, dtype: str | None = None, stream=None):
    """Sort every tensor of ``arrays`` in place, all in one batch of launches."""
    import torch
    lib = load()
    arrays = [a for a in arrays if a.numel() > 0]
    if not arrays:
        return
    dt = _key_dtype(arrays[0], dtype)
    dev = arrays[0].device
    ptrs = torch.tensor([_dev(a, "array") for a in arrays], dtype=torch.int64, device=dev)
    lens = torch.tensor([a.numel() for a in arrays], dtype=torch.int64, device=dev)
    total = sum(a.numel() for a in arrays)
    _check(lib.sr_sort_batch(dt, ptrs.data_ptr(), lens.data_ptr(), len(arrays), total, _stream(stream)),
           "sr_sort_batch")
    return ptrs, lens  # keep the device arrays alive until the stream has used them


class Server:
    """Continuous-batching sort server (see sr_server_* in include/sortrace.h)."""

    def __init__(self, hbm_budget_bytes: int, streams: int = 4, max_batch_requests: int = 64,
                 max_batch_keys: int = 1 << 25):
        self._lib = load()
        cfg = SrServerConfig(hbm_budget_bytes, streams, max_batch_requests, max_batch_keys)
        h = ctypes.c_void_p()
        _check(self._lib.sr_server_create(ctypes.byref(cfg), ctypes.byref(h)), "sr_server_create")
        self._h = h
        self._events = {}

    def now(self) -> float:
        return self._lib.sr_server_now(self._h)

    def submit(self, keys, tag: int, t_arrive: float, dtype: str | None = None, ready="current"):
        """ready: "current" records an event on the current stream now, so the
        sort waits for work already queued there on the keys; None skips the
        wait; or a torch.cuda.Event the caller recorded."""
        import torch
        if isinstance(ready, str):
            ev = torch.cuda.Event()
            ev.record(torch.cuda.current_stream())
        else:
            ev = ready
        raw = None if ev is None else ctypes.c_void_p(ev.cuda_event)
        _check(self._lib.sr_server_submit(self._h, _key_dtype(keys, dtype), _dev(keys, "keys"), keys.numel(),
                                          tag, t_arrive, raw), "sr_server_submit")
        if ev is not None:
            self._events[tag] = ev   # kept alive until the request is reported finished

    def wait_idle(self, timeout_s: float = 60.0):
        _check(self._lib.sr_server_wait_idle(self._h, timeout_s), "sr_server_wait_idle")

    def records(self) -> list:
        out = []
        buf = (SrRequestRecord * 4096)()
        while True:
            cnt = ctypes.c_size_t()
            _check(self._lib.sr_server_records(self._h, buf, 4096, ctypes.byref(cnt)), "sr_server_records")
            for i in range(cnt.value):
                r = buf[i]
                self._events.pop(r.tag, None)
                out.append({"tag": r.tag, "dtype": r.dtype, "batch": r.batch, "n": r.n, "status": r.status,
                            "t_arrive": r.t_arrive, "t_admit": r.t_admit, "t_launch": r.t_launch,
                            "t_done": r.t_done})
            if cnt.value < 4096:
                return out

    def close(self):
        if self._h:
            self._lib.sr_server_destroy(self._h)
            self._h = None
        self._events = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
