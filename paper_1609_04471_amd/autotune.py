"""Autotuner for libsortrace's launch shapes.

For each key type (int32, uint64, float32), keys-only or pairs, and each
size band, the sweep times every valid combination of the launch-shape
fields of the tuning table (``sr_tune_entry`` in ``include/sortrace.h``)
on the device and keeps the fastest (or, when it is within a 2 % margin,
the previous band's choice, so that timing noise does not flip rows):

  partition     separate Merge Path partition launch + persistent merge grid
                (1), or each merge workgroup searching its own window (0);
  nontemporal   persistent merge with nontemporal window loads and stores;
  tile_variant  32-bit keys: 512 x 16 or 1024 x 8 threads x keys per tile;
  merge_items   32-bit keys, fused merge: 8 or 16 outputs per thread;
  fan_in        keys only, with the partition launch: unset (two-way passes)
                or 4 (four-way passes, each merging two levels of the merge
                tree in one read and one write of the array).

Segmented and batched sorts (rows with "segmented": true, looked up by the
total key count) are swept separately on the batched workload's mix --
log-uniform segment lengths in [16, 262144] -- over tile_variant and
merge_items (32-bit keys, keys only).

Pairs always merge two-way.  Inputs are uniform random keys of the band's size
(the case that runs every merge pass), generated on the device from a fixed
seed.  Every candidate's output is compared byte for byte with the output
under the built-in rules, so a table can only select among shapes that sort
identically.

The result is a JSON file::

    {"format": "sortrace-tune-1", "device": ..., "arch": ..., "rows": [
        {"dtype": "int32", "pairs": false, "min_n": 0, "tile_variant": 1,
         "merge_items": 8, "partition": 0, "nontemporal": 0,
         "measured_n": 65536, "ms": ..., "builtin_ms": ...}, ...]}

``apply(path)`` loads such a file into the library (``sr_tune_set``); the
binding also applies the file named by the environment variable
``SR_TUNE_TABLE`` when it loads the library.  Run the sweep with::

    python -m paper_1609_04471_amd.autotune --out tune.json
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import sys

FORMAT = "sortrace-tune-1"
KEY_BYTES = {"int32": 4, "uint64": 8, "float32": 4}


def candidates(dtype: str, pairs: bool) -> list:
    """Every distinct launch shape of (dtype, pairs); fields that do not
    apply to a combination are left out of it."""
    out = []
    wide = KEY_BYTES[dtype] == 4 and not pairs  # tile_variant / merge_items apply
    tiles = (0, 1) if wide else (None,)
    for tile, part in itertools.product(tiles, (0, 1)):
        extra = ({"merge_items": m} for m in ((8, 16) if wide else (None,))) if part == 0 else \
            ({"nontemporal": t, **f} for t in (0, 1) for f in (({},) if pairs else ({}, {"fan_in": 4})))
        for e in extra:
            c = {"partition": part}
            if tile is not None:
                c["tile_variant"] = tile
            c.update({k: v for k, v in e.items() if v is not None})
            out.append(c)
    return out


def band_sizes(dtype: str, pairs: bool, lo: int = 16, hi: int = 28, step: int = 2) -> list:
    return [1 << b for b in range(lo, hi + 1, step)]


def band_starts(sizes: list) -> list:
    """Row start of each measured size: 0 for the first, else the geometric
    midpoint between it and the previous measured size."""
    return [0] + [int(round(math.sqrt(a * b))) for a, b in zip(sizes, sizes[1:])]


def compress(rows: list) -> list:
    """Drop rows whose fields equal the previous row of the same kind."""
    from .sortrace import TUNE_FIELDS
    out = []
    for r in rows:
        p = out[-1] if out else None
        if p and (p["dtype"], p["pairs"], p.get("segmented", False)) == \
                (r["dtype"], r["pairs"], r.get("segmented", False)) and \
                all(p.get(f) == r.get(f) for f in TUNE_FIELDS):
            continue
        out.append(r)
    return out


def validate(table: dict) -> list:
    """Rows of a tuning file, checked for format and field names."""
    from .sortrace import DTYPES, TUNE_FIELDS
    if table.get("format") != FORMAT:
        raise ValueError(f"not a {FORMAT} table")
    rows = []
    for r in table["rows"]:
        if r["dtype"] not in DTYPES:
            raise ValueError(f"bad dtype {r['dtype']!r}")
        rows.append({"dtype": r["dtype"], "pairs": bool(r["pairs"]), "segmented": bool(r.get("segmented", False)),
                     "min_n": int(r["min_n"]), **{f: int(r[f]) for f in TUNE_FIELDS if f in r}})
    return rows


def apply(path: str) -> list:
    """Load a tuning file into the library; returns its rows."""
    from . import sortrace
    with open(path) as f:
        rows = validate(json.load(f))
    sortrace.tune_set(rows)
    return rows


def _random_keys(dtype: str, n: int, seed: int, device):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    if dtype == "uint64":
        return torch.randint(-(1 << 63), (1 << 63) - 1, (n,), dtype=torch.int64, device=device, generator=g)
    bits = torch.randint(-(1 << 31), (1 << 31) - 1, (n,), dtype=torch.int32, device=device, generator=g)
    if dtype == "float32":
        # finite floats of every sign and exponent: clear one exponent bit
        bits = bits & 0x7F7FFFFF | (bits & -0x80000000)
        return bits.view(torch.float32)
    return bits


def time_shape(dtype: str, pairs: bool, src, psrc, shape, reps: int, stream):
    """Median ms of `reps` sorts of copies of src under one table row
    (shape None = no table), and the last output."""
    import torch
    from . import sortrace
    sortrace.tune_set([] if shape is None else [{"dtype": dtype, "pairs": pairs, "min_n": 0, **shape}])
    keys = torch.empty_like(src)
    pay = torch.empty_like(psrc) if pairs else None
    times = []
    with torch.cuda.stream(stream):
        for i in range(reps + 1):
            keys.copy_(src)
            if pairs:
                pay.copy_(psrc)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            if pairs:
                sortrace.sort_pairs(keys, pay, dtype=dtype, stream=stream)
            else:
                sortrace.sort_keys(keys, dtype=dtype, stream=stream)
            b.record(stream)
            b.synchronize()
            if i:  # the first sort allocates the workspace
                times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2], keys, pay


def pick(timed: list, prev: dict | None, margin: float):
    """The fastest (ms, shape) of `timed`, unless the shape of the previous
    band (or, for the first band, the first candidate) is within `margin`
    of it: then that one, so that timing noise does not flip a row."""
    from .sortrace import TUNE_FIELDS
    best = min(timed, key=lambda t: t[0])
    if prev is not None:
        ref = [t for t in timed if all(t[1].get(f) == prev.get(f) for f in TUNE_FIELDS)]
    else:
        ref = timed[:1]
    if ref and ref[0][0] <= best[0] * (1 + margin):
        return ref[0]
    return best


def sweep(dtypes=("int32", "uint64", "float32"), kinds=(False, True), lo=16, hi=28, step=2, reps=5,
          seed=1234, margin=0.02, log=print) -> dict:
    import torch
    from . import sortrace
    sortrace.load()
    for name, auto in (("partition_min_n", -1), ("tile_variant", -1), ("merge_items", 0),
                       ("merge_nontemporal", -1)):
        sortrace.set_option(name, auto)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    old = sortrace.tune_get()
    rows = []
    try:
        for dtype, pairs in itertools.product(dtypes, kinds):
            sizes = band_sizes(dtype, pairs, lo, hi, step)
            for n, start in zip(sizes, band_starts(sizes)):
                src = _random_keys(dtype, n, seed + n, dev)
                psrc = torch.arange(n, dtype=torch.int32, device=dev) if pairs else None
                torch.cuda.synchronize()
                builtin_ms, ref, refp = time_shape(dtype, pairs, src, psrc, None, reps, stream)
                timed = []
                for shape in candidates(dtype, pairs):
                    ms, out, outp = time_shape(dtype, pairs, src, psrc, shape, reps, stream)
                    same = torch.equal(out, ref) and (not pairs or torch.equal(outp, refp))
                    if not same:
                        raise RuntimeError(f"{dtype} pairs={pairs} n={n} {shape}: output differs")
                    timed.append((ms, shape))
                    del out, outp
                prev = rows[-1] if rows and (rows[-1]["dtype"], rows[-1]["pairs"]) == (dtype, pairs) else None
                best = pick(timed, prev, margin)
                row = {"dtype": dtype, "pairs": pairs, "min_n": start, **best[1], "measured_n": n,
                       "ms": round(best[0], 5), "builtin_ms": round(builtin_ms, 5)}
                log(f"[autotune] {dtype:7s} pairs={int(pairs)} n=2^{int(math.log2(n))}: {best[1]} "
                    f"{best[0]:.4f} ms (built-in {builtin_ms:.4f} ms)")
                rows.append(row)
                del src, psrc, ref, refp
                torch.cuda.empty_cache()
    finally:
        sortrace.tune_set(old)
    props = torch.cuda.get_device_properties(dev)
    return {"format": FORMAT, "device": props.name, "arch": getattr(props, "gcnArchName", ""),
            "reps": reps, "seed": seed, "margin": margin, "rows": rows}


def seg_candidates(dtype: str) -> list:
    """Launch shapes of segmented / batched sorts: 32-bit keys only."""
    if KEY_BYTES[dtype] != 4:
        return []
    return [{"tile_variant": t, "merge_items": m} for t in (0, 1) for m in (8, 16)]


def _segment_offsets(total: int, seed: int, lo: int = 16, hi: int = 262144):
    """CSR offsets of log-uniform segment lengths in [lo, hi] (the batched-sort
    workload's mix) summing to `total` (the last segment is cut)."""
    import numpy as np
    from . import inputs
    lens, got, k = [], 0, 0
    while got < total:
        for L in inputs.segment_lengths(256, seed + k, lo, hi):
            L = int(min(L, total - got))
            lens.append(L)
            got += L
            if got >= total:
                break
        k += 1
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    return off


def time_seg_shape(dtype: str, src, off, shape, reps: int, stream):
    import torch
    from . import sortrace
    sortrace.tune_set([] if shape is None else
                      [{"dtype": dtype, "pairs": False, "segmented": True, "min_n": 0, **shape}])
    keys = torch.empty_like(src)
    times = []
    with torch.cuda.stream(stream):
        for i in range(reps + 1):
            keys.copy_(src)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            sortrace.sort_segmented(keys, off, dtype=dtype, stream=stream)
            b.record(stream)
            b.synchronize()
            if i:
                times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2], keys


def sweep_segmented(dtypes=("int32", "float32"), lo=20, hi=26, step=2, reps=5, seed=4321, margin=0.02,
                    log=print) -> list:
    """Rows for segmented / batched sorts: per dtype and total-size band, the
    fastest tile shape and merge outputs per thread on the log-uniform
    segment mix, each output checked against the built-in shape's."""
    import torch
    from . import sortrace
    sortrace.load()
    for name, auto in (("tile_variant", -1), ("merge_items", 0)):
        sortrace.set_option(name, auto)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    old = sortrace.tune_get()
    rows = []
    try:
        for dtype in dtypes:
            sizes = [1 << b for b in range(lo, hi + 1, step)]
            for n, start in zip(sizes, band_starts(sizes)):
                src = _random_keys(dtype, n, seed + n, dev)
                off = torch.from_numpy(_segment_offsets(n, seed + n)).to(dev)
                torch.cuda.synchronize()
                builtin_ms, ref = time_seg_shape(dtype, src, off, None, reps, stream)
                timed = []
                for shape in seg_candidates(dtype):
                    ms, out = time_seg_shape(dtype, src, off, shape, reps, stream)
                    if not torch.equal(out, ref):
                        raise RuntimeError(f"segmented {dtype} n={n} {shape}: output differs")
                    timed.append((ms, shape))
                    del out
                prev = rows[-1] if rows and rows[-1]["dtype"] == dtype else None
                best = pick(timed, prev, margin)
                rows.append({"dtype": dtype, "pairs": False, "segmented": True, "min_n": start, **best[1],
                             "measured_n": n, "segments": int(off.numel() - 1), "ms": round(best[0], 5),
                             "builtin_ms": round(builtin_ms, 5)})
                log(f"[autotune] segmented {dtype:7s} n=2^{int(math.log2(n))} ({off.numel() - 1} segments): "
                    f"{best[1]} {best[0]:.4f} ms (built-in {builtin_ms:.4f} ms)")
                del src, off, ref
                torch.cuda.empty_cache()
    finally:
        sortrace.tune_set(old)
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--dtypes", default="int32,uint64,float32")
    ap.add_argument("--kinds", default="keys,pairs")
    ap.add_argument("--lo", type=int, default=16, help="log2 of the smallest measured size")
    ap.add_argument("--hi", type=int, default=28, help="log2 of the largest measured size")
    ap.add_argument("--step", type=int, default=2)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--margin", type=float, default=0.02,
                    help="keep the previous band's shape when it is within this fraction of the best")
    ap.add_argument("--keep-all", action="store_true", help="keep rows equal to the previous one")
    ap.add_argument("--segmented-into", default=None, metavar="TABLE",
                    help="sweep only the segmented / batched rows (total sizes 2^20 .. 2^26) and write them "
                         "with the plain rows of TABLE")
    a = ap.parse_args(argv)
    say = lambda s: print(s, flush=True)  # noqa: E731
    if a.segmented_into:
        with open(a.segmented_into) as f:
            table = json.load(f)
        validate(table)
        seg = sweep_segmented(reps=a.reps, margin=a.margin, log=say)
        table["rows"] = [r for r in table["rows"] if not r.get("segmented", False)] + \
            (seg if a.keep_all else compress(seg))
    else:
        kinds = tuple({"keys": False, "pairs": True}[k] for k in a.kinds.split(","))
        table = sweep(tuple(a.dtypes.split(",")), kinds, a.lo, a.hi, a.step, a.reps, margin=a.margin, log=say)
        table["rows"] += sweep_segmented(reps=a.reps, margin=a.margin, log=say)
        if not a.keep_all:
            table["rows"] = compress(table["rows"])
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(f"[autotune] wrote {len(table['rows'])} rows to {a.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
