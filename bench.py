"""Benchmark of libsortrace on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-big] [--no-cpu]

Workload (the step): plain in-place int32 sorts of n = 2,000,000 keys, one of
each of the four input types of Table 1 of the Sort Race paper (random,
reversely sorted, nearly sorted, few unique), inputs already resident in HBM.
``value`` is the aggregate Mkeys/s over the K timed steps (4 x 2M keys each).

Besides the JSON fields of the contract the line carries:
  per_type_2M / per_type_256M   Mkeys/s, path and passes per input type
  roofline      the dominant kernel (merge pass) on 256M random int32 keys:
                algorithmic bytes per launch (2 x n x 4) / mean launch time
                measured with HIP events on the launch stream, against 8 TB/s
  copy_GBps     a 16-byte copy kernel's rate in the same run (practical peak)
  cpu_baseline  the CPU oracle (single thread) on a bounded sample of the
                same workload
Data is synthetic (seeded generators in paper_1609_04471_amd.inputs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mkeys/s int32 sort at n=2M (4 input types), %HBM roofline; batched p99 ms"
PEAK_HBM_GBPS = 8000.0
N_SMALL = 2_000_000
N_BIG = 268_435_456


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Hash of the device code: the two device headers and the kernel half of
    sr_engine.hip (everything before its host-side marker)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1609_04471_amd", "csrc")
    for f in ("sr_device.hpp", "sr_kernels.hpp"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    eng = open(os.path.join(csrc, "sr_engine.hip"), "rb").read()
    cut = eng.find(b"\n// Host side\n")
    if cut < 0:
        raise RuntimeError("sr_engine.hip has lost its host-side marker")
    h.update(eng[:cut])
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_sha") != kernel_source_sha():
        return None
    return e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=10, help="timed reps per type at 256M")
    ap.add_argument("--no-big", action="store_true", help="skip the n=256M section")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-seg", action="store_true", help="skip the batched-segments section")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-classes", action="store_true", help="skip the Sec. 2 presorted-class section")
    ap.add_argument("--no-configs", action="store_true", help="skip the 2^20 keys and 2^24 pairs section")
    ap.add_argument("--no-lists", action="store_true", help="skip the heavy list items section")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--only", choices=["small", "big-random", "big-reversed", "big-nearly", "big-few", "seg", "serve",
                                       "classes", "configs", "lists", "comparisons"],
                    default=None,
                    help="run one section only (for profiler runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: libsortrace sorts on one GPU; runs over several GPUs are not supported "
              "(a sharded sort would sort each GPU's share, exchange key ranges once at rank "
              "splitters and merge what each GPU receives).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1609_04471_amd import inputs, sortrace

    sortrace.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    types = list(inputs.TYPES)

    def host_input(kind, n):
        return inputs.int32_of_type(kind, n, inputs.seed_for(2, types.index(kind), n))

    result = {}

    # ------------------------------------------------------------ step: 4 x 2M
    if args.only in (None, "small"):
        log("generating 2M inputs")
        pristine = {k: torch.from_numpy(host_input(k, N_SMALL)).to(dev) for k in types}
        total_steps = args.warmup + args.steps

        def time_steps():
            """(gpu ms, wall s) of args.steps timed steps after the warmup."""
            bufs = [{k: pristine[k].clone() for k in types} for _ in range(total_steps)]
            torch.cuda.synchronize()
            for s in range(args.warmup):
                for k in types:
                    sortrace.sort_keys(bufs[s][k])
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            ev0.record(stream)
            for s in range(args.warmup, total_steps):
                for k in types:
                    sortrace.sort_keys(bufs[s][k])
            ev1.record(stream)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            # correctness of the timed outputs (cheap property: nondecreasing)
            for k in types:
                b = bufs[-1][k]
                assert bool((b[1:] >= b[:-1]).all()), k
            return ev0.elapsed_time(ev1), wall

        gpu_ms, wall = time_steps()
        ms_per_step = gpu_ms / args.steps
        value = args.steps * len(types) * N_SMALL / (gpu_ms / 1e3) / 1e6
        log(f"step: {ms_per_step:.4f} ms (wall {wall * 1e3 / args.steps:.4f} ms) -> {value:.1f} Mkeys/s")
        table = sortrace.tune_get()
        tuning = {"table": os.path.relpath(os.environ.get("SR_TUNE_TABLE", sortrace.TUNE_TABLE), ROOT)
                  if table else None, "rows": len(table)}
        if table:
            # the same step under the built-in launch-shape rules, for comparison
            sortrace.tune_set([])
            try:
                b_ms, _ = time_steps()
            finally:
                sortrace.tune_set(table)
            tuning["step_ms_builtin_rules"] = round(b_ms / args.steps, 5)
            log(f"step under the built-in shape rules: {b_ms / args.steps:.4f} ms")
        result["tuning"] = tuning

        per_small = {}
        for k in types:
            reps = 30
            work = [pristine[k].clone() for _ in range(reps + 3)]
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(reps)]
            torch.cuda.synchronize()
            for i in range(3):
                sortrace.sort_keys(work[i])
            for i in range(reps):
                evs[i][0].record(stream)
                sortrace.sort_keys(work[3 + i])
                evs[i][1].record(stream)
            torch.cuda.synchronize()
            times = [a.elapsed_time(b) for a, b in evs]
            st = sortrace.last_stats()
            med = statistics.median(times)
            per_small[k] = {"ms_median": round(med, 5), "ms_min": round(min(times), 5),
                            "Mkeys_s": round(N_SMALL / (med / 1e3) / 1e6, 1),
                            "path": st["path"], "passes": st["passes"]}
            log(f"2M {k}: {per_small[k]}")
            del work
        result.update(value=value, ms_per_step=ms_per_step, per_type_2M=per_small)
        del pristine

    # ------------------------------------------------------------ 256M section
    roofline = None
    per_big = {}
    copy_gbps = None
    if not args.no_big and (args.only is None or args.only.startswith("big-")):
        big_types = types if args.only is None else [args.only[4:]]
        work = torch.empty(N_BIG, dtype=torch.int32, device=dev)
        # bandwidth reference: 16-byte copy of 1 GiB
        src = torch.empty(N_BIG, dtype=torch.int32, device=dev)
        sortrace.copy_probe(src, work)
        torch.cuda.synchronize()
        cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
        for a, b in cev:
            a.record(stream)
            sortrace.copy_probe(src, work)
            b.record(stream)
        torch.cuda.synchronize()
        cms = statistics.median([a.elapsed_time(b) for a, b in cev])
        copy_gbps = 2 * N_BIG * 4 / (cms / 1e3) / 1e9
        log(f"copy16: {copy_gbps:.0f} GB/s")
        for k in big_types:
            log(f"generating 256M {k}")
            h = host_input(k, N_BIG)
            src.copy_(torch.from_numpy(h))
            del h
            times = []
            for i in range(args.reps + 1):
                work.copy_(src)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                sortrace.sort_keys(work)
                b.record(stream)
                torch.cuda.synchronize()
                if i > 0:
                    times.append(a.elapsed_time(b))
            st = sortrace.last_stats()
            assert bool((work[1:] >= work[:-1]).all()), k
            med = statistics.median(times)
            per_big[k] = {"ms_median": round(med, 4), "ms_min": round(min(times), 4),
                          "Mkeys_s": round(N_BIG / (med / 1e3) / 1e6, 1),
                          "path": st["path"], "passes": st["passes"],
                          "algorithmic_GBps": round(st["passes"] * 2 * N_BIG * 4 / (med / 1e3) / 1e9, 1)}
            log(f"256M {k}: {per_big[k]}")
            if k == "random":
                # per-kernel times with HIP events on the launch stream
                sortrace.set_option("profile", 1)
                sortrace.profile_collect("")
                for _ in range(3):
                    work.copy_(src)
                    sortrace.sort_keys(work)
                torch.cuda.synchronize()
                kern = {}
                for name in ("probe", "tile_sort", "partition", "merge"):
                    cnt, ms = sortrace.profile_collect(name)
                    kern[name] = (cnt, ms)
                sortrace.set_option("profile", 0)
                mcnt, mms = kern["merge"]
                avg_ms = mms / max(mcnt, 1)
                alg_bytes = 2 * N_BIG * 4
                achieved = alg_bytes / (avg_ms / 1e3) / 1e9
                tcnt, tms = kern["tile_sort"]
                roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                            "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4),
                            "traffic": measured_traffic("merge_int32_256M"),
                            "kernel": "merge pass (k_merge_persist int32, 256x16 outputs per workgroup, nontemporal)",
                            "workload": "int32 random n=268435456",
                            "launch_ms_mean": round(avg_ms, 5), "launches": mcnt,
                            "algorithmic_bytes_per_launch": alg_bytes,
                            "partition_ms_mean": round(kern["partition"][1] / max(kern["partition"][0], 1), 5),
                            "probe_ms_mean": round(kern["probe"][1] / max(kern["probe"][0], 1), 5),
                            "tile_sort_ms_mean": round(tms / max(tcnt, 1), 5),
                            "tile_sort_GBps": round(alg_bytes / (tms / max(tcnt, 1) / 1e3) / 1e9, 1)}
                log(f"roofline: {roofline}")
        del work, src
        torch.cuda.synchronize()
    result.update(per_type_256M=per_big or None, roofline=roofline, copy_GBps=round(copy_gbps, 1) if copy_gbps else None)

    # ------------------------------------------------------------ 2^20 keys, 2^24 pairs
    cfgs = None
    if not args.no_configs and args.only in (None, "configs"):
        cfgs = configs_section(torch, np, inputs, sortrace, dev, stream)
    result["configs"] = cfgs

    # ------------------------------------------------------------ heavy list items
    lists = None
    if not args.no_lists and args.only in (None, "lists"):
        lists = lists_section(torch, inputs, sortrace, dev)
    result["lists"] = lists

    # ------------------------------------------------------------ Sec. 2 classes
    classes = None
    if not args.no_classes and args.only in (None, "classes"):
        classes = classes_section(args, torch, np, inputs, sortrace, dev, stream)
    result["classes"] = classes

    # ------------------------------------------------------------ batched segments
    seg = None
    if not args.no_seg and args.only in (None, "seg"):
        log("generating 4096 segments")
        hk, hoff, kinds = inputs.segments_int32(4096, seed=inputs.seed_for(4, 0, 0))
        nseg = hoff.size - 1
        pristine = torch.from_numpy(hk).to(dev)
        off = torch.from_numpy(hoff).to(dev)
        work = torch.empty_like(pristine)
        ntot = int(hoff[-1])

        def timed(fn, reps):
            out = []
            for _ in range(reps):
                work.copy_(pristine)
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                a.record(stream)
                fn()
                b.record(stream)
                torch.cuda.synchronize()
                out.append((a.elapsed_time(b), (time.perf_counter() - t0) * 1e3))
            return out

        sortrace.set_option("graph", 1)
        timed(lambda: sortrace.sort_segmented(work, off), 2)        # capture + warm-up
        bt = timed(lambda: sortrace.sort_segmented(work, off), 10)
        sortrace.set_option("graph", 0)
        batched = work.clone()
        views = [work[int(hoff[i]):int(hoff[i + 1])] for i in range(nseg)]

        def plain():
            for v in views:
                if v.numel() > 1:
                    sortrace.sort_keys(v)
        timed(plain, 1)
        pt = timed(plain, 3)
        same = bool(torch.equal(work, batched))
        bms = statistics.median([x[0] for x in bt])
        pms = statistics.median([max(x) for x in pt])
        seg = {"segments": nseg, "keys": ntot,
               "batched_graph_ms": round(bms, 4),
               "batched_Mkeys_s": round(ntot / (bms / 1e3) / 1e6, 1),
               "plain_calls_ms": round(pms, 4),
               "plain_Mkeys_s": round(ntot / (pms / 1e3) / 1e6, 1),
               "speedup": round(pms / bms, 2), "identical_results": same}
        log(f"segments: {seg}")
        assert same
        del pristine, work, off, views, batched
        torch.cuda.synchronize()
    result["segmented"] = seg

    # ------------------------------------------------------------ serving
    serving = None
    if not args.no_serve and args.only in (None, "serve"):
        serving = serve_section(args, torch, np, inputs, sortrace, dev)
    result["serving"] = serving

    # ------------------------------------------------------------ CPU baseline
    cpu = None
    if not args.no_cpu and args.only is None:
        cpu = cpu_section(args, np, inputs, types, host_input)

    comparisons = None
    if not args.no_cpu and args.only in (None, "comparisons"):
        comparisons = comparisons_section(np, inputs, types, host_input)

    line = {
        "metric": METRIC,
        "value": round(result.get("value", 0.0), 1),
        "unit": "Mkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(result.get("ms_per_step", 0.0), 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain in-place int32 sort, n=2,000,000 keys, four input types "
                               "(random, reversed, nearly sorted, few unique), keys only",
                   "n": N_SMALL, "arrays_per_step": len(types), "types": types},
        "roofline": result.get("roofline"),
        "cpu_baseline": cpu,
        "per_type_2M": result.get("per_type_2M"),
        "per_type_256M": result.get("per_type_256M"),
        "copy_GBps": result.get("copy_GBps"),
        "segmented_4096": result.get("segmented"),
        "presorted_classes": result.get("classes"),
        "keys_2p20_and_pairs_2p24": result.get("configs"),
        "heavy_lists": result.get("lists"),
        "serving": result.get("serving"),
        "paper_mergesort_comparisons": comparisons,
        "tuning": result.get("tuning"),
        "gpu": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_section(args, np, inputs, types, host_input):
    """The CPU oracle timed on this host: (1) the single-threaded mergesort on
    the four 2M inputs of the step (the reported value), (2) its task-parallel
    variant on all usable cores, same inputs, (3) one single-threaded sort of
    each 256M input, the four run side by side on four threads.  Every input
    is the same seeded array the GPU sorts."""
    import concurrent.futures as cf
    import oracle
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    hosts = {k: host_input(k, N_SMALL) for k in types}
    done, rounds, t0 = 0, 0, time.perf_counter()
    while True:
        for k in types:
            oracle.sort_keys(hosts[k])
            done += N_SMALL
        rounds += 1
        el = time.perf_counter() - t0
        if el > 12.0 or rounds >= 40:
            break
    seeds = {k: inputs.seed_for(2, types.index(k), N_SMALL) for k in types}
    cpu = {"value": round(done / el / 1e6, 3), "unit": "Mkeys/s", "cores": 1, "kind": "oracle",
           "sample": f"{rounds} round(s) of the four 2M int32 inputs ({done} keys) through the "
                     f"single-threaded oracle mergesort, {el:.1f} s",
           "nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": cpu_model(),
           "seeds_2M": {k: hex(v) for k, v in seeds.items()}}
    threads = max(1, min(usable, 64))
    done, rounds, t0 = 0, 0, time.perf_counter()
    while True:
        for k in types:
            oracle.sort_keys_parallel(hosts[k], threads)
            done += N_SMALL
        rounds += 1
        el = time.perf_counter() - t0
        if el > 6.0 or rounds >= 100:
            break
    t_used = 1 << (threads.bit_length() - 1)
    cpu["parallel"] = {"value": round(done / el / 1e6, 3), "unit": "Mkeys/s", "cores": t_used,
                       "sample": f"{rounds} round(s) of the same four 2M inputs through the task-parallel "
                                 f"variant of the oracle on {t_used} threads, {el:.1f} s"}
    # the paper's own mergesort (Sec. 3 techniques, a CPU program) on the same inputs
    import baseline
    done, rounds, ncmp, t0 = 0, 0, 0, time.perf_counter()
    while True:
        for k in types:
            _, c = baseline.sort(hosts[k])
            done += N_SMALL
            ncmp += c
        rounds += 1
        el = time.perf_counter() - t0
        if el > 6.0 or rounds >= 100:
            break
    cpu["paper_mergesort"] = {"value": round(done / el / 1e6, 3), "unit": "Mkeys/s", "cores": 1,
                              "comparisons_per_key": round(ncmp / done, 3),
                              "minrun": baseline.MINRUN, "gallop_after": baseline.GALLOP_AFTER,
                              "sample": f"{rounds} round(s) of the same four 2M inputs through the paper's "
                                        f"mergesort (Sec. 3 (a), (b), (e2), (f), (g)) as a C program, {el:.1f} s"}
    log(f"cpu baseline: {cpu}")
    if not args.no_big:
        def leg(k):
            a = host_input(k, N_BIG)
            t = time.perf_counter()
            oracle.sort_keys(a)
            return time.perf_counter() - t
        with cf.ThreadPoolExecutor(len(types)) as ex:
            secs = dict(zip(types, ex.map(leg, types)))
        cpu["legs_256M"] = {k: {"s": round(v, 2), "Mkeys_s": round(N_BIG / v / 1e6, 3), "cores": 1,
                                "seed": hex(inputs.seed_for(2, types.index(k), N_BIG))}
                            for k, v in secs.items()}
        cpu["legs_256M_note"] = ("one single-threaded oracle sort of each 268,435,456-key input, the four "
                                 "running at once on four host threads")
        log(f"cpu 256M legs: {cpu['legs_256M']}")
    return cpu


def comparisons_section(np, inputs, types, host_input):
    """Sec. 5 of the paper for its mergesort as a CPU program (baseline/):
    comparisons per key at n = 2,000,000 for random int32 keys, the four input
    types and the Sec. 2 classes (mean over k = 2^0..2^8), and the regression
    g(n) = f(n)/n = s log2(n) + t over n = j * 10^6, j = 1..5 (per class, the
    mean over k at each n).  Runs on a pool of host threads."""
    import concurrent.futures as cf
    import baseline
    classes = ("equal_teeth", "even_teeth", "sharp_teeth", "shuffled_teeth", "distance", "exchange", "limited")
    ks = [1 << i for i in range(9)]

    def count(job):
        name, n, k = job
        if name == "random_int":
            a = inputs.random_int32(n, inputs.seed_for(7, 0, n))
        elif name in types:
            a = host_input(name, n)
        else:
            a = inputs.class_int32(name, n, k, inputs.seed_for(6, classes.index(name), k))
        return job, baseline.sort(a)[1] / n

    jobs = [("random_int", j * 10**6, 0) for j in range(1, 6)]
    jobs += [(t, N_SMALL, 0) for t in types]
    jobs += [(c, j * 10**6, k) for c in classes for j in range(1, 6) for k in ks]
    t0 = time.perf_counter()
    threads = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 8))
    with cf.ThreadPoolExecutor(threads) as ex:
        got = dict(ex.map(count, jobs))
    per_n = {}
    for (name, n, k), g in got.items():
        per_n.setdefault(name, {}).setdefault(n, []).append(g)
    out = {"n": N_SMALL, "minrun": baseline.MINRUN, "gallop_after": baseline.GALLOP_AFTER,
           "per_key_2M": {}, "regression": {}}
    for name, by_n in per_n.items():
        gs = {n: float(np.mean(v)) for n, v in by_n.items()}
        if 2_000_000 in gs:
            out["per_key_2M"][name] = round(gs[2_000_000], 3)
        if len(gs) == 5:
            x = np.log2(np.array(sorted(gs)))
            y = np.array([gs[n] for n in sorted(gs)])
            s_, t_ = np.polyfit(x, y, 1)
            out["regression"][name] = {"s": round(float(s_), 3), "t": round(float(t_), 3)}
    out["host_s"] = round(time.perf_counter() - t0, 1)
    log(f"comparisons: {out}")
    return out


def lists_section(torch, inputs, sortrace, dev):
    """Heavy items of Sec. 2: random lists of 16, 64 and 256 int32 (64, 256
    and 1024 bytes), n = 200,000 (the size of Tables 2-3) and 2,000,000.
    sr_sort_lists synchronizes, so the host clock times each call; the input
    is restored (untimed) before every call.  Bytes: the prefix-key pairs
    sort plus one read and one gather write of the lists."""
    out = {}
    for n in (200_000, 2_000_000):
        for L in (16, 64, 256):
            src = torch.from_numpy(inputs.random_lists(n, L, seed=n + L)).to(dev)
            work = torch.empty_like(src)
            times = []
            for i in range(6):
                work.copy_(src)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sortrace.sort_lists(work)
                if i:
                    times.append((time.perf_counter() - t0) * 1e3)
            ok = bool(((work[1:, 0] > work[:-1, 0]) | (work[1:, 0] == work[:-1, 0])).all())
            ms = statistics.median(times)
            key = f"n{n}_words{L}"
            out[key] = {"ms_median": round(ms, 4), "Mlists_s": round(n / (ms / 1e3) / 1e6, 2),
                        "list_GBps": round(2 * n * L * 4 / (ms / 1e3) / 1e9, 1), "first_word_sorted": ok}
            log(f"lists {key}: {out[key]}")
            del src, work
    torch.cuda.synchronize()
    return out


def configs_section(torch, np, inputs, sortrace, dev, stream):
    """2^20 uniform int32 keys, and 2^24 stable (uint64 key in geometric runs
    with 10% equal steps, uint32 payload = index) pairs: Mkeys/s, path,
    passes; the pairs output is checked for sortedness and stability."""
    def timed(fn, restore, reps):
        out = []
        for i in range(reps + 2):
            restore()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            if i >= 2:
                out.append(a.elapsed_time(b))
        return statistics.median(out)

    res = {}
    n1 = 1 << 20
    src = torch.from_numpy(inputs.random_int32(n1, inputs.seed_for(1, 0, n1))).to(dev)
    work = torch.empty_like(src)
    ms = timed(lambda: sortrace.sort_keys(work), lambda: work.copy_(src), 20)
    st = sortrace.last_stats()
    assert bool((work[1:] >= work[:-1]).all())
    res["int32_random_2p20"] = {"ms_median": round(ms, 5), "Mkeys_s": round(n1 / (ms / 1e3) / 1e6, 1),
                                "path": st["path"], "passes": st["passes"]}
    log(f"2^20 keys: {res['int32_random_2p20']}")
    n3 = 1 << 24
    hk, hp = inputs.runs_uint64(n3, seed=inputs.seed_for(3, 0, n3))
    ks = torch.from_numpy(hk.view(np.int64)).to(dev)
    ps = torch.from_numpy(hp.view(np.int32)).to(dev)
    kw, pw = torch.empty_like(ks), torch.empty_like(ps)

    def restore():
        kw.copy_(ks)
        pw.copy_(ps)
    ms = timed(lambda: sortrace.sort_pairs(kw, pw, dtype="uint64"), restore, 10)
    st = sortrace.last_stats()
    gk = kw.cpu().numpy().view(np.uint64)
    gp = pw.cpu().numpy().view(np.uint32)
    ok = bool(np.all(gk[1:] >= gk[:-1])) and bool(np.all((gk[1:] != gk[:-1]) | (gp[1:] > gp[:-1])))
    ok = ok and bool(np.array_equal(gk, hk[gp]))
    res["uint64_pairs_runs_2p24"] = {"ms_median": round(ms, 4), "Mpairs_s": round(n3 / (ms / 1e3) / 1e6, 1),
                                     "path": st["path"], "passes": st["passes"],
                                     "algorithmic_GBps": round(st["bytes_moved"] / (ms / 1e3) / 1e9, 1),
                                     "stable_and_sorted": ok}
    log(f"2^24 pairs: {res['uint64_pairs_runs_2p24']}")
    assert ok
    return res


def classes_section(args, torch, np, inputs, sortrace, dev, stream):
    """The presorted classes of Sec. 2 as in Tables 2-3: n = 2M, k = 2^0..2^8,
    each input sorted by the adaptive plan and by the forced general path
    (tile sort + every merge pass); mean times over k per class.  Two 256M
    teeth inputs show the pass counts at scale."""
    names = ("equal_teeth", "even_teeth", "sharp_teeth", "shuffled_teeth", "distance", "exchange", "limited")
    ks = [1 << i for i in range(9)]

    def time_sort(src, work, reps, force=None):
        if force is not None:
            sortrace.set_option("force_path", force)
        try:
            times = []
            for i in range(reps + 1):
                work.copy_(src)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                sortrace.sort_keys(work)
                b.record(stream)
                torch.cuda.synchronize()
                if i > 0:
                    times.append(a.elapsed_time(b))
            st = sortrace.last_stats()
        finally:
            if force is not None:
                sortrace.set_option("force_path", -1)
        assert bool((work[1:] >= work[:-1]).all())
        return statistics.median(times), st

    out = {}
    n = N_SMALL
    work = torch.empty(n, dtype=torch.int32, device=dev)
    for ci, name in enumerate(names):
        rows = []
        for k in ks:
            src = torch.from_numpy(inputs.class_int32(name, n, k, inputs.seed_for(6, ci, k))).to(dev)
            ms, st = time_sort(src, work, 10)
            gms, _ = time_sort(src, work, 5, force=3)
            m = sortrace.presortedness(src, inv=True)
            rows.append((k, ms, gms, st["path"], st["passes"], (m["run"], m["mono"], m["inv"])))
        mean = statistics.mean(r[1] for r in rows)
        gmean = statistics.mean(r[2] for r in rows)
        paths = {}
        for r in rows:
            paths[r[3]] = paths.get(r[3], 0) + 1
        out[name] = {"ms_mean_over_k": round(mean, 5), "Mkeys_s": round(n / (mean / 1e3) / 1e6, 1),
                     "general_ms_mean": round(gmean, 5), "speedup_vs_general": round(gmean / mean, 2),
                     "paths": paths, "passes": {str(r[0]): r[4] for r in rows},
                     "run_mono_inv": {str(r[0]): r[5] for r in rows}}
        log(f"classes 2M {name}: {out[name]}")
    # device time of the Sec. 2 measures on one 2M input
    src = torch.from_numpy(inputs.class_int32("exchange", n, 64, 1)).to(dev)
    meas = {}
    for label, inv in (("run_mono_ms", False), ("run_mono_inv_ms", True)):
        times = []
        for i in range(6):
            t0 = time.perf_counter()
            sortrace.presortedness(src, inv=inv)   # synchronizes
            if i:
                times.append((time.perf_counter() - t0) * 1e3)
        meas[label] = round(statistics.median(times), 4)
    log(f"measures at 2M (host-timed, include allocation and the copy back): {meas}")
    out["measure_time_2M"] = meas
    del work
    big = {}
    if not args.no_big:
        work = torch.empty(N_BIG, dtype=torch.int32, device=dev)
        for name, k in (("sharp_teeth", 8), ("even_teeth", 8), ("equal_teeth", 64)):
            log(f"generating 256M {name} k={k}")
            src = torch.from_numpy(inputs.class_int32(name, N_BIG, k, 0)).to(dev)
            ms, st = time_sort(src, work, 3)
            gms, gst = time_sort(src, work, 1, force=3)
            big[f"{name}_k{k}"] = {"ms": round(ms, 4), "Mkeys_s": round(N_BIG / (ms / 1e3) / 1e6, 1),
                                   "path": st["path"], "passes": st["passes"],
                                   "merge_passes": st["merge_passes"], "leaves": st["run_leaves"],
                                   "general_ms": round(gms, 4), "general_passes": gst["passes"]}
            log(f"classes 256M {name} k={k}: {big[f'{name}_k{k}']}")
            del src
        del work
        torch.cuda.synchronize()
    return {"n": n, "k": ks, "per_class_2M": out, "n_big": N_BIG if big else None, "big": big or None}


def serve_section(args, torch, np, inputs, sortrace, dev):
    """Poisson request stream through the continuous-batching server and the
    plain one-at-a-time FIFO server (same trace, same device-resident data)."""
    R = args.serve_requests
    lo, hi = 1024, 16_777_216
    pool_n = 1 << 26
    log("serving: generating request pool")
    pool_f = torch.from_numpy(inputs.normal_float32(pool_n, seed=inputs.seed_for(5, 1, 0)).view(np.int32)).to(dev)
    pool_i = torch.from_numpy(inputs.uniform_int32(pool_n, seed=inputs.seed_for(5, 0, 0))).to(dev)
    u = inputs.unit_double(inputs.stream(inputs.seed_for(5, 2, 0), 3 * R))
    sizes = np.clip(np.floor(np.exp(np.log(lo) + u[:R] * (np.log(hi) - np.log(lo)))), lo, hi).astype(np.int64)
    is_f = u[R:2 * R] < 0.5
    starts = (u[2 * R:] * (pool_n - sizes)).astype(np.int64)
    offs = np.zeros(R + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    data = torch.empty(int(offs[-1]), dtype=torch.int32, device=dev)
    views = [data[int(offs[i]):int(offs[i + 1])] for i in range(R)]

    def restore():
        for i in range(R):
            src = pool_f if is_f[i] else pool_i
            views[i].copy_(src[int(starts[i]):int(starts[i] + sizes[i])])
        torch.cuda.synchronize()

    budget = 4 << 30
    cfg_batched = dict(streams=4, max_batch_requests=64, max_batch_keys=1 << 26)
    cfg_plain = dict(streams=1, max_batch_requests=1, max_batch_keys=hi)

    def run(cfg, arrivals):
        restore()
        with sortrace.Server(budget, **cfg) as srv:
            t0 = srv.now() + 0.02
            for i in range(R):
                srv.submit(views[i], tag=i, t_arrive=t0 + arrivals[i], dtype="float32" if is_f[i] else "int32")
            srv.wait_idle(600)
            recs = srv.records()
        assert len(recs) == R and all(r["status"] == 0 for r in recs)
        lat = np.array([r["t_done"] - r["t_arrive"] for r in recs]) * 1e3
        span = max(r["t_done"] for r in recs) - min(r["t_arrive"] for r in recs)
        return {"p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3), "throughput_req_s": round(R / span, 1),
                "Mkeys_s": round(float(sizes.sum()) / span / 1e6, 1),
                "batches": len({r["batch"] for r in recs})}

    log("serving: closed-loop capacity")
    closed = run(cfg_batched, np.zeros(R))
    cap = closed["throughput_req_s"]
    plain_closed = run(cfg_plain, np.zeros(R))
    pcap = plain_closed["throughput_req_s"]
    out = {"requests": R, "sizes": f"log-uniform [{lo}, {hi}]", "mean_keys": int(sizes.mean()),
           "dtypes": "50% float32 N(0,1)+specials, 50% int32 uniform", "hbm_budget_bytes": budget,
           "batched_config": cfg_batched, "capacity_req_s": cap,
           "capacity_Mkeys_s": closed["Mkeys_s"], "plain_capacity_req_s": pcap,
           "plain_capacity_Mkeys_s": plain_closed["Mkeys_s"],
           "loads_note": "each server at rho x its OWN closed-loop capacity; 'shared' is one absolute "
                         "rate below both capacities (0.8 x the plain server's) offered to both",
           "loads": {}}
    ea = inputs.unit_double(inputs.stream(inputs.seed_for(5, 3, 0), R))
    unit_gaps = -np.log(1.0 - ea)   # exponential inter-arrivals of mean 1

    def at(cfg, lam, own_cap):
        r = run(cfg, np.cumsum(unit_gaps / lam))
        r["offered_req_s"] = round(lam, 1)
        r["overloaded"] = bool(lam > own_cap)
        return r
    for rho in (0.5, 0.8, 0.95):
        b = at(cfg_batched, rho * cap, cap)
        p = at(cfg_plain, rho * pcap, pcap)
        out["loads"][str(rho)] = {"batched": b, "plain": p}
        log(f"serving rho={rho}: batched {b} | plain {p}")
    lam = 0.8 * min(pcap, cap)
    b = at(cfg_batched, lam, cap)
    p = at(cfg_plain, lam, pcap)
    out["loads"]["shared"] = {"offered_req_s": round(lam, 1), "batched": b, "plain": p}
    log(f"serving shared load {lam:.0f} req/s: batched {b} | plain {p}")
    # correctness: every request equals the same array sorted alone
    restore()
    with sortrace.Server(budget, **cfg_batched) as srv:
        t0 = srv.now()
        for i in range(R):
            srv.submit(views[i], tag=i, t_arrive=t0, dtype="float32" if is_f[i] else "int32")
        srv.wait_idle(600)
    mix = data.clone()
    restore()
    for i in range(R):
        sortrace.sort_keys(views[i], dtype="float32" if is_f[i] else "int32")
    torch.cuda.synchronize()
    out["alone_equals_mix"] = bool(torch.equal(mix, data))
    assert out["alone_equals_mix"]
    del data, pool_f, pool_i, mix
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    main()
