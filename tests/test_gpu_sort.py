"""GPU parity: libsortrace (through the C ABI) against the CPU oracle.

Tolerance is zero everywhere -- sorting does no arithmetic on keys, so every
output is compared bit for bit with the oracle's on the same seeded input.
Sizes span several tiles (8192 int32 keys per tile, 4096 merge outputs per
workgroup) and ragged tails.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SIZES = [2, 3, 5, 63, 64, 65, 1000, 4095, 4096, 4097, 8191, 8192, 8193, 12345, 16384,
         16385, 65537, 100_003, 262_144, 1_000_001]


def kinds_int32(n, seed):
    out = {k: inputs.int32_of_type(k, n, seed + i) for i, k in enumerate(inputs.TYPES)}
    out["sorted"] = np.arange(n, dtype=np.int32) * 3 - n
    out["equal"] = np.full(n, -7, dtype=np.int32)
    h = n // 2
    out["organ"] = np.concatenate([np.arange(h), np.arange(n - h)[::-1]]).astype(np.int32)
    m = max((n - 1) // 2, 0)
    # the 2m+1 instance on which BSD qsort degrades (Sec. 4)
    out["bsd_killer"] = np.concatenate([np.arange(m, 0, -1), [m + 1],
                                        np.arange(2 * m + 1, m + 1, -1)])[:n].astype(np.int32)
    return out


def to_dev(a: np.ndarray) -> torch.Tensor:
    view = {4: np.int32, 8: np.int64}[a.itemsize]
    return torch.from_numpy(np.ascontiguousarray(a).view(view).copy()).to(DEV)


def from_dev(t: torch.Tensor, like: np.ndarray) -> np.ndarray:
    return t.cpu().numpy().view(like.dtype)


def bits(a):
    return a.view({4: np.uint32, 8: np.uint64}[a.itemsize])


def gpu_sort_keys(gpu, a, dtype):
    t = to_dev(a)
    gpu.sort_keys(t, dtype=dtype)
    return from_dev(t, a)


def gpu_sort_pairs(gpu, k, p, dtype):
    tk, tp = to_dev(k), to_dev(p.view(np.int32))
    gpu.sort_pairs(tk, tp, dtype=dtype)
    return from_dev(tk, k), from_dev(tp, p)


@pytest.mark.parametrize("n", SIZES)
def test_int32_keys_all_kinds(gpu, n):
    for kind, a in kinds_int32(n, 1000 + n).items():
        got = gpu_sort_keys(gpu, a, "int32")
        want = oracle.sort_keys(a)
        assert np.array_equal(got, want), (kind, n)


@pytest.mark.parametrize("n", [2, 77, 4096, 8193, 65537, 300_001])
def test_float32_total_order_keys(gpu, n):
    a = inputs.normal_float32(n, seed=n)
    got = gpu_sort_keys(gpu, a, "float32")
    assert np.array_equal(bits(got), bits(oracle.sort_keys(a))), n


@pytest.mark.parametrize("n", [2, 77, 4096, 4097, 65537, 300_001])
def test_uint64_keys(gpu, n):
    k, _ = inputs.runs_uint64(n, seed=n)
    got = gpu_sort_keys(gpu, k, "uint64")
    assert np.array_equal(got, oracle.sort_keys(k)), n
    r = inputs.stream(n, n)  # full 64-bit range, top bit set half the time
    assert np.array_equal(gpu_sort_keys(gpu, r, "uint64"), oracle.sort_keys(r))


@pytest.mark.parametrize("dtype", ["int32", "float32", "uint64"])
@pytest.mark.parametrize("n", [2, 3, 100, 2047, 2048, 4097, 50_001, 262_147])
def test_pairs_stable(gpu, dtype, n):
    if dtype == "uint64":
        k, p = inputs.runs_uint64(n, seed=n, tie_stress=True)
    elif dtype == "float32":
        k = inputs.normal_float32(n, seed=n)
        k[: n // 2] = k[n // 4: n // 4 + n // 2][::-1]  # many equal keys
        p = np.arange(n, dtype=np.uint32)
    else:
        k = inputs.few_unique_int32(n, seed=n)
        p = np.arange(n, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(gpu, k, p, dtype)
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(bits(gk), bits(wk)), (dtype, n)
    assert np.array_equal(gp, wp), (dtype, n)


@pytest.mark.parametrize("n", [3, 4097, 20_000, 131_073])
def test_pairs_reversed_path_is_stable(gpu, n):
    # nonincreasing with equal groups: the REVERSED path must keep group order
    k = (np.arange(n, dtype=np.int64)[::-1] // 3).astype(np.int32)
    p = np.arange(n, dtype=np.uint32)[::-1].copy()
    gk, gp = gpu_sort_pairs(gpu, k, p, "int32")
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(gk, wk) and np.array_equal(gp, wp)
    if n > 8192:
        assert gpu.last_stats()["path"] == "reversed"


def test_unaligned_pointers(gpu):
    n = 70_001
    a = inputs.random_int32(n + 1, seed=9)
    base = to_dev(a)
    view = base[1:]  # 4-byte aligned, not 16-byte aligned
    gpu.sort_keys(view, dtype="int32")
    got = base.cpu().numpy()
    assert got[0] == a[0]
    assert np.array_equal(got[1:], oracle.sort_keys(a[1:]))


@pytest.mark.parametrize("n", [70_001, 1_000_003])
def test_unaligned_pointers_every_path(gpu, n):
    # every input type (and a 64-value few-unique input) at a base 4-byte
    # but not 16-byte aligned: the vector loads of the probe, the few-unique
    # count and the tile sort fall back to element loads
    kinds = {k: inputs.int32_of_type(k, n + 1, 40 + i) for i, k in enumerate(inputs.TYPES)}
    kinds["few64"] = inputs.few_unique_int32(n + 1, seed=3, distinct=64)
    for kind, a in kinds.items():
        for off in (1, 2, 3):
            base = to_dev(a)
            view = base[off:]
            gpu.sort_keys(view, dtype="int32")
            got = base.cpu().numpy()
            assert np.array_equal(got[:off], a[:off]), (kind, off)
            assert np.array_equal(got[off:], oracle.sort_keys(a[off:])), (kind, off, gpu.last_stats()["path"])


def test_paths_chosen(gpu):
    n = 1_000_000
    cases = {"sorted": (np.arange(n, dtype=np.int32), "sorted"),
             "reversed": (inputs.reversed_int32(n), "reversed"),
             "random": (inputs.random_int32(n, 5), "general"),
             "equal": (np.zeros(n, np.int32), "sorted")}
    for name, (a, path) in cases.items():
        got = gpu_sort_keys(gpu, a, "int32")
        assert np.array_equal(got, oracle.sort_keys(a)), name
        st = gpu.last_stats()
        assert st["path"] == path, (name, st)
    # a forced general path gives the same bytes
    gpu.set_option("force_path", 3)
    try:
        a = inputs.reversed_int32(n)
        assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a))
        assert gpu.last_stats()["path"] == "general"
    finally:
        gpu.set_option("force_path", -1)


def test_measure_counts_descents(gpu):
    for n in (2, 16, 5000, 1_000_003):
        a = inputs.nearly_sorted_int32(n, seed=n)
        d, u = gpu.measure(to_dev(a), dtype="int32")
        assert d + 1 == oracle.run(a)
        assert u == oracle.ascents(a)
    ex = np.array([1, 15, 18, 19, 20, 16, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2], np.int32)
    assert gpu.measure(to_dev(ex), dtype="int32")[0] + 1 == 12  # Run(A) of the Sec. 3 example


def test_deterministic_repeats(gpu):
    a = inputs.few_unique_int32(3_000_000, seed=42)
    outs = [gpu_sort_keys(gpu, a, "int32") for _ in range(3)]
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    assert np.array_equal(outs[0], oracle.sort_keys(a))


@pytest.mark.parametrize("kind", inputs.TYPES)
def test_two_million_four_types(gpu, kind):
    n = 2_000_000
    a = inputs.int32_of_type(kind, n, inputs.seed_for(2, inputs.TYPES.index(kind), n))
    got = gpu_sort_keys(gpu, a, "int32")
    assert np.array_equal(got, oracle.sort_keys(a)), kind


@pytest.mark.parametrize("n", [8193, 40_000, 262_147, 1_000_003])
def test_separate_partition_launch(gpu, n):
    """Merge passes with the Merge Path partition in its own launch."""
    gpu.set_option("partition_min_n", 0)
    try:
        a = inputs.random_int32(n, seed=n)
        assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a))
        k, p = inputs.runs_uint64(n, seed=n, tie_stress=True)
        gk, gp = gpu_sort_pairs(gpu, k, p, "uint64")
        wk, wp = oracle.sort_pairs(k, p)
        assert np.array_equal(gk, wk) and np.array_equal(gp, wp)
    finally:
        gpu.set_option("partition_min_n", -1)


def _near(n, seed, frac=100, ties=1):
    """0..n-1 (optionally // ties) with floor(n/frac) disjoint exchanges."""
    a = (np.arange(n, dtype=np.int64) // ties).astype(np.int32)
    rng = np.random.default_rng(seed)
    m = n // frac
    pos = rng.choice(n, size=2 * m, replace=False)
    p, q = pos[0::2], pos[1::2]
    a[p], a[q] = a[q].copy(), a[p].copy()
    return a


@pytest.mark.parametrize("n", [8193, 65_536, 300_007, 2_000_000, 5_000_011])
def test_outlier_path_nearly_sorted(gpu, n):
    for seed, (frac, ties) in enumerate([(100, 1), (100, 7), (30, 1), (1000, 3)]):
        a = _near(n, seed, frac, ties)
        got = gpu_sort_keys(gpu, a, "int32")
        assert np.array_equal(got, oracle.sort_keys(a)), (n, frac, ties)
        st = gpu.last_stats()
        if frac >= 100:  # ~2% descents: below the probe's 1/16 threshold
            assert st["path"] == "outlier", st
            assert 0 < st["outliers"] <= 4 * (n // frac) + 8, st
        else:            # ~6.7% descents: the probe may choose either path
            assert st["path"] in ("outlier", "general"), st
    b = inputs.nearly_sorted_int32(n, seed=5)
    assert np.array_equal(gpu_sort_keys(gpu, b, "int32"), oracle.sort_keys(b))
    assert gpu.last_stats()["path"] == "outlier"


def _check_pairs(gpu, k, dtype="int32", p=None):
    if p is None:
        p = np.arange(k.size, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(gpu, k, p, dtype)
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(bits(gk), bits(wk)) and np.array_equal(gp, wp), (dtype, k.size)
    return gpu.last_stats()


@pytest.mark.parametrize("n", [8193, 65_536, 300_007, 2_000_000, 5_000_011])
def test_outlier_path_pairs_stable(gpu, n):
    """Pairs on the outlier path: equal keys among the kept keys and among the
    outliers, and between the two, keep their input order (payload = input
    position, compared with the oracle's stable sort)."""
    for seed, (frac, ties) in enumerate([(100, 1), (100, 7), (200, 64), (1000, 3)]):
        a = _near(n, seed + 10, frac, ties)
        st = _check_pairs(gpu, a)
        if n >= 65_536:
            assert st["path"] == "outlier", (frac, ties, st)
            assert 0 < st["outliers"] <= n // 4, st
    b = inputs.nearly_sorted_int32(n, seed=6)
    assert _check_pairs(gpu, b)["path"] in (("outlier",) if n >= 65_536 else ("outlier", "general"))


def test_outlier_path_pairs_other_dtypes_and_payloads(gpu):
    n = 700_001
    rng = np.random.default_rng(21)
    f = np.sort(inputs.normal_float32(n, seed=9, specials=False))
    f[::1000] = np.float32(0.0)          # ties inside the kept keys and with outliers
    idx = rng.choice(n, size=2 * (n // 150), replace=False)
    f[idx[0::2]], f[idx[1::2]] = f[idx[1::2]].copy(), f[idx[0::2]].copy()
    pay = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    assert _check_pairs(gpu, f, "float32", pay)["path"] == "outlier"
    u = (np.arange(n, dtype=np.uint64) // np.uint64(5)) * np.uint64(2**35)
    u[idx[0::2]], u[idx[1::2]] = u[idx[1::2]].copy(), u[idx[0::2]].copy()
    assert _check_pairs(gpu, u, "uint64")["path"] == "outlier"


def test_outlier_path_pairs_limits(gpu):
    """More than n/4 outliers: the pairs plan falls back to GENERAL before
    writing anything; forcing OUTLIER on random pairs falls back too; the
    switch turns the path off."""
    n = 1_000_003
    a = _near(n, 3, frac=6, ties=1)       # ~1/3 of the keys displaced
    assert _check_pairs(gpu, a)["path"] != "outlier"
    gpu.set_option("force_path", 2)
    try:
        r = inputs.random_int32(300_001, seed=4)
        assert _check_pairs(gpu, r)["path"] == "general"
        assert _check_pairs(gpu, _near(400_000, 5))["path"] == "outlier"
    finally:
        gpu.set_option("force_path", -1)
    gpu.set_option("outlier_path", 0)
    try:
        assert _check_pairs(gpu, _near(400_000, 6))["path"] != "outlier"
    finally:
        gpu.set_option("outlier_path", 1)


def test_outlier_path_falls_back(gpu):
    n = 1_000_003
    rot = np.concatenate([np.arange(n // 2, n), np.arange(0, n // 2)]).astype(np.int32)
    assert np.array_equal(gpu_sort_keys(gpu, rot, "int32"), oracle.sort_keys(rot))
    # kept keys not sorted across tiles: no outlier job; the two ascending
    # runs take the run path, or the general path once that is switched off
    assert gpu.last_stats()["path"] == "runs"
    gpu.set_option("runs_path", 0)
    try:
        assert np.array_equal(gpu_sort_keys(gpu, rot, "int32"), oracle.sort_keys(rot))
        assert gpu.last_stats()["path"] == "general"
    finally:
        gpu.set_option("runs_path", 1)
    gpu.set_option("outlier_path", 0)
    try:
        a = inputs.nearly_sorted_int32(n, seed=3)
        assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a))
        assert gpu.last_stats()["path"] == "general"
    finally:
        gpu.set_option("outlier_path", 1)


def test_outlier_path_other_dtypes(gpu):
    n = 400_009
    f = np.sort(inputs.normal_float32(n, seed=8, specials=False))
    idx = np.random.default_rng(1).choice(n, size=2 * (n // 100), replace=False)
    f[idx[0::2]], f[idx[1::2]] = f[idx[1::2]].copy(), f[idx[0::2]].copy()
    f[::997] = np.float32(-0.0)
    assert np.array_equal(bits(gpu_sort_keys(gpu, f, "float32")), bits(oracle.sort_keys(f)))
    u = np.arange(n, dtype=np.uint64) * np.uint64(3) + np.uint64(2**63)
    u[idx[0::2]], u[idx[1::2]] = u[idx[1::2]].copy(), u[idx[0::2]].copy()
    assert np.array_equal(gpu_sort_keys(gpu, u, "uint64"), oracle.sort_keys(u))
    assert gpu.last_stats()["path"] == "outlier"


def test_pairs_persistent_merge_large(gpu):
    n = 4_500_001  # above the partition threshold: persistent merge for 32-bit pairs
    k = inputs.few_unique_int32(n, seed=77)
    p = np.arange(n, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(gpu, k, p, "int32")
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(gk, wk) and np.array_equal(gp, wp)


def test_outlier_path_across_workspace_growth(gpu):
    """Regression: growing the scratch between calls must not disturb the
    look-back status words of the outlier path (they are epoch-stamped)."""
    for n in (100_000, 262_144, 400_000, 600_000, 1_000_001, 262_144):
        a = inputs.int32_of_type("nearly", n, 1003 + n)
        assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a)), n
        assert gpu.last_stats()["path"] == "outlier", n


@pytest.mark.parametrize("tile_variant,merge_items", [(1, 16), (0, 8), (0, 16), (1, 8)])
def test_tuning_variants_same_bytes(gpu, tile_variant, merge_items):
    gpu.set_option("tile_variant", tile_variant)
    gpu.set_option("merge_items", merge_items)
    try:
        for n in (5000, 8192, 100_003, 2_000_000):
            for kind in ("random", "few", "reversed"):
                a = inputs.int32_of_type(kind, n, n + 11)
                assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a)), (kind, n)
            f = inputs.normal_float32(n, seed=n)
            assert np.array_equal(bits(gpu_sort_keys(gpu, f, "float32")), bits(oracle.sort_keys(f)))
    finally:
        gpu.set_option("tile_variant", -1)
        gpu.set_option("merge_items", 0)


def test_concurrent_host_threads(gpu):
    """Four host threads sort on four streams at once (ctypes drops the GIL
    during each call): keys and pairs of every kind and ragged sizes, each
    result bit-exact against the oracle."""
    import threading
    cases = []
    for t in range(4):
        mine = []
        for j, kind in enumerate(inputs.TYPES):
            n = [70_001, 300_007, 1_000_003][(t + j) % 3]
            a = inputs.int32_of_type(kind, n, 100 * t + j)
            mine.append(("keys", a, None, oracle.sort_keys(a)))
        k, p = inputs.runs_uint64(200_003, seed=60 + t, tie_stress=True)
        mine.append(("pairs", k, p, oracle.sort_pairs(k, p)))
        cases.append(mine)
    dev = [[(to_dev(a), to_dev(p.view(np.int32)) if p is not None else None) for _, a, p, _ in mine]
           for mine in cases]
    streams = [torch.cuda.Stream() for _ in range(4)]
    torch.cuda.synchronize()
    errors = []

    def worker(t):
        try:
            st = streams[t]
            for rep in range(3):
                for (what, a, p, _), (tk, tp) in zip(cases[t], dev[t]):
                    if rep:  # restore the input on this stream, then sort again
                        with torch.cuda.stream(st):
                            tk.copy_(to_dev(a))
                            if tp is not None:
                                tp.copy_(to_dev(p.view(np.int32)))
                    if what == "keys":
                        gpu.sort_keys(tk, dtype="int32", stream=st)
                    else:
                        gpu.sort_pairs(tk, tp, dtype="uint64", stream=st)
            st.synchronize()
        except Exception as e:  # reported by the main thread
            errors.append((t, repr(e)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors
    for mine, dv in zip(cases, dev):
        for (what, a, p, want), (tk, tp) in zip(mine, dv):
            if what == "keys":
                assert np.array_equal(bits(from_dev(tk, a)), bits(want)), (what, a.size)
            else:
                assert np.array_equal(bits(from_dev(tk, a)), bits(want[0]))
                assert np.array_equal(from_dev(tp, p), want[1])
    for st in streams:
        assert gpu.load().sr_release_stream(st.cuda_stream) == 0


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")  # nothing was recorded: the point
def test_plain_sort_refuses_capture_that_would_allocate(gpu):
    """On a stream without a workspace of the size, a plain sort recorded
    into a capture is refused with SR_ERR_UNSUPPORTED before anything is
    recorded; the keys stay as they were and the same call sorts once the
    capture has ended."""
    lib = gpu.load()
    a = inputs.random_int32(100_003, seed=21)
    t = to_dev(a)
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        g.capture_begin()
        try:
            rc = lib.sr_sort_keys(0, t.data_ptr(), a.size, st.cuda_stream)
            rc_pairs = lib.sr_sort_pairs(0, t.data_ptr(), t.data_ptr(), a.size, st.cuda_stream)
        finally:
            g.capture_end()
    assert rc == 2 and rc_pairs == 2, (rc, rc_pairs)
    assert b"capture" in lib.sr_last_error_message()
    torch.cuda.synchronize()
    assert np.array_equal(from_dev(t, a), a)
    gpu.sort_keys(t, dtype="int32", stream=st)
    st.synchronize()
    assert np.array_equal(from_dev(t, a), np.sort(a))
    assert lib.sr_release_stream(st.cuda_stream) == 0


@pytest.mark.parametrize("n", [300_001, 2_000_000, 9_000_001])
def test_plain_sorts_recorded_into_a_stream_capture(gpu, n):
    """Keys and pairs sorts recorded into a torch CUDA graph on a stream whose
    workspace is reserved, replayed five times on new data of every input
    type (each replay takes its own device plan), with eager sorts on the
    same stream between the replays: every replay equals the oracle."""
    lib = gpu.load()
    st = torch.cuda.Stream()
    assert lib.sr_reserve(0, n, 0, st.cuda_stream) == 0
    keys = torch.empty(n, dtype=torch.int32, device=DEV)
    pk = torch.empty(n, dtype=torch.int64, device=DEV)
    pp = torch.empty(n, dtype=torch.int32, device=DEV)
    other = torch.empty(n, dtype=torch.int32, device=DEV)
    with torch.cuda.stream(st):   # warm-up sorts size the pairs workspace too
        gpu.sort_pairs(pk, pp, dtype="uint64", stream=st)
    st.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        g.capture_begin()
        try:
            gpu.sort_keys(keys, dtype="int32", stream=st)
            gpu.sort_pairs(pk, pp, dtype="uint64", stream=st)
        finally:
            g.capture_end()
    kinds = ["random", "reversed", "nearly", "few", "random"]
    for rep, kind in enumerate(kinds):
        a = inputs.int32_of_type(kind, n, 90 + rep)
        hk, hp = inputs.runs_uint64(n, seed=rep, tie_stress=rep % 2 == 1)
        with torch.cuda.stream(st):
            keys.copy_(torch.from_numpy(a))
            pk.copy_(torch.from_numpy(hk.view(np.int64)))
            pp.copy_(torch.from_numpy(hp.view(np.int32)))
            g.replay()
            other.copy_(torch.from_numpy(inputs.random_int32(n, 7 + rep)))
            gpu.sort_keys(other, dtype="int32", stream=st)
        st.synchronize()
        assert np.array_equal(from_dev(keys, a), oracle.sort_keys(a)), (rep, kind)
        wk, wp = oracle.sort_pairs(hk, hp)
        assert np.array_equal(pk.cpu().numpy().view(np.uint64), wk), rep
        assert np.array_equal(pp.cpu().numpy().view(np.uint32), wp), rep
    del g
    torch.cuda.synchronize()
    assert lib.sr_release_stream(st.cuda_stream) == 0


def test_plain_sort_graph_cache(gpu):
    """The library's own capture-and-replay cache for plain sorts ("graph" and
    "graph_plain" options): repeated calls on one buffer with new data."""
    n = 2_000_000
    t = torch.empty(n, dtype=torch.int32, device=DEV)
    gpu.set_option("graph", 1)
    gpu.set_option("graph_plain", 1)
    try:
        for rep, kind in enumerate(["random", "few", "reversed", "nearly", "random", "few"]):
            a = inputs.int32_of_type(kind, n, 40 + rep)
            t.copy_(torch.from_numpy(a))
            gpu.sort_keys(t, dtype="int32")
            torch.cuda.synchronize()
            assert np.array_equal(from_dev(t, a), oracle.sort_keys(a)), (rep, kind)
    finally:
        gpu.set_option("graph_plain", 0)
        gpu.set_option("graph", 0)


def test_random_sizes_sweep(gpu):
    """Sixty seeded random sizes from 2 to 300,000 keys, each with a random
    dtype, input kind and keys/pairs choice: bit-exact against the oracle
    (catches size-dependent launch-shape or tail handling mistakes that the
    fixed size list misses)."""
    rng = np.random.default_rng(2024)
    for case in range(60):
        n = int(rng.integers(2, 300_001))
        kind = inputs.TYPES[int(rng.integers(0, len(inputs.TYPES)))]
        dt = ("int32", "float32", "uint64")[int(rng.integers(0, 3))]
        a = inputs.int32_of_type(kind, n, 500 + case)
        if dt == "float32":
            a = (a.astype(np.float32) * np.float32(0.25))
        elif dt == "uint64":
            a = (a.astype(np.int64).astype(np.uint64) << np.uint64(20)) ^ np.uint64(0x9E3779B9)
        if rng.random() < 0.3:
            p = np.arange(n, dtype=np.uint32)
            gk, gp = gpu_sort_pairs(gpu, a, p, dt)
            wk, wp = oracle.sort_pairs(a, p)
            assert np.array_equal(bits(gk), bits(wk)) and np.array_equal(gp, wp), (case, n, kind, dt)
        else:
            got = gpu_sort_keys(gpu, a, dt)
            assert np.array_equal(bits(got), bits(oracle.sort_keys(a))), (case, n, kind, dt)


@pytest.mark.parametrize("path", [-1, 3])
@pytest.mark.parametrize("n", [40_000, 300_001, 2_000_000, 9_000_001])
def test_largest_code_keys_through_the_merges(gpu, n, path):
    """Keys equal to the largest code of their type (INT32_MAX, 2^64 - 1, and
    the float32 NaN with every payload bit set, last in totalOrder) -- the
    value a keys-only merge stages after each run -- mixed with random keys,
    in runs of them and alone, on the device's own path (-1) and forced
    through the general merge passes (3); every size up to the separate
    partition launch's shape.  Exact against the oracle."""
    rng = np.random.default_rng(n + path)
    biggest = {"int32": np.array([2**31 - 1], np.int32),
               "uint64": np.array([2**64 - 1], np.uint64),
               "float32": np.array([0x7FFFFFFF], np.uint32).view(np.float32)}
    for dtype, big in biggest.items():
        if dtype == "uint64":
            a = rng.integers(0, 2**64 - 1, size=n, dtype=np.uint64)
        elif dtype == "int32":
            a = rng.integers(-2**31, 2**31 - 1, size=n, dtype=np.int32)
        else:
            a = inputs.normal_float32(n, seed=n + 11)
        a[rng.random(n) < 0.3] = big[0]
        a[n // 3:n // 3 + 5000] = big[0]
        gpu.set_option("force_path", path)
        try:
            got = gpu_sort_keys(gpu, a, dtype)
        finally:
            gpu.set_option("force_path", -1)
        assert np.array_equal(bits(got), bits(oracle.sort_keys(a))), (dtype, n, path)


@pytest.mark.parametrize("n", [9_000_001, 20_000_003])
def test_job_passes_on_the_partition_shape(gpu, n):
    """Sizes that take the separate partition launch (int32 keys from 2^23):
    the merge passes of an outlier job and of a few-unique job with keys
    between the sampled values, each behind its own partition launch on the
    job's short runs; keys and pairs, exact against the oracle."""
    a = _near(n, n)
    got = gpu_sort_keys(gpu, a, "int32")
    st = gpu.last_stats()
    assert st["path"] == "outlier" and st["merge_passes"] >= 3, st
    assert np.array_equal(got, oracle.sort_keys(a))
    p = np.arange(n, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(gpu, a, p, "int32")
    st = gpu.last_stats()
    assert st["path"] == "outlier", st
    wk, wp = oracle.sort_pairs(a, p)
    assert np.array_equal(gk, wk) and np.array_equal(gp, wp)
    rng = np.random.default_rng(n)
    vals = rng.integers(-2**31, 2**31, size=20, dtype=np.int64)
    b = vals[rng.integers(0, 20, size=n)]
    other = rng.random(n) < 0.03
    b[other] = rng.integers(-2**31, 2**31, size=int(other.sum()), dtype=np.int64)
    b = b.astype(np.int32)
    got = gpu_sort_keys(gpu, b, "int32")
    st = gpu.last_stats()
    assert st["path"] == "few" and st["outliers"] > 0 and st["merge_passes"] >= 3, st
    assert np.array_equal(got, oracle.sort_keys(b))
