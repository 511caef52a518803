"""GPU parity of the natural-run path (SR_PATH_RUNS) against the CPU oracle.

Inputs are the presorted classes of Sec. 2 (k-equal, k-even and k-sharp
teeth, organ pipes, k-exchange, k-distance) and random concatenations of
monotone runs with plateaus, at sizes that put run heads inside tiles, on
tile boundaries and in dense (disordered) tiles.  Every result is compared
bit for bit with the oracle; the path and pass counts are checked against
design invariants (they have no value in the paper).
"""
import numpy as np
import pytest

import oracle
from paper_1609_04471_amd import inputs

from test_gpu_sort import bits, gpu_sort_keys

pytestmark = pytest.mark.gpu


def general_passes(n, tile=8192):
    t = -(-n // tile)
    return 1 + max(0, (t - 1).bit_length())


def check(gpu, a, dtype="int32"):
    got = gpu_sort_keys(gpu, a, dtype)
    want = oracle.sort_keys(a)
    assert np.array_equal(bits(got), bits(want))
    return gpu.last_stats()


@pytest.mark.parametrize("n", [20_000, 262_147, 2_000_000])
@pytest.mark.parametrize("k", [2, 3, 8, 32])
def test_teeth_classes(gpu, n, k):
    for name in ("equal_teeth", "even_teeth", "sharp_teeth"):
        a = inputs.class_int32(name, n, k, seed=k)
        st = check(gpu, a)
        if n // k >= 3 * 8192:  # sections span several tiles: the run plan must pay
            assert st["path"] == "runs", (name, n, k, st)
            assert st["merge_passes"] < general_passes(n) - 1, (name, n, k, st)
        if name == "sharp_teeth" and st["path"] == "runs":
            # sections hold consecutive value ranges: after the reversals every
            # leaf continues the previous one, so nothing is merged
            assert st["run_leaves"] == 1 and st["merge_passes"] == 0, st


def test_sharp_teeth_large(gpu):
    n = 1 << 25
    a = inputs.sharp_teeth(n, 8)
    got = gpu_sort_keys(gpu, a, "int32")
    assert np.array_equal(got, np.arange(1, n + 1, dtype=np.int32))  # closed form
    st = gpu.last_stats()
    assert st["path"] == "runs" and st["merge_passes"] == 0, st
    assert st["passes"] <= 2, st


@pytest.mark.parametrize("seed", range(6))
def test_random_monotone_runs(gpu, seed):
    """Concatenated runs of random lengths and directions with plateaus, some
    too short for their own leaf, some disordered stretches."""
    rng = np.random.default_rng(seed)
    parts, total = [], 0
    n_target = [300_000, 1_000_000, 2_500_000][seed % 3]
    while total < n_target:
        kind = rng.integers(0, 10)
        ln = int(rng.integers(1, [60, 3000, 40_000, 200_000][rng.integers(0, 4)]))
        if kind == 0:   # disordered stretch
            x = rng.integers(-2**31, 2**31, size=ln, dtype=np.int64)
        else:
            steps = rng.integers(0, 4, size=ln)            # zero steps make plateaus
            steps[rng.random(ln) < 0.3] = 0
            x = int(rng.integers(-2**30, 2**30)) + np.cumsum(steps)
            if kind % 2:
                x = x[::-1]
        parts.append(np.clip(x, -2**31, 2**31 - 1))
        total += ln
    a = np.concatenate(parts)[:n_target].astype(np.int32)
    check(gpu, a)
    # the same runs, each shifted above the previous one: ordered leaves
    b = np.concatenate([p - p.min() + 1 + 10 * i * 2**20 // len(parts) for i, p in enumerate(parts)])
    b = np.clip(b, -2**31, 2**31 - 1)[:n_target].astype(np.int32)
    check(gpu, b)


def test_constant_stretches_carry_direction(gpu):
    """Strict directions carried across whole tiles of equal keys."""
    n1, n2, n3 = 30_000, 50_000, 40_001
    a = np.concatenate([np.arange(n1), np.full(n2, n1 + 5), np.arange(n1 + 5, n1 + 5 - n3, -1),
                        np.full(20_000, -3), np.arange(-3, 60_000)]).astype(np.int32)
    st = check(gpu, a)
    assert st["path"] == "runs", st
    b = np.concatenate([np.full(9000, 7), np.arange(7, -20_000, -1), np.full(9000, -5)]).astype(np.int32)
    check(gpu, b)


def test_heads_on_tile_boundaries(gpu):
    T = 4096
    for off in (-2, -1, 0, 1, 2):
        L = 3 * T + off
        a = np.concatenate([np.arange(L), np.arange(L)[::-1] + 10, np.arange(L) - 5,
                            np.arange(2 * L)[::-1]]).astype(np.int32)
        check(gpu, a)
        s = np.concatenate([np.arange(L)[::-1], np.arange(L, 2 * L), np.arange(3 * L - 1, 2 * L - 1, -1)])
        got = gpu_sort_keys(gpu, s.astype(np.int32), "int32")
        assert np.array_equal(got, np.arange(3 * L, dtype=np.int32))


def test_sorted_with_dense_patches(gpu):
    n = 1_500_000
    a = np.arange(n, dtype=np.int64)
    rng = np.random.default_rng(3)
    for start in (100_000, 700_001, 1_400_000):
        ln = 6000
        a[start:start + ln] = rng.integers(start - 50_000, start + 50_000, size=ln)
    st = check(gpu, a.astype(np.int32))
    assert st["path"] in ("runs", "outlier"), st


def test_forced_runs_falls_back_on_random(gpu):
    gpu.set_option("force_path", 4)
    try:
        for n in (10_000, 1_000_003):
            a = inputs.random_int32(n, seed=n)
            st = check(gpu, a)
            assert st["path"] == "general", st
        a = inputs.class_int32("even_teeth", 1_000_000, 4, seed=0)
        assert check(gpu, a)["path"] == "runs"
    finally:
        gpu.set_option("force_path", -1)


def test_exchange_prefers_outlier(gpu):
    n = 2_000_000
    for k in (1, 16, 256):
        a = inputs.class_int32("exchange", n, k, seed=k)
        st = check(gpu, a)
        # a few exchanges cost about two passes either way; many only via outliers
        assert st["path"] in (("outlier", "runs") if k == 1 else ("outlier",)), (k, st)


@pytest.mark.parametrize("name", ["distance", "limited", "shuffled_teeth"])
def test_other_classes(gpu, name):
    n = 200_003
    for k in (1, 4, 64):
        a = inputs.class_int32(name, n, k, seed=k)
        check(gpu, a)


def test_runs_other_dtypes(gpu):
    n = 1_000_001
    t = inputs.class_int32("even_teeth", n, 6, seed=0).astype(np.int64)
    f = (t.astype(np.float32) - 3e5) * np.float32(0.37)
    f[::200_003] = np.float32(-0.0)
    st = check(gpu, f, "float32")
    assert st["path"] == "runs", st
    u = (t.astype(np.uint64) << np.uint64(40)) + np.uint64(2**63 - 2**62)
    st = check(gpu, u, "uint64")
    assert st["path"] == "runs", st


def test_runs_switch_off(gpu):
    a = inputs.class_int32("sharp_teeth", 1_000_000, 4, seed=0)
    gpu.set_option("runs_path", 0)
    try:
        assert check(gpu, a)["path"] == "general"
    finally:
        gpu.set_option("runs_path", 1)
    assert check(gpu, a)["path"] == "runs"


@pytest.mark.parametrize("name,k", [("even_teeth", 8), ("equal_teeth", 64), ("even_teeth", 3)])
def test_runs_with_partition_launch(gpu, name, k):
    """With the separate partition launch the leaf merges take their co-ranks
    from it and run persistent and double-buffered."""
    n = 5_000_011
    a = inputs.class_int32(name, n, k, seed=k)
    gpu.set_option("partition_min_n", 0)
    try:
        st = check(gpu, a)
    finally:
        gpu.set_option("partition_min_n", -1)
    assert st["path"] == "runs" and st["merge_passes"] >= 2, st


def test_runs_random_mix_large(gpu):
    rng = np.random.default_rng(11)
    parts = []
    total = 0
    while total < 6_000_000:
        ln = int(rng.integers(50_000, 900_000))
        x = np.cumsum(rng.integers(0, 3, size=ln)) + int(rng.integers(-2**30, 2**30))
        parts.append(x[::-1] if rng.random() < 0.5 else x)
        total += ln
    a = np.concatenate(parts).astype(np.int32)
    st = check(gpu, a)
    assert st["path"] == "runs", st


# ------------------------------------------------------------------ pairs

from test_gpu_sort import gpu_sort_pairs  # noqa: E402


def check_pairs(gpu, k, dtype="int32"):
    p = np.arange(k.size, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(gpu, k, p, dtype)
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(bits(gk), bits(wk)) and np.array_equal(gp, wp)
    return gpu.last_stats()


def plateau_runs(n, seed, plateau_p=0.5, max_step=3):
    """Monotone runs of random directions whose steps are often zero, so the
    descending runs hold long groups of equal keys."""
    rng = np.random.default_rng(seed)
    parts, total = [], 0
    while total < n:
        ln = int(rng.integers(2, [50, 5000, 60_000][rng.integers(0, 3)]))
        steps = rng.integers(1, max_step + 1, size=ln)
        steps[rng.random(ln) < plateau_p] = 0
        x = int(rng.integers(-2**20, 2**20)) + np.cumsum(steps)
        parts.append(x[::-1] if rng.random() < 0.5 else x)
        total += ln
    return np.concatenate(parts)[:n].astype(np.int32)


@pytest.mark.parametrize("n", [20_000, 300_007, 2_000_000])
def test_pairs_take_the_run_path_stably(gpu, n):
    for k in (2, 8, 32):
        for name in ("equal_teeth", "even_teeth", "sharp_teeth"):
            st = check_pairs(gpu, inputs.class_int32(name, n, k, seed=k))
            if n // k >= 3 * 4096:
                assert st["path"] == "runs", (name, n, k, st)


@pytest.mark.parametrize("seed", range(4))
def test_pairs_plateaus_in_descending_runs(gpu, seed):
    n = [100_003, 700_001, 3_000_000, 5_000_011][seed]
    a = plateau_runs(n, seed)
    st = check_pairs(gpu, a)
    assert st["path"] in ("runs", "general", "near"), st
    # long equal groups reversed across unit and tile boundaries (51 values:
    # the few-unique path would take it, so it is switched off here)
    b = np.concatenate([np.repeat(np.arange(50, 0, -1), 3001), np.repeat(np.arange(40), 777),
                        np.repeat(np.arange(30, 0, -1), 9000)]).astype(np.int32)
    gpu.set_option("few_path", 0)
    try:
        st = check_pairs(gpu, b)
    finally:
        gpu.set_option("few_path", 1)
    assert st["path"] == "runs", st


def test_pairs_runs_with_partition_launch_and_dense(gpu):
    n = 3_000_001
    a = plateau_runs(n, 11, plateau_p=0.2)
    a[1_000_000:1_040_000] = inputs.random_int32(40_000, seed=4)   # a disordered stretch
    gpu.set_option("partition_min_n", 0)
    try:
        check_pairs(gpu, a)
    finally:
        gpu.set_option("partition_min_n", -1)
    check_pairs(gpu, a)


def test_pairs_runs_float_and_forced(gpu):
    f = plateau_runs(400_000, 3).astype(np.float32) * np.float32(0.5)
    f[::1001] = -0.0
    check_pairs(gpu, f, "float32")
    a = plateau_runs(300_000, 5)
    gpu.set_option("force_path", 4)  # SR_PATH_RUNS
    try:
        check_pairs(gpu, a)
        check_pairs(gpu, inputs.random_int32(200_000, seed=1))   # falls back when the plan cannot hold
    finally:
        gpu.set_option("force_path", -1)
    gpu.set_option("runs_path", 0)
    try:
        assert check_pairs(gpu, a)["path"] != "runs"
    finally:
        gpu.set_option("runs_path", 1)


def test_pairs_runs_uint64(gpu):
    a = plateau_runs(1_000_003, 7).astype(np.int64)
    k = (a + (1 << 40)).astype(np.uint64)
    k[::5003] = np.uint64(2**64 - 1)                 # keys above 2^63
    st = check_pairs(gpu, k, "uint64")
    assert st["path"] in ("runs", "general", "near"), st
    t = inputs.class_int32("even_teeth", 600_000, 6, seed=1).astype(np.int64).astype(np.uint64) << np.uint64(20)
    assert check_pairs(gpu, t, "uint64")["path"] == "runs"


def test_probe_skips_run_scans_that_cannot_pay(gpu):
    """Hard valleys (runs overlapping in value, never joined) seen in the
    probe's sample bound the plan's leaves from below: 1024 equal teeth in 2M
    keys need more merge passes than a scan can save, so the probe goes
    straight to the general path; their tooth boundaries are deep drops, so
    the outlier split is not tried either.  Sharp teeth have as many runs
    but no hard valleys (every run continues the previous one): still RUNS."""
    n = 2_000_000
    st = check(gpu, inputs.class_int32("equal_teeth", n, 1024, seed=1))
    assert st["path"] == "general", st
    st = check(gpu, inputs.class_int32("sharp_teeth", n, 1024, seed=1))
    assert st["path"] == "runs" and st["merge_passes"] == 0, st
    # few teeth: the scan pays, and without the outlier attempt
    st = check(gpu, inputs.class_int32("equal_teeth", 1 << 23, 128, seed=1))
    assert st["path"] == "runs", st


@pytest.mark.parametrize("n", [300_007, 2_000_000])
def test_displaced_blocks_and_the_outlier_split(gpu, n):
    """Sorted keys with blocks swapped with their neighbours.  Each swap is a
    drop that no single removal repairs; short blocks (3 keys) are still
    peeled off by the outlier split's rounds, long ones (40 keys) overlap
    further than the probe's depth test and the split is not tried (the
    run plan, the general plan or its NEAR finish follow: the blocks move
    by less than half a tile).  Whatever path follows, the result is exact."""
    rng = np.random.default_rng(n)
    for blk, paths in ((3, ("outlier",)), (40, ("runs", "general", "near"))):
        a = np.arange(n, dtype=np.int64)
        starts = np.sort(rng.choice(n // (2 * blk) - 1, size=n // (200 * blk), replace=False)) * (2 * blk)
        for p in starts:
            a[p:p + 2 * blk] = np.concatenate([a[p + blk:p + 2 * blk], a[p:p + blk]])
        st = check(gpu, a.astype(np.int32))
        assert st["path"] in paths, (blk, st)
