"""GPU parity of four-way merge passes (fan-in four) against the oracle.

A four-way pass merges each group of four neighbouring sorted runs in one
read and one write of the array: every 2048th key of every run (1024th for
64-bit keys) cuts the group where it stands in the merge order, and each
chunk between two cuts is merged as two levels in LDS.  The schedule is
forced here on sizes far below its built-in threshold (separate partition
shape, fan-in four), so that many shapes are covered quickly: one and
several four-way passes, an odd number of levels (a last two-way pass),
ragged last groups with one to four partial runs, heavy ties and the extreme
codes.  Every result is compared bit for bit with the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1609_04471_amd import inputs

from test_gpu_sort import bits, gpu_sort_keys, gpu_sort_pairs

pytestmark = pytest.mark.gpu

T32 = 8192   # int32 / float32 keys per tile
T64 = 4096   # uint64 keys per tile


@pytest.fixture
def fan4(gpu):
    gpu.set_option("partition_min_n", 0)
    gpu.set_option("fan_in", 4)
    try:
        yield gpu
    finally:
        gpu.set_option("fan_in", 0)
        gpu.set_option("partition_min_n", -1)


def levels(n, t):
    tiles = -(-n // t)
    return max(0, (tiles - 1).bit_length())


def check(g, a, dtype):
    got = gpu_sort_keys(g, a, dtype)
    assert np.array_equal(bits(got), bits(oracle.sort_keys(a))), (dtype, a.size)
    return g.last_stats()


# sizes in tiles of 8192: 2 (one pass), 2 + ragged, 3 levels (four-way +
# two-way), 4 levels, ragged last groups of 1..4 runs, 7 and 8 levels
SIZES32 = [16_385, 24_577, 32_768, 40_000, 65_536, 100_003, 3 * 32_768 + 5, 5 * 32_768 + 8_191 * 2,
           7 * 32_768 + 8_192 * 3 + 1, 262_145, 1_000_003, 2_000_000]


@pytest.mark.parametrize("n", SIZES32)
def test_int32_random(fan4, n):
    a = inputs.random_int32(n, seed=n)
    st = check(fan4, a, "int32")
    assert st["path"] == "general", st
    m = levels(n, T32)
    assert st["merge_passes"] == m // 2 + (m & 1), (st, m)


@pytest.mark.parametrize("n", [20_000, 100_003, 1_000_003])
def test_int32_ties(fan4, n):
    """Few distinct values and all-equal keys on the general path: every
    cut lands inside runs of equal keys."""
    fan4.set_option("force_path", 3)
    try:
        rng = np.random.default_rng(n)
        for a in (rng.integers(-3, 4, size=n).astype(np.int32),
                  np.full(n, 7, dtype=np.int32),
                  np.repeat(rng.integers(-2**31, 2**31, size=n // 5000 + 1), 5000)[:n].astype(np.int32)):
            check(fan4, a, "int32")
    finally:
        fan4.set_option("force_path", -1)


@pytest.mark.parametrize("n", [40_000, 262_147])
def test_int32_extreme_codes(fan4, n):
    rng = np.random.default_rng(n)
    a = rng.choice(np.array([-2**31, 2**31 - 1, 0, -1, 1], dtype=np.int64), size=n).astype(np.int32)
    a[rng.integers(0, n, size=n // 10)] = rng.integers(-2**31, 2**31, size=n // 10)
    fan4.set_option("force_path", 3)
    try:
        check(fan4, a, "int32")
    finally:
        fan4.set_option("force_path", -1)


@pytest.mark.parametrize("n", [16_385, 100_003, 300_001])
def test_float32_total_order(fan4, n):
    a = inputs.normal_float32(n, seed=n)
    rng = np.random.default_rng(n)
    pool = np.array([0x7FC00000, 0xFFC00000, 0x80000000, 0x00000000, 0x7F800000, 0xFF800000],
                    dtype=np.uint32).view(np.float32)
    idx = rng.integers(0, n, size=n // 20)
    a[idx] = pool[rng.integers(0, pool.size, size=idx.size)]
    check(fan4, a, "float32")


@pytest.mark.parametrize("n", [8_193, 12_289, 16_384, 20_001, 65_537, 300_001, 1_000_003])
def test_uint64(fan4, n):
    r = inputs.stream(n, n)
    st = check(fan4, r, "uint64")
    m = levels(n, T64)
    if m >= 2:
        assert st["merge_passes"] == m // 2 + (m & 1), (st, m)
    k, _ = inputs.runs_uint64(n, seed=n, tie_stress=True)
    check(fan4, k, "uint64")


@pytest.mark.parametrize("kind", ["reversed", "nearly", "few", "sorted", "teeth"])
def test_other_plans_under_the_four_way_schedule(fan4, kind):
    """Plans other than GENERAL keep their two-way slots; the four-way
    launches of the general schedule return at once for them."""
    n = 1_000_003
    if kind == "reversed":
        a = (np.arange(n, dtype=np.int64)[::-1] - n // 2).astype(np.int32)
    elif kind == "nearly":
        a = inputs.nearly_sorted_int32(n, seed=5)
    elif kind == "few":
        a = inputs.few_unique_int32(n, seed=5)
    elif kind == "sorted":
        a = np.arange(n, dtype=np.int32) * 2 - n
    else:
        a = inputs.class_int32("even_teeth", n, 8, seed=5)
    check(fan4, a, "int32")


def test_pairs_stay_two_way(fan4):
    n = 300_001
    k = inputs.few_unique_int32(n, seed=3)
    p = np.arange(n, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(fan4, k, p, "int32")
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(gk, wk) and np.array_equal(gp, wp)


def test_repeated_calls_and_sizes(fan4):
    """Back-to-back sorts of shrinking and growing sizes on one workspace."""
    for n in (2_000_000, 50_000, 700_001, 16_385, 2_000_000):
        a = inputs.random_int32(n, seed=n + 1)
        check(fan4, a, "int32")
