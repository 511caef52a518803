"""The NEAR plan (tile sort + two rounds of neighbour merges) on inputs whose
keys are displaced by less than half a tile (the k-distance class of Sec. 2,
Table 1's nearly sorted type): bit-exact against the oracle, the path taken
where the tiles allow it and the full merge tree where they do not."""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def dev(a):
    view = {4: np.int32, 8: np.int64}[a.itemsize]
    return torch.from_numpy(np.ascontiguousarray(a).view(view).copy()).to(DEV)


def host(t, dtype):
    return t.cpu().numpy().view(dtype)


# n chosen for odd and even merge-slot counts (T = 8192 for 32-bit keys:
# 50,000 keys = 7 tiles, 3 slots; 100,003 = 13 tiles, 4 slots; 2M = 245 tiles, 8)
@pytest.mark.parametrize("n", [50_000, 100_003, 2_000_000, 4_500_001])
@pytest.mark.parametrize("k", [1, 16, 256, 1024, 4000])
def test_k_distance_int32(gpu, n, k):
    a = inputs.class_int32("distance", n, k, seed=k + n)
    t = dev(a)
    gpu.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    st = gpu.last_stats()
    assert np.array_equal(host(t, np.int32), oracle.sort_keys(a))
    assert st["path"] == "near", st
    ntiles = -(-n // 8192)
    m = max(1, (ntiles - 1).bit_length())
    assert st["merge_passes"] == 2 + (m & 1)


@pytest.mark.parametrize("k", [6000, 20000])
def test_too_far_takes_the_tree(gpu, k):
    """Displacement beyond half a tile: the test fails somewhere and the full
    merge tree sorts (still exact)."""
    n = 1_000_000
    a = inputs.class_int32("distance", n, k, seed=3)
    t = dev(a)
    gpu.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    assert np.array_equal(host(t, np.int32), oracle.sort_keys(a))
    assert gpu.last_stats()["path"] in ("general", "near")


def test_random_and_forced_general_take_the_tree(gpu):
    a = inputs.random_int32(1_000_003, 5)
    t = dev(a)
    gpu.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    assert gpu.last_stats()["path"] == "general"
    assert np.array_equal(host(t, np.int32), oracle.sort_keys(a))
    b = inputs.class_int32("distance", 1_000_003, 64, seed=9)
    gpu.set_option("force_path", 3)
    try:
        t = dev(b)
        gpu.sort_keys(t, dtype="int32")
        torch.cuda.synchronize()
        st = gpu.last_stats()
    finally:
        gpu.set_option("force_path", -1)
    assert st["path"] == "general" and st["merge_passes"] == 7
    assert np.array_equal(host(t, np.int32), oracle.sort_keys(b))
    gpu.set_option("near_path", 0)
    try:
        t = dev(b)
        gpu.sort_keys(t, dtype="int32")
        torch.cuda.synchronize()
        assert gpu.last_stats()["path"] == "general"
    finally:
        gpu.set_option("near_path", 1)
    assert np.array_equal(host(t, np.int32), oracle.sort_keys(b))


@pytest.mark.parametrize("n", [40_000, 1_000_001])
def test_near_pairs_stable(gpu, n):
    """Pairs (uint64 keys with heavy ties, T = 4096; int32 keys): payload =
    index, compared with the oracle's stable sort."""
    base = inputs.class_int32("distance", n, 300, seed=n).astype(np.int64)
    k64 = (base // 3).astype(np.uint64) * np.uint64(2**33)     # ties in groups of three
    p = np.arange(n, dtype=np.uint32)
    tk, tp = dev(k64), dev(p)
    gpu.sort_pairs(tk, tp, dtype="uint64")
    torch.cuda.synchronize()
    st = gpu.last_stats()
    wk, wp = oracle.sort_pairs(k64, p)
    assert np.array_equal(host(tk, np.uint64), wk) and np.array_equal(host(tp, np.uint32), wp)
    assert st["path"] == "near"
    k32 = (base // 2).astype(np.int32)
    tk, tp = dev(k32), dev(p)
    gpu.sort_pairs(tk, tp, dtype="int32")
    torch.cuda.synchronize()
    wk, wp = oracle.sort_pairs(k32, p)
    assert np.array_equal(host(tk, np.int32), wk) and np.array_equal(host(tp, np.uint32), wp)


def test_near_float32_and_partition_launch(gpu):
    """float32 keys (totalOrder) on the path with the separate partition
    launch and the persistent merge."""
    n = 3_000_017
    base = inputs.class_int32("distance", n, 500, seed=1)
    f = (base.astype(np.float64) - n // 2).astype(np.float32)   # exact: |values| < 2^24
    f[f == 0] = -0.0                                              # -0 in the middle, displaced like 0
    nan = np.array([0x7FC00000, 0x7FC00001, 0x7FFFFFFF], dtype=np.uint32).view(np.float32)
    f[-3:] = nan[::-1]                                            # +NaNs (by payload) at the end, reversed
    gpu.set_option("partition_min_n", 1)
    try:
        t = dev(f)
        gpu.sort_keys(t, dtype="float32")
        torch.cuda.synchronize()
        st = gpu.last_stats()
    finally:
        gpu.set_option("partition_min_n", -1)
    assert np.array_equal(host(t, np.uint32), oracle.sort_keys(f).view(np.uint32))
    assert st["path"] == "near"
