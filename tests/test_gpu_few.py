"""GPU parity of the few-distinct-keys path (SR_PATH_FEW) against the oracle.

Few-unique inputs (the Table 1 type and the k-limited class of Sec. 2),
with and without keys that the probe's sample misses (they go through the
separate between-key sort), float32 specials and uint64 keys; key + payload
sorts, whose equal keys must keep their input order.  Every result is
compared bit for bit with the oracle; paths are checked against design
invariants.
"""
import numpy as np
import pytest

import oracle
from paper_1609_04471_amd import inputs

from test_gpu_sort import bits, gpu_sort_keys

pytestmark = pytest.mark.gpu


def check(gpu, a, dtype="int32"):
    got = gpu_sort_keys(gpu, a, dtype)
    assert np.array_equal(bits(got), bits(oracle.sort_keys(a)))
    return gpu.last_stats()


@pytest.mark.parametrize("n", [8193, 20_000, 65_537, 300_001, 2_000_000, 5_000_011])
def test_few_unique_type(gpu, n):
    a = inputs.few_unique_int32(n, seed=n)
    st = check(gpu, a)
    assert st["path"] == "few" and st["outliers"] == 0, st
    assert st["passes"] == 1, st


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 8, 10, 12, 14, 16])
def test_k_limited(gpu, k):
    n = 1_000_003
    a = inputs.class_int32("limited", n, k, seed=k)
    st = check(gpu, a)
    if k <= 12:   # at most 4096 values: the bucket pass
        assert st["path"] == "few", st
    else:         # more distinct values than splitters
        assert st["path"] != "few", st


@pytest.mark.parametrize("n", [65_537, 2_000_000, 4_500_017])
def test_twelve_limited_type(gpu, n):
    """Table 1's few-unique type is 12-limited: 4096 values.  The sample sees
    nearly all of them; the keys of the few it misses are sorted as between
    keys.  At 65,537 keys the probe's pairs hold about one equal neighbour, too
    few to call the input few-valued: exact either way."""
    a = inputs.class_int32("limited", n, 12, seed=n)
    st = check(gpu, a)
    if n >= 1_000_000:
        assert st["path"] == "few", st
        assert st["outliers"] <= n // 8, st


# The 2,000,000-key, 0.1 % case took a GPU memory fault under a rewrite of
# this path (4096 splitters) whose cause was not found; that rewrite is out
# of the library, and the case stays skipped until the cause is known.
_FAULTED = pytest.mark.skip(reason="memory fault under a withdrawn rewrite of the FEW path; cause not found")


@pytest.mark.parametrize("n,frac", [(100_000, 0.001), pytest.param(2_000_000, 0.001, marks=_FAULTED),
                                    (5_000_011, 0.001)] +
                         [(n, f) for f in (0.03, 0.3) for n in (100_000, 2_000_000, 5_000_011)])
def test_between_keys(gpu, n, frac):
    rng = np.random.default_rng(int(n * frac * 1000) % 2**32)
    vals = rng.integers(-2**31, 2**31, size=20, dtype=np.int64)
    a = vals[rng.integers(0, 20, size=n)]
    other = rng.random(n) < frac
    a[other] = rng.integers(-2**31, 2**31, size=int(other.sum()), dtype=np.int64)
    a = a.astype(np.int32)
    st = check(gpu, a)
    if frac < 0.25:
        assert st["path"] == "few", st
        assert st["outliers"] > 0, st
    else:
        assert st["path"] != "few", st


def test_rare_values_missed_by_the_sample(gpu):
    n = 3_000_001
    a = inputs.few_unique_int32(n, seed=9)
    rng = np.random.default_rng(4)
    pos = rng.choice(n, size=37, replace=False)
    a[pos] = np.arange(37, dtype=np.int32) * 1000 - 17
    st = check(gpu, a)
    assert st["path"] == "few" and 0 < st["outliers"] <= 37, st


def test_float_specials(gpu):
    n = 1_200_007
    pool = np.array([0x7FC00000, 0xFFC00000, 0x7F800001, 0xFF800000, 0x7F800000, 0x80000000, 0x00000000,
                     0x3F800000, 0xBFC00000, 0x00000001, 0x80000001], dtype=np.uint32).view(np.float32)
    rng = np.random.default_rng(5)
    f = pool[rng.integers(0, pool.size, size=n)]
    st = check(gpu, f, "float32")
    assert st["path"] == "few", st


def test_uint64(gpu):
    n = 2_000_003
    rng = np.random.default_rng(6)
    vals = rng.integers(0, 2**63, size=13, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    u = vals[rng.integers(0, 13, size=n)]
    u[::50_021] = np.uint64(2**64 - 1)
    st = check(gpu, u, "uint64")
    assert st["path"] == "few", st


def test_large_closed_form(gpu):
    n = 1 << 26
    a = inputs.few_unique_int32(n, seed=26)
    got = gpu_sort_keys(gpu, a, "int32")
    v, c = np.unique(a, return_counts=True)
    assert np.array_equal(got, np.repeat(v, c))
    st = gpu.last_stats()
    assert st["path"] == "few" and st["passes"] == 1, st


def test_forced_and_switched_off(gpu):
    gpu.set_option("force_path", 5)
    try:
        for n in (10_000, 1_000_003):
            a = inputs.random_int32(n, seed=n)
            assert check(gpu, a)["path"] == "general"  # the sample's values cover too few keys
        b = inputs.few_unique_int32(500_000, seed=1)
        assert check(gpu, b)["path"] == "few"
    finally:
        gpu.set_option("force_path", -1)
    gpu.set_option("few_path", 0)
    try:
        b = inputs.few_unique_int32(500_000, seed=2)
        assert check(gpu, b)["path"] == "general"
    finally:
        gpu.set_option("few_path", 1)


@pytest.mark.parametrize("distinct,few", [(64, True), (65, True), (3000, True), (6000, False)])
def test_distinct_count_limit(gpu, distinct, few):
    """The probe keeps FEW while its sample holds at most 4096 distinct values:
    up to 64 are sorted by one wavefront, more by the tile sorter (65 and 3000
    values); 6000 values fill the sample's limit and the sort goes general."""
    n = 1_000_003
    rng = np.random.default_rng(distinct)
    vals = np.unique(rng.integers(-2**31, 2**31, size=4 * distinct, dtype=np.int64))[:distinct]
    assert vals.size == distinct
    a = vals[rng.integers(0, distinct, size=n)].astype(np.int32)
    st = check(gpu, a, "int32")
    assert (st["path"] == "few") == few, st


def test_extreme_codes_in_the_sample(gpu):
    """Values whose order codes are the smallest and largest of their type --
    for uint64 the largest code has no code + 1 and is counted apart -- are
    found by the sample and become splitters like any other."""
    n = 800_011
    rng = np.random.default_rng(12)
    vals = np.array([0, 2**64 - 1, 5, 2**63, 2**63 - 1, 77], dtype=np.uint64)
    u = vals[rng.integers(0, vals.size, size=n)]
    st = check(gpu, u, "uint64")
    assert st["path"] == "few", st
    ivals = np.array([-2**31, 2**31 - 1, 0, -1, 1], dtype=np.int32)
    a = ivals[rng.integers(0, ivals.size, size=n)]
    st = check(gpu, a, "int32")
    assert st["path"] == "few", st


@pytest.mark.parametrize("dtype", ["float32", "uint64"])
def test_many_values_other_dtypes(gpu, dtype):
    """2000 distinct values (with the extreme codes among them) in float32 and
    uint64: splitters sorted by the tile sorter, buckets found by the
    branch-free search."""
    n = 3_000_001
    rng = np.random.default_rng(31)
    if dtype == "float32":
        vals = np.unique(rng.standard_normal(2000).astype(np.float32))
        vals[:4] = np.array([0x7FC00000, 0xFFFFFFFF, 0x80000000, 0x00000000], dtype=np.uint32).view(np.float32)
    else:
        vals = np.unique(rng.integers(1, 2**63, size=2000, dtype=np.uint64) * np.uint64(2))
        vals[:2] = np.array([0, 2**64 - 1], dtype=np.uint64)
    a = vals[rng.integers(0, vals.size, size=n)]
    st = check(gpu, a, dtype)
    assert st["path"] == "few", st


def test_forced_few_with_many_values(gpu):
    """Forced FEW on keys with more than 4096 distinct values: the splitters
    are the 64 smallest distinct values of 1024 sorted sample keys; the rest
    are between keys, too many for the bucket pass, so the plan falls back,
    exactly."""
    gpu.set_option("force_path", 5)
    try:
        a = inputs.class_int32("limited", 1_000_003, 16, seed=3)
        st = check(gpu, a)
    finally:
        gpu.set_option("force_path", -1)
    assert st["path"] in ("few", "general"), st


@pytest.mark.parametrize("n", [100_000, 2_000_000])
@pytest.mark.parametrize("frac", [0.001, 0.03])
def test_wide_between_keys(gpu, n, frac):
    """1500 values (the wide tables) and a fraction of other keys: the between
    keys are sorted on their own (several merge passes at 3 %) and placed
    between the equal buckets."""
    rng = np.random.default_rng(int(n * frac * 1000) % 2**32 + 7)
    vals = np.unique(rng.integers(-2**31, 2**31, size=1500, dtype=np.int64))
    a = vals[rng.integers(0, vals.size, size=n)]
    other = rng.random(n) < frac
    a[other] = rng.integers(-2**31, 2**31, size=int(other.sum()), dtype=np.int64)
    a = a.astype(np.int32)
    st = check(gpu, a)
    if n >= 1_000_000:
        assert st["path"] == "few" and st["outliers"] > 0, st


@pytest.mark.parametrize("k", [32, 128, 256])
def test_periodic_input_does_not_alias_the_sample(gpu, k):
    """k-even teeth at 2,000,000 keys: the tooth length is a multiple of the
    sample strata's width for these k, so evenly spaced samples saw a few
    hundred values of the 7,813..62,500 present and sent the sort into the
    bucket pass, which then fell back after a counting read whose between
    keys all went through one atomic counter (383 us of classify for
    k = 128).  Samples drawn inside their strata see the real spread; the
    classify launch stays a no-op or a run scan."""
    n = 2_000_000
    a = inputs.class_int32("even_teeth", n, k, seed=k)
    check(gpu, a)
    gpu.set_option("profile", 1)
    try:
        gpu.profile_collect("")
        for _ in range(3):
            gpu_sort_keys(gpu, a, "int32")
        cnt, ms = gpu.profile_collect("classify")
    finally:
        gpu.set_option("profile", 0)
    assert cnt == 3 and ms / cnt < 0.1, (cnt, ms)


# ------------------------------------------------------------------ pairs

from test_gpu_sort import gpu_sort_pairs  # noqa: E402


def check_pairs(gpu, k, dtype="int32", p=None):
    """Pairs against the oracle's stable sort; the payload is the input
    position unless given, so any reordering of equal keys shows."""
    if p is None:
        p = np.arange(k.size, dtype=np.uint32)
    gk, gp = gpu_sort_pairs(gpu, k, p, dtype)
    wk, wp = oracle.sort_pairs(k, p)
    assert np.array_equal(bits(gk), bits(wk)) and np.array_equal(gp, wp)
    return gpu.last_stats()


@pytest.mark.parametrize("n", [8_193, 20_000, 300_001, 2_000_000, 4_194_304])
def test_pairs_few_unique(gpu, n):
    a = inputs.few_unique_int32(n, seed=n)
    st = check_pairs(gpu, a)
    assert st["path"] == "few" and st["outliers"] == 0, st


def test_pairs_few_size_limit(gpu):
    """The count matrix holds 1024 tiles of 4096 keys: one key more and the
    pairs take the general path, exactly."""
    n = 4_194_305
    st = check_pairs(gpu, inputs.few_unique_int32(n, seed=3))
    assert st["path"] != "few", st


@pytest.mark.parametrize("n,frac", [(300_001, 0.001), (2_000_000, 0.0001), (2_000_000, 0.2)])
def test_pairs_between_keys_fall_back(gpu, n, frac):
    """Keys between the sampled values: the pairs plan needs none, so it
    turns back into GENERAL before touching the arrays."""
    rng = np.random.default_rng(int(n * frac * 1e4) % 2**32)
    vals = rng.integers(-2**31, 2**31, size=20, dtype=np.int64)
    a = vals[rng.integers(0, 20, size=n)]
    other = rng.random(n) < frac
    a[other] = rng.integers(-2**31, 2**31, size=int(other.sum()), dtype=np.int64)
    st = check_pairs(gpu, a.astype(np.int32))
    assert st["path"] != "few", st


@pytest.mark.parametrize("distinct,few", [(2, True), (64, True), (65, False)])
def test_pairs_value_count(gpu, distinct, few):
    n = 1_000_003
    rng = np.random.default_rng(distinct + 100)
    vals = np.unique(rng.integers(-2**31, 2**31, size=4 * distinct, dtype=np.int64))[:distinct]
    a = vals[rng.integers(0, distinct, size=n)].astype(np.int32)
    p = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)  # payloads not positions
    st = check_pairs(gpu, a, p=p)
    assert (st["path"] == "few") == few, st


def test_pairs_few_other_dtypes(gpu):
    n = 1_500_007
    rng = np.random.default_rng(77)
    pool = np.array([0x7FC00000, 0xFFC00000, 0x80000000, 0x00000000, 0x7F800000, 0xFF800000, 0x3F800000],
                    dtype=np.uint32).view(np.float32)
    f = pool[rng.integers(0, pool.size, size=n)]
    assert check_pairs(gpu, f, "float32")["path"] == "few"
    vals = np.array([0, 2**64 - 1, 5, 2**63, 77, 2**40 + 3], dtype=np.uint64)
    u = vals[rng.integers(0, vals.size, size=n)]
    assert check_pairs(gpu, u, "uint64")["path"] == "few"


def test_pairs_few_switched_off_and_forced(gpu):
    a = inputs.few_unique_int32(500_000, seed=8)
    gpu.set_option("few_path", 0)
    try:
        assert check_pairs(gpu, a)["path"] != "few"
    finally:
        gpu.set_option("few_path", 1)
    gpu.set_option("force_path", 5)
    try:
        assert check_pairs(gpu, a)["path"] == "few"
        r = inputs.random_int32(300_001, seed=9)
        assert check_pairs(gpu, r)["path"] == "general"   # forced, then turned back
    finally:
        gpu.set_option("force_path", -1)
