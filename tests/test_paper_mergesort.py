"""The paper's mergesort as a CPU program (baseline/): pinned against the
oracle and against definitions, with comparison counts checked on inputs
whose counts follow from the techniques of Sec. 3 by hand."""
import itertools

import numpy as np
import pytest

import baseline
import oracle
from paper_1609_04471_amd import inputs

I32 = np.array([-2**31, -7, -1, 0, 1, 2, 99, 2**31 - 1], dtype=np.int32)
U64 = np.array([0, 1, 2**32, 2**40, 2**63 - 1, 2**63, 2**64 - 2, 2**64 - 1], dtype=np.uint64)
F32 = np.array([0xFFC00000, 0xFF800000, 0xBF800000, 0x80000000, 0x00000000, 0x3F800000,
                0x7F800000, 0x7FC00000], dtype=np.uint32).view(np.float32)


@pytest.mark.parametrize("n", range(0, 9))
def test_every_permutation(n):
    for ordered in (I32[:n], U64[:n], F32[:n]):
        for perm in itertools.permutations(range(n)):
            a = ordered[list(perm)] if n else ordered[:0]
            for minrun, g in ((1, 3), (8, 7)):
                out, _ = baseline.sort(a, minrun=minrun, gallop_after=g)
                assert np.array_equal(out.view(np.uint8), ordered.view(np.uint8)), (perm, minrun)


@pytest.mark.parametrize("minrun,gallop", [(1, 1), (2, 3), (8, 7)])
def test_stable_on_every_ternary_sequence(minrun, gallop):
    """Payload = index: the output is the order of (key, index) (Python's
    sorted), including descending stretches with equal keys at their ends
    (reversed stably, reading 3)."""
    for n in range(0, 9):
        idx = np.arange(n, dtype=np.uint32)
        for seq in itertools.product(range(3), repeat=n):
            k = np.array(seq, dtype=np.int32)
            (ok, op), _ = baseline.sort(k, idx, minrun=minrun, gallop_after=gallop)
            assert list(op) == sorted(range(n), key=lambda i: (seq[i], i)), seq


@pytest.mark.parametrize("kind", ["random", "reversed", "nearly", "few"])
def test_matches_the_oracle(kind):
    for n in (1000, 4097, 65537, 300_001):
        a = inputs.int32_of_type(kind, n, n + 3)
        p = np.arange(n, dtype=np.uint32)
        for minrun, g in ((8, 7), (1, 3), (64, 2)):
            (ok, op), _ = baseline.sort(a, p, minrun=minrun, gallop_after=g)
            wk, wp = oracle.sort_pairs(a, p)
            assert np.array_equal(ok, wk) and np.array_equal(op, wp), (n, minrun)


@pytest.mark.parametrize("name", ["equal_teeth", "even_teeth", "sharp_teeth", "shuffled_teeth", "distance",
                                  "exchange", "limited"])
def test_classes_match_the_oracle(name):
    for k in (1, 2, 16, 256):
        a = inputs.class_int32(name, 50_001, k, k)
        out, _ = baseline.sort(a)
        assert np.array_equal(out, oracle.sort_keys(a)), k


def test_comparison_counts_closed_forms():
    for n in (1, 2, 3, 100, 5000):
        # one scan over a single run: n - 1 comparisons, nothing to merge
        assert baseline.sort(np.arange(n, dtype=np.int32))[1] == n - 1
        assert baseline.sort(np.arange(n, dtype=np.int32)[::-1].copy())[1] == n - 1
        assert baseline.sort(np.full(n, 4, dtype=np.int32))[1] == n - 1
    assert baseline.sort(np.zeros(0, dtype=np.int32))[1] == 0


def test_comparison_count_of_the_sec3_example():
    """Sec. 3's example, without minimum run length and galloping after three
    wins (as there).  Scan: 4 ascents and the descent that ends the first run,
    then 1 + 9 comparisons for the reversed run: 15.  Merge of (1 15 18 19 20)
    with (2 .. 11 16): trimming A's 1 takes 2 comparisons (1 <= 2, 15 > 2),
    trimming B takes 1 (16 is not above 20); A's 15..20 go to temporary
    memory; 2, 3, 4 win one by one (3); galloping places 15 between 11 and 16
    with 4 doubling probes (5, 6, 8, 16) and 2 bisection probes (10, 11),
    moving 5..11 at once (6); 15 beats 16 and 16 beats 18 (2); 18..20 follow
    uncompared.  Total 15 + 2 + 1 + 3 + 6 + 2 = 29."""
    ex = np.array([1, 15, 18, 19, 20, 16, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2], dtype=np.int32)
    out, c = baseline.sort(ex, minrun=1, gallop_after=3)
    assert list(out) == [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 15, 16, 18, 19, 20]
    assert c == 29


def test_bad_arguments():
    with pytest.raises(TypeError):
        baseline.sort(np.zeros(3, dtype=np.int16))
    with pytest.raises(ValueError):
        baseline.sort(np.zeros(3, dtype=np.int32), gallop_after=0)
