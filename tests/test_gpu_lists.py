"""GPU sort of heavy list items (Sec. 2: random lists of 16, 64 and 256
integers) through the C ABI, bit-exact against the oracle's stable
word-by-word mergesort."""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
I32 = np.iinfo(np.int32)


def gpu_sort_lists(gpu, a):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32).copy()).to(DEV)
    gpu.sort_lists(t)
    return t.cpu().numpy()


def random_lists(n, L, seed, lo=None, hi=None):
    return inputs.random_lists(n, L, seed, lo, hi)


@pytest.mark.parametrize("L", [16, 64, 256])
@pytest.mark.parametrize("n", [2, 1000, 100_003])
def test_random_lists_of_the_paper(gpu, L, n):
    a = random_lists(n, L, seed=n + L)
    assert np.array_equal(gpu_sort_lists(gpu, a), oracle.sort_lists(a))


@pytest.mark.parametrize("L", [1, 2, 3, 5, 16, 33])
def test_ties_refined_word_by_word(gpu, L):
    """Small alphabets: prefixes tie often, so the refinement rounds run."""
    for n, lo, hi in ((50_000, -1, 2), (20_011, 0, 2), (9_000, -3, 4)):
        a = random_lists(n, L, seed=L * 7 + n, lo=lo, hi=hi)
        assert np.array_equal(gpu_sort_lists(gpu, a), oracle.sort_lists(a)), (n, L, lo, hi)


def test_long_equal_prefixes(gpu):
    n, L = 30_000, 64
    a = random_lists(n, L, seed=5, lo=-2, hi=2)
    a[:, :40] = 7                          # ties through 20 refinement rounds
    a[::3, :62] = -9
    a[::11] = a[0]                         # whole-list duplicates
    assert np.array_equal(gpu_sort_lists(gpu, a), oracle.sort_lists(a))
    b = np.full((4097, 16), 3, np.int32)   # every list equal
    assert np.array_equal(gpu_sort_lists(gpu, b), b)


def test_extreme_words(gpu):
    vals = np.array([I32.min, I32.min + 1, -1, 0, 1, I32.max - 1, I32.max], np.int32)
    rng = np.random.default_rng(3)
    a = vals[rng.integers(0, vals.size, size=(40_000, 4))]
    assert np.array_equal(gpu_sort_lists(gpu, a), oracle.sort_lists(a))


def test_sorted_and_reversed_lists(gpu):
    a = oracle.sort_lists(random_lists(70_000, 16, seed=9, lo=-50, hi=50))
    assert np.array_equal(gpu_sort_lists(gpu, a), a)
    assert np.array_equal(gpu_sort_lists(gpu, a[::-1].copy()), a)


def test_million_lists(gpu):
    a = random_lists(1_000_003, 16, seed=11)
    a[::1000, :2] = 0                      # some prefix ties at scale
    assert np.array_equal(gpu_sort_lists(gpu, a), oracle.sort_lists(a))


def test_errors_and_trivial(gpu):
    lib = gpu.load()
    t = torch.zeros(8, 4, dtype=torch.int32, device=DEV)
    assert lib.sr_sort_lists(t.data_ptr(), 8, 0, None) == 1
    assert lib.sr_sort_lists(t.data_ptr() + 2, 8, 4, None) == 1
    assert lib.sr_sort_lists(None, 8, 4, None) == 1
    assert lib.sr_sort_lists(None, 1, 4, None) == 0
    one = torch.tensor([[5, -1, 2]], dtype=torch.int32, device=DEV)
    gpu.sort_lists(one)
    assert one.cpu().tolist() == [[5, -1, 2]]
