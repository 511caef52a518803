"""GPU parity at the full 256M-key size of the benchmark, in the launch
configuration bench.py times (one sr_sort_keys call on a resident array).

  random        element by element against the oracle's mergesort of the
                same 2^28 keys (run in a worker thread while the GPU works);
                as extra checks, properties that hold at any size: the
                output is nondecreasing; it is a permutation of the input
                (equal counts of every 16-bit prefix, equal sums of keys and
                of squared keys); and at 64 sampled output positions p the
                value v = out[p] has exactly the definition's rank: fewer
                than p + 1 input keys are below v and more than p are at most v
                (counted directly on the device, independent of the sort)
  reversed, nearly sorted   exactly 0 .. n-1
  few unique    exactly the input's values in order, each repeated its count
"""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu

N = 1 << 28
DEV = "cuda:0"


def sort_on_gpu(gpu, a: np.ndarray) -> torch.Tensor:
    t = torch.from_numpy(a).to(DEV)
    gpu.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    return t


@pytest.mark.timeout(900)
def test_random_256M(gpu):
    a = inputs.int32_of_type("random", N, inputs.seed_for(2, 0, N))
    ex = cf.ThreadPoolExecutor(1)
    want = ex.submit(oracle.sort_keys, a)
    print("[full-size] 256M random: oracle started", flush=True)
    src = torch.from_numpy(a).to(DEV)
    out = src.clone()
    gpu.sort_keys(out, dtype="int32")
    torch.cuda.synchronize()
    assert gpu.last_stats()["path"] == "general"
    assert bool((out[1:] >= out[:-1]).all())
    hi_in = torch.bincount(((src.to(torch.int64) + 2**31) >> 16), minlength=1 << 16)
    hi_out = torch.bincount(((out.to(torch.int64) + 2**31) >> 16), minlength=1 << 16)
    assert torch.equal(hi_in, hi_out)
    s_in, s_out = src.to(torch.int64), out.to(torch.int64)
    assert int(s_in.sum()) == int(s_out.sum())
    assert int((s_in * s_in).sum()) == int((s_out * s_out).sum())
    rng = np.random.default_rng(1)
    for p in [0, N - 1] + list(rng.integers(0, N, size=62)):
        v = int(out[int(p)])
        below = int((src < v).sum())
        at_most = int((src <= v).sum())
        assert below <= p < at_most, (p, v, below, at_most)
    got = out.cpu().numpy()
    del out, src, s_in, s_out
    print("[full-size] 256M random: GPU checks done, waiting for the oracle", flush=True)
    w = want.result()
    ex.shutdown()
    assert np.array_equal(got, w)


@pytest.mark.parametrize("kind", ["reversed", "nearly"])
def test_presorted_256M_closed_form(gpu, kind):
    a = inputs.int32_of_type(kind, N, inputs.seed_for(2, inputs.TYPES.index(kind), N))
    out = sort_on_gpu(gpu, a)
    want_path = {"reversed": "reversed", "nearly": "outlier"}[kind]
    assert gpu.last_stats()["path"] == want_path
    assert torch.equal(out, torch.arange(N, dtype=torch.int32, device=DEV))


def test_few_unique_256M(gpu):
    a = inputs.int32_of_type("few", N, inputs.seed_for(2, 3, N))
    v, c = np.unique(a, return_counts=True)
    out = sort_on_gpu(gpu, a)
    assert gpu.last_stats()["path"] == "few"
    want = torch.repeat_interleave(torch.from_numpy(v).to(DEV), torch.from_numpy(c).to(DEV))
    assert torch.equal(out, want)
