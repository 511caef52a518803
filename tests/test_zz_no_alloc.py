"""sr_sort_keys_noalloc (the allocation-free entry point) against sr_sort_keys.

Each case sorts the same input through both entry points, two calls in a row
with the second input smaller than the first (the shared scratch array keeps
the first call's contents), and compares the results bit for bit with each
other and with the oracle.  The device's free memory must not move across
calls of the allocation-free entry point."""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LIMIT_BYTES = 32 << 20


def _dev(a):
    view = {4: np.int32, 8: np.int64}[a.itemsize]
    return torch.from_numpy(np.ascontiguousarray(a).view(view).copy()).to(DEV)


def _both(gpu, a, dtype):
    """(noalloc result, sr_sort_keys result) of the host array a."""
    t1, t2 = _dev(a), _dev(a)
    gpu.sort_keys_noalloc(t1, dtype=dtype)
    gpu.sort_keys(t2, dtype=dtype)
    torch.cuda.synchronize()
    return t1.cpu().numpy().view(a.dtype), t2.cpu().numpy().view(a.dtype)


def _check(gpu, a, dtype):
    got, ref = _both(gpu, a, dtype)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
    assert np.array_equal(got.view(np.uint8), oracle.sort_keys(a).view(np.uint8))


@pytest.mark.parametrize("kind", ["random", "reversed", "nearly", "few"])
def test_noalloc_matches_sort_keys_two_calls(gpu, kind):
    for n in (5_000_003, 300_001):
        print(f"[noalloc] int32 {kind} n={n}", flush=True)
        _check(gpu, inputs.int32_of_type(kind, n, inputs.seed_for(2, inputs.TYPES.index(kind), n)), "int32")


@pytest.mark.parametrize("dtype", ["float32", "uint64"])
def test_noalloc_other_dtypes_two_calls(gpu, dtype):
    big = LIMIT_BYTES // (4 if dtype == "float32" else 8)
    for n in (big, 77_777):
        print(f"[noalloc] {dtype} n={n}", flush=True)
        a = inputs.normal_float32(n, seed=n) if dtype == "float32" else inputs.stream(n, n)
        _check(gpu, a, dtype)


def test_noalloc_limit_and_memory(gpu):
    n = LIMIT_BYTES // 4
    a = inputs.random_int32(n, seed=5)
    b = inputs.runs_uint64(300_000, seed=6)[0]
    small = inputs.class_int32("sharp_teeth", 9000, 4, 1)
    t_a, t_b, t_s = _dev(a), _dev(b), _dev(small)
    over = torch.zeros(n + 1, dtype=torch.int32, device=DEV)
    gpu.sort_keys_noalloc(_dev(small[:20_000]), dtype="int32")   # the device's one-time set-up
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    print("[noalloc] limit-size int32, then uint64 runs, then a small one", flush=True)
    gpu.sort_keys_noalloc(t_a, dtype="int32")
    gpu.sort_keys_noalloc(t_b, dtype="uint64")
    gpu.sort_keys_noalloc(t_s, dtype="int32")
    with pytest.raises(gpu.SortraceError) as e:
        gpu.sort_keys_noalloc(over, dtype="int32")
    assert "limit" in str(e.value)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert bool((over == 0).all())
    assert np.array_equal(t_a.cpu().numpy(), oracle.sort_keys(a))
    assert np.array_equal(t_b.cpu().numpy().view(np.uint64), oracle.sort_keys(b))
    assert np.array_equal(t_s.cpu().numpy(), oracle.sort_keys(small))
