"""Sorts of more than 2^31 keys, so that positions, counts and offsets pass
the int32 range, on every path of the device plan.

Each input is a permutation of a known multiset, built on the device from a
closed form, so the sorted output is known without sorting:
  general     keys p(i) - 2^30 with p(i) = (a i + b) mod n, a bijection of
              [0, n) when gcd(a, n) = 1: the output is exactly
              -2^30 .. n - 1 - 2^30
  pairs       keys p(i) >> 1 (every value twice, the last once), payload i:
              key k comes from the inputs p^-1(2k) and p^-1(2k + 1), which a
              stable sort keeps in input order
  reversed, nearly sorted (a swap every 100,003 keys), 8 interleaved teeth
              (tooth t = t, t + 8, t + 16, ...: natural runs)
              all of them permutations of -2^30 .. n - 1 - 2^30
  few unique  16 values drawn at random: the output holds each value as many
              times as the input (counted before the sort), in order
The arrays take 8.6 GB each; the test is skipped on a device with less than
96 GB free.
"""
import math

import pytest
import torch

pytestmark = pytest.mark.gpu

N = (1 << 31) + 12_345
A, B = 1_327_217_885, 987_654_321
OFF = 1 << 30
DEV = "cuda:0"
CH = 1 << 28  # chunk of the device-side generators and checks


@pytest.fixture(scope="module")
def big(gpu):
    free, _ = torch.cuda.mem_get_info()
    if free < (96 << 30):
        pytest.skip("needs 96 GB of free device memory")
    assert math.gcd(A, N) == 1
    return gpu


def perm_chunk(s, e):
    i = torch.arange(s, e, dtype=torch.int64, device=DEV)
    return (i * A + B) % N


def build(fn):
    out = torch.empty(N, dtype=torch.int32, device=DEV)
    for s in range(0, N, CH):
        e = min(N, s + CH)
        out[s:e] = fn(s, e).to(torch.int32)
    return out


def u32_bits(x):
    """int64 values in [0, 2^32) as the int32 values with the same bits."""
    return x - ((x >> 31) << 32)


def assert_arange(t, off):
    for s in range(0, N, CH):
        e = min(N, s + CH)
        want = torch.arange(s, e, dtype=torch.int64, device=DEV) - off
        got = t[s:e].to(torch.int64)
        if not torch.equal(got, want):
            bad = (got != want).nonzero()[0].item() + s
            raise AssertionError(f"first mismatch at {bad}: {t[bad].item()} != {bad - off}")


def test_general_past_int32_positions(big):
    t = build(lambda s, e: perm_chunk(s, e) - OFF)
    big.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    assert big.last_stats()["path"] == "general"
    assert_arange(t, OFF)


def test_pairs_stable_past_int32_positions(big):
    keys = build(lambda s, e: perm_chunk(s, e) >> 1)
    # payload i as uint32 bits in an int32 tensor
    pay = build(lambda s, e: u32_bits(torch.arange(s, e, dtype=torch.int64, device=DEV)))
    big.sort_pairs(keys, pay, dtype="int32")
    torch.cuda.synchronize()
    a_inv = pow(A, -1, N)
    for s in range(0, N, CH):
        e = min(N, s + CH)
        j = torch.arange(s, e, dtype=torch.int64, device=DEV)
        assert torch.equal(keys[s:e].to(torch.int64), j >> 1), s
        k = j >> 1
        i1 = ((2 * k - B) % N) * a_inv % N
        i2 = ((2 * k + 1 - B) % N) * a_inv % N
        has2 = (2 * k + 1) < N
        lo = torch.where(has2, torch.minimum(i1, i2), i1)
        hi = torch.where(has2, torch.maximum(i1, i2), i1)
        want = torch.where((j & 1) == 0, lo, hi)
        got = pay[s:e].to(torch.int64) & 0xFFFFFFFF
        assert torch.equal(got, want), s


@pytest.mark.parametrize("kind", ["reversed", "nearly", "teeth"])
def test_presorted_paths_past_int32_positions(big, kind):
    # values i - 2^30 for i in [0, n): inside the int32 range
    if kind == "reversed":
        t = build(lambda s, e: (N - 1 - OFF) - torch.arange(s, e, dtype=torch.int64, device=DEV))
        path = "reversed"
    elif kind == "nearly":
        t = build(lambda s, e: torch.arange(s, e, dtype=torch.int64, device=DEV) - OFF)
        pos = torch.arange(0, N - 8, 100_003, dtype=torch.int64, device=DEV)
        x, y = t[pos].clone(), t[pos + 7].clone()
        t[pos] = y
        t[pos + 7] = x
        path = "outlier"
    else:
        t = torch.cat([(torch.arange(r, N, 8, dtype=torch.int64, device=DEV) - OFF).to(torch.int32)
                       for r in range(8)])
        path = "runs"
    assert t.numel() == N
    big.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    assert big.last_stats()["path"] == path
    assert_arange(t, OFF)


def test_few_unique_past_int32_positions(big):
    g = torch.Generator(device=DEV)
    g.manual_seed(16)
    t = build(lambda s, e: torch.randint(0, 16, (e - s,), generator=g, device=DEV, dtype=torch.int64))
    counts = torch.zeros(16, dtype=torch.int64, device=DEV)
    for s in range(0, N, CH):
        counts += torch.bincount(t[s:s + CH].to(torch.int64), minlength=16)
    big.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    assert big.last_stats()["path"] == "few"
    start = 0
    for v, c in enumerate(counts.tolist()):
        assert bool((t[start:start + c] == v).all()), (v, start, c)
        start += c
    assert start == N
