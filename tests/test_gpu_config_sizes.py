"""GPU parity against the oracle, element by element, at the full sizes of the
benchmarked workloads and in the launch configuration bench.py times:

  2^20 uniform int32 keys, one sr_sort_keys call
  2^24 stable (uint64 key, uint32 payload = index) pairs, keys in geometric
       runs of mean length 1000 with 10 % equal steps, one sr_sort_pairs call
  4096 segments of log-uniform lengths in [16, 262144] (~107M int32 keys,
       each segment one of the four input types), one sr_sort_segmented call
       replayed from its captured hipGraph
  served requests of 1,024 .. 16,777,216 float32 (normal, totalOrder specials)
       and int32 keys through the continuous-batching server

The 256M-key random case is in test_gpu_full_size.py.  Each oracle sort runs
in a worker thread (the C oracle releases the interpreter lock) while the GPU
works, and every comparison is bitwise (tolerance 0).
"""
import concurrent.futures as cf

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(f"[config-sizes] {msg}", flush=True)


@pytest.mark.timeout(600)
def test_config_2p20_int32_keys(gpu):
    n = 1 << 20
    a = inputs.random_int32(n, inputs.seed_for(1, 0, n))
    t = torch.from_numpy(a).to(DEV)
    gpu.sort_keys(t, dtype="int32")
    torch.cuda.synchronize()
    assert gpu.last_stats()["path"] == "general"
    assert np.array_equal(t.cpu().numpy(), oracle.sort_keys(a))


@pytest.mark.timeout(600)
def test_config_2p24_uint64_pairs_in_runs(gpu):
    n = 1 << 24
    say(f"uint64 pairs n={n}: generating")
    hk, hp = inputs.runs_uint64(n, seed=inputs.seed_for(3, 0, n))
    with cf.ThreadPoolExecutor(1) as ex:
        want = ex.submit(oracle.sort_pairs, hk, hp)
        ks = torch.from_numpy(hk.view(np.int64).copy()).to(DEV)
        ps = torch.from_numpy(hp.view(np.int32).copy()).to(DEV)
        gpu.sort_pairs(ks, ps, dtype="uint64")
        torch.cuda.synchronize()
        gk = ks.cpu().numpy().view(np.uint64)
        gp = ps.cpu().numpy().view(np.uint32)
        say("uint64 pairs: GPU done, waiting for the oracle")
        wk, wp = want.result()
    assert np.array_equal(gk, wk)
    assert np.array_equal(gp, wp)
    # the properties bench.py checks, as extra asserts
    assert np.all((gk[1:] != gk[:-1]) | (gp[1:] > gp[:-1]))
    assert np.array_equal(gk, hk[gp])


@pytest.mark.timeout(900)
def test_config_4096_segments_graph(gpu):
    say("4096 segments: generating")
    hk, hoff, kinds = inputs.segments_int32(4096, seed=inputs.seed_for(4, 0, 0))
    assert hoff.size == 4097 and int(hoff[-1]) > 100_000_000
    with cf.ThreadPoolExecutor(1) as ex:
        want = ex.submit(oracle.sort_segmented, hk, hoff)
        pristine = torch.from_numpy(hk).to(DEV)
        off = torch.from_numpy(hoff).to(DEV)
        work = torch.empty_like(pristine)
        gpu.set_option("graph", 1)
        try:
            outs = []
            for rep in range(3):      # capture, then two replays with eager work between
                work.copy_(pristine)
                gpu.sort_segmented(work, off, dtype="int32")
                torch.cuda.synchronize()
                outs.append(work.cpu().numpy())
        finally:
            gpu.set_option("graph", 0)
        say("4096 segments: GPU done, waiting for the oracle")
        w = want.result()
    for rep, got in enumerate(outs):
        assert np.array_equal(got, w), f"replay {rep}"


@pytest.mark.timeout(900)
def test_config_serving_full_sizes(gpu):
    """Requests at both ends of the size range and between, both dtypes, with
    overlapping arrivals; every result equals the oracle's sort of it."""
    sizes = [16_777_216, 1024, 5_000_000, 16_777_216, 1500, 200_000, 9_999_999, 65_536, 3_000_000, 1024]
    reqs = []
    for i, n in enumerate(sizes):
        s = inputs.seed_for(5, 7, i)
        reqs.append(inputs.normal_float32(n, seed=s) if i % 2 == 0 else inputs.uniform_int32(n, seed=s))
    with cf.ThreadPoolExecutor(4) as ex:
        wants = [ex.submit(oracle.sort_keys, a) for a in reqs]
        devs = [torch.from_numpy(a.view(np.int32).copy()).to(DEV) for a in reqs]
        torch.cuda.synchronize()
        with gpu.Server(1 << 30, streams=4, max_batch_requests=64, max_batch_keys=1 << 26) as srv:
            t0 = srv.now()
            for i, (a, t) in enumerate(zip(reqs, devs)):
                srv.submit(t, tag=i, t_arrive=t0 + 0.001 * (i // 3),
                           dtype="float32" if a.dtype == np.float32 else "int32")
            srv.wait_idle(120)
            recs = srv.records()
        assert sorted(r["tag"] for r in recs) == list(range(len(reqs)))
        assert all(r["status"] == 0 for r in recs)
        say("serving: GPU done, waiting for the oracle")
        for i, (t, w) in enumerate(zip(devs, wants)):
            assert np.array_equal(t.cpu().numpy(), w.result().view(np.int32)), f"request {i} ({sizes[i]} keys)"
