"""Serving: every request's result is the same alone and in the mix.

Requests of both dtypes (int32 uniform, float32 normal with totalOrder
specials) and mixed sizes go through the continuous-batching server with
staggered arrivals; each result is compared bit for bit with the same
array sorted alone by sr_sort_keys and with the oracle (tolerance 0).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make_requests(count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(1024), np.log(400_000))))
        if i % 2:
            a = inputs.normal_float32(n, seed=seed * 1000 + i)
        else:
            a = inputs.uniform_int32(n, seed=seed * 1000 + i)
        reqs.append(a)
    return reqs


def to_dev(a):
    return torch.from_numpy(a.view(np.int32).copy()).to(DEV)


@pytest.mark.parametrize("streams,max_batch", [(4, 16), (1, 1), (2, 64)])
def test_alone_equals_mix(gpu, streams, max_batch):
    reqs = make_requests(48, seed=streams * 10 + max_batch)
    mix = [to_dev(a) for a in reqs]
    alone = [to_dev(a) for a in reqs]
    torch.cuda.synchronize()
    budget = 24 << 20  # small enough that admission binds
    with gpu.Server(budget, streams=streams, max_batch_requests=max_batch, max_batch_keys=1 << 22) as srv:
        t0 = srv.now()
        for i, (a, t) in enumerate(zip(reqs, mix)):
            # bursts of 8 simultaneous arrivals, 0.5 ms apart
            srv.submit(t, tag=i, t_arrive=t0 + 0.0005 * (i // 8), dtype="float32" if a.dtype == np.float32 else "int32")
        srv.wait_idle(60)
        recs = srv.records()
    assert sorted(r["tag"] for r in recs) == list(range(len(reqs)))
    assert all(r["status"] == 0 for r in recs)
    assert all(r["t_done"] >= r["t_launch"] >= r["t_admit"] >= r["t_arrive"] - 1e-9 for r in recs)
    if max_batch > 1:
        assert max(len([r for r in recs if r["batch"] == b]) for b in {r["batch"] for r in recs}) > 1
    for a, t in zip(reqs, alone):
        gpu.sort_keys(t, dtype="float32" if a.dtype == np.float32 else "int32")
    torch.cuda.synchronize()
    for a, m, t in zip(reqs, mix, alone):
        mb, tb = m.cpu().numpy(), t.cpu().numpy()
        assert np.array_equal(mb, tb)
        assert np.array_equal(mb, oracle.sort_keys(a).view(np.int32))


def test_sort_batch_api(gpu):
    arrays = [inputs.uniform_int32(n, seed=n) for n in (1, 2, 100, 8192, 8193, 70_000, 300_001)]
    ts = [to_dev(a) for a in arrays]
    keep = gpu.sort_batch(ts, dtype="int32")
    torch.cuda.synchronize()
    for a, t in zip(arrays, ts):
        assert np.array_equal(t.cpu().numpy(), oracle.sort_keys(a))


def test_server_rejects_oversized_request(gpu):
    with gpu.Server(1 << 20, streams=1, max_batch_requests=4, max_batch_keys=1 << 16) as srv:
        t = torch.zeros(1 << 18, dtype=torch.int32, device=DEV)
        with pytest.raises(gpu.SortraceError):
            srv.submit(t, tag=0, t_arrive=srv.now())
