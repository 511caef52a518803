"""Caller-owned scratch (sr_set_workspace) through the C ABI.

On a stream whose data scratch is a buffer the caller set: keys, pairs and
segmented sorts of every input type give the oracle's results bit for bit;
no device memory is allocated once the buffer is set (the device's free
memory does not move across the calls); a call whose scratch does not fit is
rejected before it touches the keys; NULL gives the scratch back to the
library, and sorts go on as before.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import inputs

from test_gpu_sort import bits, from_dev, to_dev

pytestmark = pytest.mark.gpu

NMAX = 3_000_000


def test_sorts_on_a_caller_workspace(gpu):
    st = torch.cuda.Stream()
    nbytes = gpu.workspace_bytes("uint64", True, NMAX, 64)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    assert buf.data_ptr() % 256 == 0
    # inputs and expected results first, so nothing below allocates on the device
    cases = []
    for n in (1000, 100_003, NMAX):
        for i, kind in enumerate(inputs.TYPES):
            a = inputs.int32_of_type(kind, n, 40 + i)
            cases.append(("keys", "int32", a, None, None, oracle.sort_keys(a)))
    k64, p64 = inputs.runs_uint64(1_000_003, seed=8, tie_stress=True)
    cases.append(("pairs", "uint64", k64, p64, None, oracle.sort_pairs(k64, p64)))
    f = inputs.normal_float32(NMAX, seed=9)
    cases.append(("keys", "float32", f, None, None, oracle.sort_keys(f)))
    sk, off, _ = inputs.segments_int32(64, seed=10, hi=65536)
    cases.append(("seg", "int32", sk, None, off, oracle.sort_segmented(sk, off)))
    orig = [(to_dev(c[2]), to_dev(c[3].view(np.int32)) if c[3] is not None else None,
             torch.from_numpy(c[4]).cuda() if c[4] is not None else None) for c in cases]
    work = [(k.clone(), p.clone() if p is not None else None, o) for k, p, o in orig]
    torch.cuda.synchronize()

    def sort_all():
        for (what, dt, *_), (tk, tp, to), (ok, op, _) in zip(cases, work, orig):
            tk.copy_(ok)
            if tp is not None:
                tp.copy_(op)
            if what == "keys":
                gpu.sort_keys(tk, dtype=dt, stream=st)
            elif what == "pairs":
                gpu.sort_pairs(tk, tp, dtype=dt, stream=st)
            else:
                gpu.sort_segmented(tk, to, dtype=dt, stream=st)
        st.synchronize()

    with torch.cuda.stream(st):
        gpu.set_workspace(buf, stream=st)
        sort_all()  # first launches of every kernel load code; then nothing may allocate
        free0, _ = torch.cuda.mem_get_info()
        sort_all()
        free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    for (what, dt, a, p, o, want), (tk, tp, to) in zip(cases, work):
        if what == "pairs":
            assert np.array_equal(bits(from_dev(tk, a)), bits(want[0])), (what, dt, a.size)
            assert np.array_equal(from_dev(tp, p), want[1]), (what, dt, a.size)
        else:
            assert np.array_equal(bits(from_dev(tk, a)), bits(want)), (what, dt, a.size)

    # a call that does not fit is rejected before anything is enqueued
    big = to_dev(inputs.random_int32(nbytes // 4 + 1000, seed=11))
    ref = big.clone()
    torch.cuda.synchronize()
    with pytest.raises(gpu.SortraceError) as err:
        gpu.sort_keys(big, dtype="int32", stream=st)
    assert err.value.status == 1 and "too small" in str(err.value)
    st.synchronize()
    assert torch.equal(big, ref)

    # NULL: the library's own scratch again, the caller's buffer unused
    gpu.set_workspace(None, stream=st)
    buf.fill_(0xA5)
    with torch.cuda.stream(st):
        gpu.sort_keys(big, dtype="int32", stream=st)
    st.synchronize()
    assert bool((buf == 0xA5).all())
    want = np.sort(ref.cpu().numpy())
    assert np.array_equal(big.cpu().numpy(), want)
    assert gpu.load().sr_release_stream(st.cuda_stream) == 0


def test_workspace_argument_errors(gpu):
    buf = torch.empty(1 << 21, dtype=torch.uint8, device="cuda:0")
    lib = gpu.load()
    assert lib.sr_set_workspace(buf.data_ptr() + 128, 1 << 20, None) == 1
    assert lib.sr_set_workspace(buf.data_ptr(), (1 << 20) - 1, None) == 1
    st = torch.cuda.Stream()
    assert lib.sr_set_workspace(buf.data_ptr(), 1 << 21, st.cuda_stream) == 0
    # the stream sorts a small array in the 2 MiB buffer, then gives it back
    t = to_dev(inputs.random_int32(50_000, seed=12))
    want = np.sort(t.cpu().numpy())
    gpu.sort_keys(t, dtype="int32", stream=st)
    st.synchronize()
    assert np.array_equal(t.cpu().numpy(), want)
    assert lib.sr_set_workspace(None, 0, st.cuda_stream) == 0
    assert lib.sr_release_stream(st.cuda_stream) == 0
