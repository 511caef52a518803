"""GPU tests of the tuning table: rows select the launch shape of a sort
(seen through the per-kernel launch record), explicit options override
rows, every shape the autotuner sweeps sorts bit-exactly like the oracle,
and a short sweep writes a table that loads back."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04471_amd import autotune, inputs

from test_gpu_sort import bits, gpu_sort_keys, gpu_sort_pairs

pytestmark = pytest.mark.gpu


@pytest.fixture
def clean(gpu):
    """No table and every shape option on auto; afterwards the table the
    library had (the shipped one) is restored."""
    saved = gpu.tune_get()
    gpu.tune_set([])
    yield gpu
    gpu.tune_set(saved)
    for name, auto in (("partition_min_n", -1), ("tile_variant", -1), ("merge_items", 0),
                       ("merge_nontemporal", -1), ("profile", 0)):
        gpu.set_option(name, auto)
    gpu.profile_collect("")


def partition_launches(gpu, a):
    """Sort a through the library with the launch record on; returns the
    number of separate partition launches and checks the result."""
    gpu.set_option("profile", 1)
    gpu.profile_collect("")
    try:
        assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a))
        torch.cuda.synchronize()
        return gpu.profile_collect("partition")[0]
    finally:
        gpu.set_option("profile", 0)


def test_rows_choose_the_partition_launch(clean):
    gpu = clean
    a = inputs.random_int32(100_003, seed=5)
    assert partition_launches(gpu, a) == 0          # built-in: fused below 2^23
    gpu.tune_set([{"dtype": "int32", "min_n": 0, "partition": 1}])
    assert partition_launches(gpu, a) == 4          # ceil(log2(13 tiles)) passes
    gpu.tune_set([{"dtype": "uint64", "min_n": 0, "partition": 1},
                  {"dtype": "int32", "pairs": True, "min_n": 0, "partition": 1}])
    assert partition_launches(gpu, a) == 0          # other kinds' rows do not apply
    gpu.tune_set([{"dtype": "int32", "min_n": 0, "partition": 0},
                  {"dtype": "int32", "min_n": 50_000, "partition": 1}])
    assert partition_launches(gpu, a[:40_000].copy()) == 0
    assert partition_launches(gpu, a[:60_000].copy()) == 3
    gpu.set_option("partition_min_n", 1 << 30)      # explicit option wins over the row
    assert partition_launches(gpu, a[:60_000].copy()) == 0
    gpu.set_option("partition_min_n", -1)
    assert partition_launches(gpu, a[:60_000].copy()) == 3


@pytest.mark.parametrize("dtype,pairs", [("int32", False), ("float32", False), ("uint64", False),
                                         ("int32", True), ("uint64", True)])
def test_every_swept_shape_matches_the_oracle(clean, dtype, pairs):
    gpu = clean
    for n in (70_001, 1_000_003):
        seed = n + 7
        if dtype == "int32":
            k = inputs.random_int32(n, seed)
        elif dtype == "float32":
            k = inputs.normal_float32(n, seed)
        else:
            k = inputs.runs_uint64(n, seed, tie_stress=True)[0]
        p = np.arange(n, dtype=np.uint32)[::-1].copy()
        want = oracle.sort_pairs(k, p) if pairs else oracle.sort_keys(k)
        for shape in autotune.candidates(dtype, pairs):
            gpu.tune_set([{"dtype": dtype, "pairs": pairs, "min_n": 0, **shape}])
            if pairs:
                gk, gp = gpu_sort_pairs(gpu, k, p, dtype)
                assert np.array_equal(bits(gk), bits(want[0])) and np.array_equal(gp, want[1]), (n, shape)
            else:
                assert np.array_equal(bits(gpu_sort_keys(gpu, k, dtype)), bits(want)), (n, shape)


def test_presorted_paths_under_every_shape(clean):
    gpu = clean
    n = 300_007
    cases = {kind: inputs.int32_of_type(kind, n, 31 + len(kind)) for kind in inputs.TYPES}
    want = {kind: oracle.sort_keys(a) for kind, a in cases.items()}
    for shape in autotune.candidates("int32", False):
        gpu.tune_set([{"dtype": "int32", "min_n": 0, **shape}])
        for kind, a in cases.items():
            assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), want[kind]), (kind, shape)


def test_short_sweep_writes_a_loadable_table(clean, tmp_path):
    gpu = clean
    table = autotune.sweep(dtypes=("int32", "uint64"), kinds=(False, True), lo=16, hi=18, step=2, reps=2,
                           log=lambda s: None)
    assert table["format"] == autotune.FORMAT and len(table["rows"]) == 8
    for r in table["rows"]:
        assert r["ms"] > 0 and r["builtin_ms"] > 0
        assert {k: v for k, v in r.items() if k in gpu.TUNE_FIELDS} in autotune.candidates(r["dtype"], r["pairs"])
    assert gpu.tune_get() == []                     # the sweep restores the table it found (none here)
    p = tmp_path / "tune.json"
    p.write_text(json.dumps(dict(table, rows=autotune.compress(table["rows"]))))
    rows = autotune.apply(str(p))
    assert len(gpu.tune_get()) == len(rows) >= 4
    a = inputs.random_int32(200_001, seed=9)
    assert np.array_equal(gpu_sort_keys(gpu, a, "int32"), oracle.sort_keys(a))


def test_shipped_table_is_valid_and_loaded(gpu):
    """The table shipped with the package names only swept shapes and is the
    one the binding applied at load (unless SR_TUNE_TABLE overrides it)."""
    import os
    rows = autotune.validate(json.load(open(gpu.TUNE_TABLE)))
    for r in rows:
        shape = {k: v for k, v in r.items() if k in gpu.TUNE_FIELDS}
        swept = autotune.seg_candidates(r["dtype"]) if r["segmented"] else autotune.candidates(r["dtype"], r["pairs"])
        assert shape in swept, r
    if "SR_TUNE_TABLE" not in os.environ:
        got = gpu.tune_get()
        want = sorted(rows, key=lambda r: (gpu.DTYPES[r["dtype"]], r["pairs"], r["segmented"], r["min_n"]))
        assert [(g["dtype"], g["pairs"], g["segmented"], g["min_n"]) for g in got] == \
            [(w["dtype"], w["pairs"], w["segmented"], w["min_n"]) for w in want]


@pytest.mark.parametrize("tile_variant,merge_items", [(0, 8), (1, 8), (1, 16), (0, 16)])
def test_segmented_rows_choose_the_batch_shape(clean, tile_variant, merge_items):
    """A segmented row of the table sets the tile shape and merge outputs of
    sr_sort_segmented / sr_sort_batch (32-bit keys): every shape sorts the
    batched-workload mix exactly as the oracle."""
    from paper_1609_04471_amd import sortrace
    keys, off, _ = inputs.segments_int32(160, seed=12)
    sortrace.tune_set([{"dtype": "int32", "pairs": False, "segmented": True, "min_n": 0,
                        "tile_variant": tile_variant, "merge_items": merge_items}])
    t = torch.from_numpy(keys.copy()).to("cuda:0")
    sortrace.sort_segmented(t, torch.from_numpy(off).to("cuda:0"), dtype="int32")
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), oracle.sort_segmented(keys, off))
    f = keys.astype(np.float32) * np.float32(0.5)
    tf = torch.from_numpy(f.copy()).to("cuda:0")
    sortrace.tune_set([{"dtype": "float32", "pairs": False, "segmented": True, "min_n": 0,
                        "tile_variant": tile_variant, "merge_items": merge_items}])
    arrays = [tf[int(off[i]):int(off[i + 1])] for i in range(0, 160, 7)]
    sortrace.sort_batch(arrays, dtype="float32")
    torch.cuda.synchronize()
    got = tf.cpu().numpy()
    for i in range(0, 160, 7):
        a, b = int(off[i]), int(off[i + 1])
        assert np.array_equal(got[a:b].view(np.uint32), oracle.sort_keys(f[a:b]).view(np.uint32))
