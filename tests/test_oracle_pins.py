"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each expected value is a
closed form, a brute-force definition written here in Python, a value the
paper prints, or a library routine (numpy's stable sort) on an order key the
test derives from the type's definition.  A mutation test at the end plants
plausible mistakes in a private copy of the oracle and checks that these
pins catch every one.
"""
import ctypes
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1609_04471_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# -------------------------------------------------------------- helpers

def total_order_key(a: np.ndarray) -> np.ndarray:
    """Unsigned key whose ascending order is the dtype's order (test-side)."""
    if a.dtype == np.int32:
        return a.view(np.uint32) ^ np.uint32(0x80000000)
    if a.dtype == np.uint64:
        return a
    if a.dtype == np.float32:
        b = a.view(np.uint32)
        neg = (b >> np.uint32(31)) == 1
        return np.where(neg, ~b, b | np.uint32(0x80000000))
    raise TypeError(a.dtype)


def bits(a: np.ndarray) -> np.ndarray:
    return a.view({4: np.uint32, 8: np.uint64}[a.itemsize])


def assert_sorted_permutation(inp, out):
    k = total_order_key(out)
    assert np.all(k[:-1] <= k[1:]), "not nondecreasing"
    u_in, c_in = np.unique(bits(inp), return_counts=True)
    u_out, c_out = np.unique(bits(out), return_counts=True)
    assert np.array_equal(u_in, u_out) and np.array_equal(c_in, c_out), "multiset changed"


# Bit patterns whose IEEE 754-2008 totalOrder (Sec. 5.10) is the list order:
# -NaN(large payload) < -NaN(small payload) < -Inf < -1 < -min subnormal <
# -0 < +0 < +min subnormal < 1 < +Inf < +NaN(small) < +NaN(large).
F32_TOTAL_ORDER = np.array([0xFFFFFFFF, 0xFFC00000, 0xFF800000, 0xBF800000, 0x80000001,
                            0x80000000, 0x00000000, 0x00000001, 0x3F800000, 0x7F800000,
                            0x7FC00000, 0x7FFFFFFF], dtype=np.uint32)
U64_ORDER = np.array([0, 1, 2**31, 2**32, 2**62, 2**63, 2**64 - 2, 2**64 - 1], dtype=np.uint64)
I32_ORDER = np.array([-2**31, -65536, -2, -1, 0, 1, 65536, 2**31 - 1], dtype=np.int32)


# ------------------------------------------------------ P1 brute force

@pytest.mark.parametrize("n", range(0, 9))
def test_all_permutations_sort_to_the_closed_form(n):
    """Every permutation of n distinct keys sorts to the known order."""
    for ordered in (I32_ORDER[:n], U64_ORDER[:n], F32_TOTAL_ORDER[:n].view(np.float32)):
        for perm in itertools.permutations(range(n)):
            a = ordered[list(perm)] if n else ordered[:0]
            out = oracle.sort_keys(a)
            assert np.array_equal(bits(out), bits(ordered)), (ordered.dtype, perm)


@pytest.mark.parametrize("n", range(0, 9))
def test_pairs_match_python_definition_on_all_ternary_inputs(n):
    """All 3^n key sequences over {0,1,2}; payload = index.  The stable result
    is the order of (key, index), computed here by Python's sorted()."""
    idx = np.arange(n, dtype=np.uint32)
    for seq in itertools.product(range(3), repeat=n):
        k = np.array(seq, dtype=np.int32)
        order = sorted(range(n), key=lambda i: (seq[i], i))
        ok, op = oracle.sort_pairs(k, idx)
        assert list(op) == order and list(ok) == [seq[i] for i in order]
        bk, bp = oracle.brute_sort(k, idx)
        assert list(bp) == order


# ------------------------------------------------- P2 insertion sort

@pytest.mark.parametrize("dtype", ["int32", "uint64", "float32"])
def test_mergesort_equals_insertion_sort(dtype):
    rng = np.random.default_rng(1609)
    for n in (0, 1, 2, 3, 17, 100, 777, 2000):
        if dtype == "int32":
            k = rng.integers(-50, 50, n).astype(np.int32) if n % 2 else \
                rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
        elif dtype == "uint64":
            k = rng.integers(0, 2**64 - 1, n, dtype=np.uint64, endpoint=True)
            k[::3] = k[0] if n else 0
        else:
            k = inputs.normal_float32(n, seed=n + 7, specials=True)
            k[::5] = F32_TOTAL_ORDER[rng.integers(0, 12, k[::5].size)].view(np.float32)
        p = np.arange(n, dtype=np.uint32)
        mk, mp = oracle.sort_pairs(k, p)
        ik, ip = oracle.insertion_sort(k, p)
        assert np.array_equal(bits(mk), bits(ik)) and np.array_equal(mp, ip)
        assert np.array_equal(bits(oracle.sort_keys(k)), bits(ik))


# ---------------------------------------------- P3 invariants, P7 library

@pytest.mark.parametrize("dtype", ["int32", "uint64", "float32"])
def test_invariants_and_numpy_stable_sort(dtype):
    rng = np.random.default_rng(4471)
    for n in (5000, 65537):
        if dtype == "int32":
            k = rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
            k[: n // 3] = k[: n // 3] % 7
        elif dtype == "uint64":
            k, _ = inputs.runs_uint64(n, seed=n, tie_stress=True)
        else:
            k = inputs.normal_float32(n, seed=n)
        p = np.arange(n, dtype=np.uint32)
        ok, op = oracle.sort_pairs(k, p)
        assert_sorted_permutation(k, ok)
        # payload is a permutation, and increases inside every equal-key group
        assert np.array_equal(np.sort(op), p)
        key = total_order_key(ok)
        same = key[1:] == key[:-1]
        assert np.all(op[1:][same] > op[:-1][same])
        # library cross-check: numpy's stable argsort of the order key
        ref = np.argsort(total_order_key(k), kind="stable")
        assert np.array_equal(op, ref.astype(np.uint32))
        assert np.array_equal(bits(oracle.sort_keys(k)), bits(ok))


# ------------------------------------------------------ P4 closed forms

@pytest.mark.parametrize("n", [0, 1, 99, 100, 101, 12345, 2_000_000])
def test_generator_closed_forms(n):
    rev = inputs.reversed_int32(n)
    near = inputs.nearly_sorted_int32(n, seed=11)
    ar = np.arange(n, dtype=np.int32)
    assert np.array_equal(oracle.sort_keys(rev), ar)
    assert np.array_equal(oracle.sort_keys(near), ar)
    # exactly 2*floor(n/100) displaced positions
    assert int(np.count_nonzero(near != ar)) == 2 * (n // 100)
    few = inputs.few_unique_int32(n, seed=12)
    vals, counts = np.unique(few, return_counts=True)
    assert vals.size <= 10
    assert np.array_equal(oracle.sort_keys(few), np.repeat(vals, counts))


def test_segmented_matches_per_segment_sort():
    keys, off, kinds = inputs.segments_int32(24, seed=5, lo=1, hi=3000)
    off[3] = off[2]  # an empty segment
    keys = keys[: off[-1]]
    out = oracle.sort_segmented(keys, off)
    for s in range(off.size - 1):
        seg = keys[off[s]:off[s + 1]]
        assert np.array_equal(out[off[s]:off[s + 1]], np.sort(seg, kind="stable"))


# ---------------------------------------------- P5 worked example (Sec. 3)

def _golden(name):
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = v.split()
    return d


def test_paper_worked_example():
    g = _golden("worked_example.txt")
    a = np.array([int(x) for x in g["input"]], dtype=np.int32)
    assert np.array_equal(oracle.sort_keys(a), np.array([int(x) for x in g["sorted"]], np.int32))
    assert oracle.run(a) == int(g["run"][0])
    assert oracle.mono(a) == int(g["mono"][0])


# ------------------------------------- P6 presortedness closed forms (Sec. 2)

def equal_teeth(n, k):
    return np.concatenate([np.arange(1, n // k + 1)] * k).astype(np.int32)


def even_teeth(n, k):
    secs = [np.arange(1, n // k + 1) for _ in range(k)]
    return np.concatenate([s[::-1] if i % 2 == 0 else s for i, s in enumerate(secs)]).astype(np.int32)


def sharp_teeth(n, k):
    secs = np.split(np.arange(1, n + 1), k)
    return np.concatenate([s[::-1] if i % 2 == 0 else s for i, s in enumerate(secs)]).astype(np.int32)


def test_presortedness_closed_forms():
    for n in (1, 2, 7, 64, 501):
        r = inputs.reversed_int32(n)
        assert oracle.inv(r) == n * (n - 1) // 2
        assert oracle.run(r) == n
        assert oracle.mono(r) == 1
        assert oracle.inv(np.sort(r)) == 0 and oracle.run(np.sort(r)) == 1
    n = 600
    organ = np.concatenate([np.arange(300), np.arange(300)[::-1]]).astype(np.int32)
    assert oracle.mono(organ) == 2
    for k in (1, 2, 3, 4, 5, 6, 10, 12, 20, 50, 100, 200):
        assert oracle.run(equal_teeth(n, k)) == k
        assert oracle.mono(equal_teeth(n, k)) == k
        assert oracle.mono(even_teeth(n, k)) == k          # k <= n/3
        assert oracle.mono(sharp_teeth(n, k)) == k          # sections of >= 3 keys
    for n in (8, 16, 400):
        a = even_teeth(n, n // 2)
        assert list(a[:8]) == [2, 1, 1, 2, 2, 1, 1, 2]
        assert oracle.mono(a) == n // 4 + 1
    rng = np.random.default_rng(3)
    for k in (1, 2, 5, 30):
        a = np.arange(500, dtype=np.int32)
        for _ in range(k):
            i, j = rng.integers(0, 500, 2)
            a[i], a[j] = a[j], a[i]
        assert oracle.mono(a) <= 2 * k + 1
        assert np.count_nonzero(a != np.arange(500)) <= 2 * k


# --------------------------- the pins catch planted mistakes in the oracle

MUTATIONS = {
    "merge_ties_go_right": ("if (r->less(a + j * rs, a + i * rs)) {",
                            "if (!r->less(a + i * rs, a + j * rs)) {"),
    "float_sign_flipped": ("return sx > sy;", "return sx < sy;"),
    "float_negative_ascending": ("return x > y;                /* both negative-signed",
                                 "return x < y;                /* both negative-signed"),
    "int32_unsigned": ("    int32_t x, y;\n    memcpy(&x, a, 4);", "    uint32_t x, y;\n    memcpy(&x, a, 4);"),
    "uint64_signed": ("    uint64_t x, y;\n    memcpy(&x, a, 8);", "    int64_t x, y;\n    memcpy(&x, a, 8);"),
    "tail_dropped": ("    while (j < hi) {\n        memcpy(tmp + k * rs, a + j * rs, rs);",
                     "    while (0) {\n        memcpy(tmp + k * rs, a + j * rs, rs);"),
    "split_off_by_one": ("    msort(r, a, tmp, mid, hi);", "    msort(r, a, tmp, mid + 1, hi);"),
}


def _mutant_sorts(tmp_path, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "sortrace_oracle.c")).read()
    old, new = MUTATIONS[name]
    assert old in src, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_sort_pairs.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]

    def sort_pairs(k, p):
        k, p = k.copy(), p.copy()
        lib.oracle_sort_pairs(oracle.DTYPES[k.dtype.name], k.ctypes.data, p.ctypes.data, k.size)
        return k, p
    return sort_pairs


def _pins_pass(sort_pairs):
    for ordered in (I32_ORDER, U64_ORDER, F32_TOTAL_ORDER[:8].view(np.float32),
                    F32_TOTAL_ORDER[4:].view(np.float32)):
        for perm in itertools.islice(itertools.permutations(range(8)), 0, 40320, 97):
            a = ordered[list(perm)]
            k, _ = sort_pairs(a, np.arange(8, dtype=np.uint32))
            if not np.array_equal(bits(k), bits(ordered)):
                return False
    for seq in itertools.product(range(3), repeat=6):
        k = np.array(seq, dtype=np.int32)
        _, p = sort_pairs(k, np.arange(6, dtype=np.uint32))
        if list(p) != sorted(range(6), key=lambda i: (seq[i], i)):
            return False
    return True


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_pins_catch_planted_mistakes(tmp_path):
    ok = _pins_pass(lambda k, p: oracle.sort_pairs(k, p))
    assert ok, "the real oracle must pass its own pins"
    for name in MUTATIONS:
        assert not _pins_pass(_mutant_sorts(tmp_path, name)), f"mutation {name} not caught"


# ------------------------------- P8 heavy list items (Sec. 2, lists of ints)

def _lists_pins_pass(sort_lists):
    """Rows of an (n, L) int32 array in word-by-word order: checked against
    numpy's lexsort (last key primary, so the columns go in reversed) and,
    for tiny cases, against Python's tuple order over every permutation."""
    rng = np.random.default_rng(8)
    for L in (1, 2, 3, 5, 16):
        for n in (0, 1, 7, 300):
            a = rng.integers(-2, 2, size=(n, L)).astype(np.int32)
            a[::5, 0] = np.iinfo(np.int32).min
            a[1::7, -1] = np.iinfo(np.int32).max
            want = a[np.lexsort(a.T[::-1])] if n else a
            if not np.array_equal(sort_lists(a), want):
                return False
    rows = [(0, 1, -1), (0, 1, 2), (-5, 9, 9), (0, 0, 7), (0, 1, -1), (3, -8, 0)]
    for perm in itertools.permutations(range(len(rows))):
        a = np.array([rows[i] for i in perm], dtype=np.int32)
        if [tuple(r) for r in sort_lists(a)] != sorted(rows):
            return False
    return True


LIST_MUTATIONS = {
    "first_word_only": ("        if (x != y)\n            return x < y;\n    }\n    return 0;",
                        "        if (x != y)\n            return x < y;\n        break;\n    }\n    return 0;"),
    "words_unsigned": ("        int32_t x, y;\n        memcpy(&x, a + 4 * w, 4);",
                       "        uint32_t x, y;\n        memcpy(&x, a + 4 * w, 4);"),
    "last_word_first": ("        memcpy(&x, a + 4 * w, 4);\n        memcpy(&y, b + 4 * w, 4);",
                        "        memcpy(&x, a + 4 * (g_list_words - 1 - w), 4);\n"
                        "        memcpy(&y, b + 4 * (g_list_words - 1 - w), 4);"),
}


def _mutant_lists(tmp_path, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "sortrace_oracle.c")).read()
    old, new = LIST_MUTATIONS[name]
    assert old in src, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    lib.oracle_sort_lists.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_size_t]

    def sort_lists(a):
        a = np.ascontiguousarray(a, dtype=np.int32).copy()
        lib.oracle_sort_lists(a.ctypes.data, a.shape[0], a.shape[1])
        return a
    return sort_lists


def test_list_sort_pins():
    assert _lists_pins_pass(oracle.sort_lists)
    a = np.arange(-50, 50, dtype=np.int32)[::-1].reshape(-1, 1)
    assert np.array_equal(oracle.sort_lists(a)[:, 0], np.sort(a[:, 0]))  # L = 1: plain int32 order


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_list_pins_catch_planted_mistakes(tmp_path):
    for name in LIST_MUTATIONS:
        assert not _lists_pins_pass(_mutant_lists(tmp_path, name)), f"mutation {name} not caught"


# ------------- P6 ascents and Inv on tied keys; segmented payloads (Sec. 2)

def _bubble_swaps(seq):
    """Adjacent exchanges a bubble sort makes, swapping only strictly greater
    left neighbours.  Each such exchange removes exactly one inversion and
    the sort ends with none, so the count equals Inv (an algorithm of its
    own, not the pair-counting definition)."""
    a = list(seq)
    swaps = 0
    for end in range(len(a) - 1, 0, -1):
        for i in range(end):
            if a[i] > a[i + 1]:
                a[i], a[i + 1] = a[i + 1], a[i]
                swaps += 1
    return swaps


def _measure_pins_pass(run, ascents, inv):
    """Closed forms of Sec. 2 plus the identity descents + ascents + equal
    neighbours = n - 1, on inputs with ties."""
    for n in (0, 1, 2, 9, 300):
        up = np.arange(n, dtype=np.int32)
        if ascents(up) != max(n - 1, 0) or ascents(up[::-1].copy()) != 0:
            return False
        eq = np.full(n, 7, dtype=np.int32)
        if ascents(eq) != 0 or inv(eq) != 0 or run(eq) != (1 if n else 0):
            return False
    # k copies of 1..q: no inversion inside a copy, q(q-1)/2 between any two
    # copies (equal values are no inversion)
    for k, q in ((1, 5), (2, 1), (2, 6), (3, 4), (5, 7)):
        a = np.tile(np.arange(1, q + 1, dtype=np.int32), k)
        if inv(a) != k * (k - 1) // 2 * q * (q - 1) // 2:
            return False
        if ascents(a) != k * (q - 1):
            return False
    # Sec. 3 worked example: 16 distinct keys, Run = 12, so 15 - 11 = 4 ascents
    g = _golden("worked_example.txt")
    ex = np.array([int(x) for x in g["input"]], dtype=np.int32)
    if ascents(ex) != int(g["ascents"][0]) or inv(ex) != _bubble_swaps(ex.tolist()):
        return False
    for dt, vals in (("int32", I32_ORDER[:3]), ("uint64", U64_ORDER[5:8]),
                     ("float32", F32_TOTAL_ORDER[4:7].view(np.float32))):
        for n in range(0, 8):
            for seq in itertools.product(range(3), repeat=n):
                a = vals[list(seq)] if n else vals[:0]
                eqn = sum(1 for i in range(n - 1) if seq[i] == seq[i + 1])
                d = (run(a) - 1) if n else 0
                if d + ascents(a) + eqn != max(n - 1, 0):
                    return False
                if inv(a) != _bubble_swaps(seq):
                    return False
    return True


def test_measures_on_tied_keys():
    assert _measure_pins_pass(oracle.run, oracle.ascents, oracle.inv)


def _segmented_pairs_pass(sort_segmented):
    """Per segment, the payload order is Python's sorted() by (key, index)."""
    rng = np.random.default_rng(44)
    for trial in range(6):
        lens = rng.integers(0, 40, 9)
        lens[trial % 9] = 0
        off = np.zeros(lens.size + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        n = int(off[-1])
        keys = rng.integers(0, 4, n).astype(np.int32)
        pay = np.arange(n, dtype=np.uint32)[::-1].copy()
        ok, op = sort_segmented(keys, off, pay)
        for s in range(lens.size):
            a, b = int(off[s]), int(off[s + 1])
            order = sorted(range(a, b), key=lambda i: (int(keys[i]), i))
            if list(op[a:b]) != [int(pay[i]) for i in order]:
                return False
            if list(ok[a:b]) != [int(keys[i]) for i in order]:
                return False
    return True


def test_segmented_pairs_match_python_definition():
    assert _segmented_pairs_pass(oracle.sort_segmented)


MEASURE_MUTATIONS = {
    "ascents_count_ties": ("        if (less(a + i * ks, a + (i + 1) * ks))\n            u++;",
                           "        if (!less(a + (i + 1) * ks, a + i * ks))\n            u++;"),
    "inv_counts_ties": ("            if (less(a + j * ks, a + i * ks))\n                c++;",
                        "            if (!less(a + i * ks, a + j * ks))\n                c++;"),
    "inv_neighbours_only": ("        for (size_t j = i + 1; j < n; j++)\n            if (less(a + j * ks, a + i * ks))",
                            "        for (size_t j = i + 1; j < n && j < i + 2; j++)\n"
                            "            if (less(a + j * ks, a + i * ks))"),
}
SEGMENT_MUTATIONS = {
    "segment_payload_not_offset": ("sort_records(dtype, k, payload + a,", "sort_records(dtype, k, payload,"),
    "segment_payload_off_by_one": ("sort_records(dtype, k, payload + a,", "sort_records(dtype, k, payload + a + 1,"),
}


def _mutant_lib(tmp_path, name, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "sortrace_oracle.c")).read()
    assert old in src, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", str(path), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    for fn in ("oracle_run", "oracle_ascents", "oracle_inv"):
        getattr(lib, fn).argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
        getattr(lib, fn).restype = ctypes.c_int64
    lib.oracle_sort_segmented.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_size_t]
    return lib


def _measure(lib, fn):
    def f(a):
        a = np.ascontiguousarray(a)
        return int(getattr(lib, fn)(oracle.DTYPES[a.dtype.name], a.ctypes.data, a.size))
    return f


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_measure_pins_catch_planted_mistakes(tmp_path):
    for name, (old, new) in MEASURE_MUTATIONS.items():
        lib = _mutant_lib(tmp_path, name, old, new)
        ok = _measure_pins_pass(_measure(lib, "oracle_run"), _measure(lib, "oracle_ascents"),
                                _measure(lib, "oracle_inv"))
        assert not ok, f"mutation {name} not caught"


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc needed")
def test_segmented_pins_catch_planted_mistakes(tmp_path):
    for name, (old, new) in SEGMENT_MUTATIONS.items():
        lib = _mutant_lib(tmp_path, name, old, new)

        def sort_segmented(keys, off, pay, lib=lib):
            k, p = keys.copy(), pay.copy()
            # the payload-off-by-one mutant reads one past the array: give it room
            buf = np.zeros(p.size + 1, dtype=np.uint32)
            buf[:p.size] = p
            lib.oracle_sort_segmented(0, k.ctypes.data, buf.ctypes.data, off.ctypes.data, off.size - 1)
            return k, buf[:p.size]
        assert not _segmented_pairs_pass(sort_segmented), f"mutation {name} not caught"


# ----------------- the multi-threaded variant used to time a CPU baseline

@pytest.mark.parametrize("dtype", ["int32", "uint64", "float32"])
def test_parallel_variant_equals_the_oracle(dtype):
    for n in (0, 1, 2, 3, 7, 100, 1001, 65537):
        for threads in (1, 2, 3, 8, 16):
            if dtype == "int32":
                a = inputs.random_int32(n, n + threads)
                a[::3] = 5
            elif dtype == "uint64":
                a = inputs.stream(n, n)
            else:
                a = inputs.normal_float32(n, seed=n + 1)
            got = oracle.sort_keys_parallel(a, threads)
            assert np.array_equal(bits(got), bits(oracle.sort_keys(a))), (n, threads)
