"""Seeded synthetic inputs for libsortrace (numpy, host side).

This module holds the input generators only -- no sorting arithmetic -- so
that the GPU path and the CPU oracle receive identical bytes.  Everything is
derived from splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used as a counter-based generator:
element i of stream ``seed`` is ``mix(seed + (i + 1) * 0x9E3779B97F4A7C15)``.
Integer ranges use a multiply-high reduction of the top 32 bits; normals use
Box-Muller in double precision rounded to float32.

Workloads (the four input types of Table 1 of the Sort Race paper, Sec. 1,
plus the batched / key-value / serving mixes):
  random        uniform over the full int32 range
  reversed      strictly descending n-1 .. 0 (k = 1 teeth, Sec. 2)
  nearly        0 .. n-1, then floor(n/100) exchanges of two positions, all
                2*floor(n/100) positions distinct (a k-exchange list, Sec. 2)
  few           every key one of 10 distinct random int32 values
  runs_u64      uint64 keys in concatenated runs of geometric length (mean
                1000), each ascending or descending, with 10% zero steps so
                equal keys occur inside runs; payload = original index
  segments      CSR batch of arrays with log-uniform lengths, each of a random
                one of the four types above
  normal_f32    standard normal float32 with 1% repeated values, signed zeros
                and NaNs of both signs (IEEE totalOrder matters)
  k-classes     the presorted classes of Sec. 2: k-equal, k-even, k-sharp and
                k-shuffled teeth, k-distance, k-exchange, k-limited
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22

TYPES = ("random", "reversed", "nearly", "few")


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64(x: int) -> int:
    """splitmix64 finaliser of one integer (used to derive seeds)."""
    with np.errstate(over="ignore"):
        return int(_mix(np.array([x & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0])


def seed_for(config: int, type_id: int, ident: int) -> int:
    """Seed per (config, input type, segment/request id)."""
    return mix64(0x1609044710 ^ (config << 56) ^ (type_id << 48) ^ ident)


def stream(seed: int, n: int, start: int = 0) -> np.ndarray:
    """n uint64 draws of splitmix64 stream ``seed`` beginning at counter ``start``."""
    out = np.empty(n, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for lo in range(0, n, _CHUNK):
            hi = min(n, lo + _CHUNK)
            idx = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            out[lo:hi] = _mix(s + idx * GOLDEN)
    return out


def below(x: np.ndarray, m: int) -> np.ndarray:
    """Multiply-high reduction of uint64 draws to [0, m), m <= 2^32."""
    assert 0 < m <= (1 << 32)
    return ((x >> np.uint64(32)) * np.uint64(m)) >> np.uint64(32)


def unit_double(x: np.ndarray) -> np.ndarray:
    """Top 53 bits as a double in [0, 1)."""
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def _distinct_positions(seed: int, count: int, n: int) -> np.ndarray:
    """``count`` distinct positions in [0, n), in first-draw order."""
    if count == 0:
        return np.empty(0, dtype=np.int64)
    assert count <= n
    got = np.empty(0, dtype=np.int64)
    start = 0
    draw = count + count // 16 + 64
    while True:
        cand = below(stream(seed, draw, start), n).astype(np.int64)
        start += draw
        allc = np.concatenate([got, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        got = allc[first]
        if got.size >= count:
            return got[:count]
        draw = 2 * (count - got.size) + 64


# --------------------------------------------------------------- int32 types

def random_int32(n: int, seed: int) -> np.ndarray:
    return (stream(seed, n) >> np.uint64(32)).astype(np.uint32).view(np.int32)


def reversed_int32(n: int) -> np.ndarray:
    return np.arange(n - 1, -1, -1, dtype=np.int64).astype(np.int32)


def nearly_sorted_int32(n: int, seed: int) -> np.ndarray:
    a = np.arange(n, dtype=np.int64).astype(np.int32)
    m = n // 100
    pos = _distinct_positions(seed, 2 * m, n)
    p, q = pos[0::2], pos[1::2]
    a[p], a[q] = a[q].copy(), a[p].copy()
    return a


def few_unique_int32(n: int, seed: int, distinct: int = 10) -> np.ndarray:
    vals = []
    start = 0
    while len(vals) < distinct:
        x = int(stream(seed ^ 0x5EED, 1, start)[0] >> np.uint64(32))
        start += 1
        v = x - (1 << 32) if x >= (1 << 31) else x
        if v not in vals:
            vals.append(v)
    v = np.array(vals, dtype=np.int32)
    return v[below(stream(seed, n), distinct).astype(np.int64)]


def int32_of_type(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "random":
        return random_int32(n, seed)
    if kind == "reversed":
        return reversed_int32(n)
    if kind == "nearly":
        return nearly_sorted_int32(n, seed)
    if kind == "few":
        return few_unique_int32(n, seed)
    raise ValueError(kind)


# ------------------------------------------- the k-classes of Sec. 2 (int32)
# Built from their definitions on 1..n without the "blow-up" maps, which are
# strictly increasing and so change no comparison between two keys.  Section
# i of k holds floor((i+1)n/k) - floor(i n/k) positions (equal sections when
# k divides n).  "Odd numbered" sections are the first, third, ... (index
# 0, 2, ... here).

CLASSES = ("equal_teeth", "even_teeth", "sharp_teeth", "shuffled_teeth", "distance", "exchange", "limited")


def _sections(n: int, k: int) -> np.ndarray:
    return (np.arange(k + 1, dtype=np.int64) * n) // k


def equal_teeth(n: int, k: int) -> np.ndarray:
    """k sections, each ascending 1 .. its length."""
    b = _sections(n, k)
    pos = np.arange(n, dtype=np.int64)
    sec = np.searchsorted(b, pos, side="right") - 1
    return (pos - b[sec] + 1).astype(np.int32)


def even_teeth(n: int, k: int) -> np.ndarray:
    """k-equal teeth with every odd-numbered section reversed (k = 2: organ pipe
    from the descending side; k = 1: reversed)."""
    b = _sections(n, k)
    pos = np.arange(n, dtype=np.int64)
    sec = np.searchsorted(b, pos, side="right") - 1
    up = pos - b[sec] + 1
    down = b[sec + 1] - pos
    return np.where(sec % 2 == 0, down, up).astype(np.int32)


def sharp_teeth(n: int, k: int) -> np.ndarray:
    """1..n in k sections, odd-numbered sections reversed (k = 1: reversed)."""
    b = _sections(n, k)
    pos = np.arange(n, dtype=np.int64)
    sec = np.searchsorted(b, pos, side="right") - 1
    mirrored = b[sec] + b[sec + 1] - 1 - pos
    return (np.where(sec % 2 == 0, mirrored, pos) + 1).astype(np.int32)


def shuffled_teeth(n: int, k: int, seed: int) -> np.ndarray:
    """The k sections of a k-sharp teeth list interleaved at random, each
    section keeping its own order: the section labels, one per key, are put in
    a uniformly random order (sorted by seeded 64-bit random keys, ties by
    position), and the keys of section s fill the positions labelled s in
    turn."""
    a = sharp_teeth(n, k)
    b = _sections(n, k)
    labels = np.repeat(np.arange(k, dtype=np.int64), np.diff(b))
    labels = labels[np.argsort(stream(seed, n), kind="stable")]
    out = np.empty(n, dtype=np.int32)
    # positions grouped by label, in increasing position order within a label
    out[np.argsort(labels, kind="stable")] = a
    return out


def distance(n: int, k: int, seed: int) -> np.ndarray:
    """1..n cut into sections of k+1 keys (the last may be shorter), each
    shuffled (Fisher-Yates, all sections at once); every key ends within k of
    its rank."""
    a = np.arange(1, n + 1, dtype=np.int64)
    w = k + 1
    full = (n // w) * w
    blk = a[:full].reshape(-1, w) if full else a[:0].reshape(0, w)
    r = stream(seed, max(1, w * max(1, blk.shape[0])))
    for j in range(w - 1, 0, -1):
        if blk.shape[0] == 0:
            break
        pick = below(r[j * blk.shape[0]:(j + 1) * blk.shape[0]], j + 1).astype(np.int64)
        rows = np.arange(blk.shape[0])
        t = blk[rows, j].copy()
        blk[rows, j] = blk[rows, pick]
        blk[rows, pick] = t
    tail = a[full:]
    rt = stream(seed ^ 0x7A11, max(1, tail.size))
    for j in range(tail.size - 1, 0, -1):
        q = int(below(rt[j:j + 1], j + 1)[0])
        tail[j], tail[q] = tail[q], tail[j]
    return np.concatenate([blk.reshape(-1), tail]).astype(np.int32)


def exchange(n: int, k: int, seed: int) -> np.ndarray:
    """1..n, then k exchanges of two uniformly drawn positions."""
    a = np.arange(1, n + 1, dtype=np.int64)
    if n > 0:
        pq = below(stream(seed, 2 * k), n).astype(np.int64)
        for p, q in zip(pq[0::2], pq[1::2]):
            a[p], a[q] = a[q], a[p]
    return a.astype(np.int32)


def limited(n: int, k: int, seed: int) -> np.ndarray:
    """At most 2^k distinct values: uniform k-bit integers; k = 0 gives all
    zeros, k >= 32 the full int32 range (random integers, as Sec. 2 notes)."""
    if k == 0:
        return np.zeros(n, dtype=np.int32)
    if k >= 32:
        return random_int32(n, seed)
    return below(stream(seed, n), 1 << k).astype(np.int64).astype(np.int32)


def class_int32(name: str, n: int, k: int, seed: int) -> np.ndarray:
    if name == "equal_teeth":
        return equal_teeth(n, k)
    if name == "even_teeth":
        return even_teeth(n, k)
    if name == "sharp_teeth":
        return sharp_teeth(n, k)
    if name == "shuffled_teeth":
        return shuffled_teeth(n, k, seed)
    if name == "distance":
        return distance(n, k, seed)
    if name == "exchange":
        return exchange(n, k, seed)
    if name == "limited":
        return limited(n, k, seed)
    raise ValueError(name)


# ------------------------------------------------------------ uint64 runs

def runs_uint64(n: int, seed: int, mean_len: int = 1000, tie_stress: bool = False):
    """Concatenated monotone runs; returns (keys uint64, payload uint32 = index).

    Run lengths are Geometric(1/mean_len) on {1, 2, ...}, truncated at n; each
    run ascends or descends with probability 1/2.  Each step inside a run is 0
    with probability 0.1 (an equal key) and otherwise uniform on [1, 2^20].
    Bases are uniform on [2^40, 2^64 - 2^40), so no run wraps around.  With
    ``tie_stress`` bases come from a pool of 64 values and steps from [0, 3],
    so equal keys also meet across runs.
    """
    keys = np.empty(n, dtype=np.uint64)
    if n == 0:
        return keys, np.empty(0, dtype=np.uint32)
    p = 1.0 / mean_len
    nruns_est = n // mean_len * 2 + 64
    lens = []
    total = 0
    start = 0
    while total < n:
        u = unit_double(stream(seed ^ 0x1111, nruns_est, start))
        start += nruns_est
        u = np.maximum(u, 1e-300)
        lg = 1 + np.floor(np.log(u) / np.log1p(-p)).astype(np.int64)
        lens.append(lg)
        total += int(lg.sum())
    lens = np.concatenate(lens)
    cum = np.cumsum(lens)
    nr = int(np.searchsorted(cum, n) + 1)
    lens = lens[:nr].copy()
    lens[-1] -= int(cum[nr - 1]) - n
    assert int(lens.sum()) == n
    rs = stream(seed ^ 0x2222, nr)
    desc = (rs >> np.uint64(63)).astype(bool)
    if tie_stress:
        pool = stream(seed ^ 0x3333, 64) | np.uint64(1 << 63)
        base = pool[below(rs, 64).astype(np.int64)]
        steps = below(stream(seed ^ 0x4444, n), 4)
    else:
        lo = np.uint64(1 << 40)
        span = (1 << 64) - (1 << 41)
        # base = lo + floor(u * span) with u from the top 53 bits
        base = lo + ((rs >> np.uint64(11)) * np.uint64(span >> 53))
        sx = stream(seed ^ 0x4444, n)
        zero = below(sx, 10) == 0
        steps = (below(sx ^ np.uint64(0xA5A5A5A5A5A5A5A5), 1 << 20) + np.uint64(1))
        steps[zero] = 0
    run_id = np.repeat(np.arange(nr), lens)
    first = np.concatenate([[0], np.cumsum(lens)[:-1]])
    steps = steps.astype(np.uint64)
    steps[first] = 0
    with np.errstate(over="ignore"):
        cs = np.cumsum(steps, dtype=np.uint64)
        run_start_cs = cs[first]
        within = cs - run_start_cs[run_id]
        b = base[run_id]
        d = desc[run_id]
        keys[~d] = b[~d] + within[~d]
        keys[d] = b[d] - within[d]
    return keys, np.arange(n, dtype=np.uint32)


# --------------------------------------------------------------- segments

def segment_lengths(nseg: int, seed: int, lo: int = 16, hi: int = 262144) -> np.ndarray:
    """Log-uniform lengths: clamp(floor(exp(U(ln lo, ln hi))), lo, hi)."""
    u = unit_double(stream(seed, nseg))
    L = np.floor(np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))).astype(np.int64)
    return np.clip(L, lo, hi)


def segments_int32(nseg: int, seed: int, lo: int = 16, hi: int = 262144):
    """CSR batch: returns (keys int32, offsets int64 [nseg+1], kinds list)."""
    L = segment_lengths(nseg, seed, lo, hi)
    kinds_idx = below(stream(seed ^ 0x7777, nseg), 4).astype(np.int64)
    offsets = np.zeros(nseg + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(L)
    keys = np.empty(int(offsets[-1]), dtype=np.int32)
    kinds = []
    for s in range(nseg):
        kind = TYPES[int(kinds_idx[s])]
        kinds.append(kind)
        keys[offsets[s]:offsets[s + 1]] = int32_of_type(kind, int(L[s]), seed_for(4, int(kinds_idx[s]), s))
    return keys, offsets, kinds


# ----------------------------------------------------------- float32 mix

def random_lists(n: int, words: int, seed: int, lo: int | None = None, hi: int | None = None) -> np.ndarray:
    """(n, words) int32 lists (the heavy items of Sec. 2): uniform over all
    int32 values, or over [lo, hi) when given (small ranges make prefixes
    tie)."""
    u = stream(seed, n * words)
    if lo is None:
        return (u & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.int32).reshape(n, words)
    return (lo + (u % np.uint64(hi - lo)).astype(np.int64)).astype(np.int32).reshape(n, words)


def normal_float32(n: int, seed: int, specials: bool = True) -> np.ndarray:
    """N(0,1) float32; with ``specials``: 1% repeats, then 0.1% each of +0,
    -0, +qNaN, -qNaN and NaNs with random sign and payload."""
    u1 = unit_double(stream(seed, n))
    u2 = unit_double(stream(seed ^ 0x9999, n))
    u1 = 1.0 - u1  # (0, 1]
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    bits = z.astype(np.float32).view(np.uint32).copy()
    if specials and n > 0:
        r = stream(seed ^ 0xABCD, n)
        rep = below(r, 100) == 0
        src = below(stream(seed ^ 0xBCDE, n), n).astype(np.int64)
        bits[rep] = bits[src[rep]]
        sel = below(stream(seed ^ 0xCDEF, n), 1000).astype(np.int64)
        bits[sel == 0] = 0x00000000
        bits[sel == 1] = 0x80000000
        bits[sel == 2] = 0x7FC00000
        bits[sel == 3] = 0xFFC00000
        rnan = stream(seed ^ 0xDEF0, n)
        mant = (below(rnan, (1 << 23) - 1) + np.uint64(1)).astype(np.uint32)
        sign = ((rnan >> np.uint64(7)) & np.uint64(1)).astype(np.uint32) << np.uint32(31)
        m4 = sel == 4
        bits[m4] = sign[m4] | np.uint32(0x7F800000) | mant[m4]
    return bits.view(np.float32)


def uniform_int32(n: int, seed: int) -> np.ndarray:
    return random_int32(n, seed)
