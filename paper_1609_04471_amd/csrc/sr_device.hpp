// sr_device.hpp -- device primitives of libsortrace (gfx950, wave64).
//
//  * key codec: an order-preserving bijection from each dtype's bit pattern
//    to an unsigned integer, so every comparison below is an unsigned
//    integer comparison (the fixed ordering of Sec. 1; float32 follows IEEE
//    754-2008 totalOrder on the bits);
//  * cross-lane exchange of a register with lane ^ M (DPP / ds_swizzle /
//    ds_bpermute, picked at compile time per mask);
//  * compare-exchange networks: Batcher's merge exchange (Knuth, TAOCP 3,
//    Sec. 5.2.2, Algorithm M) inside a thread, Batcher's bitonic merge across
//    the 64 lanes of a wavefront;
//  * Merge Path co-rank searches (Odeh, Green, Mwassi, Shmueli, Birk 2012):
//    a binary search inside LDS and a 64-ary wavefront search in global
//    memory.
// Every merge takes the left run on ties, which keeps merges stable (the
// Appendix A merge contract plus the stability of Sec. 6).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sr {

constexpr int kWave = 64;

// ------------------------------------------------------------------ codec
// S = storage type (what the user's buffer holds), U = order key.
struct CodecI32 {
    using S = uint32_t;
    using U = uint32_t;
    static __device__ __forceinline__ U enc(S x) { return x ^ 0x80000000u; }
    static __device__ __forceinline__ S dec(U u) { return u ^ 0x80000000u; }
};

struct CodecF32 {
    using S = uint32_t;
    using U = uint32_t;
    // sign clear: set the top bit; sign set: invert every bit.
    static __device__ __forceinline__ U enc(S b) {
        return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
    }
    static __device__ __forceinline__ S dec(U u) {
        return u ^ ((uint32_t)((int32_t)~u >> 31) | 0x80000000u);
    }
};

struct CodecU64 {
    using S = uint64_t;
    using U = uint64_t;
    static __device__ __forceinline__ U enc(S x) { return x; }
    static __device__ __forceinline__ S dec(U u) { return u; }
};

template <class U>
__device__ __forceinline__ U key_max() { return (U)~(U)0; }

// --------------------------------------------------- device control block
// One per workspace.  The probe's last workgroup writes the plan and clears
// the per-call counters, so every call finds them cleared.
struct Ctl {
    unsigned long long unused0[4];
    unsigned int mixed;               // some probe workgroup saw both an ascent and a descent
    unsigned int ticket;              // probe workgroups that finished
    int path;                         // sr_path chosen by the plan
    int force_path;                   // -1 or a forced sr_path
    unsigned long long m;             // OUTLIER: number of outliers
    unsigned long long n_kept;        // OUTLIER: number of kept keys (written by the last tile)
    unsigned int bad_join;            // OUTLIER: kept keys not sorted somewhere: fall back
    unsigned int ticket2;             // OUTLIER: tile ids handed out by classify
    unsigned int ticket3;             // OUTLIER: classify workgroups finished
    unsigned int epoch;               // call counter stamped into the look-back status words
    int job_passes;                   // OUTLIER: merge passes of the outlier sort
    int dual;                         // OUTLIER beside a run plan (the sample's turning points are rare)
    unsigned long long reserved[4];   // [0] descents, [1] ascents (for sr_last_stats)
    unsigned long long run[4];        // RUNS: merge leaves, merge passes, keys reversed, keys in dense pieces
    int few_wide;                     // FEW: the job uses the wide tables (more than 64 splitters)
    int pad_w;
};

// Plain relaxed agent-scope accessors (coherent across the XCDs' L2s), for
// words that other workgroups of the same launch write.  Plan fields written
// by an earlier launch on the stream are read with plain loads: the launch
// boundary orders them.
__device__ __forceinline__ unsigned int ld_agent(const unsigned int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_agent(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_agent(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Resets of words that a later launch updates with atomics are agent-scope
// atomic stores too: a plain store may sit dirty in one XCD's L2 and be
// written back after the later launch's atomics, undoing their counts.
__device__ __forceinline__ void st_agent(unsigned int* p, unsigned int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------ cross-lane exchange
// Value held by lane (lane ^ M) of the same wavefront.  DPP covers the masks
// that stay inside a row of 16 lanes (every lane has its source inside the
// row, so no "old" value is needed), ds_swizzle's bit mode the masks below
// 32, ds_bpermute the rest.  All lanes must be active.
template <int M>
__device__ __forceinline__ uint32_t xlane(uint32_t v) {
    const int x = (int)v;
    if constexpr (M == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
    } else if constexpr (M == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true);  // quad_perm 2,3,0,1
    } else if constexpr (M == 3) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x1B, 0xF, 0xF, true);  // quad_perm 3,2,1,0
    } else if constexpr (M == 7) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, true); // row_half_mirror
    } else if constexpr (M == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, true); // row_ror:8
    } else if constexpr (M == 15) {
        return (uint32_t)__builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true); // row_mirror
    } else if constexpr (M < 32) {
        // bit mode: and_mask = 0x1F, or_mask = 0, xor_mask = M
        return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x1F | (M << 10));
    } else {
        const int src = (int)(__lane_id() ^ (unsigned)M);
        return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, x);
    }
}

template <int M>
__device__ __forceinline__ uint64_t xlane(uint64_t v) {
    const uint32_t lo = xlane<M>((uint32_t)v);
    const uint32_t hi = xlane<M>((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Network element for stable (key, payload) tile sorts: the key plus the
// element's position inside the tile.  Ordering (key, position) makes every
// element distinct, so any sorting network yields the stable order.
template <class U>
struct KeyPos {
    U k;
    uint32_t p;
};

template <class U>
__device__ __forceinline__ bool lt(U a, U b) { return a < b; }
template <class U>
__device__ __forceinline__ bool lt(const KeyPos<U>& a, const KeyPos<U>& b) {
    return a.k < b.k || (a.k == b.k && a.p < b.p);
}

template <class U>
__device__ __forceinline__ U emin(U a, U b) { return a < b ? a : b; }
template <class U>
__device__ __forceinline__ U emax(U a, U b) { return a < b ? b : a; }
template <class U>
__device__ __forceinline__ KeyPos<U> emin(const KeyPos<U>& a, const KeyPos<U>& b) { return lt(b, a) ? b : a; }
template <class U>
__device__ __forceinline__ KeyPos<U> emax(const KeyPos<U>& a, const KeyPos<U>& b) { return lt(b, a) ? a : b; }

template <int M, class U>
__device__ __forceinline__ KeyPos<U> xlane(const KeyPos<U>& v) {
    return KeyPos<U>{xlane<M>(v.k), xlane<M>(v.p)};
}

// One side of a cross-lane compare-exchange: the lane holding x keeps the
// larger of (x, partner) when `upper`, else the smaller.  For 32-bit keys
// that is the median of (x, p, 0) or (x, p, ~0): one v_med3_u32 instead of a
// min, a max and a select.
template <class E>
__device__ __forceinline__ E keep_side(const E& x, const E& p, bool upper) {
    return upper ? emax(x, p) : emin(x, p);
}
__device__ __forceinline__ uint32_t keep_side(uint32_t x, uint32_t p, bool upper) {
    const uint32_t bound = upper ? 0xFFFFFFFFu : 0u;
    const uint32_t lo = x < p ? x : p;
    const uint32_t hi = x < p ? p : x;
    const uint32_t t = hi < bound ? hi : bound;
    return lo < t ? t : lo;
}

template <class E>
__device__ __forceinline__ void cmpx(E& a, E& b) {
    const E lo = emin(a, b);
    const E hi = emax(a, b);
    a = lo;
    b = hi;
}

// ----------------------------------------------- in-register sorting network
// Batcher's merge exchange for N inputs, generated at compile time in the
// order of Knuth's Algorithm M (passes p = 2^(t-1) .. 1; inner d, q, r).
template <int N>
struct MergeExchange {
    int a[N * N];
    int b[N * N];
    int count;
    constexpr MergeExchange() : a(), b(), count(0) {
        int t = 0;
        while ((1 << t) < N) ++t;
        if (t == 0) return;
        for (int p = 1 << (t - 1); p > 0; p >>= 1) {
            int q = 1 << (t - 1), r = 0, d = p;
            for (;;) {
                for (int i = 0; i + d < N; ++i) {
                    if ((i & p) == r) {
                        a[count] = i;
                        b[count] = i + d;
                        ++count;
                    }
                }
                if (q == p) break;
                d = q - p;
                q >>= 1;
                r = p;
            }
        }
    }
};

template <int N>
inline constexpr MergeExchange<N> kMergeExchange{};

template <int N, class E>
__device__ __forceinline__ void sort_in_registers(E (&v)[N]) {
    constexpr MergeExchange<N> net = kMergeExchange<N>;
#pragma unroll
    for (int c = 0; c < net.count; ++c) cmpx(v[net.a[c]], v[net.b[c]]);
}

// ----------------------------------------------- wavefront bitonic merging
// Conceptual index of v[r] in lane L is L * N + r.  Each lane starts with N
// sorted values; after wave_sort the wavefront's 64 * N values are sorted.
// Merging two sorted runs of G/2 lanes each: first the "flip" stage pairs
// index i with the mirrored index of the 2-run block (lane ^ (G-1), register
// N-1-r), then half-cleaners at lane distances G/4 .. 1, then at register
// distances N/2 .. 1 (Batcher's bitonic merge).
template <int DL, int N, class E>
__device__ __forceinline__ void half_cleaner_lanes(E (&v)[N], unsigned lane) {
    const bool upper = (lane & DL) != 0;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        const E p = xlane<DL>(v[r]);
        v[r] = keep_side(v[r], p, upper);
    }
    if constexpr (DL > 1) half_cleaner_lanes<DL / 2>(v, lane);
}

template <int N, class E>
__device__ __forceinline__ void half_cleaners_in_registers(E (&v)[N]) {
#pragma unroll
    for (int d = N / 2; d >= 1; d /= 2) {
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if ((r & d) == 0) cmpx(v[r], v[r + d]);
        }
    }
}

template <int G, int N, class E>
__device__ __forceinline__ void wave_merge_level(E (&v)[N], unsigned lane) {
    const bool upper = (lane & (G / 2)) != 0;
    E p[N];
#pragma unroll
    for (int r = 0; r < N; ++r) p[r] = xlane<G - 1>(v[N - 1 - r]);
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = keep_side(v[r], p[r], upper);
    if constexpr (G >= 4) half_cleaner_lanes<G / 4>(v, lane);
    half_cleaners_in_registers(v);
    if constexpr (G < kWave) wave_merge_level<G * 2>(v, lane);
}

template <int N, class E>
__device__ __forceinline__ void wave_sort(E (&v)[N]) {
    sort_in_registers(v);
    wave_merge_level<2>(v, __lane_id());
}

// ------------------------------------------------------- Merge Path search
// co-rank of diagonal d between sorted A[0, la) and B[0, lb): the number i of
// A elements among the first d outputs of the stable merge.  A[i] precedes
// B[d-1-i] when A[i] <= B[d-1-i].  By a single thread in global memory
// (plain binary search).
template <class C>
__device__ __forceinline__ int64_t corank_thread(const typename C::S* A, int64_t la,
                                                 const typename C::S* B, int64_t lb, int64_t d) {
    int64_t lo = d > lb ? d - lb : 0;
    int64_t hi = d < la ? d : la;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (C::enc(A[mid]) <= C::enc(B[d - 1 - mid]))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// corank_thread with a first guess, for the partition launch: when A and B
// are alike (the general plan's runs of random keys), the co-rank of d lies
// within a few sqrt(d) of d * la / (la + lb).  A window of +-(4 sqrt(d) + 64)
// around that guess is checked with two probes issued together (it holds the
// co-rank iff A[lo'-1] <= B[d-lo'] and A[hi'] > B[d-1-hi'], or it touches the
// range's ends) and then searched; when the check fails the whole range is.
// Ranges of at most 4096 are searched directly.
template <class C>
__device__ __forceinline__ int64_t corank_guess(const typename C::S* A, int64_t la, const typename C::S* B,
                                                int64_t lb, int64_t d) {
    int64_t lo = d > lb ? d - lb : 0;
    int64_t hi = d < la ? d : la;
    if (hi - lo > 4096) {
        const int64_t g = (int64_t)((double)d * (double)la / (double)(la + lb));
        const int64_t w = 4 * (int64_t)sqrt((double)d) + 64;
        const int64_t glo = g - w > lo ? g - w : lo;
        const int64_t ghi = g + w < hi ? g + w : hi;
        // the two probes' keys, loaded before either is compared; a range
        // this wide has la, lb >= 1, so index 0 stands in for an unused probe
        const typename C::U a0 = C::enc(A[glo > lo ? glo - 1 : 0]), b0 = C::enc(B[glo > lo ? d - glo : 0]);
        const typename C::U a1 = C::enc(A[ghi < hi ? ghi : 0]), b1 = C::enc(B[ghi < hi ? d - 1 - ghi : 0]);
        const bool ok_lo = glo == lo || a0 <= b0;
        const bool ok_hi = ghi == hi || !(a1 <= b1);
        if (glo <= ghi && ok_lo && ok_hi) {
            lo = glo;
            hi = ghi;
        }
    }
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (C::enc(A[mid]) <= C::enc(B[d - 1 - mid]))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Same search in global memory by one whole wavefront: each round the 64
// lanes test 64 evenly spaced candidates, so the range shrinks 64-fold per
// round.  Keys are decoded with codec C on load.  Returns the co-rank in all
// lanes.
template <class C>
__device__ __forceinline__ int64_t corank_wave(const typename C::S* A, int64_t la,
                                               const typename C::S* B, int64_t lb, int64_t d) {
    const unsigned lane = __lane_id();
    int64_t lo = d > lb ? d - lb : 0;
    int64_t hi = d < la ? d : la;
    while (lo < hi) {
        const int64_t len = hi - lo;
        const int64_t step = (len + kWave - 1) / kWave;
        const int64_t x = lo + (int64_t)lane * step;
        bool pred = false;
        if (x < hi) pred = C::enc(A[x]) <= C::enc(B[d - 1 - x]);
        const unsigned long long bal = __builtin_amdgcn_ballot_w64(pred);
        const int cnt = __builtin_popcountll(bal);  // predicate is monotone: the first cnt probes hold
        if (cnt == 0) {
            hi = lo;
        } else {
            const int64_t last_true = lo + (int64_t)(cnt - 1) * step;
            const int64_t first_false = lo + (int64_t)cnt * step;
            lo = last_true + 1;
            hi = first_false < hi ? first_false : hi;
        }
    }
    return lo;
}

}  // namespace sr
