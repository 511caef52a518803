// sr_kernels.hpp -- the sort-path kernels of libsortrace as device functions
// plus thin __global__ wrappers.  Included by the engine translation unit.
//
// Pass structure (general path): a tile sort sorts every tile of T keys
// inside one workgroup (the GPU form of the paper's base case, Sec. 3 (b):
// short runs are extended to a minimum length before merging), then
// level-synchronous merge passes pair up neighbouring sorted runs, all pairs
// of a level in one launch (Sec. 3 (e1): in each round all runs are paired
// and merged).  Each merge pass cuts its output into chunks by Merge Path, so
// the work per workgroup is equal whatever the data.
#pragma once

#include <type_traits>

#include "sr_device.hpp"

namespace sr {

// 16-byte vector of storage elements, for dwordx4 loads and stores.
template <class S>
struct alignas(16) V16 {
    S v[16 / sizeof(S)];
};

__device__ __forceinline__ bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// ------------------------------------------------------------- reductions
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
    return x;
}

// ==================================================================== tile
// Sorts one tile of `valid` (<= WG*IT) keys from src into dst (src may equal
// dst).  Keys-only: wavefront bitonic sort of 64*IT keys in registers, then
// Merge Path merges in LDS across the WG/64 wavefronts.  Pairs: the same on
// (key, tile position) elements, so the result is the stable order, and the
// payload is gathered by position at the end.
template <class C, int WG, int IT, bool PAIRS>
struct TileSort {
    using S = typename C::S;
    using U = typename C::U;
    static constexpr int T = WG * IT;
    static constexpr int VN = 16 / sizeof(S);
    static_assert(IT % VN == 0, "IT must hold whole 16-byte vectors");
    static_assert(WG % kWave == 0, "whole wavefronts");

    // LDS rows are padded by one word per 32 (pad): the per-thread runs of
    // IT consecutive elements (put) and the 16-byte output reads then hit
    // the banks at most twice per wavefront access instead of IT times.
    static constexpr int TP = T + T / 32;
    static __device__ __forceinline__ int pad(int e) { return e + (e >> 5); }

    // Keys only: a run of width w starts at logical slot G + q * (w + G) and
    // is followed by G slots holding the largest code (G more lead the first
    // run), so an exhausted run reads as the largest code and the serial
    // merge needs no bounds tests.  Ties go to the left run, so the left run
    // can be read up to IT - 1 slots past its end (only while every remaining
    // output is the largest code): G >= IT.  Logical slot l lives at pad(l),
    // like the pairs layout, so lanes whose heads lie IT/2 slots apart do not
    // meet in the same LDS banks.
    static constexpr int G = IT < 4 ? 4 : IT;
    static constexpr int TK = G + T + (T / (kWave * IT)) * G;
    static constexpr int TKP = TK + TK / 32 + 1;
    static constexpr int KW = PAIRS ? TP : (TKP > TP ? TKP : TP);
    struct Smem {
        U k[KW];
        uint32_t p[PAIRS ? TP : 1];    // tile position of each element
        uint32_t pay[PAIRS ? T : 1];   // payload, by tile position
    };

    using E = typename std::conditional<PAIRS, KeyPos<U>, U>::type;

    static __device__ __forceinline__ E make(U k, uint32_t pos) {
        if constexpr (PAIRS) return KeyPos<U>{k, pos};
        else return k;
    }
    static __device__ __forceinline__ U key_of(const E& e) {
        if constexpr (PAIRS) return e.k;
        else return e;
    }

    static __device__ __forceinline__ bool before(U ka, uint32_t pa, U kb, uint32_t pb) {
        if constexpr (PAIRS) return ka < kb || (ka == kb && pa < pb);
        else return ka < kb;
    }

    // One merge level in LDS: runs of `width` become runs of 2*width.  The
    // thread produces outputs [tid*IT, tid*IT + IT) of its 2*width group.
    static __device__ __forceinline__ void lds_level(const Smem& sm, int width, int tid, E (&v)[IT]) {
        const int out0 = tid * IT;
        const int gs = out0 & ~(2 * width - 1);
        const int d = out0 - gs;
        int lo = d > width ? d - width : 0;
        int hi = d < width ? d : width;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int xa = pad(gs + mid), xb = pad(gs + width + d - 1 - mid);
            bool a_first;
            if constexpr (PAIRS) a_first = !before(sm.k[xb], sm.p[xb], sm.k[xa], sm.p[xa]);
            else a_first = sm.k[xa] <= sm.k[xb];
            if (a_first) lo = mid + 1;
            else hi = mid;
        }
        int i = lo, j = d - lo;
        int ia = pad(gs + (i < width ? i : width - 1));
        int ib = pad(gs + width + (j < width ? j : width - 1));
        U a = sm.k[ia], b = sm.k[ib];
        uint32_t pa = 0, pb = 0;
        if constexpr (PAIRS) {
            pa = sm.p[ia];
            pb = sm.p[ib];
        }
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const bool ta = (j >= width) || (i < width && !before(b, pb, a, pa));
            if constexpr (PAIRS) v[r] = make(ta ? a : b, ta ? pa : pb);
            else v[r] = ta ? a : b;
            i += ta ? 1 : 0;
            j += ta ? 0 : 1;
            const int nx = pad(ta ? gs + (i < width ? i : width - 1) : gs + width + (j < width ? j : width - 1));
            const U kn = sm.k[nx];
            a = ta ? kn : a;
            b = ta ? b : kn;
            if constexpr (PAIRS) {
                const uint32_t pn = sm.p[nx];
                pa = ta ? pn : pa;
                pb = ta ? pb : pn;
            }
        }
    }

    // Keys only: the IT outputs of thread tid (positions tid*IT .. of runs of
    // width w) to the gapped layout; threads below the gap count fill the
    // gaps after the runs with the largest code.
    static __device__ __forceinline__ void put_k(Smem& sm, int w, int tid, const U (&v)[IT]) {
        const int out0 = tid * IT;
        const int q = out0 >> __builtin_ctz((unsigned)w);   // w is a power of two
        const int l0 = G + q * (w + G) + (out0 - q * w);
#pragma unroll
        for (int r = 0; r < IT; ++r) sm.k[pad(l0 + r)] = v[r];
        const int runs = T / w;
        if (w < T && tid < runs * G) {
            const int q2 = tid / G;
            sm.k[pad(G + q2 * (w + G) + w + (tid - q2 * G))] = key_max<U>();
        }
    }

    // Keys only: one merge level in the gapped layout, runs of width w become
    // runs of 2w; thread tid produces outputs [tid*IT, tid*IT + IT) of its
    // group.  The co-rank search takes fixed power-of-two steps (no exit
    // test per lane); the serial merge reads both run heads each step.
    // Byte offset of logical slot l in the keys-only layout, (l + l/32) *
    // sizeof(U), as one shift and one add-shift (the compiler's own form of
    // this expression takes three instructions).
    static __device__ __forceinline__ uint32_t slot_bytes(uint32_t l) {
        constexpr int SH = sizeof(U) == 8 ? 3 : 2;
        uint32_t t, r;
        asm("v_lshrrev_b32 %0, 5, %1" : "=v"(t) : "v"(l));
        asm("v_add_lshl_u32 %0, %1, %2, %3" : "=v"(r) : "v"(l), "v"(t), "i"(SH));
        return r;
    }

    static __device__ __forceinline__ void lds_level_k(const Smem& sm, int w, int tid, U (&v)[IT]) {
        using LU = const __attribute__((address_space(3))) U;   // 32-bit LDS addresses
        using LB = const __attribute__((address_space(3))) char;
        LB* kb = (LB*)sm.k;
        auto ld = [kb](int l) { return *(LU*)(kb + slot_bytes((uint32_t)l)); };
        const int out0 = tid * IT;
        const int g = out0 >> (__builtin_ctz((unsigned)w) + 1);   // w is a power of two
        const int d = out0 - g * 2 * w;
        const int a0 = G + 2 * g * (w + G);
        const int b0 = a0 + w + G;
        const int lo = d > w ? d - w : 0;
        const int hi = d < w ? d : w;
        // i = lo + the number of x in [lo, hi) with A[x] <= B[d-1-x].  Probe
        // t reads A[t-1] and B[d-t]; i <= hi <= w and s <= w keep both
        // inside [a0 - 1, b0 + w] even when t > hi (then the probe is void).
        int i = lo;
#pragma unroll 1
        for (int s = w; s >= 1; s >>= 1) {
            const int t = i + s;
            const bool ok = (t <= hi) & (ld(a0 - 1 + t) <= ld(b0 + d - t));
            i = ok ? t : i;
        }
        uint32_t pa = (uint32_t)(a0 + i), pb = (uint32_t)(b0 + d - i);   // heads
        U a = ld(pa), b = ld(pb);
        if constexpr (sizeof(U) == 4) {
            // One output in eight VALU instructions: the compare's carry bit
            // advances B's head (add with carry) or A's (subtract with
            // borrow of -1), then both padded addresses.  ALU only; the
            // loads stay with the compiler.  The compiler's own form of this
            // step takes ten to eleven.  s_nop: wait states before a VALU
            // reads VCC as a carry right after a VALU wrote it.
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                uint32_t o, xa, xb, t1, t2;
                uint64_t c;
                asm("v_cmp_lt_u32 vcc, %[b], %[a]\n\t"
                    "v_min_u32 %[o], %[b], %[a]\n\t"
                    "s_nop 1\n\t"
                    "v_addc_co_u32_e64 %[pb], %[c], %[pb], 0, vcc\n\t"
                    "v_subb_co_u32_e64 %[pa], %[c], %[pa], -1, vcc\n\t"
                    "v_lshrrev_b32 %[t1], 5, %[pa]\n\t"
                    "v_lshrrev_b32 %[t2], 5, %[pb]\n\t"
                    "v_add_lshl_u32 %[xa], %[pa], %[t1], 2\n\t"
                    "v_add_lshl_u32 %[xb], %[pb], %[t2], 2"
                    : [o] "=&v"(o), [pa] "+v"(pa), [pb] "+v"(pb), [xa] "=&v"(xa), [xb] "=&v"(xb), [t1] "=&v"(t1),
                      [t2] "=&v"(t2), [c] "=&s"(c)
                    : [a] "v"(a), [b] "v"(b)
                    : "vcc");
                v[r] = o;
                if (r + 1 < IT) {
                    a = *(LU*)(kb + xa);
                    b = *(LU*)(kb + xb);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const bool tb = b < a;
                v[r] = tb ? b : a;
                pa += tb ? 0u : 1u;
                pb += tb ? 1u : 0u;
                if (r + 1 < IT) {
                    a = ld(pa);
                    b = ld(pb);
                }
            }
        }
    }

    static __device__ __forceinline__ void put(Smem& sm, int tid, const E (&v)[IT]) {
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int x = pad(tid * IT + r);
            if constexpr (PAIRS) {
                sm.k[x] = v[r].k;
                sm.p[x] = v[r].p;
            } else {
                sm.k[x] = v[r];
            }
        }
    }

    // A segment of at most 64 * IT keys sorted by the calling wavefront alone
    // (registers and cross-lane exchanges, no LDS and no barrier); src may
    // equal dst, psrc may equal pdst.
    static constexpr int WAVE_T = kWave * IT;
    static __device__ void run_wave(const S* src, S* dst, const uint32_t* psrc, uint32_t* pdst, int valid) {
        const int lane = (int)__lane_id();
        E v[IT];
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int e = lane + r * kWave;
            v[r] = make(e < valid ? C::enc(src[e]) : key_max<U>(), (uint32_t)e);
        }
        wave_sort(v);
        // value r of lane L is output L * IT + r
        uint32_t pv[PAIRS ? IT : 1];
        if constexpr (PAIRS) {
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const int o = lane * IT + r;
                pv[r] = o < valid ? psrc[v[r].p] : 0u;  // every read before any write
            }
        }
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int o = lane * IT + r;
            if (o < valid) {
                dst[o] = C::dec(key_of(v[r]));
                if constexpr (PAIRS) pdst[o] = pv[r];
            }
        }
    }

    // desc (optional): the sorted tile's codes at positions 0, valid-1, T/2-1
    // and T/2 (the last two only when the tile holds more than T/2 keys), for
    // the NEAR test of the general plan.
    static __device__ void run(Smem& sm, const S* src, S* dst, const uint32_t* psrc, uint32_t* pdst, int valid,
                               unsigned long long* desc = nullptr) {
        body(sm, src, dst, psrc, pdst, valid, desc);
    }
    // run() inlined, for a launch's main call site: the LDS array's address
    // is then a constant that folds into the instructions' offsets.
    static __device__ __forceinline__ void body(Smem& sm, const S* src, S* dst, const uint32_t* psrc,
                                                uint32_t* pdst, int valid, unsigned long long* desc = nullptr) {
        const int tid = threadIdx.x;
        E v[IT];
        const bool vec = valid == T && aligned16(src) && (!PAIRS || aligned16(psrc));
        if (vec) {
#pragma unroll
            for (int q = 0; q < IT / VN; ++q) {
                const int e0 = (tid + q * WG) * VN;
                const V16<S> x = reinterpret_cast<const V16<S>*>(src)[tid + q * WG];
#pragma unroll
                for (int j = 0; j < VN; ++j) v[q * VN + j] = make(C::enc(x.v[j]), (uint32_t)(e0 + j));
            }
        } else {
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const int e = tid + r * WG;
                v[r] = make(e < valid ? C::enc(src[e]) : key_max<U>(), (uint32_t)e);
            }
        }
        if constexpr (PAIRS) {
            for (int e = tid; e < valid; e += WG) sm.pay[e] = psrc[e];
        }

        wave_sort(v);

        if constexpr (!PAIRS) {
            put_k(sm, kWave * IT, tid, v);
#pragma unroll 1
            for (int width = kWave * IT; width < T; width *= 2) {
                __syncthreads();
                lds_level_k(sm, width, tid, v);
                __syncthreads();
                put_k(sm, 2 * width, tid, v);
            }
        } else if constexpr (T > kWave * IT) {
            put(sm, tid, v);
#pragma unroll 1
            for (int width = kWave * IT; width < T; width *= 2) {
                __syncthreads();
                lds_level(sm, width, tid, v);
                __syncthreads();
                put(sm, tid, v);
            }
        } else {
            put(sm, tid, v);
        }
        __syncthreads();

        // position of sorted element e in LDS
        auto at = [](int e) { return PAIRS ? pad(e) : pad(G + e); };
        if (desc != nullptr && tid < 4) {
            constexpr int H = T / 2;
            const int pos = tid == 0 ? 0 : tid == 1 ? valid - 1 : tid == 2 ? H - 1 : H;
            if (tid < 2 || valid > H) desc[tid] = (unsigned long long)sm.k[at(pos)];
        }
        // store, striped so that consecutive lanes write consecutive addresses
        const bool vout = valid == T && aligned16(dst);
        if (vout) {
#pragma unroll
            for (int q = 0; q < IT / VN; ++q) {
                const int e0 = (tid + q * WG) * VN;
                V16<S> x;
#pragma unroll
                for (int j = 0; j < VN; ++j) x.v[j] = C::dec(sm.k[at(e0 + j)]);
                reinterpret_cast<V16<S>*>(dst)[tid + q * WG] = x;
            }
        } else {
            for (int e = tid; e < valid; e += WG) dst[e] = C::dec(sm.k[at(e)]);
        }
        if constexpr (PAIRS) {
            for (int e = tid; e < valid; e += WG) pdst[e] = sm.pay[sm.p[pad(e)]];
        }
    }
};

// ================================================================== merge
// One output chunk of WG*IT keys of one merge pass: the runs A = [gs, gs+w)
// and B = [gs+w, gs+2w) of src (clipped to n) are merged into dst[gs, ...).
// Phases: window bounds (two Merge Path co-ranks, precomputed or searched by
// wavefronts 0 and 1), window loads into registers, staging in LDS, a
// per-thread co-rank search inside LDS and a serial merge of IT outputs,
// then the outputs go back through LDS (padded by one slot per 16, so the
// blocked writes do not collide in banks) and out as coalesced vectors.
// Ties take A: stable.
template <class C, int WG, int IT, bool PAIRS>
struct MergeChunk {
    using S = typename C::S;
    using U = typename C::U;
    static constexpr int CH = WG * IT;
    static constexpr int ITEMS = IT;
    static constexpr int VN = 16 / sizeof(S);
    static constexpr int PADDED = CH + CH / 16;
    // keys only: GAP slots of the largest code after each staged run (A at
    // [0, na), B at [na + GAP, cnt + GAP)), so that the serial merge reads
    // past a run's end without a bounds test
    static constexpr int GAP = PAIRS ? 0 : IT;
    static_assert(WG >= 2 * kWave, "two wavefronts search the window bounds");
    static_assert(IT % VN == 0, "whole vectors per thread");
    static_assert(PADDED >= CH + 2 * GAP + 1, "both runs, their stops and one read past them fit the buffer");
    static_assert(WG >= 2 * GAP, "one thread per stop slot");

    struct Buf {
        U k[PADDED];
        uint32_t pay[PAIRS ? PADDED : 1];
    };
    struct Smem {
        Buf b;
        int64_t co[2];
    };

    static __device__ __forceinline__ int pad(int e) { return e + (e >> 4); }

    // Window of one chunk: where its inputs are and its loaded blocks.
    // A = src[gA, gA + na) and B = src[gB, gB + cnt - na) are read as the
    // aligned 16-byte blocks that cover them (RV per thread hold a window of
    // CH keys however its two parts sit on block boundaries).  A block at a
    // window edge is read whole: it never crosses a page, so the extra keys it
    // brings lie in mapped memory, and stage() drops them.  Payloads likewise,
    // in blocks of four.
    static constexpr int NBLK = CH / VN + 2;
    static constexpr int RV = (NBLK + WG - 1) / WG;
    static constexpr int RVP = PAIRS ? (CH / 4 + 2 + WG - 1) / WG : 1;
    struct Win {
        int64_t out0;   // first output of the chunk (segment-relative)
        int64_t gA;     // first A element of the window (segment-relative)
        int64_t gB;     // first B element of the window
        int na, cnt;
        int offA, offB, nbA, nbB;      // key blocks: elements before gA / gB in their first block; block counts
        int poffA, poffB, pnbA, pnbB;  // the same for the payload blocks
        V16<S> x[RV];
        uint4 px[RVP];
    };

    // Runs being merged: pairs of width `width` aligned at multiples of
    // 2*width, or, when split >= 0, the single pair [0, split), [split, n).
    static __device__ __forceinline__ void bounds(int64_t n, int64_t width, int64_t split, int64_t out0,
                                                  int64_t& gs, int64_t& la, int64_t& lb, int64_t& d0, int64_t& d1) {
        if (split >= 0) {
            gs = 0;
            la = split;
            lb = n - split;
        } else {
            // group start; the widths of level-synchronous passes are powers
            // of two, which spares the 64-bit division
            const int64_t g = 2 * width;
            gs = (g & (g - 1)) == 0 ? (out0 & ~(g - 1)) : out0 / g * g;
            la = (n - gs) < width ? (n - gs) : width;
            const int64_t rest = n - gs - la;
            lb = rest < width ? rest : width;
        }
        d0 = out0 - gs;
        d1 = (d0 + CH) < (la + lb) ? (d0 + CH) : (la + lb);
    }

    // Window of the chunk starting at out0 from precomputed co-ranks (co is
    // indexed by chunk number relative to the same array start).
    static __device__ __forceinline__ void window_from_co(int64_t n, int64_t width, int64_t split, int64_t out0,
                                                          const int64_t* co, Win& w) {
        int64_t gs, la, lb, d0, d1;
        bounds(n, width, split, out0, gs, la, lb, d0, d1);
        const int64_t c = out0 / CH;
        const int64_t i0 = co[c];
        const int64_t i1 = d1 == la + lb ? la : co[c + 1];
        w.out0 = out0;
        w.gA = gs + i0;
        w.gB = gs + la + (d0 - i0);
        w.na = (int)(i1 - i0);
        w.cnt = (int)(d1 - d0);
    }

    // Same, with the co-ranks searched here by wavefronts 0 and 1.
    static __device__ __forceinline__ void window_search(Smem& sm, const S* src, int64_t n, int64_t width,
                                                         int64_t split, int64_t out0, Win& w) {
        int64_t gs, la, lb, d0, d1;
        bounds(n, width, split, out0, gs, la, lb, d0, d1);
        const int wave = threadIdx.x / kWave;
        if (wave < 2) {
            const int64_t c = corank_wave<C>(src + gs, la, src + gs + la, lb, wave == 0 ? d0 : d1);
            if (__lane_id() == 0) sm.co[wave] = c;
        }
        __syncthreads();
        const int64_t i0 = sm.co[0], i1 = sm.co[1];
        w.out0 = out0;
        w.gA = gs + i0;
        w.gB = gs + la + (d0 - i0);
        w.na = (int)(i1 - i0);
        w.cnt = (int)(d1 - d0);
    }

    // Issue every window load of this thread (they stay in flight until stage()).
    // NT: nontemporal loads and stores, for arrays far larger than the caches
    // (the pass's data is not read again before the next pass).
    template <class T, int TN, bool NT>
    static __device__ __forceinline__ void load_blocks(const T* base, int64_t gA, int64_t gB, int na, int nb,
                                                       int& offA, int& offB, int& nbA, int& nbB,
                                                       V16<T> (&x)[(TN == 0 ? 1 : TN)]) {
        constexpr int E = 16 / (int)sizeof(T);
        const uintptr_t pa = (uintptr_t)(base + gA), pb = (uintptr_t)(base + gB);
        offA = (int)((pa & 15u) / sizeof(T));
        offB = (int)((pb & 15u) / sizeof(T));
        nbA = na > 0 ? (offA + na + E - 1) / E : 0;
        nbB = nb > 0 ? (offB + nb + E - 1) / E : 0;
        const V16<T>* bA = reinterpret_cast<const V16<T>*>(pa & ~(uintptr_t)15);
        const V16<T>* bB = reinterpret_cast<const V16<T>*>(pb & ~(uintptr_t)15);
        typedef unsigned int v4u __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int r = 0; r < TN; ++r) {
            const int blk = threadIdx.x + r * WG;
            const V16<T>* q = blk < nbA ? bA + blk : bB + (blk - nbA);
            if (blk < nbA + nbB) {
                if constexpr (NT) {
                    const v4u t = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(q));
                    x[r] = *reinterpret_cast<const V16<T>*>(&t);
                } else {
                    x[r] = *q;
                }
            }
        }
    }

    template <bool NT = false>
    static __device__ __forceinline__ void load(const S* src, const uint32_t* psrc, Win& w) {
        const int nb = w.cnt - w.na;
        load_blocks<S, RV, NT>(src, w.gA, w.gB, w.na, nb, w.offA, w.offB, w.nbA, w.nbB, w.x);
        if constexpr (PAIRS) {
            load_blocks<uint32_t, RVP, NT>(psrc, w.gA, w.gB, w.na, nb, w.poffA, w.poffB, w.pnbA, w.pnbB,
                                           reinterpret_cast<V16<uint32_t>(&)[RVP]>(w.px));
        }
    }

    // The loaded blocks into LDS: A at [0, na), B at [na + gap, cnt + gap),
    // keys encoded.
    template <class T, int TN, class F>
    static __device__ __forceinline__ void stage_blocks(const V16<T> (&x)[(TN == 0 ? 1 : TN)], int na, int nb,
                                                        int offA, int offB, int nbA, int nbB, int gap, F&& put) {
        constexpr int E = 16 / (int)sizeof(T);
#pragma unroll
        for (int r = 0; r < TN; ++r) {
            const int blk = threadIdx.x + r * WG;
            if (blk < nbA + nbB) {
                const bool inA = blk < nbA;
                const int e0 = inA ? blk * E - offA : (blk - nbA) * E - offB;  // part-relative index of x.v[0]
                const int lim = inA ? na : nb;
                const int to = inA ? 0 : na + gap;
                if (e0 >= 0 && e0 + E <= lim) {
#pragma unroll
                    for (int j = 0; j < E; ++j) put(to + e0 + j, x[r].v[j]);
                } else {
#pragma unroll
                    for (int j = 0; j < E; ++j)
                        if (e0 + j >= 0 && e0 + j < lim) put(to + e0 + j, x[r].v[j]);
                }
            }
        }
    }

    static __device__ __forceinline__ void stage(Buf& b, const Win& w) {
        const int nb = w.cnt - w.na;
        stage_blocks<S, RV>(w.x, w.na, nb, w.offA, w.offB, w.nbA, w.nbB, GAP,
                            [&](int e, S v) { b.k[e] = C::enc(v); });
        if constexpr (PAIRS) {
            stage_blocks<uint32_t, RVP>(reinterpret_cast<const V16<uint32_t>(&)[RVP]>(w.px), w.na, nb, w.poffA,
                                        w.poffB, w.pnbA, w.pnbB, 0, [&](int e, uint32_t v) { b.pay[e] = v; });
        } else {
            // the stops after A and after B
            const int t = threadIdx.x;
            if (t < 2 * GAP) b.k[t < GAP ? w.na + t : w.cnt + t] = ~(U)0;
        }
    }

    // Serial merge of this thread's IT outputs from the staged window.
    static __device__ __forceinline__ void merge(const Buf& b, int na, int cnt, U (&v)[IT], uint32_t (&pv)[IT]) {
        const int t0 = threadIdx.x * IT;
        if (t0 >= cnt) return;
        const int nb = cnt - na;
        const int b0 = na + GAP;  // first staged B slot
        int i;
        {
            // co-rank of t0 between the staged A = [0, na) and B = [b0, b0 + nb)
            int lo = t0 > nb ? t0 - nb : 0;
            int hi = t0 < na ? t0 : na;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (b.k[mid] <= b.k[b0 + t0 - 1 - mid]) lo = mid + 1;
                else hi = mid;
            }
            i = lo;
        }
        int j = t0 - i;
        if constexpr (!PAIRS) {
            // Keys only: an exhausted run reads its stops, the largest code.
            // Taking a stop instead of an equal key of the other run writes
            // the same bits, and every key still to come is then that value
            // too (both runs are sorted), so the output is exact.  A run's
            // index passes its end only while both heads hold the largest
            // code, one slot per output: with IT stops only the read after
            // the last output (never used) can land past them, at most at
            // cnt + 2 GAP, inside the buffer.
            int pa = i, pb = b0 + j;
            U a = b.k[pa], bb = b.k[pb];
#pragma unroll
            for (int r = 0; r < IT; ++r) {
                const bool ta = a <= bb;
                v[r] = ta ? a : bb;
                pa += ta ? 1 : 0;
                pb += ta ? 0 : 1;
                const U kn = b.k[ta ? pa : pb];
                a = ta ? kn : a;
                bb = ta ? bb : kn;
            }
            return;
        }
        const int last = cnt - 1;
        int ia = i < na ? i : last;
        int ib = na + (j < nb ? j : nb - 1);
        ib = ib < 0 ? 0 : ib;
        U a = b.k[ia], bb = b.k[ib];
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const bool ta = (j >= nb) || (i < na && a <= bb);
            v[r] = ta ? a : bb;
            if constexpr (PAIRS) pv[r] = b.pay[ta ? (i < na ? i : last) : (na + j < cnt ? na + j : last)];
            i += ta ? 1 : 0;
            j += ta ? 0 : 1;
            int nx = ta ? i : na + j;
            nx = nx < last ? nx : last;
            const U kn = b.k[nx];
            a = ta ? kn : a;
            bb = ta ? bb : kn;
        }
    }

    static __device__ __forceinline__ void stage_out(Buf& b, int cnt, const U (&v)[IT], const uint32_t (&pv)[IT]) {
        const int t0 = threadIdx.x * IT;
        if (t0 >= cnt) return;
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            if (t0 + r < cnt) {
                b.k[pad(t0 + r)] = v[r];
                if constexpr (PAIRS) b.pay[pad(t0 + r)] = pv[r];
            }
        }
    }

    template <bool NT = false>
    static __device__ __forceinline__ void store(const Buf& b, S* dst, uint32_t* pdst, int64_t out0, int cnt) {
        const int tid = threadIdx.x;
        S* out = dst + out0;
        if (cnt == CH && aligned16(out)) {
#pragma unroll
            for (int q = 0; q < IT / VN; ++q) {
                const int e0 = (tid + q * WG) * VN;
                V16<S> x;
#pragma unroll
                for (int j = 0; j < VN; ++j) x.v[j] = C::dec(b.k[pad(e0 + j)]);
                if constexpr (NT) {
                    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
                    __builtin_nontemporal_store(*reinterpret_cast<const v4u*>(&x),
                                                reinterpret_cast<v4u*>(out) + tid + q * WG);
                } else {
                    reinterpret_cast<V16<S>*>(out)[tid + q * WG] = x;
                }
            }
        } else {
            for (int e = tid; e < cnt; e += WG) out[e] = C::dec(b.k[pad(e)]);
        }
        if constexpr (PAIRS) {
            uint32_t* pout = pdst + out0;
            if (cnt == CH && aligned16(pout)) {
#pragma unroll
                for (int q = 0; q < IT / 4; ++q) {
                    const int e0 = (tid + q * WG) * 4;
                    uint4 x;
                    x.x = b.pay[pad(e0)];
                    x.y = b.pay[pad(e0 + 1)];
                    x.z = b.pay[pad(e0 + 2)];
                    x.w = b.pay[pad(e0 + 3)];
                    reinterpret_cast<uint4*>(pout)[tid + q * WG] = x;
                }
            } else {
                for (int e = tid; e < cnt; e += WG) pout[e] = b.pay[pad(e)];
            }
        }
    }

    // One chunk, start to end.  src/dst/psrc/pdst point at the start of the
    // (segment) array of length n; co (optional) holds precomputed co-ranks.
    // Keys only, a whole chunk into a 16-byte aligned output: each thread
    // holds IT consecutive outputs and stores them straight from registers.
    // Returns false (for the whole workgroup alike) where it does not apply.
    // Not with nontemporal stores: a wavefront's store then writes a quarter
    // of each of 64 lines, and such partial lines bypass the cache that
    // would join them (a merge pass at 256M keys took 4x as long).
    template <bool NT = false>
    static __device__ __forceinline__ bool store_direct(S* dst, int64_t out0, int cnt, const U (&v)[IT]) {
        if constexpr (PAIRS || NT) {
            return false;
        } else {
            S* out = dst + out0;
            if (cnt != CH || !aligned16(out)) return false;
            V16<S>* q = reinterpret_cast<V16<S>*>(out + threadIdx.x * IT);
#pragma unroll
            for (int k = 0; k < IT / VN; ++k) {
                V16<S> x;
#pragma unroll
                for (int j = 0; j < VN; ++j) x.v[j] = C::dec(v[k * VN + j]);
                q[k] = x;
            }
            return true;
        }
    }

    static __device__ void run(Smem& sm, const S* src, S* dst, const uint32_t* psrc, uint32_t* pdst,
                               int64_t n, int64_t width, int64_t split, int64_t out0, const int64_t* co) {
        Win w;
        if (co != nullptr) window_from_co(n, width, split, out0, co, w);
        else window_search(sm, src, n, width, split, out0, w);
        load(src, psrc, w);
        stage(sm.b, w);
        __syncthreads();
        U v[IT];
        uint32_t pv[IT];
        merge(sm.b, w.na, w.cnt, v, pv);
        if (store_direct(dst, out0, w.cnt, v)) return;
        __syncthreads();
        stage_out(sm.b, w.cnt, v, pv);
        __syncthreads();
        store(sm.b, dst, pdst, out0, w.cnt);
    }
};

// Persistent, double-buffered form of one merge pass: a workgroup walks the
// chunks c = blockIdx.x, + gridDim.x, ...; while it merges chunk c out of one
// LDS buffer, the window loads of its next chunk are already in flight into
// registers, and they are staged into the other buffer.
template <class C, int WG, int IT, bool PAIRS>
struct MergePersistent {
    using MC = MergeChunk<C, WG, IT, PAIRS>;
    using S = typename C::S;
    using U = typename C::U;
    static constexpr int CH = MC::CH;
    struct Smem {
        typename MC::Buf b[2];
    };

    template <bool NT = false>
    static __device__ __forceinline__ void run(Smem& sm, const S* src, S* dst, const uint32_t* psrc, uint32_t* pdst,
                                               int64_t n, int64_t width, int64_t split, const int64_t* co) {
        const int64_t nchunks = (n + CH - 1) / CH;
        int64_t c = blockIdx.x;
        if (c >= nchunks) return;
        typename MC::Win w;
        MC::window_from_co(n, width, split, c * CH, co, w);
        MC::template load<NT>(src, psrc, w);
        int buf = 0;
        for (;;) {
            MC::stage(sm.b[buf], w);
            const int na = w.na, cnt = w.cnt;
            const int64_t out0 = w.out0;
            __syncthreads();
            const int64_t cn = c + gridDim.x;
            if (cn < nchunks) {
                MC::window_from_co(n, width, split, cn * CH, co, w);
                MC::template load<NT>(src, psrc, w);
            }
            U v[IT];
            uint32_t pv[IT];
            MC::merge(sm.b[buf], na, cnt, v, pv);
            // the next stage() into this buffer comes after the next
            // iteration's barrier, which every thread reaches only after
            // this merge has read it
            if (!MC::template store_direct<NT>(dst, out0, cnt, v)) {
                __syncthreads();
                MC::stage_out(sm.b[buf], cnt, v, pv);
                __syncthreads();
                MC::template store<NT>(sm.b[buf], dst, pdst, out0, cnt);
            }
            if (cn >= nchunks) break;
            c = cn;
            buf ^= 1;
        }
    }
};

// ============================================================ four-way merge
// A pass of fan-in four (keys only): each group of four neighbouring runs
// R0..R3 of width w (clipped to n) becomes one sorted run of 4w, so two
// levels of the merge tree cost one read and one write of the array (the
// rounds of pairwise merging of Sec. 3 (e1), taken two at a time).
// Partition: run q is sampled every D keys from offset q*D/4 (staggered, so
// that runs of alike values do not put their samples side by side, which
// would leave most chunks nearly empty and a few full).  A sample x = R_r[o]
// cuts the group where x stands in the merge order (key, then run): the keys
// of R_q before it are those <= x for q < r and those < x for q > r, and its
// place among the group's cuts follows from those counts (the samples of R_q
// before x are those at offsets below the count).  Cut 0 is the group start.
// Between two consecutive cuts each run has fewer than D keys, so a chunk
// holds at most 4D keys.  One workgroup per chunk stages its four ranges in
// LDS, merges R0 with R1 and R2 with R3, then the two results, and writes the
// chunk at its rank.
template <class C>
struct Merge4 {
    using S = typename C::S;
    using U = typename C::U;
    static constexpr int WG = 256;
    static constexpr int D = sizeof(S) == 4 ? 2048 : 1024;  // sample stride
    static constexpr int CAP = 4 * D;                         // keys of a chunk at most
    static constexpr int ITM = CAP / WG;                      // outputs per thread at most
    struct Smem {
        U k[CAP];
    };

    static __host__ __device__ __forceinline__ int64_t run_len(int64_t n, int64_t gs, int64_t w, int q) {
        const int64_t a = n - gs - (int64_t)q * w;
        return a <= 0 ? 0 : (a < w ? a : w);
    }
    // first sampled offset of run q, and the samples of a run of l keys
    static __host__ __device__ __forceinline__ int64_t phase(int q) { return (int64_t)q * (D / 4); }
    static __host__ __device__ __forceinline__ int64_t nsamp(int64_t l, int q) {
        return l <= phase(q) ? 0 : (l - phase(q) + D - 1) / D;
    }
    // samples of run q at offsets below c
    static __device__ __forceinline__ int64_t below(int64_t c, int q) {
        return c <= phase(q) ? 0 : (c - phase(q) + D - 1) / D;
    }
    // cut slots of a full group (its samples and cut 0)
    static __host__ __device__ __forceinline__ int64_t per_group(int64_t w) { return 4 * (w / D) + 1; }

    // Chunks (= cut slots) of the pass over n keys in runs of w.
    static __host__ __device__ __forceinline__ int64_t chunks(int64_t n, int64_t w) {
        if (n <= 0) return 0;
        const int64_t G = (n + 4 * w - 1) / (4 * w);
        const int64_t gs = (G - 1) * 4 * w;
        int64_t last = 1;
        for (int q = 0; q < 4; ++q) last += nsamp(run_len(n, gs, w, q), q);
        return (G - 1) * per_group(w) + last;
    }
    // Sample threads of the pass: 4 w / D per group, a run after another.
    static __host__ __device__ __forceinline__ int64_t sample_slots(int64_t n, int64_t w) {
        return (n + 4 * w - 1) / (4 * w) * (4 * (w / D));
    }

    // Sample thread s: the cut of its sample into splits[group base + place].
    static __device__ __forceinline__ void sample(const S* src, int64_t n, int64_t w, int64_t s, uint4* splits) {
        const int64_t per_run = w / D;
        const int64_t g = s / (4 * per_run);
        const int64_t l = s - g * 4 * per_run;
        const int r = (int)(l / per_run);
        const int64_t k = l - (int64_t)r * per_run;
        const int64_t gs = g * 4 * w;
        const int64_t off = phase(r) + k * D;
        int64_t lo[4], hi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            lo[q] = 0;
            hi[q] = q == r ? 0 : run_len(n, gs, w, q);
        }
        if (off >= run_len(n, gs, w, r)) return;
        const U x = C::enc(src[gs + (int64_t)r * w + off]);
        // the three searches advance together, their loads in flight at once
        for (int step = 0; step < 40; ++step) {
            U y[4];
            bool act[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                act[q] = lo[q] < hi[q];
                const int64_t mid = (lo[q] + hi[q]) >> 1;
                y[q] = act[q] ? C::enc(src[gs + (int64_t)q * w + mid]) : (U)0;
            }
            if (!(act[0] || act[1] || act[2] || act[3])) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (act[q]) {
                    const int64_t mid = (lo[q] + hi[q]) >> 1;
                    const bool before = q < r ? y[q] <= x : y[q] < x;
                    if (before) lo[q] = mid + 1;
                    else hi[q] = mid;
                }
            }
        }
        int64_t c[4];
        int64_t pos = 1 + k;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c[q] = q == r ? off : lo[q];
            if (q != r) pos += below(c[q], q);
        }
        splits[g * per_group(w) + pos] =
            make_uint4((unsigned)c[0], (unsigned)c[1], (unsigned)c[2], (unsigned)c[3]);
    }

    // co-rank of diagonal d between k[a0, a0 + na) and k[b0, b0 + nb) in LDS
    static __device__ __forceinline__ int corank(const U* k, int a0, int na, int b0, int nb, int d) {
        int lo = d > nb ? d - nb : 0;
        int hi = d < na ? d : na;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (k[a0 + mid] <= k[b0 + d - 1 - mid]) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    }

    // Merge cursor over A = k[.., ea) and B = k[.., eb); an exhausted run reads
    // as the largest code (taking it for an equal key writes the same bits).
    struct Cur {
        int pa, ea, pb, eb;
        U a, b;
    };
    static __device__ __forceinline__ Cur cursor(const U* k, int pa, int ea, int pb, int eb) {
        constexpr U kMax = ~(U)0;
        Cur c;
        c.pa = pa;
        c.ea = ea;
        c.pb = pb;
        c.eb = eb;
        c.a = pa < ea ? k[pa] : kMax;
        c.b = pb < eb ? k[pb] : kMax;
        return c;
    }
    static __device__ __forceinline__ U next(const U* k, Cur& c) {
        constexpr U kMax = ~(U)0;
        const bool ta = c.a <= c.b;
        const U out = ta ? c.a : c.b;
        c.pa += ta ? 1 : 0;
        c.pb += ta ? 0 : 1;
        const int nx = ta ? c.pa : c.pb;
        const U kn = nx < (ta ? c.ea : c.eb) ? k[nx] : kMax;
        c.a = ta ? kn : c.a;
        c.b = ta ? c.b : kn;
        return out;
    }

    // Chunk c of the pass (one workgroup of WG threads).
    template <bool NT>
    static __device__ __forceinline__ void chunk(Smem& sm, const S* src, S* dst, int64_t n, int64_t w, int64_t c,
                                                 const uint4* splits) {
        const int tid = threadIdx.x;
        const int64_t per = per_group(w);
        const int64_t g = c / per;
        const int64_t t = c - g * per;
        const int64_t gs = g * 4 * w;
        int64_t len[4];
        int64_t ns = 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            len[q] = run_len(n, gs, w, q);
            ns += nsamp(len[q], q);
        }
        if (t >= ns) return;
        const uint4 a = t == 0 ? make_uint4(0u, 0u, 0u, 0u) : splits[c];
        const uint4 e = t + 1 < ns ? splits[c + 1]
                                   : make_uint4((unsigned)len[0], (unsigned)len[1], (unsigned)len[2], (unsigned)len[3]);
        const int64_t st[4] = {a.x, a.y, a.z, a.w};
        const int64_t en[4] = {e.x, e.y, e.z, e.w};
        // a cut out of order or past its run would be a partition error:
        // the chunk is then left unwritten rather than read out of bounds
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (st[q] > en[q] || en[q] > len[q]) return;
        const int o1 = (int)(en[0] - st[0]);
        const int o2 = o1 + (int)(en[1] - st[1]);
        const int o3 = o2 + (int)(en[2] - st[2]);
        const int cnt = o3 + (int)(en[3] - st[3]);
        if (cnt > CAP) return;
        const int64_t out0 = gs + st[0] + st[1] + st[2] + st[3];
        // where LDS position i reads from: run q's range, chosen by selects
        // (a local array indexed at run time would live in scratch)
        const S* r0 = src + gs + st[0];
        const S* r1 = src + gs + w + st[1] - o1;
        const S* r2 = src + gs + 2 * w + st[2] - o2;
        const S* r3 = src + gs + 3 * w + st[3] - o3;
        {
            // loads in batches of 8 per thread, all of a batch in flight before
            // the first is used: no branch among them (a lane past the chunk
            // rereads the chunk's last key)
            constexpr int BJ = 8;
            const int nj = (cnt + WG - 1) / WG;
            for (int j0 = 0; j0 < nj; j0 += BJ) {
                S x[BJ];
#pragma unroll
                for (int j = 0; j < BJ; ++j) {
                    const int i0 = tid + (j0 + j) * WG;
                    const int i = i0 < cnt ? i0 : cnt - 1;
                    const S* p = (i < o1 ? r0 : i < o2 ? r1 : i < o3 ? r2 : r3) + i;
                    if constexpr (NT) x[j] = __builtin_nontemporal_load(p);
                    else x[j] = *p;
                }
#pragma unroll
                for (int j = 0; j < BJ; ++j) {
                    const int i = tid + (j0 + j) * WG;
                    if (i < cnt) sm.k[i] = C::enc(x[j]);
                }
            }
        }
        __syncthreads();
        const int it = (cnt + WG - 1) / WG;
        const int p0 = tid * it;
        U v[ITM];
        // level 1: [0, o2) merges R0's range with R1's, [o2, cnt) R2's with R3's
        {
            const int d01 = p0 < o2 ? p0 : o2;
            const int d23 = p0 > o2 ? (p0 < cnt ? p0 - o2 : cnt - o2) : 0;
            const int i01 = corank(sm.k, 0, o1, o1, o2 - o1, d01);
            const int i23 = corank(sm.k, o2, o3 - o2, o3, cnt - o3, d23);
            Cur c01 = cursor(sm.k, i01, o1, o1 + (d01 - i01), o2);
            Cur c23 = cursor(sm.k, o2 + i23, o3, o3 + (d23 - i23), cnt);
#pragma unroll
            for (int r = 0; r < ITM; ++r) {
                if (r < it) {
                    const int p = p0 + r;
                    if (p < o2) v[r] = next(sm.k, c01);
                    else if (p < cnt) v[r] = next(sm.k, c23);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITM; ++r)
            if (r < it && p0 + r < cnt) sm.k[p0 + r] = v[r];
        __syncthreads();
        // level 2: k[0, o2) with k[o2, cnt)
        {
            const int d = p0 < cnt ? p0 : cnt;
            const int i = corank(sm.k, 0, o2, o2, cnt - o2, d);
            Cur cc = cursor(sm.k, i, o2, o2 + (d - i), cnt);
#pragma unroll
            for (int r = 0; r < ITM; ++r)
                if (r < it && p0 + r < cnt) v[r] = next(sm.k, cc);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ITM; ++r)
            if (r < it && p0 + r < cnt) sm.k[p0 + r] = v[r];
        __syncthreads();
        S* out = dst + out0;
        for (int i = tid; i < cnt; i += WG) {
            const S y = C::dec(sm.k[i]);
            if constexpr (NT) __builtin_nontemporal_store(y, out + i);
            else out[i] = y;
        }
    }
};

// ============================================================ NEAR plan
// Part `part` of `parts` of a copy of cn keys (and payloads when psrc is
// set): 16-byte vectors where both sides are aligned, else elements.
template <class S>
__device__ __forceinline__ void copy_part(const S* src, S* dst, const uint32_t* psrc, uint32_t* pdst, int64_t cn,
                                          int64_t part, int64_t parts) {
    constexpr int VN = 16 / (int)sizeof(S);
    const int64_t per = ((cn + parts - 1) / parts + 63) / 64 * 64;
    const int64_t a = part * per;
    const int64_t b = (a + per) < cn ? (a + per) : cn;
    if (a >= b) return;
    if (aligned16(src + a) && aligned16(dst + a)) {
        const int64_t nv = (b - a) / VN;
        const V16<S>* s16 = reinterpret_cast<const V16<S>*>(src + a);
        V16<S>* d16 = reinterpret_cast<V16<S>*>(dst + a);
        for (int64_t i = threadIdx.x; i < nv; i += blockDim.x) d16[i] = s16[i];
        for (int64_t i = a + nv * VN + threadIdx.x; i < b; i += blockDim.x) dst[i] = src[i];
    } else {
        for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) dst[i] = src[i];
    }
    if (psrc != nullptr)
        for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) pdst[i] = psrc[i];
}

// Merge slot 0 of the general plan checks whether the two-round NEAR plan
// sorts the array, from the sorted tiles' descriptors (codes at 0, last,
// T/2-1, T/2): for every tile t, (a) last(t) <= first(t+2); (b) at most T/2
// keys of tile t+1 are below last(t): key T/2 of t+1 >= last(t) (or t+1 holds
// at most T/2 keys); (c) at most T/2 keys of tile t are above first(t+1): key
// T/2-1 of t <= first(t+1).  Then after the rounds (0,1),(2,3),... and
// (1,2),(3,4),... of T-blocks every block boundary is in order.  A
// violation anywhere turns the plan back into GENERAL: every workgroup of
// slot 0 merges alike under both names, and slot 1 on reads the final one.
__device__ __forceinline__ void near_check(Ctl* ctl, const unsigned long long* td, int64_t n, int64_t T) {
    const int64_t ntiles = (n + T - 1) / T;
    const int64_t H = T / 2;
    bool bad = false;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long* d = td + 4 * t;
        if (t + 2 < ntiles && d[1] > td[4 * (t + 2)]) bad = true;
        if (t + 1 < ntiles) {
            const unsigned long long* e = d + 4;
            const int64_t next_len = (n - (t + 1) * T) < T ? (n - (t + 1) * T) : T;
            if (next_len > H && e[3] < d[1]) bad = true;   // tile t is whole: key H-1 exists
            if (d[2] > e[0]) bad = true;
        }
    }
    if (__builtin_amdgcn_ballot_w64(bad) != 0ull && __lane_id() == 0) ctl->path = 3 /* SR_PATH_GENERAL */;
}

// ============================================================ job views
// The launch sequence is fixed on the host; which data a launch works on is
// read from the plan in the control block.  GENERAL sorts the user buffer U
// with ping-pong partner S1 in M merge passes.  OUTLIER sorts the m outliers
// (stored at S1[n-m, n)) with partner U in P passes, then merge slot P merges
// the kept keys S1[0, n-m) with the sorted outliers into U (pairs: the
// outliers carry their indices in PS1[n-m, n) with partner PU, and slots P
// and P + 1 place them and the kept pairs).  FEW sorts its m between-bucket
// keys the same way; its slot P is the fill pass.
template <class S>
struct PassView {
    const S* src;
    S* dst;
    const uint32_t* psrc;
    uint32_t* pdst;
    int64_t n;
    int64_t width;
    int64_t split;
    bool active;
    // a plain copy of cn keys (and payloads) from csrc to cdst in the same slot
    const S* csrc;
    S* cdst;
    const uint32_t* cpsrc;
    uint32_t* cpdst;
    int64_t cn;
    int fan;  // 4: a four-way pass (Merge4) over runs of `width`; else two-way
};

// NEAR (the general plan's candidate, confirmed by merge slot 0 from the tile
// descriptors, which turns it back into GENERAL otherwise): slot 0 is the
// general plan's first pass; slot 1 merges the T-blocks (1,2), (3,4), ... of
// slot 0's output -- the array viewed from offset T, in groups of two blocks --
// and copies block 0; it writes U when slot 0 wrote S1 (M even), else S1, and
// then slot 2 copies S1 back to U.  Later slots do nothing.

template <class S>
__device__ __forceinline__ PassView<S> resolve_merge(const Ctl* ctl, S* U, S* S1, uint32_t* PU, uint32_t* PS1,
                                                     int64_t n, int M, int64_t T, int k, bool fan4 = false) {
    PassView<S> v{};
    v.active = false;
    v.split = -1;
    v.cn = 0;
    v.fan = 2;
    const int path = ctl->path;
    if (fan4 && path == 3 /* SR_PATH_GENERAL */) {
        // four-way schedule: slot k (even) merges the levels k and k+1 in one
        // pass, from runs of T << k to runs of T << (k+2); odd slots are
        // empty; with M odd the last slot is a two-way pass
        if ((k & 1) == 0) {
            const int P = M / 2 + (M & 1);  // passes over the array
            const int from = (P - k / 2) & 1;
            v.src = from ? S1 : U;
            v.dst = from ? U : S1;
            v.n = n;
            v.width = T << k;
            v.active = true;
            v.fan = k + 1 < M ? 4 : 2;
        }
        return v;
    }
    if (path == 6 /* SR_PATH_NEAR */ && k >= 1) {
        const bool to_s1 = (M & 1) == 0;  // slot 0 wrote S1
        S* X = to_s1 ? S1 : U;
        S* Y = to_s1 ? U : S1;
        uint32_t* PX = to_s1 ? PS1 : PU;
        uint32_t* PY = to_s1 ? PU : PS1;
        if (k == 1) {
            v.src = X + T;
            v.dst = Y + T;
            v.psrc = PX ? PX + T : nullptr;
            v.pdst = PY ? PY + T : nullptr;
            v.n = n - T;
            v.width = T;
            v.active = true;
            v.csrc = X;
            v.cdst = Y;
            v.cpsrc = PX;
            v.cpdst = PY;
            v.cn = T;
        } else if (k == 2 && !to_s1) {
            v.csrc = S1;
            v.cdst = U;
            v.cpsrc = PS1;
            v.cpdst = PU;
            v.cn = n;
        }
        return v;
    }
    if (path == 3 /* SR_PATH_GENERAL */ || path == 6 /* SR_PATH_NEAR: slot 0 */) {
        const int from = (M - k) & 1;
        v.src = from ? S1 : U;
        v.dst = from ? U : S1;
        v.psrc = from ? PS1 : PU;
        v.pdst = from ? PU : PS1;
        v.n = n;
        v.width = T << k;
        v.active = true;
    } else if (path == 2 /* SR_PATH_OUTLIER */ || path == 5 /* SR_PATH_FEW: slot P is its fill pass */) {
        const int64_t m = (int64_t)ctl->m;
        const int P = ctl->job_passes;
        S* X0 = S1 + (n - m);
        uint32_t* XP0 = PS1 != nullptr ? PS1 + (n - m) : nullptr;  // pairs: the outliers' indices
        if (k < P) {
            const int from = (P - k) & 1;
            v.src = from ? U : X0;
            v.dst = from ? X0 : U;
            v.psrc = from ? PU : XP0;
            v.pdst = from ? XP0 : PU;
            v.n = m;
            v.width = T << k;
            v.active = true;
        } else if (k == P && path == 2 && PS1 == nullptr) {  // keys; pairs place in slots P, P + 1
            v.src = S1;
            v.dst = U;
            v.n = n;
            v.width = n;
            v.split = n - m;
            v.active = true;
        }
    }
    return v;
}

template <class S>
__device__ __forceinline__ PassView<S> resolve_tile(const Ctl* ctl, S* U, S* S1, uint32_t* PU, uint32_t* PS1,
                                                    int64_t n, int M, bool fan4 = false) {
    // Every field is chosen as a scalar and the view built once at the end:
    // a view assembled field by field on different branches was kept in
    // scratch memory (a per-lane stack slot written on every launch).
    S* src = U;  // single tile (no plan): in place
    S* dst = U;
    const uint32_t* psrc = PU;
    uint32_t* pdst = PU;
    int64_t len = n;
    bool active = true;
    if (ctl != nullptr) {
        const int path = ctl->path;
        const bool general = path == 3 /* SR_PATH_GENERAL */ || path == 6 /* SR_PATH_NEAR */;
        const bool job = path == 2 /* SR_PATH_OUTLIER */ || path == 5 /* SR_PATH_FEW */;
        const int64_t m = job ? (int64_t)ctl->m : 0;
        const int P = job ? ctl->job_passes : 0;
        S* X0 = S1 + (n - m);
        // passes after the tile sort: M two-way, or M/2 four-way (+1 two-way)
        const bool odd = ((fan4 && path == 3 ? M / 2 + (M & 1) : M) & 1) != 0;
        uint32_t* XP0 = PS1 != nullptr ? PS1 + (n - m) : nullptr;  // pairs: the outliers' indices
        src = job ? X0 : U;
        dst = job ? ((P & 1) ? U : X0) : (odd ? S1 : U);
        psrc = job ? XP0 : PU;
        pdst = job ? ((P & 1) ? PU : XP0) : (odd ? PS1 : PU);
        len = job ? m : n;
        active = general || job;
    }
    PassView<S> v;
    v.src = src;
    v.dst = dst;
    v.psrc = psrc;
    v.pdst = pdst;
    v.n = len;
    v.width = 0;
    v.split = -1;
    v.active = active;
    v.csrc = nullptr;
    v.cdst = nullptr;
    v.cpsrc = nullptr;
    v.cpdst = nullptr;
    v.cn = 0;
    v.fan = 2;
    return v;
}

}  // namespace sr
