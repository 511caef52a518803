// sr_measure.hip -- presortedness measures of Sec. 2 on the device.
//
//  * Run(A): one plus the number of descents a_i > a_{i+1}; the ascents
//    a_i < a_{i+1} are counted beside it.
//  * Mono(A): the least number of contiguous pieces, each nondecreasing or
//    nonincreasing.  Cutting a piece only when the next element breaks its
//    direction is optimal (any part of a monotone piece is monotone), so
//    Mono is the result of a left-to-right scan with three states (piece
//    descending, undecided, ascending).  That scan is a finite transducer:
//    the effect of a stretch of neighbour comparisons is, for each entry
//    state, the exit state and the number of pieces opened.  These summaries
//    compose associatively, so each workgroup summarises a tile, and one
//    workgroup composes the tile summaries in order.
//  * Inv(A): the number of pairs i < j with a_i > a_j, counted by a
//    bottom-up merge sort of a copy (the classic divide-and-conquer count):
//    within runs of 16 keys, an odd-even transposition network, where every
//    exchange of neighbours removes exactly one inversion; then merge levels
//    of doubling width, where a key taken from the right run B while the
//    left run A still holds la - i keys adds la - i (the stable merge takes
//    A on ties, so every key left in A is strictly greater).
// Keys are compared through the codec of each dtype (sr_device.hpp), so the
// order is the one the sort uses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "sortrace.h"
#include "sr_internal.hpp"
#include "sr_kernels.hpp"

namespace sr {
namespace {

constexpr int kMeasWG = 256;
constexpr int kMonoPer = 16;                       // neighbour comparisons per thread
constexpr int64_t kMonoTile = kMeasWG * kMonoPer;  // per workgroup
constexpr int kMonoRedWG = 1024;
constexpr int kInvRun = 16;                        // keys per thread: base runs and merge outputs

// Scan state: 0 = piece nonincreasing (decided), 1 = undecided, 2 = piece
// nondecreasing (decided).  A comparison step is s = -1 (a_i > a_{i+1}),
// 0 (equal) or +1 (a_i < a_{i+1}).
struct Fsm {
    int o[3];                  // exit state for each entry state
    unsigned long long c[3];   // pieces opened for each entry state
};

__device__ __forceinline__ void fsm_identity(Fsm& f) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f.o[d] = d;
        f.c[d] = 0;
    }
}

__device__ __forceinline__ void fsm_step(Fsm& f, int s) {
    if (s == 0) return;
    const int dir = s + 1;  // 0 or 2
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (f.o[d] == 1) {
            f.o[d] = dir;          // an undecided piece takes the direction
        } else if (f.o[d] != dir) {
            f.o[d] = 1;            // the element opens a new, undecided piece
            f.c[d] += 1;
        }
    }
}

__device__ __forceinline__ int pick3(const int* v, int i) { return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]); }
__device__ __forceinline__ unsigned long long pick3(const unsigned long long* v, int i) {
    return i == 0 ? v[0] : (i == 1 ? v[1] : v[2]);
}

// a, then b
__device__ __forceinline__ Fsm fsm_then(const Fsm& a, const Fsm& b) {
    Fsm r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.o[d] = pick3(b.o, a.o[d]);
        r.c[d] = a.c[d] + pick3(b.c, a.o[d]);
    }
    return r;
}

// Ordered tree reduction of one Fsm per thread through LDS; thread 0 gets
// the composition in thread order.
template <int WG>
__device__ __forceinline__ Fsm fsm_block_reduce(Fsm f, int (*so)[WG], unsigned long long (*sc)[WG]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        so[d][t] = f.o[d];
        sc[d][t] = f.c[d];
    }
    for (int s = 1; s < WG; s <<= 1) {
        __syncthreads();
        if ((t & (2 * s - 1)) == 0) {
            Fsm a, b;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a.o[d] = so[d][t];
                a.c[d] = sc[d][t];
                b.o[d] = so[d][t + s];
                b.c[d] = sc[d][t + s];
            }
            const Fsm r = fsm_then(a, b);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                so[d][t] = r.o[d];
                sc[d][t] = r.c[d];
            }
        }
    }
    __syncthreads();
    Fsm r;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.o[d] = so[d][0];
        r.c[d] = sc[d][0];
    }
    return r;
}

// Tile summaries of the comparison steps i = 1 .. n-1 (a_{i-1} vs a_i), plus
// descents and ascents.  tiles: 4 words per tile (exit states packed in
// bytes, then the three piece counts, each <= kMonoTile).
template <class C>
__global__ __launch_bounds__(kMeasWG) void k_mono_tiles(const typename C::S* keys, int64_t n, uint4* tiles,
                                                        unsigned long long* counts) {
    using U = typename C::U;
    __shared__ int so[3][kMeasWG];
    __shared__ unsigned long long sc[3][kMeasWG];
    const int64_t first = 1 + (int64_t)blockIdx.x * kMonoTile + (int64_t)threadIdx.x * kMonoPer;
    Fsm f;
    fsm_identity(f);
    unsigned long long desc = 0, asc = 0;
    if (first < n) {
        U prev = C::enc(keys[first - 1]);
        const int64_t last = std::min<int64_t>(first + kMonoPer, n);
        for (int64_t i = first; i < last; ++i) {
            const U cur = C::enc(keys[i]);
            const int s = prev < cur ? 1 : (cur < prev ? -1 : 0);
            desc += s < 0 ? 1 : 0;
            asc += s > 0 ? 1 : 0;
            fsm_step(f, s);
            prev = cur;
        }
    }
    desc = wave_sum(desc);
    asc = wave_sum(asc);
    if (__lane_id() == 0) {
        if (desc) atomicAdd(&counts[0], desc);
        if (asc) atomicAdd(&counts[1], asc);
    }
    const Fsm r = fsm_block_reduce<kMeasWG>(f, so, sc);
    if (threadIdx.x == 0)
        tiles[blockIdx.x] = make_uint4((unsigned)r.o[0] | ((unsigned)r.o[1] << 8) | ((unsigned)r.o[2] << 16),
                                       (unsigned)r.c[0], (unsigned)r.c[1], (unsigned)r.c[2]);
}

// Composes the tile summaries in order; counts[2] = Mono(A) (n >= 2).
__global__ __launch_bounds__(kMonoRedWG) void k_mono_reduce(const uint4* tiles, int64_t ntiles,
                                                            unsigned long long* counts) {
    __shared__ int so[3][kMonoRedWG];
    __shared__ unsigned long long sc[3][kMonoRedWG];
    const int64_t per = (ntiles + kMonoRedWG - 1) / kMonoRedWG;
    const int64_t b = (int64_t)threadIdx.x * per, e = std::min<int64_t>(b + per, ntiles);
    Fsm f;
    fsm_identity(f);
    for (int64_t i = b; i < e; ++i) {
        const uint4 w = tiles[i];
        Fsm g;
        g.o[0] = (int)(w.x & 0xff);
        g.o[1] = (int)((w.x >> 8) & 0xff);
        g.o[2] = (int)((w.x >> 16) & 0xff);
        g.c[0] = w.y;
        g.c[1] = w.z;
        g.c[2] = w.w;
        f = fsm_then(f, g);
    }
    const Fsm r = fsm_block_reduce<kMonoRedWG>(f, so, sc);
    if (threadIdx.x == 0) counts[2] = 1 + r.c[1];  // the scan starts with one undecided piece
}

// Inversions inside runs of 16 keys: odd-even transposition sort of the
// run's codes (16 rounds sort 16 keys); every exchange removes one
// inversion.  The sorted codes go to `out`.  A short last run is padded
// with the largest code, which never exchanges (no key exceeds it).
template <class C>
__global__ __launch_bounds__(kMeasWG) void k_inv_base(const typename C::S* keys, int64_t n, typename C::U* out,
                                                      unsigned long long* counts) {
    using U = typename C::U;
    const int64_t b = ((int64_t)blockIdx.x * kMeasWG + threadIdx.x) * kInvRun;
    unsigned int c32 = 0;  // at most 120 per run
    if (b < n) {
        const int m = (int)std::min<int64_t>(kInvRun, n - b);
        U v[kInvRun];
#pragma unroll
        for (int k = 0; k < kInvRun; ++k) v[k] = k < m ? C::enc(keys[b + k]) : ~(U)0;
        auto cx = [&](int k) {
            const bool x = v[k] > v[k + 1];
            const U lo = x ? v[k + 1] : v[k], hi = x ? v[k] : v[k + 1];
            v[k] = lo;
            v[k + 1] = hi;
            c32 += x ? 1u : 0u;
        };
#pragma unroll 1
        for (int round = 0; round < kInvRun; round += 2) {  // an even and an odd round
#pragma unroll
            for (int k = 0; k + 1 < kInvRun; k += 2) cx(k);
#pragma unroll
            for (int k = 1; k + 1 < kInvRun; k += 2) cx(k);
        }
#pragma unroll
        for (int k = 0; k < kInvRun; ++k)
            if (k < m) out[b + k] = v[k];
    }
    unsigned long long c = wave_sum((unsigned long long)c32);
    if (__lane_id() == 0 && c) atomicAdd(&counts[3], c);
}

// One merge level: sorted runs of width w (the last one may be short) are
// merged in pairs; each thread writes 16 outputs of one pair (2w is a
// multiple of 16) and adds the inversions between the pair's runs that its
// B keys account for.
template <class U>
__global__ __launch_bounds__(kMeasWG) void k_inv_merge(const U* in, U* out, int64_t n, int64_t w,
                                                       unsigned long long* counts) {
    const int64_t o0 = ((int64_t)blockIdx.x * kMeasWG + threadIdx.x) * kInvRun;
    unsigned long long c = 0;
    if (o0 < n) {
        const int64_t base = o0 / (2 * w) * (2 * w);
        const int64_t la = std::min<int64_t>(w, n - base);
        const int64_t lb = std::max<int64_t>(0, std::min<int64_t>(w, n - base - w));
        const U* A = in + base;
        const U* B = A + la;
        const int64_t d = o0 - base;
        // co-rank: i = number of A keys among the pair's first d outputs
        int64_t lo = std::max<int64_t>(0, d - lb), hi = std::min<int64_t>(d, la);
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (A[mid] <= B[d - mid - 1]) lo = mid + 1;
            else hi = mid;
        }
        int64_t i = lo, j = d - lo;
        const int cnt = (int)std::min<int64_t>(kInvRun, la + lb - d);
        for (int k = 0; k < cnt; ++k) {
            if (j >= lb || (i < la && A[i] <= B[j])) {
                out[o0 + k] = A[i++];
            } else {
                out[o0 + k] = B[j++];
                c += (unsigned long long)(la - i);
            }
        }
    }
    c = wave_sum(c);
    if (__lane_id() == 0 && c) atomicAdd(&counts[3], c);
}

__global__ void k_zero4(unsigned long long* p) {
    if (threadIdx.x < 4) p[threadIdx.x] = 0;
}

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <class C>
sr_status measure_impl(const void* keys_v, int64_t n, bool want_inv, hipStream_t st, unsigned long long* host4) {
    using S = typename C::S;
    using U = typename C::U;
    const S* keys = static_cast<const S*>(keys_v);
    const int64_t ntiles = cdiv64(n - 1, kMonoTile);
    const size_t cnt_bytes = 256;
    const size_t tile_bytes = (size_t)ntiles * sizeof(uint4);
    const size_t code_bytes = want_inv ? ((size_t)n * sizeof(U) + 255) / 256 * 256 : 0;
    const size_t total = cnt_bytes + (tile_bytes + 255) / 256 * 256 + 2 * code_bytes;
    // scratch for this call only (a measure is not on the sort path)
    void* mem = nullptr;
    hipError_t e = hipMalloc(&mem, total);
    if (e != hipSuccess) return api_fail(SR_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    char* p = static_cast<char*>(mem);
    unsigned long long* counts = reinterpret_cast<unsigned long long*>(p);
    uint4* tiles = reinterpret_cast<uint4*>(p + cnt_bytes);
    U* x = reinterpret_cast<U*>(p + cnt_bytes + (tile_bytes + 255) / 256 * 256);
    U* y = reinterpret_cast<U*>(reinterpret_cast<char*>(x) + code_bytes);
    hipLaunchKernelGGL(k_zero4, dim3(1), dim3(64), 0, st, counts);
    hipLaunchKernelGGL(k_mono_tiles<C>, dim3((unsigned)ntiles), dim3(kMeasWG), 0, st, keys, n, tiles, counts);
    hipLaunchKernelGGL(k_mono_reduce, dim3(1), dim3(kMonoRedWG), 0, st, (const uint4*)tiles, ntiles, counts);
    if (want_inv) {
        const unsigned g = (unsigned)cdiv64(cdiv64(n, kInvRun), kMeasWG);
        hipLaunchKernelGGL(k_inv_base<C>, dim3(g), dim3(kMeasWG), 0, st, keys, n, x, counts);
        for (int64_t w = kInvRun; w < n; w *= 2) {
            hipLaunchKernelGGL(k_inv_merge<U>, dim3(g), dim3(kMeasWG), 0, st, (const U*)x, y, n, w, counts);
            std::swap(x, y);
        }
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host4, counts, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        // the stream may still use the scratch: keep it rather than free it under a running kernel
        return api_fail(SR_ERR_DEVICE, std::string("presortedness: ") + hipGetErrorString(e));
    }
    e = hipFree(mem);
    if (e != hipSuccess) return api_fail(SR_ERR_DEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    return SR_OK;
}

}  // namespace
}  // namespace sr

extern "C" {

sr_status sr_measure_presortedness(sr_dtype dt, const void* keys, size_t n, int32_t flags, sr_presortedness* out_host,
                                   void* stream) {
    using namespace sr;
    api_clear_error();
    sr_status s = api_check_keys(dt, keys, n);
    if (s != SR_OK) return s;
    if (!out_host) return api_fail(SR_ERR_INVALID_ARGUMENT, "out_host is NULL");
    if (flags & ~SR_MEASURE_INV) return api_fail(SR_ERR_INVALID_ARGUMENT, "unknown flag");
    const bool want_inv = (flags & SR_MEASURE_INV) != 0;
    std::memset(out_host, 0, sizeof(*out_host));
    out_host->run = (int64_t)std::min<size_t>(n, 1);
    out_host->mono = (int64_t)std::min<size_t>(n, 1);
    out_host->inv = want_inv ? 0 : -1;
    if (n <= 1) return SR_OK;
    unsigned long long h[4] = {0, 0, 0, 0};
    hipStream_t st = (hipStream_t)stream;
    switch (dt) {
    case SR_INT32: s = measure_impl<CodecI32>(keys, (int64_t)n, want_inv, st, h); break;
    case SR_FLOAT32: s = measure_impl<CodecF32>(keys, (int64_t)n, want_inv, st, h); break;
    case SR_UINT64: s = measure_impl<CodecU64>(keys, (int64_t)n, want_inv, st, h); break;
    }
    if (s != SR_OK) return s;
    out_host->descents = (int64_t)h[0];
    out_host->ascents = (int64_t)h[1];
    out_host->run = (int64_t)h[0] + 1;
    out_host->mono = (int64_t)h[2];
    if (want_inv) out_host->inv = (int64_t)h[3];
    return SR_OK;
}

}  // extern "C"
