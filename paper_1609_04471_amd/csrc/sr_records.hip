// sr_records.hip -- sorting heavy items: lists of int32 words (Sec. 2's
// random 16-, 64- and 256-integer lists), ordered word by word from the
// first, stable.
//
// A list is never moved while it is ordered.  Its first two words, each
// mapped to an order-preserving unsigned code, form a 64-bit prefix key that
// is sorted with the list's index as a stable payload (the pairs sort of
// this library).  Lists whose prefixes tie are then refined two words at a
// time: the tied positions are compacted, keyed by their next two words and
// sorted stably inside their tie groups (the segmented pairs sort), and the
// group boundaries are split where the new keys differ.  For random lists a
// 64-bit prefix almost never ties, so one pairs sort decides the order.  A
// final gather moves every list to its place.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "sortrace.h"
#include "sr_internal.hpp"
#include "sr_kernels.hpp"

namespace sr {
namespace {

constexpr int kRecWG = 256;
constexpr int kScanPer = 16;
constexpr int64_t kScanTile = (int64_t)kRecWG * kScanPer;  // flags per workgroup in the scans
constexpr int kScanTopWG = 1024;

__device__ __forceinline__ uint32_t code_i32(int32_t x) { return (uint32_t)x ^ 0x80000000u; }

// Prefix key of list r at words t, t+1 (the first word in the high half; a
// missing second word counts as the lowest code, the same for every list).
__device__ __forceinline__ uint64_t list_key(const int32_t* lists, int64_t r, int L, int t) {
    const int32_t* p = lists + r * (int64_t)L;
    const uint64_t hi = code_i32(p[t]);
    const uint64_t lo = t + 1 < L ? code_i32(p[t + 1]) : 0u;
    return hi << 32 | lo;
}

__global__ __launch_bounds__(kRecWG) void k_list_init(const int32_t* lists, int64_t n, int L, uint64_t* keys,
                                                      uint32_t* idx) {
    for (int64_t i = (int64_t)blockIdx.x * kRecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRecWG) {
        idx[i] = (uint32_t)i;
        keys[i] = list_key(lists, i, L, 0);
    }
}

// head[i] = 1 where a group of equal prefix keys starts.
__global__ __launch_bounds__(kRecWG) void k_list_heads(const uint64_t* keys, int64_t n, uint8_t* head) {
    for (int64_t i = (int64_t)blockIdx.x * kRecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRecWG)
        head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// tied[i] = 1 where i lies in a group of two or more lists.
__global__ __launch_bounds__(kRecWG) void k_list_tied(const uint8_t* head, int64_t n, uint8_t* tied) {
    for (int64_t i = (int64_t)blockIdx.x * kRecWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRecWG)
        tied[i] = (head[i] && (i + 1 == n || head[i + 1])) ? 0 : 1;
}

// Flags set per scan tile.
__global__ __launch_bounds__(kRecWG) void k_flag_count(const uint8_t* flags, int64_t n, uint32_t* bsum) {
    __shared__ unsigned long long ws[kRecWG / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    unsigned long long c = 0;
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t e = base + (int64_t)j * kRecWG + threadIdx.x;
        c += (e < n && flags[e]) ? 1 : 0;
    }
    c = wave_sum(c);
    if (__lane_id() == 0) ws[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kRecWG / kWave; ++w) t += ws[w];
        bsum[blockIdx.x] = (uint32_t)t;
    }
}

// Exclusive prefix of the nb tile counts (one workgroup); total[0] = sum.
__global__ __launch_bounds__(kScanTopWG) void k_flag_scan_top(const uint32_t* bsum, int64_t nb, uint32_t* bpre,
                                                              unsigned long long* total) {
    __shared__ unsigned long long part[kScanTopWG];
    const int64_t per = (nb + kScanTopWG - 1) / kScanTopWG;
    const int64_t b = (int64_t)threadIdx.x * per, e = std::min<int64_t>(b + per, nb);
    unsigned long long s = 0;
    for (int64_t i = b; i < e; ++i) s += bsum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (int t = 0; t < kScanTopWG; ++t) {
            const unsigned long long v = part[t];
            part[t] = run;
            run += v;
        }
        total[0] = run;
    }
    __syncthreads();
    unsigned long long run = part[threadIdx.x];
    for (int64_t i = b; i < e; ++i) {
        bpre[i] = (uint32_t)run;
        run += bsum[i];
    }
}

// Position of every set flag among the set flags, in index order: calls
// f(e, c) for each set flag e with its rank c.
template <class F>
__device__ __forceinline__ void for_each_flagged(const uint8_t* flags, int64_t n, const uint32_t* bpre, F&& f) {
    __shared__ uint32_t wt[kRecWG / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    const int wave = threadIdx.x / kWave, lane = __lane_id();
    uint32_t carry = bpre[blockIdx.x];
    for (int j = 0; j < kScanPer; ++j) {
        const int64_t e = base + (int64_t)j * kRecWG + threadIdx.x;
        const bool set = e < n && flags[e];
        const unsigned long long m = __ballot(set);
        const uint32_t below = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wt[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t off = carry, tot = 0;
        for (int w = 0; w < kRecWG / kWave; ++w) {
            off += w < wave ? wt[w] : 0u;
            tot += wt[w];
        }
        if (set) f(e, off + below);
        carry += tot;
        __syncthreads();
    }
}

// Compacts the tied positions: their list index, their key at words t, t+1,
// their position and whether they start a group.
__global__ __launch_bounds__(kRecWG) void k_list_compact(const uint8_t* tied, const uint8_t* head, const uint32_t* bpre,
                                                         int64_t n, const uint32_t* idx, const int32_t* lists, int L,
                                                         int t, uint64_t* ckey, uint32_t* cidx, int64_t* cpos,
                                                         uint8_t* gflag) {
    for_each_flagged(tied, n, bpre, [&](int64_t e, uint32_t c) {
        const uint32_t r = idx[e];
        cidx[c] = r;
        ckey[c] = list_key(lists, r, L, t);
        cpos[c] = e;
        gflag[c] = head[e];
    });
}

// Segment offsets of the compacted tie groups; off[ng] = cnt.
__global__ __launch_bounds__(kRecWG) void k_list_offsets(const uint8_t* gflag, int64_t cnt, const uint32_t* bpre,
                                                         int64_t* off, const unsigned long long* ng) {
    for_each_flagged(gflag, cnt, bpre, [&](int64_t e, uint32_t c) { off[c] = e; });
    if (blockIdx.x == 0 && threadIdx.x == 0) off[ng[0]] = cnt;
}

// Writes the refined order back and splits groups where the new keys differ.
__global__ __launch_bounds__(kRecWG) void k_list_scatter(const uint64_t* ckey, const uint32_t* cidx,
                                                         const int64_t* cpos, const uint8_t* gflag, int64_t cnt,
                                                         uint32_t* idx, uint8_t* head) {
    for (int64_t c = (int64_t)blockIdx.x * kRecWG + threadIdx.x; c < cnt; c += (int64_t)gridDim.x * kRecWG) {
        const int64_t e = cpos[c];
        idx[e] = cidx[c];
        if (!gflag[c] && ckey[c] != ckey[c - 1]) head[e] = 1;
    }
}

// dst list i = src list idx[i], one word per thread.
__global__ __launch_bounds__(kRecWG) void k_list_gather(const int32_t* src, int32_t* dst, const uint32_t* idx,
                                                        int64_t n, int L) {
    const int64_t total = n * (int64_t)L;
    for (int64_t w = (int64_t)blockIdx.x * kRecWG + threadIdx.x; w < total; w += (int64_t)gridDim.x * kRecWG) {
        const int64_t i = w / L, j = w - i * L;
        dst[w] = src[(int64_t)idx[i] * L + j];
    }
}

int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv64(work, kRecWG), 65536)); }

struct Scratch {
    void* mem = nullptr;
    ~Scratch() {
        if (mem) (void)hipFree(mem);
    }
};

sr_status dev_fail(hipError_t e, const char* what) {
    return api_fail(SR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace
}  // namespace sr

extern "C" {

sr_status sr_sort_lists(int32_t* lists, size_t n_, int32_t words, void* stream) {
    using namespace sr;
    api_clear_error();
    if (words < 1 || words > (1 << 20)) return api_fail(SR_ERR_INVALID_ARGUMENT, "words is 1 .. 2^20");
    if (n_ > 0xFFFFFFFFull) return api_fail(SR_ERR_INVALID_ARGUMENT, "n above 2^32 - 1");
    if (n_ > 1 && lists == nullptr) return api_fail(SR_ERR_INVALID_ARGUMENT, "lists is NULL");
    if (lists && ((uintptr_t)lists % 4) != 0) return api_fail(SR_ERR_INVALID_ARGUMENT, "lists not 4-byte aligned");
    if (n_ <= 1) return SR_OK;
    const int64_t n = (int64_t)n_;
    const int L = words;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nb = cdiv64(n, kScanTile);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t o_keys = 0;
    const size_t o_idx = o_keys + al(8 * (size_t)n);
    const size_t o_head = o_idx + al(4 * (size_t)n);
    const size_t o_tied = o_head + al((size_t)n);
    const size_t o_bsum = o_tied + al((size_t)n);
    const size_t o_bpre = o_bsum + al(4 * (size_t)nb);
    const size_t o_tot = o_bpre + al(4 * (size_t)nb);
    const size_t o_ckey = o_tot + 256;
    const size_t o_cidx = o_ckey + al(8 * (size_t)n);
    const size_t o_cpos = o_cidx + al(4 * (size_t)n);
    const size_t o_gflag = o_cpos + al(8 * (size_t)n);
    const size_t o_coff = o_gflag + al((size_t)n);
    const size_t o_copy = o_coff + al(8 * ((size_t)n + 1));
    const size_t total_bytes = o_copy + al(4 * (size_t)n * (size_t)L);
    Scratch sc;
    hipError_t e = hipMalloc(&sc.mem, total_bytes);
    if (e != hipSuccess) return api_fail(SR_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    char* base = static_cast<char*>(sc.mem);
    uint64_t* keys = reinterpret_cast<uint64_t*>(base + o_keys);
    uint32_t* idx = reinterpret_cast<uint32_t*>(base + o_idx);
    uint8_t* head = reinterpret_cast<uint8_t*>(base + o_head);
    uint8_t* tied = reinterpret_cast<uint8_t*>(base + o_tied);
    uint32_t* bsum = reinterpret_cast<uint32_t*>(base + o_bsum);
    uint32_t* bpre = reinterpret_cast<uint32_t*>(base + o_bpre);
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(base + o_tot);
    uint64_t* ckey = reinterpret_cast<uint64_t*>(base + o_ckey);
    uint32_t* cidx = reinterpret_cast<uint32_t*>(base + o_cidx);
    int64_t* cpos = reinterpret_cast<int64_t*>(base + o_cpos);
    uint8_t* gflag = reinterpret_cast<uint8_t*>(base + o_gflag);
    int64_t* coff = reinterpret_cast<int64_t*>(base + o_coff);
    int32_t* copy = reinterpret_cast<int32_t*>(base + o_copy);

    hipLaunchKernelGGL(k_list_init, dim3(grid_for(n)), dim3(kRecWG), 0, st, (const int32_t*)lists, n, L, keys, idx);
    if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "list keys");
    sr_status s = sr_sort_pairs(SR_UINT64, keys, idx, (size_t)n, stream);
    if (s != SR_OK) return s;
    hipLaunchKernelGGL(k_list_heads, dim3(grid_for(n)), dim3(kRecWG), 0, st, (const uint64_t*)keys, n, head);
    for (int t = 2; t < L; t += 2) {
        // tied positions and their count
        hipLaunchKernelGGL(k_list_tied, dim3(grid_for(n)), dim3(kRecWG), 0, st, (const uint8_t*)head, n, tied);
        hipLaunchKernelGGL(k_flag_count, dim3((unsigned)nb), dim3(kRecWG), 0, st, (const uint8_t*)tied, n, bsum);
        hipLaunchKernelGGL(k_flag_scan_top, dim3(1), dim3(kScanTopWG), 0, st, (const uint32_t*)bsum, nb, bpre, tot);
        unsigned long long h = 0;
        if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "list ties");
        if ((e = hipMemcpyAsync(&h, tot, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return dev_fail(e, "copy");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail(e, "list ties");
        if (h == 0) break;
        const int64_t cnt = (int64_t)h;
        hipLaunchKernelGGL(k_list_compact, dim3((unsigned)nb), dim3(kRecWG), 0, st, (const uint8_t*)tied,
                           (const uint8_t*)head, (const uint32_t*)bpre, n, (const uint32_t*)idx,
                           (const int32_t*)lists, L, t, ckey, cidx, cpos, gflag);
        // group offsets among the compacted positions
        const int64_t cb = cdiv64(cnt, kScanTile);
        hipLaunchKernelGGL(k_flag_count, dim3((unsigned)cb), dim3(kRecWG), 0, st, (const uint8_t*)gflag, cnt, bsum);
        hipLaunchKernelGGL(k_flag_scan_top, dim3(1), dim3(kScanTopWG), 0, st, (const uint32_t*)bsum, cb, bpre,
                           tot + 1);
        hipLaunchKernelGGL(k_list_offsets, dim3((unsigned)cb), dim3(kRecWG), 0, st, (const uint8_t*)gflag, cnt,
                           (const uint32_t*)bpre, coff, (const unsigned long long*)(tot + 1));
        unsigned long long ng = 0;
        if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "list groups");
        if ((e = hipMemcpyAsync(&ng, tot + 1, 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return dev_fail(e, "copy");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail(e, "list groups");
        s = sr_sort_segmented(SR_UINT64, ckey, cidx, (size_t)cnt, coff, (size_t)ng, stream);
        if (s != SR_OK) return s;
        hipLaunchKernelGGL(k_list_scatter, dim3(grid_for(cnt)), dim3(kRecWG), 0, st, (const uint64_t*)ckey,
                           (const uint32_t*)cidx, (const int64_t*)cpos, (const uint8_t*)gflag, cnt, idx, head);
    }
    if ((e = hipMemcpyAsync(copy, lists, 4 * (size_t)n * (size_t)L, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return dev_fail(e, "list copy");
    hipLaunchKernelGGL(k_list_gather, dim3(grid_for(n * L)), dim3(kRecWG), 0, st, (const int32_t*)copy, lists,
                       (const uint32_t*)idx, n, L);
    if ((e = hipGetLastError()) != hipSuccess) return dev_fail(e, "list gather");
    // the scratch is freed on return: wait until the stream is done with it
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return dev_fail(e, "list gather");
    return SR_OK;
}

}  // extern "C"
