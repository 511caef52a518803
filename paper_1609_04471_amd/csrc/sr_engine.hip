// sr_engine.hip -- kernels, host orchestration and the C ABI of libsortrace.
//
// Launch sequence of sr_sort_keys / sr_sort_pairs for n above one tile, all on
// the caller's stream and with no device-to-host traffic:
//   probe      reads the keys once (early exit once the array is known to be
//              mixed), counts ascents/descents, samples the descent rate; its
//              last workgroup writes the plan into the device control block.
//              This is the sortedness test the paper makes indispensable for
//              quicksort (Sec. 4 (f)) and the run scan of natural mergesort
//              (Sec. 1, process 1), for the whole array at once.
//   reverse    (+ regroup for pairs) only if the plan says REVERSED: a
//              nonincreasing array is one descending run, reversed in place
//              (Sec. 3 (a)); for pairs equal-key groups are reversed back, the
//              paper's "reversed twice".
//   outlier    only if the plan says OUTLIER (nearly sorted input).
//   tile_sort  + merge x M only if the plan says GENERAL.
// Kernels whose path was not chosen return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "sortrace.h"
#include "sr_kernels.hpp"

namespace sr {

// ------------------------------------------------------------- tuning
// Tile sort: WG x IT keys per workgroup; merge: WG x IT outputs per workgroup.
template <class C, bool PAIRS>
struct Tune;
template <bool PAIRS>
struct Tune32 {
    static constexpr int TWG = PAIRS ? 256 : 512, TIT = 16;
    static constexpr int MWG = 256, MIT = 16;
};
template <bool PAIRS>
struct Tune64 {
    // 4096-key tiles either way (whole run-scan tiles, so pairs can take the
    // run path too); pairs hold 8 keys per thread in registers
    static constexpr int TWG = PAIRS ? 512 : 256, TIT = PAIRS ? 8 : 16;
    static constexpr int MWG = 256, MIT = 8;
};
template <bool PAIRS>
struct Tune<CodecI32, PAIRS> : Tune32<PAIRS> {};
template <bool PAIRS>
struct Tune<CodecF32, PAIRS> : Tune32<PAIRS> {};
template <bool PAIRS>
struct Tune<CodecU64, PAIRS> : Tune64<PAIRS> {};

constexpr int kProbeWG = 256;
constexpr int64_t kProbeTile = 8192;   // keys per probe workgroup
constexpr int kProbeSample = 256;      // neighbour pairs sampled per probe workgroup
constexpr int kSampleField = 21;       // bits per sampled count in a packed sum
constexpr int kAscBits = 40;           // ascent count below the sampled deep drops in one word
constexpr int64_t kDropDepth = 16;     // a deep drop's overlap reaches at least this far
constexpr unsigned long long kSampleMask = (1ull << kSampleField) - 1;
constexpr int kRevWG = 256;
constexpr int64_t kProbeMaxGrid = 1024; // probe workgroups (grid-stride over its tiles)
static_assert(kProbeSample * kProbeMaxGrid < (1 << kSampleField), "packed sample sums fit");
static_assert(kProbeSample * kProbeMaxGrid < (1ll << (64 - kAscBits)), "sampled deep drops fit above the ascents");
constexpr unsigned int kProbeGroup = 32;  // probe workgroups per first-level ticket counter

__device__ __forceinline__ bool path_is(const Ctl* ctl, int want) {
    return ctl == nullptr || ctl->path == want;
}

// Outlier-path tile geometry (used by the RUNS job too).
constexpr int kClsWG = 256;
constexpr int kClsPer = 17;
constexpr int kClsW = kClsWG * kClsPer;  // 4352-key window
constexpr int kClsTC = 4096;             // core keys per tile
constexpr int kClsH = (kClsW - kClsTC) / 2;
constexpr int kClsMaxIter = 10;  // more rounds: not outlier-shaped (falls back)
constexpr int kClsDeepIter = 5;  // from this round on, an unrepairable descent ends the rounds

__device__ __forceinline__ int ceil_log2_dev(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) ++r;
    return r;
}

constexpr int kVerWG = 1024;
constexpr int kVerQ = 8;  // consecutive tiles per verify thread per round
constexpr int64_t kVerRound = (int64_t)kVerWG * kVerQ;

// Slot of tile t's summary words (kept count, first and last kept key).
// k_verify reads them in rounds of kVerRound tiles, thread i taking kVerQ
// consecutive tiles; keeping tile r0 + i * kVerQ + q at r0 + q * kVerWG + i
// makes each of those loads one coalesced row.  The arrays hold whole rounds.
__device__ __forceinline__ int64_t ver_slot(int64_t t) {
    const int64_t r0 = t / kVerRound * kVerRound, o = t - r0;
    return r0 + (o % kVerQ) * kVerWG + o / kVerQ;
}

// ------------------------------------------------------------ natural runs
// RUNS job: the natural runs of natural mergesort (Sec. 3) found in parallel,
// descending ones reversed in place, and a merge tree over the resulting
// sorted leaves, so presorted input skips most merge passes.  The measure it
// exploits is Mono (Sec. 2): the fewest monotone pieces of the array.
//
// Pair i is (key i, key i+1); it is strict when the two keys differ.  A
// turning is a strict pair i whose nearest earlier strict pair j points the
// other way; the keys j+1 .. i between them (equal keys) form its block, the
// peak or valley.  Every turning places one run boundary inside its block:
// the block joins the descending side (boundary at j+1 for a peak, at i+1 for
// a valley) unless that descending stretch is a single strict pair, which is
// then dropped instead (boundary at i+1 for the peak, j+1 for the valley --
// the same position).  Equal positions are kept once.  Each run then holds
// strict pairs of one direction only, so it is monotone; the count matches
// Mono on the teeth classes of Sec. 2, and on k-sharp teeth every descending
// section becomes one run whose reversal continues its neighbours.
//
// Launch order (the same fixed launches as the outlier path):
//   classify  per 4096-key tile: heads (at most kRunHeads, else the tile is
//             dense), first/last strict direction, min and max (runscan_lds)
//   verify    one workgroup: carries across tiles, the head list, singleton
//             joins, dense tiles as sorted pieces, in-order joins of adjacent
//             leaves (max of one <= min of the next), merge-tree pass count
//             and per-pass chunk prefixes; keeps RUNS only when it is cheaper
//             than the other paths (run_plan)
//   scatter   reverses the descending runs in place (runs_reverse)
//   tile sort sorts the dense pieces in place
//   merges    pass k merges leaf groups of 2^(k+1) leaves; one extra copy
//             pass when the pass count is odd lands the result in U
constexpr int kRunHeads = 8;           // turnings recorded per 4096-key tile; more: dense
constexpr int kRunMaxBase = 4096;      // runs and dense pieces a plan may hold
constexpr int kRunMaxLeaves = 2048;    // merge leaves after in-order joins
constexpr int kRunMaxPasses = 16;
constexpr int kRevPairs = 2048;        // key pairs swapped per reversal work unit
constexpr int kRevPer = kRevPairs / kClsWG;

struct RunTile {
    int nh;                         // turnings recorded, or -1: dense tile
    int fz;                         // tile-relative index of the first strict pair, -1 if none
    int lz;                         // tile-relative index of the last strict pair, -1 if none
    int signs;                      // bit 0: first strict pair descends; bit 1: last one does
    int heads[kRunHeads];           // turnings (i << 13 | j << 1 | descending), tile-relative i, j
    unsigned long long vmin, vmax;  // encoded extremes of the tile's keys
};
static_assert(sizeof(RunTile) == 64, "run descriptor is one 64-byte record");

// Plan of a RUNS sort.  Entries and boundaries pack a position with its kind
// in the top byte: 0 array start, 1 run boundary of a turning, 2 dense piece
// start, 3 end of a dense piece; entries use 4 for a valley and 5 for a peak
// (position i, with j in ent_j).
struct RunArea {
    long long L;        // merge leaves
    long long nbase;    // runs and dense pieces
    long long ndesc;    // descending runs
    long long nrev;     // reversal work units
    int npasses;        // merge passes (P, plus one copy pass when P is odd)
    int P;
    int pad0, pad1;
    long long pbase[kRunMaxPasses];    // pass k: its chunk prefix starts at pre[pbase[k]]
    long long ptotal[kRunMaxPasses];   // pass k: chunks
    long long lb[kRunMaxLeaves + 1];   // merge leaf starts, lb[L] = n
    long long pre[2 * kRunMaxLeaves + 2 * kRunMaxPasses];
    long long ent[kRunMaxBase + 2];    // turnings and dense markers in array order
    long long ent_j[kRunMaxBase + 2];
    long long bs[kRunMaxBase + 2];     // leaf boundaries
    unsigned long long bmin[kRunMaxBase], bmax[kRunMaxBase];
    long long ds[kRunMaxBase], de[kRunMaxBase];  // descending runs [ds, de)
    long long dpre[kRunMaxBase + 1];             // reversal units before descending run i
};

constexpr long long kPosMask = (1LL << 56) - 1;
__device__ __forceinline__ long long bpos(long long b) { return b & kPosMask; }
__device__ __forceinline__ int bkind(long long b) { return (int)(b >> 56); }

// Latest nonzero value among lanes 0..lane (0 if none): a scan with the
// associative "later nonzero wins".
__device__ __forceinline__ int wave_last_nonzero(int x) {
    const int lane = (int)__lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o && x == 0) x = y;
    }
    return x;
}

// Exclusive prefix of v over the workgroup's threads in order, and the total.
// s_w holds one value per wavefront.
__device__ __forceinline__ long long wg_scan_excl(long long v, long long* s_w, long long& total) {
    const int lane = (int)__lane_id();
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    long long x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) s_w[wave] = x;
    __syncthreads();
    long long pre = x - v, tot = 0;
    for (int q = 0; q < nw; ++q) {
        if (q < wave) pre += s_w[q];
        tot += s_w[q];
    }
    total = tot;
    return pre;
}

// Run descriptor of the 4096-key tile [c0, c1) from its window in LDS (sk[0]
// is key w0; the window reaches key c1 when c1 < n).  Every thread of the
// 256-thread workgroup takes 16 consecutive pairs.  A pair's previous strict
// pair comes from a max-scan of ((index + 1) << 1 | descending); the tile's
// first strict pair has its previous one in an earlier tile, so the plan
// decides whether it turns.
template <class U>
__device__ void runscan_lds(const U* sk, int64_t n, int64_t c0, int64_t c1, int64_t w0, RunTile* out) {
    constexpr int PER = kClsTC / kClsWG;
    constexpr int NW = kClsWG / kWave;
    __shared__ int s_last[NW], s_cnt[NW], s_first;
    __shared__ U s_mn[NW], s_mx[NW];
    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid / kWave;
    if (tid == 0) s_first = -1;
    const int64_t qend = c1 < n - 1 ? c1 : n - 1;  // pairs of this tile: [c0, qend)
    const int b0 = tid * PER;
    // bit r: pair b0 + r is strict / descending
    unsigned int strict = 0u, descm = 0u;
    U mn = ~(U)0, mx = 0;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int64_t q = c0 + b0 + r;
        if (q < c1) {
            const U a = sk[q - w0];
            mn = a < mn ? a : mn;
            mx = a > mx ? a : mx;
            if (q < qend) {
                const U b = sk[q - w0 + 1];
                strict |= (a != b ? 1u : 0u) << r;
                descm |= (a > b ? 1u : 0u) << r;
            }
        }
    }
    const int rl = 31 - __builtin_clz(strict | 1u);  // last strict pair (valid when strict != 0)
    const int lastv = strict ? ((b0 + rl + 1) << 1) | (int)((descm >> rl) & 1u) : 0;
    const int rf = __builtin_ctz(strict | 0x80000000u);
    const int firstv = strict ? ((b0 + rf + 1) << 1) | (int)((descm >> rf) & 1u) : 0;
    int incl = lastv;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl = y > incl ? y : incl;
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) {
        const U x = __shfl_xor(mn, o), y = __shfl_xor(mx, o);
        mn = x < mn ? x : mn;
        mx = y > mx ? y : mx;
    }
    if (lane == kWave - 1) s_last[wave] = incl;
    if (lane == 0) {
        s_mn[wave] = mn;
        s_mx[wave] = mx;
    }
    __syncthreads();
    int in = __shfl_up(incl, 1);
    if (lane == 0) in = 0;
    for (int w = 0; w < wave; ++w) in = s_last[w] > in ? s_last[w] : in;
    if (in == 0 && firstv != 0) s_first = firstv;  // the tile's first strict pair
    // turnings: strict pairs whose previous strict pair has the other direction
    int cnt = 0;
    {
        int pd = in == 0 ? -1 : (in & 1);
        for (unsigned int m = strict; m != 0u; m &= m - 1u) {
            const int r = __builtin_ctz(m);
            const int dd = (int)((descm >> r) & 1u);
            if (pd >= 0 && pd != dd) ++cnt;
            pd = dd;
        }
    }
    int xc = cnt;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(xc, o);
        if (lane >= o) xc += y;
    }
    if (lane == kWave - 1) s_cnt[wave] = xc;
    __syncthreads();
    int total = 0, hpre = xc - cnt;
    for (int w = 0; w < NW; ++w) {
        total += s_cnt[w];
        if (w < wave) hpre += s_cnt[w];
    }
    if (total <= kRunHeads && cnt > 0) {
        int pv = in;  // previous strict pair as ((index + 1) << 1 | descending)
        for (unsigned int m = strict; m != 0u; m &= m - 1u) {
            const int r = __builtin_ctz(m);
            const int dd = (int)((descm >> r) & 1u);
            if (pv != 0 && (pv & 1) != dd) out->heads[hpre++] = ((b0 + r) << 13) | (((pv >> 1) - 1) << 1) | dd;
            pv = ((b0 + r + 1) << 1) | dd;
        }
    }
    if (tid == 0) {
        int lv = 0;
        U tmn = s_mn[0], tmx = s_mx[0];
        for (int w = 0; w < NW; ++w) {
            lv = s_last[w] > lv ? s_last[w] : lv;
            tmn = s_mn[w] < tmn ? s_mn[w] : tmn;
            tmx = s_mx[w] > tmx ? s_mx[w] : tmx;
        }
        const int fv = s_first;
        out->nh = total <= kRunHeads ? total : -1;
        out->fz = fv > 0 ? (fv >> 1) - 1 : -1;
        out->lz = lv > 0 ? (lv >> 1) - 1 : -1;
        out->signs = (fv & 1) | ((lv & 1) << 1);
        out->vmin = (unsigned long long)tmn;
        out->vmax = (unsigned long long)tmx;
    }
}

// Plan of the RUNS job (one workgroup of kVerWG threads).  ocost is the
// remaining cost of the outlier job in pass-equivalents (huge if none);
// was_runs: the probe chose RUNS, so a rejected plan falls back to GENERAL.
// g = tile-sort tile / 4096 (1 or 2): a dense piece is the dense 4096-key
// tiles of one tile-sort tile.  CH = outputs per merge chunk of the merge
// launches; M = merge launches enqueued.
template <class C>
__device__ void run_plan(Ctl* ctl, int64_t n, int64_t ntiles, const typename C::S* keys, const RunTile* rd,
                         RunArea* ra, int g, int64_t CH, int M, double ocost, bool was_runs) {
    constexpr int NT = kVerWG;
    constexpr int64_t TC = kClsTC;
    __shared__ long long s_w[NT / kWave];
    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid / kWave;
    auto reject = [&]() {
        if (tid == 0 && was_runs) ctl->path = SR_PATH_GENERAL;
    };

    // A. entries in array order, in rounds of NT tiles (one tile per thread,
    //    coalesced 16-byte descriptor heads): each tile's turnings -- the
    //    first one against the last strict pair of earlier tiles, carried by a
    //    max-scan of ((index + 1) << 1 | descending) -- and the dense piece
    //    starts and ends, written at the running offset (a scan of per-tile
    //    counts).  Stops as soon as the entries or the dense keys exceed what
    //    a plan may hold.
    __shared__ long long s_carry, s_base, s_dk;
    __shared__ int s_nh[NT + 1];
    if (tid == 0) {
        s_carry = 0;
        s_base = 0;
        s_dk = 0;
    }
    __syncthreads();
    for (int64_t r0 = 0; r0 < ntiles; r0 += NT) {
        const int64_t t = r0 + tid;
        const bool have = t < ntiles;
        const int4 hd = have ? *reinterpret_cast<const int4*>(rd + t) : make_int4(0, -1, -1, 0);
        const int nh = hd.x, fz = hd.y, lz = hd.z, signs = hd.w;  // RunTile's first four fields
        s_nh[tid + 1] = nh;
        if (tid == 0) s_nh[0] = r0 > 0 ? rd[r0 - 1].nh : 0;
        const long long lv = (have && lz >= 0) ? ((((long long)(t * TC + lz)) + 1) << 1) | ((signs >> 1) & 1) : 0;
        long long incl = lv;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const long long y = __shfl_up(incl, o);
            if (lane >= o) incl = y > incl ? y : incl;
        }
        if (lane == kWave - 1) s_w[wave] = incl;
        __syncthreads();
        long long carry = __shfl_up(incl, 1);
        if (lane == 0) carry = 0;
        long long rmax = 0;
        for (int w = 0; w < NT / kWave; ++w) {
            if (w < wave) carry = s_w[w] > carry ? s_w[w] : carry;
            rmax = s_w[w] > rmax ? s_w[w] : rmax;
        }
        carry = s_carry > carry ? s_carry : carry;
        const bool pdense = t > 0 && s_nh[tid] < 0;
        int cnt = 0;
        long long dk = 0;
        bool carry_turn = false;
        if (have) {
            const int64_t st = t * TC;
            if (nh < 0) {
                if (t > 0 && ((t % g) == 0 || !pdense)) ++cnt;
                dk = ((st + TC) < n ? (st + TC) : n) - st;
            } else {
                if (pdense) ++cnt;
                if (fz >= 0 && carry != 0) {
                    const int cs = (carry & 1) ? -1 : 1, fs = (signs & 1) ? -1 : 1;
                    carry_turn = cs == -fs;
                    if (carry_turn) ++cnt;
                }
                cnt += nh;
            }
        }
        long long tot, dtot;
        long long o = s_base + wg_scan_excl(cnt, s_w, tot);
        (void)wg_scan_excl(dk, s_w, dtot);
        if (s_base + tot + 1 > kRunMaxBase || 2 * (s_dk + dtot) > n) {  // leaves = entries + 1
            reject();
            return;
        }
        if (have) {
            const int64_t st = t * TC;
            auto put = [&](long long pos, long long kind, long long j) {
                ra->ent[o] = pos | (kind << 56);
                ra->ent_j[o] = j;
                ++o;
            };
            if (nh < 0) {
                if (t > 0 && ((t % g) == 0 || !pdense)) put(st, 2, 0);
            } else {
                if (pdense) put(st, 3, 0);
                if (carry_turn) put(st + fz, (signs & 1) ? 5 : 4, (carry >> 1) - 1);
                for (int h = 0; h < nh; ++h) {
                    const int v = rd[t].heads[h];
                    put(st + (v >> 13), (v & 1) ? 5 : 4, st + ((v >> 1) & 0xFFF));
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            s_carry = rmax > s_carry ? rmax : s_carry;
            s_base += tot;
            s_dk += dtot;
        }
        __syncthreads();
    }
    const long long dense_keys = s_dk;
    if (tid == 0) ra->nbase = s_base;  // entries, for now
    __syncthreads();

    // B. leaf boundaries: dense markers, and the boundary of each turning
    //    (valley 4 at i+1 unless the descending stretch before it is a single
    //    pair, then j+1; peak 5 at j+1 unless the descending stretch after it
    //    is a single pair, then i+1), once per position; a turning whose
    //    boundary falls on or inside an adjacent dense piece adds none.
    {
        const long long ne = ra->nbase;
        auto tpos = [&](long long m) -> long long {
            const long long e = ra->ent[m];
            const long long i = bpos(e), j = ra->ent_j[m];
            long long p;
            if (bkind(e) == 5) {
                const bool single = m + 1 < ne && bkind(ra->ent[m + 1]) >= 4 && ra->ent_j[m + 1] == i;
                p = single ? i + 1 : j + 1;
            } else {
                const bool single = m > 0 && bkind(ra->ent[m - 1]) >= 4 && bpos(ra->ent[m - 1]) == j;
                p = single ? j + 1 : i + 1;
            }
            if (m > 0 && bkind(ra->ent[m - 1]) == 3 && p <= bpos(ra->ent[m - 1])) return -1;
            if (m + 1 < ne && bkind(ra->ent[m + 1]) == 2 && p >= bpos(ra->ent[m + 1])) return -1;
            return p;
        };
        auto boundary = [&](long long m) -> long long {  // packed boundary, or -1
            const long long e = ra->ent[m];
            if (bkind(e) < 4) return e;
            const long long p = tpos(m);
            if (p < 0) return -1;
            if (m > 0 && bkind(ra->ent[m - 1]) >= 4 && tpos(m - 1) == p) return -1;
            return p | (1LL << 56);
        };
        const long long pb = (ne + NT - 1) / NT;
        const long long i0 = (long long)tid * pb < ne ? (long long)tid * pb : ne;
        const long long i1 = (i0 + pb) < ne ? (i0 + pb) : ne;
        long long k = 0;
        for (long long m = i0; m < i1; ++m) k += boundary(m) >= 0 ? 1 : 0;
        long long tot;
        long long o = 1 + wg_scan_excl(k, s_w, tot);
        for (long long m = i0; m < i1; ++m) {
            const long long b = boundary(m);
            if (b >= 0) ra->bs[o++] = b;
        }
        if (tid == 0) {
            ra->bs[0] = (long long)(rd[0].nh < 0 ? 2 : 0) << 56;
            ra->bs[tot + 1] = n;
            ra->nbase = tot + 1;
        }
    }
    __syncthreads();

    // C. extremes of every leaf, descending runs and their reversal units
    const long long nl = ra->nbase;
    const long long pl = (nl + NT - 1) / NT;
    const long long l0 = (long long)tid * pl < nl ? (long long)tid * pl : nl;
    const long long l1 = (l0 + pl) < nl ? (l0 + pl) : nl;
    long long desc_keys = 0;
    {
        long long nd = 0, units = 0;
        for (long long i = l0; i < l1; ++i) {
            const long long b = ra->bs[i];
            const long long s = bpos(b), e = bpos(ra->bs[i + 1]);
            unsigned long long mn = ~0ull, mx = 0ull;
            if (bkind(b) == 2) {
                for (long long t = s / TC; t * TC < e; ++t) {
                    mn = rd[t].vmin < mn ? rd[t].vmin : mn;
                    mx = rd[t].vmax > mx ? rd[t].vmax : mx;
                }
            } else if (e > s) {
                const unsigned long long a = (unsigned long long)C::enc(keys[s]);
                const unsigned long long z = (unsigned long long)C::enc(keys[e - 1]);
                mn = a < z ? a : z;
                mx = a < z ? z : a;
                if (a > z) {
                    ++nd;
                    units += ((e - s) / 2 + kRevPairs - 1) / kRevPairs;
                    desc_keys += e - s;
                }
            }
            ra->bmin[i] = mn;
            ra->bmax[i] = mx;
        }
        long long tnd, tun, tdk;
        long long od = wg_scan_excl(nd, s_w, tnd);
        long long ou = wg_scan_excl(units, s_w, tun);
        (void)wg_scan_excl(desc_keys, s_w, tdk);
        desc_keys = tdk;
        for (long long i = l0; i < l1; ++i) {
            const long long b = ra->bs[i];
            if (bkind(b) == 2) continue;
            const long long s = bpos(b), e = bpos(ra->bs[i + 1]);
            if (e <= s) continue;
            const unsigned long long a = (unsigned long long)C::enc(keys[s]);
            const unsigned long long z = (unsigned long long)C::enc(keys[e - 1]);
            if (a > z) {
                ra->ds[od] = s;
                ra->de[od] = e;
                ra->dpre[od] = ou;
                ++od;
                ou += ((e - s) / 2 + kRevPairs - 1) / kRevPairs;
            }
        }
        if (tid == 0) {
            ra->ndesc = tnd;
            ra->nrev = tun;
            ra->dpre[tnd] = tun;
        }
    }
    __syncthreads();

    // D. in-order joins: leaf i continues leaf i-1 when max(i-1) <= min(i)
    {
        auto starts = [&](long long i) { return i == 0 || ra->bmax[i - 1] > ra->bmin[i]; };
        long long k = 0;
        for (long long i = l0; i < l1; ++i) k += starts(i) ? 1 : 0;
        long long L;
        long long o = wg_scan_excl(k, s_w, L);
        if (L > kRunMaxLeaves) {
            reject();
            return;
        }
        for (long long i = l0; i < l1; ++i)
            if (starts(i)) ra->lb[o++] = bpos(ra->bs[i]);
        if (tid == 0) {
            ra->lb[L] = n;
            ra->L = L;
        }
    }
    __syncthreads();
    const long long L = ra->L;
    const int P = ceil_log2_dev(L);
    const int np = P + (P & 1);
    const double rcost = (double)(desc_keys + dense_keys) / (double)n + np;
    const double gcost = 1.0 + M;
    if (np > M || !(rcost + 1.0 <= gcost) || !(rcost < ocost)) {  // save at least one pass
        reject();
        return;
    }

    // E. chunk prefixes of every pass: pass k merges groups of 2^(k+1)
    //    leaves (first half with second half); at k = P (odd P) one group
    //    holds every leaf as its first half: a copy back into U
    long long base = 0;
    for (int k = 0; k < np; ++k) {
        const long long G = (L + (2LL << k) - 1) >> (k + 1);
        long long ch = 0;
        if (tid < G) {
            const long long a = (long long)tid << (k + 1);
            const long long z = (a + (2LL << k)) < L ? (a + (2LL << k)) : L;
            ch = (ra->lb[z] - ra->lb[a] + CH - 1) / CH;
        }
        long long tot;
        const long long pre = wg_scan_excl(ch, s_w, tot);
        if (tid < G) ra->pre[base + tid] = pre;
        if (tid == 0) {
            ra->pre[base + G] = tot;
            ra->pbase[k] = base;
            ra->ptotal[k] = tot;
        }
        base += G + 1;
    }
    if (tid == 0) {
        ra->npasses = np;
        ra->P = P;
        ctl->path = SR_PATH_RUNS;
        ctl->run[0] = (unsigned long long)L;
        ctl->run[1] = (unsigned long long)np;
        ctl->run[2] = (unsigned long long)desc_keys;
        ctl->run[3] = (unsigned long long)dense_keys;
    }
}

// Reversal units of the descending runs (scatter launch, 256 threads):
// unit j of run [s, e) swaps the pairs (s+p, e-1-p) for p in
// [j*kRevPairs, (j+1)*kRevPairs) below (e-s)/2, every load before any store.
template <class S>
__device__ void runs_reverse(S* keys, uint32_t* pay, const RunArea* ra) {
    const long long nrev = ra->nrev, nd = ra->ndesc;
    for (long long u = blockIdx.x; u < nrev; u += gridDim.x) {
        long long lo = 0, hi = nd - 1;
        while (lo < hi) {
            const long long mid = (lo + hi + 1) >> 1;
            if (ra->dpre[mid] <= u) lo = mid;
            else hi = mid - 1;
        }
        const long long s = ra->ds[lo], e = ra->de[lo];
        const long long half = (e - s) / 2;
        const long long p0 = (u - ra->dpre[lo]) * kRevPairs;
        S a[kRevPer], b[kRevPer];
        uint32_t pa[kRevPer], pb[kRevPer];
#pragma unroll
        for (int r = 0; r < kRevPer; ++r) {
            const long long p = p0 + threadIdx.x + r * kClsWG;
            if (p < half && p < p0 + kRevPairs) {
                a[r] = keys[s + p];
                b[r] = keys[e - 1 - p];
                if (pay != nullptr) {
                    pa[r] = pay[s + p];
                    pb[r] = pay[e - 1 - p];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kRevPer; ++r) {
            const long long p = p0 + threadIdx.x + r * kClsWG;
            if (p < half && p < p0 + kRevPairs) {
                keys[s + p] = b[r];
                keys[e - 1 - p] = a[r];
                if (pay != nullptr) {
                    pay[s + p] = pb[r];
                    pay[e - 1 - p] = pa[r];
                }
            }
        }
    }
}

// Pairs: after runs_reverse every descending run is ascending, with the
// payloads of each group of equal keys in reversed input order.  Restore it:
// the payload at i trades places with the one at its mirror inside the group
// (the stable form of the reversal).  The work is cut into the reversal
// units; the last unit of an odd run also takes the middle key.
template <class C>
__device__ void runs_regroup(const typename C::S* keys, uint32_t* pay, const RunArea* ra) {
    using U = typename C::U;
    const long long nrev = ra->nrev, nd = ra->ndesc;
    for (long long u = blockIdx.x; u < nrev; u += gridDim.x) {
        long long lo = 0, hi = nd - 1;
        while (lo < hi) {
            const long long mid = (lo + hi + 1) >> 1;
            if (ra->dpre[mid] <= u) lo = mid;
            else hi = mid - 1;
        }
        const long long s = ra->ds[lo], e = ra->de[lo];
        const long long half = (e - s) / 2;
        const long long p0 = (u - ra->dpre[lo]) * kRevPairs;
        const bool mid_here = ((e - s) & 1) != 0 && p0 + kRevPairs >= half;
        for (int r = 0; r < 2 * kRevPer + 1; ++r) {
            long long i;
            if (r < 2 * kRevPer) {
                const long long p = p0 + threadIdx.x + (r >> 1) * kClsWG;
                if (!(p < half && p < p0 + kRevPairs)) continue;
                i = (r & 1) ? e - 1 - p : s + p;
            } else {
                if (!mid_here || threadIdx.x != 0) continue;
                i = s + half;
            }
            const U x = C::enc(keys[i]);
            const bool le = i > s && C::enc(keys[i - 1]) == x;
            const bool re = i + 1 < e && C::enc(keys[i + 1]) == x;
            if (!le && !re) continue;
            long long a = s, b = i;  // first key equal to x
            while (a < b) {
                const long long m = (a + b) >> 1;
                if (C::enc(keys[m]) < x) a = m + 1;
                else b = m;
            }
            const long long gs = a;
            a = i;
            b = e;  // first key above x
            while (a < b) {
                const long long m = (a + b) >> 1;
                if (C::enc(keys[m]) <= x) a = m + 1;
                else b = m;
            }
            const long long partner = gs + a - 1 - i;
            if (i < partner) {
                const uint32_t va = pay[i], vb = pay[partner];
                pay[i] = vb;
                pay[partner] = va;
            }
        }
    }
}

// Chunk c of RUNS merge pass k: its group (binary search in the pass's chunk
// prefix) as [a0, mid) + [mid, e), and the chunk's first output inside it.
struct RunChunk {
    long long a0, mid, e, out0, first;  // first: index of the group's first chunk
};
// Group of chunk c in a pass's chunk prefix: the last g < G with
// pre[g] <= c (pre[0] = 0, nondecreasing).  Wave form: a 64-ary search that
// the calling wavefront takes as a whole (every lane, c uniform) -- two
// dependent rounds for up to 4096 groups where a binary search takes twelve.
__device__ __forceinline__ long long run_group_wave(const long long* pre, long long G, long long c) {
    const int lane = (int)__lane_id();
    long long lo = 0, hi = G - 1;
    while (lo < hi) {
        const long long step = (hi - lo + kWave - 1) / kWave;
        const long long x = lo + 1 + (long long)lane * step;
        const bool pred = x <= hi && pre[x] <= c;  // true on a prefix of the lanes
        const int cnt = __builtin_popcountll(__builtin_amdgcn_ballot_w64(pred));
        if (cnt == 0) {
            hi = lo;
        } else {
            const long long nlo = lo + 1 + (long long)(cnt - 1) * step;
            hi = nlo + step - 1 < hi ? nlo + step - 1 : hi;
            lo = nlo;
        }
    }
    return lo;
}
__device__ __forceinline__ long long run_group_thread(const long long* pre, long long G, long long c) {
    long long lo = 0, hi = G - 1;
    while (lo < hi) {
        const long long mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// WAVE: the calling wavefront searches as a whole (c uniform in it).
template <bool WAVE = false>
__device__ __forceinline__ RunChunk run_chunk(const RunArea* ra, int k, long long c, long long CH) {
    const long long* pre = ra->pre + ra->pbase[k];
    const long long L = ra->L;
    const long long G = (L + (2LL << k) - 1) >> (k + 1);
    const long long lo = WAVE ? run_group_wave(pre, G, c) : run_group_thread(pre, G, c);
    const long long l0 = lo << (k + 1);
    const long long lm = (l0 + (1LL << k)) < L ? (l0 + (1LL << k)) : L;
    const long long le = (l0 + (2LL << k)) < L ? (l0 + (2LL << k)) : L;
    RunChunk r;
    r.a0 = ra->lb[l0];
    r.mid = ra->lb[lm];
    r.e = ra->lb[le];
    r.first = pre[lo];
    r.out0 = (c - pre[lo]) * CH;
    return r;
}

// RUNS merge pass k with co-ranks from the partition launch (co[c] for every
// chunk c of the pass), persistent and double-buffered like the general pass.
template <class MC, class S>
__device__ __forceinline__ void runs_merge_persist(typename MC::Buf (&buf)[2], const RunArea* ra, S* U, S* S1,
                                                   uint32_t* PU, uint32_t* PS1, int k, const int64_t* co) {
    if (k >= ra->npasses) return;
    const long long total = ra->ptotal[k];
    const S* src = (k & 1) ? S1 : U;
    S* dst = (k & 1) ? U : S1;
    const uint32_t* psrc = (k & 1) ? PS1 : PU;  // null for keys-only sorts
    uint32_t* pdst = (k & 1) ? PU : PS1;
    long long c = blockIdx.x;
    if (c >= total) return;
    typename MC::Win w;
    RunChunk rc = run_chunk<true>(ra, k, c, MC::CH);
    MC::window_from_co(rc.e - rc.a0, rc.e - rc.a0, rc.mid - rc.a0, rc.out0, co + rc.first, w);
    MC::load(src + rc.a0, psrc ? psrc + rc.a0 : nullptr, w);
    int b = 0;
    for (;;) {
        MC::stage(buf[b], w);
        const int na = w.na, cnt = w.cnt;
        const long long out0 = w.out0, a0 = rc.a0;
        __syncthreads();
        const long long cn = c + gridDim.x;
        if (cn < total) {
            rc = run_chunk<true>(ra, k, cn, MC::CH);
            MC::window_from_co(rc.e - rc.a0, rc.e - rc.a0, rc.mid - rc.a0, rc.out0, co + rc.first, w);
            MC::load(src + rc.a0, psrc ? psrc + rc.a0 : nullptr, w);
        }
        typename MC::U v[MC::ITEMS];
        uint32_t pv[MC::ITEMS];
        MC::merge(buf[b], na, cnt, v, pv);
        __syncthreads();
        MC::stage_out(buf[b], cnt, v, pv);
        __syncthreads();
        MC::store(buf[b], dst + a0, pdst ? pdst + a0 : nullptr, out0, cnt);
        if (cn >= total) break;
        c = cn;
        b ^= 1;
    }
}

// Merge pass k of the RUNS job: chunks of the pass's groups, grid-stride.
template <class MC, class S>
__device__ __forceinline__ void runs_merge(typename MC::Smem& sm, const RunArea* ra, S* U, S* S1, uint32_t* PU,
                                           uint32_t* PS1, int k) {
    if (k >= ra->npasses) return;
    const long long total = ra->ptotal[k];
    const long long* pre = ra->pre + ra->pbase[k];
    const long long L = ra->L;
    const long long G = (L + (2LL << k) - 1) >> (k + 1);
    const S* src = (k & 1) ? S1 : U;
    S* dst = (k & 1) ? U : S1;
    const uint32_t* psrc = (k & 1) ? PS1 : PU;  // null for keys-only sorts
    uint32_t* pdst = (k & 1) ? PU : PS1;
    for (long long c = blockIdx.x; c < total; c += gridDim.x) {
        const long long lo = run_group_wave(pre, G, c);
        const long long l0 = lo << (k + 1);
        const long long lm = (l0 + (1LL << k)) < L ? (l0 + (1LL << k)) : L;
        const long long le = (l0 + (2LL << k)) < L ? (l0 + (2LL << k)) : L;
        const long long a0 = ra->lb[l0], mid = ra->lb[lm], e = ra->lb[le];
        MC::run(sm, src + a0, dst + a0, psrc ? psrc + a0 : nullptr, pdst ? pdst + a0 : nullptr, e - a0, e - a0,
                mid - a0, (c - pre[lo]) * MC::CH, nullptr);
        __syncthreads();
    }
}



// -------------------------------------------------------------- few unique
// FEW job: equal buckets, the data-parallel form of the 3-way partitioning
// the paper's quicksorts use for few distinct keys (Sec. 2 k-limited class,
// Sec. 4, Appendix B).  The probe's last workgroup sorts kFewSample evenly
// spread keys and keeps their distinct values as splitters s_0 < ... <
// s_{ns-1}.  Bucket 2i+1 holds the keys equal to s_i; bucket 2i the keys
// strictly between s_{i-1} and s_i (bucket 0: below s_0, bucket 2ns: above
// s_{ns-1}).
//   classify  per 4096-key tile: each key's bucket (binary search among the
//             splitters), bucket counts, and the keys of the "between"
//             buckets appended to S1[n-m, n) (any order: keys only)
//   verify    bucket offsets; GENERAL if m > n/4 (U still untouched)
//   tile sort / merge slots 0 .. P-1: the m between keys are sorted like the
//             outlier list (U is free: every equal key is known from its
//             splitter and count)
//   merge slot P: every output position is filled from its bucket -- the
//             splitter value, or the next sorted between key
// Keys equal under the order are bit-identical, so writing the splitter
// reproduces them exactly.  For few-unique input m = 0: one read and one
// write of the array.
constexpr int kFewMax = 64;
constexpr int kFewBuckets = 2 * kFewMax + 1;
constexpr int kFewSample = 1024;
constexpr int kFewCopies = 32;  // bucket counter copies (workgroup w adds to copy w % 32)
constexpr size_t kFewLdsBytes = 8 * (2 * kFewBuckets + 1) + 8 * kFewMax;  // few_place's table copy

struct FewTable {
    unsigned long long ns;                    // splitters
    unsigned long long split[kFewMax];        // encoded, ascending, distinct
    unsigned long long cnt[kFewCopies][kFewBuckets];  // keys per bucket, spread over copies
    unsigned long long tot[kFewBuckets];      // keys per bucket
    long long off[kFewBuckets + 1];           // first output position of each bucket
    long long bpre[kFewBuckets];              // between keys in earlier buckets
    unsigned long long sample[kFewSample];    // the probe's sample, sorted in place (raw keys)
};

template <class U>
__device__ __forceinline__ int few_bucket(const U* sp, int ns, U u) {
    int lo = 0, hi = ns;  // splitters below u
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sp[mid] < u) lo = mid + 1;
        else hi = mid;
    }
    return (lo < ns && sp[lo] == u) ? 2 * lo + 1 : 2 * lo;
}

// Position of sample j of S over [0, n): a point inside stratum j drawn by a
// hash of j, so that inputs with a period dividing the stratum width (teeth
// whose length is a multiple of n/S) do not show the sample a few values
// repeated.
__device__ __forceinline__ int64_t strat_pos(int64_t j, int64_t n, int64_t S) {
    const int64_t lo = j * n / S, hi = (j + 1) * n / S;
    uint32_t h = (uint32_t)j * 0x9E3779B1u;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    return hi > lo ? lo + (int64_t)(((uint64_t)h * (uint64_t)(hi - lo)) >> 32) : lo;
}

// The between keys of a classify tile (bm[r]: wavefront ballot of the keys
// x[r] that fall between splitters) to S1[n-1-m, ...), in any order: one
// reservation per tile, and no stores once the job holds more than n/4 of
// them -- the plan then falls back to GENERAL and never reads them, so a
// wrong few-unique guess costs one counting read.  Every thread calls it.
template <class S, int R>
__device__ __forceinline__ void few_between(const S (&x)[R], const unsigned long long (&bm)[R], int64_t n,
                                            Ctl* ctl, S* s1) {
    __shared__ unsigned int s_wc[kClsWG / kWave];
    __shared__ unsigned long long s_base;
    const int lane = (int)__lane_id();
    const int wave = (int)threadIdx.x / kWave;
    unsigned int c = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) c += (unsigned int)__builtin_popcountll(bm[r]);
    if (lane == 0) s_wc[wave] = c;
    __syncthreads();
    unsigned int tot = 0, before = 0;
#pragma unroll
    for (int w = 0; w < kClsWG / kWave; ++w) {
        before += w < wave ? s_wc[w] : 0u;
        tot += s_wc[w];
    }
    if (threadIdx.x == 0) s_base = tot != 0u ? atomicAdd(&ctl->m, (unsigned long long)tot) : 0ull;
    __syncthreads();
    const unsigned long long base = s_base;
    if ((base + tot) * 4ull > (unsigned long long)n) return;
    unsigned long long off = base + before;
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if ((bm[r] >> lane) & 1ull) s1[n - 1 - (int64_t)(off + __builtin_popcountll(bm[r] & below))] = x[r];
        off += (unsigned long long)__builtin_popcountll(bm[r]);
    }
}

// LDS of the small-table counts (shares the classify launch's union).
template <class U>
struct FewLds {
    U sp[kFewMax];
    unsigned int hist[kFewBuckets];
    unsigned int between;
};

// Bucket counts and between keys of the 4096-key tile [c0, c1) (256 threads).
template <class C>
__device__ void few_count(const typename C::S* keys, int64_t n, int64_t c0, int64_t c1, Ctl* ctl, FewTable* ft,
                          typename C::S* s1, FewLds<typename C::U>& fl) {
    using U = typename C::U;
    constexpr int R = kClsTC / kClsWG;
    U* sp = fl.sp;
    unsigned int* hist = fl.hist;
    const int tid = threadIdx.x;
    const int ns = (int)ft->ns;
    const int nb = 2 * ns + 1;
    for (int i = tid; i < ns; i += kClsWG) sp[i] = (U)ft->split[i];
    for (int b = tid; b < nb; b += kClsWG) hist[b] = 0;
    typename C::S x[R];
    // a whole tile as 16-byte vectors: the order of a tile's keys matters
    // neither to its counts nor to its between keys (they are sorted later)
    constexpr int VN = 16 / (int)sizeof(typename C::S);
    const bool vec = c1 - c0 == kClsTC && aligned16(keys + c0);
    if (vec) {
#pragma unroll
        for (int u = 0; u < R / VN; ++u) {
            const V16<typename C::S> y = reinterpret_cast<const V16<typename C::S>*>(keys + c0)[u * kClsWG + tid];
#pragma unroll
            for (int j = 0; j < VN; ++j) x[u * VN + j] = y.v[j];
        }
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t q = c0 + r * kClsWG + tid;
            if (q < c1) x[r] = keys[q];
        }
    }
    __syncthreads();
    unsigned long long bm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = c0 + r * kClsWG + tid;
        bool between = false;
        if (vec || q < c1) {
            const int b = few_bucket<U>(sp, ns, C::enc(x[r]));
            atomicAdd(&hist[b], 1u);
            between = (b & 1) == 0;
        }
        bm[r] = __builtin_amdgcn_ballot_w64(between);
    }
    __syncthreads();
    unsigned long long* cc = ft->cnt[blockIdx.x % kFewCopies];
    for (int b = tid; b < nb; b += kClsWG)
        if (hist[b] != 0u) atomicAdd(&cc[b], (unsigned long long)hist[b]);
    few_between<typename C::S, R>(x, bm, n, ctl, s1);
}

// Bucket totals (the counter copies summed, one bucket per thread), then
// offsets and the job (thread 0 of the verify workgroup).
__device__ void few_plan(Ctl* ctl, int64_t n, FewTable* ft, int64_t T_sort) {
    __shared__ unsigned long long s_tot[kFewBuckets];
    const int nb = 2 * (int)ft->ns + 1;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        unsigned long long t = 0;
        for (int c = 0; c < kFewCopies; ++c) t += ld_agent(&ft->cnt[c][b]);
        s_tot[b] = t;
        ft->tot[b] = t;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const unsigned long long m = ld_agent(&ctl->m);
    long long o = 0, bp = 0;
    for (int b = 0; b < nb; ++b) {
        ft->off[b] = o;
        ft->bpre[b] = bp;
        o += (long long)s_tot[b];
        if ((b & 1) == 0) bp += (long long)s_tot[b];
    }
    ft->off[nb] = o;
    if (o != n || (unsigned long long)bp != m || 4 * m > (unsigned long long)n) {
        ctl->path = SR_PATH_GENERAL;
        ctl->m = 0;
        ctl->job_passes = 0;
        return;
    }
    ctl->job_passes = ceil_log2_dev(((int64_t)m + T_sort - 1) / T_sort);
}

// Merge slot P of the FEW job: U[p] for every p, grid-stride over blocks of
// WG x 8 outputs; lds holds the table (at least 8 * (2 * kFewBuckets + 1) +
// 8 * kFewMax bytes).
template <class C, int WG>
__device__ __forceinline__ void few_place(typename C::S* U, const typename C::S* X0, int64_t n, const FewTable* ft, void* lds) {
    using S = typename C::S;
    constexpr int IT = 8;
    long long* off = static_cast<long long*>(lds);
    long long* bpre = off + kFewBuckets + 1;
    S* spv = reinterpret_cast<S*>(bpre + kFewBuckets);
    const int tid = threadIdx.x;
    const int ns = (int)ft->ns;
    const int nb = 2 * ns + 1;
    for (int b = tid; b <= nb; b += WG) off[b] = ft->off[b];
    for (int b = tid; b < nb; b += WG) bpre[b] = ft->bpre[b];
    for (int i = tid; i < ns; i += WG) spv[i] = C::dec((typename C::U)ft->split[i]);
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * WG * IT; base < n; base += (int64_t)gridDim.x * WG * IT) {
        const int64_t p0 = base + (int64_t)tid * IT;
        if (p0 >= n) continue;
        int lo = 0, hi = nb - 1;  // last bucket starting at or before p0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= p0) lo = mid;
            else hi = mid - 1;
        }
        int b = lo;
        constexpr int VN = 16 / sizeof(S);
        V16<S> v[IT / VN];
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int64_t p = p0 + r;
            S val{};
            if (p < n) {
                while (off[b + 1] <= p) ++b;
                val = (b & 1) ? spv[b >> 1] : X0[bpre[b] + (p - off[b])];
            }
            v[r / VN].v[r % VN] = val;
        }
        if (p0 + IT <= n && aligned16(U + p0)) {
#pragma unroll
            for (int q = 0; q < IT / VN; ++q) reinterpret_cast<V16<S>*>(U + p0)[q] = v[q];
        } else {
#pragma unroll
            for (int r = 0; r < IT; ++r)
                if (p0 + r < n) U[p0 + r] = v[r / VN].v[r % VN];
        }
    }
}

// ------------------------------------------------------ few unique, pairs
// FEW for key + payload sorts, when every key equals one of at most kFewMax
// sampled values (no keys between them; otherwise the plan falls back to
// GENERAL with U untouched) and the per-tile counts fit the wide table's
// space (n <= 1024 tiles of kClsTC keys).  Equal keys must keep their input
// order, so each (value, tile) gets its own output range:
//   classify  tile t's count of each value into row i, column t of a count
//             matrix; keys between values only counted (into m)
//   verify    each value's row scanned (exclusive, in place; one thread per
//             value), the values' output offsets; GENERAL unless m == 0 and
//             the counts add up to n
//   scatter   tile t again, in input order (16 rounds of 256 keys): a key's
//             rank among the tile's earlier keys of its value (wave ballots
//             per value present, then the earlier waves' counts and the
//             earlier rounds') gives its output position; key and payload
//             go to S1 / PS1 there
//   merge slot 0: S1 / PS1 copied back to U / PU
// One read of the keys, one read and one write of keys and payloads, one
// copy: stable by construction.

// Counts of the kClsTC-key tile t = [c0, c1) (256 threads).
template <class C>
__device__ void few_count_pairs(const typename C::S* keys, int64_t c0, int64_t c1, Ctl* ctl, const FewTable* ft,
                                unsigned int* fewm, int64_t t, int64_t ncls, FewLds<typename C::U>& fl) {
    using U = typename C::U;
    constexpr int R = kClsTC / kClsWG;
    U* sp = fl.sp;
    unsigned int* hist = fl.hist;
    unsigned int& s_between = fl.between;
    const int tid = threadIdx.x;
    const int ns = (int)ft->ns;
    for (int i = tid; i < ns; i += kClsWG) {
        sp[i] = (U)ft->split[i];
        hist[i] = 0u;
    }
    if (tid == 0) s_between = 0u;
    __syncthreads();
    unsigned int nb = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = c0 + r * kClsWG + tid;
        if (q < c1) {
            const int b = few_bucket<U>(sp, ns, C::enc(keys[q]));
            if (b & 1) atomicAdd(&hist[b >> 1], 1u);
            else ++nb;
        }
    }
    if (nb != 0u) atomicAdd(&s_between, nb);
    __syncthreads();
    for (int i = tid; i < ns; i += kClsWG) fewm[(int64_t)i * ncls + t] = hist[i];
    if (tid == 0 && s_between != 0u) atomicAdd(&ctl->m, (unsigned long long)s_between);
}

// Row scans and value offsets (the verify workgroup).
__device__ void few_plan_pairs(Ctl* ctl, int64_t n, FewTable* ft, unsigned int* fewm, int64_t ncls) {
    __shared__ unsigned long long s_tot[kFewMax];
    const int ns = (int)ft->ns;
    for (int i = threadIdx.x; i < ns; i += blockDim.x) {
        unsigned int* row = fewm + (int64_t)i * ncls;
        unsigned long long run = 0;
        for (int64_t t = 0; t < ncls; ++t) {
            const unsigned int c = row[t];
            row[t] = (unsigned int)run;
            run += c;
        }
        s_tot[i] = run;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    const unsigned long long m = ld_agent(&ctl->m);
    long long o = 0;
    for (int i = 0; i < ns; ++i) {
        ft->off[2 * i + 1] = o;
        o += (long long)s_tot[i];
    }
    if (m != 0ull || o != n) {
        ctl->path = SR_PATH_GENERAL;
        ctl->m = 0;
    }
    ctl->job_passes = 0;
}

// Scatter of tile t (256 threads): keys and payloads to their places in
// S1 / PS1.
template <class C>
__device__ void few_scatter_pairs(const typename C::S* keys, const uint32_t* pay, typename C::S* s1, uint32_t* ps1,
                                  int64_t n, const FewTable* ft, const unsigned int* fewm, int64_t t,
                                  int64_t ncls) {
    using U = typename C::U;
    using S = typename C::S;
    constexpr int R = kClsTC / kClsWG;
    constexpr int NW = kClsWG / kWave;
    __shared__ U sp[kFewMax];
    __shared__ long long base[kFewMax];            // place of the tile's next key of each value
    __shared__ unsigned int wcnt[NW][kFewMax];     // keys of each value per wave, this round
    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid / kWave;
    const int64_t c0 = t * kClsTC;
    const int64_t c1 = (c0 + kClsTC) < n ? (c0 + kClsTC) : n;
    const int ns = (int)ft->ns;
    for (int i = tid; i < ns; i += kClsWG) {
        sp[i] = (U)ft->split[i];
        base[i] = ft->off[2 * i + 1] + (long long)fewm[(int64_t)i * ncls + t];
    }
    for (int i = tid; i < NW * kFewMax; i += kClsWG) wcnt[i / kFewMax][i % kFewMax] = 0u;
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r = 0; r < R; ++r) {
        const int64_t q = c0 + (int64_t)r * kClsWG + tid;
        int b = -1;  // value index; -1: no key, or a key between values (none in a FEW plan)
        S x{};
        uint32_t p = 0;
        if (q < c1) {
            x = keys[q];
            p = pay[q];
            const int bb = few_bucket<U>(sp, ns, C::enc(x));
            b = (bb & 1) ? (bb >> 1) : -1;
        }
        // one round per value present in the wavefront: its lanes' ranks,
        // and its count from its first lane
        unsigned long long rem = __builtin_amdgcn_ballot_w64(b >= 0);
        int rank = 0;
        while (rem != 0ull) {
            const int lead = __builtin_ctzll(rem);
            const int bl = __shfl(b, lead);
            const unsigned long long mk = __builtin_amdgcn_ballot_w64(b == bl);
            if (b == bl) rank = __builtin_popcountll(mk & below);
            if (lane == lead) wcnt[wave][bl] = (unsigned int)__builtin_popcountll(mk);
            rem &= ~mk;
        }
        __syncthreads();
        if (b >= 0) {
            long long pos = base[b] + rank;
            for (int w = 0; w < wave; ++w) pos += (long long)wcnt[w][b];
            if (pos >= 0 && pos < n) {
                s1[pos] = x;
                ps1[pos] = p;
            }
        }
        __syncthreads();
        for (int i = tid; i < ns; i += kClsWG) {
            unsigned int c = 0;
            for (int w = 0; w < NW; ++w) {
                c += wcnt[w][i];
                wcnt[w][i] = 0u;
            }
            base[i] += (long long)c;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------- outliers, pairs
// OUTLIER for key + payload sorts.  The kept keys are in input order and
// sorted; an outlier and a kept key with the same key must come out in input
// order, which the keys alone do not tell.  The scatter stores the outliers
// in input order, each with its index j as the payload that the outlier sort
// carries (stable: equal outliers keep their order), and beside the job its
// payload and its kept-before count kb_j (the kept keys ahead of it in the
// input).  Then, with A the kept keys and [lo, hi) the range of A equal to
// an outlier's key, the sorted outlier k goes to k + clamp(kb_j, lo, hi)
// (merge slot P), and the kept key a to the a-th position left free (slot
// P + 1).  The job is taken for m <= n/4 and P + 2 <= M merge slots.

// First index of A[0, na) whose code is not below u (strict: above u).
template <class C, bool STRICT>
__device__ __forceinline__ int64_t bound_in(const typename C::S* A, int64_t na, typename C::U u) {
    int64_t lo = 0, hi = na;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        const typename C::U y = C::enc(A[mid]);
        if (STRICT ? y <= u : y < u) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge slot P: every sorted outlier k to its place in U / PU; its place is
// kept in PS1[n-m+k] (sorted: the places increase with k) for slot P + 1.
template <class C>
__device__ void outlier_place_pairs(typename C::S* Ub, const typename C::S* S1, uint32_t* PUb, uint32_t* PS1,
                                    int64_t n, int64_t m, const uint32_t* opay, const uint32_t* okb) {
    using S = typename C::S;
    const int64_t na = n - m;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const S x = S1[na + k];
        const uint32_t j = PS1[na + k];
        const typename C::U u = C::enc(x);
        const int64_t lo = bound_in<C, false>(S1, na, u);
        // keys equal to x among the kept ones: usually none
        int64_t hi = lo;
        if (lo < na && C::enc(S1[lo]) == u) hi = lo + bound_in<C, true>(S1 + lo, na - lo, u);
        const int64_t kb = j < (uint64_t)m ? (int64_t)okb[j] : 0;
        const int64_t pos = k + (kb < lo ? lo : kb > hi ? hi : kb);
        if (pos >= 0 && pos < n && j < (uint64_t)m) {
            Ub[pos] = x;
            PUb[pos] = opay[j];
        }
        PS1[na + k] = (uint32_t)pos;
    }
}

// First k in [0, m) with B[k] >= p (B ascending), by one wavefront: 64
// probes per round narrow the range 64-fold.  Result in every lane.
__device__ __forceinline__ int64_t lower_bound_wave(const uint32_t* B, int64_t m, int64_t p) {
    const int lane = (int)__lane_id();
    int64_t lo = 0, hi = m;  // B[lo - 1] < p <= B[hi]
    while (lo < hi) {
        const int64_t len = hi - lo;
        const int64_t step = (len + kWave - 1) / kWave;
        const int64_t x = lo + (int64_t)lane * step;
        const bool below = x < hi && (int64_t)B[x] < p;
        const int cnt = __builtin_popcountll(__builtin_amdgcn_ballot_w64(below));
        if (cnt == 0) {
            hi = lo;
        } else {
            const int64_t last = lo + (int64_t)(cnt - 1) * step;
            const int64_t first_not = lo + (int64_t)cnt * step;
            lo = last + 1;
            hi = first_not < hi ? first_not : hi;
        }
    }
    return lo;
}

// Merge slot P + 1: the kept pairs into the places left free, in order:
// output p (not an outlier's place) takes A[p - (outlier places below p)].
// Chunks of WG * 16 outputs, grid-stride; a chunk's outlier places as an
// LDS bitmap with word prefix counts.
template <class C, int WG>
__device__ void outlier_fill_pairs(typename C::S* Ub, const typename C::S* S1, uint32_t* PUb, const uint32_t* PS1,
                                   int64_t n, int64_t m) {
    constexpr int CHF = WG * 16;
    constexpr int NWD = CHF / 32;
    static_assert(NWD <= WG, "one bitmap word per thread");
    __shared__ unsigned int bm[NWD];
    __shared__ unsigned int pre[NWD];
    __shared__ long long s_k[2];
    const int tid = threadIdx.x;
    const int64_t na = n - m;
    const uint32_t* B = PS1 + na;
    for (int64_t p0 = (int64_t)blockIdx.x * CHF; p0 < n; p0 += (int64_t)gridDim.x * CHF) {
        const int64_t p1 = (p0 + CHF) < n ? (p0 + CHF) : n;
        if (tid < NWD) bm[tid] = 0u;
        if (tid < 2 * kWave) {
            const int64_t kk = lower_bound_wave(B, m, tid < kWave ? p0 : p1);
            if (tid == 0) s_k[0] = kk;
            if (tid == kWave) s_k[1] = kk;
        }
        __syncthreads();
        const int64_t k0 = s_k[0], k1 = s_k[1];
        for (int64_t k = k0 + tid; k < k1; k += WG) {
            const int64_t off = (int64_t)B[k] - p0;
            if (off >= 0 && off < CHF) atomicOr(&bm[off >> 5], 1u << (off & 31));
        }
        __syncthreads();
        if (tid == 0) {
            unsigned int run = 0;
            for (int w = 0; w < NWD; ++w) {
                pre[w] = run;
                run += (unsigned int)__builtin_popcount(bm[w]);
            }
        }
        __syncthreads();
        for (int i = tid; i < (int)(p1 - p0); i += WG) {
            const unsigned int word = bm[i >> 5];
            const unsigned int bit = 1u << (i & 31);
            if (word & bit) continue;
            const int64_t before = k0 + (int64_t)pre[i >> 5] + __builtin_popcount(word & (bit - 1u));
            const int64_t a = p0 + i - before;
            if (a >= 0 && a < na) {
                Ub[p0 + i] = S1[a];
                PUb[p0 + i] = PS1[a];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ wide few unique
// The FEW job with 65 to 4096 sampled values (Table 1's few-unique type is
// 12-limited: 4096 values).  Buckets and job are those above; what changes
// with the count: the probe samples kWideSample keys into a larger hash set
// and sorts the distinct values with the tile sorter; a key's bucket is a
// branch-free binary search over the splitters in LDS; a tile's counts are
// 16-bit LDS counters (a tile holds 4096 keys) added to one global counter
// per bucket; the offsets come from a scan across the verify workgroup; the
// fill pass reads its tables through the cache.  A 16384-key sample of 4096
// values misses about 2 % of them (4096 e^-4); their keys are between keys.
constexpr int kWideMax = 4096;
constexpr int kWideBuckets = 2 * kWideMax + 1;
constexpr int kWideSample = 16384;
constexpr int kWideHash = 8192;  // LDS hash set slots (codes of the key type)

// In the look-back area of the workspace; the probe clears the counters a
// wide job will use.
struct WideTable {
    unsigned long long ns;                   // splitters
    unsigned long long split[kWideMax];      // codes, ascending, distinct
    unsigned long long cnt[kWideBuckets];    // keys per bucket
    long long off[kWideBuckets + 1];         // first output position of each bucket
    long long bpre[kWideBuckets];            // between keys in earlier buckets
    unsigned long long sample[kWideMax];     // the probe's distinct samples (raw keys), sorted in place
};

// Splitters below code u: binary search over the ns (>= 1) splitter codes
// sp[] without branches (P >= ns a power of two; positions past the
// splitters count as the largest code, their reads clamped to the last).
// The steps of at least Q = max(P / kWideIdx, 1) positions read idx[] in LDS
// (every Q-th splitter), the last log2(Q) steps read the table through the cache:
// a copy of the whole table in LDS (16 KB) halved the classify launch's
// occupancy on the outlier path, whose window shares that LDS.
constexpr int kWideIdx = 256;
template <class U>
__device__ __forceinline__ int wide_below(const unsigned long long* sp, const U* idx, int ns, int P, U u) {
    const int Q = P > kWideIdx ? P / kWideIdx : 1;
    int base = 0;
    int half = P >> 1;
    for (; half >= Q && half > 0; half >>= 1) {
        const int j = base + half;
        base = idx[j / Q] < u ? j : base;
    }
    for (; half > 0; half >>= 1) {
        const int j = base + half;
        const U y = (U)sp[j < ns ? j : ns - 1];
        base = (j < ns && y < u) ? j : base;
    }
    return base + ((U)sp[base] < u ? 1 : 0);
}

template <class U>
struct WideLds {
    unsigned int hist[(kWideBuckets + 1) / 2];   // two 16-bit counters per word
    U idx[kWideIdx];                             // every (P / kWideIdx)-th splitter code
};

// Bucket counts and between keys of the 4096-key tile [c0, c1) (256 threads).
template <class C>
__device__ void wide_count(const typename C::S* keys, int64_t n, int64_t c0, int64_t c1, Ctl* ctl, WideTable* fw,
                           typename C::S* s1, WideLds<typename C::U>& fl) {
    using U = typename C::U;
    constexpr int R = kClsTC / kClsWG;
    static_assert(kClsTC < 65536, "16-bit tile counters");
    const int tid = threadIdx.x;
    const int ns = (int)fw->ns;
    const int nb = 2 * ns + 1;
    int P = 1;
    while (P < ns) P <<= 1;
    const unsigned long long* sp = fw->split;
    for (int w = tid; w < (nb + 1) / 2; w += kClsWG) fl.hist[w] = 0u;
    static_assert(kWideIdx <= kClsWG && kWideMax / kWideIdx >= 1, "one index entry per thread");
    if (tid < kWideIdx) {
        const int j = tid * (P > kWideIdx ? P / kWideIdx : 1);
        fl.idx[tid] = j < ns ? (U)sp[j] : (U)~(U)0;
    }
    typename C::S x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = c0 + r * kClsWG + tid;
        if (q < c1) x[r] = keys[q];
    }
    __syncthreads();
    unsigned long long bm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t q = c0 + r * kClsWG + tid;
        bool between = false;
        if (q < c1) {
            const U u = C::enc(x[r]);
            const int lo = wide_below<U>(sp, fl.idx, ns, P, u);
            const int b = (lo < ns && (U)sp[lo < ns ? lo : ns - 1] == u) ? 2 * lo + 1 : 2 * lo;
            atomicAdd(&fl.hist[b >> 1], 1u << ((b & 1) * 16));
            between = (b & 1) == 0;
        }
        bm[r] = __builtin_amdgcn_ballot_w64(between);
    }
    __syncthreads();
    for (int w = tid; w < (nb + 1) / 2; w += kClsWG) {
        const unsigned int h = fl.hist[w];
        if (h & 0xFFFFu) atomicAdd(&fw->cnt[2 * w], (unsigned long long)(h & 0xFFFFu));
        if ((h >> 16) != 0u && 2 * w + 1 < nb) atomicAdd(&fw->cnt[2 * w + 1], (unsigned long long)(h >> 16));
    }
    few_between<typename C::S, R>(x, bm, n, ctl, s1);
}

// Offsets (a scan across the verify workgroup, kWideBuckets / kVerWG buckets
// per thread) and the job.
__device__ void wide_plan(Ctl* ctl, int64_t n, WideTable* fw, int64_t T_sort) {
    constexpr int PB = (kWideBuckets + kVerWG - 1) / kVerWG;
    __shared__ long long s_w[kVerWG / kWave];
    __shared__ long long s_bw[kVerWG / kWave];
    const int ns = (int)fw->ns;
    const int nb = 2 * ns + 1;
    const int b0 = (int)threadIdx.x * PB;
    unsigned long long t[PB];
    long long sum = 0, bsum = 0;
#pragma unroll
    for (int q = 0; q < PB; ++q) {
        const int b = b0 + q;
        t[q] = b < nb ? ld_agent(&fw->cnt[b]) : 0ull;
        sum += (long long)t[q];
        if ((b & 1) == 0) bsum += (long long)t[q];
    }
    long long total, btotal;
    long long o = wg_scan_excl(sum, s_w, total);
    long long bp = wg_scan_excl(bsum, s_bw, btotal);
#pragma unroll
    for (int q = 0; q < PB; ++q) {
        const int b = b0 + q;
        if (b < nb) {
            fw->off[b] = o;
            fw->bpre[b] = bp;
        }
        o += (long long)t[q];
        if ((b & 1) == 0) bp += (long long)t[q];
    }
    if (threadIdx.x != 0) return;
    fw->off[nb] = total;
    const unsigned long long m = ld_agent(&ctl->m);
    if (total != n || (unsigned long long)btotal != m || 4 * m > (unsigned long long)n) {
        ctl->path = SR_PATH_GENERAL;
        ctl->m = 0;
        ctl->job_passes = 0;
        return;
    }
    ctl->job_passes = ceil_log2_dev(((int64_t)m + T_sort - 1) / T_sort);
}

// Merge slot P of a wide FEW job: as few_place, with the tables read through
// the cache.
template <class C, int WG>
__device__ __forceinline__ void wide_place(typename C::S* U, const typename C::S* X0, int64_t n,
                                           const WideTable* fw) {
    using S = typename C::S;
    constexpr int IT = 8;
    const int tid = threadIdx.x;
    const int nb = 2 * (int)fw->ns + 1;
    const long long* off = fw->off;
    const long long* bpre = fw->bpre;
    for (int64_t base = (int64_t)blockIdx.x * WG * IT; base < n; base += (int64_t)gridDim.x * WG * IT) {
        const int64_t p0 = base + (int64_t)tid * IT;
        if (p0 >= n) continue;
        int lo = 0, hi = nb - 1;  // last bucket starting at or before p0
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= p0) lo = mid;
            else hi = mid - 1;
        }
        int b = lo;
        constexpr int VN = 16 / sizeof(S);
        V16<S> v[IT / VN];
#pragma unroll
        for (int r = 0; r < IT; ++r) {
            const int64_t p = p0 + r;
            S val{};
            if (p < n) {
                while (off[b + 1] <= p) ++b;
                val = (b & 1) ? C::dec((typename C::U)fw->split[b >> 1]) : X0[bpre[b] + (p - off[b])];
            }
            v[r / VN].v[r % VN] = val;
        }
        if (p0 + IT <= n && aligned16(U + p0)) {
#pragma unroll
            for (int q = 0; q < IT / VN; ++q) reinterpret_cast<V16<S>*>(U + p0)[q] = v[q];
        } else {
#pragma unroll
            for (int r = 0; r < IT; ++r)
                if (p0 + r < n) U[p0 + r] = v[r / VN].v[r % VN];
        }
    }
}

// ============================================================== kernels

// Tile-sort launch.  GENERAL / OUTLIER: the tile sort of the job's array
// (resolve_tile).  REVERSED: the same launch reverses the array instead --
// workgroup b swaps the pairs (i, n-1-i) for i in its half-tile share
// [b*T/2, (b+1)*T/2) of [0, n/2), in place in U.
template <class C, int WG, int IT, bool PAIRS>
__global__ __launch_bounds__(WG) void k_tile_sort(typename C::S* U, typename C::S* S1, uint32_t* PU,
                                                  uint32_t* PS1, int64_t n, int M, const Ctl* ctl,
                                                  const RunTile* rdesc, unsigned long long* tdesc = nullptr,
                                                  int fan4 = 0) {
    using TS = TileSort<C, WG, IT, PAIRS>;
    using S = typename C::S;
    __shared__ typename TS::Smem sm;
    if constexpr (TS::T >= kClsTC) {  // the RUNS job needs tiles of whole run-scan tiles
        // RUNS: sort the dense 4096-key tiles of this tile in place, both at
        // once when both are dense (the plan's dense pieces)
        if (ctl != nullptr && rdesc != nullptr && ctl->path == SR_PATH_RUNS) {
            constexpr int G = TS::T / kClsTC;
            static_assert(G == 1 || G == 2, "tile = 1 or 2 run-scan tiles");
            const int64_t ncls = (n + kClsTC - 1) / kClsTC;
            const int64_t q0 = (int64_t)blockIdx.x * G;
            const bool d0 = q0 < ncls && rdesc[q0].nh < 0;
            const bool d1 = G == 2 && q0 + 1 < ncls && rdesc[q0 + 1].nh < 0;
            int64_t s0 = -1, e0 = -1, s1 = -1, e1 = -1;
            if (d0 && d1) {
                s0 = q0 * kClsTC;
                e0 = (q0 + 2) * kClsTC;
            } else {
                if (d0) {
                    s0 = q0 * kClsTC;
                    e0 = s0 + kClsTC;
                }
                if (d1) {
                    s1 = (q0 + 1) * kClsTC;
                    e1 = s1 + kClsTC;
                }
            }
            if (s0 >= 0) {
                e0 = e0 < n ? e0 : n;
                TS::run(sm, U + s0, U + s0, PAIRS ? PU + s0 : nullptr, PAIRS ? PU + s0 : nullptr, (int)(e0 - s0));
            }
            if (s1 >= 0) {
                e1 = e1 < n ? e1 : n;
                __syncthreads();
                TS::run(sm, U + s1, U + s1, PAIRS ? PU + s1 : nullptr, PAIRS ? PU + s1 : nullptr, (int)(e1 - s1));
            }
            return;
        }
    }
    if (ctl != nullptr && ctl->path == SR_PATH_REVERSED) {
        constexpr int H = TS::T / 2;
        constexpr int R = H / WG;
        const int64_t half = n / 2;
        const int64_t i0 = (int64_t)blockIdx.x * H + threadIdx.x;
        S a[R], b[R];
        uint32_t pa[R], pb[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = i0 + (int64_t)r * WG;
            if (i < half) {
                a[r] = U[i];
                b[r] = U[n - 1 - i];
                if constexpr (PAIRS) {
                    pa[r] = PU[i];
                    pb[r] = PU[n - 1 - i];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t i = i0 + (int64_t)r * WG;
            if (i < half) {
                U[i] = b[r];
                U[n - 1 - i] = a[r];
                if constexpr (PAIRS) {
                    PU[i] = pb[r];
                    PU[n - 1 - i] = pa[r];
                }
            }
        }
        return;
    }
    const PassView<S> v = resolve_tile(ctl, U, S1, PU, PS1, n, M, fan4 != 0);
    if (!v.active) return;
    const int64_t base = (int64_t)blockIdx.x * TS::T;
    if (base >= v.n) return;
    const int valid = (int)((v.n - base) < TS::T ? (v.n - base) : TS::T);
    // the general plan's tiles describe themselves for merge slot 0's NEAR test
    unsigned long long* desc =
        (tdesc != nullptr && ctl != nullptr && ctl->path == SR_PATH_NEAR) ? tdesc + 4 * blockIdx.x : nullptr;
    TS::body(sm, v.src + base, v.dst + base, PAIRS ? v.psrc + base : nullptr, PAIRS ? v.pdst + base : nullptr,
             valid, desc);
}

// Merge Path partition of merge slot k: co[c] = co-rank of the start of
// output chunk c (c*CH) inside its pair of runs.  One thread per chunk.
template <class C>
__global__ __launch_bounds__(256) void k_partition(typename C::S* U, typename C::S* S1, int64_t n, int M,
                                                   int64_t T, int k, int CH, int64_t* co, const Ctl* ctl,
                                                   const RunArea* ra, int fan4 = 0) {
    using S = typename C::S;
    if (ra != nullptr && ctl != nullptr && ctl->path == SR_PATH_RUNS) {
        // RUNS: co-rank of every chunk of the pass inside its leaf group
        if (k >= ra->npasses) return;
        const S* src = (k & 1) ? S1 : U;
        const long long total = ra->ptotal[k];
        for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < total; c += (long long)gridDim.x * 256) {
            const RunChunk rc = run_chunk(ra, k, c, CH);
            co[c] = corank_thread<C>(src + rc.a0, rc.mid - rc.a0, src + rc.mid, rc.e - rc.mid, rc.out0);
        }
        return;
    }
    const PassView<S> v = resolve_merge(ctl, U, S1, (uint32_t*)nullptr, (uint32_t*)nullptr, n, M, T, k, fan4 != 0);
    if (!v.active || v.fan == 4) return;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c * CH >= v.n) return;
    const int64_t out0 = c * CH;
    int64_t gs, la, lb;
    if (v.split >= 0) {
        gs = 0;
        la = v.split;
        lb = v.n - v.split;
    } else {
        const int64_t g = 2 * v.width;  // a power of two on level-synchronous passes
        gs = (g & (g - 1)) == 0 ? (out0 & ~(g - 1)) : out0 / g * g;
        la = (v.n - gs) < v.width ? (v.n - gs) : v.width;
        const int64_t rest = v.n - gs - la;
        lb = rest < v.width ? rest : v.width;
    }
    co[c] = corank_guess<C>(v.src + gs, la, v.src + gs + la, lb, out0 - gs);
}

// Merge slot k, one chunk per workgroup, co-ranks searched in the workgroup.
template <class C, int WG, int IT, bool PAIRS>
__global__ __launch_bounds__(WG) void k_merge(typename C::S* U, typename C::S* S1, uint32_t* PU, uint32_t* PS1,
                                              int64_t n, int M, int64_t T, int k, const Ctl* ctl,
                                              const RunArea* ra, const FewTable* ft,
                                              const unsigned long long* tdesc = nullptr,
                                              const WideTable* fw = nullptr, const uint32_t* opay = nullptr,
                                              const uint32_t* okb = nullptr) {
    using MC = MergeChunk<C, WG, IT, PAIRS>;
    using S = typename C::S;
    __shared__ typename MC::Smem sm;
    static_assert(sizeof(sm) >= kFewLdsBytes, "fill pass table fits the merge LDS");
    if (ctl != nullptr && ra != nullptr && ctl->path == SR_PATH_RUNS) {
        runs_merge<MC, S>(sm, ra, U, S1, PU, PS1, k);
        return;
    }
    if constexpr (PAIRS) {
        // FEW of pairs: the placed keys and payloads back into the user buffers
        if (ctl != nullptr && ft != nullptr && ctl->path == SR_PATH_FEW && k == 0) {
            copy_part(S1, U, PS1, PU, n, (int64_t)blockIdx.x, (int64_t)gridDim.x);
            return;
        }
        // OUTLIER of pairs: slot P places the outliers, slot P + 1 the kept pairs
        if (ctl != nullptr && opay != nullptr && ctl->path == SR_PATH_OUTLIER) {
            const int P = ctl->job_passes;
            if (k == P) {
                outlier_place_pairs<C>(U, S1, PU, PS1, n, (int64_t)ctl->m, opay, okb);
                return;
            }
            if (k == P + 1) {
                outlier_fill_pairs<C, WG>(U, S1, PU, PS1, n, (int64_t)ctl->m);
                return;
            }
        }
    } else {
        if (ctl != nullptr) {
            const int path = ctl->path;
            if (ft != nullptr && path == SR_PATH_FEW && k == ctl->job_passes) {
                if (fw != nullptr && ctl->few_wide) wide_place<C, WG>(U, S1 + (n - (int64_t)ctl->m), n, fw);
                else few_place<C, WG>(U, S1 + (n - (int64_t)ctl->m), n, ft, &sm);
                return;
            }
        }
    }
    if (tdesc != nullptr && k == 0 && ctl->path == SR_PATH_NEAR) near_check(const_cast<Ctl*>(ctl), tdesc, n, T);
    const PassView<S> v = resolve_merge(ctl, U, S1, PU, PS1, n, M, T, k);
    const int64_t nch = v.active ? (v.n + MC::CH - 1) / MC::CH : 0;
    if (v.cn > 0 && (int64_t)blockIdx.x >= nch) {
        // workgroups past the merge's chunks copy (the grid has at least T / CH of them)
        copy_part(v.csrc, v.cdst, v.cpsrc, v.cpdst, v.cn, (int64_t)blockIdx.x - nch, (int64_t)gridDim.x - nch);
        return;
    }
    if (!v.active) return;
    const int64_t out0 = (int64_t)blockIdx.x * MC::CH;
    if (out0 >= v.n) return;
    MC::run(sm, v.src, v.dst, v.psrc, v.pdst, v.n, v.width, v.split, out0, nullptr);
}

// Merge slot k, persistent double-buffered, co-ranks from k_partition.
// RUNS passes reuse its LDS for one-chunk merges with in-kernel co-ranks.
// NT: nontemporal window loads and output stores (arrays far beyond the
// caches; keeps the partition launch's searches cached).
template <class C, int WG, int IT, bool PAIRS, bool NT = false>
__global__ __launch_bounds__(WG) void k_merge_persist(typename C::S* U, typename C::S* S1, uint32_t* PU,
                                                      uint32_t* PS1, int64_t n, int M, int64_t T, int k,
                                                      const int64_t* co, const Ctl* ctl, const RunArea* ra,
                                                      const FewTable* ft, const unsigned long long* tdesc = nullptr,
                                                      int fan4 = 0, const WideTable* fw = nullptr,
                                                      const uint32_t* opay = nullptr, const uint32_t* okb = nullptr) {
    using MP = MergePersistent<C, WG, IT, PAIRS>;
    using MC = typename MP::MC;
    using S = typename C::S;
    __shared__ union {
        typename MP::Smem p;
        typename MC::Smem c;
    } sm;
    static_assert(sizeof(sm) >= kFewLdsBytes, "fill pass table fits the merge LDS");
    if (ctl != nullptr && ra != nullptr && ctl->path == SR_PATH_RUNS) {
        runs_merge_persist<MC, S>(sm.p.b, ra, U, S1, PU, PS1, k, co);
        return;
    }
    if constexpr (PAIRS) {
        // FEW of pairs: the placed keys and payloads back into the user buffers
        if (ctl != nullptr && ft != nullptr && ctl->path == SR_PATH_FEW && k == 0) {
            copy_part(S1, U, PS1, PU, n, (int64_t)blockIdx.x, (int64_t)gridDim.x);
            return;
        }
        // OUTLIER of pairs: slot P places the outliers, slot P + 1 the kept pairs
        if (ctl != nullptr && opay != nullptr && ctl->path == SR_PATH_OUTLIER) {
            const int P = ctl->job_passes;
            if (k == P) {
                outlier_place_pairs<C>(U, S1, PU, PS1, n, (int64_t)ctl->m, opay, okb);
                return;
            }
            if (k == P + 1) {
                outlier_fill_pairs<C, WG>(U, S1, PU, PS1, n, (int64_t)ctl->m);
                return;
            }
        }
    } else {
        if (ctl != nullptr) {
            const int path = ctl->path;
            if (ft != nullptr && path == SR_PATH_FEW && k == ctl->job_passes) {
                if (fw != nullptr && ctl->few_wide) wide_place<C, WG>(U, S1 + (n - (int64_t)ctl->m), n, fw);
                else few_place<C, WG>(U, S1 + (n - (int64_t)ctl->m), n, ft, &sm);
                return;
            }
        }
    }
    if (tdesc != nullptr && k == 0 && ctl->path == SR_PATH_NEAR) near_check(const_cast<Ctl*>(ctl), tdesc, n, T);
    const PassView<S> v = resolve_merge(ctl, U, S1, PU, PS1, n, M, T, k, fan4 != 0);
    if (v.cn > 0) copy_part(v.csrc, v.cdst, v.cpsrc, v.cpdst, v.cn, (int64_t)blockIdx.x, (int64_t)gridDim.x);
    if (!v.active || v.fan == 4) return;
    MP::template run<NT>(sm.p, v.src, v.dst, v.psrc, v.pdst, v.n, v.width, v.split, co);
}

// Four-way pass at merge slot k (general plan, fan-in four): the cut of
// every sample, then one workgroup per chunk.  Both return at once unless
// slot k is a four-way pass of the plan.
template <class C>
__global__ __launch_bounds__(256) void k_part4(typename C::S* U, typename C::S* S1, int64_t n, int M, int64_t T,
                                               int k, uint4* splits, const Ctl* ctl) {
    using S = typename C::S;
    const PassView<S> v = resolve_merge(ctl, U, S1, (uint32_t*)nullptr, (uint32_t*)nullptr, n, M, T, k, true);
    if (!v.active || v.fan != 4) return;
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= Merge4<C>::sample_slots(n, v.width)) return;
    Merge4<C>::sample(v.src, n, v.width, s, splits);
}

template <class C, bool NT>
__global__ __launch_bounds__(256) void k_merge4(typename C::S* U, typename C::S* S1, int64_t n, int M, int64_t T,
                                                int k, const uint4* splits, const Ctl* ctl) {
    using S = typename C::S;
    static_assert(Merge4<C>::WG == 256, "launch shape");
    __shared__ typename Merge4<C>::Smem sm;
    const PassView<S> v = resolve_merge(ctl, U, S1, (uint32_t*)nullptr, (uint32_t*)nullptr, n, M, T, k, true);
    if (!v.active || v.fan != 4) return;
    Merge4<C>::template chunk<NT>(sm, v.src, v.dst, n, v.width, (int64_t)blockIdx.x, splits);
}

// --------------------------------------------------------------- outliers
// Nearly-sorted input (the k-exchange class of Sec. 2, tied to the Rem
// measure: the fewest keys whose removal leaves a sorted sequence).  Three
// launches after the probe chose OUTLIER:
//   k_classify  tile t (kClsTC keys plus kClsH halo keys on each side) in LDS:
//               repeatedly drop keys at descents among the keys still kept --
//               the larger key of a descent when its removal restores the
//               order, else the smaller, else both -- until no descent is
//               left, so the tile's kept keys are sorted.  Writes a kept bit
//               mask, the kept count and the first/last kept key per tile.
//   k_verify    (one workgroup) the kept keys form one sorted sequence iff
//               no tile's first kept key is below the last kept key of the
//               nearest earlier tile that kept any; prefix of the counts;
//               sets the job (OUTLIER with m outliers if the joins hold and
//               m <= n/2, else GENERAL -- U is still untouched).
//   k_scatter   kept keys to S1[0, n-m) in input order, outliers to
//               S1[n-m, n) (from the end backwards).
template <class C>
__global__ __launch_bounds__(kClsWG) void k_classify(const typename C::S* keys, int64_t n, Ctl* ctl,
                                                     unsigned int* flags, unsigned long long* tfirst,
                                                     unsigned long long* tlast, unsigned long long* tcount,
                                                     int runs_ok, RunTile* rdesc, FewTable* ft,
                                                     typename C::S* s1, WideTable* fw, unsigned int* fewm) {
    using U = typename C::U;
    // the outlier window and the few-unique counters share the launch's LDS
    __shared__ union {
        U sk[kClsW];
        WideLds<U> wide;
        FewLds<U> few;
    } cls_lds;
    const int path = ctl->path;
    if (path == SR_PATH_FEW) {
        const int64_t f0 = (int64_t)blockIdx.x * kClsTC;
        const int64_t f1 = (f0 + kClsTC) < n ? (f0 + kClsTC) : n;
        if (fewm != nullptr) few_count_pairs<C>(keys, f0, f1, ctl, ft, fewm, blockIdx.x, gridDim.x, cls_lds.few);
        else if (fw != nullptr && ctl->few_wide) wide_count<C>(keys, n, f0, f1, ctl, fw, s1, cls_lds.wide);
        else few_count<C>(keys, n, f0, f1, ctl, ft, s1, cls_lds.few);
        return;
    }
    const bool do_runs = runs_ok && (path == SR_PATH_RUNS || (path == SR_PATH_OUTLIER && ctl->dual));
    if (path != SR_PATH_OUTLIER && !do_runs) return;
    U* sk = cls_lds.sk;
    __shared__ unsigned int kw[kClsWG], rw[kClsWG];   // per-thread kept masks, removals by others
    __shared__ int wtot[kClsWG / kWave];
    __shared__ int s_flag[2], s_both[2];
    __shared__ U s_first, s_last;
    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid / kWave;
    if (tid < 2) s_flag[tid] = s_both[tid] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x;
    const int64_t c0 = t * kClsTC;
    const int64_t c1 = (c0 + kClsTC) < n ? (c0 + kClsTC) : n;
    const int64_t w0 = c0 - kClsH > 0 ? c0 - kClsH : 0;
    const int64_t w1 = (c1 + kClsH) < n ? (c1 + kClsH) : n;
    const int wn = (int)(w1 - w0);
    {
        // all window loads in flight before the first LDS store
        typename C::S xv[kClsPer];
#pragma unroll
        for (int r = 0; r < kClsPer; ++r) {
            const int j = tid + r * kClsWG;
            if (j < wn) xv[r] = keys[w0 + j];
        }
#pragma unroll
        for (int r = 0; r < kClsPer; ++r) {
            const int j = tid + r * kClsWG;
            if (j < wn) sk[j] = C::enc(xv[r]);
        }
    }
    __syncthreads();
    if (do_runs) runscan_lds<U>(sk, n, c0, c1, w0, rdesc + t);
    if (path != SR_PATH_OUTLIER) return;

    // Removal rounds on a register copy: thread tid owns window positions
    // bj .. bj+16 (bit r of km: position bj + r still kept) and their keys.
    // In a round every kept key q is compared with the next kept key j; at a
    // descent the larger key goes if dropping it restores the order with the
    // previous kept key, else the smaller if that restores it with the kept
    // key after j, else both.  A register sweep over the thread's own
    // positions finds its descents; only at those (few, on nearly sorted
    // input) are the neighbours looked up, by position, in the keys in LDS,
    // across the thread's ends through the kept masks the threads publish in
    // LDS (kw); a removal of a position another thread owns goes to that
    // thread's word rw by an LDS atomic OR.  All decisions
    // of a round use the masks of the previous round, so the result does not
    // depend on thread timing.  A round without removals means the kept keys
    // are sorted.
    const int bj = tid * kClsPer;
    U key[kClsPer];
    unsigned int km = 0u;
#pragma unroll
    for (int r = 0; r < kClsPer; ++r) {
        key[r] = sk[bj + r];  // positions >= wn are never kept
        km |= (bj + r < wn ? 1u : 0u) << r;
    }
    rw[tid] = 0u;
    const int uend = (wn + kClsPer - 1) / kClsPer;  // threads owning window positions
    bool converged = false;
    for (int iter = 0; iter <= kClsMaxIter; ++iter) {
        kw[tid] = km;
        __syncthreads();
        int r1 = -1, r2 = -1;  // first two kept positions after this thread's
        for (int u = tid + 1; km != 0u && u < uend && r2 < 0; ++u) {
            unsigned int w = kw[u];
            while (w != 0u && r2 < 0) {
                const int pos = u * kClsPer + __builtin_ctz(w);
                w &= w - 1u;
                if (r1 < 0) r1 = pos;
                else r2 = pos;
            }
        }
        int l1 = -1;  // last kept position before this thread's
        for (int u = tid - 1; km != 0u && u >= 0 && l1 < 0; --u) {
            const unsigned int w = kw[u];
            if (w != 0u) l1 = u * kClsPer + 31 - __builtin_clz(w);
        }
        // backward sweep: the descents, kept positions r whose next kept key
        // is smaller (the rare case; everything else of a round is skipped
        // for positions without one)
        unsigned int desc = 0u;
        {
            bool h = r1 >= 0;
            U k1 = h ? sk[r1] : (U)0;
#pragma unroll
            for (int r = kClsPer - 1; r >= 0; --r) {
                if ((km >> r) & 1u) {
                    desc |= (h && key[r] > k1 ? 1u : 0u) << r;
                    k1 = key[r];
                    h = true;
                }
            }
        }
        // the removals at each descent, from the previous kept key and the
        // next two kept keys (read from LDS by position)
        unsigned int own_rem = 0u;
        const bool rem = desc != 0u;
        bool both = false;
        while (desc != 0u) {
            const int r = __builtin_ctz(desc);
            desc &= desc - 1u;
            const unsigned int above = r + 1 < kClsPer ? km >> (r + 1) : 0u;
            const unsigned int below = km & ((1u << r) - 1u);
            const int na = __builtin_popcount(above);
            const int q1 = na >= 1 ? bj + r + 1 + __builtin_ctz(above) : r1;
            const int q2 = na >= 2 ? bj + r + 1 + __builtin_ctz(above & (above - 1u)) : (na == 1 ? r1 : r2);
            const U kr = sk[bj + r], n1 = sk[q1];
            const bool h2 = q2 >= 0;
            const bool hp = below != 0u || l1 >= 0;
            const U pk = below != 0u ? sk[bj + 31 - __builtin_clz(below)] : (l1 >= 0 ? sk[l1] : (U)0);
            bool ra = !hp || pk <= n1;
            bool rb = !ra && (!h2 || kr <= sk[q2]);
            if (!ra && !rb) {
                ra = rb = true;
                both = true;
            }
            if (ra) own_rem |= 1u << r;
            if (rb) {
                if (na >= 1) own_rem |= 1u << (q1 - bj);
                else atomicOr(&rw[r1 / kClsPer], 1u << (r1 % kClsPer));
            }
        }
        if (rem) s_flag[iter & 1] = 1;
        if (both) s_both[iter & 1] = 1;
        __syncthreads();
        const bool any = s_flag[iter & 1] != 0;
        const bool deep = s_both[iter & 1] != 0;
        if (tid == 0) {
            s_flag[(iter + 1) & 1] = 0;
            s_both[(iter + 1) & 1] = 0;
        }
        km &= ~(own_rem | rw[tid]);
        rw[tid] = 0u;
        if (!any) {
            converged = true;
            break;
        }
        // a descent that no single removal repairs, still there after
        // kClsDeepIter rounds, is a boundary between overlapping runs being
        // peeled key by key: the tile is not outlier-shaped
        if (deep && iter >= kClsDeepIter) break;
    }
    // the final kept masks, for the core pass below
    kw[tid] = km;
    __syncthreads();

    // the tile's core [c0, c1): this thread's 16 core positions as a bit
    // mask cut out of the owners' kept masks, kept ranks, first and last
    // kept key
    const int cs = (int)(c0 - w0), ce = (int)(c1 - w0);
    constexpr int CP = kClsTC / kClsWG;
    static_assert(CP == 16 && kClsPer >= CP, "a core stretch spans at most two owners' masks");
    unsigned int bits;
    {
        const int p0 = cs + tid * CP;
        const int u = p0 / kClsPer, o = p0 - u * kClsPer;
        unsigned int m = kw[u] >> o;
        if (u + 1 < kClsWG) m |= kw[u + 1] << (kClsPer - o);
        const int nv = ce - p0;  // core positions of this thread
        bits = nv <= 0 ? 0u : (m & (nv >= CP ? 0xFFFFu : ((1u << nv) - 1u)));
    }
    const int kl = __builtin_popcount(bits);
    int x = kl;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wtot[wave] = x;
    __syncthreads();
    int koff = x - kl, kc = 0;
#pragma unroll
    for (int w = 0; w < kClsWG / kWave; ++w) {
        kc += wtot[w];
        if (w < wave) koff += wtot[w];
    }
    if (kl > 0) {
        const int p0 = cs + tid * CP;
        if (koff == 0) s_first = sk[p0 + __builtin_ctz(bits)];
        if (koff + kl == kc) s_last = sk[p0 + 31 - __builtin_clz(bits)];
    }
    __syncthreads();

    // publish: kept flags of the core as a bit mask (bit i of word w = core key
    // 32w + i), the kept count and the first/last kept key of the tile
    {
        const unsigned int other = (unsigned int)__shfl_xor((int)bits, 1);
        if ((tid & 1) == 0) flags[t * (kClsTC / 32) + tid / 2] = bits | (other << CP);
    }
    if (tid == 0) {
        if (!converged) atomicOr(&ctl->bad_join, 1u);
        const int64_t vs = ver_slot(t);
        tcount[vs] = (unsigned long long)kc;
        tfirst[vs] = kc > 0 ? (unsigned long long)s_first : 0ull;
        tlast[vs] = kc > 0 ? (unsigned long long)s_last : 0ull;
    }
}

// Scatter of the outlier path: tile t's kept keys go to S1[kpref[t] + kept
// rank inside the tile], its outliers to S1[n-1-(outliers before)], from the
// kept bit masks of k_classify and the tile offsets of k_verify.  Keys are
// assigned striped (key e of the tile to thread e mod 256), so loads and the
// mostly consecutive kept stores coalesce; a key's kept rank is the popcount
// prefix of the tile's mask words (scanned in LDS) plus the bits below it.
// The same launch reverses the descending runs of the RUNS job.
template <class C>
__global__ __launch_bounds__(kClsWG) void k_scatter(typename C::S* keys, int64_t n, const Ctl* ctl,
                                                    typename C::S* s1, const unsigned int* flags,
                                                    const unsigned long long* kpref_t, const RunArea* ra,
                                                    uint32_t* pay, uint32_t* spay, const FewTable* ft,
                                                    const unsigned int* fewm, uint32_t* opay, uint32_t* okb) {
    using S = typename C::S;
    constexpr int CP = kClsTC / kClsWG;
    constexpr int NW = kClsTC / 32;  // mask words per tile
    static_assert(NW <= kClsWG, "one word per thread in the scan");
    const int path = ctl->path;
    if (path == SR_PATH_RUNS && ra != nullptr) {
        runs_reverse<S>(keys, pay, ra);
        return;
    }
    if (path == SR_PATH_FEW && fewm != nullptr) {
        few_scatter_pairs<C>(keys, pay, s1, spay, n, ft, fewm, blockIdx.x, gridDim.x);
        return;
    }
    if (path != SR_PATH_OUTLIER) return;
    __shared__ unsigned int sw[NW];
    __shared__ int spre[NW];
    __shared__ int wtot[kClsWG / kWave];
    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid / kWave;
    const int64_t t = blockIdx.x;
    const int64_t c0 = t * kClsTC;
    const int64_t c1 = (c0 + kClsTC) < n ? (c0 + kClsTC) : n;
    S x[CP];
#pragma unroll
    for (int r = 0; r < CP; ++r) {
        const int64_t g = c0 + r * kClsWG + tid;
        if (g < c1) x[r] = keys[g];
    }
    const unsigned int w = tid < NW ? flags[t * NW + tid] : 0u;
    if (tid < NW) sw[tid] = w;
    const int pc = __builtin_popcount(w);
    int xs = pc;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(xs, d);
        if (lane >= d) xs += y;
    }
    if (lane == kWave - 1) wtot[wave] = xs;
    __syncthreads();
    int pre = xs - pc;
    for (int q = 0; q < wave; ++q) pre += wtot[q];
    if (tid < NW) spre[tid] = pre;
    __syncthreads();
    const int64_t kpref = (int64_t)kpref_t[t];
    // pairs: outliers in input order with their index, payload and kept-before
    // count (keys only: from the end backwards)
    const bool pj = opay != nullptr;
    const int64_t mj = pj ? (int64_t)ctl->m : 0;
#pragma unroll
    for (int r = 0; r < CP; ++r) {
        const int li = r * kClsWG + tid;
        const int64_t g = c0 + li;
        if (g < c1) {
            const unsigned int word = sw[li >> 5];
            const int bit = li & 31;
            const int kr = spre[li >> 5] + __builtin_popcount(word & ((1u << bit) - 1u));
            const bool keep = ((word >> bit) & 1u) != 0u;
            const int64_t jj = (c0 - kpref) + (li - kr);  // outliers before it
            int64_t pos;
            if (keep) pos = kpref + kr;
            else pos = pj ? n - mj + jj : n - 1 - jj;
            if (pos >= 0 && pos < n) {
                s1[pos] = x[r];
                if (pj) {
                    if (keep) {
                        spay[pos] = pay[g];
                    } else if (jj < mj) {
                        spay[pos] = (uint32_t)jj;
                        opay[jj] = pay[g];
                        okb[jj] = (uint32_t)(kpref + kr);
                    }
                }
            }
        }
    }
}

// Verification and job of the outlier path (one workgroup, after classify).
// The kept keys form one sorted sequence iff every tile's first kept key is
// at least the last kept key of the nearest earlier tile that kept any.
// Then the job is OUTLIER with m = n - kept outliers when m <= n/2;
// otherwise GENERAL (the user buffer has not been written yet).
//
// With runs_ok the same workgroup then plans the RUNS job (run_plan) when the
// probe chose RUNS, or beside an OUTLIER job (unless OUTLIER was forced); the
// cheaper of the two is kept.
__device__ void verify_outliers(Ctl* ctl, int64_t n, int64_t ntiles, const unsigned long long* tfirst,
                                const unsigned long long* tlast, const unsigned long long* tcount,
                                unsigned long long* kpref_t, int64_t T_sort, double* ocost, int pairs, int M);

template <class C>
__global__ __launch_bounds__(kVerWG) void k_verify(Ctl* ctl, int64_t n, int64_t ntiles, const unsigned long long* tfirst,
                                                   const unsigned long long* tlast, const unsigned long long* tcount,
                                                   unsigned long long* kpref_t, int64_t T_sort,
                                                   const typename C::S* keys, const RunTile* rdesc, RunArea* ra,
                                                   int runs_ok, int64_t merge_ch, int M, FewTable* ft,
                                                   WideTable* fw, unsigned int* fewm, int out_pairs) {
    const int path0 = ctl->path;
    if (path0 == SR_PATH_FEW) {
        if (fewm != nullptr) few_plan_pairs(ctl, n, ft, fewm, ntiles);
        else if (fw != nullptr && ctl->few_wide) wide_plan(ctl, n, fw, T_sort);
        else few_plan(ctl, n, ft, T_sort);
        return;
    }
    const bool want_runs = runs_ok && (path0 == SR_PATH_RUNS || (path0 == SR_PATH_OUTLIER && ctl->dual));
    __shared__ double s_ocost;
    if (path0 == SR_PATH_OUTLIER)
        verify_outliers(ctl, n, ntiles, tfirst, tlast, tcount, kpref_t, T_sort, &s_ocost, out_pairs, M);
    else if (path0 == SR_PATH_RUNS && threadIdx.x == 0) s_ocost = 1e300;
    __syncthreads();
    // a run plan cannot beat an outlier job of about two passes
    if (want_runs && s_ocost > 2.5)
        run_plan<C>(ctl, n, ntiles, keys, rdesc, ra, (int)(T_sort / kClsTC), merge_ch, M, s_ocost,
                    path0 == SR_PATH_RUNS);
}

__device__ void verify_outliers(Ctl* ctl, int64_t n, int64_t ntiles, const unsigned long long* tfirst,
                                const unsigned long long* tlast, const unsigned long long* tcount,
                                unsigned long long* kpref_t, int64_t T_sort, double* ocost, int pairs, int M) {
    // Rounds of kVerWG x kVerQ consecutive tiles (each thread kVerQ
    // consecutive ones, read from the ver_slot layout so that every load of a
    // wavefront is one coalesced row): the kept prefix
    // continues a running base, and each tile's first kept key is checked
    // against the last kept key of the nearest earlier tile that kept any
    // (in this thread, in an earlier thread of the round -- a max-scan of
    // thread indices -- or in an earlier round).
    constexpr int Q = kVerQ;
    __shared__ long long s_w[kVerWG / kWave];
    __shared__ unsigned long long s_lastk[kVerWG];
    __shared__ unsigned long long s_base, s_carry_key;
    __shared__ int s_carry_has, s_bad;
    const int tid = threadIdx.x;
    const int lane = (int)__lane_id();
    const int wave = tid / kWave;
    if (tid == 0) {
        s_bad = 0;
        s_base = 0;
        s_carry_has = 0;
        s_carry_key = 0;
    }
    __syncthreads();
    for (int64_t r0 = 0; r0 < ntiles; r0 += (int64_t)kVerWG * Q) {
        const int64_t tb = r0 + (int64_t)tid * Q;
        unsigned long long cv[Q], fv[Q], lv[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const bool ok = tb + q < ntiles;
            const int64_t vs = r0 + (int64_t)q * kVerWG + tid;  // ver_slot(tb + q)
            cv[q] = ok ? tcount[vs] : 0ull;
            fv[q] = ok ? tfirst[vs] : 0ull;
            lv[q] = ok ? tlast[vs] : 0ull;
        }
        unsigned long long kept = 0, last = 0, first = 0;
        bool has = false, bad = false;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (cv[q] == 0) continue;
            if (has && fv[q] < last) bad = true;
            if (!has) first = fv[q];
            has = true;
            last = lv[q];
            kept += cv[q];
        }
        long long tot;
        long long pre = wg_scan_excl((long long)kept, s_w, tot) + (long long)s_base;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            if (tb + q < ntiles) kpref_t[tb + q] = (unsigned long long)pre;
            pre += (long long)cv[q];
        }
        // nearest earlier thread of this round that kept any key
        s_lastk[tid] = last;
        int hi = has ? tid : -1;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(hi, o);
            if (lane >= o) hi = y > hi ? y : hi;
        }
        __syncthreads();
        if (lane == kWave - 1) s_w[wave] = hi;
        __syncthreads();
        int prev = __shfl_up(hi, 1);
        if (lane == 0) prev = -1;
        int rmax = -1;
        for (int w = 0; w < kVerWG / kWave; ++w) {
            const int v = (int)s_w[w];
            if (w < wave) prev = v > prev ? v : prev;
            rmax = v > rmax ? v : rmax;
        }
        if (has) {
            if (prev >= 0) {
                if (first < s_lastk[prev]) bad = true;
            } else if (s_carry_has && first < s_carry_key) {
                bad = true;
            }
        }
        if (bad) s_bad = 1;
        __syncthreads();
        if (tid == 0) {
            s_base += (unsigned long long)tot;
            if (rmax >= 0) {
                s_carry_has = 1;
                s_carry_key = s_lastk[rmax];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        const unsigned long long total = s_base;
        const bool fail = s_bad != 0 || ld_agent(&ctl->bad_join) != 0 || total > (unsigned long long)n;
        const int64_t m = n - (int64_t)total;
        // pairs: at most n/4 outliers, and merge slots for the job's passes
        // and the two placement passes
        const int jp0 = ceil_log2_dev((m + T_sort - 1) / T_sort);
        if (fail || m > (pairs ? n / 4 : n / 2) || (pairs && jp0 + 2 > M)) {
            ctl->path = SR_PATH_GENERAL;
            ctl->m = 0;
            ctl->job_passes = 0;
            *ocost = 1e300;
        } else {
            const int jp = ceil_log2_dev((m + T_sort - 1) / T_sort);
            ctl->m = (unsigned long long)m;
            ctl->job_passes = jp;
            // scatter (1) + outlier sort (1 + jp passes over m) + final merge (1)
            *ocost = 2.0 + (1.0 + jp) * (double)m / (double)n;
        }
        ctl->n_kept = total;
        ctl->reserved[2] = fail ? 1 : 0;
        ctl->reserved[3] = (unsigned long long)m;
        ctl->ticket2 = 0;
        ctl->bad_join = 0;
    }
}

// Probe.  The array's neighbour pairs (i, i+1) are cut into probe tiles of
// kProbeTile pairs; a capped grid walks them grid-stride.  Before each tile a
// workgroup checks the global "mixed" flag and stops once some workgroup has
// seen both an ascent and a descent (then the array is neither sorted nor
// reversed).  Each workgroup first samples kProbeSample pairs at an evenly
// spread position for the descent-rate estimate, and skips the tiles at once
// when its own sample holds both.  The last workgroup to
// finish turns the counters into the plan and clears them.
template <class C>
__global__ __launch_bounds__(kProbeWG) void k_probe(const typename C::S* keys, int64_t n, Ctl* ctl,
                                                    unsigned long long* slots, int jobs_ok, int runs_pmax,
                                                    FewTable* ft, WideTable* fw) {
    using U = typename C::U;
    using S = typename C::S;
    constexpr int VN = 16 / sizeof(S);
    constexpr int Q = (int)(kProbeTile / (kProbeWG * VN));  // vectors per thread per tile
    __shared__ unsigned long long red[5][kProbeWG / kWave];
    __shared__ int skip;
    __shared__ unsigned int last;
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    const int64_t npairs = n - 1;
    const int64_t ntiles = (npairs + kProbeTile - 1) / kProbeTile;

    // sample: kProbeSample pairs around tile blockIdx * ntiles / gridDim, at an
    // offset scattered by a multiplicative hash of the workgroup index (so
    // that boundaries of inputs built on powers of two, such as tile-aligned
    // ones, are hit as often as any others)
    // sd: 21-bit fields (sums over at most 1024 samples of 256 pairs fit):
    // sampled descents, turning points (two strict neighbouring pairs that
    // point different ways), and -- added per workgroup below -- the
    // workgroup's turnings capped at 2, which counts a disordered sample
    // window like one piece rather than by its many turnings.
    // sp: 21-bit fields: pairs, equal pairs, and hard valleys -- valleys
    // x > y < z (or x > y = z < u) with x >= z (x >= u), where the stretches
    // on the two sides overlap in value, so that a run plan cannot join the
    // runs they end and start (kept only for windows with few turnings,
    // below).
    // sdd: deep drops -- descents x > y between two ascending stretches
    // (w <= x, y <= z) that removing x or y alone does not repair (w > y and
    // x > z), with the stretch after them still below x kDropDepth keys on:
    // a boundary between runs that overlap further than the outlier split
    // can peel off in its rounds (a short displaced block is not one).
    unsigned long long sd = 0, sp = 0, sdd = 0;
    bool seen_desc = false, seen_asc = false;
    {
        const int64_t t = (int64_t)blockIdx.x * ntiles / gridDim.x;
        int64_t b0 = t * kProbeTile + (int64_t)((blockIdx.x * 2654435761u) % (unsigned)kProbeTile) - kProbeSample / 2;
        b0 = std::max<int64_t>(0, std::min<int64_t>(b0, npairs - kProbeSample));
        const int64_t s1 = std::min<int64_t>(b0 + kProbeSample, npairs);
        for (int64_t i = b0 + tid; i < s1; i += kProbeWG) {
            // every key the tests below may look at, loaded together (indexes
            // clamped into the array; a test uses a key only where its index
            // was in range), so that the sample costs one round trip
            const int64_t last = n - 1;
            const U w = C::enc(keys[i > 0 ? i - 1 : 0]);
            const U x = C::enc(keys[i]), y = C::enc(keys[i + 1]);
            const U z = C::enc(keys[i + 2 < last ? i + 2 : last]);
            const U u = C::enc(keys[i + 3 < last ? i + 3 : last]);
            const U far = C::enc(keys[i + 1 + kDropDepth < last ? i + 1 + kDropDepth : last]);
            seen_desc |= x > y;
            seen_asc |= x < y;
            sd += x > y ? 1 : 0;
            sp += x == y ? (1ull << kSampleField) + 1 : 1;
            if (i + 1 < npairs) {
                if ((x > y && y < z) || (x < y && y > z)) sd += 1ull << kSampleField;
                if (x > y && y < z && x >= z) {
                    sp += 1ull << (2 * kSampleField);
                } else if (x > y && y == z && i + 2 < npairs) {  // a valley on a plateau of two
                    if (y < u && x >= u) sp += 1ull << (2 * kSampleField);
                }
                if (x > y && y <= z && x > z && i > 0 && i + 1 + kDropDepth < n)
                    sdd += (w <= x && w > y && far < x) ? 1 : 0;
            }
        }
    }
    // a workgroup whose own sample holds an ascent and a descent already
    // knows that the array is mixed: it raises the flag and skips the counts
    const int any_desc = __syncthreads_or((int)seen_desc);
    const int any_asc = __syncthreads_or((int)seen_asc);
    const bool sample_mixed = any_desc != 0 && any_asc != 0;
    // (the atomic's result is not waited for: raising the flag costs no round trip)
    if (sample_mixed && tid == 0) atomicOr(&ctl->mixed, 1u);
    unsigned long long d = 0, a = 0;
    const bool vec_ok = aligned16(keys);
    for (int64_t t = blockIdx.x; !sample_mixed && t < ntiles; t += gridDim.x) {
        __syncthreads();
        if (tid == 0) skip = ld_agent(&ctl->mixed) != 0;
        __syncthreads();
        if (skip) break;
        const int64_t b0 = t * kProbeTile;
        const int64_t b1 = std::min<int64_t>(b0 + kProbeTile, npairs);
        unsigned long long td = 0, ta = 0;
        if (vec_ok && b1 - b0 == kProbeTile) {
            // thread owns vectors q: keys [b0 + (tid + q*WG)*VN, +VN) and the key after them
            V16<S> x[Q];
            S nx[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int64_t e = b0 + (int64_t)(tid + q * kProbeWG) * VN;
                x[q] = *reinterpret_cast<const V16<S>*>(keys + e);
                nx[q] = keys[e + VN];  // e + VN <= b1 <= n - 1
            }
#pragma unroll
            for (int q = 0; q < Q; ++q) {
#pragma unroll
                for (int j = 0; j < VN; ++j) {
                    const U u = C::enc(x[q].v[j]);
                    const U w = C::enc(j + 1 < VN ? x[q].v[j + 1] : nx[q]);
                    td += u > w ? 1 : 0;
                    ta += u < w ? 1 : 0;
                }
            }
        } else {
            for (int64_t i = b0 + tid; i < b1; i += kProbeWG) {
                const U x = C::enc(keys[i]), y = C::enc(keys[i + 1]);
                td += x > y ? 1 : 0;
                ta += x < y ? 1 : 0;
            }
        }
        td = wave_sum(td);
        ta = wave_sum(ta);
        __syncthreads();
        if (__lane_id() == 0) {
            red[0][wave] = td;
            red[1][wave] = ta;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long sdn = 0, san = 0;
            for (int w = 0; w < kProbeWG / kWave; ++w) {
                sdn += red[0][w];
                san += red[1][w];
            }
            d += sdn;
            a += san;
            if (d && a) {
                atomicOr(&ctl->mixed, 1u);
                skip = 1;
            }
        }
    }
    __syncthreads();
    sd = wave_sum(sd);
    sp = wave_sum(sp);
    sdd = wave_sum(sdd);
    if (__lane_id() == 0) {
        red[2][wave] = sd;
        red[3][wave] = sp;
        red[4][wave] = sdd;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long t2 = 0, t3 = 0, t4 = 0;
        for (int w = 0; w < kProbeWG / kWave; ++w) {
            t2 += red[2][w];
            t3 += red[3][w];
            t4 += red[4][w];
        }
        const unsigned long long wturn = (t2 >> kSampleField) & kSampleMask;
        t2 += (wturn < 2 ? wturn : 2ull) << (2 * kSampleField);
        // hard valleys count only in windows that look like runs (at most two
        // turnings); a disordered window becomes one dense piece of a plan
        if (wturn > 2) t3 &= (1ull << (2 * kSampleField)) - 1;
        // per-workgroup slot (plain stores, no contention), then one ticket;
        // the ascent count (at most n <= 2^36 over all slots) shares its word
        // with the deep drops (bits kAscBits and up)
        slots[blockIdx.x * 4 + 0] = d;
        slots[blockIdx.x * 4 + 1] = a + (t4 << kAscBits);
        slots[blockIdx.x * 4 + 2] = t2;
        slots[blockIdx.x * 4 + 3] = t3;
        // release: the slot is written back to memory before the ticket moves
        // (no acquire here: nothing this workgroup reads later depends on it)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        // two-level ticket: groups of kProbeGroup workgroups share a counter
        // (each on its own 256-byte line), the last of a group bumps ctl->ticket
        const unsigned int groups = (gridDim.x + kProbeGroup - 1) / kProbeGroup;
        const unsigned int g = blockIdx.x / kProbeGroup;
        const unsigned int in_g = g + 1 < groups ? kProbeGroup : gridDim.x - g * kProbeGroup;
        unsigned int* gc = reinterpret_cast<unsigned int*>(slots + kProbeMaxGrid * 4) + g * 64;
        last = false;
        if (atomicAdd(gc, 1u) == in_g - 1) {
            st_agent(gc, 0u);  // reset for the next call (no other workgroup of this group touches it again)
            last = atomicAdd(&ctl->ticket, 1u) == groups - 1;
        }
    }
    __syncthreads();
    if (last) {
        // acquire: the slots of every workgroup, released before their tickets
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unsigned long long acc[4] = {0, 0, 0, 0};
        for (int g = tid; g < (int)gridDim.x; g += kProbeWG)
            for (int q = 0; q < 4; ++q) acc[q] += __hip_atomic_load(&slots[g * 4 + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int q = 0; q < 4; ++q) acc[q] = wave_sum(acc[q]);
        __syncthreads();
        if (__lane_id() == 0)
            for (int q = 0; q < 4; ++q) red[q][wave] = acc[q];
        __syncthreads();
    }
    __shared__ int s_path, s_force, s_dual, s_force_near;
    __shared__ unsigned long long s_desc, s_asc;
    if (last && tid == 0) {
        unsigned long long tot[4] = {0, 0, 0, 0};
        for (int w = 0; w < kProbeWG / kWave; ++w)
            for (int q = 0; q < 4; ++q) tot[q] += red[q][w];
        const unsigned long long desc = tot[0];
        const unsigned long long asc = tot[1] & ((1ull << kAscBits) - 1);
        const unsigned long long sdrop = tot[1] >> kAscBits;
        const unsigned long long sdesc = tot[2] & kSampleMask;
        const unsigned long long sturn = (tot[2] >> kSampleField) & kSampleMask;
        const unsigned long long scap = tot[2] >> (2 * kSampleField);
        const unsigned long long spairs = tot[3] & kSampleMask;
        const unsigned long long sequal = (tot[3] >> kSampleField) & kSampleMask;
        const unsigned long long shard = tot[3] >> (2 * kSampleField);
        const bool mixed = ld_agent(&ctl->mixed) != 0;
        const bool outlier_ok = (jobs_ok & 1) != 0, runs_ok = (jobs_ok & 2) != 0, few_ok = (jobs_ok & 4) != 0;
        // a run plan is worth a scan when turnings are rare in the sample, the
        // whole array would not hold clearly more run boundaries (dense
        // windows counted as pieces) than a plan can, and the leaves that the
        // hard valleys alone force (scaled to the array; trusted from two
        // sampled ones on) leave merge passes enough to save over the general
        // path to pay for the scan and plan
        const double hard = (double)shard * (double)npairs / (double)(spairs ? spairs : 1);
        const bool runs_pay = shard < 2 || ceil_log2_dev((int64_t)hard + 1) <= runs_pmax;
        const bool runs_like = runs_ok && sturn * 64 <= spairs && runs_pay &&
                               (double)scap * (double)npairs <= (double)spairs * (2.0 * kRunMaxBase);
        // the outlier split repairs descents a few keys deep; when most
        // sampled descents are deep drops it would only fall back
        const bool drops = sdrop * 2 > sdesc;
        int path;
        if (!mixed && desc == 0) path = SR_PATH_SORTED;
        else if (!mixed && asc == 0) path = SR_PATH_REVERSED;
        else if (outlier_ok && sdesc * 16 <= spairs && !drops) path = SR_PATH_OUTLIER;
        // few distinct values: equal neighbours at a rate of at least 1/16384
        // (about 1/v for v values); confirmed by the sample below
        else if (few_ok && sequal * 16384 >= spairs) path = SR_PATH_FEW;
        else if (runs_like) path = SR_PATH_RUNS;
        else path = SR_PATH_GENERAL;
        const int force = ctl->force_path;
        if (force == SR_PATH_GENERAL || (force == SR_PATH_OUTLIER && outlier_ok) || (force == SR_PATH_RUNS && runs_ok) ||
            (force == SR_PATH_FEW && few_ok))
            path = force;
        // fallback if the sample shows too many distinct keys
        s_path = path == SR_PATH_FEW && force != SR_PATH_FEW
                     ? -(runs_like ? SR_PATH_RUNS : SR_PATH_GENERAL) - 10
                     : path;
        s_force = force == SR_PATH_FEW;
        // forcing GENERAL rules NEAR out; forcing NEAR tries it on any input
        s_force_near = force == SR_PATH_GENERAL ? -1 : force == SR_PATH_NEAR ? 1 : 0;
        s_dual = path == SR_PATH_OUTLIER && force != SR_PATH_OUTLIER && runs_like;
        s_desc = desc;
        s_asc = asc;
    }
    if (last) {
        __syncthreads();
        int path = s_path;
        int few_wide = 0;
        if (path == SR_PATH_FEW || path <= -10) {
            // FEW: the distinct values among kFewSample evenly spread samples
            // become the splitters if there are at most kFewMax of them.  They
            // are counted in an LDS hash set (open addressing; a slot holds
            // the encoded key + 1, 0 for empty, and is claimed by one
            // compare-and-swap per probe, so no lane ever waits on another;
            // the 64-bit largest code, whose key + 1 wraps to 0, is a flag)
            // and, when few enough, sorted by one wavefront.  A forced FEW
            // with more distinct samples takes the kFewMax smallest, from the
            // sample sorted by the tile sorter.
            constexpr int PER = kFewSample / kProbeWG;
            constexpr int HB = 11, HS = 1 << HB;
            static_assert(HS >= 2 * kFewSample, "the hash set stays at most half full");
            static_assert(kFewMax <= kWave, "one splitter per lane");
            using FS = TileSort<C, kProbeWG, kFewSample / kProbeWG, false>;
            using FSW = TileSort<C, kProbeWG, kWideMax / kProbeWG, false>;
            static_assert(FS::T == kFewSample && FSW::T == kWideMax, "one sample tile");
            constexpr int WB = 8;  // wide sample keys per thread per round
            static_assert(kWideHash >= kWideMax + kProbeWG * WB + 1, "inserts stop before the wide hash set fills");
            // the phases run one after another, so their LDS is shared
            __shared__ union {
                unsigned long long hset[HS];
                U wh[kWideHash];
                typename FSW::Smem fsw;
                typename FS::Smem fsm;
            } few_lds;
            unsigned long long* hset = few_lds.hset;
            __shared__ unsigned long long hval[kFewMax];
            __shared__ int s_dist, s_top, s_nv, s_full;
            for (int i = tid; i < HS; i += kProbeWG) hset[i] = 0ull;
            if (tid == 0) {
                s_dist = 0;
                s_top = 0;
                s_nv = 0;
            }
            U sv[PER];
#pragma unroll
            for (int r = 0; r < PER; ++r) sv[r] = C::enc(keys[strat_pos(tid * PER + r, n, kFewSample)]);
            __syncthreads();
#pragma unroll
            for (int r = 0; r < PER; ++r) {
                const unsigned long long code = (unsigned long long)sv[r] + 1ull;
                if (code == 0ull) {
                    s_top = 1;
                    continue;
                }
                unsigned int h = (unsigned int)((code * 0x9E3779B97F4A7C15ull) >> (64 - HB));
                for (;;) {  // ends: at most kFewSample of the HS slots are ever taken
                    const unsigned long long old = atomicCAS(&hset[h], 0ull, code);
                    if (old == 0ull) {
                        atomicAdd(&s_dist, 1);
                        break;
                    }
                    if (old == code) break;
                    h = (h + 1u) & (HS - 1);
                }
            }
            __syncthreads();
            const int total = s_dist + s_top;
            int ns = -1;  // splitters taken; -1: not few-unique
            if (total <= kFewMax) {
                for (int i = tid; i < HS; i += kProbeWG) {
                    const unsigned long long c = hset[i];
                    if (c != 0ull) hval[atomicAdd(&s_nv, 1)] = c - 1ull;
                }
                __syncthreads();
                if (wave == 0) {
                    // padding with the largest code keeps the real values first
                    const int lane = (int)__lane_id();
                    U v[1] = {lane < s_dist ? (U)hval[lane] : (U)~(U)0};
                    wave_sort(v);
                    if (lane < total) ft->split[lane] = (unsigned long long)v[0];
                }
                ns = total;
            } else if (fw != nullptr && total <= kFewSample * 15 / 16) {
                // (more than 960 distinct values among 1024 samples: the
                // array holds far more than kWideMax values -- 4096 values,
                // however their frequencies, show at most about 906 +- 9)
                // wide: kWideSample keys in rounds of WB per thread into a
                // larger hash set of codes (code + 1, as above), until more
                // than kWideMax distinct ones are seen; a round starts only
                // while at most kWideMax are known, so the set never fills.
                // Up to kWideMax values are then sorted as one tile.
                __syncthreads();  // the small hash set is dead from here
                U* wh = few_lds.wh;
                for (int i = tid; i < kWideHash; i += kProbeWG) wh[i] = (U)0;
                if (tid == 0) {
                    s_dist = 0;
                    s_top = 0;
                    s_nv = 0;
                    s_full = 0;
                }
                __syncthreads();
                constexpr int PERW = kWideSample / kProbeWG;
                for (int b0 = 0; b0 < PERW; b0 += WB) {
                    if (s_full) break;
                    U sv2[WB];
#pragma unroll
                    for (int r = 0; r < WB; ++r)
                        sv2[r] = C::enc(keys[strat_pos(tid * PERW + b0 + r, n, kWideSample)]);
#pragma unroll
                    for (int r = 0; r < WB; ++r) {
                        const U code = (U)(sv2[r] + (U)1);
                        if (code == (U)0) {
                            s_top = 1;
                            continue;
                        }
                        unsigned int h =
                            (unsigned int)(((unsigned long long)code * 0x9E3779B97F4A7C15ull) >> 51) & (kWideHash - 1);
                        for (;;) {  // ends: fewer than kWideHash distinct codes are ever inserted
                            const U old = atomicCAS(&wh[h], (U)0, code);
                            if (old == (U)0) {
                                if (atomicAdd(&s_dist, 1) + 1 > kWideMax) s_full = 1;
                                break;
                            }
                            if (old == code) break;
                            h = (h + 1u) & (kWideHash - 1);
                        }
                    }
                    __syncthreads();
                }
                const int wtotal = s_dist + s_top;
                if (!s_full && wtotal <= kWideMax) {
                    S* samp = reinterpret_cast<S*>(fw->sample);
                    for (int i = tid; i < kWideHash; i += kProbeWG) {
                        const U c = wh[i];
                        if (c != (U)0) samp[atomicAdd(&s_nv, 1)] = C::dec((U)(c - (U)1));
                    }
                    if (tid == 0 && s_top) samp[s_dist] = C::dec((U)~(U)0);
                    __syncthreads();  // the hash set is dead from here: its LDS is the sorter's
                    FSW::run(few_lds.fsw, samp, samp, nullptr, nullptr, wtotal);
                    __syncthreads();
                    for (int i = tid; i < wtotal; i += kProbeWG) fw->split[i] = (unsigned long long)C::enc(samp[i]);
                    ns = wtotal;
                    few_wide = 1;
                }
                __syncthreads();
            }
            if (ns < 0 && total > kFewMax && s_force) {
                __shared__ int s_cnt[kProbeWG / kWave];
                S* samp = reinterpret_cast<S*>(ft->sample);
                for (int i = tid; i < kFewSample; i += kProbeWG) samp[i] = keys[strat_pos(i, n, kFewSample)];
                __syncthreads();
                FS::run(few_lds.fsm, samp, samp, nullptr, nullptr, kFewSample);
                __syncthreads();
                int c = 0;
                bool first[PER];
                U cur[PER];
                U prv = tid > 0 ? C::enc(samp[tid * PER - 1]) : (U)0;
#pragma unroll
                for (int r = 0; r < PER; ++r) {
                    const int i = tid * PER + r;
                    cur[r] = C::enc(samp[i]);
                    first[r] = i == 0 || cur[r] != prv;
                    prv = cur[r];
                    c += first[r] ? 1 : 0;
                }
                int xc = c;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const int y = __shfl_up(xc, o);
                    if ((int)__lane_id() >= o) xc += y;
                }
                if (__lane_id() == kWave - 1) s_cnt[wave] = xc;
                __syncthreads();
                int pre = xc - c;
                for (int w = 0; w < wave; ++w) pre += s_cnt[w];
#pragma unroll
                for (int r = 0; r < PER; ++r)
                    if (first[r] && pre < kFewMax) ft->split[pre++] = (unsigned long long)cur[r];
                ns = kFewMax;
            }
            __syncthreads();
            if (ns >= 0) {
                if (few_wide) {
                    for (int b = tid; b < 2 * ns + 1; b += kProbeWG) st_agent(&fw->cnt[b], 0ull);
                    if (tid == 0) fw->ns = (unsigned long long)ns;
                } else {
                    for (int b = tid; b < kFewCopies * (2 * ns + 1); b += kProbeWG)
                        st_agent(&ft->cnt[b / (2 * ns + 1)][b % (2 * ns + 1)], 0ull);
                    if (tid == 0) ft->ns = (unsigned long long)ns;
                }
                path = SR_PATH_FEW;
            } else {
                path = -path - 10;
            }
        }
        // a general sort is first a NEAR candidate, which merge slot 0 confirms
        // or turns back into GENERAL (the first merge pass is the same)
        if ((jobs_ok & 8) != 0 && ((path == SR_PATH_GENERAL && s_force_near >= 0) || s_force_near > 0))
            path = SR_PATH_NEAR;
        if (tid == 0) {
            ctl->path = path;
            ctl->few_wide = path == SR_PATH_FEW ? few_wide : 0;
            ctl->dual = s_dual;
            ctl->reserved[0] = s_desc;  // kept for sr_last_stats
            ctl->reserved[1] = s_asc;
            ctl->reserved[2] = 0;
            ctl->reserved[3] = 0;
            st_agent(&ctl->mixed, 0u);
            st_agent(&ctl->ticket, 0u);
            st_agent(&ctl->m, 0ull);
            ctl->job_passes = 0;
            ctl->n_kept = 0;
            st_agent(&ctl->bad_join, 0u);
            ctl->ticket2 = 0;
            unsigned int ep = (ctl->epoch + 1u) & 0xFFFFFFu;
            ctl->epoch = ep == 0u ? 1u : ep;
        }
    }
}

// After a plain reversal of a nonincreasing array of pairs, equal-key groups
// are in reversed input order; reverse each group's payloads once more.
template <class C>
__global__ __launch_bounds__(kRevWG) void k_regroup(const typename C::S* keys, uint32_t* pay, int64_t n,
                                                    const Ctl* ctl, const RunArea* ra) {
    using U = typename C::U;
    static_assert(kRevWG == kClsWG, "regroup units are the reversal units");
    if (ra != nullptr && path_is(ctl, SR_PATH_RUNS)) {
        runs_regroup<C>(keys, pay, ra);
        return;
    }
    if (!path_is(ctl, SR_PATH_REVERSED)) return;
    for (int64_t i = (int64_t)blockIdx.x * kRevWG + threadIdx.x; i < n; i += (int64_t)gridDim.x * kRevWG) {
        const U x = C::enc(keys[i]);
        const bool le = i > 0 && C::enc(keys[i - 1]) == x;
        const bool re = i + 1 < n && C::enc(keys[i + 1]) == x;
        if (!le && !re) continue;
        int64_t lo = 0, hi = i;  // first index with key == x (keys ascending now)
        while (lo < hi) {
            const int64_t m = (lo + hi) >> 1;
            if (C::enc(keys[m]) < x) lo = m + 1;
            else hi = m;
        }
        const int64_t gs = lo;
        lo = i;
        hi = n;  // first index with key > x
        while (lo < hi) {
            const int64_t m = (lo + hi) >> 1;
            if (C::enc(keys[m]) <= x) lo = m + 1;
            else hi = m;
        }
        const int64_t partner = gs + lo - 1 - i;
        if (i < partner) {
            const uint32_t a = pay[i], b = pay[partner];
            pay[i] = b;
            pay[partner] = a;
        }
    }
}

// ------------------------------------------------------------ segmented
// Batched sort of independent segments [off[s], off[s+1]) (CSR offsets in
// device memory).  k_seg_plan (one workgroup) derives each segment's tile
// count, merge-pass count P_s and merge-chunk count, with prefix sums; the
// tile-sort launch and the merge slots then walk the concatenated tile /
// chunk lists persistently (each workgroup a contiguous range), finding the
// segment of an item by binary search and then advancing linearly.  Every
// segment is sorted exactly as a plain array would be (tile sort, then P_s
// level-synchronous merge passes), with its own ping-pong parity so that its
// last pass lands in the caller's buffer.
struct SegCtl {
    long long total_tiles;
    long long total_chunks;
    int max_passes;
    int pad;
};

constexpr int kSegPlanWG = 1024;

__device__ __forceinline__ int64_t find_seg(const int64_t* pre, int64_t nseg, int64_t item) {
    // last s with pre[s] <= item (pre is nondecreasing, pre[0] = 0)
    int64_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// off: CSR offsets (nseg+1); or, when lens is not null, per-segment lengths
// whose exclusive prefix is written to off (nseg+1 entries) here.
__global__ __launch_bounds__(kSegPlanWG) void k_seg_plan(int64_t* off, const int64_t* lens, int64_t nseg, int64_t T,
                                                         int64_t CH, int64_t* tile_pre, int64_t* chunk_pre,
                                                         int* seg_passes, SegCtl* sc) {
    __shared__ long long wt[kSegPlanWG / kWave], wc[kSegPlanWG / kWave];
    __shared__ int wp[kSegPlanWG / kWave];
    __shared__ long long carry_t, carry_c, carry_l;
    __shared__ long long wl[kSegPlanWG / kWave];
    __shared__ int maxp;
    const int tid = threadIdx.x, lane = (int)__lane_id(), wave = tid / kWave;
    if (tid == 0) {
        carry_t = 0;
        carry_c = 0;
        carry_l = 0;
        maxp = 0;
    }
    __syncthreads();
    if (lens != nullptr) {
        // offsets of the segments inside the scratch: exclusive prefix of lens
        for (int64_t b = 0; b < nseg; b += kSegPlanWG) {
            const int64_t sg = b + tid;
            const long long l = sg < nseg ? lens[sg] : 0;
            long long x = l;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const long long y = __shfl_up(x, d);
                if (lane >= d) x += y;
            }
            if (lane == kWave - 1) wl[wave] = x;
            __syncthreads();
            long long pre = carry_l + x - l;
            for (int q = 0; q < wave; ++q) pre += wl[q];
            if (sg < nseg) off[sg] = pre;
            __syncthreads();
            if (tid == 0)
                for (int q = 0; q < kSegPlanWG / kWave; ++q) carry_l += wl[q];
            __syncthreads();
        }
        if (tid == 0) off[nseg] = carry_l;
        __syncthreads();
    }
    for (int64_t b = 0; b < nseg; b += kSegPlanWG) {
        const int64_t s = b + tid;
        long long tl = 0, ch = 0;
        int ps = 0;
        if (s < nseg) {
            const int64_t len = off[s + 1] - off[s];
            tl = (len + T - 1) / T;
            ps = tl > 1 ? ceil_log2_dev(tl) : 0;
            ch = ps > 0 ? (len + CH - 1) / CH : 0;
            seg_passes[s] = ps;
        }
        long long xt = tl, xc = ch;
        int xp = ps;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const long long yt = __shfl_up(xt, d), yc = __shfl_up(xc, d);
            if (lane >= d) {
                xt += yt;
                xc += yc;
            }
            const int yp = __shfl_xor(xp, d);
            xp = xp > yp ? xp : yp;
        }
        if (lane == kWave - 1) {
            wt[wave] = xt;
            wc[wave] = xc;
        }
        if (lane == 0) wp[wave] = xp;
        __syncthreads();
        long long pt = carry_t + xt - tl, pc = carry_c + xc - ch;
        for (int q = 0; q < wave; ++q) {
            pt += wt[q];
            pc += wc[q];
        }
        if (s < nseg) {
            tile_pre[s] = pt;
            chunk_pre[s] = pc;
        }
        __syncthreads();
        if (tid == 0) {
            for (int q = 0; q < kSegPlanWG / kWave; ++q) {
                carry_t += wt[q];
                carry_c += wc[q];
                maxp = maxp > wp[q] ? maxp : wp[q];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        tile_pre[nseg] = carry_t;
        chunk_pre[nseg] = carry_c;
        sc->total_tiles = carry_t;
        sc->total_chunks = carry_c;
        sc->max_passes = maxp;
    }
}

// U is the caller's array and off its CSR offsets; or, when ptrs is not
// null, segment s lives at ptrs[s] and off holds its place in the scratch.
template <class C, int WG, int IT, bool PAIRS>
__global__ __launch_bounds__(WG) void k_seg_tile(typename C::S* U, typename C::S* S1, uint32_t* PU, uint32_t* PS1,
                                                 const int64_t* off, int64_t nseg, const int64_t* tile_pre,
                                                 const int* seg_passes, const SegCtl* sc,
                                                 typename C::S* const* ptrs) {
    using TS = TileSort<C, WG, IT, PAIRS>;
    constexpr int NW = WG / kWave;
    __shared__ typename TS::Smem sm;
    __shared__ int s_small[NW];
    const int64_t total = sc->total_tiles;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per;
    const int64_t b1 = (b0 + per) < total ? (b0 + per) : total;
    if (b0 >= b1) return;
    int64_t s = find_seg(tile_pre, nseg, b0);
    const int wave = threadIdx.x / kWave;
    for (int64_t b = b0; b < b1;) {
        while (tile_pre[s + 1] <= b) ++s;
        if (off[s + 1] - off[s] <= TS::WAVE_T) {
            // Segments of at most 64 * IT keys (one tile each): this one and
            // up to NW - 1 more in a row are sorted at once, one per wavefront.
            const int64_t bw = b + wave;
            int64_t sw = s;
            int small = 0;
            if (bw < b1) {
                while (tile_pre[sw + 1] <= bw) ++sw;
                small = (off[sw + 1] - off[sw]) <= TS::WAVE_T ? 1 : 0;
            }
            if (__lane_id() == 0) s_small[wave] = small;
            __syncthreads();
            int run = 0;
            while (run < NW && s_small[run]) ++run;  // >= 1: tile b is small
            __syncthreads();
            if (wave < run) {
                const int64_t so = off[sw];
                const int len = (int)(off[sw + 1] - so);
                const bool to_s1 = (seg_passes[sw] & 1) != 0;
                if (ptrs != nullptr) {
                    typename C::S* us = ptrs[sw];
                    TS::run_wave(us, to_s1 ? S1 + so : us, nullptr, nullptr, len);
                } else {
                    typename C::S* dst = to_s1 ? S1 : U;
                    uint32_t* pdst = to_s1 ? PS1 : PU;
                    TS::run_wave(U + so, dst + so, PAIRS ? PU + so : nullptr, PAIRS ? pdst + so : nullptr, len);
                }
            }
            b += run;
            continue;
        }
        const int64_t so = off[s], len = off[s + 1] - so;
        const int64_t u = b - tile_pre[s];
        const int64_t base = so + u * TS::T;
        const int valid = (int)((len - u * TS::T) < TS::T ? (len - u * TS::T) : TS::T);
        const bool to_s1 = (seg_passes[s] & 1) != 0;
        if (ptrs != nullptr) {
            typename C::S* us = ptrs[s] + u * TS::T;
            TS::run(sm, us, to_s1 ? S1 + base : us, nullptr, nullptr, valid);
        } else {
            typename C::S* dst = to_s1 ? S1 : U;
            uint32_t* pdst = to_s1 ? PS1 : PU;
            TS::run(sm, U + base, dst + base, PAIRS ? PU + base : nullptr, PAIRS ? pdst + base : nullptr, valid);
        }
        __syncthreads();
        ++b;
    }
}

template <class C, int WG, int IT, bool PAIRS>
__global__ __launch_bounds__(WG) void k_seg_merge(typename C::S* U, typename C::S* S1, uint32_t* PU, uint32_t* PS1,
                                                  const int64_t* off, int64_t nseg, const int64_t* chunk_pre,
                                                  const int* seg_passes, const SegCtl* sc, int64_t T, int k,
                                                  typename C::S* const* ptrs) {
    using MC = MergeChunk<C, WG, IT, PAIRS>;
    if (k >= sc->max_passes) return;
    __shared__ typename MC::Smem sm;
    const int64_t total = sc->total_chunks;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = (int64_t)blockIdx.x * per;
    const int64_t c1 = (c0 + per) < total ? (c0 + per) : total;
    if (c0 >= c1) return;
    int64_t s = find_seg(chunk_pre, nseg, c0);
    for (int64_t c = c0; c < c1; ++c) {
        while (chunk_pre[s + 1] <= c) ++s;
        const int P = seg_passes[s];
        if (k >= P) continue;
        const int64_t so = off[s], len = off[s + 1] - so;
        const int from = (P - k) & 1;
        typename C::S* us = ptrs != nullptr ? ptrs[s] : U + so;
        typename C::S* src = from ? S1 + so : us;
        typename C::S* dst = from ? us : S1 + so;
        uint32_t* psrc = from ? PS1 : PU;
        uint32_t* pdst = from ? PU : PS1;
        MC::run(sm, src, dst, PAIRS ? psrc + so : nullptr, PAIRS ? pdst + so : nullptr, len, T << k, -1,
                (c - chunk_pre[s]) * MC::CH, nullptr);
        __syncthreads();
    }
}

// Exact counts of descents and ascents (sr_measure).
template <class C>
__global__ __launch_bounds__(kProbeWG) void k_count(const typename C::S* keys, int64_t n,
                                                    unsigned long long* out) {
    using U = typename C::U;
    unsigned long long d = 0, a = 0;
    for (int64_t i = (int64_t)blockIdx.x * kProbeWG + threadIdx.x; i + 1 < n; i += (int64_t)gridDim.x * kProbeWG) {
        const U x = C::enc(keys[i]), y = C::enc(keys[i + 1]);
        d += x > y ? 1 : 0;
        a += x < y ? 1 : 0;
    }
    d = wave_sum(d);
    a = wave_sum(a);
    if (__lane_id() == 0) {
        if (d) atomicAdd(&out[0], d);
        if (a) atomicAdd(&out[1], a);
    }
}

__global__ void k_fill_u64(unsigned long long* p, int n, unsigned long long v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_init_ctl(Ctl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long* w = reinterpret_cast<unsigned long long*>(ctl);
        for (size_t i = 0; i < sizeof(Ctl) / 8; ++i) w[i] = 0;
        ctl->path = SR_PATH_GENERAL;
        ctl->force_path = -1;
    }
}

__global__ void k_set_force(Ctl* ctl, int force) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->force_path = force;
}

__global__ __launch_bounds__(256) void k_copy16(uint4* dst, const uint4* src, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

}  // namespace sr

// ======================================================================
// Host side
// ======================================================================
#include "sr_internal.hpp"

namespace {

using namespace sr;

thread_local std::string g_err;

sr_status fail(sr_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

sr_status hip_fail(hipError_t e, const char* what) {
    return fail(SR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

std::mutex g_mu;
// device-time model behind the probe's run-scan gate (measured on gfx950:
// the scan, the outlier rounds it can bring along and the plan together
// against a merge pass at 2M .. 32M keys)
constexpr double kRunScanUs = 40.0;
constexpr double kPassFloorUs = 8.0;

int g_force_path = -1;
bool g_profile = false;
bool g_outlier_enabled = true;  // allow the OUTLIER path
bool g_runs_enabled = true;     // allow the RUNS path for keys-only sorts
bool g_few_enabled = true;      // allow the FEW path
bool g_near_enabled = true;     // allow the NEAR plan on general sorts
// Launch-shape options; the "auto" value defers to the tuning table, then to
// the built-in rule in resolve_shape.
int64_t g_partition_min_n = -1;  // separate Merge Path partition launch from this n on
int g_tile_variant = -1;         // 0: 512 x 16, 1: 1024 x 8 (32-bit keys only)
int g_merge_items = 0;           // fused merge: outputs per thread, 8 or 16 (32-bit keys only)
int g_nontemporal = -1;          // persistent merge: nontemporal window loads and stores
int g_fan_in = 0;                // merge fan-in of general sorts: 2, 4, 0 = auto (table, then built-in)
std::vector<sr_tune_entry> g_tune;  // sorted by (dtype, pairs, min_n)
uint64_t g_tune_version = 0;        // bumped by every sr_tune_set (captured graphs key on it)

// Built-in rules, from a sweep of random keys of each type on gfx950.
constexpr int64_t kPartitionMinN = (int64_t)1 << 23;
constexpr int64_t kMerge16MinN = (int64_t)1 << 21;     // fused merge: 16 outputs per thread from here
constexpr size_t kNontemporalBytes = (size_t)1 << 28;  // of keys: two such arrays exceed the MALL
constexpr int64_t kFan4MinN = (int64_t)1 << 62;         // four-way passes from here (set from measurements)
constexpr int64_t kTuneMaxRows = 1024;

// sr_dtype of a codec
template <class C>
struct DtypeOf;
template <>
struct DtypeOf<CodecI32> { static constexpr int value = SR_INT32; };
template <>
struct DtypeOf<CodecU64> { static constexpr int value = SR_UINT64; };
template <>
struct DtypeOf<CodecF32> { static constexpr int value = SR_FLOAT32; };

struct LaunchShape {
    bool partition;    // separate partition launch + persistent merge
    int tile_variant;  // 0: TWG x TIT, 1: 1024 x 8 (32-bit keys)
    int merge_items;   // fused merge outputs per thread (32-bit keys)
    bool nt;           // nontemporal persistent merge
    int fan_in;        // 2, or 4: four-way passes for keys-only general sorts (partition shape only)
};

// Explicit options first, then the table row of (dt, pairs) with the largest
// min_n <= n, then the built-in rules.  Caller holds g_mu.
LaunchShape resolve_shape(int dt, bool pairs, int64_t n, size_t key_bytes) {
    const sr_tune_entry* row = nullptr;
    for (const sr_tune_entry& e : g_tune)
        if (e.dtype == dt && e.pairs == (pairs ? 1 : 0) && e.segmented == 0 && e.min_n <= n) row = &e;
    LaunchShape sh;
    if (g_partition_min_n >= 0) sh.partition = n >= g_partition_min_n;
    else if (row && row->partition >= 0) sh.partition = row->partition != 0;
    else sh.partition = n >= kPartitionMinN;
    if (g_tile_variant >= 0) sh.tile_variant = g_tile_variant;
    else if (row && row->tile_variant >= 0) sh.tile_variant = row->tile_variant;
    else sh.tile_variant = sh.partition ? 0 : 1;
    if (g_merge_items > 0) sh.merge_items = g_merge_items;
    else if (row && row->merge_items > 0) sh.merge_items = row->merge_items;
    else sh.merge_items = n >= kMerge16MinN ? 16 : 8;
    if (g_nontemporal >= 0) sh.nt = g_nontemporal != 0;
    else if (row && row->nontemporal >= 0) sh.nt = row->nontemporal != 0;
    else if (!pairs) sh.nt = (size_t)n * key_bytes >= kNontemporalBytes;
    else sh.nt = key_bytes == 8 && (size_t)n * key_bytes >= kNontemporalBytes / 2;  // not for 32-bit pairs
    if (g_fan_in > 0) sh.fan_in = g_fan_in;
    else if (row && row->fan_in > 0) sh.fan_in = row->fan_in;
    else sh.fan_in = !pairs && n >= kFan4MinN ? 4 : 2;
    if (pairs) sh.fan_in = 2;
    return sh;
}

// Shape of a segmented / batched sort (32-bit keys, keys only): the tile
// sort's thread shape and the merge's outputs per thread.  Explicit options
// first, then the table's segmented row of (dt, pairs) with the largest
// min_n <= total keys, then the built-in shape (512 x 16 tiles, 16 outputs).
struct SegShape {
    int tile_variant;
    int merge_items;
};
SegShape resolve_seg_shape(int dt, bool pairs, int64_t n) {
    const sr_tune_entry* row = nullptr;
    for (const sr_tune_entry& e : g_tune)
        if (e.dtype == dt && e.pairs == (pairs ? 1 : 0) && e.segmented == 1 && e.min_n <= n) row = &e;
    SegShape sh;
    if (g_tile_variant >= 0) sh.tile_variant = g_tile_variant;
    else if (row && row->tile_variant >= 0) sh.tile_variant = row->tile_variant;
    else sh.tile_variant = 0;
    if (g_merge_items > 0) sh.merge_items = g_merge_items;
    else if (row && row->merge_items > 0) sh.merge_items = row->merge_items;
    else sh.merge_items = 16;
    return sh;
}

struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t get_event() {
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;  // this launch goes unprofiled
    }
    return e;
}

// Set while a call is recorded into a stream capture: no event records then.
thread_local bool t_no_profile = false;
struct NoProfile {
    bool prev;
    explicit NoProfile(bool on) : prev(t_no_profile) { t_no_profile = prev || on; }
    ~NoProfile() { t_no_profile = prev; }
};

// Records an event pair around one launch when profiling is on.
struct ProfScope {
    hipStream_t st;
    const char* name;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(hipStream_t s, const char* nm) : st(s), name(nm) {
        if (g_profile && !t_no_profile) {
            std::lock_guard<std::mutex> lk(g_mu);
            a = get_event();
            b = get_event();
            if (a == nullptr || b == nullptr || hipEventRecord(a, st) != hipSuccess) {
                (void)hipGetLastError();
                if (a) g_event_pool.push_back(a);
                if (b) g_event_pool.push_back(b);
                a = b = nullptr;
            }
        }
    }
    ~ProfScope() {
        if (a) {
            const bool ok = hipEventRecord(b, st) == hipSuccess;
            std::lock_guard<std::mutex> lk(g_mu);
            if (ok) {
                g_prof.push_back(ProfRec{name, a, b});
            } else {
                (void)hipGetLastError();
                g_event_pool.push_back(a);
                g_event_pool.push_back(b);
            }
        }
    }
};

// Per (device, stream): a header allocated once and never moved (control
// block with the call epoch, probe slots), the data scratch (grown on
// demand) and the zero-initialised look-back arrays of the outlier path
// (grown on demand; their status words are stamped with the epoch, which
// therefore must never restart while they live).
struct Workspace {
    void* hdr = nullptr;
    void* base = nullptr;
    size_t bytes = 0;
    Ctl* ctl = nullptr;
    int force = -2;       // force_path value last written to ctl
    void* aux = nullptr;
    size_t aux_bytes = 0;
    unsigned long long generation = 0;  // bumped whenever a buffer moves (invalidates captured graphs)
    bool external = false;              // base is the caller's buffer (sr_set_workspace): never grown or freed
};

struct LastCall {
    int64_t tile = 0;
    int64_t n = 0;
    int es = 0;
    int merge_passes = 0;
    int trivial = 1;
    bool fan4 = false;  // general passes were four-way
    bool pairs = false;
    Ctl* ctl = nullptr;
};

std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
std::map<hipStream_t, LastCall> g_last;

// Workspace header: control block, then the probe's per-workgroup slots.
constexpr size_t kCtlBytes = 256;
constexpr size_t kHdrBytes = 128 * 1024;
static_assert(sizeof(Ctl) <= kCtlBytes, "control block");
static_assert(kCtlBytes + kProbeMaxGrid * 4 * 8 + (kProbeMaxGrid / kProbeGroup + 1) * 256 <= kHdrBytes,
              "probe slots and group counters");
constexpr size_t kFewOff = 48 * 1024;  // FEW splitter table inside the header
static_assert(kCtlBytes + kProbeMaxGrid * 4 * 8 + (kProbeMaxGrid / kProbeGroup + 1) * 256 <= kFewOff &&
                  kFewOff + sizeof(FewTable) <= kHdrBytes,
              "few-unique table");

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// The path-forcing option lives in the control block: rewrite it when the
// option changed since this workspace last saw it.
void apply_force(Workspace* ws, hipStream_t st) {
    int force;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        force = g_force_path;
    }
    if (ws->force != force) {
        hipLaunchKernelGGL(k_set_force, dim3(1), dim3(1), 0, st, ws->ctl, force);
        ws->force = force;
    }
}

// Workspace of at least `data_bytes` scratch bytes and `aux_bytes` of
// zero-initialised look-back space for (device, stream).
sr_status get_workspace(hipStream_t st, size_t data_bytes, Workspace** out, size_t aux_bytes = 0) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    Workspace* ws;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Workspace*& slot = g_ws[{dev, st}];
        if (!slot) slot = new Workspace();
        ws = slot;
    }
    if (ws->hdr == nullptr) {
        e = hipMalloc(&ws->hdr, kHdrBytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SR_ERR_OUT_OF_MEMORY, "workspace header allocation failed");
        }
        ws->ctl = reinterpret_cast<Ctl*>(ws->hdr);
        hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, st, (unsigned long long*)ws->hdr,
                           (int64_t)(kHdrBytes / 8));
        hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, st, ws->ctl);
        ws->force = -1;
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "init");
    }
    const size_t need = round_up(std::max(data_bytes, (size_t)256), 256);
    if (ws->external) {
        if (ws->bytes < need)
            return fail(SR_ERR_INVALID_ARGUMENT, "caller workspace too small: the call needs " + std::to_string(need) +
                                                     " bytes, " + std::to_string(ws->bytes) + " are set");
    } else if (ws->bytes < need) {
        if (ws->base) {
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(ws->base);
            ws->base = nullptr;
            ws->bytes = 0;
        }
        const size_t alloc = std::max(need, (size_t)1 << 20);
        ws->generation++;
        e = hipMalloc(&ws->base, alloc);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SR_ERR_OUT_OF_MEMORY, "workspace allocation of " + std::to_string(alloc) + " bytes failed");
        }
        ws->bytes = alloc;
    }
    if (aux_bytes > ws->aux_bytes) {
        if (ws->aux) {
            e = hipStreamSynchronize(st);
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(ws->aux);
            ws->aux = nullptr;
            ws->aux_bytes = 0;
        }
        ws->generation++;
        const size_t alloc = round_up(std::max(aux_bytes, (size_t)1 << 16), 4096);
        e = hipMalloc(&ws->aux, alloc);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(SR_ERR_OUT_OF_MEMORY, "look-back allocation of " + std::to_string(alloc) + " bytes failed");
        }
        ws->aux_bytes = alloc;
        hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, st, (unsigned long long*)ws->aux,
                           (int64_t)(alloc / 8));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "zero");
    }
    apply_force(ws, st);
    *out = ws;
    return SR_OK;
}

// Whether (device, stream) already holds a workspace of these sizes, so a
// call would allocate nothing.
bool workspace_fits(hipStream_t st, size_t data_bytes, size_t aux_bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_ws.find({dev, st});
    if (it == g_ws.end() || it->second == nullptr) return false;
    const Workspace* ws = it->second;
    const size_t need = round_up(std::max(data_bytes, (size_t)256), 256);
    return ws->hdr != nullptr && ws->bytes >= need && ws->aux_bytes >= aux_bytes;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Look-back space of a sort of n keys with every presortedness path on (tile
// summaries in whole verify rounds, kept-key masks, run descriptors, the run
// plan): an upper bound of what sort_impl asks for.
size_t aux_bound(int64_t n) {
    const size_t ncls = (size_t)cdiv(n, kClsTC);
    const size_t cls_arr = round_up(round_up(ncls, (size_t)kVerRound) * 8, 256);
    return 4 * cls_arr + round_up(ncls * (kClsTC / 8), 256) + round_up(ncls * sizeof(RunTile), 256) +
           round_up(sizeof(RunArea), 256) + round_up((size_t)cdiv(n, 4096) * 32, 256) +
           round_up(sizeof(WideTable), 256);
}

void* ws_data(Workspace* ws) { return ws->base; }
unsigned long long* ws_slots(Workspace* ws) {
    return reinterpret_cast<unsigned long long*>((char*)ws->hdr + kCtlBytes);
}

// ------------------------------------------------ allocation-free sorts
// sr_sort_keys_noalloc keeps its whole workspace (header, look-back space,
// data scratch) in one array per device that lives in the code object, so a
// call never allocates device memory.  The array's name is a host-side
// stand-in in host code: its device address comes from hipGetSymbolAddress,
// once per device, and only that address is passed to kernels.
constexpr size_t kNoAllocKeyBytes = (size_t)32 << 20;  // largest n x key size
constexpr int64_t kNoAllocMaxN32 = (int64_t)(kNoAllocKeyBytes / 4);
constexpr size_t kNoAllocBytes = (size_t)36 << 20;
constexpr int kNoAllocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocDevice {
    bool ready = false;
    Workspace ws;  // views of the array; never grown or freed
};
NoAllocDevice g_noalloc[kNoAllocMaxDevices];
std::mutex g_noalloc_mu;

bool noalloc_ready() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) return false;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return g_noalloc[dev].ready;
}

// The device's allocation-free workspace; the first call on a device looks up
// the array's address, zeroes its header and look-back space on `st` and
// waits for that, so every later call (on any stream) finds it initialised.
sr_status noalloc_workspace(hipStream_t st, Workspace** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(SR_ERR_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    NoAllocDevice& d = g_noalloc[dev];
    if (!d.ready) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return fail(SR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        const size_t aux = round_up(aux_bound(kNoAllocMaxN32), 4096);
        if (kHdrBytes + aux + kNoAllocKeyBytes + ((size_t)1 << 20) > kNoAllocBytes)
            return fail(SR_ERR_INTERNAL, "allocation-free scratch layout does not fit its array");
        char* p = static_cast<char*>(ptr);
        Workspace& w = d.ws;
        w.hdr = p;
        w.ctl = reinterpret_cast<Ctl*>(p);
        w.aux = p + kHdrBytes;
        w.aux_bytes = aux;
        w.base = p + kHdrBytes + aux;
        w.bytes = kNoAllocBytes - kHdrBytes - aux;
        w.external = true;
        hipLaunchKernelGGL(k_zero_u64, dim3(256), dim3(256), 0, st, (unsigned long long*)p,
                           (int64_t)((kHdrBytes + aux) / 8));
        hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, st, w.ctl);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "allocation-free scratch initialisation");
        w.force = -1;
        d.ready = true;
    }
    apply_force(&d.ws, st);
    *out = &d.ws;
    return SR_OK;
}

// Resident workgroups of a kernel on the whole device (persistent grids).
template <class K>
int64_t resident_blocks(K kernel, int threads) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int64_t> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), dev);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int64_t r = (int64_t)std::max(cus, 1) * per_cu;
    cache[key] = r;
    return r;
}

int ceil_log2(int64_t x) {
    int r = 0;
    while (((int64_t)1 << r) < x) ++r;
    return r;
}


#define SR_LAUNCH_CHECK(what)                                  \
    do {                                                       \
        hipError_t e_ = hipGetLastError();                     \
        if (e_ != hipSuccess) return hip_fail(e_, what);       \
    } while (0)

// st: the caller's stream (workspace and statistics are kept per stream);
// ls: the stream the kernels are launched on (st, or a capture stream).
// noalloc: take the device's allocation-free workspace instead of the
// stream's (nothing is allocated; the call's statistics are not recorded).
template <class C, bool PAIRS>
sr_status sort_impl(void* keys_v, uint32_t* pay, int64_t n, hipStream_t st, bool prepare_only = false,
                    hipStream_t ls = nullptr, bool noalloc = false) {
    if (ls == nullptr) ls = st;
    // Recorded into the caller's stream capture, the sort enqueues the same
    // launches (replays sort whatever the buffers hold then); it must neither
    // allocate nor synchronize, so its workspace has to be in place already.
    bool capturing = false;
    {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        capturing = hipStreamIsCapturing(st, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
    }
    NoProfile np(capturing);
    using S = typename C::S;
    using TN = Tune<C, PAIRS>;
    constexpr int T = TN::TWG * TN::TIT;
    constexpr int CH = TN::MWG * TN::MIT;
    static_assert(T % CH == 0, "tile must be a whole number of merge chunks");
    S* keys = static_cast<S*>(keys_v);
    const int64_t ntiles = cdiv(n, T);
    const int M = ceil_log2(ntiles);
    LastCall lc;
    lc.n = n;
    lc.es = (int)sizeof(S) + (PAIRS ? 4 : 0);
    lc.pairs = PAIRS;
    lc.merge_passes = M;
    if (ntiles == 1) {
        if (prepare_only) return SR_OK;
        // One tile: sort in place, no probe.
        ProfScope ps(ls, "tile_sort");
        hipLaunchKernelGGL((k_tile_sort<C, TN::TWG, TN::TIT, PAIRS>), dim3(1), dim3(TN::TWG), 0, ls, keys, keys,
                           pay, pay, n, 0, (const Ctl*)nullptr, (const RunTile*)nullptr);
        SR_LAUNCH_CHECK("tile_sort");
        if (noalloc) return SR_OK;
        lc.trivial = 1;
        std::lock_guard<std::mutex> lk(g_mu);
        g_last[st] = lc;
        return SR_OK;
    }
    const int64_t nchunks = cdiv(n, CH);
    // pairs: outlier places and kept-before counts kept in 32 bits
    const bool outlier_ok = g_outlier_enabled && (!PAIRS || n <= (int64_t)UINT32_MAX);
    // keys-only sorts and pairs with tiles of whole run-scan tiles (the
    // run reversal of pairs is the stable one)
    const bool runs_ok = g_runs_enabled && T >= kClsTC;
    // pairs: equal buckets only (at most kFewMax values), their count matrix
    // (kFewMax x tiles of u32) in the wide table's space: n <= 4,194,304
    const bool few_ok =
        g_few_enabled && (!PAIRS || (size_t)cdiv(n, kClsTC) * kFewMax * sizeof(unsigned int) <= sizeof(WideTable));
    const bool scan_ok = outlier_ok || runs_ok || few_ok;
    const int64_t ncls = scan_ok ? cdiv(n, kClsTC) : 0;
    LaunchShape sh;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        sh = resolve_shape(DtypeOf<C>::value, PAIRS, n, sizeof(S));
    }
    const bool use_partition = sh.partition;
    // four-way general passes: keys only, with the partition launch shape,
    // at least one pair of levels, cuts held in 32 bits
    const bool fan4 = !PAIRS && use_partition && sh.fan_in == 4 && M >= 2 && n <= (int64_t)UINT32_MAX;
    // co-ranks of a merge pass; a RUNS pass has up to one extra chunk per leaf
    // group; a four-way pass keeps the cut of every sample (16 bytes) there
    const size_t co_bytes =
        round_up(std::max((size_t)(nchunks + 2 + kRunMaxLeaves) * 8,
                          fan4 ? (size_t)(Merge4<C>::chunks(n, (int64_t)T) + 8) * 16 : (size_t)0),
                 256);
    const size_t kbytes = round_up((size_t)n * sizeof(S), 256);
    // tile summaries (ver_slot layout: whole verify rounds) and tile prefixes
    const size_t cls_arr = round_up((size_t)round_up((size_t)ncls, (size_t)kVerRound) * 8, 256);
    Workspace* ws = nullptr;
    // aux: tile offsets, first/last kept keys, kept counts, kept bit masks
    const size_t flag_bytes = round_up((size_t)ncls * (kClsTC / 8), 256);
    // run descriptors and the run plan
    const size_t rdesc_bytes = runs_ok ? round_up((size_t)ncls * sizeof(RunTile), 256) : 0;
    const size_t rarea_bytes = runs_ok ? round_up(sizeof(RunArea), 256) : 0;
    // NEAR: four codes per sorted tile for merge slot 0's test
    bool near_ok;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        near_ok = g_near_enabled && M >= 3 && !fan4;
    }
    const size_t tdesc_bytes = near_ok ? round_up((size_t)ntiles * 32, 256) : 0;
    // FEW with more than 64 splitters: its tables
    const size_t wide_bytes = few_ok ? round_up(sizeof(WideTable), 256) : 0;
    // pairs OUTLIER: each outlier's payload and kept-before count (m <= n/4)
    const size_t ocap = PAIRS && outlier_ok ? (size_t)n / 4 + 1 : 0;
    const size_t data_need =
        co_bytes + kbytes + (PAIRS ? round_up((size_t)n * 4, 256) + round_up(ocap * 8, 256) : 0);
    const size_t aux_need = 4 * cls_arr + flag_bytes + rdesc_bytes + rarea_bytes + tdesc_bytes + wide_bytes;
    sr_status s;
    if (capturing && !(noalloc ? noalloc_ready() : workspace_fits(st, data_need, aux_need)))
        return fail(SR_ERR_UNSUPPORTED, "a sort recorded into a stream capture cannot allocate or synchronize: "
                                        "size the stream's workspace first (sr_reserve, or one sort of this "
                                        "size on the stream before the capture)");
    if (noalloc) {
        s = noalloc_workspace(st, &ws);
        if (s == SR_OK && (data_need > ws->bytes || aux_need > ws->aux_bytes))
            s = fail(SR_ERR_INTERNAL, "allocation-free scratch smaller than the call needs");
    } else {
        s = get_workspace(st, data_need, &ws, aux_need);
    }
    if (s != SR_OK || prepare_only) return s;
    Ctl* ctl = ws->ctl;
    char* wd = static_cast<char*>(ws_data(ws));
    int64_t* co = reinterpret_cast<int64_t*>(wd);
    S* skeys = reinterpret_cast<S*>(wd + co_bytes);
    uint32_t* spay = PAIRS ? reinterpret_cast<uint32_t*>(wd + co_bytes + kbytes) : nullptr;
    uint32_t* opay = ocap ? reinterpret_cast<uint32_t*>(wd + co_bytes + kbytes + round_up((size_t)n * 4, 256))
                          : nullptr;
    uint32_t* okb = ocap ? opay + ocap : nullptr;
    const bool merge8 = sizeof(S) == 4 && !PAIRS && TN::MIT == 16 && sh.merge_items == 8;
    const int64_t merge_ch = use_partition ? CH : (merge8 ? (int64_t)TN::MWG * 8 : CH);
    RunTile* rdesc = nullptr;
    RunArea* rarea = nullptr;
    FewTable* ftab = few_ok ? reinterpret_cast<FewTable*>(static_cast<char*>(ws->hdr) + kFewOff) : nullptr;
    unsigned long long* tdesc =
        near_ok ? reinterpret_cast<unsigned long long*>(static_cast<char*>(ws->aux) + 4 * cls_arr + flag_bytes +
                                                        rdesc_bytes + rarea_bytes)
                : nullptr;
    void* few_area = few_ok ? static_cast<char*>(ws->aux) + 4 * cls_arr + flag_bytes + rdesc_bytes + rarea_bytes +
                                  tdesc_bytes
                            : nullptr;
    // keys: the wide table; pairs: the count matrix of the pairs FEW job
    WideTable* fw = PAIRS ? nullptr : reinterpret_cast<WideTable*>(few_area);
    unsigned int* fewm = PAIRS ? reinterpret_cast<unsigned int*>(few_area) : nullptr;

    {
        ProfScope ps(ls, "probe");
        const unsigned g = (unsigned)std::min<int64_t>(cdiv(n - 1, kProbeTile), kProbeMaxGrid);
        // a run scan and plan cost about kRunScanUs of device time; a merge
        // pass costs a launch-bound floor plus its HBM time (about 5.5 TB/s):
        // the scan pays only if the plan's leaves leave at least that many
        // passes saved, so the leaves the probe sees forced may merge in at
        // most runs_pmax passes
        const double pass_us = kPassFloorUs + (double)n * (double)(sizeof(S) + (PAIRS ? 4 : 0)) * 2.0 / 5.5e6;
        const int runs_pmax = M - (int)std::ceil(kRunScanUs / pass_us);
        hipLaunchKernelGGL(k_probe<C>, dim3(g), dim3(kProbeWG), 0, ls, (const S*)keys, n, ctl, ws_slots(ws),
                           (outlier_ok ? 1 : 0) | (runs_ok ? 2 : 0) | (few_ok ? 4 : 0) | (near_ok ? 8 : 0), runs_pmax,
                           ftab, fw);
        SR_LAUNCH_CHECK("probe");
    }
    if (scan_ok) {
        unsigned long long* aux = static_cast<unsigned long long*>(ws->aux);
        unsigned long long* kpref_t = aux;
        unsigned long long* tfirst = aux + cls_arr / 8;
        unsigned long long* tlast = aux + 2 * (cls_arr / 8);
        unsigned long long* tcount = aux + 3 * (cls_arr / 8);
        unsigned int* flags = reinterpret_cast<unsigned int*>(aux + 4 * (cls_arr / 8));
        if (runs_ok) {
            rdesc = reinterpret_cast<RunTile*>(reinterpret_cast<char*>(flags) + flag_bytes);
            rarea = reinterpret_cast<RunArea*>(reinterpret_cast<char*>(rdesc) + rdesc_bytes);
        }
        {
            ProfScope ps(ls, "classify");
            hipLaunchKernelGGL(k_classify<C>, dim3((unsigned)ncls), dim3(kClsWG), 0, ls, (const S*)keys, n, ctl,
                               flags, tfirst, tlast, tcount, runs_ok ? 1 : 0, rdesc, ftab, skeys, fw, fewm);
            SR_LAUNCH_CHECK("classify");
        }
        {
            ProfScope ps(ls, "verify");
            hipLaunchKernelGGL(k_verify<C>, dim3(1), dim3(kVerWG), 0, ls, ctl, n, ncls,
                               (const unsigned long long*)tfirst, (const unsigned long long*)tlast,
                               (const unsigned long long*)tcount, kpref_t, (int64_t)T, (const S*)keys,
                               (const RunTile*)rdesc, rarea, runs_ok ? 1 : 0, merge_ch, M, ftab, fw, fewm,
                               ocap ? 1 : 0);
            SR_LAUNCH_CHECK("verify");
        }
        ProfScope ps(ls, "scatter");
        hipLaunchKernelGGL(k_scatter<C>, dim3((unsigned)ncls), dim3(kClsWG), 0, ls, keys, n, (const Ctl*)ctl, skeys,
                           (const unsigned int*)flags, (const unsigned long long*)kpref_t, (const RunArea*)rarea,
                           PAIRS ? pay : nullptr, spay, (const FewTable*)ftab, (const unsigned int*)fewm, opay, okb);
        SR_LAUNCH_CHECK("scatter");
    }
    {
        // GENERAL / OUTLIER: tile sort of the job; REVERSED: in-place reversal
        ProfScope ps(ls, "tile_sort");
        if constexpr (sizeof(S) == 4 && !PAIRS && TN::TWG * TN::TIT == 1024 * 8) {
            if (sh.tile_variant == 1) {
                hipLaunchKernelGGL((k_tile_sort<C, 1024, 8, PAIRS>), dim3((unsigned)ntiles), dim3(1024), 0, ls, keys,
                                   skeys, pay, spay, n, M, (const Ctl*)ctl, (const RunTile*)rdesc, tdesc,
                                   fan4 ? 1 : 0);
                SR_LAUNCH_CHECK("tile_sort");
                goto tile_done;
            }
        }
        hipLaunchKernelGGL((k_tile_sort<C, TN::TWG, TN::TIT, PAIRS>), dim3((unsigned)ntiles), dim3(TN::TWG), 0, ls,
                           keys, skeys, pay, spay, n, M, (const Ctl*)ctl, (const RunTile*)rdesc, tdesc,
                           fan4 ? 1 : 0);
        SR_LAUNCH_CHECK("tile_sort");
    }
tile_done:
    if (PAIRS) {
        ProfScope ps(ls, "regroup");
        const unsigned g = (unsigned)std::min<int64_t>(cdiv(n, kRevWG * 4), 8192);
        hipLaunchKernelGGL(k_regroup<C>, dim3(std::max(1u, g)), dim3(kRevWG), 0, ls, (const S*)keys, pay, n,
                           (const Ctl*)ctl, (const RunArea*)rarea);
        SR_LAUNCH_CHECK("regroup");
    }
    for (int k = 0; k < M; ++k) {
        if (use_partition) {
            {
                ProfScope ps(ls, "partition");
                hipLaunchKernelGGL(k_partition<C>, dim3((unsigned)cdiv(nchunks, 256)), dim3(256), 0, ls, keys, skeys,
                                   n, M, (int64_t)T, k, CH, co, (const Ctl*)ctl, (const RunArea*)rarea,
                                   fan4 ? 1 : 0);
                SR_LAUNCH_CHECK("partition");
            }
            // a general sort's four-way pass over levels k and k+1 (the two-way
            // launches of the slot then return at once; the other plans use
            // them and these return)
            const bool four = fan4 && (k & 1) == 0 && k + 1 < M;
            const int64_t nc4 = four ? Merge4<C>::chunks(n, (int64_t)T << k) : 0;
            if (four) {
                ProfScope ps(ls, "part4");
                const int64_t ns4 = Merge4<C>::sample_slots(n, (int64_t)T << k);
                hipLaunchKernelGGL(k_part4<C>, dim3((unsigned)cdiv(ns4, 256)), dim3(256), 0, ls, keys, skeys, n, M,
                                   (int64_t)T, k, reinterpret_cast<uint4*>(co), (const Ctl*)ctl);
                SR_LAUNCH_CHECK("part4");
            }
            {
                ProfScope ps(ls, "merge");
                auto kern = sh.nt ? k_merge_persist<C, TN::MWG, TN::MIT, PAIRS, true>
                                  : k_merge_persist<C, TN::MWG, TN::MIT, PAIRS, false>;
                const int64_t grid = std::min<int64_t>(nchunks, resident_blocks(kern, TN::MWG));
                hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(TN::MWG), 0, ls, keys, skeys, pay, spay, n, M,
                                   (int64_t)T, k, (const int64_t*)co, (const Ctl*)ctl, (const RunArea*)rarea,
                                   (const FewTable*)ftab, (const unsigned long long*)tdesc, fan4 ? 1 : 0,
                                   (const WideTable*)fw, (const uint32_t*)opay, (const uint32_t*)okb);
                SR_LAUNCH_CHECK("merge");
            }
            if (four) {
                ProfScope ps(ls, "merge4");
                auto kern4 = sh.nt ? k_merge4<C, true> : k_merge4<C, false>;
                hipLaunchKernelGGL(kern4, dim3((unsigned)nc4), dim3(256), 0, ls, keys, skeys, n, M, (int64_t)T, k,
                                   reinterpret_cast<const uint4*>(co), (const Ctl*)ctl);
                SR_LAUNCH_CHECK("merge4");
            }
        } else {
            ProfScope ps(ls, "merge");
            // a RUNS pass k cuts each of its <= kRunMaxLeaves / 2^(k+1) groups
            // into chunks on its own, so it may have that many chunks more
            // than a level-synchronous pass: one workgroup each, so that no
            // workgroup merges two chunks one after the other (the extra
            // workgroups of other jobs return at once)
            const int64_t extra = runs_ok ? (int64_t)(kRunMaxLeaves >> (k + 1 < 30 ? k + 1 : 30)) + 1 : 0;
            bool done = false;
            if constexpr (sizeof(S) == 4 && !PAIRS && TN::MIT == 16) {
                if (merge8) {
                    hipLaunchKernelGGL((k_merge<C, TN::MWG, 8, PAIRS>), dim3((unsigned)(cdiv(n, TN::MWG * 8) + extra)),
                                       dim3(TN::MWG), 0, ls, keys, skeys, pay, spay, n, M, (int64_t)T, k,
                                       (const Ctl*)ctl, (const RunArea*)rarea, (const FewTable*)ftab,
                                       (const unsigned long long*)tdesc, (const WideTable*)fw,
                                       (const uint32_t*)opay, (const uint32_t*)okb);
                    done = true;
                }
            }
            if (!done)
                hipLaunchKernelGGL((k_merge<C, TN::MWG, TN::MIT, PAIRS>), dim3((unsigned)(nchunks + extra)),
                                   dim3(TN::MWG), 0, ls, keys, skeys, pay, spay, n, M, (int64_t)T, k,
                                   (const Ctl*)ctl, (const RunArea*)rarea, (const FewTable*)ftab,
                                   (const unsigned long long*)tdesc, (const WideTable*)fw,
                                   (const uint32_t*)opay, (const uint32_t*)okb);
            SR_LAUNCH_CHECK("merge");
        }
    }
    if (noalloc) return SR_OK;
    lc.trivial = 0;
    lc.fan4 = fan4;
    lc.ctl = ctl;
    lc.tile = T;
    std::lock_guard<std::mutex> lk(g_mu);
    g_last[st] = lc;
    return SR_OK;
}

// Offsets mode: keys_v + off (CSR).  Batch mode: ptrs/lens (device arrays)
// give each segment's own buffer and length; n is then the total.
template <class C, bool PAIRS>
sr_status seg_impl(void* keys_v, uint32_t* pay, int64_t n, const int64_t* off, int64_t nseg, hipStream_t st,
                   bool prepare_only = false, hipStream_t ls = nullptr, void* const* ptrs = nullptr,
                   const int64_t* lens = nullptr) {
    if (ls == nullptr) ls = st;
    using S = typename C::S;
    using TN = Tune<C, PAIRS>;
    constexpr int T = TN::TWG * TN::TIT;
    // 32-bit keys-only batches take their launch shape from the table
    constexpr bool kShaped = sizeof(S) == 4 && !PAIRS && TN::TWG * TN::TIT == 1024 * 8 && TN::MIT == 16;
    SegShape sh{0, TN::MIT};
    if constexpr (kShaped) {
        std::lock_guard<std::mutex> lk(g_mu);
        sh = resolve_seg_shape(DtypeOf<C>::value, PAIRS, n);
    }
    const bool merge8 = kShaped && sh.merge_items == 8;
    const int CH = TN::MWG * (merge8 ? 8 : TN::MIT);
    S* keys = static_cast<S*>(keys_v);
    const size_t kbytes = round_up((size_t)n * sizeof(S), 256);
    const size_t pbytes = PAIRS ? round_up((size_t)n * 4, 256) : 0;
    const size_t arr = round_up((size_t)(nseg + 1) * 8, 256);
    Workspace* ws = nullptr;
    sr_status s = get_workspace(st, kbytes + pbytes + 4 * arr + 256, &ws);
    if (s != SR_OK || prepare_only) return s;
    char* wd = static_cast<char*>(ws_data(ws));
    S* skeys = reinterpret_cast<S*>(wd);
    uint32_t* spay = PAIRS ? reinterpret_cast<uint32_t*>(wd + kbytes) : nullptr;
    int64_t* tile_pre = reinterpret_cast<int64_t*>(wd + kbytes + pbytes);
    int64_t* chunk_pre = reinterpret_cast<int64_t*>(wd + kbytes + pbytes + arr);
    int* seg_passes = reinterpret_cast<int*>(wd + kbytes + pbytes + 2 * arr);
    SegCtl* sc = reinterpret_cast<SegCtl*>(wd + kbytes + pbytes + 3 * arr);
    int64_t* seg_off = reinterpret_cast<int64_t*>(wd + kbytes + pbytes + 3 * arr + 256);
    int64_t* plan_off = ptrs != nullptr ? seg_off : const_cast<int64_t*>(off);
    {
        ProfScope ps(ls, "seg_plan");
        hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(kSegPlanWG), 0, ls, plan_off, lens, nseg, (int64_t)T,
                           (int64_t)CH, tile_pre, chunk_pre, seg_passes, sc);
        SR_LAUNCH_CHECK("seg_plan");
    }
    off = plan_off;
    S* const* sptrs = reinterpret_cast<S* const*>(ptrs);
    {
        ProfScope ps(ls, "seg_tile_sort");
        auto kern = k_seg_tile<C, TN::TWG, TN::TIT, PAIRS>;
        int threads = TN::TWG;
        if constexpr (kShaped) {
            if (sh.tile_variant == 1) {
                kern = k_seg_tile<C, 1024, 8, PAIRS>;
                threads = 1024;
            }
        }
        const int64_t grid = std::min<int64_t>(cdiv(n, T) + nseg, resident_blocks(kern, threads));
        hipLaunchKernelGGL(kern, dim3((unsigned)std::max<int64_t>(grid, 1)), dim3(threads), 0, ls, keys, skeys, pay,
                           spay, off, nseg, (const int64_t*)tile_pre, (const int*)seg_passes, (const SegCtl*)sc,
                           sptrs);
        SR_LAUNCH_CHECK("seg_tile_sort");
    }
    const int Mbound = ceil_log2(cdiv(n, T));
    auto mk = k_seg_merge<C, TN::MWG, TN::MIT, PAIRS>;
    if constexpr (kShaped) {
        if (merge8) mk = k_seg_merge<C, TN::MWG, 8, PAIRS>;
    }
    const int64_t mgrid = std::max<int64_t>(1, std::min<int64_t>(cdiv(n, CH) + nseg, resident_blocks(mk, TN::MWG)));
    for (int k = 0; k < Mbound; ++k) {
        ProfScope ps(ls, "seg_merge");
        hipLaunchKernelGGL(mk, dim3((unsigned)mgrid), dim3(TN::MWG), 0, ls, keys, skeys, pay, spay, off, nseg,
                           (const int64_t*)chunk_pre, (const int*)seg_passes, (const SegCtl*)sc, (int64_t)T, k, sptrs);
        SR_LAUNCH_CHECK("seg_merge");
    }
    return SR_OK;
}

// ------------------------------------------------------------ hipGraphs
// With the "graph" option on, the launch sequence of a call is captured once
// per (entry point, dtype, buffers, sizes, stream, options, workspace
// generation) and replayed afterwards with one hipGraphLaunch.  The plan
// stays on the device, so a replay adapts to new data in the same buffers.
bool g_graph = false;
bool g_graph_plain = false;  // plain sorts captured too (both need "graph")

struct GraphKey {
    int kind, dt, dev;
    const void *keys, *pay, *off;
    int64_t n, nseg;
    hipStream_t st;
    int64_t opts[11];
    unsigned long long gen;
    bool operator<(const GraphKey& o) const {
        return std::memcmp(this, &o, sizeof(GraphKey)) < 0;
    }
};
std::map<GraphKey, hipGraphExec_t> g_graphs;

// One private capture stream per device (non-blocking, default priority):
// the legacy null stream cannot be captured.
hipStream_t capture_stream(int dev) {
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    std::lock_guard<std::mutex> lk(mu);
    auto it = streams.find(dev);
    if (it != streams.end()) return it->second;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams[dev] = cs;
    return cs;
}

template <class Launch, class Prepare>
sr_status run_maybe_graph(int kind, int dt, const void* keys, const void* pay, const void* off, int64_t n,
                          int64_t nseg, hipStream_t st, Launch&& launch, Prepare&& prepare) {
    bool use_graph;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        use_graph = g_graph;
    }
    if (!use_graph) return launch(nullptr);
    sr_status s = prepare();  // allocations happen here, outside any capture
    if (s != SR_OK) return s;
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    key.kind = kind;
    key.dt = dt;
    (void)hipGetDevice(&key.dev);
    key.keys = keys;
    key.pay = pay;
    key.off = off;
    key.n = n;
    key.nseg = nseg;
    key.st = st;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        key.opts[0] = g_force_path;
        key.opts[1] = g_partition_min_n;
        key.opts[2] = g_outlier_enabled;
        key.opts[3] = g_tile_variant;
        key.opts[4] = g_merge_items;
        key.opts[5] = g_nontemporal;
        key.opts[6] = g_runs_enabled;
        key.opts[7] = g_few_enabled;
        key.opts[8] = (int64_t)g_tune_version;
        key.opts[9] = g_near_enabled;
        key.opts[10] = g_fan_in;
        auto it = g_ws.find({key.dev, st});
        key.gen = it != g_ws.end() && it->second ? it->second->generation : 0;
    }
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find(key);
        if (it != g_graphs.end()) exec = it->second;
    }
    if (!exec) {
        bool prof;
        {
            std::lock_guard<std::mutex> lk(g_mu);
            prof = g_profile;
            g_profile = false;  // no event records inside a captured graph
        }
        hipStream_t cs = capture_stream(key.dev);
        if (cs == nullptr) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_profile = prof;
            return fail(SR_ERR_DEVICE, "could not create the capture stream");
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            std::lock_guard<std::mutex> lk(g_mu);
            g_profile = prof;
            return hip_fail(e, "hipStreamBeginCapture");
        }
        s = launch(cs);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(cs, &graph);
        {
            std::lock_guard<std::mutex> lk(g_mu);
            g_profile = prof;
        }
        if (s != SR_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        std::lock_guard<std::mutex> lk(g_mu);
        g_graphs[key] = exec;
    }
    hipError_t e = hipGraphLaunch(exec, st);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return SR_OK;
}

// Plain sorts go through the private-capture graph cache only when both the
// "graph" and "graph_plain" options are on (the segmented entry point needs
// "graph" alone); otherwise they launch directly on the caller's stream.
template <class C, bool PAIRS>
sr_status sort_dispatch(int dt, void* keys, uint32_t* pay, int64_t n, hipStream_t st) {
    bool plain_graphs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        plain_graphs = g_graph_plain;
    }
    if (!plain_graphs) return sort_impl<C, PAIRS>(keys, pay, n, st);
    return run_maybe_graph(
        PAIRS ? 1 : 0, dt, keys, pay, nullptr, n, 0, st,
        [&](hipStream_t ls) { return sort_impl<C, PAIRS>(keys, pay, n, st, false, ls); },
        [&]() { return sort_impl<C, PAIRS>(keys, pay, n, st, true); });
}

template <class C, bool PAIRS>
sr_status seg_dispatch(int dt, void* keys, uint32_t* pay, int64_t n, const int64_t* off, int64_t nseg,
                       hipStream_t st) {
    return run_maybe_graph(
        PAIRS ? 3 : 2, dt, keys, pay, off, n, nseg, st,
        [&](hipStream_t ls) { return seg_impl<C, PAIRS>(keys, pay, n, off, nseg, st, false, ls); },
        [&]() { return seg_impl<C, PAIRS>(keys, pay, n, off, nseg, st, true); });
}

int elem_bytes(sr_dtype dt) {
    switch (dt) {
    case SR_INT32: return 4;
    case SR_UINT64: return 8;
    case SR_FLOAT32: return 4;
    default: return 0;
    }
}

sr_status check_keys(sr_dtype dt, const void* keys, size_t n) {
    const int es = elem_bytes(dt);
    if (es == 0) return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (n > 1 && keys == nullptr) return fail(SR_ERR_INVALID_ARGUMENT, "keys is NULL");
    if (n > ((size_t)1 << 36)) return fail(SR_ERR_INVALID_ARGUMENT, "n too large");
    if (keys && ((uintptr_t)keys % (uintptr_t)es) != 0)
        return fail(SR_ERR_INVALID_ARGUMENT, "keys not aligned to the element size");
    return SR_OK;
}

}  // namespace

namespace sr {
sr_status api_fail(sr_status s, const std::string& msg) { return fail(s, msg); }
void api_clear_error() { g_err.clear(); }
sr_status api_check_keys(sr_dtype dt, const void* keys, size_t n) { return check_keys(dt, keys, n); }
}  // namespace sr

// ======================================================================
// C ABI
// ======================================================================
extern "C" {

sr_status sr_sort_keys(sr_dtype dt, void* keys, size_t n, void* stream) {
    g_err.clear();
    sr_status s = check_keys(dt, keys, n);
    if (s != SR_OK) return s;
    if (n <= 1) return SR_OK;
    hipStream_t st = (hipStream_t)stream;
    switch (dt) {
    case SR_INT32: return sort_dispatch<CodecI32, false>(dt, keys, nullptr, (int64_t)n, st);
    case SR_FLOAT32: return sort_dispatch<CodecF32, false>(dt, keys, nullptr, (int64_t)n, st);
    case SR_UINT64: return sort_dispatch<CodecU64, false>(dt, keys, nullptr, (int64_t)n, st);
    }
    return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
}

sr_status sr_sort_keys_noalloc(sr_dtype dt, void* keys, size_t n, void* stream) {
    g_err.clear();
    sr_status s = check_keys(dt, keys, n);
    if (s != SR_OK) return s;
    if (n * (size_t)elem_bytes(dt) > kNoAllocKeyBytes)
        return fail(SR_ERR_INVALID_ARGUMENT, "sr_sort_keys_noalloc: " + std::to_string(n) + " keys of " +
                                                 std::to_string(elem_bytes(dt)) + " bytes exceed its limit of " +
                                                 std::to_string(kNoAllocKeyBytes) + " bytes of keys");
    if (n <= 1) return SR_OK;
    hipStream_t st = (hipStream_t)stream;
    switch (dt) {
    case SR_INT32: return sort_impl<CodecI32, false>(keys, nullptr, (int64_t)n, st, false, nullptr, true);
    case SR_FLOAT32: return sort_impl<CodecF32, false>(keys, nullptr, (int64_t)n, st, false, nullptr, true);
    case SR_UINT64: return sort_impl<CodecU64, false>(keys, nullptr, (int64_t)n, st, false, nullptr, true);
    }
    return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
}

sr_status sr_sort_pairs(sr_dtype dt, void* keys, uint32_t* payload, size_t n, void* stream) {
    g_err.clear();
    sr_status s = check_keys(dt, keys, n);
    if (s != SR_OK) return s;
    if (n > 1 && payload == nullptr) return fail(SR_ERR_INVALID_ARGUMENT, "payload is NULL");
    if (payload && ((uintptr_t)payload & 3u)) return fail(SR_ERR_INVALID_ARGUMENT, "payload not 4-byte aligned");
    if (n <= 1) return SR_OK;
    hipStream_t st = (hipStream_t)stream;
    switch (dt) {
    case SR_INT32: return sort_dispatch<CodecI32, true>(dt, keys, payload, (int64_t)n, st);
    case SR_FLOAT32: return sort_dispatch<CodecF32, true>(dt, keys, payload, (int64_t)n, st);
    case SR_UINT64: return sort_dispatch<CodecU64, true>(dt, keys, payload, (int64_t)n, st);
    }
    return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
}

sr_status sr_sort_segmented(sr_dtype dt, void* keys, uint32_t* payload, size_t n, const int64_t* offsets,
                            size_t nseg, void* stream) {
    g_err.clear();
    sr_status s = check_keys(dt, keys, n);
    if (s != SR_OK) return s;
    if (nseg == 0 || n <= 1) return SR_OK;
    if (offsets == nullptr) return fail(SR_ERR_INVALID_ARGUMENT, "offsets is NULL");
    if ((uintptr_t)offsets & 7u) return fail(SR_ERR_INVALID_ARGUMENT, "offsets not 8-byte aligned");
    if (nseg > ((size_t)1 << 31)) return fail(SR_ERR_INVALID_ARGUMENT, "too many segments");
    if (payload && ((uintptr_t)payload & 3u)) return fail(SR_ERR_INVALID_ARGUMENT, "payload not 4-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nn = (int64_t)n, ns = (int64_t)nseg;
    if (payload) {
        switch (dt) {
        case SR_INT32: return seg_dispatch<CodecI32, true>(dt, keys, payload, nn, offsets, ns, st);
        case SR_FLOAT32: return seg_dispatch<CodecF32, true>(dt, keys, payload, nn, offsets, ns, st);
        case SR_UINT64: return seg_dispatch<CodecU64, true>(dt, keys, payload, nn, offsets, ns, st);
        }
    } else {
        switch (dt) {
        case SR_INT32: return seg_dispatch<CodecI32, false>(dt, keys, nullptr, nn, offsets, ns, st);
        case SR_FLOAT32: return seg_dispatch<CodecF32, false>(dt, keys, nullptr, nn, offsets, ns, st);
        case SR_UINT64: return seg_dispatch<CodecU64, false>(dt, keys, nullptr, nn, offsets, ns, st);
        }
    }
    return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
}

sr_status sr_sort_batch(sr_dtype dt, void* const* keys_ptrs, const int64_t* lens, size_t nseg, size_t total,
                        void* stream) {
    g_err.clear();
    if (elem_bytes(dt) == 0) return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
    if (nseg == 0 || total == 0) return SR_OK;
    if (!keys_ptrs || !lens) return fail(SR_ERR_INVALID_ARGUMENT, "keys_ptrs or lens is NULL");
    if (((uintptr_t)keys_ptrs & 7u) || ((uintptr_t)lens & 7u))
        return fail(SR_ERR_INVALID_ARGUMENT, "keys_ptrs/lens not 8-byte aligned");
    if (total > ((size_t)1 << 36) || nseg > ((size_t)1 << 31)) return fail(SR_ERR_INVALID_ARGUMENT, "batch too large");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nn = (int64_t)total, ns = (int64_t)nseg;
    switch (dt) {
    case SR_INT32: return seg_impl<CodecI32, false>(nullptr, nullptr, nn, nullptr, ns, st, false, nullptr, keys_ptrs, lens);
    case SR_FLOAT32: return seg_impl<CodecF32, false>(nullptr, nullptr, nn, nullptr, ns, st, false, nullptr, keys_ptrs, lens);
    case SR_UINT64: return seg_impl<CodecU64, false>(nullptr, nullptr, nn, nullptr, ns, st, false, nullptr, keys_ptrs, lens);
    }
    return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
}

sr_status sr_reserve(sr_dtype dt, size_t n, size_t nseg, void* stream) {
    g_err.clear();
    if (elem_bytes(dt) == 0) return fail(SR_ERR_INVALID_ARGUMENT, "unknown dtype");
    hipStream_t st = (hipStream_t)stream;
    const int64_t nn = (int64_t)std::max<size_t>(n, 2), ns = (int64_t)std::max<size_t>(nseg, 1);
    sr_status s = SR_OK;
    switch (dt) {
    case SR_INT32:
        s = seg_impl<CodecI32, false>(nullptr, nullptr, nn, nullptr, ns, st, true);
        if (s == SR_OK) s = sort_impl<CodecI32, false>(nullptr, nullptr, nn, st, true);
        break;
    case SR_FLOAT32:
        s = seg_impl<CodecF32, false>(nullptr, nullptr, nn, nullptr, ns, st, true);
        if (s == SR_OK) s = sort_impl<CodecF32, false>(nullptr, nullptr, nn, st, true);
        break;
    case SR_UINT64:
        s = seg_impl<CodecU64, false>(nullptr, nullptr, nn, nullptr, ns, st, true);
        if (s == SR_OK) s = sort_impl<CodecU64, false>(nullptr, nullptr, nn, st, true);
        break;
    }
    return s;
}

sr_status sr_set_workspace(void* buf, size_t bytes, void* stream) {
    g_err.clear();
    if (buf && ((uintptr_t)buf & 255u)) return fail(SR_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
    if (buf && bytes < ((size_t)1 << 20)) return fail(SR_ERR_INVALID_ARGUMENT, "workspace smaller than 1 MiB");
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    // no call in flight on the stream may still use the scratch being replaced
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    Workspace* ws;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        Workspace*& slot = g_ws[{dev, st}];
        if (!slot) slot = new Workspace();
        ws = slot;
    }
    if (ws->base && !ws->external) (void)hipFree(ws->base);
    ws->base = buf;
    ws->bytes = buf ? bytes : 0;
    ws->external = buf != nullptr;
    ws->generation++;
    if (!buf) return SR_OK;
    // the header and the look-back space stay the library's: allocate them
    // now, for the largest sort the buffer can serve (at most bytes / 4 keys)
    Workspace* w = nullptr;
    return get_workspace(st, 256, &w, aux_bound((int64_t)(bytes / 4)));
}

sr_status sr_release_stream(void* stream) {
    g_err.clear();
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    (void)hipGetDevice(&dev);
    Workspace* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find({dev, st});
        if (it == g_ws.end()) return SR_OK;
        ws = it->second;
        g_ws.erase(it);
        g_last.erase(st);
        for (auto gi = g_graphs.begin(); gi != g_graphs.end();) {
            if (gi->first.st == st && gi->first.dev == dev) {
                (void)hipGraphExecDestroy(gi->second);
                gi = g_graphs.erase(gi);
            } else {
                ++gi;
            }
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (ws->hdr) (void)hipFree(ws->hdr);
    if (ws->base && !ws->external) (void)hipFree(ws->base);
    if (ws->aux) (void)hipFree(ws->aux);
    delete ws;
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return SR_OK;
}

sr_status sr_measure(sr_dtype dt, const void* keys, size_t n, int64_t* out_host, void* stream) {
    g_err.clear();
    sr_status s = check_keys(dt, keys, n);
    if (s != SR_OK) return s;
    if (!out_host) return fail(SR_ERR_INVALID_ARGUMENT, "out_host is NULL");
    out_host[0] = out_host[1] = 0;
    if (n <= 1) return SR_OK;
    hipStream_t st = (hipStream_t)stream;
    Workspace* ws = nullptr;
    s = get_workspace(st, 256, &ws);
    if (s != SR_OK) return s;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(ws_data(ws));
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, cnt, 2, 0ull);
    const unsigned g = (unsigned)std::min<int64_t>(cdiv((int64_t)n, kProbeWG * 8), 16384);
    switch (dt) {
    case SR_INT32: hipLaunchKernelGGL(k_count<CodecI32>, dim3(g), dim3(kProbeWG), 0, st, (const uint32_t*)keys, (int64_t)n, cnt); break;
    case SR_FLOAT32: hipLaunchKernelGGL(k_count<CodecF32>, dim3(g), dim3(kProbeWG), 0, st, (const uint32_t*)keys, (int64_t)n, cnt); break;
    case SR_UINT64: hipLaunchKernelGGL(k_count<CodecU64>, dim3(g), dim3(kProbeWG), 0, st, (const uint64_t*)keys, (int64_t)n, cnt); break;
    }
    SR_LAUNCH_CHECK("count");
    unsigned long long h[2];
    hipError_t e = hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    out_host[0] = (int64_t)h[0];
    out_host[1] = (int64_t)h[1];
    return SR_OK;
}

sr_status sr_workspace_bytes(sr_dtype dt, int with_payload, size_t n, size_t nseg, size_t* bytes) {
    g_err.clear();
    const int es = elem_bytes(dt);
    if (es == 0 || !bytes) return fail(SR_ERR_INVALID_ARGUMENT, "bad argument");
    // upper bound of what sort_impl / seg_impl allocate, over every tuning:
    // header; co-ranks (smallest merge chunk 2048, plus one per run leaf
    // group); the partner array (keys, payload); outlier / run-scan tile
    // arrays per 4096 keys (4 words, a 512-byte kept mask, a RunTile) and the
    // run plan; segment plan arrays
    const size_t ncls = n / kClsTC + 1;
    size_t b = kHdrBytes + round_up((n / 2048 + 2 + kRunMaxLeaves) * 8, 256);
    b += round_up(n * (size_t)es, 256) +
         (with_payload ? round_up(n * 4, 256) + round_up((n / 4 + 1) * 8, 256) : 0);
    b += 4 * round_up(round_up(ncls, (size_t)kVerRound) * 8, 256) + round_up(ncls * (kClsTC / 8), 256);
    b += round_up(ncls * sizeof(RunTile), 256) + round_up(sizeof(RunArea), 256);
    b += round_up((nseg + 1) * 8 * 4, 256);
    *bytes = std::max(b, (size_t)1 << 20);
    return SR_OK;
}

sr_status sr_last_stats(void* stream, sr_stats* out) {
    g_err.clear();
    if (!out) return fail(SR_ERR_INVALID_ARGUMENT, "out is NULL");
    hipStream_t st = (hipStream_t)stream;
    LastCall lc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_last.find(st);
        if (it == g_last.end()) return fail(SR_ERR_INVALID_ARGUMENT, "no sort on this stream yet");
        lc = it->second;
    }
    std::memset(out, 0, sizeof(*out));
    out->n = lc.n;
    if (lc.trivial) {
        out->path = SR_PATH_TRIVIAL;
        out->passes = 1;
    } else {
        Ctl h;
        hipError_t e = hipMemcpyAsync(&h, lc.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        out->path = h.path;
        out->descents = (int64_t)h.reserved[0];
        double eq = 0;  // read+write passes over n, as a real number
        switch (h.path) {
        case SR_PATH_SORTED: eq = 0; break;
        case SR_PATH_REVERSED: eq = 1; break;
        case SR_PATH_OUTLIER: {
            const double m = (double)h.m;
            out->outliers = (int64_t)h.m;
            // classify (n read, n written) + outlier sort (tile + P merges on m)
            // + final merge of kept and outliers (n read, n written); pairs:
            // two placement passes, the outliers' (m) and the kept pairs' (n)
            out->merge_passes = h.job_passes + (lc.pairs ? 2 : 1);
            eq = 2.0 + (lc.pairs ? 2.0 + h.job_passes : 1.0 + h.job_passes) * m / (double)lc.n;
            break;
        }
        case SR_PATH_FEW: {
            // keys: bucket count (n read, m written) + sort of the m between
            // keys + fill (n written, m read); pairs (m = 0): count (keys
            // read) + placement (n read, n written) + copy back
            const double m = (double)h.m;
            out->outliers = (int64_t)h.m;
            out->merge_passes = h.job_passes + 1;
            eq = lc.pairs ? 2.0 + 0.5 * (double)(lc.es - 4) / (double)lc.es
                          : 1.0 + (2.0 + h.job_passes) * m / (double)lc.n;
            break;
        }
        case SR_PATH_NEAR:
            // tile sort, two neighbour rounds, and a copy back when the
            // second round had to write the partner buffer
            out->merge_passes = 2 + (lc.merge_passes & 1);
            eq = 1 + out->merge_passes;
            break;
        case SR_PATH_RUNS: {
            // run scan (n read) + reversal and dense tile sorts + merge tree
            out->run_leaves = (int64_t)h.run[0];
            out->merge_passes = (int32_t)h.run[1];
            eq = 0.5 + (double)(h.run[2] + h.run[3]) / (double)lc.n + (double)h.run[1];
            break;
        }
        default:
            // four-way passes merge two levels each (the last alone when odd)
            out->merge_passes = lc.fan4 ? lc.merge_passes / 2 + (lc.merge_passes & 1) : lc.merge_passes;
            eq = 1 + out->merge_passes;
            break;
        }
        out->passes = (int32_t)std::ceil(eq - 1e-9);
        out->bytes_moved = eq * 2.0 * (double)lc.n * (double)lc.es;
        return SR_OK;
    }
    out->bytes_moved = (double)out->passes * 2.0 * (double)lc.n * (double)lc.es;
    return SR_OK;
}

const char* sr_status_str(sr_status s) {
    switch (s) {
    case SR_OK: return "ok";
    case SR_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SR_ERR_UNSUPPORTED: return "unsupported";
    case SR_ERR_OUT_OF_MEMORY: return "out of memory";
    case SR_ERR_DEVICE: return "device error";
    case SR_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* sr_last_error_message(void) { return g_err.c_str(); }

sr_status sr_set_option(const char* name, int64_t value) {
    g_err.clear();
    if (!name) return fail(SR_ERR_INVALID_ARGUMENT, "name is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    if (std::strcmp(name, "force_path") == 0) {
        if (value < -1 || value > SR_PATH_NEAR) return fail(SR_ERR_INVALID_ARGUMENT, "bad force_path");
        g_force_path = (int)value;
        return SR_OK;
    }
    if (std::strcmp(name, "partition_min_n") == 0) {
        if (value < -1) return fail(SR_ERR_INVALID_ARGUMENT, "partition_min_n >= -1");
        g_partition_min_n = value;
        return SR_OK;
    }
    if (std::strcmp(name, "graph") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "graph is 0 or 1");
        g_graph = value != 0;
        return SR_OK;
    }
    if (std::strcmp(name, "graph_plain") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "graph_plain is 0 or 1");
        g_graph_plain = value != 0;
        return SR_OK;
    }
    if (std::strcmp(name, "tile_variant") == 0) {
        if (value < -1 || value > 1) return fail(SR_ERR_INVALID_ARGUMENT, "tile_variant is -1, 0 or 1");
        g_tile_variant = (int)value;
        return SR_OK;
    }
    if (std::strcmp(name, "merge_items") == 0) {
        if (value != 0 && value != 8 && value != 16)
            return fail(SR_ERR_INVALID_ARGUMENT, "merge_items is 0, 8 or 16");
        g_merge_items = (int)value;
        return SR_OK;
    }
    if (std::strcmp(name, "merge_nontemporal") == 0) {
        if (value < -1 || value > 1) return fail(SR_ERR_INVALID_ARGUMENT, "merge_nontemporal is -1, 0 or 1");
        g_nontemporal = (int)value;
        return SR_OK;
    }
    if (std::strcmp(name, "fan_in") == 0) {
        if (value != 0 && value != 2 && value != 4) return fail(SR_ERR_INVALID_ARGUMENT, "fan_in is 0, 2 or 4");
        g_fan_in = (int)value;
        return SR_OK;
    }
    if (std::strcmp(name, "outlier_path") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "outlier_path is 0 or 1");
        g_outlier_enabled = value != 0;
        return SR_OK;
    }
    if (std::strcmp(name, "near_path") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "near_path is 0 or 1");
        g_near_enabled = value != 0;
        return SR_OK;
    }
    if (std::strcmp(name, "few_path") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "few_path is 0 or 1");
        g_few_enabled = value != 0;
        return SR_OK;
    }
    if (std::strcmp(name, "runs_path") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "runs_path is 0 or 1");
        g_runs_enabled = value != 0;
        return SR_OK;
    }
    if (std::strcmp(name, "profile") == 0) {
        if (value != 0 && value != 1) return fail(SR_ERR_INVALID_ARGUMENT, "profile is 0 or 1");
        g_profile = value != 0;
        return SR_OK;
    }
    return fail(SR_ERR_INVALID_ARGUMENT, std::string("unknown option ") + name);
}

sr_status sr_tune_set(const sr_tune_entry* entries, int64_t count) {
    g_err.clear();
    if (count < 0 || count > kTuneMaxRows) return fail(SR_ERR_INVALID_ARGUMENT, "count is 0..1024");
    if (count > 0 && !entries) return fail(SR_ERR_INVALID_ARGUMENT, "entries is NULL");
    std::vector<sr_tune_entry> rows(entries, entries + count);
    for (int64_t i = 0; i < count; ++i) {
        const sr_tune_entry& e = rows[(size_t)i];
        const std::string at = "tuning row " + std::to_string(i) + ": ";
        if (e.dtype < SR_INT32 || e.dtype > SR_FLOAT32) return fail(SR_ERR_INVALID_ARGUMENT, at + "bad dtype");
        if (e.pairs != 0 && e.pairs != 1) return fail(SR_ERR_INVALID_ARGUMENT, at + "pairs is 0 or 1");
        if (e.min_n < 0) return fail(SR_ERR_INVALID_ARGUMENT, at + "min_n < 0");
        if (e.tile_variant < -1 || e.tile_variant > 1)
            return fail(SR_ERR_INVALID_ARGUMENT, at + "tile_variant is -1, 0 or 1");
        if (e.merge_items != 0 && e.merge_items != 8 && e.merge_items != 16)
            return fail(SR_ERR_INVALID_ARGUMENT, at + "merge_items is 0, 8 or 16");
        if (e.partition < -1 || e.partition > 1) return fail(SR_ERR_INVALID_ARGUMENT, at + "partition is -1, 0 or 1");
        if (e.nontemporal < -1 || e.nontemporal > 1)
            return fail(SR_ERR_INVALID_ARGUMENT, at + "nontemporal is -1, 0 or 1");
        if (e.segmented != 0 && e.segmented != 1) return fail(SR_ERR_INVALID_ARGUMENT, at + "segmented is 0 or 1");
        if (e.segmented && (e.partition != -1 || e.nontemporal != -1))
            return fail(SR_ERR_INVALID_ARGUMENT, at + "segmented rows leave partition and nontemporal unset");
        if (e.fan_in != 0 && e.fan_in != 2 && e.fan_in != 4)
            return fail(SR_ERR_INVALID_ARGUMENT, at + "fan_in is 0, 2 or 4");
        if ((e.segmented || e.pairs) && e.fan_in == 4)
            return fail(SR_ERR_INVALID_ARGUMENT, at + "fan_in 4 is for plain keys-only sorts");
    }
    auto before = [](const sr_tune_entry& a, const sr_tune_entry& b) {
        if (a.dtype != b.dtype) return a.dtype < b.dtype;
        if (a.pairs != b.pairs) return a.pairs < b.pairs;
        if (a.segmented != b.segmented) return a.segmented < b.segmented;
        return a.min_n < b.min_n;
    };
    std::sort(rows.begin(), rows.end(), before);
    for (size_t i = 1; i < rows.size(); ++i)
        if (!before(rows[i - 1], rows[i]))
            return fail(SR_ERR_INVALID_ARGUMENT, "two tuning rows with the same dtype, pairs, segmented and min_n");
    std::lock_guard<std::mutex> lk(g_mu);
    g_tune.swap(rows);
    ++g_tune_version;
    return SR_OK;
}

sr_status sr_tune_get(sr_tune_entry* out, int64_t cap, int64_t* count) {
    g_err.clear();
    if (!count) return fail(SR_ERR_INVALID_ARGUMENT, "count is NULL");
    if (cap < 0 || (cap > 0 && !out)) return fail(SR_ERR_INVALID_ARGUMENT, "bad output buffer");
    std::lock_guard<std::mutex> lk(g_mu);
    *count = (int64_t)g_tune.size();
    for (int64_t i = 0; i < cap && i < (int64_t)g_tune.size(); ++i) out[i] = g_tune[(size_t)i];
    return SR_OK;
}

sr_status sr_profile_collect(const char* prefix, int64_t* launches, double* total_ms) {
    g_err.clear();
    if (!launches || !total_ms) return fail(SR_ERR_INVALID_ARGUMENT, "NULL output");
    const size_t pl = prefix ? std::strlen(prefix) : 0;
    std::vector<ProfRec> mine;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        std::vector<ProfRec> keep;
        for (auto& r : g_prof) {
            if (pl == 0 || r.name.compare(0, pl, prefix) == 0) mine.push_back(r);
            else keep.push_back(r);
        }
        g_prof.swap(keep);
    }
    int64_t cnt = 0;
    double ms = 0;
    sr_status st = SR_OK;
    for (auto& r : mine) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess && st == SR_OK) st = hip_fail(e, "hipEventSynchronize");
        float t = 0;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
            ms += t;
            cnt++;
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto& r : mine) {
            g_event_pool.push_back(r.a);
            g_event_pool.push_back(r.b);
        }
    }
    *launches = cnt;
    *total_ms = ms;
    return st;
}

sr_status sr_copy_bandwidth_probe(void* dst, const void* src, size_t bytes, void* stream) {
    g_err.clear();
    if (!dst || !src || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return fail(SR_ERR_INVALID_ARGUMENT, "copy probe needs 16-byte aligned buffers and size");
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return SR_OK;
    ProfScope ps((hipStream_t)stream, "copy16");
    // one 16-byte element per thread over the whole range: the fastest copy
    // shape measured on MI355X (grid-stride grids of 1K-64K workgroups are
    // 8-25 % slower)
    const unsigned g = (unsigned)std::min<int64_t>(cdiv(n16, 256), (int64_t)1 << 30);
    hipLaunchKernelGGL(k_copy16, dim3(g), dim3(256), 0, (hipStream_t)stream, (uint4*)dst, (const uint4*)src, n16);
    SR_LAUNCH_CHECK("copy16");
    return SR_OK;
}

}  // extern "C"
