/*
 * sortrace.h -- C ABI of libsortrace, an MI355X (gfx950) adaptive merge sort.
 *
 * The problem every call solves is the one stated in Sec. 1 and Appendix A
 * of Zhang, Meng, Liang, "Sort Race" (arXiv 1609.04471): n elements are put
 * into ascending order under one fixed ordering, in place, through a
 * qsort-like call.  Here the ordering is fixed per dtype instead of a
 * comparison function:
 *   SR_INT32    two's-complement signed order
 *   SR_UINT64   unsigned order
 *   SR_FLOAT32  IEEE 754-2008 totalOrder on the bit pattern (-NaN < -Inf <
 *               ... < -0 < +0 < ... < +Inf < +NaN, payloads ordered); bits are
 *               never changed, so the sorted output is unique.
 * Key+payload sorts are stable (Sec. 6: stability is the mergesort property
 * that matters; Sec. 3 (a): equal elements keep their input order).
 *
 * Conventions shared by every call:
 *  - Pointers to keys, payloads and offsets are DEVICE pointers owned by the
 *    caller (for example torch.Tensor.data_ptr()); the library never frees
 *    them.  Keys need their natural alignment (4 bytes for 32-bit dtypes, 8
 *    for SR_UINT64), payloads 4 bytes; 16-byte alignment is not required.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls are asynchronous: they return once the work is enqueued on
 *    `stream`, and the result is in place when the stream reaches that point.
 *    No call in the sort path copies data back to the host or synchronizes.
 *    Other streams must not touch the buffers meanwhile.  Host threads may
 *    call concurrently on different streams.
 *  - Scratch memory: the library owns one workspace per (device, stream),
 *    grown on demand (a call that grows it synchronizes `stream` once first).
 *  - Errors: everything checkable on the host is checked before anything is
 *    enqueued, so on error the inputs are untouched.  n <= 1 (or nseg == 0)
 *    is a no-op returning SR_OK.  A failed HIP launch returns SR_ERR_DEVICE
 *    with the HIP message in sr_last_error_message().
 */
#ifndef SORTRACE_H
#define SORTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SR_INT32 = 0, SR_UINT64 = 1, SR_FLOAT32 = 2 } sr_dtype;

typedef enum {
    SR_OK = 0,
    SR_ERR_INVALID_ARGUMENT = 1,
    SR_ERR_UNSUPPORTED = 2,
    SR_ERR_OUT_OF_MEMORY = 3,
    SR_ERR_DEVICE = 4,
    SR_ERR_INTERNAL = 5
} sr_status;

/* The path the device plan chose for the last sort on a stream. */
typedef enum {
    SR_PATH_TRIVIAL = -1,  /* n <= 1, or small enough for one tile: no probe */
    SR_PATH_SORTED = 0,    /* already nondecreasing: nothing written */
    SR_PATH_REVERSED = 1,  /* nonincreasing: reversed in place (stable for pairs) */
    SR_PATH_OUTLIER = 2,   /* nearly sorted: outliers split off, sorted, merged back
                              (pairs: at most n/4 outliers, n < 2^32; an outlier
                              and a kept key with equal keys keep input order) */
    SR_PATH_GENERAL = 3,   /* tile sort + merge passes */
    SR_PATH_RUNS = 4,      /* natural runs (keys and pairs; for pairs the reversal
                              keeps equal keys in input order):
                              descending runs reversed in
                              place, disordered tiles sorted, runs whose values are
                              already in order joined, then a merge tree over the
                              remaining leaves (Sec. 3 natural runs, Sec. 2 Mono) */
    SR_PATH_FEW = 5,       /* few distinct keys: equal buckets around at most 4096
                              sampled values -- the GPU form of 3-way partitioning
                              (Sec. 4, k-limited of Sec. 2, Table 1's 12-limited
                              few-unique type); keys between the sampled values
                              are sorted separately.  Pairs: at most 64 values,
                              every key equal to one of them, n <= 4,194,304;
                              each key and payload is placed in input order among
                              its equals (stable) */
    SR_PATH_NEAR = 6       /* tile sort, then two rounds of neighbour merges: tile
                              pairs (0,1),(2,3),... and then (1,2),(3,4),...; taken
                              when the sorted tiles show that every tile overlaps
                              only its neighbours, by at most half a tile (keys
                              displaced by less than half a tile: the k-distance
                              class of Sec. 2, Table 1's nearly sorted type); keys
                              and pairs.  Reported on the general plan's launches:
                              a sort that is not NEAR-shaped takes the full merge
                              tree instead */
} sr_path;

typedef struct {
    int32_t path;          /* sr_path */
    int32_t passes;        /* read+write passes over the n keys, rounded up; a pass
                              over m < n keys counts m/n (the probe's reads are
                              not counted) */
    int64_t n;             /* keys sorted by the call */
    int64_t descents;      /* probe: descents seen (exact when path is SORTED/REVERSED) */
    int64_t outliers;      /* OUTLIER path: keys moved to the outlier list; FEW path:
                              keys not equal to any sampled value */
    double bytes_moved;    /* algorithmic HBM bytes: unrounded passes x 2 x n x element bytes */
    int64_t run_leaves;    /* RUNS path: sorted leaves left after the in-order joins */
    int32_t merge_passes;  /* merge passes of the chosen path (RUNS: over its leaves;
                              GENERAL with fan-in four: passes over the array, a
                              four-way pass counting once) */
    int32_t pad;
} sr_stats;

/*
 * Sort n keys of type dt in place at device pointer `keys`.  The
 * ascending order of Sec. 1; equal keys are bit-identical, so the result is
 * the unique sorted permutation.
 * Errors: SR_ERR_INVALID_ARGUMENT for keys == NULL with n > 1, a bad dtype or
 * a misaligned pointer; SR_ERR_UNSUPPORTED when `stream` is capturing into a
 * graph (plain sorts are launched directly; sr_sort_segmented has a graph
 * option of its own), before anything is enqueued.
 */
sr_status sr_sort_keys(sr_dtype dt, void *keys, size_t n, void *stream);

/*
 * Stable sort of (key, payload) records in place: keys at `keys` (type dt),
 * payload[i] travels with keys[i].  Among equal keys the input order is kept
 * (Sec. 3 (a), Sec. 6).  payload must not be NULL when n > 1.  Errors as
 * sr_sort_keys.
 */
sr_status sr_sort_pairs(sr_dtype dt, void *keys, uint32_t *payload, size_t n, void *stream);

/*
 * Segmented sort: every segment [offsets[s], offsets[s+1]) of `keys` (and of
 * `payload` when it is not NULL, stable) is sorted on its own, all in one
 * batch of launches.  `offsets` is a DEVICE array of nseg + 1 int64 with
 * offsets[0] == 0, nondecreasing, offsets[nseg] == n; empty segments are
 * allowed.  These preconditions are the caller's: they are not checked on the
 * device.
 */
sr_status sr_sort_segmented(sr_dtype dt, void *keys, uint32_t *payload, size_t n,
                            const int64_t *offsets, size_t nseg, void *stream);

/*
 * Heavy items (Sec. 2: random lists of 16, 64 or 256 integers): n lists of
 * `words` int32 each, row-major at device pointer `lists` (list i at
 * lists + i * words), sorted in place into word-by-word order from the first
 * word (each word a signed int32; the first unequal word decides), stable
 * (equal lists keep their input order).  The lists are ordered through
 * 64-bit prefix keys of two words with the list index as payload (a stable
 * pairs sort), ties refined two words at a time by segmented sorts of the
 * tied positions, then gathered once.  The call allocates its scratch with
 * hipMalloc (about 40 bytes per list plus one copy of the lists), reads the
 * tie count back after each refinement round, and synchronizes `stream`.
 * Errors: words outside 1 .. 2^20, n above 2^32 - 1, NULL or misaligned
 * lists (SR_ERR_INVALID_ARGUMENT); no memory (SR_ERR_OUT_OF_MEMORY).
 */
sr_status sr_sort_lists(int32_t *lists, size_t n, int32_t words, void *stream);

/*
 * Batched sort of nseg independent arrays, each in its own device buffer:
 * array s starts at keys_ptrs[s] and has lens[s] keys of type dt.  keys_ptrs
 * and lens are DEVICE arrays (8-byte aligned) of nseg entries; total is the
 * sum of lens (known to the caller; it sizes the launch and the scratch).
 * Each array ends up sorted in place exactly as sr_sort_keys would leave it
 * (Sec. 1's problem, once per array), all of them in one set of launches.
 * Keys only.  The lens must sum to total; this is not checked on the device.
 */
sr_status sr_sort_batch(sr_dtype dt, void *const *keys_ptrs, const int64_t *lens, size_t nseg, size_t total,
                        void *stream);

/*
 * Sizes the workspace of `stream` for keys-only sorts of up to n keys (and
 * batches of up to nseg arrays), so that later calls up to that size never
 * allocate or synchronize.  May synchronize `stream` once.
 */
sr_status sr_reserve(sr_dtype dt, size_t n, size_t nseg, void *stream);

/*
 * Hands the library a caller-owned device buffer of `bytes` bytes at `buf` as
 * the data scratch of `stream` on the current device (merge co-ranks, the
 * partner array of the merge passes, segment plans): later calls on the
 * stream use it instead of scratch of their own, so an application can
 * budget, pool or place that memory itself.  buf must be 256-byte aligned and
 * bytes >= 1 MiB; sr_workspace_bytes gives a sufficient size for a call
 * shape.  The library keeps a fixed 128 KiB header and the look-back arrays
 * of the presortedness paths (about 3.5 % of bytes) in memory of its own,
 * allocated by this call for up to bytes / 4 keys, so a later sort whose
 * scratch fits allocates nothing; one that does not fit returns
 * SR_ERR_INVALID_ARGUMENT before it enqueues anything (the keys untouched).
 * The call synchronizes `stream` and frees data scratch the library held for
 * it.  buf == NULL gives the scratch back to the library (the next call
 * allocates its own).  The caller keeps ownership: the buffer must stay
 * allocated and untouched until the stream has finished its last call and
 * another buffer, NULL, or sr_release_stream has replaced it.  sr_sort_lists
 * and sr_measure_presortedness allocate their own extra scratch regardless.
 */
sr_status sr_set_workspace(void *buf, size_t bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code recorded into a
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * sr_sort_keys with no allocation.  Same arguments, order and result as
 * sr_sort_keys, but its whole workspace (control block, look-back space and
 * the merge passes' partner array) is one fixed array of 36 MiB per device
 * that the library's code object holds until the process ends, so no call
 * allocates or frees anything.  Limit: n x element size <= 32 MiB (8,388,608
 * int32 or float32 keys, 4,194,304 uint64 keys); a larger n returns
 * SR_ERR_INVALID_ARGUMENT before anything is enqueued.  The first call on a
 * device initialises that device's array on `stream` and waits for it (one
 * synchronization, ever).  Every call on a device shares its one array, which
 * keeps the last call's contents: calls whose work overlaps on one device --
 * on different streams, or from different host threads, without ordering
 * between them -- race and give wrong results; order them on one stream.
 * sr_last_stats does not report these calls.  Errors as sr_sort_keys.
 */
sr_status sr_sort_keys_noalloc(sr_dtype dt, void *keys, size_t n, void *stream);

/* Frees the workspace the library holds for `stream` on the current device
 * (after synchronizing it; a buffer set by sr_set_workspace is the caller's
 * and is not freed).  Call before destroying a stream that sorted. */
sr_status sr_release_stream(void *stream);

/*
 * Continuous-batching sort server (serving).  Requests reference keys that
 * already reside in device memory and carry an arrival time (seconds on the
 * server's clock, sr_server_now()); submit them in arrival order.  A worker
 * thread admits arrived requests in FIFO order while the HBM footprint of
 * admitted, unfinished requests (2 x n x element bytes: keys plus scratch)
 * stays within hbm_budget_bytes, groups admitted requests of one dtype into a
 * batch (up to max_batch_requests arrays and max_batch_keys keys) whenever
 * one of its `streams` streams is idle, and sorts the batch there with
 * sr_sort_batch (sr_sort_keys for a batch of one).  Batches on different
 * streams overlap on the device.  streams = 1 with max_batch_requests = 1 is
 * the plain one-at-a-time FIFO server.  Every result is what sr_sort_keys
 * gives for the same array alone.  Scratch: sr_server_create reserves, on
 * every stream, the workspace of a batch of max_batch_keys keys of each
 * dtype (int32, float32, uint64), so the worker never allocates; the
 * footprint charged per request (2 x n x element bytes) is the admission
 * rule's bookkeeping of the keys plus the share of that reserved scratch its
 * sort uses.
 */
typedef struct sr_server sr_server;

typedef struct {
    size_t hbm_budget_bytes;   /* admission budget for keys + scratch of unfinished requests */
    int streams;               /* 1..16 batches in flight */
    int max_batch_requests;    /* arrays per batch (>= 1) */
    size_t max_batch_keys;     /* keys per batch, also the largest admissible request */
} sr_server_config;

typedef struct {
    uint64_t tag;
    int32_t dtype;
    int32_t batch;             /* batch id the request ran in */
    int64_t n;
    int32_t status;            /* sr_status of its sort */
    int32_t pad;
    double t_arrive, t_admit, t_launch, t_done;  /* seconds, server clock; t_done from the batch's completion event */
} sr_request_record;

sr_status sr_server_create(const sr_server_config *cfg, sr_server **out);
/* ready_event: NULL, or a hipEvent_t recorded on the producer's stream after
 * the keys were written; the batch's stream waits for it before the sort, so
 * keys produced asynchronously are never sorted early.  The event must stay
 * valid until the request is reported finished.  Errors: a request whose
 * footprint exceeds the budget or max_batch_keys, or an arrival earlier than
 * the previous submission's. */
sr_status sr_server_submit(sr_server *s, sr_dtype dt, void *keys, size_t n, uint64_t tag, double t_arrive,
                           void *ready_event);
double sr_server_now(sr_server *s);
/* Waits until every submitted request has finished (SR_ERR_INTERNAL on timeout). */
sr_status sr_server_wait_idle(sr_server *s, double timeout_s);
/* Moves up to cap finished requests (completion order) into out (host memory). */
sr_status sr_server_records(sr_server *s, sr_request_record *out, size_t cap, size_t *count);
sr_status sr_server_destroy(sr_server *s);

/*
 * Presortedness of keys (Sec. 2): out_host[0] = number of descents
 * a_i > a_{i+1} (Run(A) = descents + 1), out_host[1] = number of ascents
 * a_i < a_{i+1}.  out_host is HOST memory; this call synchronizes `stream`.
 */
sr_status sr_measure(sr_dtype dt, const void *keys, size_t n, int64_t *out_host, void *stream);

/*
 * The three presortedness measures of Sec. 2 on the device (keys are not
 * modified; they are compared in the order the sort uses):
 *   Run(A)  = |{i : a_i > a_{i+1}}| + 1;
 *   Mono(A) = the least k such that A is a concatenation of k contiguous
 *             pieces, each sorted or reversely sorted (nondecreasing or
 *             nonincreasing; a piece of equal keys is both);
 *   Inv(A)  = |{(i, j) : i < j, a_i > a_j}|, only when flags has
 *             SR_MEASURE_INV (it costs a merge sort of a copy:
 *             log2(n/16) + 1 launches over 2 x n x key-size bytes of scratch).
 * For n = 0 every measure is 0; for n = 1, run = mono = 1.
 * out_host is HOST memory; the call allocates its scratch with hipMalloc,
 * frees it, and synchronizes `stream`.  Errors: bad arguments as for
 * sr_sort_keys, an unknown flag, NULL out_host (SR_ERR_INVALID_ARGUMENT);
 * no memory for the scratch (SR_ERR_OUT_OF_MEMORY).
 */
typedef struct {
    int64_t descents;  /* |{i : a_i > a_{i+1}}| */
    int64_t ascents;   /* |{i : a_i < a_{i+1}}| */
    int64_t run;       /* Run(A) */
    int64_t mono;      /* Mono(A) */
    int64_t inv;       /* Inv(A); -1 when not asked for */
} sr_presortedness;

#define SR_MEASURE_INV 1

sr_status sr_measure_presortedness(sr_dtype dt, const void *keys, size_t n, int32_t flags,
                                   sr_presortedness *out_host, void *stream);

/* Workspace bytes the library would hold for a call of this shape (an upper
 * bound; also a sufficient `bytes` for sr_set_workspace). */
sr_status sr_workspace_bytes(sr_dtype dt, int with_payload, size_t n, size_t nseg, size_t *bytes);

/*
 * Statistics of the last sr_sort_keys / sr_sort_pairs on `stream`.  Reads
 * the device plan back, so it synchronizes `stream`.  out is host memory.
 */
sr_status sr_last_stats(void *stream, sr_stats *out);

/* Static text for a status code. */
const char *sr_status_str(sr_status s);

/* Detail of the last error on the calling host thread ("" if none). */
const char *sr_last_error_message(void);

/*
 * Options (process-wide).  Names:
 *   "force_path"  -1 = let the device plan decide (default); otherwise an
 *                 sr_path value the plan is forced to when it is safe
 *                 (SR_PATH_GENERAL is always safe; forcing it also rules out
                 SR_PATH_NEAR, so the full merge tree runs).
 *   "profile"     1 = record a HIP event pair around every kernel the sort
 *                 path launches (on the caller's stream); 0 = off (default).
 *   "outlier_path" 1 = sorts may take SR_PATH_OUTLIER (default);
 *                 0 = never (nearly sorted input then takes SR_PATH_GENERAL).
 *   "few_path"    1 = sorts may take SR_PATH_FEW (default); 0 = never.
 *                 A forced SR_PATH_FEW still falls back to SR_PATH_GENERAL when
 *                 more than a quarter of the keys miss the sampled values.
 *   "near_path"   1 = general sorts may finish as SR_PATH_NEAR when their
 *                 sorted tiles allow it (default); 0 = never.
 *   "runs_path"   1 = keys-only and pairs sorts may take SR_PATH_RUNS
 *                 (default); 0 = never.
 *                 A forced SR_PATH_RUNS still falls back to SR_PATH_GENERAL
 *                 when the run plan exceeds its limits (4096 runs and dense
 *                 pieces, 2048 leaves, half the keys in dense tiles).
 *   "graph"       1 = sr_sort_segmented captures its launch sequence in a
 *                 hipGraph the first time a (dtype, buffers, sizes, stream,
 *                 options) combination is seen, and replays it afterwards
 *                 with one hipGraphLaunch (the segment plan is recomputed on
 *                 the device, so new data and new offsets in the same buffers
 *                 are handled); 0 = plain launches (default).
 *   "graph_plain" 1 = with "graph" on, sr_sort_keys / sr_sort_pairs use the
 *                 same capture-and-replay cache; 0 = they launch directly
 *                 (default).
 * Recording into the caller's own stream capture: sr_sort_keys,
 * sr_sort_pairs and sr_sort_keys_noalloc may be called on a capturing stream
 * when they need no allocation there -- the stream's workspace already holds
 * the size (sr_reserve, sr_set_workspace, or an earlier sort of that size on
 * the stream; for sr_sort_keys_noalloc, an earlier call on the device) --
 * else they return SR_ERR_UNSUPPORTED and record nothing.  Each replay sorts
 * the buffers as they are at replay time.
 * The four launch-shape options below default to "auto": the matching row
 * of the tuning table (sr_tune_set) decides, else the built-in rule given
 * with each.  A value set here overrides the table for every sort.
 *   "tile_variant" 32-bit keys only: 0 = tile sort by 512 threads x 16 keys,
 *                 1 = 1024 threads x 8 keys (same 8192-key tile), -1 = auto
 *                 (built-in: 1 without a partition launch, else 0).
 *   "merge_items"  32-bit keys only, merge passes without a partition
 *                 launch: outputs per thread, 8 or 16; 0 = auto (built-in:
 *                 16 from n = 2^21 on, else 8).
 *   "partition_min_n"  from this n on, every merge pass is preceded by a
 *                 separate Merge Path partition launch and merged by a
 *                 persistent grid; below it each merge workgroup searches
 *                 its own window bounds.  -1 = auto (built-in 2^23).
 *   "merge_nontemporal"  persistent merge passes load their windows and
 *                 store their output with nontemporal hints: 1 = on, 0 = off,
 *                 -1 = auto (built-in: on for keys-only sorts from 256 MiB
 *                 of keys, for uint64 pairs from 128 MiB of keys, never for
 *                 32-bit pairs).
 *   "fan_in"      merge fan-in of keys-only general sorts that use the
 *                 partition shape: 4 = four-way passes (each group of four
 *                 neighbouring runs is cut at every 2048th key of each run --
 *                 every 1024th for 64-bit keys -- and merged as two levels in
 *                 LDS, so two levels of the merge tree cost one pass over the
 *                 array; a sort that takes this schedule does not try the
 *                 NEAR plan), 2 = two-way, 0 = auto (tuning table, then
 *                 built-in).  Pairs always merge two-way.
 * Returns SR_ERR_INVALID_ARGUMENT for an unknown name or value.
 */
sr_status sr_set_option(const char *name, int64_t value);

/*
 * Tuning table: launch shapes per key type, keys-only or pairs, and size
 * band, as written by the package's autotuner (a sweep of these fields over
 * timed sorts on the device).  A sort of n keys uses the row of its dtype and
 * kind with the largest min_n <= n; a field left at its "unset" value, or a
 * sort no row matches, takes the built-in rule of the option of the same
 * name (sr_set_option).  Fields that do not apply to a key type (tile_variant
 * and merge_items for uint64 keys and for pairs) are ignored.
 */
typedef struct {
    int32_t dtype;         /* sr_dtype */
    int32_t pairs;         /* 0 = sr_sort_keys, 1 = sr_sort_pairs */
    int64_t min_n;         /* the band starts here (>= 0) */
    int32_t tile_variant;  /* 0 or 1; -1 = unset */
    int32_t merge_items;   /* 8 or 16; 0 = unset */
    int32_t partition;     /* 1 = separate partition launch, 0 = fused search; -1 = unset */
    int32_t nontemporal;   /* 1 or 0; -1 = unset */
    int32_t segmented;     /* 0 = plain sorts; 1 = sr_sort_segmented / sr_sort_batch, whose
                              rows are looked up by the total key count and use only
                              tile_variant and merge_items (32-bit keys, keys only;
                              partition and nontemporal must be unset there) */
    int32_t fan_in;        /* merge fan-in of plain keys-only sorts with the partition shape:
                              4 = four-way passes (each merges two levels of the merge
                              tree in one read and one write of the array), 2 = two-way;
                              0 = unset.  Must be 0 or 2 for pairs and segmented rows. */
} sr_tune_entry;

/* Replaces the process-wide tuning table with `count` rows copied from host
 * memory (count 0 clears it; entries may then be NULL).  Rows are validated
 * first: a bad dtype, a negative min_n, a field outside its values, or two
 * rows with the same (dtype, pairs, segmented, min_n) return SR_ERR_INVALID_ARGUMENT and
 * leave the table unchanged.  At most 1024 rows. */
sr_status sr_tune_set(const sr_tune_entry *entries, int64_t count);

/* Copies up to `cap` rows of the table (sorted by dtype, pairs, segmented, min_n) to
 * host memory and stores the row count in *count. */
sr_status sr_tune_get(sr_tune_entry *out, int64_t cap, int64_t *count);

/*
 * With "profile" on: sums the device time of the recorded launches whose
 * kernel name starts with `prefix` ("" = all) and forgets those launches
 * (the others stay recorded).  Synchronizes on the recorded events.  launches and total_ms are
 * host memory.  Kernel names: "probe", "tile_sort" (also carries the
 * reversal), "regroup", "partition", "merge", "classify", "merge_outliers",
 * "seg_plan", "seg_tile_sort", "seg_merge".
 */
sr_status sr_profile_collect(const char *prefix, int64_t *launches, double *total_ms);

/* Device copy kernel (16-byte vectors) used as a bandwidth reference:
 * copies `bytes` (a multiple of 16) from src to dst on `stream`. */
sr_status sr_copy_bandwidth_probe(void *dst, const void *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SORTRACE_H */
