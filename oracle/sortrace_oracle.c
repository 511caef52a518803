/*
 * sortrace_oracle.c -- CPU oracle for libsortrace.  TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct definition that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the HIP library under paper_1609_04471_amd/csrc, and
 * the library never calls it.
 *
 * What it computes (Zhang, Meng, Liang, "Sort Race", arXiv 1609.04471):
 *   - Sec. 1 states the problem: comparison-based internal sorting of n
 *     elements into one fixed order, in place, through a qsort-like call
 *     (array, n, element size, comparison function).  Appendix A fixes the
 *     merge contract: merge(arr, l, m, r) combines the sorted halves
 *     arr[l, m) and arr[m, r) into arr[l, r).
 *   - Sec. 6 names stability as the mergesort property, and Sec. 3 (a)
 *     requires equal elements to keep their input order.
 *   So the keys-only result is the unique nondecreasing permutation of the
 *   input; the key+payload result is the unique stable one (lexicographic on
 *   (key, original index)).
 *
 * The order per dtype is written here from each type's own definition:
 *   int32   two's-complement "<"
 *   uint64  unsigned "<"
 *   float32 IEEE 754-2008 totalOrder on the bit pattern (Sec. 5.10 of that
 *           standard): a negative-signed value precedes a positive-signed
 *           one; among positive-signed patterns a larger bit pattern is
 *           larger; among negative-signed ones a larger pattern is smaller.
 *           The paper compares doubles through a comparator and says nothing
 *           of NaN or signed zero; totalOrder is the reading taken.
 *
 * Functions:
 *   oracle_sort_keys / oracle_sort_pairs   plain stable top-down mergesort
 *                                          (the paper's mergesort is a
 *                                          participant of the race, Sec. 1;
 *                                          merge contract of Appendix A)
 *   oracle_sort_segmented                  the same, per CSR segment
 *   oracle_insertion_sort                  insertion sort (Sec. 1, Sec. 3 (b),
 *                                          Appendix B isort): shifts only
 *                                          while the left neighbour is
 *                                          strictly greater, hence stable
 *   oracle_brute_sort                      O(n^2) definition: repeatedly
 *                                          take the minimum (key, index)
 *   oracle_sort_lists                      the heavy items of Sec. 2: lists
 *                                          of int32 compared word by word
 *                                          (lexicographic), same mergesort
 *   oracle_run / oracle_inv / oracle_mono  presortedness measures of Sec. 2
 *                                          (Run, Inv, Mono)
 *   oracle_sort_keys_parallel              the same mergesort on several host
 *                                          threads (chunks sorted in parallel,
 *                                          then each merge round's merges cut
 *                                          into equal parts by Merge Path
 *                                          co-ranks); used only to time a CPU
 *                                          baseline on all host cores, and
 *                                          checked against oracle_sort_keys
 *
 * Every pointer is host memory owned by the caller.  Return value 0 = OK,
 * -1 = bad argument.  Build: gcc -O2 -shared -fPIC.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_INT32 = 0, OR_UINT64 = 1, OR_FLOAT32 = 2 };

/* ---------------------------------------------------------------- order */

/* One record = key bytes followed by the payload (uint32) when present.  The
 * records are sorted through a comparison function pointer, the interface
 * the paper uses for every method (Sec. 5, Appendix A). */
typedef int (*less_fn)(const unsigned char *a, const unsigned char *b);

static int less_int32(const unsigned char *a, const unsigned char *b)
{
    int32_t x, y;
    memcpy(&x, a, 4);
    memcpy(&y, b, 4);
    return x < y;
}

static int less_uint64(const unsigned char *a, const unsigned char *b)
{
    uint64_t x, y;
    memcpy(&x, a, 8);
    memcpy(&y, b, 8);
    return x < y;
}

static int less_float32_total(const unsigned char *a, const unsigned char *b)
{
    uint32_t x, y;
    memcpy(&x, a, 4);
    memcpy(&y, b, 4);
    unsigned sx = x >> 31, sy = y >> 31;
    if (sx != sy)
        return sx > sy;          /* the negative-signed one is less */
    if (sx == 0)
        return x < y;            /* both positive-signed: ascending bits */
    return x > y;                /* both negative-signed: descending bits */
}

static int key_size(int dtype)
{
    switch (dtype) {
    case OR_INT32: return 4;
    case OR_UINT64: return 8;
    case OR_FLOAT32: return 4;
    default: return 0;
    }
}

static less_fn less_for(int dtype)
{
    switch (dtype) {
    case OR_INT32: return less_int32;
    case OR_UINT64: return less_uint64;
    case OR_FLOAT32: return less_float32_total;
    default: return NULL;
    }
}

/* ------------------------------------------------------ record packing */

typedef struct {
    size_t ks;      /* key bytes */
    size_t rs;      /* record bytes */
    int with_payload;
    less_fn less;
} rec_t;

static unsigned char *pack(const rec_t *r, const void *keys,
                           const uint32_t *payload, size_t n)
{
    unsigned char *buf = (unsigned char *)malloc(n ? n * r->rs : 1);
    if (!buf)
        return NULL;
    for (size_t i = 0; i < n; i++) {
        memcpy(buf + i * r->rs, (const unsigned char *)keys + i * r->ks, r->ks);
        if (r->with_payload)
            memcpy(buf + i * r->rs + r->ks, payload + i, 4);
    }
    return buf;
}

static void unpack(const rec_t *r, const unsigned char *buf, void *keys,
                   uint32_t *payload, size_t n)
{
    for (size_t i = 0; i < n; i++) {
        memcpy((unsigned char *)keys + i * r->ks, buf + i * r->rs, r->ks);
        if (r->with_payload)
            memcpy(payload + i, buf + i * r->rs + r->ks, 4);
    }
}

static int setup(rec_t *r, int dtype, int with_payload)
{
    r->ks = (size_t)key_size(dtype);
    r->less = less_for(dtype);
    if (r->ks == 0 || r->less == NULL)
        return -1;
    r->with_payload = with_payload;
    r->rs = r->ks + (with_payload ? 4 : 0);
    return 0;
}

/* ------------------------------------------------- top-down mergesort */

/* merge(a, lo, mid, hi): the sorted a[lo, mid) and a[mid, hi) become the
 * sorted a[lo, hi) (the Appendix A contract).  On equal keys the left run
 * goes first, so the sort is stable. */
static void merge(const rec_t *r, unsigned char *a, unsigned char *tmp,
                  size_t lo, size_t mid, size_t hi)
{
    size_t i = lo, j = mid, k = lo, rs = r->rs;
    while (i < mid && j < hi) {
        if (r->less(a + j * rs, a + i * rs)) {
            memcpy(tmp + k * rs, a + j * rs, rs);
            j++;
        } else {
            memcpy(tmp + k * rs, a + i * rs, rs);
            i++;
        }
        k++;
    }
    while (i < mid) {
        memcpy(tmp + k * rs, a + i * rs, rs);
        i++;
        k++;
    }
    while (j < hi) {
        memcpy(tmp + k * rs, a + j * rs, rs);
        j++;
        k++;
    }
    memcpy(a + lo * rs, tmp + lo * rs, (hi - lo) * rs);
}

static void msort(const rec_t *r, unsigned char *a, unsigned char *tmp,
                  size_t lo, size_t hi)
{
    if (hi - lo < 2)
        return;
    size_t mid = lo + (hi - lo) / 2;
    msort(r, a, tmp, lo, mid);
    msort(r, a, tmp, mid, hi);
    merge(r, a, tmp, lo, mid, hi);
}

static int sort_records(int dtype, void *keys, uint32_t *payload, size_t n,
                        int with_payload)
{
    rec_t r;
    if (setup(&r, dtype, with_payload) != 0)
        return -1;
    if (n == 0)
        return 0;
    if (keys == NULL || (with_payload && payload == NULL))
        return -1;
    unsigned char *a = pack(&r, keys, payload, n);
    unsigned char *tmp = (unsigned char *)malloc(n * r.rs);
    if (!a || !tmp) {
        free(a);
        free(tmp);
        return -1;
    }
    msort(&r, a, tmp, 0, n);
    unpack(&r, a, keys, payload, n);
    free(a);
    free(tmp);
    return 0;
}

int oracle_sort_keys(int dtype, void *keys, size_t n)
{
    return sort_records(dtype, keys, NULL, n, 0);
}

int oracle_sort_pairs(int dtype, void *keys, uint32_t *payload, size_t n)
{
    return sort_records(dtype, keys, payload, n, 1);
}

/* Each segment [offsets[s], offsets[s+1]) is sorted on its own.  offsets has
 * nseg + 1 entries, starts at 0 and never decreases.  payload may be NULL. */
int oracle_sort_segmented(int dtype, void *keys, uint32_t *payload,
                          const int64_t *offsets, size_t nseg)
{
    int ks = key_size(dtype);
    if (ks == 0)
        return -1;
    if (nseg == 0)
        return 0;
    if (offsets == NULL || offsets[0] != 0)
        return -1;
    for (size_t s = 0; s < nseg; s++) {
        int64_t a = offsets[s], b = offsets[s + 1];
        if (b < a)
            return -1;
        unsigned char *k = (unsigned char *)keys + (size_t)a * (size_t)ks;
        int rc = payload ? sort_records(dtype, k, payload + a, (size_t)(b - a), 1)
                         : sort_records(dtype, k, NULL, (size_t)(b - a), 0);
        if (rc != 0)
            return rc;
    }
    return 0;
}

/* ------------------------------------------- multi-threaded (timing only) */

typedef struct {
    const rec_t *r;
    unsigned char *a, *tmp;
    size_t lo, hi;
} sort_part;

static void *sort_part_run(void *p)
{
    sort_part *j = (sort_part *)p;
    msort(j->r, j->a, j->tmp, j->lo, j->hi);
    return NULL;
}

/* Of the first d records of the stable merge of a[alo, ahi) and a[blo, bhi),
 * how many come from the first run (ties go to the first run). */
static size_t co_rank(const rec_t *r, const unsigned char *a, size_t alo, size_t ahi,
                      size_t blo, size_t bhi, size_t d)
{
    size_t na = ahi - alo, nb = bhi - blo, rs = r->rs;
    size_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
    while (lo < hi) {
        size_t mid = lo + (hi - lo) / 2;
        /* a[alo + mid] is among the first d unless b[blo + d - 1 - mid] precedes it */
        if (!r->less(a + (blo + d - 1 - mid) * rs, a + (alo + mid) * rs))
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

typedef struct {
    const rec_t *r;
    const unsigned char *src;
    unsigned char *dst;
    size_t alo, ahi, blo, bhi, out;
} merge_part;

static void *merge_part_run(void *p)
{
    merge_part *j = (merge_part *)p;
    size_t i = j->alo, k = j->blo, o = j->out, rs = j->r->rs;
    while (i < j->ahi && k < j->bhi) {
        if (j->r->less(j->src + k * rs, j->src + i * rs)) {
            memcpy(j->dst + o * rs, j->src + k * rs, rs);
            k++;
        } else {
            memcpy(j->dst + o * rs, j->src + i * rs, rs);
            i++;
        }
        o++;
    }
    memcpy(j->dst + o * rs, j->src + i * rs, (j->ahi - i) * rs);
    o += j->ahi - i;
    memcpy(j->dst + o * rs, j->src + k * rs, (j->bhi - k) * rs);
    return NULL;
}

/* Keys only, on up to `threads` host threads (rounded down to a power of
 * two, at most 256).  The result is the same unique sorted permutation as
 * oracle_sort_keys. */
int oracle_sort_keys_parallel(int dtype, void *keys, size_t n, int threads)
{
    rec_t r;
    if (setup(&r, dtype, 0) != 0 || threads < 1)
        return -1;
    if (n == 0)
        return 0;
    if (keys == NULL)
        return -1;
    int t = 1;
    while (t * 2 <= threads && t < 256)
        t *= 2;
    unsigned char *a = (unsigned char *)keys; /* keys-only records are the keys */
    unsigned char *tmp = (unsigned char *)malloc(n * r.rs);
    size_t *b = (size_t *)malloc((size_t)(t + 1) * sizeof(size_t));
    pthread_t *th = (pthread_t *)malloc((size_t)t * sizeof(pthread_t));
    sort_part *sp = (sort_part *)malloc((size_t)t * sizeof(sort_part));
    merge_part *mp = (merge_part *)malloc((size_t)t * sizeof(merge_part));
    if (!tmp || !b || !th || !sp || !mp) {
        free(tmp); free(b); free(th); free(sp); free(mp);
        return -1;
    }
    for (int i = 0; i <= t; i++)
        b[i] = n / (size_t)t * (size_t)i + (n % (size_t)t) * (size_t)i / (size_t)t;
    for (int i = 0; i < t; i++) {
        sp[i] = (sort_part){&r, a, tmp, b[i], b[i + 1]};
        pthread_create(&th[i], NULL, sort_part_run, &sp[i]);
    }
    for (int i = 0; i < t; i++)
        pthread_join(th[i], NULL);
    unsigned char *src = a, *dst = tmp;
    for (int runs = t; runs > 1; runs /= 2) {
        int per = t / (runs / 2); /* threads per merge */
        for (int g = 0; g < runs / 2; g++) {
            size_t alo = b[2 * g], mid = b[2 * g + 1], bhi = b[2 * g + 2], len = bhi - alo;
            for (int q = 0; q < per; q++) {
                size_t d0 = len * (size_t)q / (size_t)per, d1 = len * (size_t)(q + 1) / (size_t)per;
                size_t i0 = co_rank(&r, src, alo, mid, mid, bhi, d0);
                size_t i1 = co_rank(&r, src, alo, mid, mid, bhi, d1);
                mp[g * per + q] = (merge_part){&r, src, dst, alo + i0, alo + i1,
                                               mid + (d0 - i0), mid + (d1 - i1), alo + d0};
            }
        }
        for (int i = 0; i < t; i++)
            pthread_create(&th[i], NULL, merge_part_run, &mp[i]);
        for (int i = 0; i < t; i++)
            pthread_join(th[i], NULL);
        for (int g = 0; g <= runs / 2; g++)
            b[g] = b[2 * g];
        unsigned char *x = src;
        src = dst;
        dst = x;
    }
    if (src != a)
        memcpy(a, src, n * r.rs);
    free(tmp); free(b); free(th); free(sp); free(mp);
    return 0;
}

/* ------------------------------------------------------ insertion sort */

/* Each element moves left past neighbours that are strictly greater, so
 * equal keys keep their order.  payload may be NULL. */
int oracle_insertion_sort(int dtype, void *keys, uint32_t *payload, size_t n)
{
    rec_t r;
    if (setup(&r, dtype, payload != NULL) != 0)
        return -1;
    if (n == 0)
        return 0;
    if (keys == NULL)
        return -1;
    unsigned char *a = pack(&r, keys, payload, n);
    unsigned char *hold = (unsigned char *)malloc(r.rs);
    if (!a || !hold) {
        free(a);
        free(hold);
        return -1;
    }
    for (size_t i = 1; i < n; i++) {
        memcpy(hold, a + i * r.rs, r.rs);
        size_t j = i;
        while (j > 0 && r.less(hold, a + (j - 1) * r.rs)) {
            memcpy(a + j * r.rs, a + (j - 1) * r.rs, r.rs);
            j--;
        }
        memcpy(a + j * r.rs, hold, r.rs);
    }
    unpack(&r, a, keys, payload, n);
    free(a);
    free(hold);
    return 0;
}

/* ------------------------------------------------- brute-force definition */

/* The output position p receives the least remaining element, where
 * "least" is the smallest key and, among equal keys, the smallest original
 * index.  O(n^2); for tiny inputs only. */
int oracle_brute_sort(int dtype, void *keys, uint32_t *payload, size_t n)
{
    rec_t r;
    if (setup(&r, dtype, payload != NULL) != 0)
        return -1;
    if (n == 0)
        return 0;
    unsigned char *a = pack(&r, keys, payload, n);
    unsigned char *out = (unsigned char *)malloc(n * r.rs);
    unsigned char *used = (unsigned char *)calloc(n, 1);
    if (!a || !out || !used) {
        free(a);
        free(out);
        free(used);
        return -1;
    }
    for (size_t p = 0; p < n; p++) {
        size_t best = n;
        for (size_t i = 0; i < n; i++) {
            if (used[i])
                continue;
            /* strictly-less keeps the earliest index among equal keys */
            if (best == n || r.less(a + i * r.rs, a + best * r.rs))
                best = i;
        }
        used[best] = 1;
        memcpy(out + p * r.rs, a + best * r.rs, r.rs);
    }
    unpack(&r, out, keys, payload, n);
    free(a);
    free(out);
    free(used);
    return 0;
}

/* ------------------------------------------------ presortedness measures */

/* Run(A) of Sec. 2: the number of descents a_i > a_{i+1}, plus one.  An
 * empty array has no runs (reading: the +1 counts the first run, and there
 * is none). */
/* ------------------------------------------------- lists (heavy items) */

/* Sec. 2 lists its first classes with items that are lists of integers of
 * 64, 256 or 1024 bytes.  The order taken for them: word by word from the
 * first, each word a signed int32; the first unequal word decides (equal
 * lists are equal).  The comparator needs the list length, which this
 * single-threaded test oracle keeps in a file-scope variable for the
 * duration of one call. */
static size_t g_list_words;

static int less_list(const unsigned char *a, const unsigned char *b)
{
    for (size_t w = 0; w < g_list_words; w++) {
        int32_t x, y;
        memcpy(&x, a + 4 * w, 4);
        memcpy(&y, b + 4 * w, 4);
        if (x != y)
            return x < y;
    }
    return 0;
}

int oracle_sort_lists(int32_t *lists, size_t n, size_t words)
{
    if (words == 0)
        return -1;
    if (n == 0)
        return 0;
    if (lists == NULL)
        return -1;
    rec_t r;
    r.ks = 4 * words;
    r.rs = 4 * words;
    r.with_payload = 0;
    r.less = less_list;
    g_list_words = words;
    unsigned char *tmp = (unsigned char *)malloc(n * r.rs);
    if (!tmp)
        return -1;
    msort(&r, (unsigned char *)lists, tmp, 0, n);
    free(tmp);
    return 0;
}

int64_t oracle_run(int dtype, const void *keys, size_t n)
{
    less_fn less = less_for(dtype);
    size_t ks = (size_t)key_size(dtype);
    if (!less)
        return -1;
    if (n == 0)
        return 0;
    const unsigned char *a = (const unsigned char *)keys;
    int64_t d = 0;
    for (size_t i = 0; i + 1 < n; i++)
        if (less(a + (i + 1) * ks, a + i * ks))
            d++;
    return d + 1;
}

/* Number of ascents a_i < a_{i+1}: Run of the mirrored order, minus one. */
int64_t oracle_ascents(int dtype, const void *keys, size_t n)
{
    less_fn less = less_for(dtype);
    size_t ks = (size_t)key_size(dtype);
    if (!less)
        return -1;
    const unsigned char *a = (const unsigned char *)keys;
    int64_t u = 0;
    for (size_t i = 0; i + 1 < n; i++)
        if (less(a + i * ks, a + (i + 1) * ks))
            u++;
    return u;
}

/* Inv(A) of Sec. 2: pairs i < j with a_i > a_j.  O(n^2), by definition. */
int64_t oracle_inv(int dtype, const void *keys, size_t n)
{
    less_fn less = less_for(dtype);
    size_t ks = (size_t)key_size(dtype);
    if (!less)
        return -1;
    const unsigned char *a = (const unsigned char *)keys;
    int64_t c = 0;
    for (size_t i = 0; i < n; i++)
        for (size_t j = i + 1; j < n; j++)
            if (less(a + j * ks, a + i * ks))
                c++;
    return c;
}

/* Mono(A) of Sec. 2: the least k such that A splits into k contiguous pieces
 * each sorted or reversely sorted (nondecreasing or nonincreasing).  Any
 * contiguous part of a monotone piece is monotone, so cutting each piece as
 * late as possible is optimal: scan left to right and start a new piece
 * exactly when the next element would break monotonicity.  A piece whose
 * elements are all equal is still undecided. */
int64_t oracle_mono(int dtype, const void *keys, size_t n)
{
    less_fn less = less_for(dtype);
    size_t ks = (size_t)key_size(dtype);
    if (!less)
        return -1;
    if (n == 0)
        return 0;
    const unsigned char *a = (const unsigned char *)keys;
    int64_t pieces = 1;
    int dir = 0; /* 0 undecided, +1 nondecreasing, -1 nonincreasing */
    for (size_t i = 1; i < n; i++) {
        const unsigned char *p = a + (i - 1) * ks, *q = a + i * ks;
        int step = less(p, q) ? 1 : (less(q, p) ? -1 : 0);
        if (step == 0)
            continue;
        if (dir == 0)
            dir = step;
        else if (step != dir) {
            pieces++;   /* element i opens a new piece */
            dir = 0;
        }
    }
    return pieces;
}
