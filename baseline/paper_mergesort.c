/*
 * paper_mergesort.c -- the paper's own adaptive mergesort as a CPU program
 * (a comparison point for the GPU library; it shares no code with it or with
 * the test oracle).
 *
 * Zhang, Meng, Liang, "Sort Race" (arXiv 1609.04471), Sec. 3 selects a
 * natural mergesort built from these techniques (the variant the paper calls
 * mer6, whose code its Appendix A prints):
 *   (a) a descending stretch found while scanning is reversed in place to
 *       make a longer run; for stability, each group of equal elements inside
 *       it is reversed twice, so equal elements keep their input order
 *       (every group, including one that ends the stretch);
 *   (b) a run shorter than the minimum run length is extended by insertion
 *       sort (linear insertion: an element moves left past strictly greater
 *       ones);
 *   (e2) runs are kept on a "half-down list": each run is at most half as
 *       long as the run before it; a new run longer than half its
 *       predecessor is merged with it, repeatedly; at the end the list is
 *       merged from the last run to the first;
 *   (f) a merge of neighbouring runs A and B leaves out the elements of A
 *       not greater than B's first element and the elements of B greater
 *       than A's last element, and copies only the shorter remaining part to
 *       temporary memory;
 *   (g) a merge switches to galloping once one side has won a number of
 *       times in a row (three in the Sec. 3 example): a binary search finds
 *       how many further elements of the winning side precede the other
 *       side's current element, and that block moves at once.
 * The minimum run length is not given by the paper; it is a parameter here.
 *
 * Every comparison goes through one comparison function and is counted
 * (Sec. 5 counts comparisons per element).  Elements are records of `es`
 * bytes whose key comes first: int32, uint64 or float32 (IEEE totalOrder on
 * the bits), optionally followed by a payload the comparison ignores.
 * Build: gcc -O3 -shared -fPIC.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int (*pm_cmp)(const void *, const void *);

static int cmp_i32(const void *p, const void *q)
{
    int32_t x, y;
    memcpy(&x, p, 4);
    memcpy(&y, q, 4);
    return (x > y) - (x < y);
}

static int cmp_u64(const void *p, const void *q)
{
    uint64_t x, y;
    memcpy(&x, p, 8);
    memcpy(&y, q, 8);
    return (x > y) - (x < y);
}

/* totalOrder on binary32: map the bits to an unsigned rank */
static uint32_t f32_rank(uint32_t b) { return (b >> 31) ? ~b : (b | 0x80000000u); }

static int cmp_f32(const void *p, const void *q)
{
    uint32_t x, y;
    memcpy(&x, p, 4);
    memcpy(&y, q, 4);
    x = f32_rank(x);
    y = f32_rank(y);
    return (x > y) - (x < y);
}

typedef struct {
    unsigned char *a;   /* the array */
    unsigned char *t;   /* temporary memory (n records) */
    size_t es;
    pm_cmp cmp;
    uint64_t ncmp;
    size_t gallop_after;
} ctx;

#define AT(c, i) ((c)->a + (size_t)(i) * (c)->es)

static int cmp_p(ctx *c, const void *p, const void *q)
{
    c->ncmp++;
    return c->cmp(p, q);
}

static void swap_rec(ctx *c, size_t i, size_t j)
{
    unsigned char tmp[64];
    memcpy(tmp, AT(c, i), c->es);
    memcpy(AT(c, i), AT(c, j), c->es);
    memcpy(AT(c, j), tmp, c->es);
}

/* reverse a[lo .. hi] (inclusive bounds) */
static void reverse_range(ctx *c, size_t lo, size_t hi)
{
    while (lo < hi)
        swap_rec(c, lo++, hi--);
}

/* Elements of the sorted block p[0, len) that are smaller than key
 * (left = 1) or not greater than key (left = 0): a doubling search probes
 * p[0], p[1], p[3], p[7], ... until one fails, then a binary search finishes
 * between the last success and that failure. */
static size_t gallop_fwd(ctx *c, const unsigned char *p, size_t len, const void *key, int left)
{
    size_t lo = 0, hi = len, off = 1;   /* p[0, lo) qualify; p[hi] does not (hi < len) */
    while (off <= len) {
        int r = cmp_p(c, p + (off - 1) * c->es, key);
        if (left ? r < 0 : r <= 0) {
            lo = off;
            off *= 2;
        } else {
            hi = off - 1;
            break;
        }
    }
    while (lo < hi) {
        size_t mid = lo + (hi - lo) / 2;
        int r = cmp_p(c, p + mid * c->es, key);
        if (left ? r < 0 : r <= 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* Elements at the end of the sorted block p[0, len) that are greater than
 * key (left = 0) or not smaller than key (left = 1): the same search from the
 * block's end. */
static size_t gallop_bwd(ctx *c, const unsigned char *p, size_t len, const void *key, int left)
{
    size_t lo = 0, hi = len, off = 1;   /* counted from the end */
    while (off <= len) {
        int r = cmp_p(c, p + (len - off) * c->es, key);
        if (left ? r >= 0 : r > 0) {
            lo = off;
            off *= 2;
        } else {
            hi = off - 1;
            break;
        }
    }
    while (lo < hi) {
        size_t mid = lo + (hi - lo) / 2;
        int r = cmp_p(c, p + (len - 1 - mid) * c->es, key);
        if (left ? r >= 0 : r > 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

/* Merge of the neighbouring sorted runs a[lo, mid) and a[mid, hi) with the
 * trims of (f) and the galloping of (g); equal elements keep A first. */
static void merge_runs(ctx *c, size_t lo, size_t mid, size_t hi)
{
    const size_t es = c->es;
    /* (f): A's elements not greater than B's first are already in place */
    lo += gallop_fwd(c, AT(c, lo), mid - lo, AT(c, mid), 0);
    if (lo == mid)
        return;
    /* (f): B's elements greater than A's last are already in place */
    hi -= gallop_bwd(c, AT(c, mid), hi - mid, AT(c, mid - 1), 0);
    if (hi == mid)
        return;
    size_t na = mid - lo, nb = hi - mid;
    const size_t G = c->gallop_after;
    if (na <= nb) {
        /* A to temporary memory, merge forward */
        memcpy(c->t, AT(c, lo), na * es);
        size_t i = 0, j = mid, o = lo, wa = 0, wb = 0;
        while (i < na && j < hi) {
            if (cmp_p(c, AT(c, j), c->t + i * es) < 0) {
                memmove(AT(c, o++), AT(c, j++), es);
                wb++;
                wa = 0;
            } else {
                memcpy(AT(c, o++), c->t + i * es, es);
                i++;
                wa++;
                wb = 0;
            }
            if (wb >= G && i < na && j < hi) {
                size_t k = gallop_fwd(c, AT(c, j), hi - j, c->t + i * es, 1);  /* B's smaller than A[i] */
                memmove(AT(c, o), AT(c, j), k * es);
                o += k;
                j += k;
                wb = 0;
            } else if (wa >= G && i < na && j < hi) {
                size_t k = gallop_fwd(c, c->t + i * es, na - i, AT(c, j), 0);   /* A's not greater than B[j] */
                memcpy(AT(c, o), c->t + i * es, k * es);
                o += k;
                i += k;
                wa = 0;
            }
        }
        memcpy(AT(c, o), c->t + i * es, (na - i) * es);   /* B's rest is in place */
    } else {
        /* B to temporary memory, merge backward */
        memcpy(c->t, AT(c, mid), nb * es);
        size_t i = mid, j = nb, o = hi, wa = 0, wb = 0;   /* i, j: one past the next candidates */
        while (i > lo && j > 0) {
            if (cmp_p(c, AT(c, i - 1), c->t + (j - 1) * es) > 0) {
                memmove(AT(c, --o), AT(c, --i), es);
                wa++;
                wb = 0;
            } else {
                memcpy(AT(c, --o), c->t + (--j) * es, es);
                wb++;
                wa = 0;
            }
            if (wa >= G && i > lo && j > 0) {
                size_t k = gallop_bwd(c, AT(c, lo), i - lo, c->t + (j - 1) * es, 0);  /* A's greater than B[j-1] */
                o -= k;
                i -= k;
                memmove(AT(c, o), AT(c, i), k * es);
                wa = 0;
            } else if (wb >= G && i > lo && j > 0) {
                size_t k = gallop_bwd(c, c->t, j, AT(c, i - 1), 1);   /* B's not smaller than A[i-1] */
                o -= k;
                j -= k;
                memcpy(AT(c, o), c->t + j * es, k * es);
                wb = 0;
            }
        }
        memcpy(AT(c, lo), c->t, j * es);   /* A's rest is in place */
    }
}

/* (b): a[lo, sorted_end) is sorted; insert a[sorted_end, end) one by one. */
static void insertion_extend(ctx *c, size_t lo, size_t sorted_end, size_t end)
{
    unsigned char hold[64];
    for (size_t i = sorted_end; i < end; i++) {
        memcpy(hold, AT(c, i), c->es);
        size_t j = i;
        while (j > lo && cmp_p(c, AT(c, j - 1), hold) > 0) {
            memcpy(AT(c, j), AT(c, j - 1), c->es);
            j--;
        }
        memcpy(AT(c, j), hold, c->es);
    }
}

/* (a): the run starting at s; returns its end.  A stretch that starts with a
 * descent extends while nonincreasing and is reversed stably. */
static size_t take_run(ctx *c, size_t s, size_t n)
{
    if (s + 1 >= n)
        return n;
    size_t e = s + 2;
    if (cmp_p(c, AT(c, s), AT(c, s + 1)) <= 0) {
        while (e < n && cmp_p(c, AT(c, e - 1), AT(c, e)) <= 0)
            e++;
        return e;
    }
    /* nonincreasing: pre-reverse each group of equal elements, then the whole;
     * a[s] > a[s+1], so the first group is a[s] alone */
    size_t g = s + 1;   /* start of the current equal group */
    while (e < n) {
        int r = cmp_p(c, AT(c, e - 1), AT(c, e));
        if (r < 0)
            break;
        if (r > 0) {
            if (e - 1 > g)
                reverse_range(c, g, e - 1);
            g = e;
        }
        e++;
    }
    if (e - 1 > g)
        reverse_range(c, g, e - 1);
    reverse_range(c, s, e - 1);
    return e;
}

/* Sorts n records of es bytes (es <= 64) in place; returns 0, or -1 on a bad
 * argument or failed allocation.  *ncmp receives the number of comparisons. */
int pm_sort(int dtype, void *keys, size_t n, size_t es, size_t minrun, size_t gallop_after, uint64_t *ncmp)
{
    ctx c;
    switch (dtype) {
    case 0: c.cmp = cmp_i32; if (es < 4) return -1; break;
    case 1: c.cmp = cmp_u64; if (es < 8) return -1; break;
    case 2: c.cmp = cmp_f32; if (es < 4) return -1; break;
    default: return -1;
    }
    if (es > 64 || gallop_after < 1 || (n > 0 && keys == NULL))
        return -1;
    c.a = (unsigned char *)keys;
    c.es = es;
    c.ncmp = 0;
    c.gallop_after = gallop_after;
    if (ncmp)
        *ncmp = 0;
    if (n < 2)
        return 0;
    c.t = (unsigned char *)malloc(n * es);
    size_t cap = 2, top = 0;    /* half-down list: run starts, newest last */
    size_t *run = (size_t *)malloc((cap + 1) * sizeof(size_t));
    if (!c.t || !run) {
        free(c.t);
        free(run);
        return -1;
    }
    size_t s = 0;
    while (s < n) {
        size_t e = take_run(&c, s, n);
        if (e - s < minrun && e < n) {
            size_t want = s + minrun < n ? s + minrun : n;
            insertion_extend(&c, s, e, want);
            e = want;
            /* the run goes on while the input keeps ascending */
            while (e < n && cmp_p(&c, AT(&c, e - 1), AT(&c, e)) <= 0)
                e++;
        }
        if (top + 2 > cap) {
            size_t *grown = (size_t *)realloc(run, (2 * cap + 1) * sizeof(size_t));
            if (!grown) {
                free(c.t);
                free(run);
                return -1;
            }
            run = grown;
            cap *= 2;
        }
        run[top++] = s;   /* runs: [run[i], run[i+1]), the last ends at e */
        run[top] = e;
        /* (e2): while the newest run is longer than half its predecessor, merge them */
        while (top >= 2 && run[top] - run[top - 1] > (run[top - 1] - run[top - 2]) / 2) {
            merge_runs(&c, run[top - 2], run[top - 1], run[top]);
            run[top - 1] = run[top];
            top--;
        }
        s = e;
    }
    /* merge the list from the last run to the first */
    while (top >= 2) {
        merge_runs(&c, run[top - 2], run[top - 1], run[top]);
        run[top - 1] = run[top];
        top--;
    }
    free(run);
    free(c.t);
    if (ncmp)
        *ncmp = c.ncmp;
    return 0;
}
