/*
 * oracle.c -- CPU oracle for sort-based duplicate removal, grouping and
 * aggregation (Do, Graefe, Naughton, "Efficient sorting, duplicate removal,
 * grouping, and aggregation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke entry point and the
 * benchmark's CPU-baseline leg do.  It shares no code with the GPU path.
 *
 * What it computes is the plain definition of grouped aggregation: for every
 * distinct key k of the input multiset, one output row
 *     (k, |R_k|, sum of v_i64 over R_k mod 2^64, exact sum of v_f64 over R_k
 *      rounded once to nearest-even, min v_i64, max v_i64)
 * in ascending key order, where R_k is the set of input rows whose key is k.
 *
 * How it computes it is the traditional path the paper uses as its baseline
 * (Section 1, Figure 2, the "sort, then aggregate in-stream" plan; Section 2.1
 * on in-stream grouping of sorted input): sort all input rows on the grouping
 * key, then make one pass in which every row either continues the group of its
 * predecessor or opens a new group.  No blocking, fusion or reordering beyond
 * that.
 *
 * Readings of points the paper leaves open (listed in the design notes):
 *   - keys compare as unsigned 64-bit integers, output ascending;
 *   - the int64 sum wraps modulo 2^64 (two's complement);
 *   - the fp64 sum is the exact real sum rounded once to nearest-even;
 *     non-finite inputs follow IEEE addition (any NaN gives NaN,
 *     +Inf plus -Inf gives NaN);
 *   - min and max apply to the int64 value column;
 *   - an empty input yields zero groups.
 *
 * Pair keys (grouping on two int32 columns A, B): the output is ordered
 * lexicographically on (A, B) with both compared as signed 32-bit integers.
 */
#define _POSIX_C_SOURCE 200809L
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>
#include <unistd.h>

/* ------------------------------------------------------------------------ */
/* Exact fp64 summation: a long fixed-point accumulator (Kulisch's exact     */
/* dot-product accumulator; see also Neal 2015, "Fast exact summation using  */
/* small and large superaccumulators").  Every finite double is an integer   */
/* multiple of 2^-1074, so a wide enough fixed-point integer holds any sum    */
/* of them exactly; the sum is rounded to double once, at the end.           */
/* ------------------------------------------------------------------------ */

/* Limb i holds bits [32*i, 32*i+32) of the fixed-point integer whose unit is
 * 2^-EXACT_BIAS.  68 limbs cover 2^-1100 .. 2^1076, enough for 2^40 sums of
 * the largest finite double.  Limbs are signed and may run outside [0,2^32)
 * between normalisations. */
#define EXACT_LIMBS 68
#define EXACT_BIAS 1100

typedef struct {
    int64_t limb[EXACT_LIMBS];
    uint64_t adds_since_norm;
    int has_special;   /* a non-finite value was added */
    double special;    /* IEEE sum of the non-finite values */
} exact_acc;

static void exact_init(exact_acc* a) {
    memset(a, 0, sizeof(*a));
}

/* Propagate carries so that limbs 0..n-2 lie in [0, 2^32); the top limb keeps
 * the sign of the whole number. */
static void exact_normalise(exact_acc* a) {
    for (int i = 0; i < EXACT_LIMBS - 1; ++i) {
        int64_t c = a->limb[i] >> 32; /* floor division by 2^32 */
        a->limb[i] -= c * ((int64_t)1 << 32);
        a->limb[i + 1] += c;
    }
    a->adds_since_norm = 0;
}

static void exact_add(exact_acc* a, double x) {
    if (!isfinite(x)) {
        a->special = a->has_special ? a->special + x : x;
        a->has_special = 1;
        return;
    }
    if (x == 0.0) return;
    int e;
    double fr = frexp(x, &e);           /* x = fr * 2^e, 0.5 <= |fr| < 1 */
    /* m = integer mantissa, x = m * 2^(e-53); m exact in 53 bits */
    double mm = ldexp(fabs(fr), 53);
    uint64_t m = (uint64_t)mm;
    int p = e - 53 + EXACT_BIAS;        /* bit position of m's unit */
    if (p < 0) {                        /* subnormal: m has trailing zeros */
        m >>= -p;
        p = 0;
    }
    int q = p / 32, r = p % 32;
    /* m << r spans at most 53 + 31 = 84 bits: three 32-bit pieces */
    unsigned __int128 w = (unsigned __int128)m << r;
    uint64_t lo = (uint64_t)(w & 0xffffffffu);
    uint64_t mid = (uint64_t)((w >> 32) & 0xffffffffu);
    uint64_t hi = (uint64_t)((w >> 64) & 0xffffffffu);
    int64_t s = (x < 0) ? -1 : 1;
    a->limb[q] += s * (int64_t)lo;
    if (q + 1 < EXACT_LIMBS) a->limb[q + 1] += s * (int64_t)mid;
    if (q + 2 < EXACT_LIMBS) a->limb[q + 2] += s * (int64_t)hi;
    if (++a->adds_since_norm >= ((uint64_t)1 << 30)) exact_normalise(a);
}

/* bit k of a non-negative normalised magnitude */
static int mag_bit(const uint64_t* mag, int k) {
    return (int)((mag[k / 32] >> (k % 32)) & 1u);
}

/* Round the exact sum to the nearest double, ties to even. */
static double exact_round(exact_acc* a) {
    if (a->has_special) return a->special;
    exact_normalise(a);
    uint64_t mag[EXACT_LIMBS];
    int neg = a->limb[EXACT_LIMBS - 1] < 0;
    if (neg) {
        /* two's complement negation over 32-bit digits */
        uint64_t carry = 1;
        for (int i = 0; i < EXACT_LIMBS; ++i) {
            uint64_t d = (~(uint64_t)a->limb[i]) & 0xffffffffull;
            d += carry;
            carry = d >> 32;
            mag[i] = d & 0xffffffffull;
        }
    } else {
        for (int i = 0; i < EXACT_LIMBS; ++i) mag[i] = (uint64_t)a->limb[i] & 0xffffffffull;
    }
    int top = -1;
    for (int i = EXACT_LIMBS - 1; i >= 0; --i)
        if (mag[i]) { top = i; break; }
    if (top < 0) return 0.0;
    int msb = top * 32 + 31;
    while (!mag_bit(mag, msb)) --msb;
    /* lowest representable bit: 52 below the msb for normal results, fixed
     * at 2^-1074 (position 1100-1074 = 26) for subnormal results */
    int lsb = msb - 52;
    if (lsb < EXACT_BIAS - 1074) lsb = EXACT_BIAS - 1074;
    uint64_t mant = 0;
    for (int k = msb; k >= lsb; --k) mant = (mant << 1) | (uint64_t)mag_bit(mag, k);
    int round_bit = (lsb >= 1) ? mag_bit(mag, lsb - 1) : 0;
    int sticky = 0;
    for (int k = lsb - 2; k >= 0 && !sticky; --k) sticky = mag_bit(mag, k);
    if (round_bit && (sticky || (mant & 1u))) mant += 1;
    double r = ldexp((double)mant, lsb - EXACT_BIAS);
    return neg ? -r : r;
}

/* Exposed for the tests: exact sum of an array, rounded once. */
double oracle_exact_sum(const double* x, uint64_t n) {
    exact_acc* a = (exact_acc*)malloc(sizeof(exact_acc));
    exact_init(a);
    for (uint64_t i = 0; i < n; ++i) exact_add(a, x[i]);
    double r = exact_round(a);
    free(a);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Stable sort of row indices: a plain top-down merge sort.                  */
/* ------------------------------------------------------------------------ */

typedef int (*row_less_fn)(const void* ctx, uint64_t a, uint64_t b);

static void merge_sort_rec(uint64_t* idx, uint64_t* tmp, uint64_t lo, uint64_t hi,
                           row_less_fn less, const void* ctx) {
    if (hi - lo < 2) return;
    uint64_t mid = lo + (hi - lo) / 2;
    merge_sort_rec(idx, tmp, lo, mid, less, ctx);
    merge_sort_rec(idx, tmp, mid, hi, less, ctx);
    uint64_t i = lo, j = mid, k = lo;
    while (i < mid && j < hi) {
        /* take from the right half only if strictly smaller: stability */
        if (less(ctx, idx[j], idx[i])) tmp[k++] = idx[j++];
        else tmp[k++] = idx[i++];
    }
    while (i < mid) tmp[k++] = idx[i++];
    while (j < hi) tmp[k++] = idx[j++];
    memcpy(idx + lo, tmp + lo, (hi - lo) * sizeof(uint64_t));
}

static uint64_t* sorted_row_order(uint64_t n, row_less_fn less, const void* ctx) {
    uint64_t* idx = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t* tmp = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) idx[i] = i;
    merge_sort_rec(idx, tmp, 0, n, less, ctx);
    free(tmp);
    return idx;
}

static int key_less(const void* ctx, uint64_t a, uint64_t b) {
    const uint64_t* k = (const uint64_t*)ctx;
    return k[a] < k[b];
}

typedef struct { const int32_t* a; const int32_t* b; } pair_ctx;

static int pair_less(const void* ctx, uint64_t x, uint64_t y) {
    const pair_ctx* p = (const pair_ctx*)ctx;
    if (p->a[x] != p->a[y]) return p->a[x] < p->a[y];
    return p->b[x] < p->b[y];
}

/* ------------------------------------------------------------------------ */
/* In-stream aggregation over the sorted row order.                          */
/* ------------------------------------------------------------------------ */

/* One open group of the in-stream scan. */
typedef struct {
    uint64_t count;
    uint64_t sum;   /* int64 sum carried as uint64 so that it wraps */
    int64_t mn, mx;
    exact_acc* fsum;
} group_state;

static void group_open(group_state* g) {
    g->count = 0;
    g->sum = 0;
    g->mn = INT64_MAX;
    g->mx = INT64_MIN;
    exact_init(g->fsum);
}

static void group_add(group_state* g, const int64_t* v, const double* f, uint64_t r) {
    g->count += 1;
    if (v) {
        g->sum += (uint64_t)v[r];
        if (v[r] < g->mn) g->mn = v[r];
        if (v[r] > g->mx) g->mx = v[r];
    }
    if (f) exact_add(g->fsum, f[r]);
}

static void group_emit(const group_state* g, uint64_t o, uint64_t* out_count,
                       int64_t* out_sum, double* out_fsum, int64_t* out_min,
                       int64_t* out_max) {
    if (out_count) out_count[o] = g->count;
    if (out_sum) out_sum[o] = (int64_t)g->sum;
    if (out_fsum) out_fsum[o] = exact_round(g->fsum);
    if (out_min) out_min[o] = g->mn;
    if (out_max) out_max[o] = g->mx;
}

/*
 * In-stream aggregation of rows taken in the order idx[0..n) (sorted on the
 * key): every row either continues the group of its predecessor or opens a
 * new one.  Returns the number of groups written.
 */
static uint64_t group_scan(const uint64_t* idx, uint64_t n, const uint64_t* keys,
                           const int64_t* v_i64, const double* v_f64, uint64_t* out_keys,
                           uint64_t* out_count, int64_t* out_sum, double* out_fsum,
                           int64_t* out_min, int64_t* out_max) {
    if (n == 0) return 0;
    group_state g;
    g.fsum = (exact_acc*)malloc(sizeof(exact_acc));
    uint64_t groups = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t r = idx[i];
        if (i == 0 || keys[r] != keys[idx[i - 1]]) {
            if (i > 0) {
                group_emit(&g, groups, out_count, out_sum, v_f64 ? out_fsum : NULL,
                           out_min, out_max);
                groups++;
            }
            group_open(&g);
            if (out_keys) out_keys[groups] = keys[r];
        }
        group_add(&g, v_i64, v_f64, r);
    }
    group_emit(&g, groups, out_count, out_sum, v_f64 ? out_fsum : NULL, out_min, out_max);
    groups++;
    free(g.fsum);
    return groups;
}

/*
 * Group n rows on a uint64 key.  v_i64 and v_f64 may be NULL (then the
 * aggregates over them are not produced).  Output pointers may be NULL to skip
 * a column; every non-NULL output array must hold at least the number of
 * distinct keys (n is always enough).  Returns the number of groups.
 */
uint64_t oracle_group_by(uint64_t n, const uint64_t* keys, const int64_t* v_i64,
                         const double* v_f64, uint64_t* out_keys, uint64_t* out_count,
                         int64_t* out_sum, double* out_fsum, int64_t* out_min,
                         int64_t* out_max) {
    if (n == 0) return 0;
    uint64_t* idx = sorted_row_order(n, key_less, keys);
    uint64_t groups = group_scan(idx, n, keys, v_i64, v_f64, out_keys, out_count, out_sum,
                                 out_fsum, out_min, out_max);
    free(idx);
    return groups;
}

/* ------------------------------------------------------------------------ */
/* The same plan on several host threads: the key space is cut into ranges  */
/* at splitters drawn from a sample of the keys, the rows of each range are   */
/* collected in input order, and each thread sorts and scans one range.     */
/* Every group lies in one range and the ranges are concatenated in key      */
/* order, so the result is the single-threaded one, bit for bit.             */
/* ------------------------------------------------------------------------ */

typedef struct {
    const uint64_t* keys;
    const int64_t* v;
    const double* f;
    uint64_t* rows;   /* the range's row ids, in input order; sorted in place */
    uint64_t n;
    uint64_t* ok;
    uint64_t* oc;
    int64_t* os;
    double* of;
    int64_t* omn;
    int64_t* omx;
    uint64_t groups;
} range_job;

static void* range_worker(void* arg) {
    range_job* j = (range_job*)arg;
    if (j->n) {
        uint64_t* tmp = (uint64_t*)malloc(j->n * sizeof(uint64_t));
        merge_sort_rec(j->rows, tmp, 0, j->n, key_less, j->keys);
        free(tmp);
    }
    j->groups = group_scan(j->rows, j->n, j->keys, j->v, j->f, j->ok, j->oc, j->os, j->of,
                           j->omn, j->omx);
    return NULL;
}

static int u64_cmp(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

int oracle_nproc(void) {
    long p = sysconf(_SC_NPROCESSORS_ONLN);
    return p > 0 ? (int)p : 1;
}

#define MAX_RANGES 256

uint64_t oracle_group_by_parallel(uint64_t n, const uint64_t* keys, const int64_t* v_i64,
                                  const double* v_f64, uint64_t* out_keys, uint64_t* out_count,
                                  int64_t* out_sum, double* out_fsum, int64_t* out_min,
                                  int64_t* out_max, int threads) {
    if (n == 0) return 0;
    if (threads <= 0) threads = oracle_nproc();
    if (threads > MAX_RANGES) threads = MAX_RANGES;
    /* splitters: equally spaced order statistics of a strided key sample,
     * duplicates dropped; range r holds keys in [spl[r-1], spl[r]) */
    uint64_t ns = (uint64_t)threads * 64;
    if (ns > n) ns = n;
    uint64_t* sample = (uint64_t*)malloc(ns * sizeof(uint64_t));
    for (uint64_t i = 0; i < ns; ++i) sample[i] = keys[i * (n / ns)];
    qsort(sample, ns, sizeof(uint64_t), u64_cmp);
    uint64_t spl[MAX_RANGES];
    int nspl = 0;
    for (int r = 1; r < threads; ++r) {
        uint64_t x = sample[(uint64_t)r * ns / (uint64_t)threads];
        if (nspl == 0 || x > spl[nspl - 1]) spl[nspl++] = x;
    }
    free(sample);
    const int nr = nspl + 1;
    /* range of every row (count of splitters <= key), then a stable scatter */
    uint8_t* rid = (uint8_t*)malloc(n);
    uint64_t cnt[MAX_RANGES + 1];
    memset(cnt, 0, sizeof(cnt));
    for (uint64_t i = 0; i < n; ++i) {
        int lo = 0, hi = nspl;
        while (lo < hi) {
            int mid = (lo + hi) / 2;
            if (spl[mid] <= keys[i]) lo = mid + 1;
            else hi = mid;
        }
        rid[i] = (uint8_t)lo;
        cnt[lo]++;
    }
    uint64_t start[MAX_RANGES + 1], fill[MAX_RANGES];
    start[0] = 0;
    for (int r = 0; r < nr; ++r) start[r + 1] = start[r] + cnt[r];
    memcpy(fill, start, sizeof(uint64_t) * (size_t)nr);
    uint64_t* rows = (uint64_t*)malloc(n * sizeof(uint64_t));
    for (uint64_t i = 0; i < n; ++i) rows[fill[rid[i]]++] = i;
    free(rid);
    /* each range writes its groups at its first row's position (a range has
     * no more groups than rows); the ranges are then packed in order */
    range_job job[MAX_RANGES];
    pthread_t tid[MAX_RANGES];
    int started[MAX_RANGES];
    for (int r = 0; r < nr; ++r) {
        const uint64_t o = start[r];
        range_job* j = &job[r];
        j->keys = keys;
        j->v = v_i64;
        j->f = v_f64;
        j->rows = rows + o;
        j->n = cnt[r];
        j->ok = out_keys ? out_keys + o : NULL;
        j->oc = out_count ? out_count + o : NULL;
        j->os = out_sum ? out_sum + o : NULL;
        j->of = out_fsum ? out_fsum + o : NULL;
        j->omn = out_min ? out_min + o : NULL;
        j->omx = out_max ? out_max + o : NULL;
        j->groups = 0;
        started[r] = pthread_create(&tid[r], NULL, range_worker, j) == 0;
        if (!started[r]) range_worker(j);
    }
    for (int r = 0; r < nr; ++r)
        if (started[r]) pthread_join(tid[r], NULL);
    uint64_t groups = 0;
    for (int r = 0; r < nr; ++r) {
        const uint64_t o = start[r], g = job[r].groups;
        if (groups != o) {
            if (out_keys) memmove(out_keys + groups, out_keys + o, g * sizeof(uint64_t));
            if (out_count) memmove(out_count + groups, out_count + o, g * sizeof(uint64_t));
            if (out_sum) memmove(out_sum + groups, out_sum + o, g * sizeof(int64_t));
            if (out_fsum && v_f64) memmove(out_fsum + groups, out_fsum + o, g * sizeof(double));
            if (out_min) memmove(out_min + groups, out_min + o, g * sizeof(int64_t));
            if (out_max) memmove(out_max + groups, out_max + o, g * sizeof(int64_t));
        }
        groups += g;
    }
    free(rows);
    return groups;
}

/*
 * Group n rows on the pair (a, b) of signed int32 columns, aggregating the
 * int64 column v.  Output ordered by (a, b), both signed.
 */
uint64_t oracle_group_by_pairs(uint64_t n, const int32_t* a, const int32_t* b,
                               const int64_t* v, int32_t* out_a, int32_t* out_b,
                               uint64_t* out_count, int64_t* out_sum,
                               int64_t* out_min, int64_t* out_max) {
    if (n == 0) return 0;
    pair_ctx ctx = {a, b};
    uint64_t* idx = sorted_row_order(n, pair_less, &ctx);
    group_state g;
    g.fsum = (exact_acc*)malloc(sizeof(exact_acc));
    uint64_t groups = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t r = idx[i];
        uint64_t p = (i > 0) ? idx[i - 1] : 0;
        if (i == 0 || a[r] != a[p] || b[r] != b[p]) {
            if (i > 0) {
                group_emit(&g, groups, out_count, out_sum, NULL, out_min, out_max);
                groups++;
            }
            group_open(&g);
            if (out_a) out_a[groups] = a[r];
            if (out_b) out_b[groups] = b[r];
        }
        group_add(&g, v, NULL, r);
    }
    group_emit(&g, groups, out_count, out_sum, NULL, out_min, out_max);
    groups++;
    free(g.fsum);
    free(idx);
    return groups;
}

/*
 * count(*) and count(distinct x) per group g in one sort (the paper's
 * Section 2.2 use of a single sort on (group, user) for duplicate removal
 * followed by grouping): rows are sorted on (g, x); a group's row count is its
 * run length, its distinct count the number of x-changes within the run.
 */
static int u64pair_less(const void* ctx, uint64_t x, uint64_t y) {
    const uint64_t* const* p = (const uint64_t* const*)ctx;
    if (p[0][x] != p[0][y]) return p[0][x] < p[0][y];
    return p[1][x] < p[1][y];
}

uint64_t oracle_count_distinct(uint64_t n, const uint64_t* g, const uint64_t* x,
                               uint64_t* out_g, uint64_t* out_count,
                               uint64_t* out_distinct) {
    if (n == 0) return 0;
    const uint64_t* ctx[2] = {g, x};
    uint64_t* idx = sorted_row_order(n, u64pair_less, ctx);
    uint64_t groups = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t r = idx[i];
        uint64_t p = (i > 0) ? idx[i - 1] : 0;
        if (i == 0 || g[r] != g[p]) {
            out_g[groups] = g[r];
            out_count[groups] = 0;
            out_distinct[groups] = 0;
            groups++;
        }
        out_count[groups - 1] += 1;
        if (i == 0 || g[r] != g[p] || x[r] != x[p]) out_distinct[groups - 1] += 1;
    }
    free(idx);
    return groups;
}
