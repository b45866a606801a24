/*
 * oracle.c -- plain, slow, single-threaded CPU reference for the two integer
 * sorts compared in "Comparison of Bucket Sort and RADIX Sort"
 * (P. Horsmalahti, arXiv 1206.3511).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library product calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU path.
 *
 * What is computed (section 2 of the paper):
 *   - Sorting (section 2): the output is the permutation of the input that is
 *     in nondecreasing order.  With a payload the permutation is the stable
 *     one: equal keys keep their input order (section 2, definition of a
 *     stable sort).  For every input there is exactly one such output.
 *   - RADIX-SORT (Algorithm 4): for digit 1 (least significant) to d, stably
 *     sort the whole array on that digit.  The per-digit stable sort is
 *     COUNTING-SORT (Algorithm 3): zero the counts, count every digit value,
 *     turn counts into inclusive prefix sums, then place elements from the
 *     last one to the first, decrementing the count of the element's digit.
 *   - Keys that are not unsigned (signed integers, IEEE 754 floats): the same
 *     definition of sorting under the order those bit patterns denote (signed
 *     value; IEEE 754-2019 totalOrder), by a plain stable merge sort.
 *   - BUCKET-SORT (Algorithm 2): drop every element, in input order, into the
 *     bucket its value selects; sort every bucket with INSERTION-SORT
 *     (Algorithm 1, whose strict '>' keeps it stable); concatenate buckets.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *   - Digits are binary, r bits wide: digit_p(k) = (k >> p*r) & (2^r - 1).
 *     The number of passes is d = ceil(key_bits / r) unless the caller asks
 *     for the paper's "digits of the largest integer" reading (Algorithm 4's
 *     d), in which case d = ceil(bits(max) / r).
 *   - The bucket of key k is floor((k - min) * B / (max - min + 1)) computed
 *     exactly in 128-bit integers, with min and max taken from the input.
 *     This is the paper's n*A[i]/M (Algorithm 2) with the value range
 *     measured instead of assumed, and with B a parameter instead of n.
 *   - Buckets are contiguous runs of one output-sized array instead of linked
 *     lists; they are filled in input order, so their contents and order are
 *     those the paper's lists would hold.
 *   - A bucket of at most `cutoff` elements is sorted with Algorithm 1 as
 *     printed.  A larger one is sorted with a plain bottom-up stable merge
 *     sort, because insertion sort of a 10^5-element bucket is quadratic.
 *     Both are stable, so the result is the same.
 *
 * Keys are handled internally as uint64_t; 32-bit keys are widened on the
 * way in and narrowed on the way out.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum { ORACLE_OK = 0, ORACLE_EINVAL = 1, ORACLE_ENOMEM = 2 };

/* ---------------------------------------------------------------- helpers */

static uint64_t load_key(const void *keys, uint64_t i, int key_bytes)
{
    if (key_bytes == 4) return ((const uint32_t *)keys)[i];
    return ((const uint64_t *)keys)[i];
}

static void store_key(void *keys, uint64_t i, uint64_t v, int key_bytes)
{
    if (key_bytes == 4) ((uint32_t *)keys)[i] = (uint32_t)v;
    else ((uint64_t *)keys)[i] = v;
}

static uint64_t *widen(const void *keys, uint64_t n, int key_bytes)
{
    uint64_t *a = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    if (!a) return NULL;
    for (uint64_t i = 0; i < n; i++) a[i] = load_key(keys, i, key_bytes);
    return a;
}

static void narrow(const uint64_t *a, void *keys, uint64_t n, int key_bytes)
{
    for (uint64_t i = 0; i < n; i++) store_key(keys, i, a[i], key_bytes);
}

/* number of significant bits of x (0 for x == 0) */
static unsigned bit_length(uint64_t x)
{
    unsigned b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

/* ---------------------------------------------------- Algorithm 3 (digit) */

/*
 * COUNTING-SORT of A[0..n-1] into B[0..n-1] on the digit (a >> shift) & (k-1),
 * k = 2^r, carrying the optional payload VA -> VB.  The steps are those of
 * Algorithm 3: zero C, count, inclusive prefix, then place from the last
 * element to the first with a decrement before the store (0-based form of
 * "B[C[A[j]]] <- A[j]; C[A[j]] <- C[A[j]] - 1").  If `counts` is not NULL it
 * receives the k digit counts taken before the prefix step.
 */
static void counting_sort_digit(const uint64_t *A, uint64_t *B,
                                const uint32_t *VA, uint32_t *VB, uint64_t n,
                                unsigned shift, unsigned r, uint64_t *C,
                                uint64_t *counts)
{
    const uint64_t k = (uint64_t)1 << r;
    const uint64_t mask = k - 1;

    for (uint64_t i = 0; i < k; i++) C[i] = 0;
    for (uint64_t j = 0; j < n; j++) C[(A[j] >> shift) & mask] += 1;
    if (counts) memcpy(counts, C, k * sizeof(uint64_t));
    for (uint64_t i = 1; i < k; i++) C[i] += C[i - 1];
    for (uint64_t j = n; j-- > 0;) {
        uint64_t dg = (A[j] >> shift) & mask;
        C[dg] -= 1;
        B[C[dg]] = A[j];
        if (VA) VB[C[dg]] = VA[j];
    }
}

/* ------------------------------------------------------ Algorithm 4 (LSD) */

/*
 * RADIX-SORT: d stable counting-sort passes, least significant digit first.
 *   keys_in/keys_out : n keys of key_bytes (4 or 8) each; may be the same.
 *   vals_in/vals_out : optional uint32 payload (both NULL or both set).
 *   r                : digit width in bits, 1..16.
 *   d_from_max       : 0 -> d = ceil(8*key_bytes / r);
 *                      1 -> d = ceil(bits(max key) / r) (Algorithm 4's d).
 *   pass_counts      : optional, d * 2^r counts (pass-major).
 *   pass_keys        : optional, d * n keys (uint64) holding the array after
 *                      every pass.
 *   passes_out       : optional, receives d.
 */
int oracle_radix_lsd(const void *keys_in, void *keys_out, int key_bytes,
                     const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                     int r, int d_from_max, uint64_t *pass_counts,
                     uint64_t *pass_keys, int *passes_out)
{
    if (key_bytes != 4 && key_bytes != 8) return ORACLE_EINVAL;
    if (r < 1 || r > 16) return ORACLE_EINVAL;
    if ((vals_in == NULL) != (vals_out == NULL)) return ORACLE_EINVAL;
    if (n > 0 && (!keys_in || !keys_out)) return ORACLE_EINVAL;

    const unsigned key_bits = 8u * (unsigned)key_bytes;
    uint64_t *A = widen(keys_in, n, key_bytes);
    uint64_t *B = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint32_t *VA = NULL, *VB = NULL;
    uint64_t *C = (uint64_t *)malloc(((uint64_t)1 << r) * sizeof(uint64_t));
    if (vals_in) {
        VA = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
        VB = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    }
    if (!A || !B || !C || (vals_in && (!VA || !VB))) {
        free(A); free(B); free(C); free(VA); free(VB);
        return ORACLE_ENOMEM;
    }
    if (vals_in) memcpy(VA, vals_in, n * sizeof(uint32_t));

    unsigned d;
    if (d_from_max) {
        uint64_t mx = 0;
        for (uint64_t i = 0; i < n; i++) if (A[i] > mx) mx = A[i];
        d = (bit_length(mx) + (unsigned)r - 1) / (unsigned)r;
    } else {
        d = (key_bits + (unsigned)r - 1) / (unsigned)r;
    }

    for (unsigned p = 0; p < d; p++) {
        counting_sort_digit(A, B, VA, VB, n, p * (unsigned)r, (unsigned)r, C,
                            pass_counts ? pass_counts + (uint64_t)p * ((uint64_t)1 << r) : NULL);
        uint64_t *t = A; A = B; B = t;
        uint32_t *tv = VA; VA = VB; VB = tv;
        if (pass_keys) memcpy(pass_keys + (uint64_t)p * n, A, n * sizeof(uint64_t));
    }

    narrow(A, keys_out, n, key_bytes);
    if (vals_out) memcpy(vals_out, VA, n * sizeof(uint32_t));
    if (passes_out) *passes_out = (int)d;
    free(A); free(B); free(C); free(VA); free(VB);
    return ORACLE_OK;
}

/* --------------------------------------------- Algorithm 1 and its backup */

/*
 * INSERTION-SORT (Algorithm 1) on a[0..m-1] with an optional payload v that
 * moves with its key.  The strict '>' in the inner loop is what keeps equal
 * keys in their input order.
 */
static void insertion_sort(uint64_t *a, uint32_t *v, uint64_t m)
{
    for (uint64_t j = 1; j < m; j++) {
        uint64_t key = a[j];
        uint32_t val = v ? v[j] : 0;
        int64_t i = (int64_t)j - 1;
        while (i >= 0 && a[i] > key) {
            a[i + 1] = a[i];
            if (v) v[i + 1] = v[i];
            i--;
        }
        a[i + 1] = key;
        if (v) v[i + 1] = val;
    }
}

/*
 * Bottom-up stable merge sort of a[0..m-1] (payload v optional) using the
 * scratch arrays ta/tv of m elements.  Equal keys are taken from the left
 * run first, which keeps the sort stable.
 */
static void merge_sort_stable(uint64_t *a, uint32_t *v, uint64_t m,
                              uint64_t *ta, uint32_t *tv)
{
    uint64_t *src = a, *dst = ta;
    uint32_t *vsrc = v, *vdst = tv;
    for (uint64_t width = 1; width < m; width *= 2) {
        for (uint64_t lo = 0; lo < m; lo += 2 * width) {
            uint64_t mid = lo + width < m ? lo + width : m;
            uint64_t hi = lo + 2 * width < m ? lo + 2 * width : m;
            uint64_t i = lo, j = mid, o = lo;
            while (i < mid && j < hi) {
                if (src[i] <= src[j]) {
                    dst[o] = src[i];
                    if (v) vdst[o] = vsrc[i];
                    i++;
                } else {
                    dst[o] = src[j];
                    if (v) vdst[o] = vsrc[j];
                    j++;
                }
                o++;
            }
            while (i < mid) { dst[o] = src[i]; if (v) vdst[o] = vsrc[i]; i++; o++; }
            while (j < hi) { dst[o] = src[j]; if (v) vdst[o] = vsrc[j]; j++; o++; }
        }
        uint64_t *t = src; src = dst; dst = t;
        uint32_t *tt = vsrc; vsrc = vdst; vdst = tt;
    }
    if (src != a) {
        memcpy(a, src, m * sizeof(uint64_t));
        if (v) memcpy(v, vsrc, m * sizeof(uint32_t));
    }
}

/* ------------------------------------------------------ Algorithm 2 (bucket) */

/*
 * Bucket of key k for the value range [mn, mx] and B buckets:
 * floor((k - mn) * B / (mx - mn + 1)), exact in 128-bit arithmetic.  The
 * range mx - mn + 1 can be 2^64 for 64-bit keys, which only u128 holds.
 */
static uint64_t bucket_of(uint64_t k, uint64_t mn, uint64_t mx, uint64_t B)
{
    u128 range = (u128)mx - (u128)mn + 1;
    u128 num = (u128)(k - mn) * (u128)B;
    return (uint64_t)(num / range);
}

uint64_t oracle_bucket_index(uint64_t k, uint64_t mn, uint64_t mx, uint64_t B)
{
    return bucket_of(k, mn, mx, B);
}

/*
 * BUCKET-SORT.
 *   nbuckets   : B >= 1.
 *   cutoff     : buckets of at most this many elements use Algorithm 1,
 *                larger ones the stable merge sort.
 *   key_bound  : 0 = the range is the keys' own [min, max]; otherwise the
 *                range is declared to be [0, key_bound] (the bound M of
 *                section 2.3), and a key above it goes to the last bucket.
 *   minmax     : optional [2] -> the range used (0, 0 for n == 0).
 *   counts     : optional [B] bucket sizes.
 *   offsets    : optional [B+1] exclusive prefix of counts (offsets[B] = n).
 *   scat_keys  : optional [n] uint64 keys after the scatter (buckets filled,
 *                not yet sorted).
 *   scat_vals  : optional [n] payload after the scatter.
 */
int oracle_bucket(const void *keys_in, void *keys_out, int key_bytes,
                  const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                  uint64_t nbuckets, uint64_t cutoff, uint64_t key_bound, uint64_t *minmax,
                  uint64_t *counts, uint64_t *offsets, uint64_t *scat_keys,
                  uint32_t *scat_vals)
{
    if (key_bytes != 4 && key_bytes != 8) return ORACLE_EINVAL;
    if (nbuckets < 1) return ORACLE_EINVAL;
    if ((vals_in == NULL) != (vals_out == NULL)) return ORACLE_EINVAL;
    if (n > 0 && (!keys_in || !keys_out)) return ORACLE_EINVAL;

    uint64_t *A = widen(keys_in, n, key_bytes);
    uint64_t *S = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t *T = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
    uint64_t *cnt = (uint64_t *)calloc(nbuckets, sizeof(uint64_t));
    uint64_t *off = (uint64_t *)malloc((nbuckets + 1) * sizeof(uint64_t));
    uint64_t *next = (uint64_t *)malloc(nbuckets * sizeof(uint64_t));
    uint32_t *SV = NULL, *TV = NULL;
    if (vals_in) {
        SV = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
        TV = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
    }
    if (!A || !S || !T || !cnt || !off || !next || (vals_in && (!SV || !TV))) {
        free(A); free(S); free(T); free(cnt); free(off); free(next);
        free(SV); free(TV);
        return ORACLE_ENOMEM;
    }

    /* value range: declared, or that of the input */
    uint64_t mn = 0, mx = 0;
    if (key_bound) {
        mx = key_bound;
    } else if (n > 0) {
        mn = A[0]; mx = A[0];
        for (uint64_t i = 1; i < n; i++) {
            if (A[i] < mn) mn = A[i];
            if (A[i] > mx) mx = A[i];
        }
    }
    /* keys above a declared bound join the last bucket */
#define BUCKET(k) (((k) > mx) ? nbuckets - 1 : bucket_of((k), mn, mx, nbuckets))

    /* bucket sizes, then where each bucket starts in the concatenation */
    for (uint64_t i = 0; i < n; i++) cnt[BUCKET(A[i])] += 1;
    off[0] = 0;
    for (uint64_t b = 0; b < nbuckets; b++) off[b + 1] = off[b] + cnt[b];

    /* insert every element into its bucket in input order */
    for (uint64_t b = 0; b < nbuckets; b++) next[b] = off[b];
    for (uint64_t i = 0; i < n; i++) {
        uint64_t b = BUCKET(A[i]);
        S[next[b]] = A[i];
        if (vals_in) SV[next[b]] = vals_in[i];
        next[b] += 1;
    }
    if (scat_keys) memcpy(scat_keys, S, n * sizeof(uint64_t));
    if (scat_vals && vals_in) memcpy(scat_vals, SV, n * sizeof(uint32_t));

    /* sort every bucket; the concatenation is the array itself */
    for (uint64_t b = 0; b < nbuckets; b++) {
        uint64_t m = cnt[b];
        uint64_t *a = S + off[b];
        uint32_t *v = vals_in ? SV + off[b] : NULL;
        if (m <= cutoff) insertion_sort(a, v, m);
        else merge_sort_stable(a, v, m, T, TV);
    }

    narrow(S, keys_out, n, key_bytes);
    if (vals_out) memcpy(vals_out, SV, n * sizeof(uint32_t));
    if (minmax) { minmax[0] = mn; minmax[1] = mx; }
    if (counts) memcpy(counts, cnt, nbuckets * sizeof(uint64_t));
    if (offsets) memcpy(offsets, off, (nbuckets + 1) * sizeof(uint64_t));
    free(A); free(S); free(T); free(cnt); free(off); free(next);
    free(SV); free(TV);
#undef BUCKET
    return ORACLE_OK;
}

/* ---------------------------------------------------------- segmented */

/*
 * Sort every segment [offsets[s], offsets[s+1]) of the packed array on its
 * own, with RADIX-SORT (algo 0) or BUCKET-SORT (algo 1).  Segments are
 * independent: nothing moves between them.  offsets must be nondecreasing,
 * start at 0 and end at n_total.
 */
int oracle_segmented(const void *keys_in, void *keys_out, int key_bytes,
                     const uint32_t *vals_in, uint32_t *vals_out,
                     uint64_t n_total, const uint64_t *offsets,
                     uint64_t num_segments, int algo, int r,
                     uint64_t nbuckets, uint64_t cutoff)
{
    if (key_bytes != 4 && key_bytes != 8) return ORACLE_EINVAL;
    if (num_segments > 0 && !offsets) return ORACLE_EINVAL;
    if (num_segments > 0 && (offsets[0] != 0 || offsets[num_segments] != n_total))
        return ORACLE_EINVAL;
    for (uint64_t s = 0; s < num_segments; s++)
        if (offsets[s + 1] < offsets[s]) return ORACLE_EINVAL;

    for (uint64_t s = 0; s < num_segments; s++) {
        uint64_t lo = offsets[s], m = offsets[s + 1] - lo;
        const char *kin = (const char *)keys_in + lo * (uint64_t)key_bytes;
        char *kout = (char *)keys_out + lo * (uint64_t)key_bytes;
        const uint32_t *vin = vals_in ? vals_in + lo : NULL;
        uint32_t *vout = vals_out ? vals_out + lo : NULL;
        int rc;
        if (algo == 0)
            rc = oracle_radix_lsd(kin, kout, key_bytes, vin, vout, m, r, 0,
                                  NULL, NULL, NULL);
        else
            rc = oracle_bucket(kin, kout, key_bytes, vin, vout, m, nbuckets,
                               cutoff, 0, NULL, NULL, NULL, NULL, NULL);
        if (rc != ORACLE_OK) return rc;
    }
    return ORACLE_OK;
}

/* ------------------------------------------ signed and floating-point keys */

/*
 * The paper's keys are integers (section 2) and its algorithms compare them
 * by value.  For keys that are not unsigned, "nondecreasing" needs an order
 * on the bit patterns:
 *   order 0: unsigned integers;
 *   order 1: two's-complement signed integers, by value;
 *   order 2: IEEE 754 binary32/binary64 in the totalOrder predicate of
 *            IEEE 754-2019 section 5.10: a key with the sign bit set comes
 *            before one without; between two keys without it the smaller
 *            magnitude (the remaining bits read as an unsigned integer)
 *            comes first; between two with it the larger magnitude comes
 *            first.  This places -NaN < -inf < negatives < -0 < +0 <
 *            positives < +inf < +NaN, NaNs ordered by their payload bits.
 * key_before(a, b) is the strict "a comes before b" of that order.
 */
static int key_before(uint64_t a, uint64_t b, int key_bytes, int order)
{
    const unsigned top = 8u * (unsigned)key_bytes - 1u;
    if (order == 0) return a < b;
    if (order == 1) {
        int64_t sa, sb;
        if (key_bytes == 4) { sa = (int32_t)(uint32_t)a; sb = (int32_t)(uint32_t)b; }
        else { sa = (int64_t)a; sb = (int64_t)b; }
        return sa < sb;
    }
    const uint64_t neg_a = (a >> top) & 1u, neg_b = (b >> top) & 1u;
    const uint64_t mag_mask = (top == 63u) ? ~(uint64_t)0 >> 1 : (((uint64_t)1 << top) - 1u);
    const uint64_t ma = a & mag_mask, mb = b & mag_mask;
    if (neg_a != neg_b) return neg_a > neg_b;
    if (neg_a) return ma > mb;
    return ma < mb;
}

/*
 * Stable sort of n keys in the order above (payload optional): a bottom-up
 * merge sort that takes the right run's key only when it comes strictly
 * before the left run's, so keys with equal bits keep their input order --
 * the stable permutation of section 2's definition, unique for each input.
 */
int oracle_sort_ordered(const void *keys_in, void *keys_out, int key_bytes, int order,
                        const uint32_t *vals_in, uint32_t *vals_out, uint64_t n)
{
    if (key_bytes != 4 && key_bytes != 8) return ORACLE_EINVAL;
    if (order < 0 || order > 2) return ORACLE_EINVAL;
    if ((vals_in == NULL) != (vals_out == NULL)) return ORACLE_EINVAL;
    if (n == 0) return ORACLE_OK;
    if (!keys_in || !keys_out) return ORACLE_EINVAL;
    uint64_t *a = widen(keys_in, n, key_bytes);
    uint64_t *t = (uint64_t *)malloc(n * sizeof(uint64_t));
    uint32_t *v = NULL, *tv = NULL;
    if (vals_in) {
        v = (uint32_t *)malloc(n * sizeof(uint32_t));
        tv = (uint32_t *)malloc(n * sizeof(uint32_t));
        if (v) memcpy(v, vals_in, n * sizeof(uint32_t));
    }
    if (!a || !t || (vals_in && (!v || !tv))) {
        free(a); free(t); free(v); free(tv);
        return ORACLE_ENOMEM;
    }
    uint64_t *src = a, *dst = t;
    uint32_t *vs = v, *vd = tv;
    for (uint64_t width = 1; width < n; width *= 2) {
        for (uint64_t lo = 0; lo < n; lo += 2 * width) {
            uint64_t mid = lo + width < n ? lo + width : n;
            uint64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            uint64_t i = lo, j = mid, o = lo;
            while (i < mid || j < hi) {
                int right = i == mid || (j < hi && key_before(src[j], src[i], key_bytes, order));
                uint64_t from = right ? j++ : i++;
                dst[o] = src[from];
                if (v) vd[o] = vs[from];
                o++;
            }
        }
        uint64_t *x = src; src = dst; dst = x;
        uint32_t *y = vs; vs = vd; vd = y;
    }
    narrow(src, keys_out, n, key_bytes);
    if (vals_out) memcpy(vals_out, vs, n * sizeof(uint32_t));
    free(a); free(t); free(v); free(tv);
    return ORACLE_OK;
}
