// bucket_sort.hip -- BUCKET-SORT (section 2.3, Algorithm 2) for gfx950.
//
// Algorithm 2 drops every key, in input order, into the bucket its value
// selects, sorts every bucket (insertion sort, Algorithm 1) and concatenates
// the buckets.  On the GPU:
//   1. min and max of the keys (the value range the paper assumes known);
//   2. the histogram of the exact bucket index b(k) = floor((k-min)*B/R);
//   3. offsets: where every bucket starts in the concatenation (exclusive
//      scan of the histogram) -- concatenation costs no data movement;
//   4. a stable scatter by b(k): keys keep their input order inside each
//      bucket, as the paper's lists do.  B <= 2048 takes one pass whose digit
//      is b(k) itself; up to 65536 buckets take two stable 8-bit passes over
//      b(k), after which the bucket starts are found where b changes;
//   5. every bucket is sorted on its own by the segmented sort (buckets that
//      fit on chip by one workgroup in LDS, larger ones by all workgroups).
// Every step keeps its data on the device; the host never waits.

#include <stdint.h>

#include <algorithm>

#include "bucket_map.hpp"
#include "device_common.hpp"
#include "intsort.h"
#include "internal.hpp"
#include "onesweep.hpp"
#include "sort_plans.hpp"

namespace intsort {

constexpr int BK_THREADS = 256;
constexpr uint32_t SUBHIST_WORDS = 2 * 256;

// counts of the low and the high byte of b(k), for the two scatter passes
template <typename K>
__global__ __launch_bounds__(BK_THREADS) void k_bucket_subhist(const K *__restrict__ keys, uint64_t n,
                                                               const uint64_t *__restrict__ minmax, uint32_t B,
                                                               uint32_t *__restrict__ subhist)
{
    __shared__ uint32_t s_h[SUBHIST_WORDS];
    const BucketMap m = make_bucket_map(minmax[0], minmax[1], B);
    for (uint32_t i = threadIdx.x; i < SUBHIST_WORDS; i += BK_THREADS) s_h[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * BK_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * BK_THREADS + threadIdx.x; i < n; i += stride) {
        const uint32_t b = bucket_of(m, keys[i]);
        atomicAdd(&s_h[b & 255u], 1u);
        atomicAdd(&s_h[256 + (b >> 8)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < SUBHIST_WORDS; i += BK_THREADS)
        if (s_h[i]) atomicAdd(&subhist[i], s_h[i]);
}

// One workgroup: exclusive offsets of the scatter digit(s), the bucket
// starts when the scatter is a single pass, and the plan words.
struct BucketPlanArgs {
    const uint32_t *counts;   // [B], when the full histogram was taken
    const uint32_t *subhist;  // [2][256], when only the byte histograms were
    uint32_t *excl;           // [passes][radix]
    uint64_t *offsets;        // [B + 1]
    uint32_t *plan;
    uint32_t B, radix, passes;
    uint32_t full;            // counts holds the full histogram
    uint64_t n;
};

__global__ __launch_bounds__(BK_THREADS) void k_bucket_plan(BucketPlanArgs a)
{
    __shared__ uint32_t s_scan[BK_THREADS / WAVE + 1];
    __shared__ uint32_t s_byte[2 * 256];
    const uint32_t tid = threadIdx.x;
    if (a.full) {
        // bucket starts: exclusive scan of the full histogram (B <= 16384:
        // 64 buckets per thread at most)
        const uint32_t per = (a.B + BK_THREADS - 1) / BK_THREADS;
        uint32_t mine = 0;
        for (uint32_t i = 0; i < per; i++) {
            const uint32_t b = tid * per + i;
            if (b < a.B) mine += a.counts[b];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<BK_THREADS>(mine, s_scan, &total);
        for (uint32_t i = 0; i < per; i++) {
            const uint32_t b = tid * per + i;
            if (b < a.B) {
                a.offsets[b] = run;
                run += a.counts[b];
            }
        }
        if (tid == 0) a.offsets[a.B] = a.n;
        // counts of the low and the high byte of the bucket index
        for (uint32_t i = tid; i < 512u; i += BK_THREADS) s_byte[i] = 0;
        __syncthreads();
        for (uint32_t b = tid; b < a.B; b += BK_THREADS) {
            const uint32_t c = a.counts[b];
            if (c) {
                atomicAdd(&s_byte[b & 255u], c);
                atomicAdd(&s_byte[256 + (b >> 8)], c);
            }
        }
        __syncthreads();
    }
    for (uint32_t p = 0; p < a.passes; p++) {
        const uint32_t d = tid;   // radix 256: one digit per thread
        const uint32_t c = a.full ? s_byte[p * 256 + d] : a.subhist[p * 256 + d];
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<BK_THREADS>(c, s_scan, &total);
        a.excl[p * a.radix + d] = ex;
    }
    if (tid == 0) {
        uint32_t *w = a.plan;
        if (a.passes == 1) {
            w[0] = 1; w[1] = BUF_IN; w[2] = BUF_OUT; w[3] = 0;
        } else {
            w[0] = 1; w[1] = BUF_IN; w[2] = BUF_TMP; w[3] = 0;
            w += PLAN_WORDS;
            w[0] = 1; w[1] = BUF_TMP; w[2] = BUF_OUT; w[3] = 1;
        }
    }
}

// after a two-pass scatter the keys are grouped by bucket: a bucket starts
// where b changes (offsets were filled with n beforehand)
template <typename K>
__global__ __launch_bounds__(BK_THREADS) void k_bucket_bounds(const K *__restrict__ keys, uint64_t n,
                                                              const uint64_t *__restrict__ minmax, uint32_t B,
                                                              uint64_t *__restrict__ offsets)
{
    const BucketMap m = make_bucket_map(minmax[0], minmax[1], B);
    const uint64_t stride = (uint64_t)gridDim.x * BK_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * BK_THREADS + threadIdx.x; i < n; i += stride) {
        const uint32_t b = bucket_of(m, keys[i]);
        if (i == 0 || bucket_of(m, keys[i - 1]) != b) offsets[b] = i;
    }
}

// an empty bucket starts where the next nonempty one does: offsets[b] =
// min(offsets[b], offsets[b + 1]) from the end (one workgroup)
__global__ __launch_bounds__(1024) void k_suffix_min(uint64_t *offsets, uint32_t count)
{
    __shared__ uint64_t s_m[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (count + 1023) / 1024;
    const uint32_t lo = tid * per, hi = min(count, lo + per);
    uint64_t run = ~0ull;
    for (uint32_t i = hi; i-- > lo;) run = min(run, offsets[i]);
    s_m[tid] = run;
    __syncthreads();
    if (tid == 0) {
        uint64_t r = ~0ull;
        for (int t = 1023; t >= 0; t--) {
            const uint64_t x = s_m[t];
            s_m[t] = r;   // minimum over the chunks after t
            r = min(r, x);
        }
    }
    __syncthreads();
    run = s_m[tid];
    for (uint32_t i = hi; i-- > lo;) {
        run = min(run, offsets[i]);
        offsets[i] = run;
    }
}

// ------------------------------------------------------------------ host

static uint32_t scatter_bits(uint32_t) { return 8u; }
constexpr uint32_t BUCKET_LDS_HIST_MAX = 16384;   // bucket_histogram_run's on-chip limit

template <typename K>
static uint64_t scatter_tile(uint32_t) { return PassCfg<K, 8>::TILE; }

BucketLayout bucket_layout(int key_bytes, bool pairs, uint64_t n, const intsort_options &o)
{
    BucketLayout L{};
    L.buckets = o.num_buckets;
    L.bits = scatter_bits(L.buckets);
    L.scatter_passes = L.buckets <= 256 ? 1u : 2u;
    const uint64_t tile = key_bytes == 4 ? scatter_tile<uint32_t>(L.bits) : scatter_tile<uint64_t>(L.bits);
    L.num_tiles = (n + tile - 1) / tile;
    const uint64_t radix = 1ull << L.bits;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes, 256); return at; };
    L.counters = take((size_t)CTR_WORDS * 4);
    L.plan = take((size_t)(MAX_PASSES + 1) * PLAN_WORDS * 4);
    L.minmax = take(16);
    L.counts = take((size_t)L.buckets * 4);
    L.subhist = take((size_t)SUBHIST_WORDS * 4);
    L.excl = take((size_t)2 * radix * 4);
    L.offsets = take((size_t)(L.buckets + 1) * 8);
    L.status0 = take((size_t)L.num_tiles * (radix + 1) * 4);
    L.status1 = take((size_t)L.num_tiles * (radix + 1) * 4);
    L.tmpb_keys = take(n * (size_t)key_bytes);
    L.tmpb_vals = take(pairs ? n * 4 : 0);
    intsort_options so = o;
    so.digit_bits = 8;
    L.S = segmented_layout(key_bytes, pairs, n, L.buckets, so);
    L.seg = take(L.S.total);
    L.total = off;
    return L;
}

template <typename K, bool PAIRS, int BITS>
static hipError_t bucket_run_typed(const BucketCall &c, hipStream_t s)
{
    using C = PassCfg<K, BITS>;
    const BucketLayout &L = c.L;
    char *ws = c.ws;
    Timer *tm = c.timer;
    const uint32_t B = L.buckets;
    uint32_t *counters = reinterpret_cast<uint32_t *>(ws + L.counters);
    uint32_t *plan = reinterpret_cast<uint32_t *>(ws + L.plan);
    uint64_t *minmax = reinterpret_cast<uint64_t *>(ws + L.minmax);
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + L.counts);
    uint32_t *subhist = reinterpret_cast<uint32_t *>(ws + L.subhist);
    uint32_t *excl = reinterpret_cast<uint32_t *>(ws + L.excl);
    uint64_t *offsets = reinterpret_cast<uint64_t *>(ws + L.offsets);
    uint32_t *status0 = reinterpret_cast<uint32_t *>(ws + L.status0);
    uint32_t *status1 = reinterpret_cast<uint32_t *>(ws + L.status1);
    K *tmpb = reinterpret_cast<K *>(ws + L.tmpb_keys);
    uint32_t *tmpb_v = reinterpret_cast<uint32_t *>(ws + L.tmpb_vals);
    char *segws = ws + L.seg;
    K *tmpc = reinterpret_cast<K *>(segws + L.S.tmp_keys);       // free until the bucket sorts start
    uint32_t *tmpc_v = reinterpret_cast<uint32_t *>(segws + L.S.tmp_vals);
    const bool scatter_only = c.opts.max_passes == 1;
    int dev = 0;
    (void)hipGetDevice(&dev);
    const uint32_t fill_grid = (uint32_t)device_cu_count(dev) * 4;

    if (tm) tm->start(s);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, s, counters, (uint64_t)CTR_WORDS, 0u);
    hipError_t e = minmax_run((int)sizeof(K), c.keys_in, c.n, minmax, s);
    if (e != hipSuccess) return e;
    if (tm) tm->mark(INTSORT_KERNEL_MINMAX, 0, s);
    const bool full_hist = B <= BUCKET_LDS_HIST_MAX;
    if (full_hist) {
        e = bucket_histogram_run((int)sizeof(K), c.keys_in, c.n, minmax, B, counts, s);
    } else {
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(2), dim3(256), 0, s, subhist, (uint64_t)SUBHIST_WORDS, 0u);
        uint64_t blocks = std::min<uint64_t>((c.n + BK_THREADS - 1) / BK_THREADS, (uint64_t)fill_grid * 2);
        hipLaunchKernelGGL((k_bucket_subhist<K>), dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(BK_THREADS), 0,
                           s, static_cast<const K *>(c.keys_in), c.n, minmax, B, subhist);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (tm) tm->mark(INTSORT_KERNEL_BUCKET_HISTOGRAM, 0, s);
    BucketPlanArgs pa{counts, subhist, excl, offsets, plan, B, (uint32_t)C::RADIX, L.scatter_passes,
                      full_hist ? 1u : 0u, c.n};
    hipLaunchKernelGGL(k_bucket_plan, dim3(1), dim3(BK_THREADS), 0, s, pa);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(fill_grid), dim3(256), 0, s, status0,
                       (uint64_t)L.num_tiles * (C::RADIX + 1), 0u);
    if (tm) tm->mark(INTSORT_KERNEL_PLAN, 0, s);

    // the stable scatter by bucket
    PassArgs<K> a{};
    a.in = static_cast<const K *>(c.keys_in);
    a.out = scatter_only ? static_cast<K *>(c.keys_out) : tmpb;
    a.tmp = tmpc;
    a.vin = c.vals_in;
    a.vout = scatter_only ? c.vals_out : tmpb_v;
    a.vtmp = tmpc_v;
    a.status0 = status0;
    a.status1 = status1;
    a.counters = counters;
    a.n = (uint32_t)c.n;
    a.tile_capacity = (uint32_t)L.num_tiles;
    for (uint32_t p = 0; p < L.scatter_passes; p++) {
        a.plan = plan + p * PLAN_WORDS;
        a.pass = p;
        const BucketDigitArgs dg{minmax, B, 8u * p, (uint32_t)(C::RADIX - 1)};
        const PlainTiles tl{(uint32_t)c.n, (uint32_t)L.num_tiles, excl + p * C::RADIX};
        hipLaunchKernelGGL((k_onesweep<K, BITS, PAIRS, BucketDigitArgs, PlainTiles>), dim3((uint32_t)L.num_tiles),
                           dim3(C::NT), 0, s, a, dg, tl);
        if (tm) tm->mark(INTSORT_KERNEL_BUCKET_SCATTER, p, s);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (scatter_only) return hipSuccess;

    if (!full_hist) {
        hipLaunchKernelGGL(k_fill<uint64_t>, dim3((B + 256) / 256), dim3(256), 0, s, offsets, (uint64_t)B + 1,
                           (uint64_t)c.n);
        uint64_t blocks = std::min<uint64_t>((c.n + BK_THREADS - 1) / BK_THREADS, (uint64_t)fill_grid * 2);
        hipLaunchKernelGGL((k_bucket_bounds<K>), dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(BK_THREADS), 0,
                           s, tmpb, c.n, minmax, B, offsets);
        hipLaunchKernelGGL(k_suffix_min, dim3(1), dim3(1024), 0, s, offsets, B + 1);
        if (tm) tm->mark(INTSORT_KERNEL_PLAN, 1, s);
    }

    // every bucket sorted on its own: buckets are the segments
    SegCall sc{};
    sc.keys_in = tmpb;
    sc.keys_out = c.keys_out;
    sc.vals_in = PAIRS ? tmpb_v : nullptr;
    sc.vals_out = PAIRS ? c.vals_out : nullptr;
    sc.n = c.n;
    sc.num_segments = B;
    sc.offsets = offsets;
    sc.key_bytes = (int)sizeof(K);
    sc.pairs = PAIRS;
    sc.opts = c.opts;
    sc.opts.digit_bits = 8;
    sc.L = L.S;
    sc.ws = segws;
    sc.timer = tm;
    return segmented_sort_run(sc, s);
}

template <typename K, bool PAIRS>
static hipError_t bucket_run_bits(const BucketCall &c, hipStream_t s)
{
    return bucket_run_typed<K, PAIRS, 8>(c, s);
}

hipError_t bucket_sort_run(const BucketCall &c, hipStream_t s)
{
    if (c.key_bytes == 4) return c.pairs ? bucket_run_bits<uint32_t, true>(c, s) : bucket_run_bits<uint32_t, false>(c, s);
    return c.pairs ? bucket_run_bits<uint64_t, true>(c, s) : bucket_run_bits<uint64_t, false>(c, s);
}

}  // namespace intsort
