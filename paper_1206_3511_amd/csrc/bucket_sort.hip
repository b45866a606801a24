// bucket_sort.hip -- BUCKET-SORT (section 2.3, Algorithm 2) for gfx950.
//
// Algorithm 2 drops every key, in input order, into the bucket its value
// selects, sorts every bucket (insertion sort, Algorithm 1) and concatenates
// the buckets.  On the GPU:
//   1. min and max of the keys (the value range the paper assumes known),
//      and whether they are already in nondecreasing order: then b(k) is
//      nondecreasing too, the scatter and every bucket sort are the
//      identity, and all later stages are skipped for one copy (with a
//      declared range the bucket histogram finds the order instead);
//   2. the histogram of the exact bucket index b(k) = floor((k-min)*B/R);
//   3. offsets: where every bucket starts in the concatenation (exclusive
//      scan of the histogram) -- concatenation costs no data movement;
//   4. a stable scatter by b(k): keys keep their input order inside each
//      bucket, as the paper's lists do.  It takes one stable 8-bit pass per
//      byte of b(k) (1 to 4); with more than 16384 buckets the bucket starts
//      are then found where b changes;
//   5. every bucket is sorted on its own by the segmented sort (on chip up
//      to one workgroup's capacity, by all workgroups above).  Buckets are
//      value ranges in order, so sorting a run of whole buckets by key sorts
//      each of them: with many tiny buckets (the paper's B = n) the small
//      ones are sorted in windows of consecutive buckets instead, one
//      workgroup in LDS each.
// Every step keeps its data on the device; the host never waits.

#include <stdint.h>

#include <algorithm>

#include "bucket_map.hpp"
#include "device_common.hpp"
#include "intsort.h"
#include "internal.hpp"
#include "lds_sort.hpp"
#include "onesweep.hpp"
#include "sort_plans.hpp"

namespace intsort {

constexpr int BK_THREADS = 256;
constexpr uint32_t SUBHIST_WORDS = 4 * 256;
constexpr uint32_t SUBHIST_COPIES = 8;     // 32 KB of LDS counts per workgroup
constexpr uint64_t WINDOW_AVG = 64;       // below this many keys per bucket, windows

// counts of every byte of b(k) that a scatter pass sorts on
template <typename K, bool ABOVE>
__global__ __launch_bounds__(BK_THREADS) void k_bucket_subhist(const K *__restrict__ keys, uint64_t n,
                                                               const uint64_t *__restrict__ minmax, uint32_t B,
                                                               uint32_t passes, uint32_t *__restrict__ subhist,
                                                               const uint64_t *skip, uint64_t *order,
                                                               uint64_t *above)
{
    // SUBHIST_COPIES copies of the counts, lane l adding into copy
    // l % SUBHIST_COPIES: lanes of one instruction meet on a bank or a word
    // a few times at most, whatever the keys (sorted runs of a few values
    // included), where one shared copy serialises them
    __shared__ uint32_t s_h[SUBHIST_WORDS * SUBHIST_COPIES];
    if (skip && *skip) return;   // keys already sorted
    // with `order`, also whether the keys are already sorted
    // (and with ABOVE, whether a key exceeds the range's maximum)
    const bool check = order != nullptr;
    bool order_ok = true;
    K seen = 0;   // largest key this thread counted (ABOVE)
    const BucketMap m = make_bucket_map(minmax[0], minmax[1], B);
    for (uint32_t i = threadIdx.x; i < SUBHIST_WORDS * SUBHIST_COPIES; i += BK_THREADS) s_h[i] = 0;
    __syncthreads();
    uint32_t *my_h = s_h + threadIdx.x % SUBHIST_COPIES;
    auto count = [&](K k) {
        const uint32_t b = bucket_of(m, k);
        if (ABOVE) seen = seen > k ? seen : k;
        for (uint32_t p = 0; p < passes; p++) atomicAdd(my_h + (p * 256 + ((b >> (8 * p)) & 255u)) * SUBHIST_COPIES, 1u);
    };
    constexpr int KPV = 16 / (int)sizeof(K);
    struct alignas(16) Vec { K v[KPV]; };
    const uint64_t nvec = n / KPV;
    const Vec *vk = reinterpret_cast<const Vec *>(keys);
    const uint64_t stride = (uint64_t)gridDim.x * BK_THREADS;
    for (uint64_t v = (uint64_t)blockIdx.x * BK_THREADS + threadIdx.x; v < nvec; v += stride) {
        const Vec x = vk[v];
        if (check && !vector_in_order<K, KPV>(x.v, keys, v, nvec)) order_ok = false;
#pragma unroll
        for (int e = 0; e < KPV; e++) count(x.v[e]);
    }
    for (uint64_t i = nvec * KPV + (uint64_t)blockIdx.x * BK_THREADS + threadIdx.x; i < n; i += stride) {
        count(keys[i]);
        if (check && i > 0 && keys[i] < keys[i - 1]) order_ok = false;
    }
    if (check) {
        if (__syncthreads_or(!order_ok) && threadIdx.x == 0) *order = 0;
    } else {
        __syncthreads();
    }
    if (ABOVE && __syncthreads_or(seen > (K)minmax[1]) && threadIdx.x == 0) *above = 1;
    for (uint32_t i = threadIdx.x; i < SUBHIST_WORDS; i += BK_THREADS) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t q = 0; q < SUBHIST_COPIES; q++) c += s_h[i * SUBHIST_COPIES + (q + i) % SUBHIST_COPIES];
        if (c) atomicAdd(&subhist[i], c);
    }
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
    const uint64_t *skip;     // nonzero: the keys are already sorted, no pass runs
    uint32_t in_place;        // the passes write the caller's output, which aliases its
                              // input (keys or values): start in the scratch buffer
    const uint64_t *minmax;
    uint64_t *bucket_skip;    // set here: what the per-bucket sorts do (BSKIP_*)
    const uint64_t *above;    // declared range: nonzero when some key lies above it
};

// the per-bucket stage after the scatter: BSKIP_NONE sorts every bucket;
// BSKIP_SORTED does nothing (the input was already in order and is copied);
// BSKIP_SINGLE does nothing either, because B >= R: then b(k) is strictly
// increasing on [min, max], every bucket holds copies of one key value, and
// the scattered keys are already the sorted output (they are copied there).
// Keys above a declared bound all go to the last bucket, which can then hold
// several values: with any such key the buckets are sorted as usual.
constexpr uint64_t BSKIP_NONE = 0, BSKIP_SORTED = 1, BSKIP_SINGLE = 2;

__global__ __launch_bounds__(BK_THREADS) void k_bucket_plan(BucketPlanArgs a)
{
    __shared__ uint32_t s_scan[BK_THREADS / WAVE + 1];
    __shared__ uint32_t s_byte[2 * 256];
    const uint32_t tid = threadIdx.x;
    uint32_t *f = a.plan + MAX_PASSES * PLAN_WORDS;   // final-copy words
    if (tid == 0) {
        const uint64_t range_m1 = a.minmax[1] - a.minmax[0];   // R - 1
        const bool single = range_m1 < (uint64_t)a.B && !(a.above && *a.above);
        *a.bucket_skip = *a.skip ? BSKIP_SORTED : (single ? BSKIP_SINGLE : BSKIP_NONE);
    }
    if (*a.skip) {
        if (tid == 0) {
            for (uint32_t q = 0; q < a.passes; q++) a.plan[q * PLAN_WORDS] = 0;
            f[0] = 0;
        }
        return;
    }
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
        // passes alternate so that the last one lands in the output; in
        // place, no pass may read and write one buffer, so they alternate
        // from the scratch buffer and a copy follows when the last one
        // lands there
        uint32_t prev = BUF_IN;
        for (uint32_t q = 0; q < a.passes; q++) {
            uint32_t *w = a.plan + q * PLAN_WORDS;
            uint32_t dst;
            if (a.in_place) dst = (q % 2 == 0) ? BUF_TMP : BUF_OUT;
            else dst = ((a.passes - 1 - q) % 2 == 0) ? BUF_OUT : BUF_TMP;
            w[0] = 1; w[1] = prev; w[2] = dst; w[3] = q;
            prev = dst;
        }
        f[0] = prev == BUF_TMP ? (COPY_KEYS | COPY_VALS) : 0u;
        f[1] = BUF_TMP;
        f[2] = BUF_OUT;
        f[3] = a.passes;
    }
}

// After the scatter the keys are grouped by bucket, in bucket order, so
// bucket b starts at the first position whose bucket is at least b (an empty
// bucket where the next nonempty one does, offsets[B] = n).  With
// c(p) = b(p) + 1, c(-1) = 0 and c(n) = B + 1, position p therefore starts
// buckets c(p-1) .. c(p)-1, and every offset has exactly one such position.
// A lane takes BS_V consecutive positions (vector loads), a wave 64 BS_V; a
// wave whose positions start no bucket (most of them when B is much smaller
// than n) writes nothing.  Otherwise the runs of its positions are adjacent,
// in position order, so the wave writes them together: lane t takes the t-th
// offset of the runs, finds its position by a binary search over the runs'
// running lengths, and the stores of a wave are contiguous.  A run longer
// than START_RUN (a wide gap of empty buckets) is cut into pieces of
// START_RUN and listed for k_bucket_start_runs instead.
constexpr uint64_t START_RUN = 1024;
constexpr int CTR_START_RUNS = 48;   // counter word: pieces listed
static_assert(CTR_START_RUNS < CTR_WORDS && CTR_START_RUNS > CTR_ERROR, "a free counter word");
constexpr int BS_V = 8;                 // positions per lane
constexpr int BS_WP = WAVE * BS_V;      // positions per wave and step

struct StartRun {
    uint64_t lo, hi, p;   // offsets[lo .. hi) = p
};

static uint64_t start_run_cap(uint64_t B)
{
    // pieces <= (sum of the long runs) / START_RUN + (number of long runs),
    // both at most (B + 1) / START_RUN
    return 2 * ((B + 1) / START_RUN) + 2;
}

template <typename K>
__global__ __launch_bounds__(BK_THREADS) void k_bucket_starts(const K *__restrict__ keys, uint64_t n,
                                                              const uint64_t *__restrict__ minmax, uint32_t B,
                                                              uint64_t *__restrict__ offsets, StartRun *runs,
                                                              uint32_t *counters, uint64_t run_cap,
                                                              const uint64_t *skip)
{
    constexpr int NW = BK_THREADS / WAVE;
    __shared__ uint32_t s_excl[NW][BS_WP + 1];   // running run length before each position
    __shared__ uint64_t s_lo[NW][BS_WP];         // first offset of each position's run
    if (*skip) return;   // keys already sorted: no bucket starts needed
    const BucketMap m = make_bucket_map(minmax[0], minmax[1], B);
    const uint32_t lane = lane_id(), wave = threadIdx.x / WAVE;
    uint32_t *w_excl = s_excl[wave];
    uint64_t *w_lo = s_lo[wave];
    const uint64_t end = (uint64_t)B + 1;   // c(n), and c of every position past n
    const uint64_t stride = (uint64_t)gridDim.x * NW * BS_WP;
    // the same trip count for every lane of a wave
    for (uint64_t base = ((uint64_t)blockIdx.x * NW + wave) * BS_WP; base <= n; base += stride) {
        const uint64_t p0 = base + (uint64_t)lane * BS_V;
        uint64_t c[BS_V];
        if (p0 + BS_V <= n) {
            // whole vectors (p0 is a multiple of 8, the buffer 16-byte aligned)
            constexpr int NV = BS_V * (int)sizeof(K) / 16;
            const uint4 *vp = reinterpret_cast<const uint4 *>(keys + p0);
            uint4 w[NV];
#pragma unroll
            for (int q = 0; q < NV; q++) w[q] = vp[q];
            K key[BS_V];
            __builtin_memcpy(key, w, sizeof(key));
#pragma unroll
            for (int i = 0; i < BS_V; i++) c[i] = (uint64_t)bucket_of(m, key[i]) + 1;
        } else {
#pragma unroll
            for (int i = 0; i < BS_V; i++) c[i] = p0 + i < n ? (uint64_t)bucket_of(m, keys[p0 + i]) + 1 : end;
        }
        // c of the position before the lane's first one
        uint64_t cprev = __shfl_up(c[BS_V - 1], 1, WAVE);
        if (lane == 0) cprev = p0 == 0 ? 0 : (p0 - 1 < n ? (uint64_t)bucket_of(m, keys[p0 - 1]) + 1 : end);
        uint32_t len[BS_V];
        uint32_t mine = 0;
#pragma unroll
        for (int i = 0; i < BS_V; i++) {
            const uint64_t lo = i == 0 ? cprev : c[i - 1], hi = c[i];
            len[i] = 0;
            if (hi < lo) {   // not grouped by bucket: cannot happen after the scatter
                atomicOr(&counters[CTR_ERROR], DEVERR_SCATTER_RANGE);
            } else if (hi - lo <= START_RUN) {
                len[i] = (uint32_t)(hi - lo);
            } else {
                const uint64_t pieces = (hi - lo + START_RUN - 1) / START_RUN;
                const uint64_t at = atomicAdd(&counters[CTR_START_RUNS], (uint32_t)pieces);
                for (uint64_t q = 0; q < pieces; q++) {
                    if (at + q >= run_cap) {   // sized so that this cannot happen
                        atomicOr(&counters[CTR_ERROR], DEVERR_SCATTER_RANGE);
                        break;
                    }
                    const uint64_t a = lo + q * START_RUN;
                    runs[at + q] = StartRun{a, min(hi, a + START_RUN), p0 + i};
                }
            }
            mine += len[i];
        }
        if (ballot(mine != 0) == 0) continue;   // no bucket starts here
        const uint32_t incl = wave_inclusive_scan(mine);
        const uint32_t total = __shfl(incl, WAVE - 1, WAVE);
        uint32_t run = incl - mine;
#pragma unroll
        for (int i = 0; i < BS_V; i++) {
            w_excl[lane * BS_V + i] = run;
            w_lo[lane * BS_V + i] = i == 0 ? cprev : c[i - 1];
            run += len[i];
        }
        if (lane == WAVE - 1) w_excl[BS_WP] = total;
        wave_sync();
        for (uint32_t u = lane; u < total; u += WAVE) {
            // the last position whose runs start at or before offset u owns
            // it (a position with an empty run shares its start with the next)
            uint32_t x = 0, y = BS_WP - 1;
            while (x < y) {
                const uint32_t mid = (x + y + 1) / 2;
                if (w_excl[mid] <= u) x = mid;
                else y = mid - 1;
            }
            offsets[w_lo[x] + (u - w_excl[x])] = base + x;
        }
        wave_sync();
    }
}

// one workgroup per listed piece of a long run of bucket starts
__global__ __launch_bounds__(BK_THREADS) void k_bucket_start_runs(const StartRun *runs, const uint32_t *counters,
                                                                  uint64_t run_cap, uint64_t *__restrict__ offsets,
                                                                  const uint64_t *skip)
{
    if (*skip) return;
    const uint64_t listed = min((uint64_t)counters[CTR_START_RUNS], run_cap);
    for (uint64_t r = blockIdx.x; r < listed; r += gridDim.x) {
        const StartRun e = runs[r];
        for (uint64_t b = e.lo + threadIdx.x; b < e.hi; b += BK_THREADS) offsets[b] = e.p;
    }
}

// the declared range [0, key_bound] in place of a measured one; whether
// the keys are in order is then found by the bucket histogram
__global__ void k_set_range(uint64_t *minmax, uint64_t lo, uint64_t hi, uint64_t *sorted, uint64_t *above)
{
    minmax[0] = lo;
    minmax[1] = hi;
    *sorted = 1;
    *above = 0;
}

// With one key value per bucket the scattered keys (and values) are the
// sorted output
template <typename K>
__global__ __launch_bounds__(BK_THREADS) void k_copy_if_single(const uint64_t *bucket_skip, const K *__restrict__ kin,
                                                               K *__restrict__ kout, const uint32_t *__restrict__ vin,
                                                               uint32_t *__restrict__ vout, uint64_t n)
{
    if (*bucket_skip != BSKIP_SINGLE) return;
    const uint64_t stride = (uint64_t)gridDim.x * BK_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * BK_THREADS + threadIdx.x; i < n; i += stride) {
        kout[i] = kin[i];
        if (vout) vout[i] = vin[i];
    }
}

// When the keys were already in order, the sort is the identity: the
// output is a copy of the input (the stages before left it untouched)
template <typename K>
__global__ __launch_bounds__(BK_THREADS) void k_copy_if_sorted(const uint64_t *sorted, const K *__restrict__ kin,
                                                               K *__restrict__ kout, const uint32_t *__restrict__ vin,
                                                               uint32_t *__restrict__ vout, uint64_t n)
{
    if (!*sorted) return;
    const uint64_t stride = (uint64_t)gridDim.x * BK_THREADS;
    for (uint64_t i = (uint64_t)blockIdx.x * BK_THREADS + threadIdx.x; i < n; i += stride) {
        if (kout != kin) kout[i] = kin[i];
        if (vout && vout != vin) vout[i] = vin[i];
    }
}

// Windows of consecutive small buckets.  Window g holds the buckets that
// start in positions [g*half, (g+1)*half) of the scattered array, less a
// last bucket longer than half (that one goes to the segmented sort).  A
// bucket start is found from the key at a position: the bucket b of the key
// at p starts at offsets[b]; the first bucket starting at or after p starts
// at p if offsets[b] == p, else at offsets[b + 1].  A window holds at most
// half + half keys.
template <typename K>
struct WindowSrc {
    const K *keys;              // scattered keys, grouped by bucket
    K *out;
    const uint32_t *vin;
    uint32_t *vout;
    const uint64_t *offsets;    // [B + 1], nondecreasing
    const uint64_t *minmax;
    uint32_t B;
    uint32_t half;
    uint64_t n;
    const uint64_t *skip;       // nonzero: keys already sorted, every window empty
    __device__ __forceinline__ uint64_t start_at_or_after(const BucketMap &m, uint64_t p) const
    {
        if (p >= n) return n;
        const uint32_t b = bucket_of(m, keys[p]);
        const uint64_t s = offsets[b];
        return s == p ? p : offsets[b + 1];
    }
    template <typename KK>
    __device__ __forceinline__ void seg(uint64_t g, const KK *&kin, KK *&kout, const uint32_t *&vi, uint32_t *&vo,
                                        uint32_t &mlen, uint32_t &base) const
    {
        if (*skip) {
            mlen = 0;
            base = 0;
            kin = reinterpret_cast<const KK *>(keys);
            kout = reinterpret_cast<KK *>(out);
            vi = vin;
            vo = vout;
            return;
        }
        const BucketMap m = make_bucket_map(minmax[0], minmax[1], B);
        const uint64_t lo = start_at_or_after(m, g * half);
        uint64_t hi = start_at_or_after(m, (g + 1) * half);
        if (hi > lo) {
            const uint64_t sl = offsets[bucket_of(m, keys[hi - 1])];
            if (hi - sl > half) hi = sl > lo ? sl : lo;
        }
        mlen = hi > lo ? (uint32_t)(hi - lo) : 0u;
        base = (uint32_t)lo;
        kin = reinterpret_cast<const KK *>(keys) + lo;
        kout = reinterpret_cast<KK *>(out) + lo;
        vi = vin ? vin + lo : nullptr;
        vo = vout ? vout + lo : nullptr;
    }
};

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
    // one 8-bit pass per byte of the largest bucket index
    L.scatter_passes = 1;
    while (L.scatter_passes < 4 && ((uint64_t)(L.buckets - 1) >> (8 * L.scatter_passes)) != 0) L.scatter_passes++;
    const uint64_t tile = key_bytes == 4 ? scatter_tile<uint32_t>(L.bits) : scatter_tile<uint64_t>(L.bits);
    L.num_tiles = (n + tile - 1) / tile;
    const uint64_t radix = 1ull << L.bits;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes, 256); return at; };
    L.counters = take((size_t)CTR_WORDS * 4);
    L.plan = take((size_t)(MAX_PASSES + 1) * PLAN_WORDS * 4);
    L.minmax = take(40);   // min, max, whether the keys are already sorted, the per-bucket stage,
                           // whether a key lies above a declared range
    L.counts = take(L.buckets <= BUCKET_LDS_HIST_MAX ? (size_t)L.buckets * 4 : 0);
    L.subhist = take((size_t)SUBHIST_WORDS * 4);
    L.excl = take((size_t)L.scatter_passes * radix * 4);
    L.offsets = take((size_t)(L.buckets + 1) * 8);
    L.runs = take(L.buckets > BUCKET_LDS_HIST_MAX ? (size_t)start_run_cap(L.buckets) * sizeof(StartRun) : 0);
    L.status0 = take((size_t)L.num_tiles * radix * 4);
    L.status1 = take((size_t)L.num_tiles * radix * 4);
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
    uint64_t *sorted = minmax + 2;
    uint64_t *bskip = minmax + 3;
    uint64_t *above = minmax + 4;
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
    hipError_t e = hipSuccess;
    // the keys' range and whether they are already in order, found by the
    // first kernel that reads every key (min/max, or with a declared range
    // the bucket histogram): then every later stage finds nothing to do and
    // the output is a copy of the input
    const bool bound = c.opts.key_bound != 0;
    if (bound) hipLaunchKernelGGL(k_set_range, dim3(1), dim3(1), 0, s, minmax, 0ull, c.opts.key_bound, sorted, above);
    else e = minmax_run((int)sizeof(K), c.keys_in, c.n, minmax, s, sorted);
    if (e != hipSuccess) return e;
    const uint64_t *hist_skip = bound ? nullptr : sorted;
    uint64_t *hist_order = bound ? sorted : nullptr;
    uint64_t *hist_above = bound ? above : nullptr;   // measured: no key lies above the maximum
    auto copy_if_sorted = [&]() {
        if (c.keys_in == c.keys_out && (!PAIRS || c.vals_in == c.vals_out)) return;
        const uint64_t blocks = std::min<uint64_t>((c.n + BK_THREADS - 1) / BK_THREADS, (uint64_t)fill_grid * 2);
        hipLaunchKernelGGL((k_copy_if_sorted<K>), dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(BK_THREADS), 0,
                           s, sorted, static_cast<const K *>(c.keys_in), static_cast<K *>(c.keys_out),
                           PAIRS ? c.vals_in : nullptr, PAIRS ? c.vals_out : nullptr, c.n);
    };
    if (tm) tm->mark(INTSORT_KERNEL_MINMAX, 0, s);
    const bool full_hist = B <= BUCKET_LDS_HIST_MAX;
    if (full_hist) {
        e = bucket_histogram_run_above((int)sizeof(K), c.keys_in, c.n, minmax, B, counts, s, hist_skip, hist_order,
                                       hist_above);
    } else {
        hipLaunchKernelGGL(k_fill<uint32_t>, dim3(4), dim3(256), 0, s, subhist, (uint64_t)SUBHIST_WORDS, 0u);
        uint64_t blocks = std::min<uint64_t>((c.n + BK_THREADS - 1) / BK_THREADS, (uint64_t)fill_grid * 2);
        const dim3 g((uint32_t)std::max<uint64_t>(blocks, 1)), t(BK_THREADS);
        if (hist_above)
            hipLaunchKernelGGL((k_bucket_subhist<K, true>), g, t, 0, s, static_cast<const K *>(c.keys_in), c.n, minmax,
                               B, L.scatter_passes, subhist, hist_skip, hist_order, hist_above);
        else
            hipLaunchKernelGGL((k_bucket_subhist<K, false>), g, t, 0, s, static_cast<const K *>(c.keys_in), c.n, minmax,
                               B, L.scatter_passes, subhist, hist_skip, hist_order, hist_above);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if (tm) tm->mark(INTSORT_KERNEL_BUCKET_HISTOGRAM, 0, s);
    // only the scatter-only form writes the caller's output (the full sort
    // scatters into its own buffers)
    const bool alias = c.keys_in == c.keys_out || (PAIRS && c.vals_in == c.vals_out);
    BucketPlanArgs pa{counts, subhist, excl, offsets, plan, B, (uint32_t)C::RADIX, L.scatter_passes,
                      full_hist ? 1u : 0u, c.n, sorted, scatter_only && alias ? 1u : 0u, minmax, bskip,
                      bound ? above : nullptr};
    hipLaunchKernelGGL(k_bucket_plan, dim3(1), dim3(BK_THREADS), 0, s, pa);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(fill_grid), dim3(256), 0, s, status0,
                       (uint64_t)L.num_tiles * C::RADIX, 0u);
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
    if (scatter_only) {
        // in place, an odd number of passes leaves the scatter in scratch
        const uint64_t blocks = std::min<uint64_t>((c.n + 255) / 256, (uint64_t)fill_grid);
        hipLaunchKernelGGL((k_plan_final_copy<K, PAIRS>), dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(256), 0,
                           s, a.in, a.out, a.tmp, a.vin, a.vout, a.vtmp, plan + MAX_PASSES * PLAN_WORDS, (uint32_t)c.n);
        copy_if_sorted();
        return hipGetLastError();
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;

    if (!full_hist) {
        StartRun *runs = reinterpret_cast<StartRun *>(ws + L.runs);
        const uint64_t cap = start_run_cap(B);
        const uint64_t per_block = (uint64_t)BK_THREADS * BS_V;
        uint64_t blocks = std::min<uint64_t>((c.n + 1 + per_block - 1) / per_block, (uint64_t)fill_grid * 2);
        hipLaunchKernelGGL((k_bucket_starts<K>), dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(BK_THREADS), 0,
                           s, tmpb, c.n, minmax, B, offsets, runs, counters, cap, (const uint64_t *)bskip);
        hipLaunchKernelGGL(k_bucket_start_runs, dim3((uint32_t)std::min<uint64_t>(cap, (uint64_t)fill_grid * 4)),
                           dim3(BK_THREADS), 0, s, runs, counters, cap, offsets, (const uint64_t *)bskip);
        if (tm) tm->mark(INTSORT_KERNEL_PLAN, 1, s);
    }

    // every bucket sorted on its own.  With many tiny buckets (fewer than
    // WINDOW_AVG keys each on average) the small ones go in windows of whole
    // consecutive buckets, one workgroup in LDS each, and only the rest are
    // segments; otherwise every bucket is a segment of its own size class.
    using CL = SegClasses<K>;
    constexpr uint32_t HALF = CL::LDS_MAX / 2;
    const bool windows = c.n < (uint64_t)B * WINDOW_AVG;
    if (windows) {
        LdsSortArgs<WindowSrc<K>> la{};
        la.src = WindowSrc<K>{tmpb, static_cast<K *>(c.keys_out), PAIRS ? tmpb_v : nullptr,
                              PAIRS ? c.vals_out : nullptr, offsets, minmax, B, HALF, c.n, bskip};
        la.list = nullptr;
        la.direct_count = (uint32_t)((c.n + HALF - 1) / HALF);
        hipLaunchKernelGGL((k_lds_sort<K, PAIRS, 512, CL::LDS_MAX / 512, WindowSrc<K>>), dim3(la.direct_count),
                           dim3(512), 0, s, la);
        if (tm) tm->mark(INTSORT_KERNEL_SEGMENT_SORT, 1, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
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
    sc.opts.flags &= ~INTSORT_FLAG_CHECK_SEGMENTS;   // the bucket starts are computed here, not given
    sc.L = L.S;
    sc.ws = segws;
    sc.timer = tm;
    sc.min_size = windows ? HALF : 0u;   // the windows took these
    sc.skip = bskip;
    if ((e = segmented_sort_run(sc, s)) != hipSuccess) return e;
    {
        const uint64_t blocks = std::min<uint64_t>((c.n + BK_THREADS - 1) / BK_THREADS, (uint64_t)fill_grid * 2);
        hipLaunchKernelGGL((k_copy_if_single<K>), dim3((uint32_t)std::max<uint64_t>(blocks, 1)), dim3(BK_THREADS), 0,
                           s, (const uint64_t *)bskip, (const K *)tmpb, static_cast<K *>(c.keys_out),
                           PAIRS ? (const uint32_t *)tmpb_v : nullptr, PAIRS ? c.vals_out : nullptr, c.n);
    }
    copy_if_sorted();
    return hipGetLastError();
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
