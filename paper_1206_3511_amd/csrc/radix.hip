// radix.hip -- LSD radix sort for gfx950 (MI355X).
//
// The method is RADIX-SORT (section 2.5, Algorithm 4): d passes, least
// significant r-bit digit first, each a stable sort of the whole array on one
// digit.  The paper's per-digit stable sort is COUNTING-SORT (section 2.4,
// Algorithm 3): count digit values, prefix-sum the counts, place every
// element at its digit's running offset.  Here that one-digit counting sort
// is split across the GPU as follows:
//
//   k_digit_histogram   the count loop of Algorithm 3 for ALL d digits in one
//                       read of the keys; its last workgroup turns the counts
//                       into exclusive prefix sums (where every digit's run
//                       starts in the output) and plans the passes.
//   k_onesweep (x d)    one pass = placement loop of Algorithm 3.  The array is
//                       cut into tiles; a tile ranks its keys stably inside
//                       LDS, publishes its per-digit counts, and obtains the
//                       counts of all earlier tiles through a decoupled
//                       look-back over per-(tile, digit) status words (a
//                       chained scan across tiles).  Keys then go through LDS
//                       in digit order so that global stores are contiguous.
//   k_final_copy        moves the result into the output buffer when the pass
//                       count left it in the scratch buffer.
//
// Placement is forward with exclusive offsets instead of Algorithm 3's
// backward walk with inclusive offsets; both give the same stable order.
// A pass whose digit has a single value over the whole input (its count is n)
// is the identity permutation and is skipped on the device unless the caller
// disables skipping; the output does not change.

#include <stdint.h>

#include "device_common.hpp"
#include "intsort.h"
#include "internal.hpp"

namespace intsort {

template <typename K>
__device__ __forceinline__ uint32_t digit_at(K k, uint32_t shift, uint32_t mask)
{
    return (uint32_t)(k >> shift) & mask;
}

// tile shape of the pass kernel for a key type and digit width
template <typename K, int BITS>
struct PassCfg {
    static constexpr int WAVES = (BITS > 8) ? 4 : 8;
    // keys per thread: large tiles keep the number of tiles, and with it the
    // look-back traffic between them, small
    static constexpr int IPT = sizeof(K) == 4 ? (BITS > 8 ? 16 : 32) : 16;
    static constexpr int NT = WAVES * WAVE;
    static constexpr int TILE = NT * IPT;
    static constexpr int RADIX = 1 << BITS;
    static constexpr int PASSES = (8 * (int)sizeof(K) + BITS - 1) / BITS;
};

constexpr int HIST_THREADS = 256;
#ifndef HIST_UNROLL
#define HIST_UNROLL 4
#endif
#ifndef HIST_BLOCKS_PER_CU
#define HIST_BLOCKS_PER_CU 4
#endif
#ifndef HIST_COPIES
#define HIST_COPIES 4
#endif
constexpr uint32_t LOOKBACK_SPIN_LIMIT = 1u << 20;
#ifndef LOOKBACK_WINDOW
#define LOOKBACK_WINDOW 4
#endif
#ifndef LOOKBACK_SPAN
#define LOOKBACK_SPAN 32
#endif

// ------------------------------------------------------------------ init

__global__ __launch_bounds__(256) void k_init(uint32_t *__restrict__ counters,
                                              uint32_t *__restrict__ hist, uint32_t hist_words)
{
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < (uint32_t)CTR_WORDS; i += blockDim.x) counters[i] = 0;
    for (uint32_t i = g; i < hist_words; i += gridDim.x * blockDim.x) hist[i] = 0;
}

// ------------------------------------------------------------- histogram

struct HistArgs {
    uint32_t *hist;        // [passes][radix], zero on entry
    uint32_t *excl;        // [passes][radix], written by the last workgroup
    uint32_t *plan;        // [(MAX_PASSES + 1) * PLAN_WORDS]
    uint32_t *counters;
    uint32_t *status0;     // look-back words of the first active pass, cleared here
    uint64_t status0_words;
    uint32_t n;
    uint32_t max_passes;   // passes allowed to run (<= passes)
    uint32_t skip;         // skip passes whose digit is constant
    uint32_t in_place;     // keys_in == keys_out
    uint32_t finalize;     // 0: only count (step-level entry point), no plan
    uint32_t copies;       // histogram copies the workgroups spread their adds over
};

// add one key's digit for pass p to the LDS histogram; a wave whose lanes all
// hold the same digit adds once instead of colliding 64 times on one word
template <int RADIX>
__device__ __forceinline__ void hist_add(uint32_t *s_h, uint32_t d)
{
    const uint32_t d0 = first_lane_value(d);
    const uint64_t act = ballot(true);
    if (ballot(d != d0) == 0) {
        if (mbcnt(act) == 0) atomicAdd(&s_h[d0], popc64(act));
    } else {
        atomicAdd(&s_h[d], 1u);
    }
}

template <typename K, int BITS>
__global__ __launch_bounds__(HIST_THREADS) void k_digit_histogram(const K *__restrict__ keys, HistArgs a)
{
    constexpr int RADIX = 1 << BITS;
    constexpr int PASSES = PassCfg<K, BITS>::PASSES;
    constexpr uint32_t MASK = RADIX - 1;
    constexpr int KPV = 16 / (int)sizeof(K);
    struct alignas(16) Vec { K v[KPV]; };

    __shared__ uint32_t s_h[PASSES * RADIX];

    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (uint32_t)(PASSES * RADIX); i += HIST_THREADS) s_h[i] = 0;
    {
        const uint64_t stride = (uint64_t)gridDim.x * HIST_THREADS;
        for (uint64_t i = (uint64_t)blockIdx.x * HIST_THREADS + tid; i < a.status0_words; i += stride)
            a.status0[i] = 0;
    }
    __syncthreads();

    const uint32_t n = a.n;
    const uint32_t nvec = n / KPV;
    const Vec *vk = reinterpret_cast<const Vec *>(keys);
    // HIST_UNROLL vector loads in flight per thread before any counting
    const uint32_t step = gridDim.x * HIST_THREADS * HIST_UNROLL;
    for (uint32_t v0 = blockIdx.x * HIST_THREADS * HIST_UNROLL + tid; v0 < nvec; v0 += step) {
        Vec x[HIST_UNROLL];
#pragma unroll
        for (int u = 0; u < HIST_UNROLL; u++) {
            const uint32_t v = v0 + u * HIST_THREADS;
            if (v < nvec) x[u] = vk[v];
        }
#pragma unroll
        for (int u = 0; u < HIST_UNROLL; u++) {
            if (v0 + u * HIST_THREADS < nvec) {
#pragma unroll
                for (int e = 0; e < KPV; e++) {
#pragma unroll
                    for (int p = 0; p < PASSES; p++)
                        hist_add<RADIX>(s_h + p * RADIX, digit_at<K>(x[u].v[e], (uint32_t)(p * BITS), MASK));
                }
            }
        }
    }
    if (blockIdx.x == 0) {
        for (uint32_t i = nvec * KPV + tid; i < n; i += HIST_THREADS) {
            K k = keys[i];
#pragma unroll
            for (int p = 0; p < PASSES; p++)
                hist_add<RADIX>(s_h + p * RADIX, digit_at<K>(k, (uint32_t)(p * BITS), MASK));
        }
    }
    __syncthreads();
    // workgroups add into one of a.copies copies of the histogram, so that
    // fewer of them queue on the same device-wide address
    uint32_t *hdst = a.hist + (blockIdx.x % a.copies) * (uint32_t)(PASSES * RADIX);
    for (uint32_t i = tid; i < (uint32_t)(PASSES * RADIX); i += HIST_THREADS) {
        uint32_t c = s_h[i];
        if (c) atomicAdd(&hdst[i], c);
    }
}

// Turns the digit counts into exclusive offsets (where the run of every digit
// value starts in the output of its pass) and plans the passes: which run,
// which buffer each reads and writes.  One workgroup; runs after the
// histogram kernel, so every count is complete and visible.
template <typename K, int BITS>
__global__ __launch_bounds__(HIST_THREADS) void k_digit_plan(HistArgs a)
{
    constexpr int RADIX = 1 << BITS;
    constexpr int PASSES = PassCfg<K, BITS>::PASSES;
    constexpr int DPT = RADIX > HIST_THREADS ? RADIX / HIST_THREADS : 1;
    __shared__ uint32_t s_scan[HIST_THREADS / WAVE + 1];
    __shared__ uint32_t s_const[MAX_PASSES];
    const uint32_t tid = threadIdx.x;
    const uint32_t n = a.n;

    if (tid < (uint32_t)MAX_PASSES) s_const[tid] = 0;
    __syncthreads();
    for (int p = 0; p < PASSES; p++) {
        uint32_t c[DPT];
        uint32_t mine = 0;
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const uint32_t d = tid * DPT + i;
            c[i] = 0;
            if (d < (uint32_t)RADIX)
                for (uint32_t cp = 0; cp < a.copies; cp++)
                    c[i] += a.hist[cp * (uint32_t)(PASSES * RADIX) + p * RADIX + d];
            if (c[i] == n) s_const[p] = 1;
            mine += c[i];
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<HIST_THREADS>(mine, s_scan, &total);
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const uint32_t d = tid * DPT + i;
            if (d < (uint32_t)RADIX) a.excl[p * RADIX + d] = run;
            run += c[i];
        }
    }
    __syncthreads();
    if (tid == 0) {
        // which passes run, and which buffer each reads and writes: the last
        // active pass must land in the output buffer
        uint32_t act[MAX_PASSES];
        uint32_t A = 0;
        for (int p = 0; p < PASSES; p++) {
            act[p] = ((uint32_t)p < a.max_passes) && !(a.skip && s_const[p]);
            A += act[p];
        }
        uint32_t q = 0, prev_dst = BUF_IN;
        for (int p = 0; p < PASSES; p++) {
            uint32_t *w = a.plan + p * PLAN_WORDS;
            if (!act[p]) { w[0] = 0; w[1] = 0; w[2] = 0; w[3] = 0; continue; }
            uint32_t dst;
            if (a.in_place) dst = (q % 2 == 0) ? BUF_TMP : BUF_OUT;
            else dst = ((A - 1 - q) % 2 == 0) ? BUF_OUT : BUF_TMP;
            w[0] = 1; w[1] = prev_dst; w[2] = dst; w[3] = q;
            prev_dst = dst;
            q++;
        }
        uint32_t *f = a.plan + MAX_PASSES * PLAN_WORDS;
        if (A == 0) { f[0] = a.in_place ? 0u : 1u; f[1] = BUF_IN; f[2] = BUF_OUT; }
        else if (prev_dst == BUF_TMP) { f[0] = 1; f[1] = BUF_TMP; f[2] = BUF_OUT; }
        else { f[0] = 0; f[1] = 0; f[2] = 0; }
        f[3] = A;
    }
}

// ------------------------------------------------------------- one pass

template <typename K>
struct PassArgs {
    const K *in;
    K *out;
    K *tmp;
    const uint32_t *vin;
    uint32_t *vout;
    uint32_t *vtmp;
    const uint32_t *excl;   // this pass's exclusive digit offsets [radix]
    const uint32_t *plan;   // this pass's plan words
    uint32_t *status0;      // look-back words for even / odd active passes
    uint32_t *status1;
    uint32_t *counters;
    uint32_t n;
    uint32_t shift;
    uint32_t pass;
    uint32_t num_tiles;
};

// Sum of the counts of digit d in tiles 0 .. tile-1.
//
// Every tile publishes, per digit, an aggregate word (its own count) and
// later an inclusive word (count of all tiles up to and including it); after
// its inclusive words it also raises a per-tile flag.  The walk first reads
// the flags of the 64 previous tiles (one load per lane) to find the nearest
// tile that has finished, then fetches the status words of the whole span to
// it in one batch.  The flag is only a hint: the status words alone decide,
// and when the hint is missing, stale or too far away the walk falls back to
// reading LOOKBACK_WINDOW words per round trip: aggregates are added and the
// walk goes on, an inclusive word ends it, an unpublished word is polled
// again (bounded: on timeout an error bit is set).
template <int RADIX>
__device__ __forceinline__ uint32_t look_back(const uint32_t *status, const uint32_t *tflag, uint32_t tile,
                                              uint32_t d, uint32_t *err)
{
    constexpr int W = LOOKBACK_WINDOW;
    constexpr int SPAN = LOOKBACK_SPAN;
    uint32_t prefix = 0;
    int64_t t = (int64_t)tile - 1;
    {
        const int64_t q = (int64_t)tile - 1 - (int64_t)lane_id();
        const bool f = q >= 0 && load_agent(&tflag[q]) != 0u;
        const uint64_t m = ballot(f);
        if (m != 0) {
            // lanes read tiles tile-1, tile-2, ...: the lowest set lane is
            // the nearest finished tile
            const int span = __builtin_ctzll(m) + 1;   // words tile-1 down to that tile
            if (span <= SPAN) {
                uint32_t sw[SPAN];
#pragma unroll
                for (int k = 0; k < SPAN; k++)
                    sw[k] = k < span ? load_agent(&status[(uint64_t)(t - k) * RADIX + d]) : 0u;
                bool stop = false, done = false;
                int consumed = 0;
#pragma unroll
                for (int k = 0; k < SPAN; k++) {
                    if (!stop && k < span) {
                        const uint32_t fl = sw[k] >> FLAG_SHIFT;
                        if (fl == 0) {
                            stop = true;
                        } else {
                            prefix += sw[k] & COUNT_MASK;
                            consumed++;
                            if (fl & 2u) { stop = true; done = true; }
                        }
                    }
                }
                if (done) return prefix;
                t -= consumed;
            }
        }
    }
    uint32_t spins = 0;
    while (t >= 0) {
        uint32_t s[W];
#pragma unroll
        for (int w = 0; w < W; w++) {
            const int64_t tt = t - w;
            // below tile 0 reads as an empty inclusive word (tile 0 always
            // publishes an inclusive word, so a correct walk stops earlier)
            s[w] = tt >= 0 ? load_agent(&status[(uint64_t)tt * RADIX + d]) : FLAG_INC;
        }
        bool stop = false, done = false;
        int consumed = 0;
#pragma unroll
        for (int w = 0; w < W; w++) {
            if (!stop) {
                const uint32_t f = s[w] >> FLAG_SHIFT;
                if (f == 0) {
                    stop = true;
                } else {
                    prefix += s[w] & COUNT_MASK;
                    consumed++;
                    if (f & 2u) { stop = true; done = true; }
                }
            }
        }
        if (done) return prefix;
        t -= consumed;
        if (t < 0) break;
        if (consumed == 0) {
            if (++spins > LOOKBACK_SPIN_LIMIT) { atomicOr(err, DEVERR_LOOKBACK_TIMEOUT); return prefix; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    atomicOr(err, DEVERR_BAD_TILE);
    return prefix;
}

template <typename K, int BITS, bool PAIRS>
__global__ __launch_bounds__((PassCfg<K, BITS>::NT)) void k_onesweep(PassArgs<K> a)
{
    using C = PassCfg<K, BITS>;
    constexpr int RADIX = C::RADIX, NT = C::NT, WAVES = C::WAVES, IPT = C::IPT, TILE = C::TILE;
    constexpr uint32_t MASK = RADIX - 1;
    constexpr int BM = BITS > 8 ? 256 : RADIX;          // peer bitmap words per wave
    constexpr int DPT = RADIX > NT ? RADIX / NT : 1;    // digits per thread in digit phases
    static_assert(TILE * sizeof(K) >= WAVES * BM * sizeof(uint64_t), "bitmaps alias the stage");
    static_assert(RADIX <= NT * DPT, "digit phase covers every digit");

    __shared__ alignas(16) unsigned char s_raw[TILE * sizeof(K)];
    __shared__ uint32_t s_wcnt[WAVES * RADIX];
    __shared__ uint32_t s_tile_excl[RADIX];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_scan[NT / WAVE + 1];
    __shared__ uint32_t s_tile;
    K *s_stage = reinterpret_cast<K *>(s_raw);
    uint64_t *s_bits = reinterpret_cast<uint64_t *>(s_raw);

    if (a.plan[0] == 0) return;   // pass skipped: the same for every workgroup
    const uint32_t srcc = a.plan[1], dstc = a.plan[2], ord = a.plan[3];
    const K *src = srcc == BUF_IN ? a.in : (srcc == BUF_OUT ? a.out : a.tmp);
    K *dst = dstc == BUF_OUT ? a.out : a.tmp;
    const uint32_t *vsrc = nullptr;
    uint32_t *vdst = nullptr;
    if (PAIRS) {
        vsrc = srcc == BUF_IN ? a.vin : (srcc == BUF_OUT ? a.vout : a.vtmp);
        vdst = dstc == BUF_OUT ? a.vout : a.vtmp;
    }
    uint32_t *status = (ord & 1) ? a.status1 : a.status0;
    uint32_t *status_next = (ord & 1) ? a.status0 : a.status1;
    // per-tile "inclusive words published" flags follow each status array
    uint32_t *tflag = status + (uint64_t)a.num_tiles * RADIX;
    uint32_t *tflag_next = status_next + (uint64_t)a.num_tiles * RADIX;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = tid / WAVE;
    const uint32_t shift = a.shift;
    const uint32_t n = a.n;

    for (uint32_t i = tid; i < (uint32_t)(WAVES * RADIX); i += NT) s_wcnt[i] = 0;
    for (uint32_t i = tid; i < (uint32_t)(WAVES * BM); i += NT) s_bits[i] = 0;
    if (tid == 0) s_tile = atomicAdd(&a.counters[CTR_TILE + a.pass], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= a.num_tiles) {   // only if the counters were not reset: never index past the arrays
        if (tid == 0) atomicOr(&a.counters[CTR_ERROR], DEVERR_BAD_TILE);
        return;
    }
    const uint32_t base = tile * (uint32_t)TILE;
    const uint32_t valid = min((uint32_t)TILE, n - base);

    // ---- load: wave-striped, so (wave, item, lane) order is index order
    K k[IPT];
    uint32_t v[PAIRS ? IPT : 1];
    const uint32_t wofs = base + wave * (IPT * WAVE) + lane;
    if (valid == (uint32_t)TILE) {
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            k[j] = src[wofs + j * WAVE];
            if (PAIRS) v[j] = vsrc[wofs + j * WAVE];
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            const uint32_t idx = wofs + j * WAVE;
            // keys past the end take the largest digit, so they rank last
            k[j] = idx < n ? src[idx] : ~K(0);
            if (PAIRS) v[j] = idx < n ? vsrc[idx] : 0u;
        }
    }

    // ---- stable rank inside the wave: peers with the same digit come from a
    // per-wave LDS bitmap that every lane ORs its bit into
    uint32_t rk[IPT];
    uint32_t *wcnt = s_wcnt + wave * RADIX;
    uint64_t *bits = s_bits + wave * BM;
    const uint64_t lanebit = 1ull << lane;
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const uint32_t d = digit_at<K>(k[j], shift, MASK);
        const uint32_t d0 = first_lane_value(d);
        if (ballot(d != d0) == 0) {
            const uint32_t c = wcnt[d0];
            rk[j] = c + lane;
            wave_sync();
            if (lane == 0) wcnt[d0] = c + WAVE;
            wave_sync();
        } else {
            const uint32_t h = BITS > 8 ? (d & 255u) : d;
            atomicOr(reinterpret_cast<unsigned long long *>(&bits[h]), (unsigned long long)lanebit);
            wave_sync();
            uint64_t peers = __hip_atomic_load(&bits[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            if (BITS > 8) {
#pragma unroll
                for (int b = 8; b < BITS; b++) {
                    const bool on = (d >> b) & 1u;
                    const uint64_t bb = ballot(on);
                    peers &= on ? bb : ~bb;
                }
            }
            const uint32_t below = mbcnt(peers);
            const uint32_t c = wcnt[d];
            rk[j] = c + below;
            wave_sync();
            if (below == 0) {
                wcnt[d] = c + popc64(peers);
                __hip_atomic_store(&bits[h], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
            wave_sync();
        }
    }
    __syncthreads();

    // ---- per digit: offsets of every wave inside the tile and the tile's
    // count, published at once so that later tiles can look back over it
    uint32_t tcnt[DPT];
    uint32_t mine = 0;
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t d = tid * DPT + i;
        tcnt[i] = 0;
        if (d < (uint32_t)RADIX) {
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < WAVES; w++) {
                const uint32_t c = s_wcnt[w * RADIX + d];
                s_wcnt[w * RADIX + d] = run;
                run += c;
            }
            tcnt[i] = run;
            store_agent(&status[(uint64_t)tile * RADIX + d], (tile == 0 ? FLAG_INC : FLAG_AGG) | run);
        }
        mine += tcnt[i];
    }
    uint32_t total_unused;
    uint32_t texcl[DPT];
    texcl[0] = block_exclusive_scan<NT>(mine, s_scan, &total_unused);
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t d = tid * DPT + i;
        if (i > 0) texcl[i] = texcl[i - 1] + tcnt[i - 1];
        if (d < (uint32_t)RADIX) s_tile_excl[d] = texcl[i];
    }
    __syncthreads();

    // ---- reorder the tile through LDS into digit order; this needs only
    // tile-local offsets, so it runs before the look-back
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const uint32_t d = digit_at<K>(k[j], shift, MASK);
        rk[j] += s_tile_excl[d] + s_wcnt[wave * RADIX + d];
        s_stage[rk[j]] = k[j];
    }

    // ---- look-back: the counts of this digit in all earlier tiles
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t d = tid * DPT + i;
        if (d < (uint32_t)RADIX) {
            uint32_t prefix = 0;
            if (tile > 0) {
                prefix = look_back<RADIX>(status, tflag, tile, d, &a.counters[CTR_ERROR]);
                store_agent(&status[(uint64_t)tile * RADIX + d], FLAG_INC | (prefix + tcnt[i]));
            }
            s_gbase[d] = a.excl[d] + prefix - texcl[i];
            store_agent(&status_next[(uint64_t)tile * RADIX + d], 0u);
        }
    }
    __syncthreads();
    if (tid == 0) {
        store_agent(&tflag[tile], 1u);
        store_agent(&tflag_next[tile], 0u);
    }

    // ---- contiguous runs of each digit go to their global offsets
    uint32_t dest[PAIRS ? IPT : 1];
    bool bad = false;
#pragma unroll
    for (int m = 0; m < IPT; m++) {
        const uint32_t i = m * NT + tid;
        if (PAIRS) dest[m] = n;
        if (i < valid) {
            const K key = s_stage[i];
            const uint32_t g = s_gbase[digit_at<K>(key, shift, MASK)] + i;
            if (g < n) {
                dst[g] = key;
                if (PAIRS) dest[m] = g;
            } else {
                bad = true;
            }
        }
    }
    if (bad) atomicOr(&a.counters[CTR_ERROR], DEVERR_SCATTER_RANGE);
    if (PAIRS) {
        uint32_t *s_v = reinterpret_cast<uint32_t *>(s_raw);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++) s_v[rk[j]] = v[j];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < IPT; m++) {
            const uint32_t i = m * NT + tid;
            if (i < valid && dest[m] < n) vdst[dest[m]] = s_v[i];
        }
    }
}

// ------------------------------------------------------------- final copy

template <typename K, bool PAIRS>
__global__ __launch_bounds__(256) void k_final_copy(const K *in, K *out, K *tmp, const uint32_t *vin,
                                                    uint32_t *vout, uint32_t *vtmp, const uint32_t *f,
                                                    uint32_t n)
{
    if (f[0] == 0) return;
    const K *src = f[1] == BUF_IN ? in : tmp;
    const uint32_t *vsrc = f[1] == BUF_IN ? vin : vtmp;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        out[i] = src[i];
        if (PAIRS) vout[i] = vsrc[i];
    }
}

// ------------------------------------------------------------------ host

template <typename K, int BITS>
static RadixGeom geom_of()
{
    using C = PassCfg<K, BITS>;
    return RadixGeom{BITS, C::RADIX, C::PASSES, C::NT, C::TILE};
}

RadixGeom radix_geometry(int key_bytes, int bits)
{
    if (key_bytes == 4) {
        if (bits == 4) return geom_of<uint32_t, 4>();
        if (bits == 11) return geom_of<uint32_t, 11>();
        return geom_of<uint32_t, 8>();
    }
    if (bits == 4) return geom_of<uint64_t, 4>();
    if (bits == 11) return geom_of<uint64_t, 11>();
    return geom_of<uint64_t, 8>();
}

RadixLayout radix_layout(int key_bytes, bool pairs, uint64_t n, int bits)
{
    RadixLayout L{};
    L.g = radix_geometry(key_bytes, bits);
    L.n = n;
    L.num_tiles = (n + L.g.tile - 1) / L.g.tile;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes, 256); return at; };
    L.counters = take((size_t)CTR_WORDS * 4);   // always first: fixed error-word offset
    L.tmp_keys = take(n * (size_t)key_bytes);
    L.tmp_vals = take(pairs ? n * 4 : 0);
    L.hist = take((size_t)HIST_COPIES * L.g.passes * L.g.radix * 4);
    L.excl = take((size_t)L.g.passes * L.g.radix * 4);
    L.plan = take((size_t)(MAX_PASSES + 1) * PLAN_WORDS * 4);
    L.status0 = take((size_t)L.num_tiles * (L.g.radix + 1) * 4);
    L.status1 = take((size_t)L.num_tiles * (L.g.radix + 1) * 4);
    L.total = off;
    return L;
}

static int g_cu_count[64];

int device_cu_count(int device)
{
    if (device < 0 || device >= 64) return 256;
    if (g_cu_count[device] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
            cus = 256;
        g_cu_count[device] = cus;
    }
    return g_cu_count[device];
}

static int current_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    return device_cu_count(dev);
}

template <typename K, int BITS>
static hipError_t launch_histogram(const RadixCall &c, uint32_t *hist, bool finalize, hipStream_t s)
{
    using C = PassCfg<K, BITS>;
    const RadixLayout &L = c.L;
    char *ws = c.ws;
    uint32_t *counters = reinterpret_cast<uint32_t *>(ws + L.counters);
    Timer *t = c.timer;
    if (t) t->start(s);
    const uint32_t copies = finalize ? (uint32_t)HIST_COPIES : 1u;
    const uint32_t hist_words = copies * (uint32_t)(C::PASSES * C::RADIX);
    hipLaunchKernelGGL(k_init, dim3((hist_words + 255) / 256), dim3(256), 0, s, counters, hist, hist_words);
    if (t) t->mark(INTSORT_KERNEL_INIT, 0, s);
    HistArgs h{};
    h.hist = hist;
    h.excl = reinterpret_cast<uint32_t *>(ws + L.excl);
    h.plan = reinterpret_cast<uint32_t *>(ws + L.plan);
    h.counters = counters;
    h.status0 = finalize ? reinterpret_cast<uint32_t *>(ws + L.status0) : nullptr;
    h.status0_words = finalize ? L.num_tiles * (uint64_t)(C::RADIX + 1) : 0;
    h.n = (uint32_t)c.n;
    h.max_passes = (uint32_t)c.max_passes;
    h.skip = c.skip_constant_digits ? 1u : 0u;
    h.in_place = c.keys_in == c.keys_out ? 1u : 0u;
    h.finalize = finalize ? 1u : 0u;
    h.copies = copies;
    const uint64_t nvec = c.n / (16 / sizeof(K));
    uint64_t blocks = (nvec + HIST_THREADS * HIST_UNROLL - 1) / (HIST_THREADS * HIST_UNROLL);
    const uint64_t cap = (uint64_t)current_cus() * HIST_BLOCKS_PER_CU;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL((k_digit_histogram<K, BITS>), dim3((uint32_t)blocks), dim3(HIST_THREADS), 0, s,
                       static_cast<const K *>(c.keys_in), h);
    if (t) t->mark(INTSORT_KERNEL_DIGIT_HISTOGRAM, 0, s);
    if (finalize) {
        hipLaunchKernelGGL((k_digit_plan<K, BITS>), dim3(1), dim3(HIST_THREADS), 0, s, h);
        if (t) t->mark(INTSORT_KERNEL_PLAN, 0, s);
    }
    return hipGetLastError();
}

template <typename K, int BITS, bool PAIRS>
static hipError_t run_typed(const RadixCall &c, hipStream_t s)
{
    using C = PassCfg<K, BITS>;
    const RadixLayout &L = c.L;
    char *ws = c.ws;
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    hipError_t e = launch_histogram<K, BITS>(c, hist, true, s);
    if (e != hipSuccess) return e;

    PassArgs<K> a{};
    a.in = static_cast<const K *>(c.keys_in);
    a.out = static_cast<K *>(c.keys_out);
    a.tmp = reinterpret_cast<K *>(ws + L.tmp_keys);
    a.vin = c.vals_in;
    a.vout = c.vals_out;
    a.vtmp = reinterpret_cast<uint32_t *>(ws + L.tmp_vals);
    a.status0 = reinterpret_cast<uint32_t *>(ws + L.status0);
    a.status1 = reinterpret_cast<uint32_t *>(ws + L.status1);
    a.counters = reinterpret_cast<uint32_t *>(ws + L.counters);
    a.n = (uint32_t)c.n;
    a.num_tiles = (uint32_t)L.num_tiles;
    const uint32_t *excl = reinterpret_cast<const uint32_t *>(ws + L.excl);
    const uint32_t *plan = reinterpret_cast<const uint32_t *>(ws + L.plan);
    for (int p = 0; p < C::PASSES && p < c.max_passes; p++) {
        a.excl = excl + p * C::RADIX;
        a.plan = plan + p * PLAN_WORDS;
        a.shift = (uint32_t)(p * BITS);
        a.pass = (uint32_t)p;
        hipLaunchKernelGGL((k_onesweep<K, BITS, PAIRS>), dim3((uint32_t)L.num_tiles), dim3(C::NT), 0, s, a);
        if (c.timer) c.timer->mark(INTSORT_KERNEL_PASS, (uint32_t)p, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    uint64_t blocks = (c.n + 255) / 256;
    const uint64_t cap = (uint64_t)current_cus() * 4;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL((k_final_copy<K, PAIRS>), dim3((uint32_t)blocks), dim3(256), 0, s, a.in, a.out, a.tmp,
                       a.vin, a.vout, a.vtmp, plan + MAX_PASSES * PLAN_WORDS, (uint32_t)c.n);
    if (c.timer) c.timer->mark(INTSORT_KERNEL_COPY, 0, s);
    return hipGetLastError();
}

template <typename K, bool PAIRS>
static hipError_t run_bits(const RadixCall &c, hipStream_t s)
{
    switch (c.bits) {
    case 4: return run_typed<K, 4, PAIRS>(c, s);
    case 11: return run_typed<K, 11, PAIRS>(c, s);
    default: return run_typed<K, 8, PAIRS>(c, s);
    }
}

hipError_t radix_sort_run(const RadixCall &c, hipStream_t s)
{
    if (c.key_bytes == 4) return c.pairs ? run_bits<uint32_t, true>(c, s) : run_bits<uint32_t, false>(c, s);
    return c.pairs ? run_bits<uint64_t, true>(c, s) : run_bits<uint64_t, false>(c, s);
}

hipError_t digit_histogram_run(const RadixCall &c, uint32_t *counts, hipStream_t s)
{
    if (c.key_bytes == 4) {
        switch (c.bits) {
        case 4: return launch_histogram<uint32_t, 4>(c, counts, false, s);
        case 11: return launch_histogram<uint32_t, 11>(c, counts, false, s);
        default: return launch_histogram<uint32_t, 8>(c, counts, false, s);
        }
    }
    switch (c.bits) {
    case 4: return launch_histogram<uint64_t, 4>(c, counts, false, s);
    case 11: return launch_histogram<uint64_t, 11>(c, counts, false, s);
    default: return launch_histogram<uint64_t, 8>(c, counts, false, s);
    }
}

}  // namespace intsort
