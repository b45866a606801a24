// onesweep.hpp -- one stable counting-sort pass over tiles of keys, shared by
// the radix sort, the bucket scatter of bucket sort and the large segments of
// the segmented sort.
//
// A pass places every key at (start of its digit's run) + (number of keys
// with the same digit before it): the placement loop of COUNTING-SORT
// (section 2.4, Algorithm 3), done for all tiles of the input at once.  Each
// workgroup takes the next tile, ranks its keys stably in LDS, publishes its
// per-digit counts, learns the counts of all earlier tiles of its segment by
// a decoupled look-back over per-(tile, digit) status words, reorders the
// tile in LDS into digit order and writes every digit's run contiguously.
//
// Two policies make the kernel serve several callers:
//   Digit  maps a key to its digit: an r-bit field of the key (radix sort)
//          or an 8-bit field of the exact bucket index (bucket sort).
//   Tiles  maps a tile id to its keys and to the global start of every digit
//          run: one array cut into equal tiles, or a list of tiles of many
//          independent segments (a look-back never leaves its segment).
#pragma once

#include <stdint.h>

#include <type_traits>

#include "bucket_map.hpp"
#include "device_common.hpp"
#include "internal.hpp"

namespace intsort {

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

constexpr uint32_t LOOKBACK_SPIN_LIMIT = 1u << 20;
// status words a look-back reads per round trip: a walk is bound by the
// round trips, and wider windows made each round trip slower (measured with
// 4, 8, 16 and 32 on 10^8 keys)
#ifndef LOOKBACK_WINDOW
#define LOOKBACK_WINDOW 4
#endif

// ---------------------------------------------------------------- digits

template <typename K>
__device__ __forceinline__ uint32_t digit_at(K k, uint32_t shift, uint32_t mask)
{
    return (uint32_t)(k >> shift) & mask;
}

// Order of the keys' bit patterns: 0 unsigned; 1 two's-complement signed;
// 2 IEEE 754 totalOrder (binary32/binary64: -NaN < -inf < ... < -0 < +0 <
// ... < +inf < +NaN).  ordered(k) maps a key to an unsigned value with the
// same order: signed keys flip the sign bit, floats flip the sign bit of a
// positive value and every bit of a negative one.
template <int ORDER>
struct KeyOrder {
    template <typename K>
    __device__ __forceinline__ static K ordered(K k)
    {
        constexpr int TOP = 8 * (int)sizeof(K) - 1;
        constexpr K SIGN = K(1) << TOP;
        if (ORDER == 1) return k ^ SIGN;
        if (ORDER == 2) {
            using S = std::make_signed_t<K>;
            return k ^ ((K)((S)k >> TOP) | SIGN);
        }
        return k;
    }
    // the key whose ordered value is all ones: it sorts after every key
    template <typename K>
    __device__ __forceinline__ static K largest()
    {
        return ORDER == 0 ? ~K(0) : (K)(~K(0) >> 1);
    }
};

// digit p of radix sort: (ordered(k) >> p*r) & (2^r - 1)
template <int ORDER>
struct OrderedDigit {
    // padding past a tile's end is the largest key, whose digit is the
    // largest: it needs no separate check
    static constexpr bool PAD_IS_MAX = true;
    uint32_t shift, mask;
    __device__ OrderedDigit prepare() const { return *this; }
    template <typename K>
    __device__ __forceinline__ uint32_t operator()(K k) const
    {
        // 32-bit keys: one bit-field extract (mask + 1 is a power of two)
        if constexpr (sizeof(K) == 4)
            return __builtin_amdgcn_ubfe((uint32_t)KeyOrder<ORDER>::ordered(k), shift, __popc(mask));
        return digit_at<K>(KeyOrder<ORDER>::ordered(k), shift, mask);
    }
    // bits lo .. lo+w-1 of the digit
    template <typename K>
    __device__ __forceinline__ uint32_t sub(K k, uint32_t lo, uint32_t w) const
    {
        return (uint32_t)(KeyOrder<ORDER>::ordered(k) >> (shift + lo)) & ((1u << w) - 1u);
    }
    template <typename K>
    __device__ __forceinline__ K pad() const { return KeyOrder<ORDER>::template largest<K>(); }
};
using RadixDigit = OrderedDigit<0>;

// an 8-bit field of the bucket index b(k) of bucket sort; min and max are
// read from device memory when the kernel starts
struct BucketDigitArgs {
    const uint64_t *minmax;
    uint32_t buckets, shift, mask;
    struct Fn {
        static constexpr bool PAD_IS_MAX = false;
        BucketMap m;
        uint32_t shift, mask;
        template <typename K>
        __device__ __forceinline__ uint32_t operator()(K k) const { return (bucket_of(m, k) >> shift) & mask; }
        // padding past a tile's end: any key; its digit is replaced by the largest
        template <typename K>
        __device__ __forceinline__ K pad() const { return ~K(0); }
    };
    __device__ Fn prepare() const { return Fn{make_bucket_map(minmax[0], minmax[1], buckets), shift, mask}; }
};

// ---------------------------------------------------------------- tiles

struct TileInfo {
    uint32_t start;       // index of the tile's first key
    uint32_t count;       // keys in the tile (<= TILE)
    uint32_t first_tile;  // id of the first tile of the tile's segment
    uint32_t base;        // index of the segment's first key
    const uint32_t *excl; // exclusive digit offsets inside the segment
    const uint32_t *excl2; // offsets added to excl when not null
    const void *in;       // the three key buffers the indices refer to
    void *out;
    void *tmp;
    uint32_t limit;       // every store index stays below this
    uint32_t slot;        // segment row (segmented tiles only)
};

// one array of n keys in tiles of TILE keys
struct PlainTiles {
    uint32_t n, num_tiles;
    const uint32_t *excl;   // [radix] exclusive digit offsets of this pass
    template <int TILE>
    __device__ __forceinline__ bool get(uint32_t t, TileInfo &ti) const
    {
        if (t >= num_tiles) return false;
        ti.start = t * (uint32_t)TILE;
        ti.count = min((uint32_t)TILE, n - ti.start);
        ti.first_tile = 0;
        ti.base = 0;
        ti.excl = excl;
        return true;
    }
    // every tile runs the pass with the buffers of the pass's plan
    __device__ bool route(const TileInfo &, uint32_t, uint32_t &, uint32_t &) const { return true; }
    __device__ bool missing_is_error() const { return true; }
    __device__ uint32_t listed() const { return num_tiles; }
};

// tiles of one array whose digit offsets were found before the pass: the
// histogram kernel counted every tile's digits and a scan over the tiles
// turned the counts into offsets, so no tile looks back (each one is the
// first of its own run of tiles)
struct ScannedTiles {
    uint32_t n, num_tiles;
    const uint32_t *offs;        // [tile][radix]: the tile's digit offsets inside its chunk
    const uint32_t *chunk_offs;  // [chunk][radix]: where each chunk's run of each digit starts
    uint32_t radix;
    uint32_t tiles_per_chunk;
    template <int TILE>
    __device__ __forceinline__ bool get(uint32_t t, TileInfo &ti) const
    {
        if (t >= num_tiles) return false;
        ti.start = t * (uint32_t)TILE;
        ti.count = min((uint32_t)TILE, n - ti.start);
        ti.first_tile = t;
        ti.base = 0;
        ti.excl = offs + (uint64_t)t * radix;
        ti.excl2 = chunk_offs + (uint64_t)(t / tiles_per_chunk) * radix;
        return true;
    }
    __device__ bool route(const TileInfo &, uint32_t, uint32_t &, uint32_t &) const { return true; }
    __device__ bool missing_is_error() const { return true; }
    __device__ uint32_t listed() const { return num_tiles; }
};

// tiles of many segments, listed on the device; the tiles of one segment
// have consecutive ids
struct TileDesc {
    uint32_t slot;        // row of the segment in seg_excl
    uint32_t first_tile;
    uint32_t start;
    uint32_t count;
    uint32_t base;
    uint32_t pad[3];
};

// Which buffers an active pass of one segment reads and writes, when the
// segment runs only the passes in `mask` (the others have a constant digit
// inside it): the last active pass lands in the output, or, in place, the
// passes alternate scratch / output starting with the scratch.
__device__ __forceinline__ void segment_route(uint32_t mask, uint32_t pass, bool in_place, uint32_t &srcc,
                                              uint32_t &dstc)
{
    const uint32_t A = (uint32_t)__popc(mask);
    auto dst_of = [&](uint32_t q) -> uint32_t {
        if (in_place) return (q % 2 == 0) ? BUF_TMP : BUF_OUT;
        return ((A - 1 - q) % 2 == 0) ? BUF_OUT : BUF_TMP;
    };
    const uint32_t q = (uint32_t)__popc(mask & ((1u << pass) - 1u));
    srcc = q == 0 ? BUF_IN : dst_of(q - 1);
    dstc = dst_of(q);
}

// where a segment's keys are after its active passes
__device__ __forceinline__ uint32_t segment_result(uint32_t mask, bool in_place)
{
    const uint32_t A = (uint32_t)__popc(mask);
    if (A == 0) return BUF_IN;
    if (in_place) return ((A - 1) % 2 == 0) ? BUF_TMP : BUF_OUT;
    return BUF_OUT;
}

struct SegTiles {
    const TileDesc *desc;
    const uint32_t *num_tiles;   // device count of listed tiles
    const uint32_t *seg_excl;    // [slot][radix] for this pass
    uint32_t radix;
    const uint32_t *slot_mask;   // [slot] passes the segment runs
    uint32_t in_place;
    template <int TILE>
    __device__ __forceinline__ bool get(uint32_t t, TileInfo &ti) const
    {
        if (t >= *num_tiles) return false;
        const TileDesc d = desc[t];
        ti.start = d.start;
        ti.count = d.count;
        ti.first_tile = d.first_tile;
        ti.base = d.base;
        ti.excl = seg_excl + (uint64_t)d.slot * radix;
        ti.slot = d.slot;
        return true;
    }
    __device__ bool route(const TileInfo &ti, uint32_t pass, uint32_t &srcc, uint32_t &dstc) const
    {
        const uint32_t mask = slot_mask[ti.slot];
        if (!((mask >> pass) & 1u)) return false;
        segment_route(mask, pass, in_place != 0, srcc, dstc);
        return true;
    }
    __device__ bool missing_is_error() const { return false; }
    __device__ uint32_t listed() const { return *num_tiles; }
};

// key buffers of one segment of a batch of separate arrays
struct SegBuf {
    const void *in;
    void *out;
    void *tmp;
    uint64_t n;
};

// tiles of a batch of separate arrays: indices are local to each array and
// every array brings its own input, output and scratch buffers
struct DescTiles {
    const TileDesc *desc;
    const uint32_t *num_tiles;
    const uint32_t *seg_excl;
    uint32_t radix;
    const uint32_t *slot_mask;
    uint32_t in_place;        // unused: each array says for itself
    const SegBuf *bufs;       // [slot]
    template <int TILE>
    __device__ __forceinline__ bool get(uint32_t t, TileInfo &ti) const
    {
        if (t >= *num_tiles) return false;
        const TileDesc d = desc[t];
        const SegBuf b = bufs[d.slot];
        ti.start = d.start;
        ti.count = d.count;
        ti.first_tile = d.first_tile;
        ti.base = d.base;
        ti.excl = seg_excl + (uint64_t)d.slot * radix;
        ti.in = b.in;
        ti.out = b.out;
        ti.tmp = b.tmp;
        ti.limit = (uint32_t)b.n;
        ti.slot = d.slot;
        return true;
    }
    __device__ bool route(const TileInfo &ti, uint32_t pass, uint32_t &srcc, uint32_t &dstc) const
    {
        const uint32_t mask = slot_mask[ti.slot];
        if (!((mask >> pass) & 1u)) return false;
        segment_route(mask, pass, ti.in == ti.out, srcc, dstc);
        return true;
    }
    __device__ bool missing_is_error() const { return false; }
    __device__ uint32_t listed() const { return *num_tiles; }
};

// ---------------------------------------------------------------- ranking

// Stable rank of one slot of a wave (64 keys, one per lane, in lane order)
// among the keys the wave has ranked so far, by one LDS atomic add per key on
// the wave's counter of the key's digit: the lanes of one add instruction
// that hit the same counter are served in lane order (intsort_create checks
// this on its device), so the old value an add returns counts the same-digit
// keys of the earlier slots plus the lanes below with the same digit.  A
// slot whose lanes all hold one digit adds once for all of them (adds on one
// word from many lanes are served one after another).
__device__ __forceinline__ uint32_t wave_rank_atomic(uint32_t d, uint32_t *wcnt)
{
    const uint32_t d0 = first_lane_value(d);
    const uint64_t act = ballot(true);
    if (ballot(d != d0) == 0) {
        const uint32_t below = mbcnt(act);
        uint32_t c = 0;
        if (below == 0) c = atomicAdd(&wcnt[d0], popc64(act));
        return first_lane_value(c) + below;
    }
    return atomicAdd(&wcnt[d], 1u);
}

// ---------------------------------------------------------------- look-back

// Sum of the counts of digit d in tiles first_tile .. tile-1 of one segment.
//
// Every tile publishes, per digit, an aggregate word (its own count) and
// later an inclusive word (count of all tiles of its segment up to and
// including it; the first tile of a segment publishes its inclusive word at
// once).  The walk reads LOOKBACK_WINDOW words per round trip, nearest tile
// first: aggregates are added and the walk goes on, an inclusive word ends
// it, an unpublished word is polled again (bounded: on timeout an error bit
// is set).
template <int RADIX>
__device__ __forceinline__ uint32_t look_back(const uint32_t *status, uint32_t tile, uint32_t first_tile, uint32_t d,
                                              uint32_t *err)
{
    constexpr int W = LOOKBACK_WINDOW;
    uint32_t prefix = 0;
    int64_t t = (int64_t)tile - 1;
    const int64_t lo = first_tile;
    uint32_t spins = 0;
    while (t >= lo) {
        uint32_t s[W];
#pragma unroll
        for (int w = 0; w < W; w++) {
            const int64_t tt = t - w;
            // before the segment's first tile reads as an empty inclusive
            // word (that tile's own word is inclusive, so a correct walk
            // stops there)
            s[w] = tt >= lo ? load_agent(&status[(uint64_t)tt * RADIX + d]) : FLAG_INC;
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
        if (consumed == 0) {
            if (++spins > LOOKBACK_SPIN_LIMIT) { atomicOr(err, DEVERR_LOOKBACK_TIMEOUT); return prefix; }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    atomicOr(err, DEVERR_BAD_TILE);
    return prefix;
}

// ---------------------------------------------------------------- the pass

// A raw buffer over the first n 4-byte elements of an array (n < 2^30, so the
// byte range fits the 32-bit record count).  The fourth descriptor word is
// the usual one of gfx9 parts (32-bit data format).  A store at a byte offset
// at or past the range (~0u, say) is dropped by the hardware.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(T *base, uint32_t n)
{
    static_assert(sizeof(T) == 4, "4-byte elements");
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<std::remove_const_t<T> *>(base), 0, (int)(n * 4u),
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ void buffer_store(__amdgpu_buffer_rsrc_t rs, uint32_t off, T v)
{
    static_assert(sizeof(T) == 4, "4-byte elements");
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, (int)off, 0, 0);
}


template <typename K>
struct PassArgs {
    const K *in;
    K *out;
    K *tmp;
    const uint32_t *vin;
    uint32_t *vout;
    uint32_t *vtmp;
    const uint32_t *plan;   // this pass's plan words: active, src, dst, ordinal
    uint32_t *status0;      // look-back words [tile][radix] for even / odd active passes
    uint32_t *status1;
    uint32_t *counters;
    uint32_t n;             // keys in the whole buffer (bound of every store)
    uint32_t pass;
    uint32_t tile_capacity; // tiles the status arrays hold
};

template <typename K, int BITS, bool PAIRS, class DigitArgs, class Tiles>
__global__ __launch_bounds__((PassCfg<K, BITS>::NT)) void k_onesweep(PassArgs<K> a, DigitArgs da, Tiles tl)
{
    using C = PassCfg<K, BITS>;
    constexpr int RADIX = C::RADIX, NT = C::NT, WAVES = C::WAVES, IPT = C::IPT, TILE = C::TILE;
    constexpr uint32_t MASK = RADIX - 1;
    constexpr int DPT = RADIX > NT ? RADIX / NT : 1;    // digits per thread in digit phases
    static_assert(RADIX <= NT * DPT, "digit phase covers every digit");

    __shared__ alignas(16) unsigned char s_raw[TILE * sizeof(K)];
    __shared__ uint32_t s_wcnt[WAVES * RADIX];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_scan[NT / WAVE + 1];
    __shared__ uint32_t s_tile;
    K *s_stage = reinterpret_cast<K *>(s_raw);

    if (a.plan[0] == 0) return;   // pass skipped: the same for every workgroup
    uint32_t srcc = a.plan[1], dstc = a.plan[2];
    const uint32_t ord = a.plan[3];
    uint32_t *status = (ord & 1) ? a.status1 : a.status0;
    uint32_t *status_next = (ord & 1) ? a.status0 : a.status1;
    const auto dg = da.prepare();

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = tid / WAVE;

    // a grid sized for the most tiles possible: workgroups beyond the listed
    // tiles leave before the shared counter, so exactly the listed ids are
    // handed out (in the order workgroups reach the counter)
    if (blockIdx.x >= tl.listed()) return;
    if (tid == 0) s_tile = atomicAdd(&a.counters[CTR_TILE + a.pass], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    TileInfo ti;
    ti.excl2 = nullptr;
    ti.in = a.in;
    ti.out = a.out;
    ti.tmp = a.tmp;
    ti.limit = a.n;
    if (tile >= a.tile_capacity || !tl.template get<TILE>(tile, ti)) {
        // past the listed tiles (a grid sized for the most tiles possible),
        // or counters that were not reset: never index past the arrays
        if (tid == 0 && (tile >= a.tile_capacity || tl.missing_is_error()))
            atomicOr(&a.counters[CTR_ERROR], DEVERR_BAD_TILE);
        return;
    }
    if (!tl.route(ti, a.pass, srcc, dstc)) {
        // the tile's segment has a constant digit here: nothing moves, but
        // the tile's look-back words for the next pass start clear
        for (uint32_t d = tid; d < (uint32_t)RADIX; d += NT) store_agent(&status_next[(uint64_t)tile * RADIX + d], 0u);
        return;
    }
    const uint32_t *vsrc = nullptr;
    uint32_t *vdst = nullptr;
    if (PAIRS) {
        vsrc = srcc == BUF_IN ? a.vin : (srcc == BUF_OUT ? a.vout : a.vtmp);
        vdst = dstc == BUF_OUT ? a.vout : a.vtmp;
    }
    for (uint32_t i = tid; i < (uint32_t)(WAVES * RADIX); i += NT) s_wcnt[i] = 0;
    __syncthreads();
    const K *src = static_cast<const K *>(srcc == BUF_IN ? ti.in : (srcc == BUF_OUT ? ti.out : ti.tmp));
    K *dst = static_cast<K *>(dstc == BUF_OUT ? ti.out : ti.tmp);
    const uint32_t n = ti.limit;
    const uint32_t valid = ti.count;
    const bool first = tile == ti.first_tile;
    // where each digit's run of the tile would start without the earlier
    // tiles of the segment: loaded before the keys, so that these loads are
    // done by the time the look-back needs them
    uint32_t gofs[DPT];
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t d = tid * DPT + i;
        gofs[i] = d < (uint32_t)RADIX ? ti.base + ti.excl[d] + (ti.excl2 ? ti.excl2[d] : 0u) : 0u;
    }

    // ---- load: wave-striped, so (wave, item, lane) order is index order.
    // With 32-bit keys, keys, values and ranks in registers at once would not
    // fit in 128 VGPRs (two workgroups per CU): their values are loaded after
    // the keys have gone to LDS, and each staged key keeps only its digit
    // (four to a word) to find its value's destination
    constexpr bool COMPACT = PAIRS && sizeof(K) == 4;
    static_assert(!COMPACT || BITS <= 8, "digits pack four to a word");
    K k[IPT];
    uint32_t v[PAIRS ? IPT : 1];
    const uint32_t lofs = wave * (IPT * WAVE) + lane;   // tile-local index of item 0
    const uint32_t wofs = ti.start + lofs;
    if (valid == (uint32_t)TILE) {
        // one base address per thread, item offsets as immediates
        const K *sp = src + wofs;
        const uint32_t *vp = PAIRS && !COMPACT ? vsrc + wofs : nullptr;
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            k[j] = sp[j * WAVE];
            if (PAIRS && !COMPACT) v[j] = vp[j * WAVE];
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            const bool in = lofs + j * WAVE < valid;
            k[j] = in ? src[wofs + j * WAVE] : dg.template pad<K>();
            if (PAIRS && !COMPACT) v[j] = in ? vsrc[wofs + j * WAVE] : 0u;
        }
    }
    // keys past the end of the tile take the largest digit and so rank last
    using DG = std::remove_cv_t<decltype(dg)>;
    auto digit_of = [&](int j) -> uint32_t {
        if (DG::PAD_IS_MAX) return dg(k[j]);
        return (valid == (uint32_t)TILE || lofs + j * WAVE < valid) ? dg(k[j]) : MASK;
    };

    // ---- stable rank inside the wave
    uint32_t rk[IPT];
    uint32_t *wcnt = s_wcnt + wave * RADIX;
#pragma unroll
    for (int j = 0; j < IPT; j++) rk[j] = wave_rank_atomic(digit_of(j), wcnt);
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
            store_agent(&status[(uint64_t)tile * RADIX + d], (first ? FLAG_INC : FLAG_AGG) | run);
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
        if (d < (uint32_t)RADIX) {
            // every wave's offset of the digit inside the tile, so that the
            // reorder reads one word per key
#pragma unroll
            for (int w = 0; w < WAVES; w++) s_wcnt[w * RADIX + d] += texcl[i];
        }
    }
    __syncthreads();

    // ---- reorder the tile through LDS into digit order; this needs only
    // tile-local offsets, so it runs before the look-back
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const uint32_t d = digit_of(j);
        rk[j] += s_wcnt[wave * RADIX + d];
        s_stage[rk[j]] = k[j];
    }
    if constexpr (COMPACT) {
        // the value loads complete during the look-back
        if (valid == (uint32_t)TILE) {
            const uint32_t *vp = vsrc + wofs;
#pragma unroll
            for (int j = 0; j < IPT; j++) v[j] = vp[j * WAVE];
        } else {
#pragma unroll
            for (int j = 0; j < IPT; j++) v[j] = lofs + j * WAVE < valid ? vsrc[wofs + j * WAVE] : 0u;
        }
    }

    // ---- look-back: the counts of this digit in the earlier tiles of the
    // segment.  The digit's keys of this tile go to [start, start + count):
    // one range test per digit stands for a test per key.  4-byte keys keep
    // byte offsets in s_gbase (the buffer stores below take byte offsets)
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t d = tid * DPT + i;
        if (d < (uint32_t)RADIX) {
            uint32_t prefix = 0;
            if (!first) {
                prefix = look_back<RADIX>(status, tile, ti.first_tile, d, &a.counters[CTR_ERROR]);
                store_agent(&status[(uint64_t)tile * RADIX + d], FLAG_INC | (prefix + tcnt[i]));
            }
            const uint32_t start = gofs[i] + prefix;
            // padding past the tile's end is counted with the largest digit
            const uint32_t real = tcnt[i] - (d == MASK ? (uint32_t)TILE - valid : 0u);
            if ((uint64_t)start + real > n) atomicOr(&a.counters[CTR_ERROR], DEVERR_SCATTER_RANGE);
            s_gbase[d] = sizeof(K) == 4 ? (start - texcl[i]) << 2 : start - texcl[i];
            store_agent(&status_next[(uint64_t)tile * RADIX + d], 0u);
        }
    }
    __syncthreads();

    // ---- contiguous runs of each digit go to their global offsets.
    // 4-byte elements go through buffer stores whose range is the n
    // elements of the buffer; a key past the tile's end (only the last tile
    // of an array or a segment has any) gets an offset past every range, and
    // the hardware drops its store, so no store needs a branch
    uint32_t dest[PAIRS && !COMPACT ? IPT : 1];   // where each staged key went
    uint32_t dpk[COMPACT ? (IPT + 3) / 4 : 1];     // or its digit, four to a word
    if (COMPACT)
#pragma unroll
        for (int q = 0; q < (IPT + 3) / 4; q++) dpk[q] = 0;
    const uint32_t tid4 = tid * 4u;
    if constexpr (sizeof(K) == 4) {
        const auto rs = buffer_rsrc(dst, n);
        // groups of keys: their stage reads, then their run starts, then
        // their stores, so that LDS latency is paid once per group (small
        // groups with values, whose registers are live here)
        auto write_keys = [&](auto partial) {
            constexpr int G = COMPACT ? 2 : 8;
            static_assert(IPT % G == 0, "whole groups");
#pragma unroll
            for (int m0 = 0; m0 < IPT; m0 += G) {
                K key[G];
                uint32_t d[G], off[G];
#pragma unroll
                for (int u = 0; u < G; u++) key[u] = s_stage[(m0 + u) * NT + tid];
#pragma unroll
                for (int u = 0; u < G; u++) {
                    d[u] = dg(key[u]) & MASK;
                    off[u] = s_gbase[d[u]] + tid4 + (uint32_t)((m0 + u) * NT * 4);
                }
#pragma unroll
                for (int u = 0; u < G; u++) {
                    if (decltype(partial)::value && (m0 + u) * NT + tid >= valid) off[u] = ~0u;
                    buffer_store(rs, off[u], key[u]);
                    if (COMPACT) dpk[(m0 + u) / 4] |= d[u] << (8 * ((m0 + u) % 4));
                }
            }
        };
        if (valid == (uint32_t)TILE) write_keys(std::false_type{});
        else write_keys(std::true_type{});
    } else {
#pragma unroll
        for (int m = 0; m < IPT; m++) {
            const uint32_t i = m * NT + tid;
            if (PAIRS) dest[m] = ~0u;
            if (i < valid) {
                const K key = s_stage[i];
                const uint32_t g = s_gbase[dg(key)] + i;
                if (g < n) {
                    dst[g] = key;
                    if (PAIRS) dest[m] = g << 2;
                }
            }
        }
    }
    if (PAIRS) {
        uint32_t *s_v = reinterpret_cast<uint32_t *>(s_raw);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++) s_v[rk[j]] = v[j];
        __syncthreads();
        // (a branch per value: without it the compiler keeps every value and
        // offset of the thread in registers at once)
#pragma unroll
        for (int m = 0; m < IPT; m++) {
            const uint32_t i = m * NT + tid;
            if (i >= valid) continue;
            const uint32_t off = COMPACT ? s_gbase[(dpk[m / 4] >> (8 * (m % 4))) & 255u] + (i << 2) : dest[m];
            if (off < n * 4u) *reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(vdst) + off) = s_v[i];
        }
    }
}

// Moves a sort's result into the output buffers when its passes left it
// elsewhere, as the plan's final-copy words f[0..1] say: f[0] & COPY_KEYS
// moves the keys, f[0] & COPY_VALS the values, from buffer f[1] (the input
// when no pass ran, else the scratch buffer).  Keys and values are decided
// apart, because either may be sorted in place while the other is not.
template <typename K, bool PAIRS>
__global__ __launch_bounds__(256) void k_plan_final_copy(const K *in, K *out, K *tmp, const uint32_t *vin,
                                                         uint32_t *vout, uint32_t *vtmp, const uint32_t *f,
                                                         uint32_t n)
{
    const uint32_t what = f[0];
    if (what == 0) return;
    const bool from_in = f[1] == BUF_IN;
    const K *src = from_in ? in : tmp;
    const uint32_t *vsrc = from_in ? vin : vtmp;
    const bool keys = (what & COPY_KEYS) != 0;
    const bool vals = PAIRS && (what & COPY_VALS) != 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (keys) out[i] = src[i];
        if (vals) vout[i] = vsrc[i];
    }
}

}  // namespace intsort
