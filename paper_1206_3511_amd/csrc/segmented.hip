// segmented.hip -- sorts every segment [offsets[s], offsets[s+1]) of a packed
// array on its own, with no host read-back of the segment sizes.
//
// The offsets live on the device, so the device itself splits the segments
// into size classes:
//   tiny / small / medium / big   sorted by one workgroup each, entirely in
//                                 LDS (k_lds_sort), reading the input and
//                                 writing the output once;
//   large                         cut into tiles that get consecutive ids;
//                                 per-tile digit counts are summed per
//                                 segment into digit offsets, then every
//                                 digit pass runs k_onesweep over the tile
//                                 list with its look-back bounded by the
//                                 segment's first tile.  A segment skips
//                                 the passes whose digit is constant inside
//                                 it, with its own scratch/output ping-pong.
// Every launch has a grid sized for the most work the class can hold; work
// groups past the class's device-side count return at once.  Each segment is
// sorted with the stable LSD radix sort of section 2.5 (Algorithm 4), so the
// result is the segment's unique stable order.

#include <stdint.h>

#include <algorithm>

#include "device_common.hpp"
#include "intsort.h"
#include "internal.hpp"
#include "lds_sort.hpp"
#include "onesweep.hpp"
#include "sort_plans.hpp"

namespace intsort {

constexpr int SEG_HIST_THREADS = 256;

struct SegWs {
    uint32_t *counters;
    uint32_t *plan;
    uint32_t *lists;          // [NCLASS][list_stride]
    uint32_t list_stride;
    TileDesc *tiles;          // [tile_cap]
    uint32_t *tile_hist;      // [tile_cap][passes][radix]
    uint32_t *seg_excl;       // [passes][slot_cap][radix]
    uint32_t *status0;
    uint32_t *status1;
    uint32_t tile_cap;
    uint32_t slot_cap;
    SegBuf *bufs;             // [slot_cap] separate arrays only, else null
    void *tmp;                // scratch keys of the large segments
    uint32_t lds_cutoff;      // longer segments take the multi-workgroup path
    uint32_t *slot_mask;      // [slot_cap] digit passes each large segment runs
    uint32_t skip;            // leave out passes whose digit is constant in the segment
    uint32_t min_size;        // segments of at most this many keys are left alone
    uint32_t check;           // k_seg_check ran: sort nothing if it found a bad segment
    uint64_t n_total;         // keys of the whole call (the bound of the length sum)
    const uint64_t *sorted_in; // a device word; nonzero: sort nothing (the input is already in order)
};

// error-word bit: a segment (or array) the caller described would reach
// outside its buffers; with INTSORT_FLAG_CHECK_SEGMENTS nothing is sorted
constexpr uint32_t DEVERR_BAD_SEGMENTS = 8u;
static_assert(DEVERR_BAD_SEGMENTS == INTSORT_DEVERR_BAD_SEGMENTS, "public error bit matches");

// One thread per segment: the caller's segment layout, checked before any
// kernel uses it (INTSORT_FLAG_CHECK_SEGMENTS).  Each segment must be valid
// on its own, and the lengths together at most n: k_seg_classify compares
// the sum collected here.
template <class Src>
__global__ __launch_bounds__(256) void k_seg_check(Src src, uint64_t num_segments, uint64_t n, uint32_t *counters)
{
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t len = 0;
    if (s < num_segments && !src.valid(s, num_segments, n, len)) atomicOr(&counters[CTR_ERROR], DEVERR_BAD_SEGMENTS);
    // lengths are below 2^32 and segments at most 2^32: no overflow
    for (int o = WAVE / 2; o > 0; o /= 2) len += __shfl_xor(len, o, WAVE);
    if (lane_id() == 0 && len)
        atomicAdd(reinterpret_cast<unsigned long long *>(counters + CTR_SEG_SUM), (unsigned long long)len);
}

// One thread per segment: classify by size; a large segment reserves a run
// of consecutive tile ids and writes their descriptors (and, for separate
// arrays, its buffers and a slice of the scratch buffer).  Thread 0 also
// writes the plan words of the digit passes: every pass is launched (its
// ordinal picks the look-back words); which buffers a tile reads and writes
// follow from the passes its own segment runs.
template <typename K, class Src>
__global__ __launch_bounds__(256) void k_seg_classify(Src src, uint64_t num_segments, SegWs w, uint32_t passes)
{
    using CL = SegClasses<K>;
    constexpr uint32_t TILE = PassCfg<K, 8>::TILE;
    const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s == 0) {
        uint32_t prev = BUF_IN;
        for (uint32_t q = 0; q < passes; q++) {
            uint32_t *pw = w.plan + q * PLAN_WORDS;
            const uint32_t dst = (q % 2 == 0) ? BUF_TMP : BUF_OUT;
            pw[0] = 1; pw[1] = prev; pw[2] = dst; pw[3] = q;
            prev = dst;
        }
    }
    // nothing to sort, or a bad layout found by k_seg_check: no segment is
    // listed, so every later kernel finds nothing to do
    if (w.sorted_in && *w.sorted_in) return;
    if (w.check) {
        const uint64_t sum = *reinterpret_cast<const uint64_t *>(w.counters + CTR_SEG_SUM);
        const bool bad_sum = sum > w.n_total;
        if (bad_sum && s == 0) atomicOr(&w.counters[CTR_ERROR], DEVERR_BAD_SEGMENTS);
        if (bad_sum || (w.counters[CTR_ERROR] & DEVERR_BAD_SEGMENTS)) return;
    }
    const K *kin = nullptr;
    K *kout = nullptr;
    const uint32_t *vin;
    uint32_t *vout;
    uint32_t m = 0, lo = 0;
    int cls = -1;
    if (s < num_segments) {
        src.template seg<K>(s, kin, kout, vin, vout, m, lo);
        if (m <= w.min_size) cls = -1;
        else if (m > w.lds_cutoff) cls = 4;
        else if (m <= CL::CAP0) cls = 0;
        else if (m <= CL::CAP1) cls = 1;
        else if (m <= CL::CAP2) cls = 2;
        else if (m <= CL::CAP3) cls = 3;
        else cls = 4;
    }
    // one atomic per wave and class: the wave's lanes of a class take
    // consecutive list entries
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint64_t mine = ballot(cls == c);
        if (mine == 0) continue;
        uint32_t base = 0;
        if (mbcnt(mine) == 0 && cls == c) base = atomicAdd(&w.counters[CTR_SEG_CLASS + c], popc64(mine));
        base = __shfl(base, __builtin_ctzll(mine), WAVE);
        if (cls == c) {
            const uint32_t at = base + mbcnt(mine);
            if (at < w.list_stride) w.lists[c * w.list_stride + at] = (uint32_t)s;
        }
    }
    if (cls != 4) return;
    const uint32_t nt = (m + TILE - 1) / TILE;
    const uint32_t slot = atomicAdd(&w.counters[CTR_SEG_SLOTS], 1u);
    const uint32_t first = atomicAdd(&w.counters[CTR_SEG_TILES], nt);
    if (slot >= w.slot_cap || first + nt > w.tile_cap) {   // sized on the host so that this cannot happen
        atomicOr(&w.counters[CTR_ERROR], DEVERR_BAD_TILE);
        return;
    }
    if (w.bufs) {
        const uint32_t toff = atomicAdd(&w.counters[CTR_SEG_TMP], m);
        SegBuf b;
        b.in = kin;
        b.out = kout;
        b.tmp = static_cast<K *>(w.tmp) + toff;
        b.n = m;
        w.bufs[slot] = b;
    }
    for (uint32_t t = 0; t < nt; t++) {
        TileDesc d;
        d.slot = slot;
        d.first_tile = first;
        d.start = lo + t * TILE;
        d.count = min(TILE, m - t * TILE);
        d.base = lo;
        d.pad[0] = d.pad[1] = d.pad[2] = 0;
        w.tiles[first + t] = d;
    }
}

// per listed tile: the digit counts of every pass (one read of its keys);
// also clears the tile's look-back words for the first pass, and the first
// tile of each segment clears the segment's digit totals, which
// k_seg_slot_sum adds up next
template <typename K, int BITS>
__global__ __launch_bounds__(SEG_HIST_THREADS) void k_seg_tile_hist(const K *__restrict__ keys, SegWs w)
{
    constexpr int PASSES = 8 * (int)sizeof(K) / BITS;
    constexpr uint32_t RADIX = 1u << BITS;
    __shared__ uint32_t s_h[(sizeof(K) == 4 && BITS == 8) ? 1 : PASSES * RADIX];
    const uint32_t t = blockIdx.x;
    if (t >= w.counters[CTR_SEG_TILES]) return;
    const TileDesc d = w.tiles[t];
    const K *kp = w.bufs ? static_cast<const K *>(w.bufs[d.slot].in) : keys;
    if (t == d.first_tile)
        for (uint32_t i = threadIdx.x; i < PASSES * RADIX; i += SEG_HIST_THREADS)
            w.seg_excl[((uint64_t)(i / RADIX) * w.slot_cap + d.slot) * RADIX + i % RADIX] = 0;
    for (uint32_t i = threadIdx.x; i < RADIX; i += SEG_HIST_THREADS) w.status0[(uint64_t)t * RADIX + i] = 0;
    uint32_t *out = w.tile_hist + (uint64_t)t * PASSES * RADIX;
    if constexpr (sizeof(K) == 4 && BITS == 8) {
        // 32-bit keys: HC copies of the counts, lane l adding into copy
        // l % HC, two 16-bit counts to a word (word (p, v / 2, copy) holds
        // digit value v of pass p in half v % 2): at most a few lanes of an
        // add meet on a word whatever the keys.  The tile is read as
        // 16-byte vectors after the keys before the first 16-byte boundary.
        constexpr int HC = 16, HALF = (int)RADIX / 2;
        // one copy counts SEG_HIST_THREADS / HC threads' keys of one tile
        static_assert((uint64_t)PassCfg<K, BITS>::TILE / HC < 65536u, "16-bit counts cannot overflow");
        __shared__ uint32_t s_c[PASSES * HALF * HC];
        for (uint32_t i = threadIdx.x; i < (uint32_t)(PASSES * HALF * HC); i += SEG_HIST_THREADS) s_c[i] = 0;
        __syncthreads();
        uint32_t *my_c = s_c + threadIdx.x % HC;
        auto count_key = [&](uint32_t k) {
#pragma unroll
            for (int p = 0; p < PASSES; p++) {
                const uint32_t v = (k >> (BITS * p)) & (RADIX - 1);
                atomicAdd(my_c + (p * HALF + (v >> 1)) * HC, 1u << (16 * (v & 1)));
            }
        };
        const uint32_t *kt = reinterpret_cast<const uint32_t *>(kp + d.start);
        const uint32_t head = min(d.count, (uint32_t)((4u - ((uint32_t)(reinterpret_cast<uintptr_t>(kt) >> 2) & 3u)) & 3u));
        if (threadIdx.x < head) count_key(kt[threadIdx.x]);
        const uint32_t nv = (d.count - head) / 4;
        const uint4 *vp = reinterpret_cast<const uint4 *>(kt + head);
        constexpr int VU = 4;   // vectors in flight per thread
        for (uint32_t v0 = threadIdx.x; v0 < nv; v0 += SEG_HIST_THREADS * VU) {
            uint4 x[VU];
#pragma unroll
            for (int u = 0; u < VU; u++)
                if (v0 + u * SEG_HIST_THREADS < nv) x[u] = vp[v0 + u * SEG_HIST_THREADS];
#pragma unroll
            for (int u = 0; u < VU; u++) {
                if (v0 + u * SEG_HIST_THREADS < nv) {
                    count_key(x[u].x);
                    count_key(x[u].y);
                    count_key(x[u].z);
                    count_key(x[u].w);
                }
            }
        }
        for (uint32_t i = head + nv * 4 + threadIdx.x; i < d.count; i += SEG_HIST_THREADS) count_key(kt[i]);
        __syncthreads();
        // the sum of the copies (read from a rotated start, so that the
        // threads spread over the banks)
        for (uint32_t i = threadIdx.x; i < PASSES * RADIX; i += SEG_HIST_THREADS) {
            const uint32_t p = i / RADIX, v = i % RADIX;
            const uint32_t *wd = s_c + (p * HALF + (v >> 1)) * HC;
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < HC; q++) c += (wd[(q + (v >> 1)) % HC] >> (16 * (v & 1))) & 0xffffu;
            out[i] = c;
        }
        return;
    }
    for (uint32_t i = threadIdx.x; i < PASSES * RADIX; i += SEG_HIST_THREADS) s_h[i] = 0;
    __syncthreads();
    // U loads in flight per thread (segments start anywhere, so 4- or
    // 8-byte loads)
    constexpr int U = 8;
    for (uint32_t i0 = threadIdx.x; i0 < d.count; i0 += SEG_HIST_THREADS * U) {
        K x[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t i = i0 + u * SEG_HIST_THREADS;
            x[u] = i < d.count ? kp[d.start + i] : K(0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (i0 + u * SEG_HIST_THREADS < d.count) {
#pragma unroll
                for (int p = 0; p < PASSES; p++)
                    lds_count(s_h + p * RADIX, digit_at<K>(x[u], (uint32_t)(BITS * p), RADIX - 1));
            }
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < PASSES * RADIX; i += SEG_HIST_THREADS) out[i] = s_h[i];
}

// Digit totals of every large segment: each workgroup adds up the counts of
// SUM_TILES consecutive listed tiles (a segment's tiles have consecutive
// ids), one thread per digit, and adds each segment's part into its totals
// in seg_excl.  A segment of thousands of tiles is spread over many
// workgroups instead of being walked by one.
constexpr uint32_t SUM_TILES = 32;

template <typename K, int BITS>
__global__ __launch_bounds__(256) void k_seg_slot_sum(SegWs w)
{
    constexpr int PASSES = 8 * (int)sizeof(K) / BITS;
    constexpr uint32_t RADIX = 1u << BITS;
    static_assert(RADIX <= 256, "one thread per digit");
    const uint32_t listed = min(w.counters[CTR_SEG_TILES], w.tile_cap);
    const uint32_t t0 = blockIdx.x * SUM_TILES;
    if (t0 >= listed) return;
    const uint32_t t1 = min(listed, t0 + SUM_TILES);
    const uint32_t d = threadIdx.x;
    if (d >= RADIX) return;
    uint32_t acc[PASSES];
    auto flush = [&](uint32_t slot) {
#pragma unroll
        for (int p = 0; p < PASSES; p++) {
            if (acc[p]) atomicAdd(&w.seg_excl[((uint64_t)p * w.slot_cap + slot) * RADIX + d], acc[p]);
            acc[p] = 0;
        }
    };
#pragma unroll
    for (int p = 0; p < PASSES; p++) acc[p] = 0;
    uint32_t cur = w.tiles[t0].slot;
    for (uint32_t t = t0; t < t1; t++) {
        const uint32_t slot = w.tiles[t].slot;
        if (slot != cur) {
            flush(cur);
            cur = slot;
        }
#pragma unroll
        for (int p = 0; p < PASSES; p++) acc[p] += w.tile_hist[((uint64_t)t * PASSES + p) * RADIX + d];
    }
    flush(cur);
}

// per large segment: exclusive scan of its digit totals per pass, and the
// passes whose digit is not constant inside it
template <typename K, int BITS>
__global__ __launch_bounds__(256) void k_seg_scan(SegWs w)
{
    constexpr int PASSES = 8 * (int)sizeof(K) / BITS;
    constexpr uint32_t RADIX = 1u << BITS;
    static_assert(PASSES <= 32, "one mask bit per pass");
    __shared__ uint32_t s_scan[256 / WAVE + 1];
    __shared__ uint32_t s_const;
    const uint32_t slot = blockIdx.x;
    if (slot >= w.counters[CTR_SEG_SLOTS] || slot >= w.slot_cap) return;
    const uint32_t d = threadIdx.x;   // a digit (threads past the radix count nothing)
    uint32_t mask = 0;
    for (int p = 0; p < PASSES; p++) {
        uint32_t *e = w.seg_excl + ((uint64_t)p * w.slot_cap + slot) * RADIX;
        const uint32_t c = d < RADIX ? e[d] : 0u;
        if (d == 0) s_const = 0;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan<256>(c, s_scan, &total);
        if (d < RADIX) e[d] = ex;
        // a digit that takes one value in the whole segment leaves the
        // segment's order as it is: the pass has nothing to do for it
        if (d < RADIX && c == total) s_const = 1;
        __syncthreads();
        if (!(w.skip && s_const)) mask |= 1u << p;
        __syncthreads();
    }
    if (d == 0) w.slot_mask[slot] = mask;
}

// Moves every large segment whose keys did not end in the output there: all
// its digits were constant (then only what is not sorted in place moves), or
// its passes ran from the scratch buffer (keys or values in place) and an
// odd number of them left it there (then keys and values move).
template <typename K, bool PAIRS, class TilesT>
__global__ __launch_bounds__(256) void k_seg_final_copy(PassArgs<K> a, TilesT tl)
{
    constexpr int TILE = PassCfg<K, 8>::TILE;
    if (blockIdx.x >= tl.listed()) return;
    TileInfo ti;
    ti.in = a.in;
    ti.out = a.out;
    ti.tmp = a.tmp;
    ti.limit = a.n;
    if (!tl.template get<TILE>(blockIdx.x, ti)) return;
    const bool keys_alias = ti.in == ti.out;
    const bool vals_alias = PAIRS && a.vin == a.vout;
    const uint32_t where = segment_result(tl.slot_mask[ti.slot], keys_alias || vals_alias);
    if (where == BUF_OUT) return;
    const bool keys = where == BUF_TMP || !keys_alias;
    const bool vals = PAIRS && (where == BUF_TMP || !vals_alias);
    if (!keys && !vals) return;
    const K *src = static_cast<const K *>(where == BUF_IN ? ti.in : ti.tmp);
    K *dst = static_cast<K *>(ti.out);
    const uint32_t *vsrc = where == BUF_IN ? a.vin : a.vtmp;
    for (uint32_t i = threadIdx.x; i < ti.count; i += 256) {
        const uint32_t g = ti.start + i;
        if (g < ti.limit) {
            if (keys) dst[g] = src[g];
            if (vals) a.vout[g] = vsrc[g];
        }
    }
}

// ------------------------------------------------------------------ host

template <typename K>
static uint32_t seg_cutoff(uint32_t requested)
{
    using CL = SegClasses<K>;
    return (requested == 0 || requested > CL::LDS_MAX) ? CL::LDS_MAX : requested;
}

template <typename K, bool PAIRS>
static SegLayout seg_layout_typed(uint64_t n, uint64_t S, uint32_t cutoff_req)
{
    constexpr uint32_t TILE = PassCfg<K, 8>::TILE;
    constexpr int PASSES = (int)sizeof(K);
    SegLayout L{};
    L.lds_cutoff = seg_cutoff<K>(cutoff_req);
    // no more segments than this can be longer than the cutoff
    L.slot_cap = (uint32_t)std::min<uint64_t>(S, n / ((uint64_t)L.lds_cutoff + 1));
    L.tile_cap = (uint32_t)((n + TILE - 1) / TILE + L.slot_cap);
    L.list_stride = (uint32_t)S;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off += align_up(bytes, 256); return at; };
    L.counters = take((size_t)CTR_WORDS * 4);
    L.plan = take((size_t)(MAX_PASSES + 1) * PLAN_WORDS * 4);
    L.lists = take((size_t)SegClasses<K>::NCLASS * S * 4);
    L.tiles = take((size_t)L.tile_cap * sizeof(TileDesc));
    L.bufs = take((size_t)L.slot_cap * sizeof(SegBuf));
    // sized for 8-bit digits; the 4-bit counts (twice the passes, a
    // sixteenth of the digits) fit in the same arrays
    L.tile_hist = take((size_t)L.tile_cap * PASSES * 256 * 4);
    L.seg_excl = take((size_t)PASSES * L.slot_cap * 256 * 4);
    L.slot_mask = take((size_t)L.slot_cap * 4);
    L.status0 = take((size_t)L.tile_cap * 256 * 4);
    L.status1 = take((size_t)L.tile_cap * 256 * 4);
    L.tmp_keys = take(n * sizeof(K));
    L.tmp_vals = take(PAIRS ? n * 4 : 0);
    L.total = off;
    return L;
}

SegLayout segmented_layout(int key_bytes, bool pairs, uint64_t n, uint64_t num_segments, const intsort_options &o)
{
    const uint32_t c = o.lds_cutoff;
    if (key_bytes == 4) return pairs ? seg_layout_typed<uint32_t, true>(n, num_segments, c)
                                     : seg_layout_typed<uint32_t, false>(n, num_segments, c);
    return pairs ? seg_layout_typed<uint64_t, true>(n, num_segments, c)
                 : seg_layout_typed<uint64_t, false>(n, num_segments, c);
}

template <typename K, bool PAIRS, int NT, int IPT, class Src>
static void launch_lds_class(const LdsSortArgs<Src> &la, uint32_t grid, hipStream_t s)
{
    if (grid == 0) return;
    // 64-bit keys differ in up to eight bytes: their passes move indices
    if constexpr (sizeof(K) == 8) hipLaunchKernelGGL((k_lds_sort_idx<K, PAIRS, NT, IPT, Src>), dim3(grid), dim3(NT), 0, s, la);
    else hipLaunchKernelGGL((k_lds_sort<K, PAIRS, NT, IPT, Src>), dim3(grid), dim3(NT), 0, s, la);
}

static void set_bufs(SegTiles &, const SegBuf *) {}
static void set_bufs(DescTiles &t, const SegBuf *b) { t.bufs = b; }

// the whole segmented sort for one key type; Src says where segments live,
// Tiles how the digit passes of the large ones find their buffers
template <typename K, bool PAIRS, class Src, class TilesT, int BITS>
static hipError_t seg_run_typed(const SegCall &c, const Src &src, bool separate, hipStream_t s)
{
    using CL = SegClasses<K>;
    using PC = PassCfg<K, BITS>;
    static_assert(PassCfg<K, BITS>::TILE == PassCfg<K, 8>::TILE, "tiles listed at the 8-bit size");
    constexpr int PASSES = 8 * (int)sizeof(K) / BITS;
    constexpr uint32_t RADIX = 1u << BITS;
    const SegLayout &L = c.L;
    char *ws = c.ws;
    Timer *tm = c.timer;
    SegWs w{};
    w.counters = reinterpret_cast<uint32_t *>(ws + L.counters);
    w.plan = reinterpret_cast<uint32_t *>(ws + L.plan);
    w.lists = reinterpret_cast<uint32_t *>(ws + L.lists);
    w.list_stride = L.list_stride;
    w.tiles = reinterpret_cast<TileDesc *>(ws + L.tiles);
    w.tile_hist = reinterpret_cast<uint32_t *>(ws + L.tile_hist);
    w.seg_excl = reinterpret_cast<uint32_t *>(ws + L.seg_excl);
    w.status0 = reinterpret_cast<uint32_t *>(ws + L.status0);
    w.status1 = reinterpret_cast<uint32_t *>(ws + L.status1);
    w.tile_cap = L.tile_cap;
    w.slot_cap = L.slot_cap;
    w.bufs = separate ? reinterpret_cast<SegBuf *>(ws + L.bufs) : nullptr;
    w.tmp = ws + L.tmp_keys;
    w.lds_cutoff = L.lds_cutoff;
    w.slot_mask = reinterpret_cast<uint32_t *>(ws + L.slot_mask);
    w.skip = (c.opts.flags & INTSORT_FLAG_NO_PASS_SKIP) ? 0u : 1u;
    w.min_size = c.min_size;
    w.check = (c.opts.flags & INTSORT_FLAG_CHECK_SEGMENTS) ? 1u : 0u;
    w.n_total = c.n;
    w.sorted_in = c.skip;

    if (tm) tm->start(s);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(1), dim3(256), 0, s, w.counters, (uint64_t)CTR_WORDS, 0u);
    const uint32_t cgrid = (uint32_t)((c.num_segments + 255) / 256);
    if (w.check)
        hipLaunchKernelGGL((k_seg_check<Src>), dim3(cgrid), dim3(256), 0, s, src, c.num_segments, c.n, w.counters);
    hipLaunchKernelGGL((k_seg_classify<K, Src>), dim3(cgrid), dim3(256), 0, s, src, c.num_segments, w,
                       (uint32_t)PASSES);
    if (tm) tm->mark(INTSORT_KERNEL_PLAN, 0, s);

    // the four on-chip classes
    LdsSortArgs<Src> la{};
    la.src = src;
    const uint64_t S = c.num_segments;
    auto grid_for = [&](uint32_t lo_exclusive, uint32_t cap) {
        // at most this many segments can be longer than lo_exclusive; none
        // longer than the cutoff, and none up to min_size, reaches an
        // on-chip class
        if (lo_exclusive >= L.lds_cutoff || cap <= c.min_size) return 0u;
        lo_exclusive = std::max(lo_exclusive, c.min_size);
        const uint64_t by_n = c.n / (uint64_t)(lo_exclusive + 1);
        return (uint32_t)std::min<uint64_t>(S, lo_exclusive == 0 ? S : by_n);
    };
    la.list = w.lists + 0 * L.list_stride;
    la.list_count = w.counters + CTR_SEG_CLASS + 0;
    launch_lds_class<K, PAIRS, 64, 4>(la, grid_for(0, CL::CAP0), s);
    la.list = w.lists + 1 * L.list_stride;
    la.list_count = w.counters + CTR_SEG_CLASS + 1;
    launch_lds_class<K, PAIRS, 256, 8>(la, grid_for(CL::CAP0, CL::CAP1), s);
    la.list = w.lists + 2 * L.list_stride;
    la.list_count = w.counters + CTR_SEG_CLASS + 2;
    launch_lds_class<K, PAIRS, 512, 16>(la, grid_for(CL::CAP1, CL::CAP2), s);
    if (CL::CAP3 > CL::CAP2) {
        la.list = w.lists + 3 * L.list_stride;
        la.list_count = w.counters + CTR_SEG_CLASS + 3;
        launch_lds_class<K, PAIRS, 512, (CL::CAP3 > CL::CAP2 ? 32 : 16)>(la, grid_for(CL::CAP2, CL::CAP3), s);
    }
    if (tm) tm->mark(INTSORT_KERNEL_SEGMENT_SORT, 0, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (L.slot_cap == 0) return hipSuccess;   // no segment can be large

    // the large segments: digit counts per tile, offsets per segment, passes
    hipLaunchKernelGGL((k_seg_tile_hist<K, BITS>), dim3(L.tile_cap), dim3(SEG_HIST_THREADS), 0, s,
                       static_cast<const K *>(c.keys_in), w);
    if (tm) tm->mark(INTSORT_KERNEL_DIGIT_HISTOGRAM, 0, s);
    hipLaunchKernelGGL((k_seg_slot_sum<K, BITS>), dim3((L.tile_cap + SUM_TILES - 1) / SUM_TILES), dim3(256), 0, s, w);
    hipLaunchKernelGGL((k_seg_scan<K, BITS>), dim3(L.slot_cap), dim3(256), 0, s, w);
    if (tm) tm->mark(INTSORT_KERNEL_PLAN, 1, s);

    PassArgs<K> a{};
    a.in = static_cast<const K *>(c.keys_in);
    a.out = static_cast<K *>(c.keys_out);
    a.tmp = reinterpret_cast<K *>(ws + L.tmp_keys);
    a.vin = c.vals_in;
    a.vout = c.vals_out;
    a.vtmp = reinterpret_cast<uint32_t *>(ws + L.tmp_vals);
    a.status0 = w.status0;
    a.status1 = w.status1;
    a.counters = w.counters;
    a.n = (uint32_t)c.n;
    a.tile_capacity = L.tile_cap;
    TilesT tl{};
    tl.desc = w.tiles;
    tl.num_tiles = w.counters + CTR_SEG_TILES;
    tl.radix = RADIX;
    tl.slot_mask = w.slot_mask;
    // a pass must not read and write one buffer: keys or values in place
    // route every large segment's passes from the scratch buffer
    tl.in_place = (c.keys_in == c.keys_out || (PAIRS && c.vals_in == c.vals_out)) ? 1u : 0u;
    set_bufs(tl, w.bufs);
    for (int p = 0; p < PASSES; p++) {
        a.plan = w.plan + p * PLAN_WORDS;
        a.pass = (uint32_t)p;
        const RadixDigit dg{(uint32_t)(BITS * p), RADIX - 1};
        tl.seg_excl = w.seg_excl + (uint64_t)p * L.slot_cap * RADIX;
        hipLaunchKernelGGL((k_onesweep<K, BITS, PAIRS, RadixDigit, TilesT>), dim3(L.tile_cap), dim3(PC::NT), 0, s,
                           a, dg, tl);
        if (tm) tm->mark(INTSORT_KERNEL_PASS, (uint32_t)p, s);
    }
    hipLaunchKernelGGL((k_seg_final_copy<K, PAIRS, TilesT>), dim3(L.tile_cap), dim3(256), 0, s, a, tl);
    if (tm) tm->mark(INTSORT_KERNEL_COPY, 1, s);
    return hipGetLastError();
}

template <int BITS>
static hipError_t segmented_sort_bits(const SegCall &c, hipStream_t s)
{
    if (c.descs) {
        if (c.pairs) return hipErrorNotSupported;
        const DescSrc src{c.descs};
        if (c.key_bytes == 4) return seg_run_typed<uint32_t, false, DescSrc, DescTiles, BITS>(c, src, true, s);
        return seg_run_typed<uint64_t, false, DescSrc, DescTiles, BITS>(c, src, true, s);
    }
    const PackedSrc src{c.keys_in, c.keys_out, c.vals_in, c.vals_out, c.offsets};
    if (c.key_bytes == 4)
        return c.pairs ? seg_run_typed<uint32_t, true, PackedSrc, SegTiles, BITS>(c, src, false, s)
                       : seg_run_typed<uint32_t, false, PackedSrc, SegTiles, BITS>(c, src, false, s);
    return c.pairs ? seg_run_typed<uint64_t, true, PackedSrc, SegTiles, BITS>(c, src, false, s)
                   : seg_run_typed<uint64_t, false, PackedSrc, SegTiles, BITS>(c, src, false, s);
}

// The multi-workgroup passes of the large segments take 4- or 8-bit digits
// (the on-chip classes sort with 8-bit digits whatever the width: any stable
// sort gives the same bytes).
hipError_t segmented_sort_run(const SegCall &c, hipStream_t s)
{
    if (c.opts.digit_bits == 8) return segmented_sort_bits<8>(c, s);
    if (c.opts.digit_bits == 4) return segmented_sort_bits<4>(c, s);
    return hipErrorNotSupported;
}

}  // namespace intsort
