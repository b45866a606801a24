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

#include <algorithm>

#include "device_common.hpp"
#include "intsort.h"
#include "internal.hpp"
#include "chunk_sort.hpp"
#include "onesweep.hpp"

namespace intsort {

constexpr int HIST_THREADS = 256;
// most first-pass tiles one histogram workgroup counts (a chunk: the scan
// over chunks is shorter the more tiles each holds)
constexpr uint32_t FIRST_PASS_TILES_PER_CHUNK = 8;
#ifndef HIST_UNROLL
#define HIST_UNROLL 4
#endif
#ifndef HIST_BLOCKS_PER_CU
#define HIST_BLOCKS_PER_CU 4
#endif
#ifndef HIST_COPIES
#define HIST_COPIES 4
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
    uint32_t keys_alias;   // keys_in == keys_out
    uint32_t vals_alias;   // key-value sort with vals_in == vals_out
    uint32_t finalize;     // 0: only count (step-level entry point), no plan
    uint32_t copies;       // histogram copies the workgroups spread their adds over
    uint32_t *tile_counts; // [tile][radix] first pass: each tile's digit offsets inside its chunk, or null
    uint32_t *chunk_sums;  // [chunk][radix] first pass: digit counts of each chunk of tiles
    uint32_t num_tiles;    // tiles of the first pass (with tile_counts)
    uint32_t tiles_per_wg; // tiles per chunk (<= FIRST_PASS_TILES_PER_CHUNK): one workgroup each
    uint32_t num_chunks;   // chunks (histogram workgroups) of the first pass
};

// PER_TILE: the first pass's digits are counted per tile (a.tile_counts set)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename K, int BITS, int ORDER, bool PER_TILE>
__global__ __launch_bounds__(HIST_THREADS) void k_digit_histogram(const K *__restrict__ keys, HistArgs a)
{
    constexpr int RADIX = 1 << BITS;
    constexpr int PASSES = PassCfg<K, BITS>::PASSES;
    constexpr uint32_t MASK = RADIX - 1;
    constexpr int KPV = 16 / (int)sizeof(K);
    struct alignas(16) Vec { K v[KPV]; };

    __shared__ uint32_t s_h[PASSES * RADIX];
    constexpr bool TILED = PER_TILE && RADIX <= HIST_THREADS && sizeof(K) == 4;   // one thread per digit
    // The first-pass digits of the tile being read go to HT copies of its
    // counts, lane l adding into copy l % HT at word (digit * HT + copy): a
    // digit costs two integer instructions and one LDS add, and the lanes
    // of one add meet on a word only when digit and copy agree.  The other
    // passes' digits count for the whole chunk in HC copies, two 16-bit
    // counts to a word: word (p - 1, v / 2, copy) holds digit value v of
    // pass p in half v % 2, so that at most four lanes of an add share a
    // word even when every lane holds the same digit (sorted or
    // narrow-range keys).
    constexpr int HT = 8;
    constexpr int HC = 16;
    constexpr int HALF = RADIX / 2;
    static_assert(!TILED || HIST_THREADS % HC == 0, "every copy has the same threads");
    // one copy counts at most HIST_THREADS / HC threads' keys of one chunk
    static_assert(!TILED || (uint64_t)FIRST_PASS_TILES_PER_CHUNK * PassCfg<K, BITS>::TILE / HC < 65536u,
                  "16-bit counts cannot overflow");
    __shared__ uint32_t s_t[TILED ? RADIX * HT : 1];
    __shared__ uint32_t s_c[TILED ? (PASSES - 1) * HALF * HC : 1];

    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (uint32_t)(PASSES * RADIX); i += HIST_THREADS) s_h[i] = 0;
    if (TILED) {
        for (uint32_t i = tid; i < (uint32_t)(RADIX * HT); i += HIST_THREADS) s_t[i] = 0;
        for (uint32_t i = tid; i < (uint32_t)((PASSES - 1) * HALF * HC); i += HIST_THREADS) s_c[i] = 0;
    }
    {
        const uint64_t stride = (uint64_t)gridDim.x * HIST_THREADS;
        for (uint64_t i = (uint64_t)blockIdx.x * HIST_THREADS + tid; i < a.status0_words; i += stride)
            a.status0[i] = 0;
    }
    __syncthreads();

    const uint32_t n = a.n;
    if constexpr (TILED) if (a.tile_counts) {
        // one chunk of consecutive first-pass tiles, read tile by tile: the
        // first-pass digits count per tile, the other digits for the chunk
        constexpr uint32_t TILE = PassCfg<K, BITS>::TILE;
        constexpr int VPTH = (int)(TILE / KPV / HIST_THREADS);   // vectors per thread and tile
        static_assert(TILE % (KPV * HIST_THREADS) == 0, "tiles of whole vectors per thread");
        const uint32_t t0 = blockIdx.x * a.tiles_per_wg;
        const uint32_t t1 = min(a.num_tiles, t0 + a.tiles_per_wg);
        uint32_t *my_t = s_t + tid % HT;
        uint32_t *my_c = s_c + tid % HC;
        auto count_key = [&](K key) {
            const K k = KeyOrder<ORDER>::ordered(key);
            atomicAdd(my_t + digit_at<K>(k, 0u, MASK) * HT, 1u);
#pragma unroll
            for (int p = 1; p < PASSES; p++) {
                const uint32_t d = digit_at<K>(k, (uint32_t)(p * BITS), MASK);
                atomicAdd(my_c + ((p - 1) * HALF + (d >> 1)) * HC, 1u << (16 * (d & 1)));
            }
        };
        uint32_t acc = 0;   // thread d < RADIX: digit d's count in the chunk's earlier tiles
        for (uint32_t t = t0; t < t1; t++) {
            const uint32_t k0 = t * TILE;
            const uint32_t cnt = min(n - k0, TILE);
            if (cnt == TILE) {
                // every vector of the thread's share of the tile in flight at once
                const Vec *tv = reinterpret_cast<const Vec *>(keys + k0) + tid;
                Vec x[VPTH];
#pragma unroll
                for (int j = 0; j < VPTH; j++) {
                    // non-temporal: the keys do not take last-level cache
                    // lines, so the lines the previous kernel left dirty
                    // there are not evicted (written back) under this read
                    // (the write-back moves into the first pass, which
                    // costs less than it saves here)
                    const u32x4 t = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(tv + j * HIST_THREADS));
                    __builtin_memcpy(&x[j], &t, sizeof(t));
                }
#pragma unroll
                for (int j = 0; j < VPTH; j++)
#pragma unroll
                    for (int e = 0; e < KPV; e++) count_key(x[j].v[e]);
            } else {
                for (uint32_t i = tid; i < cnt; i += HIST_THREADS) count_key(keys[k0 + i]);
            }
            __syncthreads();
            if (tid < (uint32_t)RADIX) {
                // the tile's count of digit tid: the sum of its copies (read
                // from a rotated start, so that the threads spread over the
                // banks), which start clear for the next tile
                uint32_t c = 0;
#pragma unroll
                for (int q = 0; q < HT; q++) {
                    const uint32_t w = tid * HT + (q + tid) % HT;
                    c += s_t[w];
                    s_t[w] = 0;
                }
                a.tile_counts[(uint64_t)t * RADIX + tid] = acc;
                acc += c;
            }
            __syncthreads();
        }
        if (tid < (uint32_t)RADIX) {
            a.chunk_sums[(uint64_t)blockIdx.x * RADIX + tid] = acc;
            s_h[tid] = acc;
        }
        // the other passes' counts: the sum of the copies (read from a
        // rotated start, so that the threads spread over the banks)
        for (uint32_t i = tid; i < (uint32_t)((PASSES - 1) * RADIX); i += HIST_THREADS) {
            const uint32_t p1 = i / RADIX, v = i % RADIX;
            const uint32_t *w = s_c + (p1 * HALF + (v >> 1)) * HC;
            uint32_t c = 0;
#pragma unroll
            for (int q = 0; q < HC; q++) c += (w[(q + (v >> 1)) % HC] >> (16 * (v & 1))) & 0xffffu;
            s_h[RADIX + i] = c;
        }
        __syncthreads();
        uint32_t *hdst = a.hist + (blockIdx.x % a.copies) * (uint32_t)(PASSES * RADIX);
        for (uint32_t i = tid; i < (uint32_t)(PASSES * RADIX); i += HIST_THREADS) {
            uint32_t c = s_h[i];
            if (c) atomicAdd(&hdst[i], c);
        }
        return;
    }
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
                        lds_count(s_h + p * RADIX,
                                  digit_at<K>(KeyOrder<ORDER>::ordered(x[u].v[e]), (uint32_t)(p * BITS), MASK));
                }
            }
        }
    }
    if (blockIdx.x == 0) {
        for (uint32_t i = nvec * KPV + tid; i < n; i += HIST_THREADS) {
            const K k = KeyOrder<ORDER>::ordered(keys[i]);
#pragma unroll
            for (int p = 0; p < PASSES; p++)
                lds_count(s_h + p * RADIX, digit_at<K>(k, (uint32_t)(p * BITS), MASK));
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
// which buffer each reads and writes.  The plan is the last workgroup's; with
// a first pass whose tiles were counted by the histogram kernel, workgroup d
// < radix also turns the chunk totals of first-pass digit d into where each
// chunk's run of d starts (the digit's start plus its counts in the earlier
// chunks), so that a tile's start is its chunk's plus its own offset inside
// the chunk.  Runs after the histogram kernel, so every count is complete
// and visible.
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

    if (blockIdx.x + 1 < gridDim.x) {
        // chunk scan of first-pass digit d (the grid has radix + 1 workgroups
        // only when RADIX <= HIST_THREADS)
        const uint32_t d = blockIdx.x;
        __shared__ uint32_t s_start;
        uint32_t c = 0;
        if (tid < (uint32_t)RADIX)
            for (uint32_t cp = 0; cp < a.copies; cp++) c += a.hist[cp * (uint32_t)(PASSES * RADIX) + tid];
        uint32_t total_unused;
        const uint32_t ex = block_exclusive_scan<HIST_THREADS>(c, s_scan, &total_unused);
        if (tid == d) s_start = ex;
        __syncthreads();
        const uint32_t chunks = a.num_chunks;
        const uint32_t per = (chunks + HIST_THREADS - 1) / HIST_THREADS;
        const uint32_t j0 = min(chunks, tid * per), j1 = min(chunks, j0 + per);
        uint32_t sum = 0;
        for (uint32_t j = j0; j < j1; j++) sum += a.chunk_sums[(uint64_t)j * RADIX + d];
        uint32_t run = s_start + block_exclusive_scan<HIST_THREADS>(sum, s_scan, &total_unused);
        for (uint32_t j = j0; j < j1; j++) {
            const uint32_t v = a.chunk_sums[(uint64_t)j * RADIX + d];
            a.chunk_sums[(uint64_t)j * RADIX + d] = run;
            run += v;
        }
        return;
    }
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
        // active pass must land in the output buffer.  When either the keys
        // or the values are sorted in place, no pass may read and write one
        // buffer, so the first pass goes to the scratch buffer and the
        // passes alternate from there.
        const bool in_place = a.keys_alias || a.vals_alias;
        uint32_t act[MAX_PASSES];
        uint32_t A = 0;
        for (int p = 0; p < PASSES; p++) {
            act[p] = ((uint32_t)p < a.max_passes) && !(a.skip && s_const[p]);
            A += act[p];
        }
        if (A == 0 && !in_place && a.max_passes > 0) {
            // every digit is constant: the last allowed pass still runs (the
            // identity permutation), so the keys land in the output without
            // a copy and the host never needs to launch one
            act[min((uint32_t)PASSES, a.max_passes) - 1] = 1;
            A = 1;
        }
        uint32_t q = 0, prev_dst = BUF_IN;
        for (int p = 0; p < PASSES; p++) {
            uint32_t *w = a.plan + p * PLAN_WORDS;
            if (!act[p]) { w[0] = 0; w[1] = 0; w[2] = 0; w[3] = 0; continue; }
            uint32_t dst;
            if (in_place) dst = (q % 2 == 0) ? BUF_TMP : BUF_OUT;
            else dst = ((A - 1 - q) % 2 == 0) ? BUF_OUT : BUF_TMP;
            w[0] = 1; w[1] = prev_dst; w[2] = dst; w[3] = q;
            prev_dst = dst;
            q++;
        }
        // final copy: bit 0 moves the keys, bit 1 the values, from f[1]
        uint32_t *f = a.plan + MAX_PASSES * PLAN_WORDS;
        if (A == 0) {
            // nothing moved: copy whatever is not already in place
            f[0] = (a.keys_alias ? 0u : COPY_KEYS) | (a.vals_alias ? 0u : COPY_VALS);
            f[1] = BUF_IN;
        } else if (prev_dst == BUF_TMP) {
            f[0] = COPY_KEYS | COPY_VALS;
            f[1] = BUF_TMP;
        } else {
            f[0] = 0;
            f[1] = 0;
        }
        f[2] = BUF_OUT;
        f[3] = A;
    }
}

// ------------------------------------------------------------------ host

// 11-bit digits take the chunked reduce-then-scan pass, narrower ones the
// onesweep pass
template <int BITS>
constexpr bool chunked_pass() { return BITS == 11; }

template <typename K, int BITS>
static RadixGeom geom_of()
{
    using C = PassCfg<K, BITS>;
    if (chunked_pass<BITS>()) {
        using H = ChunkCfg<K, BITS>;
        return RadixGeom{BITS, H::RADIX, C::PASSES, H::NT, H::TILE, true};
    }
    return RadixGeom{BITS, C::RADIX, C::PASSES, C::NT, C::TILE, false};
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

// The histogram kernel counts the first pass's digits in chunks of
// consecutive tiles, one chunk per workgroup: about FIRST_PASS_CHUNKS chunks,
// of at most FIRST_PASS_TILES_PER_CHUNK tiles
constexpr uint64_t FIRST_PASS_CHUNKS = 1024;
// ... for 32-bit keys (with or without values) and at least this many
// tiles: there the first pass without look-back saves more than the scan
// over chunks costs (measured on 100M keys: keys only, the pass 0.286 ->
// 0.239 ms for 0.020 ms more in the histogram and the scan; with values
// 0.427 -> 0.411 ms; with 64-bit keys and values the first pass got slower)
constexpr uint64_t FIRST_PASS_MIN_TILES = 2048;

static bool scanned_first_pass(int key_bytes, bool, uint64_t tiles, bool chunked)
{
    return !chunked && key_bytes == 4 && tiles >= FIRST_PASS_MIN_TILES;
}

static uint32_t first_pass_tiles_per_chunk(uint64_t tiles)
{
    const uint64_t per = (tiles + FIRST_PASS_CHUNKS - 1) / FIRST_PASS_CHUNKS;
    return (uint32_t)std::min<uint64_t>(FIRST_PASS_TILES_PER_CHUNK, std::max<uint64_t>(1, per));
}

static uint32_t first_pass_chunks(uint64_t tiles)
{
    const uint64_t per = first_pass_tiles_per_chunk(tiles);
    return (uint32_t)std::max<uint64_t>(1, (tiles + per - 1) / per);
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
    if (L.g.chunked) {
        // per chunk and digit: counts, and where the chunk's runs start
        const uint64_t chunks = std::min<uint64_t>(L.num_tiles, ChunkCfg<uint32_t, 11>::MAX_CHUNKS);
        L.status_words = chunks * (uint64_t)L.g.radix;
    } else {
        // per tile and digit: one look-back word
        L.status_words = L.num_tiles * (uint64_t)L.g.radix;
    }
    L.status0 = take((size_t)L.status_words * 4);
    L.status1 = take((size_t)L.status_words * 4);
    // first pass, per tile and per chunk of tiles: digit offsets
    const bool scanned = scanned_first_pass(key_bytes, pairs, L.num_tiles, L.g.chunked);
    L.tile_offs = take(scanned ? (size_t)L.num_tiles * L.g.radix * 4 : 0);
    L.chunk_offs = take(scanned ? (size_t)first_pass_chunks(L.num_tiles) * L.g.radix * 4 : 0);
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

template <typename K, int BITS, int ORDER = 0>
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
    h.status0_words = finalize ? L.status_words : 0;
    h.n = (uint32_t)c.n;
    h.max_passes = (uint32_t)c.max_passes;
    h.skip = c.skip_constant_digits ? 1u : 0u;
    h.keys_alias = c.keys_in == c.keys_out ? 1u : 0u;
    h.vals_alias = c.pairs && c.vals_in == c.vals_out ? 1u : 0u;
    h.finalize = finalize ? 1u : 0u;
    h.copies = copies;
    const uint64_t nvec = c.n / (16 / sizeof(K));
    uint64_t blocks = (nvec + HIST_THREADS * HIST_UNROLL - 1) / (HIST_THREADS * HIST_UNROLL);
    const uint64_t cap = (uint64_t)current_cus() * HIST_BLOCKS_PER_CU;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    if (finalize && scanned_first_pass(c.key_bytes, c.pairs, L.num_tiles, chunked_pass<BITS>())) {
        // one chunk of whole tiles per workgroup, so that every tile's
        // first-pass counts come out of the same read
        h.tile_counts = reinterpret_cast<uint32_t *>(ws + L.tile_offs);
        h.chunk_sums = reinterpret_cast<uint32_t *>(ws + L.chunk_offs);
        h.num_tiles = (uint32_t)L.num_tiles;
        h.tiles_per_wg = first_pass_tiles_per_chunk(L.num_tiles);
        blocks = first_pass_chunks(L.num_tiles);
        h.num_chunks = (uint32_t)blocks;
    }
    bool launched = false;
    if constexpr (sizeof(K) == 4 && C::RADIX <= HIST_THREADS) {
        if (h.tile_counts) {
            hipLaunchKernelGGL((k_digit_histogram<K, BITS, ORDER, true>), dim3((uint32_t)blocks), dim3(HIST_THREADS),
                               0, s, static_cast<const K *>(c.keys_in), h);
            launched = true;
        }
    }
    if (!launched)
        hipLaunchKernelGGL((k_digit_histogram<K, BITS, ORDER, false>), dim3((uint32_t)blocks), dim3(HIST_THREADS), 0,
                           s, static_cast<const K *>(c.keys_in), h);
    if (t) t->mark(INTSORT_KERNEL_DIGIT_HISTOGRAM, 0, s);
    if (finalize) {
        // one workgroup plans; with per-tile first-pass counts, one more per
        // digit scans the chunk totals
        const uint32_t grid = h.tile_counts && C::RADIX <= HIST_THREADS ? (uint32_t)C::RADIX + 1 : 1u;
        hipLaunchKernelGGL((k_digit_plan<K, BITS>), dim3(grid), dim3(HIST_THREADS), 0, s, h);
        if (t) t->mark(INTSORT_KERNEL_PLAN, 0, s);
    }
    return hipGetLastError();
}

template <typename K, int BITS, bool PAIRS, int ORDER = 0>
static hipError_t run_typed(const RadixCall &c, hipStream_t s)
{
    using C = PassCfg<K, BITS>;
    const RadixLayout &L = c.L;
    char *ws = c.ws;
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    hipError_t e = launch_histogram<K, BITS, ORDER>(c, hist, true, s);
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
    a.tile_capacity = (uint32_t)L.num_tiles;
    const uint32_t *excl = reinterpret_cast<const uint32_t *>(ws + L.excl);
    const uint32_t *plan = reinterpret_cast<const uint32_t *>(ws + L.plan);
    for (int p = 0; p < C::PASSES && p < c.max_passes; p++) {
        a.plan = plan + p * PLAN_WORDS;
        a.pass = (uint32_t)p;
        using DG = OrderedDigit<ORDER>;
        const DG dg{(uint32_t)(p * BITS), (uint32_t)(C::RADIX - 1)};
        if constexpr (chunked_pass<BITS>()) {
            using H = ChunkCfg<K, BITS>;
            ChunkArgs ca{};
            ca.plan = a.plan;
            ca.n = (uint32_t)c.n;
            ca.tiles = (uint32_t)L.num_tiles;
            const uint64_t want =
                std::min<uint64_t>({L.num_tiles, (uint64_t)current_cus() * H::WG_PER_CU, (uint64_t)H::MAX_CHUNKS});
            ca.tpc = (uint32_t)((L.num_tiles + want - 1) / want);
            ca.chunks = (uint32_t)((L.num_tiles + ca.tpc - 1) / ca.tpc);
            ca.cnt = a.status0;
            ca.off = a.status1;
            ca.excl = excl + p * C::RADIX;
            ca.counters = a.counters;
            hipLaunchKernelGGL((k_chunk_count<K, BITS, DG>), dim3(ca.chunks), dim3(512), 0, s, a, ca, dg);
            hipLaunchKernelGGL(k_chunk_scan, dim3(C::RADIX), dim3(256), 0, s, ca, (uint32_t)C::RADIX);
            hipLaunchKernelGGL((k_chunk_sort<K, BITS, PAIRS, DG>), dim3(ca.chunks), dim3(H::NT), 0, s, a, ca, dg);
        } else {
            bool scanned = false;
            if constexpr (sizeof(K) == 4) {
                if (p == 0 && scanned_first_pass(c.key_bytes, c.pairs, L.num_tiles, false)) {
                    // the first pass's per-tile offsets are known: no look-back
                    const ScannedTiles tl{(uint32_t)c.n, (uint32_t)L.num_tiles,
                                          reinterpret_cast<const uint32_t *>(ws + L.tile_offs),
                                          reinterpret_cast<const uint32_t *>(ws + L.chunk_offs), (uint32_t)C::RADIX,
                                          first_pass_tiles_per_chunk(L.num_tiles)};
                    hipLaunchKernelGGL((k_onesweep<K, BITS, PAIRS, DG, ScannedTiles>), dim3((uint32_t)L.num_tiles),
                                       dim3(C::NT), 0, s, a, dg, tl);
                    scanned = true;
                }
            }
            if (!scanned) {
                const PlainTiles tl{(uint32_t)c.n, (uint32_t)L.num_tiles, excl + p * C::RADIX};
                hipLaunchKernelGGL((k_onesweep<K, BITS, PAIRS, DG, PlainTiles>), dim3((uint32_t)L.num_tiles),
                                   dim3(C::NT), 0, s, a, dg, tl);
            }
        }
        if (c.timer) c.timer->mark(INTSORT_KERNEL_PASS, (uint32_t)p, s);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // Out of place with at least one pass allowed, the plan routes the last
    // pass that runs (one always does) into the output, so nothing is left
    // to copy; otherwise the plan's final-copy words say what moves
    const bool in_place = c.keys_in == c.keys_out || (c.pairs && c.vals_in == c.vals_out);
    if (in_place || c.max_passes <= 0) {
        uint64_t blocks = (c.n + 255) / 256;
        const uint64_t cap = (uint64_t)current_cus() * 4;
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL((k_plan_final_copy<K, PAIRS>), dim3((uint32_t)blocks), dim3(256), 0, s, a.in, a.out,
                           a.tmp, a.vin, a.vout, a.vtmp, plan + MAX_PASSES * PLAN_WORDS, (uint32_t)c.n);
    }
    if (c.timer) c.timer->mark(INTSORT_KERNEL_COPY, 0, s);
    return hipGetLastError();
}

template <typename K, bool PAIRS>
static hipError_t run_bits(const RadixCall &c, hipStream_t s)
{
    // signed and floating-point keys: 8-bit digits
    if (c.order != 0) {
        if (c.bits != 8) return hipErrorNotSupported;
        return c.order == 1 ? run_typed<K, 8, PAIRS, 1>(c, s) : run_typed<K, 8, PAIRS, 2>(c, s);
    }
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
