// chunk_sort.hpp -- one LSD radix pass as reduce-then-scan, used for 11-bit
// digits.
//
// The pass is the placement loop of COUNTING-SORT (section 2.4, Algorithm 3)
// over the whole array, split the other way round from the onesweep kernel:
//
//   k_chunk_count  the digit counts of every chunk (a run of consecutive
//                  tiles), one read of the keys
//   k_chunk_scan   for every digit, where each chunk's run of that digit
//                  starts: the pass's global digit offset plus the counts of
//                  the digit in all earlier chunks
//   k_chunk_sort   every workgroup walks the tiles of its chunk in order; it
//                  sorts a tile stably by the digit in LDS, writes each
//                  digit's run at the chunk's running offset, and advances
//                  the offsets by the tile's counts
//
// With 2^11 digits a decoupled look-back between tiles has to move 8 KB of
// status per tile and step; here no workgroup ever waits for another, at the
// price of one more read of the keys per pass.
//
// The in-tile sort is itself an LSD sort by SB-bit sub-digits: every thread
// holds IPT consecutive keys of the tile, counts its sub-digits in private
// LDS counters (an atomic add returns the key's rank among the thread's
// earlier keys with the same sub-digit), a raking scan over (sub-digit,
// thread) turns the counts into offsets, and the keys move to their places
// through the stage.
#pragma once

#include <stdint.h>

#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"
#include "onesweep.hpp"

namespace intsort {

template <typename K, int BITS>
struct ChunkCfg {
    static constexpr int NT = 512;
    static constexpr int IPT = 96 / (int)sizeof(K);   // 96 bytes of keys per thread
    static constexpr int TILE = NT * IPT;
    static constexpr int RADIX = 1 << BITS;
    static constexpr int SB = 4;                        // bits per in-tile sub-pass
    static constexpr int SR = 1 << SB;
    static constexpr int SUBS = (BITS + SB - 1) / SB;
    static constexpr int WG_PER_CU = 2;                 // two workgroups fill a CU's LDS
    static constexpr uint32_t MAX_CHUNKS = 4096;
};

struct ChunkArgs {
    const uint32_t *plan;    // this pass's plan words: active, src, dst, ordinal
    uint32_t n;              // keys
    uint32_t tiles;          // tiles of the array
    uint32_t tpc;            // tiles per chunk
    uint32_t chunks;
    uint32_t *cnt;           // [digit][chunk] counts
    uint32_t *off;           // [chunk][digit] start of the chunk's run
    const uint32_t *excl;    // [digit] exclusive global offsets of this pass
    uint32_t *counters;
};

// word w of the (sub-digit, thread) counter table; the 16-byte groups of
// every 32-word row are XOR-swizzled by the row, so that a thread reading its
// own 16 consecutive words and 32 threads reading one word each of a row
// both spread over the banks
__device__ __forceinline__ uint32_t cnt_word(uint32_t w) { return w ^ (((w >> 5) & 7u) << 2); }

// x[0..N) = elements t*N .. t*N+N-1 of an array of T in LDS
template <typename T, int N>
__device__ __forceinline__ void blocked_from_lds(const unsigned char *s, uint32_t t, T (&x)[N])
{
    static_assert((N * sizeof(T)) % 16 == 0, "whole 16-byte groups");
    constexpr int Q = N * sizeof(T) / 16;
    constexpr int PER = 16 / sizeof(T);
    const uint4 *p = reinterpret_cast<const uint4 *>(s + t * (uint32_t)(N * sizeof(T)));
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const uint4 v = p[q];
        const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
        for (int i = 0; i < PER; i++) x[q * PER + i] = e[i];
    }
}

// x[0..N) = g[0..N) with 16-byte loads (g 16-byte aligned)
template <typename T, int N>
__device__ __forceinline__ void blocked_from_global(const T *g, T (&x)[N])
{
    constexpr int Q = N * sizeof(T) / 16;
    constexpr int PER = 16 / sizeof(T);
    const uint4 *p4 = reinterpret_cast<const uint4 *>(g);
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const uint4 v = p4[q];
        const T *e = reinterpret_cast<const T *>(&v);
#pragma unroll
        for (int i = 0; i < PER; i++) x[q * PER + i] = e[i];
    }
}

// a tile of `valid` elements (padded with `fill`) in blocked order, read
// striped from global memory and transposed through LDS
template <typename T, int N, int NT>
__device__ __forceinline__ void blocked_via_lds(const T *src, uint32_t valid, T fill, unsigned char *s, T (&x)[N])
{
    const uint32_t tid = threadIdx.x;
    T *st = reinterpret_cast<T *>(s);
#pragma unroll
    for (int j = 0; j < N; j++) {
        const uint32_t i = j * NT + tid;
        st[i] = i < valid ? src[i] : fill;
    }
    __syncthreads();
    blocked_from_lds<T, N>(s, tid, x);
    __syncthreads();
}

// digit counts of every chunk
template <typename K, int BITS, class DG>
__global__ __launch_bounds__(512) void k_chunk_count(PassArgs<K> a, ChunkArgs ca, DG dg)
{
    using C = ChunkCfg<K, BITS>;
    constexpr int RADIX = C::RADIX, TILE = C::TILE;
    constexpr int NW = 512 / WAVE;
    constexpr int KPV = 16 / (int)sizeof(K);
    constexpr int U = 4;   // 16-byte loads in flight per thread
    __shared__ uint32_t s_h[NW * RADIX];   // one histogram per wave
    if (ca.plan[0] == 0) return;
    const K *src = ca.plan[1] == BUF_IN ? a.in : (ca.plan[1] == BUF_OUT ? a.out : a.tmp);
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < (uint32_t)(NW * RADIX); i += 512) s_h[i] = 0;
    __syncthreads();
    uint32_t *h = s_h + (tid / WAVE) * RADIX;
    const uint64_t lo = (uint64_t)blockIdx.x * ca.tpc * TILE;
    const uint64_t hi = min((uint64_t)ca.n, lo + (uint64_t)ca.tpc * TILE);
    // lo is a multiple of the tile, so the chunk starts 16-byte aligned
    const uint32_t nv = lo < hi ? (uint32_t)((hi - lo) / KPV) : 0u;
    const uint4 *v4 = reinterpret_cast<const uint4 *>(src + lo);
    for (uint32_t v0 = tid; v0 < nv; v0 += 512 * U) {
        uint4 x[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            if (v0 + u * 512 < nv) x[u] = v4[v0 + u * 512];
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (v0 + u * 512 < nv) {
                const K *e = reinterpret_cast<const K *>(&x[u]);
#pragma unroll
                for (int q = 0; q < KPV; q++) lds_count(h, dg(e[q]));
            }
        }
    }
    for (uint64_t i = lo + (uint64_t)nv * KPV + tid; i < hi; i += 512) lds_count(h, dg(src[i]));
    __syncthreads();
    for (uint32_t d = tid; d < (uint32_t)RADIX; d += 512) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) s += s_h[w * RADIX + d];
        ca.cnt[(uint64_t)d * ca.chunks + blockIdx.x] = s;
    }
}

// one workgroup per digit: exclusive scan of the digit's chunk counts,
// starting at the digit's global offset
__global__ __launch_bounds__(256) void k_chunk_scan(ChunkArgs ca, uint32_t radix)
{
    __shared__ uint32_t s_tmp[256 / WAVE];
    if (ca.plan[0] == 0) return;
    const uint32_t d = blockIdx.x, tid = threadIdx.x;
    const uint32_t per = (ca.chunks + 255) / 256;
    const uint32_t c0 = tid * per;
    const uint32_t *cnt = ca.cnt + (uint64_t)d * ca.chunks;
    uint32_t sum = 0;
    for (uint32_t i = 0; i < per; i++)
        if (c0 + i < ca.chunks) sum += cnt[c0 + i];
    uint32_t run = block_scan_1b<256>(sum, s_tmp) + ca.excl[d];
    for (uint32_t i = 0; i < per; i++) {
        if (c0 + i < ca.chunks) {
            ca.off[(uint64_t)(c0 + i) * radix + d] = run;
            run += cnt[c0 + i];
        }
    }
}

template <typename K, int BITS, bool PAIRS, class DG>
__global__ __launch_bounds__((ChunkCfg<K, BITS>::NT), (PAIRS ? 2 : 4)) void k_chunk_sort(PassArgs<K> a, ChunkArgs ca,
                                                                                     DG dg)
{
    using C = ChunkCfg<K, BITS>;
    constexpr int RADIX = C::RADIX, NT = C::NT, IPT = C::IPT, TILE = C::TILE;
    constexpr int SB = C::SB, SR = C::SR, SUBS = C::SUBS;
    constexpr int DPT = RADIX > NT ? RADIX / NT : 1;   // digits per thread
    constexpr int CWORDS = SR * NT;
    constexpr int STAGE = TILE * (int)sizeof(K);
    constexpr int HIST0 = 64;                          // word offset of the tile histogram in the stage
    static_assert(RADIX <= NT * DPT, "every digit has a thread");
    static_assert(RADIX <= CWORDS, "digit bases fit the counter area");
    static_assert(NT / WAVE <= HIST0 && (HIST0 + RADIX) * 4 <= STAGE, "histogram fits the stage");
    static_assert(SR == 16 && (NT % 256) == 0, "counter layout");
    static_assert(TILE * sizeof(uint32_t) <= STAGE, "values fit the stage");

    __shared__ alignas(16) unsigned char s_stage[STAGE];
    __shared__ alignas(16) uint32_t s_cnt[CWORDS];
    // the stage is idle while these are live
    uint32_t *s_scan = reinterpret_cast<uint32_t *>(s_stage);
    uint32_t *s_hist = reinterpret_cast<uint32_t *>(s_stage) + HIST0;
    // after the last sub-pass the counters hold the global base of every run
    uint32_t *s_gbase = s_cnt;
    K *s_keys = reinterpret_cast<K *>(s_stage);
    uint32_t *s_vals = reinterpret_cast<uint32_t *>(s_stage);

    if (ca.plan[0] == 0) return;   // pass skipped
    const uint32_t srcc = ca.plan[1], dstc = ca.plan[2];
    const K *src = srcc == BUF_IN ? a.in : (srcc == BUF_OUT ? a.out : a.tmp);
    K *dst = dstc == BUF_OUT ? a.out : a.tmp;
    const uint32_t *vsrc = nullptr;
    uint32_t *vdst = nullptr;
    if (PAIRS) {
        vsrc = srcc == BUF_IN ? a.vin : (srcc == BUF_OUT ? a.vout : a.vtmp);
        vdst = dstc == BUF_OUT ? a.vout : a.vtmp;
    }
    const uint32_t tid = threadIdx.x;
    const uint32_t n = ca.n;
    // this thread's counter of sub-digit s is word s*NT + ccol (the swizzle
    // term depends on the thread only, NT being a multiple of 256)
    const uint32_t ccol = cnt_word(tid);

    // running start of every digit's run for this chunk
    uint32_t run[DPT];
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const uint32_t d = tid * DPT + i;
        run[i] = d < (uint32_t)RADIX ? ca.off[(uint64_t)blockIdx.x * RADIX + d] : 0u;
    }

    const uint32_t t_end = min(ca.tiles, (blockIdx.x + 1) * ca.tpc);
    for (uint32_t tile = blockIdx.x * ca.tpc; tile < t_end; tile++) {
        const uint32_t start = tile * (uint32_t)TILE;
        const uint32_t valid = min((uint32_t)TILE, n - start);
#pragma unroll
        for (int d = 0; d < SR; d++) s_cnt[d * NT + ccol] = 0;
        for (uint32_t d = tid; d < (uint32_t)RADIX; d += NT) s_hist[d] = 0;
        __syncthreads();

        // ---- the tile in blocked order: thread t holds positions t*IPT ..;
        // padding past the end is the largest key, whose digit is the
        // largest, so it sorts after every key
        K k[IPT];
        uint32_t v[IPT];
        if (valid == (uint32_t)TILE) {
            blocked_from_global<K, IPT>(src + start + (uint64_t)tid * IPT, k);
            if constexpr (PAIRS) blocked_from_global<uint32_t, IPT>(vsrc + start + (uint64_t)tid * IPT, v);
        } else {
            blocked_via_lds<K, IPT, NT>(src + start, valid, dg.template pad<K>(), s_stage, k);
            if constexpr (PAIRS) blocked_via_lds<uint32_t, IPT, NT>(vsrc + start, valid, 0u, s_stage, v);
            for (uint32_t d = tid; d < (uint32_t)RADIX; d += NT) s_hist[d] = 0;
            __syncthreads();
        }

        // ---- the tile's digit counts and their exclusive scan
#pragma unroll
        for (int j = 0; j < IPT; j++)
            if (tid * IPT + j < valid) lds_count(s_hist, dg(k[j]));
        __syncthreads();
        uint32_t tcnt[DPT], texcl[DPT];
        {
            uint32_t mine = 0;
#pragma unroll
            for (int i = 0; i < DPT; i++) {
                const uint32_t d = tid * DPT + i;
                tcnt[i] = d < (uint32_t)RADIX ? s_hist[d] : 0u;
                mine += tcnt[i];
            }
            texcl[0] = block_scan_1b<NT>(mine, s_scan);
#pragma unroll
            for (int i = 1; i < DPT; i++) texcl[i] = texcl[i - 1] + tcnt[i - 1];
        }

        // ---- stable in-tile sort by the digit, SB bits at a time, least
        // significant first.  A thread's counters are touched by other
        // threads only between the two barriers around the raking scan.
        uint32_t rk[IPT];
#pragma unroll
        for (int sp = 0; sp < SUBS; sp++) {
            const uint32_t lo = sp * SB;
            const uint32_t w = (BITS - (int)lo) < SB ? (BITS - lo) : SB;
#pragma unroll
            for (int j = 0; j < IPT; j++)
                rk[j] = __hip_atomic_fetch_add(&s_cnt[dg.sub(k[j], lo, w) * NT + ccol], 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
            __syncthreads();
            {
                // thread t rakes counter words 16t .. 16t+15 (one sub-digit
                // row, consecutive threads): exclusive offsets in
                // (sub-digit, thread) order
                uint32_t x[SR];
                const uint32_t r0 = cnt_word(tid * SR);
#pragma unroll
                for (int q = 0; q < SR / 4; q++) {
                    const uint4 g = *reinterpret_cast<const uint4 *>(&s_cnt[r0 ^ (4u * q)]);
                    x[4 * q] = g.x;
                    x[4 * q + 1] = g.y;
                    x[4 * q + 2] = g.z;
                    x[4 * q + 3] = g.w;
                }
                uint32_t sum = 0;
#pragma unroll
                for (int i = 0; i < SR; i++) {
                    const uint32_t c = x[i];
                    x[i] = sum;
                    sum += c;
                }
                const uint32_t base = block_scan_1b<NT>(sum, s_scan);
#pragma unroll
                for (int q = 0; q < SR / 4; q++)
                    *reinterpret_cast<uint4 *>(&s_cnt[r0 ^ (4u * q)]) =
                        make_uint4(base + x[4 * q], base + x[4 * q + 1], base + x[4 * q + 2], base + x[4 * q + 3]);
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IPT; j++) {
                rk[j] += s_cnt[dg.sub(k[j], lo, w) * NT + ccol];
                s_keys[rk[j]] = k[j];
            }
            if (sp + 1 < SUBS) {
#pragma unroll
                for (int d = 0; d < SR; d++) s_cnt[d * NT + ccol] = 0;
            }
            __syncthreads();
            if (sp + 1 < SUBS) {
                blocked_from_lds<K, IPT>(s_stage, tid, k);
                if constexpr (PAIRS) {
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < IPT; j++) s_vals[rk[j]] = v[j];
                    __syncthreads();
                    blocked_from_lds<uint32_t, IPT>(s_stage, tid, v);
                }
            }
        }

        // ---- the tile is in digit order: digit d's run goes to
        // run[d] .. run[d] + tcnt[d]
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const uint32_t d = tid * DPT + i;
            if (d < (uint32_t)RADIX) {
                s_gbase[d] = run[i] - texcl[i];
                run[i] += tcnt[i];
            }
        }
#pragma unroll
        for (int m = 0; m < IPT; m++) k[m] = s_keys[m * NT + tid];
        __syncthreads();
        if constexpr (PAIRS) {
#pragma unroll
            for (int j = 0; j < IPT; j++) s_vals[rk[j]] = v[j];
            __syncthreads();
        }
        bool bad = false;
#pragma unroll
        for (int m = 0; m < IPT; m++) {
            const uint32_t i = m * NT + tid;
            if (i < valid) {
                const uint32_t g = s_gbase[dg(k[m])] + i;
                if (g < n) {
                    dst[g] = k[m];
                    if constexpr (PAIRS) vdst[g] = s_vals[i];
                } else {
                    bad = true;
                }
            }
        }
        if (bad) atomicOr(&ca.counters[CTR_ERROR], DEVERR_SCATTER_RANGE);
        // the next tile reuses the stage and the counters
        __syncthreads();
    }
}

}  // namespace intsort
