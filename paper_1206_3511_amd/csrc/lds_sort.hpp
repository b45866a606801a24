// lds_sort.hpp -- one workgroup sorts one short segment entirely on chip.
//
// This is the per-bucket sort of bucket sort (section 2.3, Algorithm 2 sorts
// every bucket with insertion sort, Algorithm 1) and the small-segment path of
// the segmented sort.  Any stable sort gives the same bytes; here it is an LSD
// radix sort over 8-bit digits whose passes never leave LDS: each pass ranks
// the keys stably (wave_rank_atomic plus a scan over digits and waves) and reorders
// them through LDS.  A digit that is the same for every key of the segment
// leaves it unchanged, so its pass is skipped.
#pragma once

#include <stdint.h>

#include "device_common.hpp"
#include "intsort.h"
#include "internal.hpp"
#include "onesweep.hpp"

namespace intsort {

// size classes of the on-chip sort: the capacity of one workgroup each
template <typename K>
struct SegClasses {
    static constexpr int NCLASS = 4;
    static constexpr uint32_t CAP0 = 64 * 4;       // one wave
    static constexpr uint32_t CAP1 = 256 * 8;
    static constexpr uint32_t CAP2 = 512 * 16;
    static constexpr uint32_t CAP3 = sizeof(K) == 4 ? 512 * 32 : 512 * 16;
    static constexpr uint32_t LDS_MAX = CAP3;      // above: the multi-workgroup path
};

// where the keys of segment s live: one packed array cut by offsets ...
struct PackedSrc {
    const void *in;
    void *out;
    const uint32_t *vin;
    uint32_t *vout;
    const uint64_t *offsets;     // [segments + 1]
    template <typename K>
    __device__ __forceinline__ void seg(uint64_t s, const K *&kin, K *&kout, const uint32_t *&vi, uint32_t *&vo,
                                        uint32_t &m, uint32_t &base) const
    {
        const uint64_t lo = offsets[s], hi = offsets[s + 1];
        m = hi > lo ? (uint32_t)(hi - lo) : 0u;
        base = (uint32_t)lo;
        kin = static_cast<const K *>(in) + lo;
        kout = static_cast<K *>(out) + lo;
        vi = vin ? vin + lo : nullptr;
        vo = vout ? vout + lo : nullptr;
    }
    // segment s keeps inside [0, n): offsets nondecreasing from 0 to n;
    // len is its length when it is valid
    __device__ bool valid(uint64_t s, uint64_t segments, uint64_t n, uint64_t &len) const
    {
        const uint64_t lo = offsets[s], hi = offsets[s + 1];
        len = hi > lo ? hi - lo : 0;
        return lo <= hi && hi <= n && (s != 0 || lo == 0) && (s + 1 != segments || hi == n);
    }
};

// ... or separate arrays, one descriptor each (keys only)
struct DescSrc {
    const intsort_segment_desc *d;
    template <typename K>
    __device__ __forceinline__ void seg(uint64_t s, const K *&kin, K *&kout, const uint32_t *&vi, uint32_t *&vo,
                                        uint32_t &m, uint32_t &base) const
    {
        const intsort_segment_desc e = d[s];
        m = (uint32_t)e.n;
        base = 0;
        kin = static_cast<const K *>(e.keys_in);
        kout = static_cast<K *>(e.keys_out);
        vi = nullptr;
        vo = nullptr;
    }
    // one array: at most n keys (the batch total), and 16-byte aligned,
    // non-null buffers when it is not empty; len is its length
    __device__ bool valid(uint64_t s, uint64_t, uint64_t n, uint64_t &len) const
    {
        const intsort_segment_desc e = d[s];
        len = e.n;
        if (e.n == 0) return true;
        const uintptr_t a = reinterpret_cast<uintptr_t>(e.keys_in), b = reinterpret_cast<uintptr_t>(e.keys_out);
        return e.n <= n && a != 0 && b != 0 && (a & 15u) == 0 && (b & 15u) == 0;
    }
};

template <class Src>
struct LdsSortArgs {
    Src src;
    const uint32_t *list;        // segment ids of this size class, or null:
    const uint32_t *list_count;  // device count of listed segments
    uint32_t direct_count;       // without a list, segments 0 .. direct_count-1
};

template <typename K, bool PAIRS, int NT, int IPT, class Src>
__global__ __launch_bounds__(NT) void k_lds_sort(LdsSortArgs<Src> a)
{
    constexpr int WAVES = NT / WAVE;
    constexpr int TILE = NT * IPT;
    constexpr int RADIX = 256;
    constexpr int PASSES = (int)sizeof(K);
    constexpr int DPT = RADIX > NT ? RADIX / NT : 1;
    __shared__ alignas(16) unsigned char s_raw[TILE * sizeof(K)];
    __shared__ uint32_t s_vstage[PAIRS ? TILE : 1];
    __shared__ uint32_t s_wcnt[WAVES * RADIX];
    __shared__ uint32_t s_excl[RADIX];
    __shared__ uint32_t s_scan[WAVES + 1];
    __shared__ K s_diff[WAVES];
    K *s_stage = reinterpret_cast<K *>(s_raw);

    uint32_t seg;
    if (a.list) {
        if (blockIdx.x >= *a.list_count) return;
        seg = a.list[blockIdx.x];
    } else {
        if (blockIdx.x >= a.direct_count) return;
        seg = blockIdx.x;
    }
    const K *kin;
    K *kout;
    const uint32_t *vin;
    uint32_t *vout;
    uint32_t m, base_unused;
    a.src.template seg<K>(seg, kin, kout, vin, vout, m, base_unused);   // m <= TILE by classification
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t lofs = wave * (IPT * WAVE) + lane;

    K k[IPT];
    uint32_t v[PAIRS ? IPT : 1];
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        const bool in = lofs + j * WAVE < m;
        k[j] = in ? kin[lofs + j * WAVE] : ~K(0);
        if (PAIRS) v[j] = in ? vin[lofs + j * WAVE] : 0u;
    }

    // bits in which some key differs from the first one
    const K ref = m > 0 ? kin[0] : K(0);
    K diff = 0;
#pragma unroll
    for (int j = 0; j < IPT; j++)
        if (lofs + j * WAVE < m) diff |= k[j] ^ ref;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) diff |= __shfl_xor(diff, off, WAVE);
    if (lane == 0) s_diff[wave] = diff;
    __syncthreads();
    diff = 0;
#pragma unroll
    for (int w = 0; w < WAVES; w++) diff |= s_diff[w];

    uint32_t *wcnt = s_wcnt + wave * RADIX;
    // slot j of this wave holds keys (index < m) or only padding; slots of
    // padding alone are neither ranked nor placed (the ranked slots are the
    // first ceil(m / 64) of the segment, so the placed keys take positions
    // 0 .. 64 ceil(m / 64) - 1, the real ones 0 .. m - 1)
    const uint32_t wbase = __builtin_amdgcn_readfirstlane(wave * (uint32_t)(IPT * WAVE));
    auto live = [&](int j) { return wbase + (uint32_t)(j * WAVE) < m; };

    // One stable counting pass on bits shift .. shift+7: every key's new
    // position goes to LDS (s_stage, s_vstage).
    auto rank_place = [&](uint32_t shift) {
        for (uint32_t i = tid; i < (uint32_t)(WAVES * RADIX); i += NT) s_wcnt[i] = 0;
        __syncthreads();
        uint32_t rk[IPT];
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            rk[j] = 0;
            if (!live(j)) continue;
            const uint32_t d = lofs + j * WAVE < m ? digit_at<K>(k[j], shift, 0xffu) : 0xffu;
            rk[j] = wave_rank_atomic(d, wcnt);
        }
        __syncthreads();
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
            }
            mine += tcnt[i];
        }
        uint32_t total_unused;
        uint32_t ex = block_exclusive_scan<NT>(mine, s_scan, &total_unused);
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const uint32_t d = tid * DPT + i;
            if (d < (uint32_t)RADIX) s_excl[d] = ex;
            ex += tcnt[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            if (!live(j)) continue;
            const uint32_t d = lofs + j * WAVE < m ? digit_at<K>(k[j], shift, 0xffu) : 0xffu;
            const uint32_t pos = s_excl[d] + s_wcnt[wave * RADIX + d] + rk[j];
            s_stage[pos] = k[j];
            if (PAIRS) s_vstage[pos] = v[j];
        }
        __syncthreads();
    };
    // padding keys took the largest digit and the last positions, so the
    // first m positions hold the segment in its new order
    auto read_back = [&]() {
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            if (!live(j)) continue;
            k[j] = s_stage[lofs + j * WAVE];
            if (PAIRS) v[j] = s_vstage[lofs + j * WAVE];
        }
        __syncthreads();
    };

    for (int p = 0; p < PASSES; p++) {
        const uint32_t shift = 8u * (uint32_t)p;
        if (((diff >> shift) & 0xffu) == 0) continue;   // the same for every workgroup thread
        rank_place(shift);
        read_back();
    }
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        if (lofs + j * WAVE < m) {
            kout[lofs + j * WAVE] = k[j];
            if (PAIRS) vout[lofs + j * WAVE] = v[j];
        }
    }
}

// The same sort for segments of 64-bit keys, which differ in up to eight
// bytes.  Every key's varying bytes go once into byte planes in LDS, and the
// passes move 16-bit element indices instead of the keys and values: a pass
// reads one digit byte and writes and reads one index per key, against eight
// key and four value bytes written and read.  At the end the keys go back
// into LDS (where the byte planes were) and the sorted keys are gathered
// from there, the values from the segment's input (every gather is done
// before any store, so the sort may run in place).
template <typename K, bool PAIRS, int NT, int IPT, class Src>
__global__ __launch_bounds__(NT) void k_lds_sort_idx(LdsSortArgs<Src> a)
{
    constexpr int WAVES = NT / WAVE;
    constexpr int TILE = NT * IPT;
    constexpr int RADIX = 256;
    constexpr int KB = (int)sizeof(K);
    constexpr int DPT = RADIX > NT ? RADIX / NT : 1;
    static_assert(TILE <= 65536, "16-bit element indices");
    // byte p of element e at s_dig[p * TILE + e]; after the passes, the keys
    __shared__ alignas(16) uint8_t s_dig[KB * TILE];
    __shared__ uint16_t s_idx[TILE];
    __shared__ uint32_t s_wcnt[WAVES * RADIX];
    __shared__ uint32_t s_excl[RADIX];
    __shared__ uint32_t s_scan[WAVES + 1];
    __shared__ K s_diff[WAVES];

    uint32_t seg;
    if (a.list) {
        if (blockIdx.x >= *a.list_count) return;
        seg = a.list[blockIdx.x];
    } else {
        if (blockIdx.x >= a.direct_count) return;
        seg = blockIdx.x;
    }
    const K *kin;
    K *kout;
    const uint32_t *vin;
    uint32_t *vout;
    uint32_t m, base_unused;
    a.src.template seg<K>(seg, kin, kout, vin, vout, m, base_unused);   // m <= TILE by classification
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
    const uint32_t lofs = wave * (IPT * WAVE) + lane;
    // slots of padding alone (index >= m for the whole wave) are skipped,
    // as in k_lds_sort
    const uint32_t wbase = __builtin_amdgcn_readfirstlane(wave * (uint32_t)(IPT * WAVE));
    auto live = [&](int j) { return wbase + (uint32_t)(j * WAVE) < m; };

    K k[IPT];
#pragma unroll
    for (int j = 0; j < IPT; j++) k[j] = lofs + j * WAVE < m ? kin[lofs + j * WAVE] : ~K(0);
    const K ref = m > 0 ? kin[0] : K(0);
    K diff = 0;
#pragma unroll
    for (int j = 0; j < IPT; j++)
        if (lofs + j * WAVE < m) diff |= k[j] ^ ref;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) diff |= __shfl_xor(diff, off, WAVE);
    if (lane == 0) s_diff[wave] = diff;
    __syncthreads();
    diff = 0;
#pragma unroll
    for (int w = 0; w < WAVES; w++) diff |= s_diff[w];

    // byte planes of the bytes that vary (padding keys are all ones, so
    // their digits are the largest and they rank last)
#pragma unroll
    for (int p = 0; p < KB; p++) {
        if (((diff >> (8 * p)) & 0xffu) == 0) continue;
#pragma unroll
        for (int j = 0; j < IPT; j++)
            if (live(j)) s_dig[p * TILE + lofs + j * WAVE] = (uint8_t)(k[j] >> (8 * p));
    }
    uint32_t e[IPT];   // the element at each of this thread's positions
#pragma unroll
    for (int j = 0; j < IPT; j++) e[j] = lofs + j * WAVE;
    __syncthreads();

    uint32_t *wcnt = s_wcnt + wave * RADIX;
    for (int p = 0; p < KB; p++) {
        if (((diff >> (8 * p)) & 0xffu) == 0) continue;   // the same for every workgroup thread
        for (uint32_t i = tid; i < (uint32_t)(WAVES * RADIX); i += NT) s_wcnt[i] = 0;
        __syncthreads();
        const uint8_t *plane = s_dig + p * TILE;
        uint32_t d[IPT], rk[IPT];
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            d[j] = 0;
            rk[j] = 0;
            if (!live(j)) continue;
            d[j] = plane[e[j]];
            rk[j] = wave_rank_atomic(d[j], wcnt);
        }
        __syncthreads();
        uint32_t tcnt[DPT];
        uint32_t mine = 0;
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const uint32_t dd = tid * DPT + i;
            tcnt[i] = 0;
            if (dd < (uint32_t)RADIX) {
                uint32_t run = 0;
#pragma unroll
                for (int w = 0; w < WAVES; w++) {
                    const uint32_t c = s_wcnt[w * RADIX + dd];
                    s_wcnt[w * RADIX + dd] = run;
                    run += c;
                }
                tcnt[i] = run;
            }
            mine += tcnt[i];
        }
        uint32_t total_unused;
        uint32_t ex = block_exclusive_scan<NT>(mine, s_scan, &total_unused);
#pragma unroll
        for (int i = 0; i < DPT; i++) {
            const uint32_t dd = tid * DPT + i;
            if (dd < (uint32_t)RADIX) s_excl[dd] = ex;
            ex += tcnt[i];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++) {
            if (!live(j)) continue;
            s_idx[s_excl[d[j]] + s_wcnt[wave * RADIX + d[j]] + rk[j]] = (uint16_t)e[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; j++)
            if (live(j)) e[j] = s_idx[lofs + j * WAVE];
        __syncthreads();
    }
    // the first m positions hold the real elements in sorted order; every
    // gather completes before the barrier, so no store overwrites a key or
    // value another thread still reads
    K *s_keys = reinterpret_cast<K *>(s_dig);   // TILE keys fill the planes' bytes
#pragma unroll
    for (int j = 0; j < IPT; j++)
        if (lofs + j * WAVE < m) s_keys[lofs + j * WAVE] = k[j];
    __syncthreads();
    uint32_t v[PAIRS ? IPT : 1];
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        if (lofs + j * WAVE < m) {
            k[j] = s_keys[e[j]];
            if (PAIRS) v[j] = vin[e[j]];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; j++) {
        if (lofs + j * WAVE < m) {
            kout[lofs + j * WAVE] = k[j];
            if (PAIRS) vout[lofs + j * WAVE] = v[j];
        }
    }
}

}  // namespace intsort
