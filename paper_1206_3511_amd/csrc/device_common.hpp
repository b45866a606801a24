// device_common.hpp -- wave64 and workgroup primitives shared by the gfx950
// kernels of the sort library (no sorting arithmetic lives here).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace intsort {

constexpr int WAVE = 64;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// number of set bits of `mask` in lanes below the calling lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t first_lane_value(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

// compiler-level ordering point for LDS traffic of one wave (LDS operations
// of a wave execute in issue order in hardware)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- device-wide (agent scope) relaxed atomics on status words; every XCD
// sees them, whatever L2 the writer sits behind
__device__ __forceinline__ uint32_t load_agent(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint32_t *p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// inclusive scan across the 64 lanes of a wave (every lane active): sums
// inside rows of 16 lanes by shifted DPP adds, then each row adds the total of
// the rows before it through the row broadcasts of lanes 15 and 31
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x)
{
    // DPP controls: row_shr:n = 0x110 + n, row_bcast:15 = 0x142, row_bcast:31 = 0x143;
    // lanes without a source (or in rows the row mask leaves out) add 0
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    return x;
}

// Exclusive scan of one value per thread over a workgroup of NT threads.
// s_tmp needs NT/64 + 1 words.  Returns the exclusive prefix; *total gets the
// sum of all values.  Contains barriers: every thread must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total)
{
    constexpr int NW = NT / WAVE;
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / WAVE;
    uint32_t incl = wave_inclusive_scan(v);
    if (lane == WAVE - 1) s_tmp[wave] = incl;
    __syncthreads();
    if (threadIdx.x < WAVE) {
        uint32_t t = (lane < (uint32_t)NW) ? s_tmp[lane] : 0u;
        uint32_t ti = wave_inclusive_scan(t);
        if (lane < (uint32_t)NW) s_tmp[lane] = ti - t;
        if (lane == (uint32_t)NW - 1) s_tmp[NW] = ti;
    }
    __syncthreads();
    uint32_t res = incl - v + s_tmp[wave];
    *total = s_tmp[NW];
    __syncthreads();
    return res;
}

// Exclusive scan of one value per thread over NT threads with a single
// barrier.  s_tmp needs NT/64 words and must not be written again before the
// caller's next barrier.
template <int NT>
__device__ __forceinline__ uint32_t block_scan_1b(uint32_t v, uint32_t *s_tmp)
{
    constexpr int NW = NT / WAVE;
    const uint32_t wave = threadIdx.x / WAVE;
    const uint32_t incl = wave_inclusive_scan(v);
    if (lane_id() == WAVE - 1) s_tmp[wave] = incl;
    __syncthreads();
    uint32_t below = 0;
#pragma unroll
    for (int w = 0; w < NW; w++)
        if ((uint32_t)w < wave) below += s_tmp[w];
    return below + incl - v;
}

// Adds one to bin d of an LDS histogram.  Lanes that hit one word in one
// atomic instruction are served one after another, so the lanes that share
// the first active lane's bin add as one group: that lane adds the group's
// size, and every lane with another bin adds one, all in one instruction.  A
// wave of sorted or nearly sorted keys then costs one or a few adds instead
// of up to 64 on one word; keys spread over many bins pay one compare more.
__device__ __forceinline__ void lds_count(uint32_t *s_h, uint32_t d)
{
    const uint32_t lane = lane_id();
    const bool lead = lane == first_lane_value(lane);   // the lane d0 comes from
    const uint32_t d0 = first_lane_value(d);
    const uint64_t same = ballot(d == d0);
    if (d != d0 || lead) atomicAdd(&s_h[d], lead ? popc64(same) : 1u);
}

}  // namespace intsort

namespace intsort {

// fills p[0..n) with v (grid-stride); a kernel, so that it can sit in a
// captured graph where memset nodes are avoided
template <typename T>
__global__ void k_fill(T *p, uint64_t n, T v)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

}  // namespace intsort
