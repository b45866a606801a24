// rank_check.hip -- the device self-test behind the choice of the stable
// in-wave rank of the pass kernel.
//
// The pass ranks a key by one LDS atomic add with return on its wave's digit
// counter.  That rank is stable only if the lanes of one add instruction that
// hit the same counter receive the old values in lane order.  The ISA does
// not state that order, so intsort_create runs this check on its device
// once: every wave of a grid adds into its own LDS counters with many digit
// patterns (one to 256 distinct counters, some lanes switched off) and
// compares each returned value with the rank that ballots give.  A device
// with any mismatch is refused (intsort_create returns
// INTSORT_ERR_UNSUPPORTED) rather than sorted unstably.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.hpp"
#include "internal.hpp"

namespace intsort {

namespace {

constexpr int CHECK_BLOCKS = 1024;
constexpr int CHECK_THREADS = 256;
constexpr int CHECK_ITERS = 256;

__device__ __forceinline__ uint64_t check_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(CHECK_THREADS) void k_rank_order_check(uint32_t *mismatches)
{
    constexpr int WAVES = CHECK_THREADS / WAVE;
    __shared__ uint32_t cnt[WAVES * 256];
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / WAVE;
    uint32_t *c = cnt + wave * 256;
    for (uint32_t i = lane; i < 256; i += WAVE) c[i] = 0;
    wave_sync();
    uint32_t bad = 0;
    for (int it = 0; it < CHECK_ITERS; it++) {
        const uint64_t h = check_mix(((uint64_t)blockIdx.x << 24) ^ ((uint64_t)it << 10) ^ threadIdx.x);
        const uint64_t hw = check_mix(((uint64_t)blockIdx.x << 24) ^ ((uint64_t)it << 10) ^ (wave + 512));
        const uint32_t kind = (uint32_t)(hw & 7);
        const uint32_t width = kind == 0 ? 0u : kind == 1 ? 1u : kind == 2 ? 2u : kind == 3 ? 4u : 8u;
        uint32_t d = (uint32_t)(h >> 32) & ((1u << width) - 1u);
        if (kind == 5) d = (lane * 7u + (uint32_t)(hw >> 8)) & 255u;
        if (kind == 6) d = (uint32_t)(hw >> 16) & 255u;
        if (kind == 7) d = ((h >> 40) & 1) ? (uint32_t)(hw >> 24) & 255u : (uint32_t)(hw >> 32) & 255u;
        const bool on = ((hw >> 48) & 3) != 0 || ((h >> 20) & 1);
        // peers of the lane by ballots over the counter index
        uint64_t peers = ballot(on);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool set = (d >> b) & 1u;
            const uint64_t m = ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t before = c[d];
        wave_sync();
        if (on) {
            const uint32_t r = atomicAdd(&c[d], 1u);
            if (r != before + mbcnt(peers)) bad++;
        }
        wave_sync();
        if ((it & 63) == 63) {
            for (uint32_t i = lane; i < 256; i += WAVE) c[i] = 0;
            wave_sync();
        }
    }
    if (bad) atomicAdd(mismatches, bad);
}

std::mutex g_lock;
int g_state[64];   // 0 not checked, 1 lane-ordered atomics, 2 not

}  // namespace

hipError_t rank_check(int device, bool *ok)
{
    *ok = false;
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_lock);
    if (g_state[device] != 0) {
        *ok = g_state[device] == 1;
        return hipSuccess;
    }
    hipError_t e;
    uint32_t *d = nullptr;
    uint32_t h = 1;
    if ((e = hipMalloc(&d, sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMemset(d, 0, sizeof(uint32_t))) == hipSuccess) {
        hipLaunchKernelGGL(k_rank_order_check, dim3(CHECK_BLOCKS), dim3(CHECK_THREADS), 0, 0, d);
        if ((e = hipGetLastError()) == hipSuccess) e = hipMemcpy(&h, d, sizeof(uint32_t), hipMemcpyDeviceToHost);
    }
    hipFree(d);
    if (e != hipSuccess) return e;
    g_state[device] = h == 0 ? 1 : 2;
    *ok = h == 0;
    return hipSuccess;
}

}  // namespace intsort
