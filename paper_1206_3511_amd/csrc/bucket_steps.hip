// bucket_steps.hip -- the first two steps of bucket sort (section 2.3,
// Algorithm 2) as stand-alone kernels: the value range of the keys (min and
// max, which replace the paper's assumed bound M), and the histogram of the
// exact bucket index b(k) = floor((k - min) * B / (max - min + 1)).

#include <stdint.h>

#include "bucket_map.hpp"
#include "device_common.hpp"
#include "internal.hpp"
#include "sort_plans.hpp"

namespace intsort {

// one workgroup per CU: every workgroup ends with one atomic min and max on
// the same two words, so fewer, larger workgroups queue less there
constexpr int MM_THREADS = 1024;
constexpr int MM_UNROLL = 4;

__global__ void k_minmax_init(uint64_t *minmax, uint64_t *sorted)
{
    minmax[0] = ~0ull;
    minmax[1] = 0;
    if (sorted) *sorted = 1;
}

// min and max over all keys: per-thread, per-wave, per-workgroup, then one
// pair of device-wide atomics per workgroup.  With `sorted`, also whether
// the keys are already in nondecreasing order: a workgroup that sees a key
// smaller than the one before it clears the flag.
template <typename K>
__global__ __launch_bounds__(MM_THREADS) void k_minmax(const K *__restrict__ keys, uint64_t n,
                                                       uint64_t *__restrict__ minmax, uint64_t *sorted)
{
    constexpr int KPV = 16 / (int)sizeof(K);
    struct alignas(16) Vec { K v[KPV]; };
    __shared__ uint64_t s_min[MM_THREADS / WAVE], s_max[MM_THREADS / WAVE];
    K lo = ~K(0), hi = 0;
    bool order_ok = true;
    const bool check = sorted != nullptr;
    const uint64_t nvec = n / KPV;
    const Vec *vk = reinterpret_cast<const Vec *>(keys);
    // MM_UNROLL 16-byte loads in flight per thread
    const uint64_t step = (uint64_t)gridDim.x * MM_THREADS * MM_UNROLL;
    for (uint64_t v0 = (uint64_t)blockIdx.x * MM_THREADS * MM_UNROLL + threadIdx.x; v0 < nvec; v0 += step) {
        Vec x[MM_UNROLL];
#pragma unroll
        for (int u = 0; u < MM_UNROLL; u++)
            if (v0 + (uint64_t)u * MM_THREADS < nvec) x[u] = vk[v0 + (uint64_t)u * MM_THREADS];
#pragma unroll
        for (int u = 0; u < MM_UNROLL; u++) {
            const uint64_t v = v0 + (uint64_t)u * MM_THREADS;
            if (check && !vector_in_order<K, KPV>(x[u].v, keys, v, nvec)) order_ok = false;
            if (v < nvec) {
#pragma unroll
                for (int e = 0; e < KPV; e++) {
                    lo = x[u].v[e] < lo ? x[u].v[e] : lo;
                    hi = x[u].v[e] > hi ? x[u].v[e] : hi;
                }
            }
        }
    }
    const uint64_t stride = (uint64_t)gridDim.x * MM_THREADS;
    for (uint64_t i = nvec * KPV + (uint64_t)blockIdx.x * MM_THREADS + threadIdx.x; i < n; i += stride) {
        lo = keys[i] < lo ? keys[i] : lo;
        hi = keys[i] > hi ? keys[i] : hi;
        if (check && i > 0 && keys[i] < keys[i - 1]) order_ok = false;
    }
    if (check && __syncthreads_or(!order_ok) && threadIdx.x == 0) *sorted = 0;
    uint64_t l = lo, h = hi;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        uint64_t l2 = __shfl_xor(l, off, WAVE), h2 = __shfl_xor(h, off, WAVE);
        l = l2 < l ? l2 : l;
        h = h2 > h ? h2 : h;
    }
    const uint32_t wave = threadIdx.x / WAVE;
    if (lane_id() == 0) { s_min[wave] = l; s_max[wave] = h; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < MM_THREADS / WAVE; w++) {
            l = s_min[w] < l ? s_min[w] : l;
            h = s_max[w] > h ? s_max[w] : h;
        }
        // 32-bit keys keep their all-ones "no key seen" value out of the max
        atomicMin(reinterpret_cast<unsigned long long *>(&minmax[0]), (unsigned long long)l);
        atomicMax(reinterpret_cast<unsigned long long *>(&minmax[1]), (unsigned long long)h);
    }
}

hipError_t minmax_run(int key_bytes, const void *keys, uint64_t n, uint64_t *minmax, hipStream_t s,
                      uint64_t *sorted)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    uint64_t blocks = (n / (16 / key_bytes) + MM_THREADS * MM_UNROLL - 1) / (MM_THREADS * MM_UNROLL);
    const uint64_t cap = (uint64_t)device_cu_count(dev);
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_minmax_init, dim3(1), dim3(1), 0, s, minmax, sorted);
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_minmax<uint32_t>, dim3((uint32_t)blocks), dim3(MM_THREADS), 0, s,
                           static_cast<const uint32_t *>(keys), n, minmax, sorted);
    else
        hipLaunchKernelGGL(k_minmax<uint64_t>, dim3((uint32_t)blocks), dim3(MM_THREADS), 0, s,
                           static_cast<const uint64_t *>(keys), n, minmax, sorted);
    return hipGetLastError();
}

// ------------------------------------------------------- bucket histogram

constexpr int BH_THREADS = 512;
constexpr int BH_UNROLL = 2;
constexpr uint32_t BH_LDS_BUCKETS = 16384;   // 64 KB of LDS counters

__global__ void k_zero_u32(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

template <typename K, bool LDS, bool ABOVE>
__global__ __launch_bounds__(BH_THREADS) void k_bucket_histogram(const K *__restrict__ keys, uint64_t n,
                                                                 const uint64_t *__restrict__ minmax,
                                                                 uint32_t B, uint32_t *__restrict__ counts,
                                                                 const uint64_t *skip, uint64_t *order,
                                                                 uint64_t *above)
{
    __shared__ uint32_t s_c[LDS ? BH_LDS_BUCKETS : 1];
    if (skip && *skip) return;   // keys already sorted: nothing to count
    // with `order`, also whether the keys are already sorted (cleared by a
    // workgroup that finds a key smaller than the one before it); with
    // ABOVE, whether a key exceeds the range's maximum (*above set to 1 by a
    // workgroup that finds one: a declared bound the keys do not keep)
    const bool check = order != nullptr;
    bool order_ok = true;
    K seen = 0;   // largest key this thread counted (ABOVE)
    const BucketMap m = make_bucket_map(minmax[0], minmax[1], B);
    if (LDS) {
        for (uint32_t i = threadIdx.x; i < B; i += BH_THREADS) s_c[i] = 0;
        __syncthreads();
    }
    auto count = [&](K k) {
        const uint32_t b = bucket_of(m, k);
        if (ABOVE) seen = seen > k ? seen : k;
        if (LDS) lds_count(s_c, b);
        else atomicAdd(&counts[b], 1u);
    };
    constexpr int KPV = 16 / (int)sizeof(K);
    struct alignas(16) Vec { K v[KPV]; };
    const uint64_t nvec = n / KPV;
    const Vec *vk = reinterpret_cast<const Vec *>(keys);
    // BH_UNROLL 16-byte loads in flight per thread
    const uint64_t step = (uint64_t)gridDim.x * BH_THREADS * BH_UNROLL;
    for (uint64_t v0 = (uint64_t)blockIdx.x * BH_THREADS * BH_UNROLL + threadIdx.x; v0 < nvec; v0 += step) {
        Vec x[BH_UNROLL];
#pragma unroll
        for (int u = 0; u < BH_UNROLL; u++)
            if (v0 + (uint64_t)u * BH_THREADS < nvec) x[u] = vk[v0 + (uint64_t)u * BH_THREADS];
#pragma unroll
        for (int u = 0; u < BH_UNROLL; u++) {
            const uint64_t v = v0 + (uint64_t)u * BH_THREADS;
            if (check && !vector_in_order<K, KPV>(x[u].v, keys, v, nvec)) order_ok = false;
            if (v < nvec) {
#pragma unroll
                for (int e = 0; e < KPV; e++) count(x[u].v[e]);
            }
        }
    }
    const uint64_t stride = (uint64_t)gridDim.x * BH_THREADS;
    for (uint64_t i = nvec * KPV + (uint64_t)blockIdx.x * BH_THREADS + threadIdx.x; i < n; i += stride) {
        count(keys[i]);
        if (check && i > 0 && keys[i] < keys[i - 1]) order_ok = false;
    }
    if (check && __syncthreads_or(!order_ok) && threadIdx.x == 0) *order = 0;
    if (ABOVE && __syncthreads_or(seen > (K)minmax[1]) && threadIdx.x == 0) *above = 1;
    if (LDS) {
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < B; i += BH_THREADS) {
            const uint32_t c = s_c[i];
            if (c) atomicAdd(&counts[i], c);
        }
    }
}

hipError_t bucket_histogram_run(int key_bytes, const void *keys, uint64_t n, const uint64_t *minmax,
                                uint32_t B, uint32_t *counts, hipStream_t s, const uint64_t *skip,
                                uint64_t *order)
{
    return bucket_histogram_run_above(key_bytes, keys, n, minmax, B, counts, s, skip, order, nullptr);
}

hipError_t bucket_histogram_run_above(int key_bytes, const void *keys, uint64_t n, const uint64_t *minmax,
                                      uint32_t B, uint32_t *counts, hipStream_t s, const uint64_t *skip,
                                      uint64_t *order, uint64_t *above)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipLaunchKernelGGL(k_zero_u32, dim3((B + 255) / 256), dim3(256), 0, s, counts, B);
    uint64_t blocks = (n / (16 / key_bytes) + BH_THREADS * BH_UNROLL - 1) / (BH_THREADS * BH_UNROLL);
    const uint64_t cap = (uint64_t)device_cu_count(dev) * 2;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    const bool lds = B <= BH_LDS_BUCKETS;
    auto go = [&](auto key_tag) {
        using K = decltype(key_tag);
        auto kp = static_cast<const K *>(keys);
        const dim3 g((uint32_t)blocks), t(BH_THREADS);
        if (lds && above) hipLaunchKernelGGL((k_bucket_histogram<K, true, true>), g, t, 0, s, kp, n, minmax, B, counts, skip, order, above);
        else if (lds) hipLaunchKernelGGL((k_bucket_histogram<K, true, false>), g, t, 0, s, kp, n, minmax, B, counts, skip, order, above);
        else if (above) hipLaunchKernelGGL((k_bucket_histogram<K, false, true>), g, t, 0, s, kp, n, minmax, B, counts, skip, order, above);
        else hipLaunchKernelGGL((k_bucket_histogram<K, false, false>), g, t, 0, s, kp, n, minmax, B, counts, skip, order, above);
    };
    if (key_bytes == 4) go(uint32_t{});
    else go(uint64_t{});
    return hipGetLastError();
}

}  // namespace intsort
