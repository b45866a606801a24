// bucket_map.hpp -- the exact bucket index of bucket sort on the device.
//
// Bucket sort (section 2.3, Algorithm 2) sends key A[i] to bucket n*A[i]/M
// for keys in [0, M].  With the value range measured instead of assumed and
// B buckets, the bucket of key k is
//     b(k) = floor((k - min) * B / R),   R = max - min + 1,
// which is nondecreasing in k, maps min to 0 and stays below B.  With B up to
// 2^30 the product (k - min) * B needs up to 62 bits for 32-bit keys and up
// to 94 bits for 64-bit keys, and R can be 2^64.  A double-precision quotient gives an estimate that
// is at most one away from b(k); exact integer arithmetic then corrects it, so
// the result is exact for every key.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace intsort {

struct BucketMap {
    uint64_t mn;
    uint64_t range_m1;    // R - 1 = max - min (R itself may be 2^64)
    uint32_t buckets;     // B >= 1
    double scale;         // B / R in double precision (64-bit keys)
    uint64_t inv;         // floor((2^64 - 1) / R) (32-bit keys, R <= 2^32)
    uint64_t mul;         // floor(2^64 B / R) + 1 when fast32
    bool full64;          // R == 2^64
    bool fast32;          // R <= 2^32 and B < R: 32-bit keys use mul
    bool fast64;          // R <= 2^62: 64-bit keys need one correction only
};

__device__ __forceinline__ BucketMap make_bucket_map(uint64_t mn, uint64_t mx, uint32_t B)
{
    BucketMap m;
    m.mn = mn;
    m.range_m1 = mx - mn;
    m.buckets = B;
    m.full64 = (m.range_m1 == ~0ull);
    // R as a double: exact for R <= 2^53, correctly rounded above
    const double R = m.full64 ? 18446744073709551616.0 : (double)m.range_m1 + 1.0;
    m.scale = (double)B / R;
    m.inv = m.full64 ? 1ull : ~0ull / (m.range_m1 + 1);
    m.fast32 = !m.full64 && m.range_m1 <= 0xffffffffull && (uint64_t)B <= m.range_m1;
    m.fast64 = !m.full64 && m.range_m1 < (1ull << 62);
    m.mul = 0;
    if (m.fast32) {
        // 2^64 = q R + r with 0 <= r < R, from floor((2^64 - 1) / R)
        const uint64_t Rr = m.range_m1 + 1;
        uint64_t q = m.inv, r = ~0ull - m.inv * Rr;
        if (r == Rr - 1) {
            q += 1;
            r = 0;
        } else {
            r += 1;
        }
        // floor(2^64 B / R) = q B + floor(r B / R); below 2^64 because B < R
        m.mul = q * B + (r * B) / Rr + 1;
    }
    return m;
}

// b(k) for 32-bit keys.  With B < R one fixed-point product gives it (below).
// Otherwise num = (k - min) * B is below 2^62; with inv = floor((2^64 - 1) / R)
// the estimate floor(num * inv / 2^64) is either the exact quotient or one
// less (num * inv / 2^64 lies below num / R and within 2 num / 2^64 < 1/2 of
// it), so one remainder check makes it exact.  The result is clamped so that
// a key outside [min, max] cannot index past B.
__device__ __forceinline__ uint32_t bucket_of(const BucketMap &m, uint32_t k)
{
    if (m.fast32) {
        // b(k) = floor(x * mul / 2^64) with mul = floor(2^64 B / R) + 1: the
        // product exceeds x B / R by less than x / 2^64 < 2^-32 <= 1 / R,
        // while x B / R sits at least 1/R below the next integer, so the
        // floor is exact.  x * mul / 2^64 is taken as
        // (x * mul_hi + floor(x * mul_lo / 2^32)) / 2^32, which fits 64 bits.
        const uint32_t x = k - (uint32_t)m.mn;
        const uint64_t t = (uint64_t)x * (m.mul >> 32) + __umulhi(x, (uint32_t)m.mul);
        const uint32_t q = (uint32_t)(t >> 32);
        return q < m.buckets ? q : m.buckets - 1;
    }
    const uint64_t x = (uint64_t)(k - (uint32_t)m.mn);
    const uint64_t num = x * (uint64_t)m.buckets;
    const uint64_t R = m.range_m1 + 1;   // <= 2^32 for 32-bit keys
    uint64_t q = __umul64hi(num, m.inv);
    if (num - q * R >= R) q++;
    return (uint32_t)(q < m.buckets ? q : m.buckets - 1);
}

// b(k) for 64-bit keys: 128-bit products decide the exact floor
__device__ __forceinline__ uint32_t bucket_of(const BucketMap &m, uint64_t k)
{
    const uint64_t x = k - m.mn;
    const uint64_t B = m.buckets;
    if (m.full64) return (uint32_t)__umul64hi(x, B);   // x * B / 2^64
    const uint64_t R = m.range_m1 + 1;
    if (m.fast64) {
        // keys above the range (a declared bound) take the last bucket
        if (x >= R) return (uint32_t)(B - 1);
        // The double estimate is within one of b(k): its relative error is
        // a few 2^-53 and b(k) < 2^30.  The remainder x B - q R then lies in
        // (-R, 2R), which for R <= 2^62 is exact in wrapping 64-bit
        // arithmetic read as signed, so one correction makes q exact.
        int64_t q = (int64_t)((double)x * m.scale);
        const int64_t r = (int64_t)(x * B - (uint64_t)q * R);
        if (r < 0) q--;
        else if (r >= (int64_t)R) q++;
        return (uint32_t)(q < 0 ? 0 : (q < (int64_t)B ? q : (int64_t)B - 1));
    }
    // P = x * B as (phi, plo)
    const uint64_t plo = x * B, phi = __umul64hi(x, B);
    uint64_t q = (uint64_t)((double)x * m.scale);
    if (q >= B) q = B - 1;
    // decrease while q * R > P, increase while (q + 1) * R <= P
    for (int it = 0; it < 4; it++) {
        const uint64_t lo = q * R, hi = __umul64hi(q, R);
        if (hi > phi || (hi == phi && lo > plo)) {
            if (q == 0) break;
            q--;
            continue;
        }
        const uint64_t lo2 = lo + R, hi2 = hi + (lo2 < lo ? 1u : 0u);
        if (hi2 < phi || (hi2 == phi && lo2 <= plo)) { q++; continue; }
        break;
    }
    return (uint32_t)(q < B ? q : B - 1);
}

// Whether vector v of an array (its KPV keys x) is in nondecreasing order,
// inside and against the key before it.  The lanes of a wave hold
// consecutive vectors, so a lane takes that key from the lane below and
// lane 0 loads it.  Every lane whose vector is valid calls it together with
// all lanes below it; lanes with v >= nvec get true.
template <typename K, int KPV>
__device__ __forceinline__ bool vector_in_order(const K *x, const K *keys, uint64_t v, uint64_t nvec)
{
    K prev = __shfl_up(x[KPV - 1], 1, WAVE);
    if (lane_id() == 0 && v > 0 && v < nvec) prev = keys[v * KPV - 1];
    if (v >= nvec) return true;
    bool ok = v == 0 || x[0] >= prev;
#pragma unroll
    for (int e = 1; e < KPV; e++) ok = ok && x[e] >= x[e - 1];
    return ok;
}

}  // namespace intsort
