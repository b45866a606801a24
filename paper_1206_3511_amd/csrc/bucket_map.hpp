// bucket_map.hpp -- the exact bucket index of bucket sort on the device.
//
// Bucket sort (section 2.3, Algorithm 2) sends key A[i] to bucket n*A[i]/M
// for keys in [0, M].  With the value range measured instead of assumed and
// B buckets, the bucket of key k is
//     b(k) = floor((k - min) * B / R),   R = max - min + 1,
// which is nondecreasing in k, maps min to 0 and stays below B.  With B up to
// 2^30 the product (k - min) * B needs up to 62 bits for 32-bit keys and up
// to 94 bits for 64-bit keys, and R can be 2^64.  32-bit keys take one
// exact fixed-point product; 64-bit keys take a double-precision estimate
// that is at most one away from b(k) and one exact remainder check.  Neither
// branches, so the result is exact for every key and costs the same for every
// range.  The map and the index are host and device functions, so that a host
// program can check them against exact 128-bit arithmetic.
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
    uint32_t a32;         // floor(B / R) (32-bit keys: R <= 2^32)
    uint64_t mul;         // floor(2^64 c / R) + 1 with c = B - a32 R (32-bit keys)
    uint64_t r_lo;        // R as a 96-bit number: low 64 bits (0 when R = 2^64)
    uint32_t r_hi;        // and bits 64..95 (1 when R = 2^64)
};

__host__ __device__ __forceinline__ BucketMap make_bucket_map(uint64_t mn, uint64_t mx, uint32_t B)
{
    BucketMap m;
    m.mn = mn;
    m.range_m1 = mx - mn;
    m.buckets = B;
    const bool full64 = m.range_m1 == ~0ull;   // R = 2^64
    // R as a double: exact for R <= 2^53, correctly rounded above
    const double R = full64 ? 18446744073709551616.0 : (double)m.range_m1 + 1.0;
    m.scale = (double)B / R;
    m.r_lo = m.range_m1 + 1;
    m.r_hi = full64 ? 1u : 0u;
    m.a32 = 0;
    m.mul = 0;
    if (m.range_m1 <= 0xffffffffull) {
        // B = a R + c with 0 <= c < R
        const uint64_t Rr = m.range_m1 + 1;
        const uint64_t a = Rr > B ? 0 : (uint32_t)B / (uint32_t)Rr;   // R <= B <= 2^30 in the division
        const uint64_t c = B - a * Rr;
        // 2^64 = q R + r with 0 <= r < R, from floor((2^64 - 1) / R)
        const uint64_t inv = ~0ull / Rr;
        uint64_t q = inv, r = ~0ull - inv * Rr;
        if (r == Rr - 1) {
            q += 1;
            r = 0;
        } else {
            r += 1;
        }
        // floor(2^64 c / R) = q c + floor(r c / R): r c < R^2 <= 2^64, and
        // the sum plus one stays below 2^64 because c < R <= 2^32
        m.a32 = (uint32_t)a;
        m.mul = q * c + (r * c) / Rr + 1;
    }
    return m;
}

// b(k) for 32-bit keys (R <= 2^32), with no branch on the map: for x = k - min
// in [0, R) and B = a R + c (0 <= c < R),
//     b(k) = floor(x B / R) = a x + floor(x c / R),
// and floor(x c / R) = floor(x * mul / 2^64) with mul = floor(2^64 c / R) + 1:
// the product exceeds x c / R by less than x / 2^64 < 2^-32 <= 1 / R, while
// x c / R sits at least 1/R below the next integer, so the floor is exact
// (c = 0 gives mul = 1 and 0).  x * mul / 2^64 is taken as
// (x * mul_hi + floor(x * mul_lo / 2^32)) / 2^32, which fits 64 bits.  A key
// outside [min, max] (x >= R, also when it lies below min) takes B - 1.
__host__ __device__ __forceinline__ uint32_t bucket_of(const BucketMap &m, uint32_t k)
{
    const uint32_t x = k - (uint32_t)m.mn;
    const uint64_t t = (uint64_t)x * (m.mul >> 32) + (((uint64_t)x * (uint32_t)m.mul) >> 32);
    const uint32_t q = (uint32_t)(t >> 32) + x * m.a32;
    return x <= (uint32_t)m.range_m1 ? q : m.buckets - 1;
}

// b(k) for 64-bit keys, with no branch on the map and none per key.  The
// double product x * (B / R) is within one of b(k): (double)x, B / R and the
// product each carry a relative error of at most 2^-53, so the estimate is off
// by less than 2^-21 from x B / R < 2^30, and its floor qe is b(k) - 1, b(k)
// or b(k) + 1.  The remainder r = x B - qe R (|r| < 2R <= 2^65) then says
// which: r < 0 means qe is one too large, r >= R one too small.  x B and qe R
// are below 2^95, and r is taken exactly as a 96-bit two's-complement number
// (64-bit low part, 32-bit high part) from four 32 x 32 -> 64-bit products.
// A key outside [min, max] (x >= R, also when it lies below min) takes B - 1.
__host__ __device__ __forceinline__ uint32_t bucket_of(const BucketMap &m, uint64_t k)
{
    const uint64_t x = k - m.mn;
    const uint32_t B = m.buckets;
    // (the clamp keeps the conversion defined for keys outside [min, max])
    const uint32_t qe = (uint32_t)fmin((double)x * m.scale, 2147483648.0);   // <= 2^30 + 1 in range
    // x B = p0 + p1 2^32
    const uint64_t p0 = (uint64_t)(uint32_t)x * B, p1 = (uint64_t)(uint32_t)(x >> 32) * B;
    const uint64_t xl = p0 + (p1 << 32);
    const uint32_t xh = (uint32_t)(p1 >> 32) + (xl < p0 ? 1u : 0u);
    // qe R = qe (R - 1) + qe = m0 + m1 2^32
    const uint64_t m0 = (uint64_t)qe * (uint32_t)m.range_m1 + qe;
    const uint64_t m1 = (uint64_t)qe * (uint32_t)(m.range_m1 >> 32);
    const uint64_t ql = m0 + (m1 << 32);
    const uint32_t qh = (uint32_t)(m1 >> 32) + (ql < m0 ? 1u : 0u);
    // r = x B - qe R, and the high word of r - R
    const uint64_t rl = xl - ql;
    const uint32_t rh = xh - qh - (xl < ql ? 1u : 0u);
    const uint32_t sh = rh - m.r_hi - (rl < m.r_lo ? 1u : 0u);
    const uint32_t q = qe - ((int32_t)rh < 0 ? 1u : 0u) + ((int32_t)sh >= 0 ? 1u : 0u);
    return x <= m.range_m1 ? q : B - 1;
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
