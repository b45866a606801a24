// Checks the library's bucket index (make_bucket_map and bucket_of in
// bucket_map.hpp, the same source the kernels compile) on the host against
// exact 128-bit arithmetic: b(k) = floor((k - min) * B / R), R = max - min + 1,
// and B - 1 for a key outside [min, max].  Every key of every range R <= 300
// with every B <= 300 at five offsets (32- and 64-bit keys), then random
// ranges up to R = 2^64 with keys at both sides of sampled bucket boundaries.
#include <stdint.h>
#include <stdio.h>

#include <random>

#include "bucket_map.hpp"

typedef unsigned __int128 u128;

static uint32_t exact(uint64_t mn, uint64_t mx, uint32_t B, uint64_t k, bool below)
{
    const u128 R = (u128)(mx - mn) + 1;
    if (below) return B - 1;
    const u128 x = (u128)(k - mn);
    if (x >= R) return B - 1;
    return (uint32_t)(x * B / R);
}

static long bad = 0, checked = 0;

static void check(uint64_t mn, uint64_t mx, uint32_t B, uint64_t k)
{
    const intsort::BucketMap m = intsort::make_bucket_map(mn, mx, B);
    const uint32_t e = exact(mn, mx, B, k, k < mn);
    const uint32_t g64 = intsort::bucket_of(m, k);
    checked++;
    if (g64 != e) {
        if (bad < 10) printf("u64 mn=%llu mx=%llu B=%u k=%llu: %u, exact %u\n", (unsigned long long)mn,
                             (unsigned long long)mx, B, (unsigned long long)k, g64, e);
        bad++;
    }
    if (mx <= 0xffffffffull && k <= 0xffffffffull) {
        const uint32_t g32 = intsort::bucket_of(m, (uint32_t)k);
        if (g32 != e) {
            if (bad < 10) printf("u32 mn=%llu mx=%llu B=%u k=%llu: %u, exact %u\n", (unsigned long long)mn,
                                 (unsigned long long)mx, B, (unsigned long long)k, g32, e);
            bad++;
        }
    }
}

int main()
{
    const uint64_t offsets[] = {0, 5, 0xfffffff0ull, 1ull << 40, ~0ull - 400};
    for (uint64_t mn : offsets)
        for (uint64_t R = 1; R <= 300; R++) {
            const uint64_t mx = mn + (R - 1);
            if (mx < mn) continue;
            for (uint32_t B = 1; B <= 300; B++)
                for (uint64_t x = 0; x < R + 2 && mn + x >= mn; x++) check(mn, mx, B, mn + x);
        }
    std::mt19937_64 g(1);
    const uint32_t Bs[] = {1, 2, 3, 255, 256, 1000, 1024, 65535, 65536, 100003, 1u << 20, (1u << 30) - 1, 1u << 30};
    for (int trial = 0; trial < 4000; trial++) {
        uint64_t mn, mx;
        const uint64_t a = g(), b = g();
        switch (trial % 8) {
        case 0: mn = 0; mx = ~0ull; break;                                   // R = 2^64
        case 1: mn = a >> 1; mx = mn + (b >> (b % 64)); break;
        case 2: mn = a >> 2; mx = mn + (1ull << 62) + (b % 1000); break;       // just above 2^62
        case 3: mn = 0; mx = (1ull << (g() % 64)) - 1 + (g() % 3); break;
        case 4: mn = a % 1000; mx = mn + (b % 5000); break;
        case 5: mn = 0; mx = 0xffffffffull - (b % 3); break;                 // 32-bit ranges
        case 6: mn = a; mx = a; break;                                       // one value
        default: mn = 3; mx = (1ull << 63) + (1ull << 61); break;
        }
        if (mx < mn) { const uint64_t t = mn; mn = mx; mx = t; }
        const uint32_t B = Bs[g() % 13];
        const uint64_t rm = mx - mn;
        for (int i = 0; i < 200; i++) check(mn, mx, B, mn + (rm == ~0ull ? g() : g() % (rm + 1)));
        check(mn, mx, B, mn);
        check(mn, mx, B, mx);
        if (mx < ~0ull) check(mn, mx, B, mx + 1);   // above the range: B - 1
        if (mn > 0) check(mn, mx, B, mn - 1);       // below the range: B - 1
        const u128 R = (u128)rm + 1;
        for (int i = 0; i < 50; i++) {
            // the first key of bucket j, ceil(j R / B) above min, and its neighbours
            const uint32_t j = (uint32_t)(g() % B);
            const u128 x = ((u128)j * R + B - 1) / B;
            if (x < R) {
                check(mn, mx, B, mn + (uint64_t)x);
                if (x > 0) check(mn, mx, B, mn + (uint64_t)x - 1);
                if (x + 1 < R) check(mn, mx, B, mn + (uint64_t)x + 1);
            }
        }
    }
    printf("%ld of %ld keys wrong\n", bad, checked);
    return bad != 0;
}
