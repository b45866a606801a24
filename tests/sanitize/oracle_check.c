/* Runs every entry point of the CPU oracle on small seeded inputs, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds
 * access, overflow the C standard leaves undefined, or leak aborts the run.
 * Results are checked only for the properties every sort must have (output
 * nondecreasing, values travelling with their keys); exact parity with the
 * paper is what the Python pins check. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_radix_lsd(const void *keys_in, void *keys_out, int key_bytes, const uint32_t *vals_in,
                     uint32_t *vals_out, uint64_t n, int r, int d_from_max, uint64_t *pass_counts,
                     uint64_t *pass_keys, int *passes_out);
uint64_t oracle_bucket_index(uint64_t k, uint64_t mn, uint64_t mx, uint64_t B);
int oracle_bucket(const void *keys_in, void *keys_out, int key_bytes, const uint32_t *vals_in,
                  uint32_t *vals_out, uint64_t n, uint64_t nbuckets, uint64_t cutoff, uint64_t key_bound,
                  uint64_t *minmax, uint64_t *counts, uint64_t *offsets, uint64_t *scat_keys,
                  uint32_t *scat_vals);
int oracle_segmented(const void *keys_in, void *keys_out, int key_bytes, const uint32_t *vals_in,
                     uint32_t *vals_out, uint64_t n_total, const uint64_t *offsets, uint64_t num_segments,
                     int algo, int r, uint64_t nbuckets, uint64_t cutoff);
int oracle_sort_ordered(const void *keys_in, void *keys_out, int key_bytes, int order, const uint32_t *vals_in,
                        uint32_t *vals_out, uint64_t n);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int failures = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            failures++;                                               \
        }                                                             \
    } while (0)

static uint64_t key_at(const void *a, int w, uint64_t i)
{
    return w == 4 ? ((const uint32_t *)a)[i] : ((const uint64_t *)a)[i];
}

/* keys nondecreasing; every value names the input key that sits beside it */
static void check_sorted_pairs(const void *in, const void *out, const uint32_t *vout, int w, uint64_t n)
{
    for (uint64_t i = 1; i < n; i++) CHECK(key_at(out, w, i - 1) <= key_at(out, w, i));
    if (vout)
        for (uint64_t i = 0; i < n; i++) CHECK(vout[i] < n && key_at(in, w, vout[i]) == key_at(out, w, i));
}

static void fill(void *a, int w, uint64_t n, int shift)
{
    for (uint64_t i = 0; i < n; i++) {
        const uint64_t r = next() >> shift;
        if (w == 4) ((uint32_t *)a)[i] = (uint32_t)r;
        else ((uint64_t *)a)[i] = r;
    }
}

int main(void)
{
    const uint64_t sizes[] = {0, 1, 2, 3, 17, 255, 256, 257, 1000, 4099};
    for (int wi = 0; wi < 2; wi++) {
        const int w = wi ? 8 : 4;
        for (size_t si = 0; si < sizeof(sizes) / sizeof(sizes[0]); si++) {
            const uint64_t n = sizes[si];
            for (int shift = 0; shift < 64; shift += 21) {
                void *in = malloc(n * 8 + 8), *out = malloc(n * 8 + 8);
                uint32_t *vin = malloc(n * 4 + 4), *vout = malloc(n * 4 + 4);
                fill(in, w, n, w == 4 ? 32 + shift / 2 : shift);
                for (uint64_t i = 0; i < n; i++) vin[i] = (uint32_t)i;
                const int rs[] = {1, 4, 8, 11, 16};
                for (int ri = 0; ri < 5; ri++) {
                    int d = 0;
                    CHECK(oracle_radix_lsd(in, out, w, vin, vout, n, rs[ri], 0, NULL, NULL, &d) == 0);
                    check_sorted_pairs(in, out, vout, w, n);
                    const int passes = (8 * w + rs[ri] - 1) / rs[ri];
                    uint64_t *pc = malloc(sizeof(uint64_t) * (size_t)passes << rs[ri]);
                    uint64_t *pk = malloc(sizeof(uint64_t) * (size_t)passes * (n + 1));
                    CHECK(oracle_radix_lsd(in, out, w, NULL, NULL, n, rs[ri], 1, pc, pk, &d) == 0);
                    check_sorted_pairs(in, out, NULL, w, n);
                    free(pc);
                    free(pk);
                }
                const uint64_t bs[] = {1, 2, 1024, 65536, n + 1};
                for (int bi = 0; bi < 5; bi++) {
                    const uint64_t B = bs[bi];
                    uint64_t mm[2];
                    uint64_t *counts = malloc(8 * B), *offs = malloc(8 * (B + 1));
                    uint64_t *sk = malloc(8 * n + 8);
                    uint32_t *sv = malloc(4 * n + 4);
                    CHECK(oracle_bucket(in, out, w, vin, vout, n, B, 32, 0, mm, counts, offs, sk, sv) == 0);
                    check_sorted_pairs(in, out, vout, w, n);
                    CHECK(oracle_bucket(in, out, w, NULL, NULL, n, B, 0, w == 4 ? 0xffffffffull : ~0ull, NULL, NULL,
                                        NULL, NULL, NULL) == 0);
                    check_sorted_pairs(in, out, NULL, w, n);
                    free(counts);
                    free(offs);
                    free(sk);
                    free(sv);
                }
                for (int order = 0; order < 3; order++) {
                    CHECK(oracle_sort_ordered(in, out, w, order, vin, vout, n) == 0);
                    for (uint64_t i = 0; i < n; i++) CHECK(vout[i] < n && key_at(in, w, vout[i]) == key_at(out, w, i));
                }
                /* segments: cut at seeded positions, some empty */
                uint64_t offsets[6] = {0, n / 5, n / 5, n / 2, (3 * n) / 4, n};
                for (int algo = 0; algo < 2; algo++) {
                    CHECK(oracle_segmented(in, out, w, vin, vout, n, offsets, 5, algo, 8, 64, 16) == 0);
                    for (int s = 0; s < 5; s++)
                        for (uint64_t i = offsets[s] + 1; i < offsets[s + 1]; i++)
                            CHECK(key_at(out, w, i - 1) <= key_at(out, w, i));
                }
                free(in);
                free(out);
                free(vin);
                free(vout);
            }
        }
    }
    /* the exact bucket map at the edges of its 64-bit range */
    CHECK(oracle_bucket_index(0, 0, ~0ull, 65536) == 0);
    CHECK(oracle_bucket_index(~0ull, 0, ~0ull, 65536) == 65535);
    CHECK(oracle_bucket_index(5, 5, 5, 7) == 0);
    CHECK(oracle_bucket_index(1ull << 62, 0, 1ull << 62, 3) == 2);
    /* argument errors are reported, not crashed on */
    CHECK(oracle_radix_lsd(NULL, NULL, 3, NULL, NULL, 4, 8, 0, NULL, NULL, NULL) != 0);
    CHECK(oracle_radix_lsd(NULL, NULL, 4, NULL, NULL, 4, 8, 0, NULL, NULL, NULL) != 0);
    CHECK(oracle_bucket(NULL, NULL, 4, NULL, NULL, 0, 0, 0, 0, NULL, NULL, NULL, NULL, NULL) != 0);
    CHECK(oracle_sort_ordered(NULL, NULL, 4, 7, NULL, NULL, 0) != 0);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle checks passed\n");
    return 0;
}
