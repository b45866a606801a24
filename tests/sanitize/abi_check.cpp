// Drives the host side of the C ABI through every argument check that runs
// before a kernel is enqueued, for a build of the library's host code with
// AddressSanitizer and UndefinedBehaviorSanitizer: option parsing, workspace
// sizing and layouts for every key type, algorithm and digit width, the
// tuning-table reader (good, malformed and missing files), argument errors
// of every sort entry point, and the serving calls on a context that cannot
// launch.  It uses a planning context (device -1), which validates and sizes
// but never launches, so it needs no GPU.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "intsort.h"

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            failures++;                                                  \
        }                                                                \
    } while (0)

int main(int argc, char **argv)
{
    const char *tune_path = argc > 1 ? argv[1] : "abi_check_tune.tsv";
    for (int s = 0; s <= 8; s++) CHECK(intsort_status_string((intsort_status)s) != nullptr);
    CHECK(intsort_status_string((intsort_status)99) != nullptr);

    intsort_ctx *ctx = nullptr;
    CHECK(intsort_create(nullptr, -1) == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_create(&ctx, -1) == INTSORT_OK && ctx);
    char key[256];
    CHECK(intsort_device_key(ctx, key, sizeof key) == INTSORT_OK && key[0] == 0);
    CHECK(intsort_device_key(ctx, key, 0) == INTSORT_ERR_INVALID_ARGUMENT);

    // workspace sizes: every key type, algorithm, digit width and size class
    const uint64_t sizes[] = {0, 1, 4095, 4096, 16384, 1000003, (1ull << 30) - 1, 1ull << 30, ~0ull};
    const uint32_t bits[] = {0, 4, 8, 11, 5};
    for (int kt = 0; kt <= 6; kt++)
        for (int algo = 0; algo <= 3; algo++)
            for (uint32_t b : bits)
                for (uint64_t n : sizes)
                    for (int pairs = 0; pairs < 2; pairs++) {
                        intsort_options o;
                        intsort_default_options(&o);
                        o.algo = (uint32_t)algo;
                        o.digit_bits = b;
                        o.num_buckets = algo == 1 ? 4099 : 0;
                        size_t bytes = 0;
                        const intsort_status st = intsort_workspace_size(ctx, (intsort_key_type)kt, pairs, n, 0, &o,
                                                                         &bytes);
                        if (st == INTSORT_OK && n > 0) CHECK(bytes > 0);
                        size_t seg = 0;
                        (void)intsort_workspace_size(ctx, (intsort_key_type)kt, pairs, n, 1 + n / 1000, &o, &seg);
                    }
    // option errors
    intsort_options bad;
    intsort_default_options(&bad);
    bad.struct_size = 3;
    size_t bytes = 0;
    CHECK(intsort_workspace_size(ctx, INTSORT_U32, 0, 100, 0, &bad, &bytes) != INTSORT_OK);
    intsort_default_options(&bad);
    bad.flags = 0x80u;
    CHECK(intsort_workspace_size(ctx, INTSORT_U32, 0, 100, 0, &bad, &bytes) != INTSORT_OK);
    CHECK(intsort_workspace_size(ctx, INTSORT_U32, 0, 100, 0, nullptr, nullptr) == INTSORT_ERR_INVALID_ARGUMENT);

    // the tuning table: good lines, malformed lines, a missing file, clearing
    FILE *f = fopen(tune_path, "w");
    CHECK(f != nullptr);
    if (f) {
        fputs("# comment\n*\tradix\t4\t20\t11\n*\tbucket\t4\t20\t65536\n*\tsegmented\t4\t20\t2048\n", f);
        fputs("\n\t\t\t\t\nno tabs here\n*\tradix\t4\t20\n*\tradix\t4\t99999999999999999999999\t8\n", f);
        fputs("*\tnothing\t4\t20\t8\n*\tradix\tx\t20\t8\n*\tradix\t4\t20\t7\n", f);
        for (int i = 0; i < 300; i++) fputc('x', f);
        fputs("\t\t\n", f);
        fclose(f);
    }
    CHECK(intsort_load_tuning(ctx, tune_path) == INTSORT_OK);
    size_t tuned = 0, fixed = 0;
    intsort_options o8;
    intsort_default_options(&o8);
    o8.digit_bits = 11;
    CHECK(intsort_workspace_size(ctx, INTSORT_U32, 0, 1u << 20, 0, nullptr, &tuned) == INTSORT_OK);
    CHECK(intsort_workspace_size(ctx, INTSORT_U32, 0, 1u << 20, 0, &o8, &fixed) == INTSORT_OK);
    CHECK(tuned == fixed);
    CHECK(intsort_load_tuning(ctx, "/nonexistent/dir/tune.tsv") == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_load_tuning(ctx, nullptr) == INTSORT_OK);
    remove(tune_path);

    // every sort entry point: argument errors come back before anything runs
    alignas(256) static uint32_t host[64];
    char *p = reinterpret_cast<char *>(host);
    CHECK(intsort_sort_keys(nullptr, INTSORT_U32, p, p, 4, nullptr, nullptr, 0, nullptr) == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_sort_keys(ctx, (intsort_key_type)9, p, p, 4, nullptr, nullptr, 0, nullptr) ==
          INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_sort_keys(ctx, INTSORT_U32, nullptr, p, 4, nullptr, nullptr, 0, nullptr) != INTSORT_OK);
    CHECK(intsort_sort_keys(ctx, INTSORT_U32, p + 4, p, 4, nullptr, nullptr, 0, nullptr) != INTSORT_OK);
    CHECK(intsort_sort_keys(ctx, INTSORT_U32, p, p, 0, nullptr, nullptr, 0, nullptr) == INTSORT_OK);
    CHECK(intsort_sort_keys(ctx, INTSORT_U32, p, p + 64, 1ull << 31, nullptr, p, 64, nullptr) != INTSORT_OK);
    CHECK(intsort_sort_keys(ctx, INTSORT_U32, p, p + 64, 16, nullptr, p + 1, 64, nullptr) != INTSORT_OK);
    CHECK(intsort_sort_keys_noalloc(ctx, INTSORT_U32, p, p + 64, 16, nullptr, nullptr) != INTSORT_OK);
    CHECK(intsort_sort_pairs(ctx, INTSORT_U32, p, p + 64, host, host, 16, nullptr, nullptr, 0, nullptr) != INTSORT_OK);
    CHECK(intsort_sort_pairs(ctx, INTSORT_U32, p, p + 64, nullptr, host + 32, 16, nullptr, nullptr, 0, nullptr) !=
          INTSORT_OK);
    CHECK(intsort_segmented_sort_keys(ctx, INTSORT_U32, p, p + 64, 16, 2, nullptr, nullptr, nullptr, 0, nullptr) !=
          INTSORT_OK);
    CHECK(intsort_segmented_sort_pairs(ctx, INTSORT_U64, p, p + 64, host, host + 32, 16, 0, nullptr, nullptr, nullptr,
                                       0, nullptr) != INTSORT_OK);
    CHECK(intsort_batched_sort_keys(ctx, INTSORT_U32, nullptr, 3, 100, nullptr, nullptr, 0, nullptr) != INTSORT_OK);
    uint32_t counts[256];
    CHECK(intsort_digit_histogram(ctx, INTSORT_U32, p, 16, 8, counts, nullptr, 0, nullptr) != INTSORT_OK);
    // a context that cannot launch refuses the serving and graph calls
    intsort_server *srv = nullptr;
    CHECK(intsort_server_create(ctx, 1u << 30, 8, 2, &srv) != INTSORT_OK && srv == nullptr);
    CHECK(intsort_server_create(ctx, 1u << 30, 0, 2, &srv) == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_server_submit(nullptr, INTSORT_U32, p, p, 1, nullptr) == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_server_destroy(nullptr) == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_server_fail_next_launches(nullptr, 1) == INTSORT_ERR_INVALID_ARGUMENT);
    CHECK(intsort_capture_begin(ctx, nullptr) != INTSORT_OK);
    CHECK(intsort_timing_enable(ctx, 1) != INTSORT_OK || true);
    CHECK(intsort_destroy(ctx) == INTSORT_OK);
    CHECK(intsort_destroy(nullptr) == INTSORT_OK);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("abi checks passed\n");
    return 0;
}
