// sort_plans.hpp -- host-side plans of the bucket and segmented sorts.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "intsort.h"
#include "internal.hpp"

namespace intsort {

constexpr uint32_t MAX_BUCKETS = 1u << 20;
constexpr uint64_t MAX_SEGMENTS = 1ull << 24;

struct BucketLayout {
    size_t counters, total;
};

struct BucketCall {
    const void *keys_in;
    void *keys_out;
    const uint32_t *vals_in;
    uint32_t *vals_out;
    uint64_t n;
    int key_bytes;
    bool pairs;
    intsort_options opts;
    BucketLayout L;
    char *ws;
};

BucketLayout bucket_layout(int key_bytes, bool pairs, uint64_t n, const intsort_options &o);
hipError_t bucket_sort_run(const BucketCall &c, hipStream_t s);

struct SegLayout {
    size_t counters, total;
};

struct SegCall {
    const void *keys_in;
    void *keys_out;
    const uint32_t *vals_in;
    uint32_t *vals_out;
    uint64_t n;
    uint64_t num_segments;
    const uint64_t *offsets;
    int key_bytes;
    bool pairs;
    intsort_options opts;
    SegLayout L;
    char *ws;
};

SegLayout segmented_layout(int key_bytes, bool pairs, uint64_t n, uint64_t num_segments,
                           const intsort_options &o);
hipError_t segmented_sort_run(const SegCall &c, hipStream_t s);

}  // namespace intsort
