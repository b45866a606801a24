// sort_plans.hpp -- host-side plans of the bucket and segmented sorts.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "intsort.h"
#include "internal.hpp"

namespace intsort {

constexpr uint32_t MAX_BUCKETS = 1u << 30;
constexpr uint64_t MAX_SEGMENTS = 1ull << 24;

struct SegLayout {
    size_t counters, plan, lists, tiles, bufs, tile_hist, seg_excl, slot_mask, status0, status1;
    size_t tmp_keys, tmp_vals, total;
    uint32_t slot_cap, tile_cap, list_stride, lds_cutoff;
};

struct BucketLayout {
    size_t counters, plan, minmax, counts, subhist, excl, offsets, runs, status0, status1, tmpb_keys, tmpb_vals,
        seg, total;
    uint32_t buckets, bits, scatter_passes;
    uint64_t num_tiles;
    SegLayout S;
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
    Timer *timer;
};

BucketLayout bucket_layout(int key_bytes, bool pairs, uint64_t n, const intsort_options &o);
hipError_t bucket_sort_run(const BucketCall &c, hipStream_t s);
// bucket_histogram_run that also sets *above to 1 when some key exceeds
// minmax[1] (above may be null)
hipError_t bucket_histogram_run_above(int key_bytes, const void *keys, uint64_t n, const uint64_t *minmax,
                                      uint32_t B, uint32_t *counts, hipStream_t s, const uint64_t *skip,
                                      uint64_t *order, uint64_t *above);


struct SegCall {
    const void *keys_in;
    void *keys_out;
    const uint32_t *vals_in;
    uint32_t *vals_out;
    uint64_t n;
    uint64_t num_segments;
    const uint64_t *offsets;
    const intsort_segment_desc *descs;   // separate arrays instead of offsets, or null
    int key_bytes;
    bool pairs;
    intsort_options opts;
    SegLayout L;
    char *ws;
    Timer *timer;
    uint32_t min_size;   // segments of at most this many keys are left as they are
    const uint64_t *skip = nullptr;   // device word: nonzero means sort nothing
};

SegLayout segmented_layout(int key_bytes, bool pairs, uint64_t n, uint64_t num_segments,
                           const intsort_options &o);
hipError_t segmented_sort_run(const SegCall &c, hipStream_t s);

}  // namespace intsort
