// plans_stub.cpp -- placeholders for plans that are not built yet.
#include "sort_plans.hpp"

namespace intsort {

BucketLayout bucket_layout(int, bool, uint64_t, const intsort_options &) { return BucketLayout{0, 256}; }
hipError_t bucket_sort_run(const BucketCall &, hipStream_t) { return hipErrorNotSupported; }
SegLayout segmented_layout(int, bool, uint64_t, uint64_t, const intsort_options &) { return SegLayout{0, 256}; }
hipError_t segmented_sort_run(const SegCall &, hipStream_t) { return hipErrorNotSupported; }

}  // namespace intsort
