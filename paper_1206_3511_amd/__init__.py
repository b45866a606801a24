"""MI355X (gfx950) integer sorting: LSD radix sort and bucket sort from
"Comparison of Bucket Sort and RADIX Sort" (arXiv 1206.3511), as HIP kernels
behind the C ABI of include/intsort.h.  Importing the package loads nothing;
the first call loads libintsort.so (built by paper_1206_3511_amd/build.py)."""

from .intsort import (  # noqa: F401
    Context, IntsortError, Server, batched_sort, bucket_histogram, context, device_error, digit_histogram, lib,
    make_options, minmax, segmented_sort, sort, sort_pairs, status_string,
)
