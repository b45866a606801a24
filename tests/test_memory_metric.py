"""Device memory of one sort call (the analogue of the paper's memory table,
section 3.2, Table 2): input, output and the workspace the library asks for.
Planning context only, no GPU."""
import pytest

import bench


@pytest.mark.parametrize("width,pairs", [(4, False), (4, True), (8, False), (8, True)])
@pytest.mark.parametrize("n", [1000, 1 << 20, 100_000_000])
def test_radix_workspace_holds_one_scratch_copy(width, pairs, n):
    for bits in (4, 8, 11):
        m = bench._memory(width, pairs, n, algo="radix", digit_bits=bits)
        scratch = n * (width + (4 if pairs else 0))
        assert m["workspace_bytes"] >= scratch
        # the rest (histograms, plans, status words) stays a small fraction at scale
        if n >= 1 << 26:
            assert m["workspace_bytes"] <= scratch * 1.25
        assert m["peak_device_bytes"] == m["workspace_bytes"] + 2 * scratch


@pytest.mark.parametrize("width,pairs", [(4, False), (8, True)])
def test_bucket_workspace_holds_scratch_for_scatter_and_bucket_sort(width, pairs):
    n = 1 << 22
    for B in (256, 1024, 65536):
        m = bench._memory(width, pairs, n, algo="bucket", num_buckets=B)
        assert m["workspace_bytes"] >= 2 * n * (width + (4 if pairs else 0))


def test_workspace_grows_with_n():
    prev = 0
    for n in (1, 1000, 1 << 16, 1 << 20, 1 << 24):
        m = bench._memory(4, False, n, algo="radix", digit_bits=8)
        assert m["workspace_bytes"] >= prev
        prev = m["workspace_bytes"]


def test_segmented_workspace_counts_segments():
    a = bench._memory(4, False, 1 << 22, 16)
    b = bench._memory(4, False, 1 << 22, 1 << 16)
    assert b["workspace_bytes"] > a["workspace_bytes"]


def test_bucket_workspace_holds_bucket_starts():
    """More buckets than the on-chip histogram holds: the workspace grows by
    at least the bucket starts (8 bytes for each of B + 1) and the list of
    long runs of empty buckets (24 bytes for each of 2*floor((B+1)/1024) + 2
    pieces)."""
    n = 1 << 20
    small = bench._memory(4, False, n, algo="bucket", num_buckets=16384)["workspace_bytes"]
    for B in (1 << 17, 1 << 20, 100_000_000):
        large = bench._memory(4, False, n, algo="bucket", num_buckets=B)["workspace_bytes"]
        assert large - small >= 8 * (B - 16384) + 24 * (2 * ((B + 1) // 1024) + 2)
