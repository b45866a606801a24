"""GPU parity of bucket sort (HIP path through the C ABI) against the CPU
oracle: the min/max and bucket-index steps, the stable scatter (buckets
filled in input order, Algorithm 2 before its per-bucket sort), and the
final sorted keys and values, bit-exact.  Also the shortcut for keys already
in order (and single inversions where the order check changes hands), and
bucket starts across wide gaps of empty buckets."""
import numpy as np
import pytest

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host, rand_keys

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("B", [1, 7, 256, 1000, 1024, 2048, 3000, 65536])
@pytest.mark.parametrize("n", [1, 2, 17, 1000, 16385, 100_003])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_bucket_pairs_parity(B, n, dtype):
    print(f"bucket pairs B={B} n={n} {np.dtype(dtype).name}", flush=True)
    rng = np.random.default_rng(B * 7 + n)
    keys = rand_keys(rng, n, dtype, hi=None if n % 2 else max(2, n // 3))
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B)
    ref = oracle.radix_lsd(keys, vals)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    out = I.sort(dev(keys), algo="bucket", num_buckets=B)
    np.testing.assert_array_equal(host(out), ref.keys)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("B", [7, 1024, 2048, 65536])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_bucket_scatter_intermediate(B, dtype):
    """Stopping after the scatter gives the oracle's bucketed array: the
    stable partition of the input by bucket index."""
    n = 50_021
    keys = rand_keys(np.random.default_rng(B), n, dtype)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.bucket(keys, vals, num_buckets=B, want_intermediates=True)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B, max_passes=1)
    np.testing.assert_array_equal(host(ok), ref.scat_keys)
    np.testing.assert_array_equal(host(ov), ref.scat_vals)


@pytest.mark.parametrize("dist", range(7))
@pytest.mark.parametrize("B", [1024, 65536])
def test_bucket_distributions(dist, B):
    n = (1 << 20) + 123
    print(f"bucket dist={workloads.DISTRIBUTIONS[dist]} B={B}", flush=True)
    keys = workloads.config2_keys(dist, n)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B)
    ref = oracle.radix_lsd(keys, vals)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)


def test_bucket_special_and_in_place():
    for dtype in (np.uint32, np.uint64):
        mx = int(np.iinfo(dtype).max)
        special = [0, 1, 2**31 - 1, 2**31, 2**32 - 1] + ([2**63, mx - 1, mx] if dtype == np.uint64 else [])
        a = np.tile(np.array(special, dtype=dtype), 2000)
        np.random.default_rng(1).shuffle(a)
        for B in (3, 1024, 65536):
            t = dev(a)
            I.sort(t, out=t, algo="bucket", num_buckets=B)
            np.testing.assert_array_equal(host(t), np.sort(a))
        same = np.full(10_000, 12345, dtype=dtype)
        np.testing.assert_array_equal(host(I.sort(dev(same), algo="bucket")), same)


def test_config1_bucket():
    """1,000,000 uniform uint32 keys, seed 0, 1024 buckets."""
    keys = workloads.config2_keys(0, 1_000_000, seed=0)
    out = host(I.sort(dev(keys), algo="bucket", num_buckets=1024))
    np.testing.assert_array_equal(out, oracle.bucket(keys, num_buckets=1024).keys)


@pytest.mark.parametrize("dist", range(7))
def test_config2_bucket_full_size(dist):
    n = 100_000_000
    print(f"bucket full size dist={workloads.DISTRIBUTIONS[dist]}", flush=True)
    keys = workloads.config2_keys(dist, n)
    out = host(I.sort(dev(keys), algo="bucket", num_buckets=1024))
    np.testing.assert_array_equal(out, oracle.radix_lsd(keys).keys)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("B,n", [(70_000, 65_537), (100_000, 300_007), ((1 << 24) + 5, 1 << 21)])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_bucket_three_and_four_byte_indices(B, n, dtype):
    """More than 65536 buckets take three or four 8-bit scatter passes: the
    scattered array and the sorted pairs equal the oracle's."""
    print(f"bucket B={B} n={n} {np.dtype(dtype).name}", flush=True)
    keys = rand_keys(np.random.default_rng(B + n), n, dtype)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.bucket(keys, vals, num_buckets=B, want_intermediates=True)
    sk, sv = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B, max_passes=1)
    np.testing.assert_array_equal(host(sk), ref.scat_keys)
    np.testing.assert_array_equal(host(sv), ref.scat_vals)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("case", range(1, 7))
@pytest.mark.parametrize("n", [100_003, 1_000_000, 10_000_000])
def test_paper_map_with_declared_bound(case, n):
    """Section 4's cases sorted with section 2.3's map: B = n buckets and the
    declared range [0, M], b(k) = floor(n*k/(M+1)).  The scatter and the
    sorted pairs equal the oracle's under the same declared range."""
    keys, M = workloads.paper_case(case, n)
    print(f"paper case {case} n={n} M={M}", flush=True)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.bucket(keys, vals, num_buckets=n, key_bound=M, want_intermediates=True)
    sk, sv = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=n, key_bound=M, max_passes=1)
    np.testing.assert_array_equal(host(sk), ref.scat_keys)
    np.testing.assert_array_equal(host(sv), ref.scat_vals)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=n, key_bound=M)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    out = I.sort(dev(keys), algo="bucket", num_buckets=n, key_bound=M)
    np.testing.assert_array_equal(host(out), ref.keys)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("case", [1, 2, 5])
def test_paper_map_at_1e8(case):
    """The paper's largest size, n = 10^8 with B = n buckets over [0, M]:
    uniform keys below 10^6 (about 100 copies of each value), the same keys
    sorted, and uniform keys below 10^8.  Sorted pairs equal the oracle's."""
    n = 100_000_000
    keys, M = workloads.paper_case(case, n)
    print(f"paper case {case} n={n} M={M}", flush=True)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=n, key_bound=M)
    gk, gv = host(ok), host(ov)
    del ok, ov
    assert I.device_error(0) == 0
    print(f"paper case {case} n={n}: oracle", flush=True)
    ref = oracle.bucket(keys, vals, num_buckets=n, key_bound=M)
    np.testing.assert_array_equal(gk, ref.keys)
    np.testing.assert_array_equal(gv, ref.vals)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_windows_and_large_buckets_mixed(dtype):
    """Small buckets go through windows of whole consecutive buckets, buckets
    above half a workgroup's capacity through the segmented sort: a mix of
    a few huge runs of equal or close keys with many small buckets."""
    rng = np.random.default_rng(11)
    n = 1_500_000
    parts = [rng.integers(0, 1 << 30, n // 2, dtype=np.uint64),
             np.full(n // 6, 12345, dtype=np.uint64),
             rng.integers(1 << 29, (1 << 29) + 20_000, n // 6, dtype=np.uint64)]
    parts.append(rng.integers(0, 1 << 30, n - sum(len(p) for p in parts), dtype=np.uint64))
    keys = np.concatenate(parts)
    rng.shuffle(keys)
    keys = keys.astype(dtype)
    vals = np.arange(n, dtype=np.uint32)
    for B in (4096, 65536, 300_000):
        ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B)
        ref = oracle.radix_lsd(keys, vals)
        np.testing.assert_array_equal(host(ok), ref.keys)
        np.testing.assert_array_equal(host(ov), ref.vals)
    assert I.device_error(0) == 0


def _sorted_keys(dtype, n, seed):
    rng = np.random.default_rng(seed)
    k = np.sort(rand_keys(rng, n, dtype, hi=None if dtype == np.uint32 else 1 << 40))
    k[: n // 3] = k[0]   # a long run of equal keys
    return np.maximum(k, 1).astype(dtype)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("B", [1024, 65536])
@pytest.mark.parametrize("bound", [False, True])
def test_sorted_input_is_copied(dtype, B, bound):
    """Keys already in nondecreasing order (found by the min/max kernel, or by
    the order check with a declared range) skip every stage: the output is
    the input, values included, also in place and for the scatter alone."""
    n = 200_003
    keys = _sorted_keys(dtype, n, B + bound)
    vals = np.arange(n, dtype=np.uint32)
    opt = dict(algo="bucket", num_buckets=B, key_bound=int(keys[-1]) + 5 if bound else 0)
    print(f"sorted input {np.dtype(dtype).name} B={B} bound={bound}", flush=True)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), **opt)
    np.testing.assert_array_equal(host(ok), keys)
    np.testing.assert_array_equal(host(ov), vals)
    np.testing.assert_array_equal(host(I.sort(dev(keys), **opt)), keys)
    d = dev(keys)
    I.sort(d, out=d, **opt)
    np.testing.assert_array_equal(host(d), keys)
    sk, sv = I.sort_pairs(dev(keys), dev(vals), max_passes=1, **opt)
    np.testing.assert_array_equal(host(sk), keys)
    np.testing.assert_array_equal(host(sv), vals)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("bound", [False, True])
def test_one_inversion_is_sorted(dtype, bound):
    """A single key smaller than the one before it, placed where the order
    check changes hands (inside a 16-byte vector, between lanes, at a wave's
    first lane, at the next grid step, in the tail past the last whole
    vector): the check must see it and the full sort run."""
    n = 200_003
    kpv = 16 // np.dtype(dtype).itemsize
    for i in (1, kpv, 64 * kpv, 1024 * 4 * kpv, 1024 * 4 * kpv * 7 + 64 * kpv, n - 1, n // 2 + 1):
        print(f"one inversion {np.dtype(dtype).name} at {i} bound={bound}", flush=True)
        keys = _sorted_keys(dtype, n, i)
        keys[i - 1] = keys[i] + 1 if keys[i] < keys[-1] else keys[i - 1]
        keys[i] = keys[i - 1] - 1 if keys[i] >= keys[i - 1] else keys[i]
        assert keys[i] < keys[i - 1]
        vals = np.arange(n, dtype=np.uint32)
        opt = dict(algo="bucket", num_buckets=1024, key_bound=int(keys.max()) + 5 if bound else 0)
        ok, ov = I.sort_pairs(dev(keys), dev(vals), **opt)
        ref = oracle.radix_lsd(keys, vals)
        np.testing.assert_array_equal(host(ok), ref.keys)
        np.testing.assert_array_equal(host(ov), ref.vals)
        assert I.device_error(0) == 0


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("case", ["few_values", "two_ends", "one_value_bound"])
def test_bucket_starts_with_wide_gaps(dtype, case):
    """More buckets than the on-chip histogram holds, and keys that leave long
    runs of empty buckets: the bucket starts of those runs are listed in
    pieces and written by a second kernel.  Unsorted inputs, so no stage is
    skipped; keys and stable values bit-exact against the oracle."""
    n = 300_007
    rng = np.random.default_rng(len(case))
    top = (1 << 32) - 1 if dtype == np.uint32 else (1 << 40)
    bound = 0
    if case == "few_values":          # 50 values spread over the range: gaps of ~40K buckets
        values = np.sort(rng.integers(0, top, 50, dtype=np.uint64))
        values[0], values[-1] = 0, top
        keys = values[rng.integers(0, 50, n)]
    elif case == "two_ends":          # first and last bucket only
        keys = np.where(rng.integers(0, 2, n) == 1, top, 0).astype(np.uint64)
    else:                             # one value in the middle of a declared range
        keys = np.full(n, top // 2, dtype=np.uint64)
        keys[::7] = top // 3          # unsorted: two values, alternating runs
        bound = int(top)
    keys = keys.astype(dtype)
    vals = np.arange(n, dtype=np.uint32)
    B = (1 << 21) + 3
    print(f"wide gaps {case} {np.dtype(dtype).name} B={B}", flush=True)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B, key_bound=bound)
    ref = oracle.radix_lsd(keys, vals)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("span,B", [(4999, 5000), (5000, 5000), (5000, 4999), (200_000, 65536), (60_000, 65536),
                                    (3000, 1 << 20)])
@pytest.mark.parametrize("in_place", [False, True])
def test_one_value_per_bucket(dtype, span, B, in_place):
    """B >= R makes b(k) strictly increasing, so every bucket holds copies of
    one key value and the per-bucket sorts are skipped; B one below R (and
    B well below R) takes the usual path.  Both equal the oracle."""
    n = 300_007
    rng = np.random.default_rng(span + B)
    base = 7 if dtype == np.uint32 else (1 << 40) + 3
    keys = (rng.integers(0, span, n) + base).astype(dtype)
    keys[:2] = [base, base + span - 1]   # R = span exactly
    vals = np.arange(n, dtype=np.uint32)
    kd, vd = dev(keys), dev(vals)
    if in_place:
        ok, ov = I.sort_pairs(kd, vd, out_keys=kd, out_vals=vd, algo="bucket", num_buckets=B)
    else:
        ok, ov = I.sort_pairs(kd, vd, algo="bucket", num_buckets=B)
    ref = oracle.radix_lsd(keys, vals)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    out = I.sort(dev(keys), algo="bucket", num_buckets=B)
    np.testing.assert_array_equal(host(out), ref.keys)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("bound,B", [(999, 1000), (999, 4096), (59_999, 65536), (59_999, 60_000)])
def test_keys_above_declared_bound(dtype, bound, B):
    """A declared bound the keys do not keep: keys above it go to the last
    bucket, which then holds several values although B >= bound + 1, so the
    buckets must still be sorted.  Keys within the bound alone take the
    one-value-per-bucket shortcut."""
    n = 200_003
    rng = np.random.default_rng(bound + B)
    keys = rng.integers(0, bound + 1, n).astype(dtype)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.radix_lsd(keys, vals)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="bucket", num_buckets=B, key_bound=bound)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    hi = keys.copy()
    pos = rng.choice(n, 50, replace=False)
    hi[pos] = (rng.integers(bound + 1, 4 * bound, 50)).astype(dtype)
    ref = oracle.radix_lsd(hi, vals)
    ok, ov = I.sort_pairs(dev(hi), dev(vals), algo="bucket", num_buckets=B, key_bound=bound)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    out = I.sort(dev(hi), algo="bucket", num_buckets=B, key_bound=bound)
    np.testing.assert_array_equal(host(out), ref.keys)
    assert I.device_error(0) == 0
