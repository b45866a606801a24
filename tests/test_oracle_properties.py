"""Property tests of the CPU oracle (hypothesis): for random inputs of up to a
few thousand keys, every oracle sort equals the library stable sort, which is
what the definition of sorting (section 2) and stability reduce to, whatever
the digit width, bucket count, cutoff or declared range."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle

SETTINGS = settings(max_examples=60, deadline=None)


def _keys(draw, dtype, n):
    bits = 8 * np.dtype(dtype).itemsize
    # a random key width makes long runs of equal high digits likely
    width = draw(st.integers(1, bits))
    seed = draw(st.integers(0, 2**32 - 1))
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 1 << min(width, 63), n, dtype=np.uint64)
    if width == 64:
        k = k * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    return k.astype(dtype)


@st.composite
def inputs(draw, dtypes=(np.uint32, np.uint64)):
    dtype = draw(st.sampled_from(dtypes))
    n = draw(st.integers(0, 3000))
    return _keys(draw, dtype, n)


def _stable(k, v):
    o = np.argsort(k, kind="stable")
    return k[o], v[o]


@SETTINGS
@given(inputs(), st.sampled_from([1, 3, 4, 8, 11, 16]), st.booleans())
def test_radix_equals_stable_sort(k, r, d_from_max):
    v = np.arange(k.size, dtype=np.uint32)
    res = oracle.radix_lsd(k, v, r=r, d_from_max=d_from_max)
    ek, ev = _stable(k, v)
    np.testing.assert_array_equal(res.keys, ek)
    np.testing.assert_array_equal(res.vals, ev)


@SETTINGS
@given(inputs(), st.sampled_from([1, 2, 3, 7, 1024, 65536]), st.sampled_from([0, 1, 8, 32, 10_000]))
def test_bucket_equals_stable_sort(k, B, cutoff):
    v = np.arange(k.size, dtype=np.uint32)
    res = oracle.bucket(k, v, num_buckets=B, cutoff=cutoff)
    ek, ev = _stable(k, v)
    np.testing.assert_array_equal(res.keys, ek)
    np.testing.assert_array_equal(res.vals, ev)


@SETTINGS
@given(inputs(dtypes=(np.uint32,)), st.integers(1, 5000), st.integers(0, 2**32 - 1))
def test_bucket_with_declared_range_equals_stable_sort(k, B, bound):
    """Keys above the declared bound join the last bucket; the output is
    still the stable sort."""
    v = np.arange(k.size, dtype=np.uint32)
    res = oracle.bucket(k, v, num_buckets=B, key_bound=max(bound, 1))
    ek, ev = _stable(k, v)
    np.testing.assert_array_equal(res.keys, ek)
    np.testing.assert_array_equal(res.vals, ev)


@SETTINGS
@given(st.sampled_from([np.int32, np.int64]), st.integers(0, 3000), st.integers(0, 2**32 - 1))
def test_signed_order_equals_stable_sort(dtype, n, seed):
    info = np.iinfo(dtype)
    rng = np.random.default_rng(seed)
    k = rng.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
    if n:
        k[rng.integers(0, n, n // 3)] = k[0]
    v = np.arange(n, dtype=np.uint32)
    got_k, got_v = oracle.sort_ordered(k, v)
    ek, ev = _stable(k, v)
    np.testing.assert_array_equal(got_k, ek)
    np.testing.assert_array_equal(got_v, ev)


@SETTINGS
@given(st.sampled_from([np.float32, np.float64]), st.integers(0, 3000), st.integers(0, 2**32 - 1))
def test_float_order_without_specials_equals_stable_sort(dtype, n, seed):
    """Finite keys and infinities, no NaN and no -0: totalOrder is the numeric
    order there."""
    rng = np.random.default_rng(seed)
    k = (rng.standard_normal(n) * np.exp(rng.uniform(-20, 20, n))).astype(dtype)
    if n > 4:
        k[rng.integers(0, n, n // 5)] = k[1]
        k[0], k[1] = np.inf, -np.inf
    k[k == 0] = 0.0
    v = np.arange(n, dtype=np.uint32)
    got_k, got_v = oracle.sort_ordered(k, v)
    ek, ev = _stable(k, v)
    ut = np.uint32 if dtype == np.float32 else np.uint64
    np.testing.assert_array_equal(got_k.view(ut), ek.view(ut))
    np.testing.assert_array_equal(got_v, ev)


@SETTINGS
@given(inputs(dtypes=(np.uint32,)), st.lists(st.integers(0, 3000), max_size=12))
def test_segmented_equals_per_segment_sort(k, cuts):
    n = k.size
    offs = np.array(sorted({0, n, *[c % (n + 1) for c in cuts]}), dtype=np.uint64)
    v = np.arange(n, dtype=np.uint32)
    for algo in ("radix", "bucket"):
        got_k, got_v = oracle.segmented(k, offs, v, algo=algo)
        for a, b in zip(offs[:-1].astype(np.int64), offs[1:].astype(np.int64)):
            ek, ev = _stable(k[a:b], v[a:b])
            np.testing.assert_array_equal(got_k[a:b], ek)
            np.testing.assert_array_equal(got_v[a:b], ev)


@SETTINGS
@given(inputs(), st.sampled_from([1, 7, 1024, 65536]), st.booleans())
def test_sorted_input_scatter_is_identity(k, B, bound):
    """Nondecreasing keys have nondecreasing bucket indices, so the stable
    scatter by bucket and every bucket's sort leave them in place: bucket
    sort of sorted keys is the identity, values included (the reasoning
    behind skipping every stage for already-sorted input)."""
    k = np.sort(k)
    v = np.arange(k.size, dtype=np.uint32)
    kb = int(k.max()) if (bound and k.size) else 0
    res = oracle.bucket(k, v, num_buckets=B, key_bound=kb, want_intermediates=True)
    np.testing.assert_array_equal(res.scat_keys, k)
    np.testing.assert_array_equal(res.scat_vals, v)
    np.testing.assert_array_equal(res.keys, k)
    np.testing.assert_array_equal(res.vals, v)
