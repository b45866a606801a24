"""Pins of the CPU oracle against facts fixed outside it.

The oracle's results are checked against:
  * library sorts (numpy's stable sort, Python's stable ``sorted``), which is
    what the paper's definition of sorting (section 2) reduces to;
  * brute force over every short sequence on a tiny alphabet and every
    permutation of small multisets;
  * the invariants the paper states: the output is a nondecreasing
    permutation (section 2), equal keys keep their input order (stability,
    section 2), and after pass p of LSD radix the array is stably sorted on
    its low (p+1) digits (section 2.5, Algorithm 4);
  * exact big-integer arithmetic for the bucket map (Algorithm 2's index with
    the measured range), at every bucket boundary.
"""
import itertools

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(12345)


def stable_ref(keys, vals=None):
    order = np.argsort(keys, kind="stable")
    return keys[order], (None if vals is None else vals[order])


def rand_keys(n, dtype, hi=None):
    if dtype == np.uint32:
        hi = (1 << 32) if hi is None else hi
        return RNG.integers(0, hi, n, dtype=np.uint64).astype(np.uint32)
    if hi is None:
        return RNG.integers(0, 1 << 63, n, dtype=np.uint64) * np.uint64(2) + \
            RNG.integers(0, 2, n, dtype=np.uint64)
    return RNG.integers(0, hi, n, dtype=np.uint64)


# ------------------------------------------------------------------ radix

@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("r", [1, 3, 4, 5, 8, 11, 16])
@pytest.mark.parametrize("n,hi", [(0, None), (1, None), (2, 3), (1000, None), (4097, 50), (3000, 1 << 20)])
def test_radix_equals_library_stable_sort(dtype, r, n, hi):
    keys = rand_keys(n, dtype, hi)
    vals = RNG.permutation(n).astype(np.uint32)
    ref_k, ref_v = stable_ref(keys, vals)
    res = oracle.radix_lsd(keys, vals, r=r)
    assert res.keys.dtype == keys.dtype
    np.testing.assert_array_equal(res.keys, ref_k)
    np.testing.assert_array_equal(res.vals, ref_v)
    assert res.passes == -(-8 * keys.dtype.itemsize // r)
    np.testing.assert_array_equal(oracle.radix_lsd(keys, r=r).keys, ref_k)


@pytest.mark.parametrize("dtype,r", [(np.uint32, 8), (np.uint32, 11), (np.uint64, 8), (np.uint64, 11), (np.uint32, 3)])
def test_radix_pass_invariant_and_counts(dtype, r):
    """After pass p the array is the stable sort by key mod 2^((p+1) r)
    (the LSD invariant behind Algorithm 4); the pass-p counts are the
    histogram of digit p, which sums to n."""
    n = 2500
    keys = rand_keys(n, dtype, None if r != 3 else 1 << 10)
    res = oracle.radix_lsd(keys, r=r, want_counts=True, want_passes=True)
    bits = 8 * keys.dtype.itemsize
    for p in range(res.passes):
        low = min(bits, (p + 1) * r)
        masked = keys.astype(np.uint64) & np.uint64((1 << low) - 1 if low < 64 else (1 << 64) - 1)
        expect = keys[np.argsort(masked, kind="stable")]
        np.testing.assert_array_equal(res.pass_keys[p], expect)
        digit = (keys.astype(np.uint64) >> np.uint64(p * r)) & np.uint64((1 << r) - 1)
        np.testing.assert_array_equal(res.pass_counts[p], np.bincount(digit.astype(np.int64), minlength=1 << r))
        assert int(res.pass_counts[p].sum()) == n


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_radix_d_from_max(dtype):
    """Algorithm 4's d (digits of the largest key) gives the same output."""
    for hi, r in [(1 << 10, 8), (1 << 17, 4), (1, 8), (5, 2)]:
        keys = rand_keys(777, dtype, hi)
        res = oracle.radix_lsd(keys, r=r, d_from_max=True)
        mx = int(keys.max())
        assert res.passes == -(-mx.bit_length() // r)
        np.testing.assert_array_equal(res.keys, np.sort(keys))


# ------------------------------------------------------------------ brute force

def _all_sequences(max_len, alphabet):
    for n in range(max_len + 1):
        yield from itertools.product(range(alphabet), repeat=n)


def test_brute_force_every_short_sequence():
    """Every sequence of length 0..6 over {0,1,2,3}: both sorts with the
    index payload equal Python's stable sorted() for every digit width and
    bucket count tried."""
    for seq in _all_sequences(6, 4):
        n = len(seq)
        keys = np.array(seq, dtype=np.uint32)
        vals = np.arange(n, dtype=np.uint32)
        order = sorted(range(n), key=lambda i: seq[i])
        ek = np.array([seq[i] for i in order], dtype=np.uint32)
        ev = np.array(order, dtype=np.uint32)
        for r in (1, 2, 3):
            res = oracle.radix_lsd(keys, vals, r=r)
            assert res.keys.tolist() == ek.tolist() and res.vals.tolist() == ev.tolist(), (seq, r)
        for B in (1, 2, 3, 7):
            res = oracle.bucket(keys, vals, num_buckets=B, cutoff=32)
            assert res.keys.tolist() == ek.tolist() and res.vals.tolist() == ev.tolist(), (seq, B)


@pytest.mark.parametrize("multiset", [(0, 0, 1, 1, 2, 2, 3, 3), (7, 7, 7, 1, 1, 0, 9, 9), (5, 4, 3, 2, 1, 0, 0, 6)])
def test_every_permutation_of_small_multisets(multiset):
    seen = set()
    for perm in itertools.permutations(multiset):
        if perm in seen:
            continue
        seen.add(perm)
        keys = np.array(perm, dtype=np.uint64)
        vals = np.arange(len(perm), dtype=np.uint32)
        order = sorted(range(len(perm)), key=lambda i: perm[i])
        for res in (oracle.radix_lsd(keys, vals, r=2), oracle.bucket(keys, vals, num_buckets=3, cutoff=4)):
            assert res.keys.tolist() == sorted(perm)
            assert res.vals.tolist() == order


def test_special_keys():
    u32 = [0, 1, 2**31 - 1, 2**31, 2**32 - 1]
    u64 = u32 + [2**63 - 1, 2**63, 2**64 - 2, 2**64 - 1]
    for dtype, vals in ((np.uint32, u32), (np.uint64, u64)):
        keys = np.array(vals * 5, dtype=dtype)
        RNG.shuffle(keys)
        pay = np.arange(keys.size, dtype=np.uint32)
        ek, ev = stable_ref(keys, pay)
        for res in (oracle.radix_lsd(keys, pay, r=8), oracle.radix_lsd(keys, pay, r=11),
                    oracle.bucket(keys, pay, num_buckets=1024), oracle.bucket(keys, pay, num_buckets=65536)):
            np.testing.assert_array_equal(res.keys, ek)
            np.testing.assert_array_equal(res.vals, ev)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 127, 128, 129])
def test_all_equal_and_tiny(n):
    for dtype in (np.uint32, np.uint64):
        for v in (0, 12345, int(np.iinfo(dtype).max)):
            keys = np.full(n, v, dtype=dtype)
            pay = np.arange(n, dtype=np.uint32)
            for res in (oracle.radix_lsd(keys, pay), oracle.bucket(keys, pay, num_buckets=7)):
                np.testing.assert_array_equal(res.keys, keys)
                np.testing.assert_array_equal(res.vals, pay)


# ------------------------------------------------------------------ bucket

def _py_bucket(k, mn, mx, B):
    return (k - mn) * B // (mx - mn + 1)


def test_bucket_index_exact_random():
    for _ in range(3000):
        bits = int(RNG.choice([8, 32, 64]))
        a, b = (int(x) for x in RNG.integers(0, 1 << min(bits, 63), 2, dtype=np.uint64))
        if bits == 64:
            a, b = a * 2 + int(RNG.integers(0, 2)), b * 2 + int(RNG.integers(0, 2))
        mn, mx = min(a, b), max(a, b)
        k = mn + (int(RNG.integers(0, 1 << 62)) % (mx - mn + 1))
        B = int(RNG.choice([1, 2, 3, 7, 1000, 1024, 65536, 1 << 20]))
        assert oracle.bucket_index(k, mn, mx, B) == _py_bucket(k, mn, mx, B)
    # the full 64-bit range, whose size 2^64 fits no 64-bit word
    mx = (1 << 64) - 1
    for k in (0, 1, 1 << 63, mx - 1, mx):
        for B in (1, 1024, 65536):
            assert oracle.bucket_index(k, 0, mx, B) == k * B >> 64


@pytest.mark.parametrize("mn,mx,B", [(0, 2**32 - 1, 1024), (17, 1040, 7), (5, 5, 3), (0, 2**64 - 1, 65536),
                                     (2**40 + 3, 2**41, 1000), (0, 999, 1024)])
def test_bucket_boundaries(mn, mx, B):
    """The first key of bucket j is mn + ceil(j R / B); the key before it is
    in an earlier bucket.  Checked at every boundary (sampled for large B)."""
    R = mx - mn + 1
    js = range(1, B) if B <= 1024 else list(range(1, 200)) + list(range(B - 200, B))
    prev = 0
    for j in js:
        first = mn + -(-j * R // B)
        if first > mx:
            continue
        bj = oracle.bucket_index(first, mn, mx, B)
        assert bj == _py_bucket(first, mn, mx, B)
        assert bj >= j and bj >= prev
        if first - 1 >= mn:
            assert oracle.bucket_index(first - 1, mn, mx, B) < bj
        prev = bj
    assert oracle.bucket_index(mn, mn, mx, B) == 0
    assert oracle.bucket_index(mx, mn, mx, B) == B - 1 if R >= B else True
    assert oracle.bucket_index(mx, mn, mx, B) < B


@pytest.mark.parametrize("dtype,B,hi", [(np.uint32, 1024, None), (np.uint32, 7, 100), (np.uint64, 65536, None),
                                        (np.uint64, 1000, 1 << 40), (np.uint32, 1, None)])
def test_bucket_intermediates(dtype, B, hi):
    """min/max, bucket sizes, offsets and the scatter (= stable partition of
    the input by bucket, the buckets of Algorithm 2 filled in input order)."""
    n = 5000
    keys = rand_keys(n, dtype, hi)
    pay = np.arange(n, dtype=np.uint32)
    res = oracle.bucket(keys, pay, num_buckets=B, cutoff=16, want_intermediates=True)
    mn, mx = int(keys.min()), int(keys.max())
    assert (res.kmin, res.kmax) == (mn, mx)
    b = np.array([_py_bucket(int(k), mn, mx, B) for k in keys], dtype=np.int64)
    np.testing.assert_array_equal(res.counts, np.bincount(b, minlength=B))
    np.testing.assert_array_equal(res.offsets[1:], np.cumsum(np.bincount(b, minlength=B)))
    assert int(res.offsets[0]) == 0 and int(res.offsets[-1]) == n
    order = np.argsort(b, kind="stable")
    np.testing.assert_array_equal(res.scat_keys, keys[order])
    np.testing.assert_array_equal(res.scat_vals, pay[order])
    ek, ev = stable_ref(keys, pay)
    np.testing.assert_array_equal(res.keys, ek)
    np.testing.assert_array_equal(res.vals, ev)


@pytest.mark.parametrize("cutoff", [0, 1, 32, 10**9])
def test_bucket_cutoff_does_not_change_result(cutoff):
    """Insertion sort (Algorithm 1) and the merge sort are both stable, so
    the per-bucket choice cannot change the output."""
    keys = rand_keys(3000, np.uint32, 300)
    pay = np.arange(3000, dtype=np.uint32)
    res = oracle.bucket(keys, pay, num_buckets=10, cutoff=cutoff)
    ek, ev = stable_ref(keys, pay)
    np.testing.assert_array_equal(res.keys, ek)
    np.testing.assert_array_equal(res.vals, ev)


# ------------------------------------------------------------------ segmented

@pytest.mark.parametrize("algo", ["radix", "bucket"])
def test_segmented_equals_per_segment_sort(algo):
    sizes = [0, 5, 1, 0, 300, 17, 1000, 0]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    keys = rand_keys(int(offsets[-1]), np.uint32, 1 << 12)
    pay = np.arange(keys.size, dtype=np.uint32)
    out_k, out_v = oracle.segmented(keys, offsets, pay, algo=algo)
    for s in range(len(sizes)):
        a, b = int(offsets[s]), int(offsets[s + 1])
        ek, ev = stable_ref(keys[a:b], pay[a:b])
        np.testing.assert_array_equal(out_k[a:b], ek)
        np.testing.assert_array_equal(out_v[a:b], ev)


def test_segmented_rejects_bad_offsets():
    keys = np.zeros(10, dtype=np.uint32)
    with pytest.raises(RuntimeError):
        oracle.segmented(keys, np.array([0, 6, 4, 10], dtype=np.uint64))
    with pytest.raises(RuntimeError):
        oracle.segmented(keys, np.array([0, 4, 9], dtype=np.uint64))


# ---- declared range: the bound M of section 2.3 and the map with B = n


@pytest.mark.parametrize("M,n", [(10**4, 5000), (10**6, 20_000), (10**8, 3000), (7, 100)])
def test_bucket_declared_bound_paper_map(M, n):
    """With B = n buckets and the range declared as [0, M], the bucket of k
    is floor(n*k/(M+1)) (checked with Python integers), every bucket holds
    its keys in input order, and the result is the library's stable sort."""
    rng = np.random.default_rng(M + n)
    keys = rng.integers(0, M + 1, size=n, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(n, dtype=np.uint32)
    r = oracle.bucket(keys, vals, num_buckets=n, key_bound=M, want_intermediates=True)
    assert (r.kmin, r.kmax) == (0, M)
    want = np.zeros(n, dtype=np.uint64)
    for k in keys.tolist():
        want[(n * k) // (M + 1)] += 1
    np.testing.assert_array_equal(r.counts, want)
    b = np.array([(n * k) // (M + 1) for k in keys.tolist()], dtype=np.int64)
    order = np.argsort(b, kind="stable")
    np.testing.assert_array_equal(r.scat_keys, keys[order])
    np.testing.assert_array_equal(r.scat_vals, vals[order])
    o = np.argsort(keys, kind="stable")
    np.testing.assert_array_equal(r.keys, keys[o])
    np.testing.assert_array_equal(r.vals, vals[o])


def test_bucket_keys_above_declared_bound_join_last_bucket():
    keys = np.array([5, 100, 3, 1000, 7, 2**32 - 1, 50], dtype=np.uint32)
    r = oracle.bucket(keys, num_buckets=4, key_bound=99, want_intermediates=True)
    np.testing.assert_array_equal(r.keys, np.sort(keys))
    # 5, 3, 7 -> bucket 0; 50 -> floor(4*50/100) = 2; 100, 1000, 2^32-1 lie
    # above the bound -> bucket 3
    assert r.counts.tolist() == [3, 0, 1, 3]


# ------------------------------------------- signed and floating-point keys

# IEEE 754 binary32 / binary64 bit patterns in ascending totalOrder
# (IEEE 754-2019 section 5.10), written from the formats' fields
# (sign | exponent | fraction): -NaN with the largest payload, -qNaN, -sNaN,
# -inf, -max, -1, -min normal, -max subnormal, -min subnormal, -0, and the
# mirror images ascending.
F32_LADDER = [0xFFFFFFFF, 0xFFC00000, 0xFF800001, 0xFF800000, 0xFF7FFFFF, 0xBF800000, 0x80800000,
              0x807FFFFF, 0x80000001, 0x80000000,
              0x00000000, 0x00000001, 0x007FFFFF, 0x00800000, 0x3F800000, 0x7F7FFFFF, 0x7F800000,
              0x7F800001, 0x7FC00000, 0x7FFFFFFF]
F64_LADDER = [0xFFFFFFFFFFFFFFFF, 0xFFF8000000000000, 0xFFF0000000000001, 0xFFF0000000000000,
              0xFFEFFFFFFFFFFFFF, 0xBFF0000000000000, 0x8010000000000000, 0x800FFFFFFFFFFFFF,
              0x8000000000000001, 0x8000000000000000,
              0x0000000000000000, 0x0000000000000001, 0x000FFFFFFFFFFFFF, 0x0010000000000000,
              0x3FF0000000000000, 0x7FEFFFFFFFFFFFFF, 0x7FF0000000000000, 0x7FF0000000000001,
              0x7FF8000000000000, 0x7FFFFFFFFFFFFFFF]


def _ladder(fdt):
    bits = np.array(F32_LADDER if fdt == np.float32 else F64_LADDER,
                    dtype=np.uint32 if fdt == np.float32 else np.uint64)
    return bits.view(fdt)


@pytest.mark.parametrize("fdt", [np.float32, np.float64])
def test_float_ladder_is_what_it_claims(fdt):
    """The hand-written ladder: NaNs at both ends, the finite values and the
    infinities strictly ascending by value except -0 == +0, -0 carrying the
    sign bit."""
    v = _ladder(fdt)
    nan = np.isnan(v)
    assert nan[:3].all() and nan[-3:].all() and not nan[3:-3].any()
    assert np.signbit(v[:10]).all() and not np.signbit(v[10:]).any()
    mid = v[3:-3].astype(np.float64)
    d = np.diff(mid)
    assert (d[d != 0] > 0).all() and np.count_nonzero(d == 0) == 1
    assert v[3] == -np.inf and v[-4] == np.inf


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("n", [0, 1, 5, 4097])
def test_signed_order_matches_library(dtype, n):
    info = np.iinfo(dtype)
    k = RNG.integers(info.min, info.max, n, dtype=dtype, endpoint=True)
    if n > 8:
        k[:6] = [info.min, info.max, -1, 0, 1, info.min]
        k[::9] = k[4]
    v = np.arange(n, dtype=np.uint32)
    got_k, got_v = oracle.sort_ordered(k, v)
    ek, ev = stable_ref(k, v)
    np.testing.assert_array_equal(got_k, ek)
    np.testing.assert_array_equal(got_v, ev)


@pytest.mark.parametrize("fdt", [np.float32, np.float64])
def test_float_finite_order_matches_library(fdt):
    """Finite keys without -0: totalOrder is the numeric order, and the stable
    library sort fixes the payload order of equal keys."""
    n = 5000
    k = (RNG.standard_normal(n) * np.exp(RNG.uniform(-30, 30, n))).astype(fdt)
    k[::11] = k[3]
    k[::13] = 0.0
    k[k == 0] = 0.0          # no -0: numeric order cannot tell it from +0
    v = np.arange(n, dtype=np.uint32)
    got_k, got_v = oracle.sort_ordered(k, v)
    ek, ev = stable_ref(k, v)
    np.testing.assert_array_equal(got_k.view(np.uint8), ek.view(np.uint8))
    np.testing.assert_array_equal(got_v, ev)


@pytest.mark.parametrize("fdt", [np.float32, np.float64])
def test_float_specials_follow_total_order(fdt):
    """Every ladder entry, repeated and shuffled: the output lists the ladder
    in order (by bit pattern) and keeps the input order of repeats."""
    lad = _ladder(fdt)
    ut = np.uint32 if fdt == np.float32 else np.uint64
    idx = np.repeat(np.arange(lad.size), 3)
    RNG.shuffle(idx)
    k = lad[idx]
    v = np.arange(idx.size, dtype=np.uint32)
    got_k, got_v = oracle.sort_ordered(k, v)
    order = np.argsort(idx, kind="stable")
    np.testing.assert_array_equal(got_k.view(ut), lad[idx[order]].view(ut))
    np.testing.assert_array_equal(got_v, v[order])


@pytest.mark.parametrize("fdt", [np.float32, np.float64])
def test_float_order_brute_force_on_ladder(fdt):
    """Every sequence of length <= 4 over six ladder entries (-NaN, -inf, -0,
    +0, +inf, +NaN and neighbours): the result is the stable sort by ladder
    position."""
    lad = _ladder(fdt)
    pick = [1, 3, 9, 10, 16, 18]
    ut = np.uint32 if fdt == np.float32 else np.uint64
    for m in range(5):
        for seq in itertools.product(range(len(pick)), repeat=m):
            pos = np.array([pick[s] for s in seq], dtype=np.int64)
            k = lad[pos]
            got_k, got_v = oracle.sort_ordered(k, np.arange(m, dtype=np.uint32))
            order = sorted(range(m), key=lambda i: pos[i])
            assert got_k.view(ut).tolist() == lad[pos[order]].view(ut).tolist()
            assert got_v.tolist() == order


def test_unsigned_order_equals_radix():
    k = rand_keys(3000, np.uint64)
    k[::5] = k[2]
    v = np.arange(3000, dtype=np.uint32)
    got_k, got_v = oracle.sort_ordered(k, v)
    ek, ev = stable_ref(k, v)
    np.testing.assert_array_equal(got_k, ek)
    np.testing.assert_array_equal(got_v, ev)


@pytest.mark.parametrize("dtype,r", [(np.uint32, 8), (np.uint32, 4), (np.uint64, 11), (np.uint64, 8)])
def test_full_declared_range_buckets_are_top_bits(dtype, r):
    """With the declared range [0, 2^W - 1] and 2^r buckets the bucket of k is
    floor(k * 2^r / 2^W) = k >> (W - r), its top r bits: the scatter is the
    stable partition on the most significant digit."""
    n = 4000
    k = rand_keys(n, dtype)
    W = 8 * k.dtype.itemsize
    res = oracle.bucket(k, np.arange(n, dtype=np.uint32), num_buckets=1 << r, key_bound=(1 << W) - 1,
                        want_intermediates=True)
    top = (k >> k.dtype.type(W - r)).astype(np.int64)
    order = np.argsort(top, kind="stable")
    np.testing.assert_array_equal(res.scat_keys, k[order])
    np.testing.assert_array_equal(res.scat_vals, order.astype(np.uint32))
    np.testing.assert_array_equal(res.counts.astype(np.int64), np.bincount(top, minlength=1 << r))


@pytest.mark.parametrize("B", [3, 1024, 1 << 16, 1 << 20])
def test_bucket_starts_are_first_positions(B):
    """Bucket b starts at the first position of the scattered array whose
    bucket is at least b, so an empty bucket starts where the next nonempty
    one does and offsets[B] = n; equivalently position p starts the buckets
    b(p-1)+1 .. b(p) (b(-1) = -1, b(n) = B), each exactly once.  Both
    readings of the concatenation give the oracle's offsets, also across wide
    gaps of empty buckets (few distinct keys, many buckets)."""
    n = 3000
    rng = np.random.default_rng(B)
    keys = rng.choice(np.array([0, 7, 1 << 20, (1 << 31) + 5, (1 << 32) - 1], dtype=np.uint64), n).astype(np.uint32)
    res = oracle.bucket(keys, num_buckets=B, want_intermediates=True)
    mn, mx = int(keys.min()), int(keys.max())
    bs = np.array([_py_bucket(int(k), mn, mx, B) for k in res.scat_keys], dtype=np.int64)
    assert np.all(np.diff(bs) >= 0)                        # grouped by bucket, in bucket order
    first = np.searchsorted(bs, np.arange(B + 1), side="left")
    np.testing.assert_array_equal(res.offsets, first.astype(res.offsets.dtype))
    written = np.full(B + 1, -1, dtype=np.int64)
    ext = np.concatenate([[-1], bs, [B]])
    for p in range(n + 1):
        for b in range(ext[p] + 1, ext[p + 1] + 1):
            assert written[b] == -1                        # one writer per offset
            written[b] = p
    np.testing.assert_array_equal(written, res.offsets.astype(np.int64))
