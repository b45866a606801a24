"""GPU parity of the first bucket-sort steps (value range and bucket-index
histogram) against the oracle's intermediates, including the exact bucket
map at every bucket boundary and the full 64-bit range."""
import numpy as np
import pytest

import oracle
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host, rand_keys

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("n", [1, 2, 15, 1000, 100_003])
def test_minmax_parity(dtype, n):
    keys = rand_keys(np.random.default_rng(n), n, dtype)
    mm = host(I.minmax(dev(keys)))
    assert (int(mm[0]), int(mm[1])) == (int(keys.min()), int(keys.max()))


@pytest.mark.parametrize("dtype,B,hi", [(np.uint32, 1024, None), (np.uint32, 7, 1000), (np.uint32, 65536, None),
                                        (np.uint64, 65536, None), (np.uint64, 1000, 1 << 40), (np.uint32, 1, None)])
def test_bucket_histogram_parity(dtype, B, hi):
    n = 200_003
    keys = rand_keys(np.random.default_rng(B), n, dtype, hi)
    ref = oracle.bucket(keys, num_buckets=B, want_intermediates=True)
    d = dev(keys)
    mm = I.minmax(d)
    counts = host(I.bucket_histogram(d, mm, B)).astype(np.uint64)
    np.testing.assert_array_equal(counts, ref.counts)


@pytest.mark.parametrize("dtype,mn,mx,B", [(np.uint32, 0, 2**32 - 1, 1024), (np.uint32, 17, 1040, 7),
                                           (np.uint64, 0, 2**64 - 1, 65536), (np.uint64, 2**40 + 3, 2**41, 1000),
                                           (np.uint32, 5, 5, 3), (np.uint32, 0, 999, 1024),
                                           # 32-bit keys with B >= R (a = floor(B / R) of 3 and 1) and B = 2^24
                                           (np.uint32, 100, 399, 1000), (np.uint32, 7, 7 + 2**20 - 1, 2**20),
                                           (np.uint32, 0, 2**32 - 1, 2**24),
                                           # 64-bit ranges above 2^62: the remainder needs more than 64 bits
                                           (np.uint64, 3, 2**63 + 2**61 + 2, 1000),
                                           (np.uint64, 3, 2**63 + 2**61 + 2, 65536),
                                           (np.uint64, 2**64 - 2**62 - 7, 2**64 - 1, 777),
                                           # R = 2^62 (the double estimate's last range) and 2^62 + 1
                                           (np.uint64, 0, 2**62 - 1, 1000), (np.uint64, 0, 2**62, 1000),
                                           (np.uint64, 10, 2**62 + 10, 3), (np.uint64, 5, 2**62 + 4, 65536)])
def test_bucket_map_at_boundaries(dtype, mn, mx, B):
    """Keys on both sides of every bucket boundary (sampled for large B),
    plus min and max: the device histogram of these keys equals the oracle's.
    For 64-bit keys the device takes b(k) from a double estimate and one
    exact 96-bit remainder check, whose operands grow with R: ranges on
    either side of 2^62 and up to 2^64 are covered; 32-bit keys take one
    fixed-point product, also with B >= R (a = floor(B / R) > 0)."""
    R = mx - mn + 1
    js = range(1, B) if B <= 1024 else list(range(1, 300)) + list(range(B - 300, B))
    ks = [mn, mx]
    for j in js:
        f = mn + -(-j * R // B)
        if mn <= f <= mx:
            ks.append(f)
        if mn <= f - 1 <= mx:
            ks.append(f - 1)
    keys = np.array(ks, dtype=dtype)
    ref = oracle.bucket(keys, num_buckets=B, want_intermediates=True)
    assert (ref.kmin, ref.kmax) == (mn, mx)
    d = dev(keys)
    counts = host(I.bucket_histogram(d, I.minmax(d), B)).astype(np.uint64)
    np.testing.assert_array_equal(counts, ref.counts)
