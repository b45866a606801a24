"""GPU parity of the LSD radix sort (HIP path through the C ABI) against the
CPU oracle: bit-exact keys, and for pairs bit-exact (stable) values, on the
same seeded inputs.  Sizes span several tiles and ragged tails; the
intermediate arrays after every digit pass and the one-read digit histogram
are checked against the oracle's intermediates."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host, rand_keys

pytestmark = pytest.mark.gpu

TILE32 = 8192     # keys per tile of the 32-bit, 8-bit-digit pass kernel
SIZES = [1, 2, 3, 17, 64, 1000, TILE32 - 1, TILE32, TILE32 + 1, 3 * TILE32 + 5, 100_003]


def _rng(*salt):
    return np.random.default_rng(abs(hash(salt)) % (1 << 32))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype,bits", [(np.uint32, 8), (np.uint32, 4), (np.uint32, 11),
                                        (np.uint64, 8), (np.uint64, 11), (np.uint64, 4)])
def test_radix_keys_parity(n, dtype, bits):
    print(f"radix keys n={n} {np.dtype(dtype).name} r={bits}", flush=True)
    keys = rand_keys(np.random.default_rng(n * 31 + bits), n, dtype)
    out = host(I.sort(dev(keys), algo="radix", digit_bits=bits))
    ref = oracle.radix_lsd(keys, r=bits).keys
    np.testing.assert_array_equal(out, ref)


@pytest.mark.parametrize("n", [5, 1000, TILE32 + 1, 3 * TILE32 + 5, 100_003])
@pytest.mark.parametrize("dtype,bits", [(np.uint32, 8), (np.uint32, 11), (np.uint64, 8), (np.uint64, 11)])
def test_radix_pairs_stable_parity(n, dtype, bits):
    print(f"radix pairs n={n} {np.dtype(dtype).name} r={bits}", flush=True)
    rng = np.random.default_rng(n + bits)
    keys = rand_keys(rng, n, dtype, hi=max(2, n // 7))   # many equal keys
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="radix", digit_bits=bits)
    ref = oracle.radix_lsd(keys, vals, r=bits)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)


@pytest.mark.parametrize("dist", range(7))
def test_radix_distributions(dist):
    n = (1 << 20) + 123
    print(f"radix dist={workloads.DISTRIBUTIONS[dist]} n={n}", flush=True)
    keys = workloads.config2_keys(dist, n)
    out = host(I.sort(dev(keys), algo="radix"))
    np.testing.assert_array_equal(out, oracle.radix_lsd(keys, r=8).keys)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="radix")
    ref = oracle.radix_lsd(keys, vals, r=8)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)


@pytest.mark.parametrize("dtype,bits", [(np.uint32, 8), (np.uint64, 11), (np.uint32, 4)])
def test_pass_intermediates(dtype, bits):
    """After p passes the array is the oracle's array after pass p (the LSD
    invariant of Algorithm 4): checks every pass kernel on its own."""
    n = 3 * TILE32 + 77
    print(f"intermediates {np.dtype(dtype).name} r={bits}", flush=True)
    keys = rand_keys(np.random.default_rng(7), n, dtype)
    vals = np.arange(n, dtype=np.uint32)
    ref = oracle.radix_lsd(keys, vals, r=bits, want_passes=True)
    for p in range(1, ref.passes + 1):
        ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="radix", digit_bits=bits, max_passes=p)
        np.testing.assert_array_equal(host(ok), ref.pass_keys[p - 1])


@pytest.mark.parametrize("dtype,bits", [(np.uint32, 8), (np.uint32, 11), (np.uint64, 8), (np.uint64, 4)])
@pytest.mark.parametrize("n", [1, 1001, 100_003])
def test_digit_histogram_parity(dtype, bits, n):
    keys = rand_keys(np.random.default_rng(n), n, dtype, hi=None if n > 2000 else 5000)
    counts = host(I.digit_histogram(dev(keys), bits)).astype(np.uint64)
    ref = oracle.radix_lsd(keys, r=bits, want_counts=True).pass_counts
    np.testing.assert_array_equal(counts, ref)


def test_in_place_and_streams():
    n = 50_000
    keys = workloads.config2_keys(0, n)
    ref = oracle.radix_lsd(keys).keys
    t = dev(keys)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        I.sort(t, out=t, algo="radix", stream=s)
    s.synchronize()
    np.testing.assert_array_equal(host(t), ref)
    # small range: two of four passes skipped, with and without skipping
    small = workloads.config2_keys(1, n)
    for skip in (True, False):
        t = dev(small)
        I.sort(t, out=t, skip_passes=skip)
        np.testing.assert_array_equal(host(t), np.sort(small))
        np.testing.assert_array_equal(host(I.sort(dev(small), skip_passes=skip)), oracle.radix_lsd(small).keys)


def test_all_equal_and_special_keys():
    for dtype in (np.uint32, np.uint64):
        mx = int(np.iinfo(dtype).max)
        for n in (1, 63, 64, 65, TILE32 + 3):
            a = np.full(n, mx, dtype=dtype)
            np.testing.assert_array_equal(host(I.sort(dev(a))), a)
        special = np.array([0, 1, 2**31 - 1, 2**31, 2**32 - 1] + ([2**63, mx - 1, mx] if dtype == np.uint64 else []),
                           dtype=dtype)
        a = np.tile(special, 3000)
        np.random.default_rng(3).shuffle(a)
        vals = np.arange(a.size, dtype=np.uint32)
        ok, ov = I.sort_pairs(dev(a), dev(vals))
        ref = oracle.radix_lsd(a, vals)
        np.testing.assert_array_equal(host(ok), ref.keys)
        np.testing.assert_array_equal(host(ov), ref.vals)


def test_repeatable_and_no_device_error():
    keys = workloads.config2_keys(6, 300_000)
    a = host(I.sort(dev(keys)))
    b = host(I.sort(dev(keys)))
    assert a.tobytes() == b.tobytes()
    assert I.device_error(0) == 0


def test_config1_full():
    """1,000,000 uniform uint32 keys, seed 0, 8-bit digits, 4 passes."""
    keys = workloads.config2_keys(0, 1_000_000, seed=0)
    out = host(I.sort(dev(keys), digit_bits=8))
    np.testing.assert_array_equal(out, oracle.radix_lsd(keys, r=8).keys)


@pytest.mark.parametrize("dist", range(7))
def test_config2_full_size(dist):
    """100,000,000 uint32 keys of each distribution, radix, in the launch
    configuration the benchmark times; compared element by element with the
    oracle."""
    n = 100_000_000
    print(f"full size dist={workloads.DISTRIBUTIONS[dist]}", flush=True)
    keys = workloads.config2_keys(dist, n)
    out = host(I.sort(dev(keys), algo="radix"))
    ref = oracle.radix_lsd(keys, r=8).keys
    np.testing.assert_array_equal(out, ref)
    assert I.device_error(0) == 0


# 32-bit key sorts (keys alone or with values) of at least 2048 tiles take
# the first pass without a look-back: its per-tile digit offsets come from the histogram kernel and a
# scan over chunks of tiles
SCANNED_N = 2048 * 16384 + 4099


@pytest.mark.parametrize("case", ["uniform", "low_byte_constant", "small_range"])
def test_scanned_first_pass(case):
    print(f"scanned first pass n={SCANNED_N} case={case}", flush=True)
    keys = workloads.config2_keys(0, SCANNED_N, seed=21)
    if case == "low_byte_constant":
        keys = (keys & np.uint32(0xFFFFFF00)) | np.uint32(0x5A)   # pass 0 skipped: look-back from pass 1
    elif case == "small_range":
        keys = keys >> np.uint32(22)                             # passes 2 and 3 skipped
    out = host(I.sort(dev(keys)))
    np.testing.assert_array_equal(out, oracle.radix_lsd(keys, r=8).keys)
    assert I.device_error(0) == 0
    # the intermediate array after the first pass alone
    one = host(I.sort(dev(keys), digit_bits=8, max_passes=1))
    np.testing.assert_array_equal(one, oracle.radix_lsd(keys, r=8, want_passes=True).pass_keys[0])


@pytest.mark.parametrize("case", ["uniform", "small_range"])
def test_scanned_first_pass_pairs(case):
    """Key-value sorts through the first pass without a look-back: keys and
    stable values bit-exact against the oracle."""
    print(f"scanned first pass pairs n={SCANNED_N} case={case}", flush=True)
    keys = workloads.config2_keys(0, SCANNED_N, seed=22)
    if case == "small_range":
        keys = keys >> np.uint32(22)
    vals = np.arange(SCANNED_N, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals))
    ref = oracle.radix_lsd(keys, vals, r=8)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    assert I.device_error(0) == 0
