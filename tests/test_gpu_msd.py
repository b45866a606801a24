"""GPU parity of the most-significant-digit-first radix sort (a stable pass on
the top r bits, then each of the 2^r buckets sorted on its remaining bits)
against the oracle: the final keys and stable values, and the array after
the top-digit pass, which is the oracle's bucket scatter over the declared
range [0, 2^key_bits - 1] with 2^r buckets."""
import numpy as np
import pytest

import oracle
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host, rand_keys

pytestmark = pytest.mark.gpu

SIZES = [1, 17, 1000, 8193, 100_003, (1 << 21) + 9]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype,bits", [(np.uint32, 8), (np.uint32, 4), (np.uint32, 11),
                                        (np.uint64, 8), (np.uint64, 11)])
def test_msd_pairs_parity(n, dtype, bits):
    print(f"msd pairs n={n} {np.dtype(dtype).name} r={bits}", flush=True)
    rng = np.random.default_rng(n * 7 + bits)
    keys = rand_keys(rng, n, dtype)
    keys[::5] = keys[-1]
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="msd", digit_bits=bits)
    ref = oracle.radix_lsd(keys, vals, r=8)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
    out = host(I.sort(dev(keys), algo="msd", digit_bits=bits))
    np.testing.assert_array_equal(out, ref.keys)


@pytest.mark.parametrize("dtype,bits", [(np.uint32, 8), (np.uint64, 11)])
def test_msd_top_digit_pass_is_the_scatter(dtype, bits):
    n = 200_003
    print(f"msd top pass n={n} {np.dtype(dtype).name} r={bits}", flush=True)
    keys = rand_keys(np.random.default_rng(bits), n, dtype)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="msd", digit_bits=bits, max_passes=1)
    top = (1 << (8 * keys.dtype.itemsize)) - 1
    ref = oracle.bucket(keys, vals, num_buckets=1 << bits, key_bound=top, want_intermediates=True)
    np.testing.assert_array_equal(host(ok), ref.scat_keys)
    np.testing.assert_array_equal(host(ov), ref.scat_vals)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_msd_all_keys_in_one_bucket(dtype):
    """Keys below 2^20 share the top digit: one bucket holds everything."""
    n = 1_000_003
    print(f"msd one bucket n={n} {np.dtype(dtype).name}", flush=True)
    keys = rand_keys(np.random.default_rng(5), n, dtype, hi=1 << 20)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="msd")
    ref = oracle.radix_lsd(keys, vals, r=8)
    np.testing.assert_array_equal(host(ok), ref.keys)
    np.testing.assert_array_equal(host(ov), ref.vals)
