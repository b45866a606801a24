"""GPU parity of radix sort on signed and IEEE 754 keys (HIP path through the
C ABI) against the oracle's stable sort under signed order and IEEE 754-2019
totalOrder: bit-exact keys (every NaN payload and the sign of zero survive)
and, for pairs, bit-exact stable values.  Sizes span several tiles and
ragged tails; inputs include every special value class, keys that share
their high digits (so digit passes are skipped) and the extremes of each
type."""
import numpy as np
import pytest

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

TILE32 = 8192
SIZES = [1, 2, 17, 1000, TILE32 + 1, 3 * TILE32 + 5, 100_003, (1 << 20) + 77]


def _bits(a):
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def _check(keys, vals=None):
    ref_k, ref_v = oracle.sort_ordered(keys, vals)
    if vals is None:
        out = host(I.sort(dev(keys), algo="radix"))
        np.testing.assert_array_equal(_bits(out), _bits(ref_k))
        return
    ok, ov = I.sort_pairs(dev(keys), dev(vals), algo="radix")
    np.testing.assert_array_equal(_bits(host(ok)), _bits(ref_k))
    np.testing.assert_array_equal(host(ov), ref_v)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("width", [32, 64])
def test_signed_keys_parity(n, width):
    print(f"signed keys n={n} int{width}", flush=True)
    _check(workloads.signed_keys(n, width, seed=n + width))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("width", [32, 64])
def test_ieee_keys_parity(n, width):
    print(f"ieee keys n={n} float{width}", flush=True)
    _check(workloads.ieee_keys(n, width, seed=n + width))


@pytest.mark.parametrize("n", [5, TILE32 + 1, 100_003])
@pytest.mark.parametrize("kind", ["int32", "int64", "float32", "float64"])
def test_ordered_pairs_stable_parity(n, kind):
    print(f"ordered pairs n={n} {kind}", flush=True)
    width = 32 if kind.endswith("32") else 64
    if kind.startswith("int"):
        keys = workloads.signed_keys(n, width, seed=3 * n, spread_bits=6)   # many equal keys
    else:
        keys = workloads.ieee_keys(n, width, seed=3 * n, special_share=4)
    _check(keys, np.arange(n, dtype=np.uint32))


@pytest.mark.parametrize("kind", ["int32", "int64", "float32", "float64"])
def test_ordered_narrow_range_skips_passes(kind):
    """Keys near zero of both signs share their high digits after the order
    transform only within each sign: mixed signs must still sort across the
    boundary, and one-signed inputs exercise the skipped passes."""
    n = 300_001
    width = 32 if kind.endswith("32") else 64
    for sign in (0, -1, 1):
        print(f"narrow {kind} sign={sign}", flush=True)
        if kind.startswith("int"):
            k = workloads.signed_keys(n, width, seed=11, spread_bits=12)
            k = np.abs(k) if sign == 1 else (-np.abs(k) if sign == -1 else k)
        else:
            k = workloads.ieee_keys(n, width, seed=11, special_share=1 << 30)
            k = (np.abs(k) % 3.0 + 1.0).astype(k.dtype)          # [1, 4): few exponents
            k = k if sign == 1 else (-k if sign == -1 else np.where(np.arange(n) % 2 == 0, k, -k))
        _check(np.ascontiguousarray(k), np.arange(n, dtype=np.uint32))


@pytest.mark.parametrize("kind", ["int32", "int64", "float32", "float64"])
def test_ordered_extremes_and_constant(kind):
    width = 32 if kind.endswith("32") else 64
    dt = np.dtype(kind)
    if kind.startswith("int"):
        info = np.iinfo(dt)
        ext = np.array([info.min, info.max, -1, 0, 1, info.min + 1, info.max - 1], dtype=dt)
    else:
        ut = np.uint32 if width == 32 else np.uint64
        top = 1 << (width - 1)
        inf = 0x7F800000 if width == 32 else 0x7FF0000000000000
        quiet = 1 << (22 if width == 32 else 51)
        # +0, -0, +inf, -inf, +sNaN, -sNaN, +qNaN, -NaN with every payload
        # bit set, the smallest subnormals of both signs
        ext = np.array([0, top, inf, inf | top, inf | 1, inf | 1 | top, inf | quiet,
                        (1 << width) - 1, 1, top | 1], dtype=np.uint64).astype(ut).view(dt)
    rng = np.random.default_rng(width)
    for n in (len(ext), 4097, 70_001):
        print(f"extremes {kind} n={n}", flush=True)
        k = ext[rng.integers(0, len(ext), n)] if n > len(ext) else ext.copy()
        _check(k, np.arange(n, dtype=np.uint32))
    print(f"constant {kind}", flush=True)
    _check(np.full(50_000, ext[3], dtype=dt), np.arange(50_000, dtype=np.uint32))


def test_ordered_empty_and_unsupported():
    for dt in (np.int32, np.int64, np.float32, np.float64):
        e = np.empty(0, dtype=dt)
        assert host(I.sort(dev(e), algo="radix")).size == 0
        k = dev(np.zeros(10, dtype=dt))
        with pytest.raises(RuntimeError):
            I.sort(k, algo="bucket")
        with pytest.raises(RuntimeError):
            I.sort(k, algo="radix", digit_bits=11)


@pytest.mark.parametrize("kind", ["int32", "float32"])
def test_ordered_scanned_first_pass(kind):
    """32-bit sorts of at least 2048 tiles take the first pass without a
    look-back; signed and IEEE keys through that path."""
    n = 2048 * 16384 + 777
    print(f"ordered scanned first pass n={n} {kind}", flush=True)
    keys = workloads.signed_keys(n, 32, seed=5) if kind == "int32" else workloads.ieee_keys(n, 32, seed=5)
    _check(keys)
