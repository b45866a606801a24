"""Key-value sorts where only one of keys and values is sorted in place.

The header allows keys and values to alias independently (keys_in ==
keys_out, vals_in == vals_out, or both, or neither).  No pass may then read
and write one buffer, and the final copy must move exactly what is not
already in place.  Every mix is checked element by element against the
oracle's stable sort (section 2, stability), on inputs whose active pass
count is odd (the last pass lands in scratch), even, and zero (no pass runs,
so only a copy can put the result in place)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host, rand_keys

pytestmark = pytest.mark.gpu

# 32-bit key sorts of at least 2048 tiles of 16384 keys take the first pass
# without a look-back
SCANNED_N = 2048 * 16384 + 4099


def _mix_call(fn, keys, vals, mix):
    """Runs fn(k, v, out_keys, out_vals) with the aliasing `mix` and returns
    host copies of the results."""
    k, v = dev(keys), dev(vals)
    ok = k if mix in ("keys", "both") else torch.empty_like(k)
    ov = v if mix in ("vals", "both") else torch.empty_like(v)
    rk, rv = fn(k, v, ok, ov)
    assert rk.data_ptr() == ok.data_ptr() and rv.data_ptr() == ov.data_ptr()
    if mix in ("keys", "both"):
        assert ok.data_ptr() == k.data_ptr()
    out = host(ok), host(ov)
    # the input that was not aliased is left as it was
    if mix == "vals":
        np.testing.assert_array_equal(host(k), keys)
    if mix == "keys":
        np.testing.assert_array_equal(host(v), vals)
    return out


def _case_keys(case, n):
    rng = np.random.default_rng(abs(hash(case)) % (1 << 32))
    if case == "u32_24bit":      # r=8: three active passes (odd)
        return rng.integers(0, 1 << 24, n, dtype=np.uint64).astype(np.uint32), 8
    if case == "u32_r11":        # r=11: three passes
        return rand_keys(rng, n, np.uint32), 11
    if case == "u32_full":       # r=8: four passes (even)
        return rand_keys(rng, n, np.uint32), 8
    if case == "u64_r8_40bit":   # r=8: five active passes
        return rng.integers(0, 1 << 40, n, dtype=np.uint64), 8
    if case == "equal":          # every digit constant: no pass runs
        return np.full(n, 0x12345678, dtype=np.uint32), 8
    raise ValueError(case)


@pytest.mark.parametrize("mix", ["keys", "vals", "both"])
@pytest.mark.parametrize("case", ["u32_24bit", "u32_r11", "u32_full", "u64_r8_40bit", "equal"])
@pytest.mark.parametrize("n", [1, 100_003])
def test_radix_pairs_mixed_aliasing(mix, case, n):
    print(f"radix aliasing mix={mix} case={case} n={n}", flush=True)
    keys, r = _case_keys(case, n)
    vals = np.arange(n, dtype=np.uint32)[::-1].copy()
    ok, ov = _mix_call(lambda k, v, a, b: I.sort_pairs(k, v, algo="radix", digit_bits=r, out_keys=a,
                                                       out_vals=b), keys, vals, mix)
    ref = oracle.radix_lsd(keys, vals, r=r)
    np.testing.assert_array_equal(ok, ref.keys)
    np.testing.assert_array_equal(ov, ref.vals)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("mix", ["keys", "vals"])
def test_radix_pairs_mixed_aliasing_first_pass_without_look_back(mix):
    """The large 32-bit path (per-tile first-pass offsets) with an odd number
    of active passes."""
    print(f"radix aliasing scanned mix={mix}", flush=True)
    keys = workloads.config2_keys(0, SCANNED_N, seed=31) >> np.uint32(8)   # three active passes
    vals = np.arange(SCANNED_N, dtype=np.uint32)
    ok, ov = _mix_call(lambda k, v, a, b: I.sort_pairs(k, v, out_keys=a, out_vals=b), keys, vals, mix)
    ref = oracle.radix_lsd(keys, vals, r=8)
    np.testing.assert_array_equal(ok, ref.keys)
    np.testing.assert_array_equal(ov, ref.vals)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("mix", ["keys", "vals", "both"])
@pytest.mark.parametrize("case", ["equal", "u32_24bit", "u32_full"])
def test_segmented_pairs_mixed_aliasing(mix, case):
    """Large segments (past one workgroup's LDS) take the multi-workgroup
    passes with their own scratch/output ping-pong; small ones sort on chip."""
    print(f"segmented aliasing mix={mix} case={case}", flush=True)
    sizes = [70_000, 17, 40_000, 0, 5_000, 90_001]
    n = sum(sizes)
    keys, _ = _case_keys(case, n)
    vals = np.arange(n, dtype=np.uint32)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    ok, ov = _mix_call(lambda k, v, a, b: I.segmented_sort(k, offs, vals=v, out_keys=a, out_vals=b),
                       keys, vals, mix)
    rk, rv = oracle.segmented(keys, offsets, vals)
    np.testing.assert_array_equal(ok, rk)
    np.testing.assert_array_equal(ov, rv)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("mix", ["keys", "vals", "both"])
@pytest.mark.parametrize("algo,buckets,dtype", [("bucket", 256, np.uint32), ("bucket", 70_000, np.uint32),
                                                ("bucket", 1024, np.uint64), ("msd", 0, np.uint32)])
def test_bucket_scatter_only_in_place(mix, algo, buckets, dtype):
    """max_passes = 1 stops after the stable scatter, which writes the
    caller's output directly: 1 pass (B = 256, MSD r = 8), 2 passes
    (B = 1024) or 3 passes (B = 70,000), on unsorted keys."""
    n = 100_003
    print(f"bucket scatter in place mix={mix} {algo} B={buckets} {np.dtype(dtype).name}", flush=True)
    keys = rand_keys(np.random.default_rng(buckets + n), n, dtype)
    vals = np.arange(n, dtype=np.uint32)
    opt = dict(max_passes=1)
    if algo == "bucket":
        opt["num_buckets"] = buckets
    ok, ov = _mix_call(lambda k, v, a, b: I.sort_pairs(k, v, algo=algo, out_keys=a, out_vals=b, **opt),
                       keys, vals, mix)
    if algo == "msd":
        top = (1 << (8 * keys.dtype.itemsize)) - 1
        ref = oracle.bucket(keys, vals, num_buckets=256, want_intermediates=True, key_bound=top)
    else:
        ref = oracle.bucket(keys, vals, num_buckets=buckets, want_intermediates=True)
    np.testing.assert_array_equal(ok, ref.scat_keys)
    np.testing.assert_array_equal(ov, ref.scat_vals)
    assert I.device_error(0) == 0


@pytest.mark.parametrize("algo", ["bucket", "msd"])
def test_bucket_scatter_only_in_place_keys_only(algo):
    n = 100_003
    print(f"bucket scatter in place keys only {algo}", flush=True)
    keys = rand_keys(np.random.default_rng(5), n, np.uint32)
    t = dev(keys)
    opt = dict(max_passes=1)
    if algo == "bucket":
        opt["num_buckets"] = 256
    I.sort(t, algo=algo, out=t, **opt)
    ref = oracle.bucket(keys, num_buckets=256, want_intermediates=True,
                        key_bound=(1 << 32) - 1 if algo == "msd" else 0)
    np.testing.assert_array_equal(host(t), ref.scat_keys)
    assert I.device_error(0) == 0
