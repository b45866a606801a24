"""The largest input a call takes, 2^30 - 1 keys (a tile's 30-bit status count
bounds n), and the 100M-key uint64 key-value configuration.

At 2^30 - 1 keys the results are checked through properties that hold at
any size and fix the stable sort completely: the output is nondecreasing
and a permutation of the input (for keys alone: equal to the library sort,
torch.sort on the device), and for key-value sorts every value is the index
of the input key that lands beside it (keys_in[vals] == keys), with indices
increasing inside every run of equal keys (stability).  The 100M-key
key-value configuration is compared with the oracle element by element (a
few GB of host memory and seconds of oracle time per case)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1206_3511_amd import intsort as I

pytestmark = pytest.mark.gpu

N_MAX = (1 << 30) - 1


def _i64(t):
    return t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF


def _check_keys(keys, out):
    a, b = _i64(out), _i64(keys)
    assert bool((a[1:] >= a[:-1]).all())
    assert torch.equal(a, torch.sort(b).values)


@pytest.mark.parametrize("algo", ["radix", "bucket"])
def test_max_size_keys(algo):
    print(f"max size keys {algo} n={N_MAX}", flush=True)
    keys = workloads.device_keys(0, N_MAX, 77, 4, "cuda:0")
    out = I.sort(keys, algo=algo)
    torch.cuda.synchronize()
    assert I.device_error(0) == 0
    _check_keys(keys, out)


def test_max_size_pairs_stable():
    print(f"max size pairs n={N_MAX}", flush=True)
    keys = workloads.device_keys(1, N_MAX, 78, 4, "cuda:0")     # [0, 1024): long runs of equal keys
    vals = torch.arange(N_MAX, dtype=torch.int32, device="cuda:0").view(torch.uint32)
    ok, ov = I.sort_pairs(keys, vals)
    torch.cuda.synchronize()
    assert I.device_error(0) == 0
    k, v = _i64(ok), _i64(ov)
    assert bool((k[1:] >= k[:-1]).all())
    assert torch.equal(_i64(keys)[v], k)                          # every value names its key
    same = k[1:] == k[:-1]
    assert bool((v[1:][same] > v[:-1][same]).all())              # stable inside runs
    del same
    assert torch.equal(torch.sort(v).values, torch.arange(N_MAX, device="cuda:0"))   # a permutation


def _check_pairs(keys64, ok, ov):
    """Stable key-value sort of 64-bit keys with the index as value."""
    k = ok.view(torch.int64)
    flip = -(1 << 63)
    ks = k ^ flip                                   # signed order of the unsigned keys
    assert bool((ks[1:] >= ks[:-1]).all())
    v = ov.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    assert torch.equal(keys64.view(torch.int64)[v], k)
    same = k[1:] == k[:-1]
    assert bool((v[1:][same] > v[:-1][same]).all())
    assert torch.equal(torch.sort(v).values, torch.arange(k.numel(), device=k.device))


_CONFIG3 = {}


def _config3(variant):
    """The 100M-key input of a variant, made once per process."""
    if variant not in _CONFIG3:
        _CONFIG3.clear()
        _CONFIG3[variant] = workloads.config3_pairs(variant, 100_000_000)
    return _CONFIG3[variant]


@pytest.mark.parametrize("variant,algo,bits", [("full", "radix", 8), ("full", "radix", 11), ("full", "bucket", 8),
                                               ("b40", "radix", 8), ("b40", "radix", 11), ("b40", "bucket", 8)])
def test_config3_full_size_pairs(variant, algo, bits):
    """100,000,000 uint64 keys with the uint32 index as payload, in the launch
    configuration the benchmark times (65536 buckets for bucket sort): keys
    and values equal the oracle's element by element (radix sort with the
    same digit width, or bucket sort with the same bucket count), after the
    properties that fix a stable sort are checked on the device."""
    print(f"config3 {variant} {algo} r={bits}", flush=True)
    kh, vh = _config3(variant)
    keys = torch.from_numpy(kh).to("cuda:0")
    vals = torch.from_numpy(vh).to("cuda:0")
    B = 65536 if algo == "bucket" else 0
    ok, ov = I.sort_pairs(keys, vals, algo=algo, digit_bits=bits, num_buckets=B)
    torch.cuda.synchronize()
    assert I.device_error(0) == 0
    _check_pairs(keys, ok, ov)
    gk, gv = ok.cpu().numpy(), ov.cpu().numpy()
    del keys, vals, ok, ov
    print(f"config3 {variant} {algo} r={bits}: oracle", flush=True)
    ref = oracle.radix_lsd(kh, vh, r=bits) if algo == "radix" else oracle.bucket(kh, vh, num_buckets=B)
    np.testing.assert_array_equal(gk, ref.keys)
    np.testing.assert_array_equal(gv, ref.vals)
