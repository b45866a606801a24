"""The device form of the input generators against the host form.

The serving benchmark and the largest tests make their keys on the device
(PCIe cannot feed them); parity is always checked on the exact bytes the GPU
sorted, but the inputs should still be the workloads the host generators
define.  The counter-based stream must match value for value (it is integer
only), and so must every distribution that is a plain function of it.  Two
distributions are defined differently on the device on purpose or by
arithmetic:
- "swaps" exchanges floor(n/100) disjoint position pairs (the host makes the
  same number of sequential swaps, which a device cannot do in parallel): the
  result must be the sorted keys with at most 2*floor(n/100) positions moved;
- "gaussian" goes through log and cos, which torch and numpy need not round
  alike in the last place: keys may differ by one where x + 0.5 lands on an
  integer boundary, and only on a tiny share of the keys."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

N = 200_003


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("seed,stream,start", [(0, 0, 0), (7, 3, 0), (5, 1, 123_456_789), (2**40 + 1, 4, 5)])
def test_device_stream_equals_host_stream(seed, stream, start):
    d = _u64(workloads.device_u64_stream(seed, stream, N, "cuda:0", start=start))
    h = workloads.u64_stream(seed, stream, N, start=start)
    np.testing.assert_array_equal(d, h)


@pytest.mark.parametrize("dist", [0, 1, 2, 3, 4])
def test_device_keys_u32_equal_host(dist):
    d = workloads.device_keys(dist, N, dist, 4, "cuda:0").cpu().numpy()
    h = workloads.config2_keys(dist, N, seed=dist)
    assert d.dtype == np.uint32
    np.testing.assert_array_equal(d, h)


@pytest.mark.parametrize("dist,shift", [(0, 0), (1, 54), (2, 48)])
def test_device_keys_u64_fields(dist, shift):
    d = workloads.device_keys(dist, N, 11, 8, "cuda:0").cpu().numpy()
    r = workloads.u64_stream(11, 0, N)
    np.testing.assert_array_equal(d, r >> np.uint64(shift))


@pytest.mark.parametrize("width", [4, 8])
def test_device_sorted_and_reverse_u64(width):
    for dist in (3, 4):
        d = workloads.device_keys(dist, N, 13, width, "cuda:0").cpu().numpy()
        r = workloads.u64_stream(13, 0, N)
        base = np.sort(r if width == 8 else (r >> np.uint64(32)).astype(np.uint32))
        np.testing.assert_array_equal(d, base if dist == 3 else base[::-1])


@pytest.mark.parametrize("width", [4, 8])
def test_device_swaps_moves_few_positions(width):
    d = workloads.device_keys(5, N, 5, width, "cuda:0").cpu().numpy()
    r = workloads.u64_stream(5, 0, N)
    base = np.sort(r if width == 8 else (r >> np.uint64(32)).astype(np.uint32))
    np.testing.assert_array_equal(np.sort(d), base)              # a permutation of the sorted keys
    moved = np.count_nonzero(d != base)
    assert 0 < moved <= 2 * (N // 100)


def test_device_gaussian_close_to_host():
    d = workloads.device_keys(6, N, 6, 4, "cuda:0").cpu().numpy().astype(np.int64)
    h = workloads.config2_keys(6, N, seed=6).astype(np.int64)
    diff = np.abs(d - h)
    assert diff.max() <= 1
    assert np.count_nonzero(diff) <= N // 10_000
