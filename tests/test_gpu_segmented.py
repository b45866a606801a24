"""GPU parity of the segmented sort: every segment sorted on its own,
bit-exact against the oracle's per-segment sort, across the on-chip size
classes and the multi-workgroup path, with empty segments, segments at the
class boundaries, and the batched workload's log-uniform size mix."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from paper_1206_3511_amd import intsort as I
from gpu_util import dev, host, rand_keys

pytestmark = pytest.mark.gpu

BOUNDARY_SIZES = [0, 1, 2, 255, 256, 257, 2048, 2049, 8192, 8193, 16384, 16385, 40000, 100_000, 0, 5, 3]


def _offsets(sizes):
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)


def _run(keys, offsets, vals=None, **opt):
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    if vals is None:
        return host(I.segmented_sort(dev(keys), offs, **opt)), None
    ok, ov = I.segmented_sort(dev(keys), offs, dev(vals), **opt)
    return host(ok), host(ov)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("pairs", [False, True])
def test_segment_class_boundaries(dtype, pairs):
    offsets = _offsets(BOUNDARY_SIZES)
    n = int(offsets[-1])
    keys = rand_keys(np.random.default_rng(5), n, dtype, hi=None if dtype == np.uint32 else 1 << 40)
    vals = np.arange(n, dtype=np.uint32) if pairs else None
    ok, ov = _run(keys, offsets, vals)
    rk, rv = oracle.segmented(keys, offsets, vals)
    np.testing.assert_array_equal(ok, rk)
    if pairs:
        np.testing.assert_array_equal(ov, rv)


@pytest.mark.parametrize("cutoff", [1, 256, 2048, 8192, 0])
@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_lds_cutoff_does_not_change_result(dtype, cutoff):
    """Every segment size class boundary moved by the cutoff option (longer
    segments take the multi-workgroup path): same bytes as the oracle."""
    offsets = _offsets(BOUNDARY_SIZES)
    n = int(offsets[-1])
    keys = rand_keys(np.random.default_rng(6), n, dtype)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = _run(keys, offsets, vals, lds_cutoff=cutoff)
    rk, rv = oracle.segmented(keys, offsets, vals)
    np.testing.assert_array_equal(ok, rk)
    np.testing.assert_array_equal(ov, rv)


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_log_uniform_mix(dtype):
    sizes, dists = workloads.segment_plan(300, seed=11, lo=16, base=4096)
    offsets = _offsets(sizes)
    n = int(offsets[-1])
    keys = np.empty(n, dtype=dtype)
    for j in range(len(sizes)):
        a, b = int(offsets[j]), int(offsets[j + 1])
        keys[a:b] = workloads.config2_keys(int(dists[j]), b - a, 2000 + j).astype(dtype)
    vals = np.arange(n, dtype=np.uint32)
    ok, ov = _run(keys, offsets, vals)
    rk, rv = oracle.segmented(keys, offsets, vals)
    np.testing.assert_array_equal(ok, rk)
    np.testing.assert_array_equal(ov, rv)


def test_in_place_and_all_empty():
    sizes = [3000, 0, 20000, 7]
    offsets = _offsets(sizes)
    keys = rand_keys(np.random.default_rng(9), int(offsets[-1]), np.uint32)
    t = dev(keys)
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    I.segmented_sort(t, offs, out_keys=t)
    np.testing.assert_array_equal(host(t), oracle.segmented(keys, offsets)[0])
    z = np.zeros(0, dtype=np.uint32)
    out = I.segmented_sort(torch.empty(0, dtype=torch.uint32, device="cuda:0"),
                           torch.zeros(4, dtype=torch.int64, device="cuda:0"))
    assert out.numel() == 0 and z.size == 0


def _seg_hash(a, offsets):
    h = workloads.mix64(a.astype(np.uint64) * workloads.GAMMA)
    return np.add.reduceat(h, offsets[:-1].astype(np.int64)) if a.size else h


def test_config4_full_batch():
    """10,000 uint32 arrays, sizes log-uniform in [16, 2^20), distributions
    from the seven of the 100M workload: every segment nondecreasing with the
    same multiset as its input (order-independent hash), and 200 sampled
    segments plus the largest compared element by element with the oracle."""
    keys, offsets = workloads.segmented_keys()
    print(f"config4: {keys.size} keys", flush=True)
    out, _ = _run(keys, offsets)
    n = keys.size
    d = np.diff(out.astype(np.int64))
    starts = offsets[1:-1].astype(np.int64) - 1
    d[starts[(starts >= 0) & (starts < n - 1)]] = 0
    assert np.all(d >= 0)
    sizes = np.diff(offsets.astype(np.int64))
    nz = sizes > 0
    hi = _seg_hash(keys, offsets)[nz[:len(offsets) - 1]]
    ho = _seg_hash(out, offsets)[nz[:len(offsets) - 1]]
    np.testing.assert_array_equal(hi, ho)
    rng = np.random.default_rng(4)
    sample = list(rng.choice(len(sizes), 200, replace=False)) + [int(np.argmax(sizes))]
    for s in sample:
        a, b = int(offsets[s]), int(offsets[s + 1])
        np.testing.assert_array_equal(out[a:b], oracle.radix_lsd(keys[a:b]).keys)
    assert I.device_error(0) == 0
