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


def test_config4_full_batch():
    """10,000 uint32 arrays, sizes log-uniform in [16, 2^20), distributions
    from the seven of the 100M workload, sorted in one segmented call: every
    one of the 10,000 segments equals the oracle's element by element (the
    oracle sorts each segment on its own, about 9.4e8 keys in all)."""
    keys, offsets = workloads.segmented_keys()
    print(f"config4: {keys.size} keys", flush=True)
    out, _ = _run(keys, offsets)
    assert I.device_error(0) == 0
    print("config4: oracle", flush=True)
    ref, _ = oracle.segmented(keys, offsets)
    np.testing.assert_array_equal(out, ref)


def test_check_segments_flag():
    """With INTSORT_FLAG_CHECK_SEGMENTS the segment layout is checked on the
    device first: a valid one sorts as usual with a clean error word; a bad
    one (decreasing offsets, an end past the keys, a start other than 0) sets
    the bad-segments bit and nothing is sorted.  A valid call afterwards is
    correct again."""
    n = 50_000
    keys = rand_keys(np.random.default_rng(12), n, np.uint32)
    good = np.array([0, 100, 20_000, n], dtype=np.uint64)
    out, _ = _run(keys, good, check_segments=True)
    np.testing.assert_array_equal(out, oracle.segmented(keys, good)[0])
    assert I.device_error(0) == 0
    for bad in ([0, 30_000, 20_000, n], [0, 100, n + 10_000], [5, 100, n]):
        print(f"bad layout {bad}", flush=True)
        _run(keys, np.array(bad, dtype=np.uint64), check_segments=True)
        assert I.device_error(0) & I.DEVERR_BAD_SEGMENTS
    out, _ = _run(keys, good, check_segments=True)
    np.testing.assert_array_equal(out, oracle.segmented(keys, good)[0])
    assert I.device_error(0) == 0


def test_check_segments_flag_batched():
    """The same check for separate arrays: a descriptor whose buffer is not
    16-byte aligned, or lengths that add up past total_keys, are reported and
    nothing is sorted; a good batch afterwards sorts."""
    import ctypes
    a = dev(rand_keys(np.random.default_rng(13), 4096, np.uint32))
    b = torch.empty_like(a)
    ctx = I.context(0)
    o = I.make_options(check_segments=True)
    p, q = a.data_ptr(), b.data_ptr()
    cases = [([[p, q, 1000]], 4096, False),
             ([[p + 4, q, 1000]], 4096, True),                      # misaligned input
             ([[p, q, 1000], [p + 4096, q + 4096, 1000]], 1500, True),   # 2000 keys > total 1500
             ([[p, q, 2000], [p + 8000, q + 8000, 2096]], 4096, False)]
    for rows, total, expect_bad in cases:
        print(f"batched check {rows} total={total}", flush=True)
        desc = torch.tensor(rows, dtype=torch.int64).to("cuda:0")
        ws = ctx.workspace(ctx.workspace_size(I.U32, False, total, len(rows), o))
        rc = I.lib().intsort_batched_sort_keys(ctx.handle, I.U32, desc.data_ptr(), len(rows), total, ctypes.byref(o),
                                               ws.data_ptr(), ws.numel(), None)
        assert rc == I.OK
        torch.cuda.synchronize()
        assert bool(I.device_error(0) & I.DEVERR_BAD_SEGMENTS) == expect_bad
        if not expect_bad:
            ha, hb = host(a), host(b)
            at = 0
            for r in rows:
                m = r[2]
                np.testing.assert_array_equal(hb[at:at + m], np.sort(ha[at:at + m]))
                at += m


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
@pytest.mark.parametrize("pairs", [False, True])
@pytest.mark.parametrize("cutoff", [1, 0])
def test_four_bit_digits(dtype, pairs, cutoff):
    """Segmented sorts with 4-bit digits (twice the passes of the longer
    segments, 16 digits each): the same bytes as the oracle, with every
    segment on the multi-workgroup path (cutoff 1) or only the long ones,
    and with keys whose top nibbles are constant (passes skipped)."""
    offsets = _offsets(BOUNDARY_SIZES)
    n = int(offsets[-1])
    for hi in (None, 1 << 20):
        keys = rand_keys(np.random.default_rng(7), n, dtype, hi=hi)
        vals = np.arange(n, dtype=np.uint32) if pairs else None
        ok, ov = _run(keys, offsets, vals, digit_bits=4, lds_cutoff=cutoff)
        rk, rv = oracle.segmented(keys, offsets, vals)
        np.testing.assert_array_equal(ok, rk)
        if pairs:
            np.testing.assert_array_equal(ov, rv)
    with pytest.raises(I.IntsortError) as e:
        _run(keys, offsets, vals, digit_bits=11)
    assert e.value.status == I.ERR_UNSUPPORTED


@pytest.mark.parametrize("dtype", [np.uint32, np.uint64])
def test_four_bit_digits_batched_and_in_place(dtype):
    sizes = [70_000, 1, 0, 16_385, 300_001, 9000]
    arrays = [rand_keys(np.random.default_rng(11 + i), m, dtype) for i, m in enumerate(sizes) if m]
    ins = [dev(a) for a in arrays]
    outs = I.batched_sort(ins, digit_bits=4, lds_cutoff=2048)
    for a, o in zip(arrays, outs):
        np.testing.assert_array_equal(host(o), np.sort(a))
    offsets = _offsets(sizes)
    keys = np.concatenate(arrays)
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    t = dev(keys)
    I.segmented_sort(t, offs, out_keys=t, digit_bits=4, lds_cutoff=1)
    np.testing.assert_array_equal(host(t), oracle.segmented(keys, offsets)[0])


def test_tuned_digit_width_is_taken(tmp_path):
    """A tuning-table entry for segmented digit width 4 makes a call with a
    zero digit_bits run 4-bit passes (8 launches for 32-bit keys)."""
    sizes = [100_000, 50_000]
    offsets = _offsets(sizes)
    n = int(offsets[-1])
    keys = rand_keys(np.random.default_rng(3), n, np.uint32)
    cls = int(np.floor(np.log2(n)))
    path = tmp_path / "tune.tsv"
    path.write_text(f"*\tsegmented_bits\t4\t{cls}\t4\n")
    ctx = I.context(0)
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    try:
        ctx.load_tuning(str(path))
        ctx.timing(True)
        ctx.kernel_times()
        out = I.segmented_sort(dev(keys), offs, lds_cutoff=1)
        passes = {i for kind, i, _ in ctx.kernel_times() if kind == "pass"}
    finally:
        ctx.timing(False)
        ctx.load_tuning(None)
    np.testing.assert_array_equal(host(out), oracle.segmented(keys, offsets)[0])
    assert passes == set(range(8))
