"""The seeded input generator: SplitMix64 known answers, determinism,
counter-based random access, distribution shapes and recorded checksums."""
import json
import os

import numpy as np

import workloads as w

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_known_answers():
    # SplitMix64 started from state 0 (Steele, Lea, Flood 2014): the first
    # three outputs, as widely reproduced from the published generator
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [w.mix64_int((i + 1) * int(w.GAMMA) & ((1 << 64) - 1)) for i in range(3)]
    assert got == expect
    arr = w.mix64(np.arange(1, 4, dtype=np.uint64) * w.GAMMA)
    assert [int(x) for x in arr] == expect


def test_counter_based_random_access():
    full = w.u64_stream(3, 1, 1000)
    np.testing.assert_array_equal(full[400:700], w.u64_stream(3, 1, 300, start=400))
    assert not np.array_equal(w.u64_stream(3, 1, 10), w.u64_stream(3, 2, 10))
    assert not np.array_equal(w.u64_stream(3, 1, 10), w.u64_stream(4, 1, 10))


def test_distribution_shapes():
    n = 1 << 15
    k = [w.config2_keys(d, n) for d in range(7)]
    assert all(a.dtype == np.uint32 and a.size == n for a in k)
    assert k[1].max() < 1024 and k[2].max() < (1 << 16)
    assert np.all(np.diff(k[3].astype(np.int64)) >= 0)
    assert np.all(np.diff(k[4].astype(np.int64)) <= 0)
    inv = np.count_nonzero(np.diff(k[5].astype(np.int64)) < 0)
    assert 0 < inv <= 2 * (n // 100) * 2
    np.testing.assert_array_equal(np.sort(k[5]), np.sort(w.uniform_u32(n, 5)))
    # gaussian clusters: the keys concentrate near at most 16 centres
    hist = np.bincount((k[6] >> 24).astype(np.int64), minlength=256)
    assert np.count_nonzero(hist) <= 16 * 2 + 4


def test_determinism_and_recorded_checksums():
    g = json.load(open(os.path.join(HERE, "golden", "input_checksums.json")))
    n = g["n"]
    for d, name in enumerate(w.DISTRIBUTIONS):
        a = w.config2_keys(d, n)
        np.testing.assert_array_equal(a, w.config2_keys(d, n))
        assert hex(w.checksum(a)) == g["config2"][name], name
    for v in ("full", "b40"):
        k, p = w.config3_pairs(v, n)
        assert hex(w.checksum(k)) == g["config3"][v]
        np.testing.assert_array_equal(p, np.arange(n, dtype=np.uint32))
    sizes, dists = w.segment_plan(64)
    assert [int(x) for x in sizes] == g["segment_plan_64"]["sizes"]
    assert [int(x) for x in dists] == g["segment_plan_64"]["dists"]
    assert sizes.min() >= 16 and sizes.max() < 16 * 65536


def test_segmented_keys_layout():
    keys, off = w.segmented_keys(num_segments=20, lo=16, base=64)
    assert off.dtype == np.uint64 and off[0] == 0 and int(off[-1]) == keys.size
    assert np.all(np.diff(off.astype(np.int64)) >= 16)


def test_paper_cases_shapes_and_checksums():
    """The six input cases of section 3.1: range, order, repeated value, and
    the recorded checksums of their first 2^16-key instances."""
    gold = json.load(open(os.path.join(HERE, "golden", "input_checksums.json")))["paper_cases"]
    n = 1 << 16
    for c in range(1, 7):
        k, M = w.paper_case(c, n)
        assert k.dtype == np.uint32 and k.shape == (n,)
        assert int(k.max()) <= M
        assert hex(w.checksum(k)) == gold[str(c)]
    assert w.PAPER_CASE_M == {1: 10**6, 2: 10**6, 3: 10**6, 4: 10**4, 5: 10**8, 6: 10**6}
    k2, _ = w.paper_case(2, n)
    assert np.all(np.diff(k2.astype(np.int64)) >= 0)
    k3, _ = w.paper_case(3, n)
    # at least 90% of adjacent pairs stay in order (n/20 replaced positions)
    assert (np.diff(k3.astype(np.int64)) >= 0).mean() > 0.9
    k6, M = w.paper_case(6, n)
    assert int((k6 == M // 2).sum()) == n // 3
    others = k6[k6 != M // 2]
    assert np.unique(others).size == others.size   # distinct when they fit
    big, _ = w.paper_case(6, 3 * 10**6)            # 2*10^6 others cannot be distinct in [0, 10^6]
    assert int((big == 500_000).sum()) == 10**6


def test_signed_and_ieee_generators():
    """Recorded checksums, value classes and the repeats the tests rely on."""
    gold = json.load(open(os.path.join(HERE, "golden", "input_checksums.json")))["signed_ieee"]
    n = 1 << 16
    assert hex(w.checksum(w.signed_keys(n, 32, seed=1))) == gold["int32"]
    assert hex(w.checksum(w.signed_keys(n, 64, seed=1))) == gold["int64"]
    b = w.signed_keys(n, 32, seed=1, spread_bits=12)
    assert hex(w.checksum(b)) == gold["int32_b12"]
    assert b.dtype == np.int32 and b.min() >= -(1 << 12) and b.max() < (1 << 12) and (b < 0).any()
    for width, name in ((32, "float32"), (64, "float64")):
        f = w.ieee_keys(n, width, seed=1)
        assert hex(w.checksum(f)) == gold[name]
        ut = np.uint32 if width == 32 else np.uint64
        bits = f.view(ut)
        sign = ut(1) << ut(width - 1)
        # every special class occurs: +-0, +-inf, NaNs of both signs, subnormals
        assert (bits == 0).any() and (bits == sign).any()
        assert np.isposinf(f).any() and np.isneginf(f).any()
        nan = np.isnan(f)
        assert (nan & ((bits & sign) != 0)).any() and (nan & ((bits & sign) == 0)).any()
        tiny = np.finfo(f.dtype).tiny
        assert ((np.abs(f) < tiny) & (f != 0)).any()
        # every ninth key repeats the key four places earlier
        np.testing.assert_array_equal(bits[9::9], bits[5:-4:9][: bits[9::9].size])
