"""The tuning table (no GPU): the autotuner's file format, and zero option
fields of the C library taking its choices (a planning context, whose device
key is empty, takes the entries for every device, '*')."""
import ctypes
import importlib

import pytest

from paper_1206_3511_amd import intsort as I


def test_table_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("INTSORT_TUNE_FILE", str(tmp_path / "t.tsv"))
    at = importlib.import_module("paper_1206_3511_amd.autotune")
    assert at.load() == []
    assert at.size_class(1) == 0 and at.size_class(1024) == 10 and at.size_class(1025) == 10
    monkeypatch.setattr(at, "_device_key", lambda device=0: "dev|gfx|hip 1")
    assert at._record("radix", 4, 100_000_000, 11, 0, reload=False) == {"digit_bits": 11}
    assert at.tuned_options("radix", 4, 120_000_000) == {"digit_bits": 11}   # same size class
    assert at.tuned_options("radix", 4, 1000) == {}
    assert at.tuned_options("bucket", 4, 100_000_000) == {}
    at._record("radix", 4, 100_000_000, 8, 0, reload=False)                   # replaces the entry
    assert at.load() == [("dev|gfx|hip 1", "radix", 4, 26, 8)]
    assert at._record("segmented_bits", 4, 1 << 30, 4, 0, reload=False) == {"digit_bits": 4}
    assert at.tuned_options("segmented_bits", 4, (1 << 30) + 5) == {"digit_bits": 4}
    assert at.tuned_options("segmented", 4, 1 << 30) == {}


def test_candidates_are_supported_options():
    at = importlib.import_module("paper_1206_3511_amd.autotune")
    assert set(at.RADIX_BITS) <= {4, 8, 11}
    assert set(at.SEG_BITS) <= {4, 8}          # what segmented and batched calls take
    assert max(at.BUCKETS) <= 65536
    assert max(at.CUTOFFS) <= 16384


def _ws(ctx, kt, pairs, n, segs=0, **opt):
    b = ctypes.c_size_t(0)
    o = I.make_options(**opt)
    assert I.lib().intsort_workspace_size(ctx.handle, kt, int(pairs), n, segs, ctypes.byref(o),
                                          ctypes.byref(b)) == I.OK
    return b.value


def test_zero_fields_take_the_tuned_values(tmp_path):
    ctx = I.Context(-1)
    assert ctx.device_key() == ""
    n = 3_000_000                       # size class 21
    path = tmp_path / "tune.tsv"
    path.write_text("# a comment line\n"
                    "*\tradix\t4\t21\t11\n"
                    "*\tbucket\t4\t21\t65536\n"
                    "*\tsegmented\t4\t21\t2048\n"
                    "some other device|gfx1|hip 9\tradix\t8\t21\t4\n"
                    "*\tradix\t8\t21\t5\n"          # not a digit width: ignored
                    "bad line without tabs\n")
    before = (_ws(ctx, I.U32, False, n), _ws(ctx, I.U32, False, n, algo="bucket"),
              _ws(ctx, I.U32, False, n, segs=20000))
    ctx.load_tuning(str(path))
    assert _ws(ctx, I.U32, False, n) == _ws(ctx, I.U32, False, n, digit_bits=11) != before[0]
    assert _ws(ctx, I.U32, False, n, algo="bucket") == _ws(ctx, I.U32, False, n, algo="bucket",
                                                            num_buckets=65536) != before[1]
    assert _ws(ctx, I.U32, False, n, segs=20000) == _ws(ctx, I.U32, False, n, segs=20000, lds_cutoff=2048) != before[2]
    # an explicit field wins; other widths and size classes keep the defaults
    assert _ws(ctx, I.U32, False, n, digit_bits=8) == before[0]
    assert _ws(ctx, I.U64, False, n) == _ws(ctx, I.U64, False, n, digit_bits=8)
    assert _ws(ctx, I.U32, False, 1 << 23) == _ws(ctx, I.U32, False, 1 << 23, digit_bits=8)
    # segmented calls never take a tuned digit width (they use 8-bit digits)
    assert _ws(ctx, I.U32, False, n, segs=20000) == _ws(ctx, I.U32, False, n, segs=20000, lds_cutoff=2048,
                                                      digit_bits=8)
    # signed keys take radix sort with 8-bit digits whatever the table says
    assert _ws(ctx, I.I32, False, n) == _ws(ctx, I.I32, False, n, digit_bits=8)
    ctx.load_tuning(None)
    assert _ws(ctx, I.U32, False, n) == before[0]
    with pytest.raises(I.IntsortError):
        ctx.load_tuning(str(tmp_path / "missing.tsv"))
