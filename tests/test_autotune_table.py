"""The autotuner's table logic (no GPU): keys, size classes, save/load."""
import importlib

import pytest


def test_table_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("INTSORT_TUNE_FILE", str(tmp_path / "t.json"))
    at = importlib.import_module("paper_1206_3511_amd.autotune")
    assert at.load() == {}
    assert at.size_class(1) == 0 and at.size_class(1024) == 10 and at.size_class(1025) == 10
    monkeypatch.setattr(at, "_device_key", lambda device=0: "dev|hip x")
    at._record("radix", 4, 100_000_000, {"digit_bits": 8}, {"8": 1.3}, 0)
    assert at.tuned_options("radix", 4, 120_000_000) == {"digit_bits": 8}   # same size class
    assert at.tuned_options("radix", 4, 1000) == {}
    assert at.tuned_options("bucket", 4, 100_000_000) == {}
    assert at.load()["dev|hip x"]["radix|w4|c26"]["n"] == 100_000_000


def test_candidates_are_supported_options():
    at = importlib.import_module("paper_1206_3511_amd.autotune")
    assert set(at.RADIX_BITS) <= {4, 8, 11}
    assert max(at.BUCKETS) <= 65536
    assert max(at.CUTOFFS) <= 16384
