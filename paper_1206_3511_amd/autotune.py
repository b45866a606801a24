"""Autotuner for the sort library's run-time choices.

It times candidate settings on the device, on synthetic keys of the shape
asked for, and keeps the fastest in a JSON table keyed by device name, HIP
version, kind, key width and size class (floor(log2 n)):

  radix      digit width r in {4, 8, 11}
  bucket     number of buckets B
  segmented  LDS cutoff: segments up to it are sorted by one workgroup in
             LDS, longer ones by all workgroups

The table lives in $INTSORT_TUNE_FILE, else ~/.cache/intsort/tune.json.
Every candidate produces the same bytes (the sorts are exact), so a choice
only changes speed; ``tuned_options`` returns {} where nothing was tuned.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import intsort as I

RADIX_BITS = (4, 8, 11)
BUCKETS = (256, 1024, 4096, 16384, 65536)
CUTOFFS = (256, 2048, 8192, 16384)


def table_path() -> str:
    return os.environ.get("INTSORT_TUNE_FILE", os.path.expanduser("~/.cache/intsort/tune.json"))


def _device_key(device: int = 0) -> str:
    return f"{torch.cuda.get_device_name(device)}|hip {torch.version.hip}"


def size_class(n: int) -> int:
    return int(math.floor(math.log2(max(1, n))))


def load() -> dict:
    try:
        with open(table_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save(table: dict) -> None:
    path = table_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _entry_key(kind: str, width: int, n: int) -> str:
    return f"{kind}|w{width}|c{size_class(n)}"


def _time(fn, reps: int = 5) -> float:
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def _keys(width: int, n: int, device: int):
    import workloads
    return workloads.device_keys(0, n, 99, width, f"cuda:{device}")


def _record(kind: str, width: int, n: int, choice: dict, timings: dict, device: int) -> dict:
    table = load()
    dev = table.setdefault(_device_key(device), {})
    dev[_entry_key(kind, width, n)] = {"choice": choice, "ms": timings, "n": n}
    save(table)
    return choice


def tune_radix(width: int, n: int, device: int = 0) -> dict:
    keys = _keys(width, n, device)
    out = torch.empty_like(keys)
    ms = {r: _time(lambda: I.sort(keys, out=out, digit_bits=r)) for r in RADIX_BITS}
    best = min(ms, key=ms.get)
    return _record("radix", width, n, {"digit_bits": best}, {str(k): round(v, 4) for k, v in ms.items()}, device)


def tune_bucket(width: int, n: int, device: int = 0) -> dict:
    keys = _keys(width, n, device)
    out = torch.empty_like(keys)
    ms = {B: _time(lambda: I.sort(keys, out=out, algo="bucket", num_buckets=B)) for B in BUCKETS}
    best = min(ms, key=ms.get)
    return _record("bucket", width, n, {"num_buckets": best}, {str(k): round(v, 4) for k, v in ms.items()},
                   device)


def tune_segmented(keys: torch.Tensor, offsets: torch.Tensor, device: int = 0) -> dict:
    """Tunes the LDS cutoff on a real batch (keys packed, device offsets)."""
    out = torch.empty_like(keys)
    width = keys.element_size()
    ms = {}
    for c in CUTOFFS:
        if width == 8 and c > 8192:
            continue
        ms[c] = _time(lambda: I.segmented_sort(keys, offsets, out_keys=out, lds_cutoff=c), reps=3)
    best = min(ms, key=ms.get)
    return _record("segmented", width, keys.numel(), {"lds_cutoff": best},
                   {str(k): round(v, 4) for k, v in ms.items()}, device)


def tuned_options(kind: str, width: int, n: int, device: int = 0) -> dict:
    """The stored choice for this kind, key width and size class, or {}."""
    dev = load().get(_device_key(device), {})
    e = dev.get(_entry_key(kind, width, n))
    return dict(e["choice"]) if e else {}
