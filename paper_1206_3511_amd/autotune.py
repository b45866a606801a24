"""Autotuner for the sort library's run-time choices.

It times candidate settings on the device, on synthetic keys of the shape
asked for, and keeps the fastest in the library's tuning table: a text file,
one tab-separated line per entry (device key, kind, key bytes, size class
floor(log2 n), value), which the C library reads at intsort_create and
whenever intsort_load_tuning is called.  Zero option fields then take the
choice:

  radix      digit width r in {4, 8, 11}      (digit_bits)
  bucket     number of buckets B               (num_buckets)
  segmented  LDS cutoff: segments up to it are sorted by one workgroup in
             LDS, longer ones by all workgroups (lds_cutoff)
  segmented_bits  digit width r in {4, 8} of those longer segments' passes
             (digit_bits of segmented and batched calls)

The table lives in $INTSORT_TUNE_FILE, else ~/.cache/intsort/tune.tsv.  The
device key comes from the library (intsort_device_key), so both sides agree
on it.  Every candidate produces the same bytes (the sorts are exact), so a
choice only changes speed; ``tuned_options`` returns {} where nothing was
tuned.
"""
from __future__ import annotations

import math
import os

import torch

from . import intsort as I

RADIX_BITS = (4, 8, 11)
SEG_BITS = (4, 8)
BUCKETS = (256, 1024, 4096, 16384, 65536)
CUTOFFS = (256, 2048, 8192, 16384)
FIELDS = {"radix": "digit_bits", "bucket": "num_buckets", "segmented": "lds_cutoff",
          "segmented_bits": "digit_bits"}


def table_path() -> str:
    return os.environ.get("INTSORT_TUNE_FILE", os.path.expanduser("~/.cache/intsort/tune.tsv"))


def _device_key(device: int = 0) -> str:
    return I.context(device).device_key()


def size_class(n: int) -> int:
    return int(math.floor(math.log2(max(1, n))))


def load() -> list:
    """The table's entries: (device key, kind, key bytes, size class, value)."""
    rows = []
    try:
        with open(table_path()) as f:
            for line in f:
                p = line.rstrip("\n").split("\t")
                if len(p) == 5 and not p[0].startswith("#") and p[1] in FIELDS:
                    try:
                        rows.append((p[0], p[1], int(p[2]), int(p[3]), int(p[4])))
                    except ValueError:
                        pass
    except OSError:
        pass
    return rows


def save(rows: list) -> None:
    path = table_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write("# device key\tkind\tkey bytes\tsize class\tvalue  (intsort tuning table)\n")
        for r in sorted(rows):
            f.write("\t".join(str(x) for x in r) + "\n")
    os.replace(tmp, path)


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


def _record(kind: str, width: int, n: int, value: int, device: int, reload: bool = True) -> dict:
    key = _device_key(device)
    cls = size_class(n)
    rows = [r for r in load() if not (r[0] == key and r[1] == kind and r[2] == width and r[3] == cls)]
    rows.append((key, kind, width, cls, int(value)))
    save(rows)
    if reload:
        # the library's context takes the new choice at once
        I.context(device).load_tuning(table_path())
    return {FIELDS[kind]: int(value)}


def tune_radix(width: int, n: int, device: int = 0) -> dict:
    keys = _keys(width, n, device)
    out = torch.empty_like(keys)
    ms = {r: _time(lambda: I.sort(keys, out=out, digit_bits=r)) for r in RADIX_BITS}
    return _record("radix", width, n, min(ms, key=ms.get), device)


def tune_bucket(width: int, n: int, device: int = 0) -> dict:
    keys = _keys(width, n, device)
    out = torch.empty_like(keys)
    ms = {B: _time(lambda: I.sort(keys, out=out, algo="bucket", num_buckets=B)) for B in BUCKETS}
    return _record("bucket", width, n, min(ms, key=ms.get), device)


def tune_segmented(keys: torch.Tensor, offsets: torch.Tensor, device: int = 0) -> dict:
    """Tunes the LDS cutoff, then the digit width of the longer segments'
    passes with that cutoff, on a real batch (keys packed, device offsets)."""
    out = torch.empty_like(keys)
    width = keys.element_size()
    ms = {}
    for c in CUTOFFS:
        if width == 8 and c > 8192:
            continue
        ms[c] = _time(lambda: I.segmented_sort(keys, offsets, out_keys=out, lds_cutoff=c, digit_bits=8), reps=3)
    cut = min(ms, key=ms.get)
    msr = {r: _time(lambda: I.segmented_sort(keys, offsets, out_keys=out, lds_cutoff=cut, digit_bits=r), reps=3)
           for r in SEG_BITS}
    _record("segmented", width, keys.numel(), cut, device, reload=False)
    return {**_record("segmented_bits", width, keys.numel(), min(msr, key=msr.get), device),
            "lds_cutoff": cut}


def tuned_options(kind: str, width: int, n: int, device: int = 0) -> dict:
    """The stored choice for this kind, key width and size class, or {}."""
    key = _device_key(device)
    cls = size_class(n)
    for r in load():
        if r[0] in (key, "*") and r[1] == kind and r[2] == width and r[3] == cls:
            return {FIELDS[kind]: r[4]}
    return {}
