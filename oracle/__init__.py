"""CPU oracle for the integer sorts of "Comparison of Bucket Sort and RADIX Sort".

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The library under
``paper_1206_3511_amd/`` never imports it, and it imports nothing from there.

The arithmetic lives in ``oracle.c`` (plain single-threaded C, built into
``liboracle.so`` by ``oracle/build.py``); this module only marshals numpy
arrays.  Every function follows a passage of the paper:

* ``radix_lsd``  -- RADIX-SORT (Algorithm 4) over COUNTING-SORT (Algorithm 3).
* ``bucket``     -- BUCKET-SORT (Algorithm 2) with INSERTION-SORT (Algorithm 1)
                    for small buckets and a stable merge sort for large ones.
* ``segmented``  -- either sort applied to every segment of a packed array.
* ``bucket_index`` -- the exact bucket map floor((k-min)*B/(max-min+1)).
* ``sort_ordered`` -- the definition of sorting (section 2) for signed and
                    IEEE 754 keys: a stable merge sort under signed order or
                    IEEE 754-2019 totalOrder.

All results are pinned by ``tests/test_oracle_pins.py`` against library sorts,
brute force and the invariants the paper states (sortedness, permutation,
stability).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p


def _load(path: str | None = None):
    """Load liboracle.so (building it first if needed).  ``path`` loads
    another build of oracle.c instead; the mutation test uses it to run the
    pins against deliberately broken copies."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None:
        path = _LIB_PATH
        if not os.path.exists(path):
            from . import build as _build

            _build.build()
    lib = ctypes.CDLL(path)
    lib.oracle_radix_lsd.argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_uint64,
                                     ctypes.c_int, ctypes.c_int, _vp, _vp,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.oracle_radix_lsd.restype = ctypes.c_int
    lib.oracle_bucket.argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _vp, _vp, _vp, _vp, _vp]
    lib.oracle_bucket.restype = ctypes.c_int
    lib.oracle_bucket_index.argtypes = [ctypes.c_uint64] * 4
    lib.oracle_bucket_index.restype = ctypes.c_uint64
    lib.oracle_segmented.argtypes = [_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_uint64, _vp,
                                     ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_segmented.restype = ctypes.c_int
    lib.oracle_sort_ordered.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_uint64]
    lib.oracle_sort_ordered.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_vp)


def _keys(keys) -> np.ndarray:
    keys = np.ascontiguousarray(keys)
    if keys.dtype not in (np.uint32, np.uint64):
        raise TypeError(f"keys must be uint32 or uint64, got {keys.dtype}")
    return keys


def _vals(vals, n):
    if vals is None:
        return None
    vals = np.ascontiguousarray(vals, dtype=np.uint32)
    if vals.shape != (n,):
        raise ValueError("payload must have one uint32 per key")
    return vals


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")


@dataclass
class RadixResult:
    keys: np.ndarray
    vals: np.ndarray | None
    passes: int
    pass_counts: np.ndarray | None = None   # [passes, 2^r] digit counts
    pass_keys: np.ndarray | None = None     # [passes, n] array after each pass


def radix_lsd(keys, vals=None, r: int = 8, d_from_max: bool = False,
              want_counts: bool = False, want_passes: bool = False) -> RadixResult:
    """RADIX-SORT (Algorithm 4): d passes of COUNTING-SORT (Algorithm 3) on
    r-bit digits, least significant first.  d = ceil(key_bits/r), or the
    number of r-bit digits of the largest key when ``d_from_max``."""
    lib = _load()
    keys = _keys(keys)
    n = keys.shape[0]
    w = keys.dtype.itemsize
    vals = _vals(vals, n)
    out = np.empty_like(keys)
    vout = None if vals is None else np.empty_like(vals)
    max_passes = -(-8 * w // r)
    counts = np.zeros((max_passes, 1 << r), dtype=np.uint64) if want_counts else None
    passes = np.zeros((max_passes, n), dtype=np.uint64) if want_passes else None
    d = ctypes.c_int(0)
    _check(lib.oracle_radix_lsd(_ptr(keys), _ptr(out), w, _ptr(vals), _ptr(vout), n, r,
                                int(d_from_max), _ptr(counts), _ptr(passes), ctypes.byref(d)))
    d = d.value
    return RadixResult(out, vout, d,
                       None if counts is None else counts[:d],
                       None if passes is None else passes[:d].astype(keys.dtype))


@dataclass
class BucketResult:
    keys: np.ndarray
    vals: np.ndarray | None
    kmin: int = 0
    kmax: int = 0
    counts: np.ndarray | None = None      # [B] bucket sizes
    offsets: np.ndarray | None = None     # [B+1] exclusive prefix, offsets[B] = n
    scat_keys: np.ndarray | None = None   # keys after the scatter, before bucket sorts
    scat_vals: np.ndarray | None = None


def bucket(keys, vals=None, num_buckets: int = 1024, cutoff: int = 32,
           want_intermediates: bool = False, key_bound: int = 0) -> BucketResult:
    """BUCKET-SORT (Algorithm 2) with the exact bucket map of ``bucket_index``,
    buckets filled in input order and sorted by INSERTION-SORT (Algorithm 1)
    when they hold at most ``cutoff`` keys, else by a stable merge sort.
    ``key_bound`` = M > 0 declares the range [0, M] (section 2.3) instead of
    the keys' own [min, max]; keys above M join the last bucket."""
    lib = _load()
    keys = _keys(keys)
    n = keys.shape[0]
    w = keys.dtype.itemsize
    vals = _vals(vals, n)
    out = np.empty_like(keys)
    vout = None if vals is None else np.empty_like(vals)
    mm = np.zeros(2, dtype=np.uint64)
    cnt = off = sk = sv = None
    if want_intermediates:
        cnt = np.zeros(num_buckets, dtype=np.uint64)
        off = np.zeros(num_buckets + 1, dtype=np.uint64)
        sk = np.zeros(n, dtype=np.uint64)
        sv = None if vals is None else np.zeros(n, dtype=np.uint32)
    _check(lib.oracle_bucket(_ptr(keys), _ptr(out), w, _ptr(vals), _ptr(vout), n,
                             num_buckets, cutoff, key_bound, _ptr(mm), _ptr(cnt), _ptr(off), _ptr(sk),
                             _ptr(sv)))
    return BucketResult(out, vout, int(mm[0]), int(mm[1]), cnt, off,
                        None if sk is None else sk.astype(keys.dtype), sv)


def bucket_index(k: int, kmin: int, kmax: int, num_buckets: int) -> int:
    """floor((k - kmin) * B / (kmax - kmin + 1)) in exact 128-bit arithmetic."""
    return int(_load().oracle_bucket_index(k, kmin, kmax, num_buckets))


def segmented(keys, offsets, vals=None, algo: str = "radix", r: int = 8,
              num_buckets: int = 1024, cutoff: int = 32):
    """Sort every segment [offsets[s], offsets[s+1]) on its own."""
    lib = _load()
    keys = _keys(keys)
    n = keys.shape[0]
    w = keys.dtype.itemsize
    vals = _vals(vals, n)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    s = offsets.shape[0] - 1
    out = np.empty_like(keys)
    vout = None if vals is None else np.empty_like(vals)
    _check(lib.oracle_segmented(_ptr(keys), _ptr(out), w, _ptr(vals), _ptr(vout), n,
                                _ptr(offsets), s, 0 if algo == "radix" else 1, r,
                                num_buckets, cutoff))
    return out, vout


# numpy dtype -> key order understood by oracle_sort_ordered
_ORDERS = {np.dtype(np.uint32): 0, np.dtype(np.uint64): 0, np.dtype(np.int32): 1, np.dtype(np.int64): 1,
           np.dtype(np.float32): 2, np.dtype(np.float64): 2}


def sort_ordered(keys, vals=None):
    """Stable nondecreasing sort of unsigned, signed (by value) or IEEE 754
    keys (totalOrder: -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN, NaNs
    by payload).  Returns (keys, vals) with the input's bit patterns."""
    lib = _load()
    keys = np.ascontiguousarray(keys)
    if keys.dtype not in _ORDERS:
        raise TypeError(f"unsupported key dtype {keys.dtype}")
    n = keys.shape[0]
    vals = _vals(vals, n)
    out = np.empty_like(keys)
    vout = None if vals is None else np.empty_like(vals)
    _check(lib.oracle_sort_ordered(_ptr(keys), _ptr(out), keys.dtype.itemsize, _ORDERS[keys.dtype],
                                   _ptr(vals), _ptr(vout), n))
    return out, vout
