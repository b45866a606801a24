"""Seeded synthetic inputs shaped like the paper's test cases (section 3.1).

This module only makes inputs.  It holds none of the sorting arithmetic, and it
is the one module that both the GPU library's tests/benchmark and the CPU
oracle's callers share.

Random numbers come from SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), used as a
counter-based generator:

    mix64(z)  = the SplitMix64 output function (two xor-shift-multiply rounds
                and a final xor-shift, constants from the publication)
    base(seed, stream) = mix64(seed * GAMMA + stream)          (mod 2^64)
    value(seed, stream, i) = mix64(base + (i + 1) * GAMMA)     (mod 2^64)

so element i of any stream can be produced independently (and in any order).

Distributions (``DISTRIBUTIONS``), each drawn for n keys from one seed:
    0 uniform   : r >> 32                       uniform on [0, 2^32)
    1 small     : r >> 54                       uniform on [0, 1024)
    2 mid       : r >> 48                       uniform on [0, 2^16)
    3 sorted    : distribution 0, sorted ascending
    4 reverse   : distribution 0, sorted descending
    5 swaps     : distribution 3, then floor(n/100) sequential swaps of
                  positions i, j = ((r >> 32) * n) >> 32 from stream 1
    6 gaussian  : 16 cluster means mu_c = r >> 32 (stream 2); key i picks
                  c = r_i >> 60 (stream 0) and z by Box-Muller from
                  u1 = ((r >> 11) + 1) / 2^53 (stream 3), u2 = (r >> 11) / 2^53
                  (stream 4); k = clamp(round(mu_c + 2^20 z), 0, 2^32 - 1),
                  rounding half away from zero.
The paper's cases map onto these: case 1 (uniform) -> 0/2, case 2 (sorted)
-> 3, case 3 (mostly sorted) -> 5, case 4 (small range) -> 1, case 5 (large
range) -> 0.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22

DISTRIBUTIONS = ("uniform", "small", "mid", "sorted", "reverse", "swaps", "gaussian")


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def mix64_int(z: int) -> int:
    """Scalar form of ``mix64`` on Python ints (used for stream bases)."""
    m = (1 << 64) - 1
    z &= m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def stream_base(seed: int, stream: int) -> int:
    return mix64_int((seed * int(GAMMA) + stream) & ((1 << 64) - 1))


def u64_stream(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Elements start .. start+n-1 of the counter-based stream (seed, stream)."""
    base = np.uint64(stream_base(seed, stream))
    out = np.empty(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        for lo in range(0, n, _CHUNK):
            hi = min(n, lo + _CHUNK)
            ctr = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            out[lo:hi] = mix64(base + ctr * GAMMA)
    return out


def _shifted(seed: int, stream: int, n: int, shift: int, dtype) -> np.ndarray:
    out = np.empty(n, dtype=dtype)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        out[lo:hi] = (u64_stream(seed, stream, hi - lo, lo) >> np.uint64(shift)).astype(dtype)
    return out


def uniform_u32(n: int, seed: int) -> np.ndarray:
    return _shifted(seed, 0, n, 32, np.uint32)


def _swaps(a: np.ndarray, seed: int) -> None:
    n = a.shape[0]
    m = n // 100
    if m == 0:
        return
    r = u64_stream(seed, 1, 2 * m) >> np.uint64(32)
    idx = ((r * np.uint64(n)) >> np.uint64(32)).astype(np.int64)
    # the swaps are sequential by definition; a Python loop keeps that exact
    for t in range(m):
        i = idx[2 * t]
        j = idx[2 * t + 1]
        a[i], a[j] = a[j], a[i]


def _gaussian(n: int, seed: int) -> np.ndarray:
    mu = (u64_stream(seed, 2, 16) >> np.uint64(32)).astype(np.float64)
    out = np.empty(n, dtype=np.uint32)
    two53 = float(1 << 53)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        c = (u64_stream(seed, 0, hi - lo, lo) >> np.uint64(60)).astype(np.int64)
        u1 = ((u64_stream(seed, 3, hi - lo, lo) >> np.uint64(11)).astype(np.float64) + 1.0) / two53
        u2 = (u64_stream(seed, 4, hi - lo, lo) >> np.uint64(11)).astype(np.float64) / two53
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
        x = mu[c] + float(1 << 20) * z
        x = np.where(x >= 0, np.floor(x + 0.5), np.ceil(x - 0.5))
        out[lo:hi] = np.clip(x, 0.0, float((1 << 32) - 1)).astype(np.uint32)
    return out


def config2_keys(dist: int | str, n: int, seed: int | None = None) -> np.ndarray:
    """n uint32 keys of one of the seven distributions (seed defaults to the
    distribution index)."""
    if isinstance(dist, str):
        dist = DISTRIBUTIONS.index(dist)
    if seed is None:
        seed = dist
    if dist == 0:
        return uniform_u32(n, seed)
    if dist == 1:
        return _shifted(seed, 0, n, 54, np.uint32)
    if dist == 2:
        return _shifted(seed, 0, n, 48, np.uint32)
    if dist in (3, 4, 5):
        a = np.sort(uniform_u32(n, seed), kind="stable")
        if dist == 4:
            a = np.ascontiguousarray(a[::-1])
        elif dist == 5:
            _swaps(a, seed)
        return a
    if dist == 6:
        return _gaussian(n, seed)
    raise ValueError(f"unknown distribution {dist}")


# ---- the paper's six input cases (section 3.1): n keys in [0, M]

PAPER_CASE_M = {1: 10**6, 2: 10**6, 3: 10**6, 4: 10**4, 5: 10**8, 6: 10**6}


def _uniform_upto(seed: int, stream: int, n: int, M: int) -> np.ndarray:
    """n keys uniform in [0, M]: floor(u * (M + 1)) for a 32-bit u, exact."""
    out = np.empty(n, dtype=np.uint32)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        u = u64_stream(seed, stream, hi - lo, lo) >> np.uint64(32)
        out[lo:hi] = ((u * np.uint64(M + 1)) >> np.uint64(32)).astype(np.uint32)
    return out


def _distinct_below(seed: int, count: int, U: int) -> np.ndarray:
    """count distinct values in [0, U) (count <= U): the first count values of
    x -> (a*x + c) mod 2^b restricted to [0, U) by cycle walking, a odd."""
    b = max(1, (U - 1).bit_length())
    mask = np.uint64((1 << b) - 1)
    a = np.uint64((stream_base(seed, 7) | 1) & int(mask))
    c = np.uint64(stream_base(seed, 8) & int(mask))
    x = np.arange(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        y = (x * a + c) & mask
        bad = y >= np.uint64(U)
        while bad.any():
            y[bad] = (y[bad] * a + c) & mask
            bad = y >= np.uint64(U)
    return y


def paper_case(case: int, n: int, seed: int | None = None):
    """(keys, M) for input case 1..6 of section 3.1 at size n, uint32 keys:
      1  uniform in [0, M], M = 10^6
      2  case 1 sorted
      3  case 1 sorted, then n/20 positions (stream 1) take new uniform values
         (stream 2): 95% of the keys stay in sorted order
      4  uniform, M = 10^4
      5  uniform, M = 10^8
      6  n/3 keys equal to k = M/2, the rest distinct values in [0, M] other
         than k when they fit (n - n/3 <= M), else uniform in [0, M] without
         k; positions shuffled (stream 3), M = 10^6
    seed defaults to 10 + case."""
    if seed is None:
        seed = 10 + case
    M = PAPER_CASE_M[case]
    if case in (1, 4, 5):
        return _uniform_upto(seed, 0, n, M), M
    if case in (2, 3):
        a = np.sort(_uniform_upto(seed, 0, n, M), kind="stable")
        if case == 3 and n >= 20:
            m = n // 20
            r = u64_stream(seed, 1, m) >> np.uint64(32)
            pos = ((r * np.uint64(n)) >> np.uint64(32)).astype(np.int64)
            a[pos] = _uniform_upto(seed, 2, m, M)
        return a, M
    if case == 6:
        k = M // 2
        same = n // 3
        rest = n - same
        if rest <= M:
            v = _distinct_below(seed, rest, M)             # [0, M)
        else:
            v = _uniform_upto(seed, 4, rest, M - 1).astype(np.uint64)
        v = v + (v >= np.uint64(k))                        # skip k: [0, M] without k
        keys = np.concatenate([np.full(same, k, dtype=np.uint64), v]).astype(np.uint32)
        order = np.argsort(u64_stream(seed, 3, n), kind="stable")
        return np.ascontiguousarray(keys[order]), M
    raise ValueError(f"unknown case {case}")


def config3_pairs(variant: str, n: int):
    """uint64 keys (variant 'full': uniform [0, 2^64), seed 0; 'b40': uniform
    [0, 2^40), seed 1) with the uint32 payload 0..n-1."""
    if variant == "full":
        keys = np.empty(n, dtype=np.uint64)
        for lo in range(0, n, _CHUNK):
            hi = min(n, lo + _CHUNK)
            keys[lo:hi] = u64_stream(0, 0, hi - lo, lo)
    elif variant == "b40":
        keys = _shifted(1, 0, n, 24, np.uint64)
    else:
        raise ValueError(variant)
    return keys, np.arange(n, dtype=np.uint32)


def signed_keys(n: int, width: int, seed: int, spread_bits: int | None = None) -> np.ndarray:
    """Two's-complement keys (int32 or int64) from stream 5 of ``seed``: the
    full range, or uniform on [-2^b, 2^b) for ``spread_bits`` = b < width."""
    r = u64_stream(seed, 5, n)
    if spread_bits is None:
        u = r if width == 64 else (r >> np.uint64(32)).astype(np.uint32)
        return u.view(np.int64 if width == 64 else np.int32)
    v = (r >> np.uint64(63 - spread_bits)).astype(np.int64) - (1 << spread_bits)
    return v.astype(np.int64 if width == 64 else np.int32)


def ieee_keys(n: int, width: int, seed: int, special_share: int = 16) -> np.ndarray:
    """IEEE 754 keys (float32 or float64).  For key i, stream 6 gives r and
    stream 7 gives q.  One key in ``special_share`` (r >> 60 == 0 when the
    share is 16) is a special value chosen by q >> 61: +-0, +-inf, a NaN of
    either sign with payload q (nonzero), a subnormal of either sign; the
    rest are (-1)^s 2^e (1 + f) with s = bit 0 of r, e uniform on
    [-E, E] (E = 60 for float32, 500 for float64) and f from q.  Every ninth
    key repeats the key four places earlier, so equal keys occur."""
    ut, ft = (np.uint32, np.float32) if width == 32 else (np.uint64, np.float64)
    mant = 23 if width == 32 else 52
    expo = 0x7F800000 if width == 32 else 0x7FF0000000000000
    sign = np.uint64(1) << np.uint64(width - 1)
    E = 60 if width == 32 else 500
    r = u64_stream(seed, 6, n)
    q = u64_stream(seed, 7, n)
    s = (r & np.uint64(1)).astype(np.float64)
    e = ((r >> np.uint64(1)) % np.uint64(2 * E + 1)).astype(np.int64) - E
    f = (q >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    out = (np.where(s == 1, -1.0, 1.0) * np.ldexp(1.0 + f, e)).astype(ft).view(ut).astype(np.uint64)
    special = ((r >> np.uint64(32)) % np.uint64(special_share)) == 0
    kind = q >> np.uint64(61)
    payload = (q & np.uint64((1 << mant) - 1)) | np.uint64(1)
    neg = np.where((q >> np.uint64(60)) & np.uint64(1) == 1, sign, np.uint64(0))
    spec = np.select([kind == 0, kind == 1, kind == 2, kind == 3, kind < 6],
                     [np.uint64(0), sign, np.uint64(expo), np.uint64(expo) | sign,
                      np.uint64(expo) | payload | neg],
                     default=payload | neg)
    out = np.where(special, spec, out).astype(ut)
    rep = np.arange(9, n, 9)
    out[rep] = out[rep - 4]
    return out.view(ft)


def log_uniform_sizes(count: int, seed: int, lo: int, hi_exp_base: int) -> np.ndarray:
    """floor(lo * base^u) with u = (r >> 11) / 2^53 from stream 0 of seed."""
    u = (u64_stream(seed, 0, count) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    return np.floor(lo * np.power(float(hi_exp_base), u)).astype(np.int64)


def segment_plan(num_segments: int = 10000, seed: int = 4, lo: int = 16, base: int = 65536):
    """Sizes (log-uniform in [lo, lo*base)) and distribution index of every
    segment of the batched workload."""
    sizes = log_uniform_sizes(num_segments, seed, lo, base)
    r = u64_stream(seed, 1, num_segments) >> np.uint64(32)
    dists = ((r * np.uint64(7)) >> np.uint64(32)).astype(np.int64)
    return sizes, dists


def segmented_keys(num_segments: int = 10000, seed: int = 4, lo: int = 16,
                   base: int = 65536, first_array_seed: int = 1000):
    """Packed uint32 keys of all segments and the uint64 offsets [S+1]."""
    sizes, dists = segment_plan(num_segments, seed, lo, base)
    offsets = np.zeros(num_segments + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes, dtype=np.uint64)
    keys = np.empty(int(offsets[-1]), dtype=np.uint32)
    for j in range(num_segments):
        a, b = int(offsets[j]), int(offsets[j + 1])
        keys[a:b] = config2_keys(int(dists[j]), b - a, first_array_seed + j)
    return keys, offsets


def checksum(a: np.ndarray) -> int:
    """Order-dependent 64-bit checksum of an array's bytes, for recording
    which exact input a run used."""
    v = np.frombuffer(np.ascontiguousarray(a).tobytes(), dtype=np.uint8)
    h = 0xCBF29CE484222325
    # FNV-1a over 8-byte words of the buffer (zero padded), folded with mix64
    pad = (-v.shape[0]) % 8
    words = np.frombuffer(np.concatenate([v, np.zeros(pad, np.uint8)]).tobytes(), dtype=np.uint64)
    idx = np.arange(1, words.shape[0] + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        folded = mix64(words ^ (idx * GAMMA))
    return mix64_int(h ^ int(np.bitwise_xor.reduce(folded)) if folded.size else h)


# ----------------------------------------------------------------------------
# Device-side generation (torch), for workloads too large to feed over PCIe.
# The same counter-based SplitMix64 on int64 tensors: products wrap modulo
# 2^64 and right shifts are made logical with a mask.  Outputs are int64
# tensors holding the 64-bit patterns.

def _lsr(x, s: int):
    import torch
    return (x >> s) & ((1 << (64 - s)) - 1)


def _to_i64(u: int) -> int:
    return u - (1 << 64) if u >= (1 << 63) else u


def device_u64_stream(seed: int, stream: int, n: int, device, start: int = 0):
    """Elements start .. start+n-1 of stream (seed, stream), as int64 bit
    patterns on `device` (equal to u64_stream's values)."""
    import torch
    base = torch.tensor(_to_i64(stream_base(seed, stream)), dtype=torch.int64, device=device)
    g = torch.tensor(_to_i64(int(GAMMA)), dtype=torch.int64, device=device)
    m1 = torch.tensor(_to_i64(int(_M1)), dtype=torch.int64, device=device)
    m2 = torch.tensor(_to_i64(int(_M2)), dtype=torch.int64, device=device)
    z = base + torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device) * g
    z = (z ^ _lsr(z, 30)) * m1
    z = (z ^ _lsr(z, 27)) * m2
    return z ^ _lsr(z, 31)


def device_keys(dist: int, n: int, seed: int, width: int, device):
    """n keys of one of the seven distributions made on the device, as a
    torch uint32 (width 4) or uint64 (width 8) tensor.  For 64-bit keys the
    fields are taken from the top of the 64-bit random value: uniform r,
    small r >> 54, mid r >> 48; sorted/reverse sort the uniform keys as
    unsigned; 'swaps' exchanges floor(n/100) disjoint position pairs (drawn
    from stream 1) of the sorted keys; 'gaussian' puts 16 clusters of width
    2^20 (32-bit) or 2^52 (64-bit) at uniform means."""
    import math
    import torch
    r = device_u64_stream(seed, 0, n, device)
    if width == 4:
        top = _lsr(r, 32)
        keys = {0: top, 1: _lsr(r, 54), 2: _lsr(r, 48)}.get(dist)
        full_bits = 32
    else:
        keys = {0: r, 1: _lsr(r, 54), 2: _lsr(r, 48)}.get(dist)
        full_bits = 64
    if dist in (3, 4, 5):
        u = r if width == 8 else _lsr(r, 32)
        flip = (-(1 << 63)) if width == 8 else 0
        keys = torch.sort(u ^ flip).values ^ flip
        if dist == 4:
            keys = keys.flip(0)
        elif dist == 5 and n >= 2:
            m = n // 100
            if m:
                pos = torch.argsort(_lsr(device_u64_stream(seed, 1, n, device), 1))[: 2 * m]
                i, j = pos[0::2], pos[1::2]
                ki, kj = keys[i].clone(), keys[j].clone()
                keys[i], keys[j] = kj, ki
    if dist == 6:
        mu = _lsr(device_u64_stream(seed, 2, 16, device), 64 - full_bits).to(torch.float64)
        if width == 8:
            mu = torch.where(mu < 0, mu + 2.0 ** 64, mu)
        c = _lsr(r, 60)
        u1 = (_lsr(device_u64_stream(seed, 3, n, device), 11).to(torch.float64) + 1.0) / float(1 << 53)
        u2 = _lsr(device_u64_stream(seed, 4, n, device), 11).to(torch.float64) / float(1 << 53)
        z = torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)
        x = mu[c] + float(1 << (20 if width == 4 else 52)) * z
        x = torch.where(x >= 0, torch.floor(x + 0.5), torch.ceil(x - 0.5))
        hi = float((1 << 32) - 1) if width == 4 else float(2 ** 64 - 2048)
        x = torch.clamp(x, 0.0, hi)
        if width == 4:
            keys = x.to(torch.int64)
        else:
            big = x >= 2.0 ** 63
            keys = torch.where(big, (x - 2.0 ** 63).to(torch.int64) ^ (-(1 << 63)), x.to(torch.int64))
    if width == 4:
        return keys.to(torch.int32).view(torch.uint32) if keys.dtype == torch.int64 else keys
    return keys.view(torch.uint64)


def serving_trace(rate: float = 2000.0, seconds: float = 60.0, seed: int = 5, lo: int = 1024,
                  base: int = 65536):
    """Poisson arrivals (exponential gaps) over `seconds`, each request
    (arrival time, key width 4 or 8 by coin flip, n = floor(lo * base^u),
    distribution index)."""
    count = int(rate * seconds * 1.5) + 16
    g = (u64_stream(seed, 0, count) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    gaps = -np.log1p(-g) / rate
    t = np.cumsum(gaps)
    keep = t < seconds
    t = t[keep]
    k = t.size
    w = np.where((u64_stream(seed, 1, k) >> np.uint64(63)) == 1, 8, 4)
    u = (u64_stream(seed, 2, k) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    n = np.floor(lo * np.power(float(base), u)).astype(np.int64)
    d = ((u64_stream(seed, 3, k) >> np.uint64(32)) * np.uint64(7) >> np.uint64(32)).astype(np.int64)
    return t, w, n, d
