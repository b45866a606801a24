"""Benchmark of the MI355X integer sort.

One step = one complete sort (every kernel of the method) of data already
resident in HBM, out of place from a pristine input.  The default workload is
the headline: 100,000,000 uint32 keys drawn uniformly from [0, 2^32) (seed 0),
LSD radix sort with 8-bit digits (4 passes).  It prints one JSON line with the
throughput (Gkeys/s), the roofline figure of the dominant kernel (the digit
pass), and the single-threaded CPU oracle timed on the same input.

Other workloads (``--workload NAME``, or ``--workload all``; one JSON line
each): the seven 100M-key distributions under radix and bucket sort, 100M
uint64 keys with a uint32 payload (radix with 8- and 11-bit digits, bucket
sort with 65536 buckets), the batched sort of 10,000 arrays against one launch
per array, and the serving trace (Poisson arrivals) through the continuous-
batching server against the plain one-request-per-launch path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Sources the digit-pass kernel is compiled from: the HBM traffic measured with
# hardware counters is reported only while they are unchanged.
PASS_SOURCES = ("paper_1206_3511_amd/csrc/onesweep.hpp", "paper_1206_3511_amd/csrc/radix.hip",
                "paper_1206_3511_amd/csrc/device_common.hpp", "paper_1206_3511_amd/csrc/internal.hpp")
TRAFFIC_FILE = "profiles/onesweep_u32_100M_r8_hbm_traffic.md"
# longest array the segmented sort of 32-bit keys sorts in one workgroup's
# LDS when no cutoff is given
SEG_LDS_MAX_U32 = 16384
DISTS = ("uniform", "small", "mid", "sorted", "reverse", "swaps", "gaussian")


def _workloads():
    w = {"uniform_u32_100M_radix_r8": ("plain", dict(dist=0, n=100_000_000, algo="radix", bits=8, B=0))}
    w["config1_u32_1M_radix_r8"] = ("plain", dict(dist=0, n=1_000_000, algo="radix", bits=8, B=0))
    w["uniform_u32_100M_radix_r11"] = ("plain", dict(dist=0, n=100_000_000, algo="radix", bits=11, B=0))
    w["config1_u32_1M_bucket_B1024"] = ("plain", dict(dist=0, n=1_000_000, algo="bucket", bits=8, B=1024))
    for e, n in ((6, 1_000_000), (7, 10_000_000), (8, 100_000_000)):
        w[f"uniform_u32_1e{e}_msd_r8"] = ("plain", dict(dist=0, n=n, algo="msd", bits=8, B=0))
    w["signed_i32_100M_radix_r8"] = ("plain", dict(dist=0, n=100_000_000, algo="radix", bits=8, B=0, kind="i32"))
    w["ieee_f32_100M_radix_r8"] = ("plain", dict(dist=0, n=100_000_000, algo="radix", bits=8, B=0, kind="f32"))
    for d, name in enumerate(DISTS):
        w[f"config2_{name}_u32_100M_radix_r8"] = ("plain", dict(dist=d, n=100_000_000, algo="radix", bits=8, B=0))
        w[f"config2_{name}_u32_100M_bucket_B1024"] = ("plain", dict(dist=d, n=100_000_000, algo="bucket", bits=8,
                                                                    B=1024))
    for v in ("full", "b40"):
        for algo, bits, B in (("radix", 8, 0), ("radix", 11, 0), ("bucket", 8, 65536)):
            tag = f"radix_r{bits}" if algo == "radix" else f"bucket_B{B}"
            w[f"config3_{v}_u64pairs_100M_{tag}"] = ("pairs", dict(variant=v, n=100_000_000, algo=algo, bits=bits,
                                                                   B=B))
    for c in range(1, 7):
        for e in (6, 7, 8):
            for algo in ("radix", "bucket"):
                w[f"paper_case{c}_n1e{e}_{algo}"] = ("paper", dict(case=c, n=10 ** e, algo=algo))
    w["config4_batched_10k"] = ("batched", {})
    w["config5_serving"] = ("serving", {})
    return w


WORKLOADS = _workloads()
HEADLINE = "uniform_u32_100M_radix_r8"


_STEPS_MS = []   # per-step times of the last _timed call


def _timed(fn, steps, warmup):
    """Mean milliseconds per step over exactly `steps` steps after `warmup`
    untimed ones; an event after every step also gives each step's time."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    _STEPS_MS[:] = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    return ev[0].elapsed_time(ev[steps]) / steps


def _step_stats():
    import statistics
    if not _STEPS_MS:
        return {}
    return {"ms_median": round(statistics.median(_STEPS_MS), 5), "ms_min": round(min(_STEPS_MS), 5)}


def _copy_ceiling(t):
    """Read+write bandwidth of a plain device copy of `t` (torch's copy
    kernel), the practical ceiling of a streaming pass, in GB/s."""
    import torch
    dst = torch.empty_like(t)
    for _ in range(2):
        dst.copy_(t)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    s.record()
    for _ in range(reps):
        dst.copy_(t)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del dst
    return round(2 * t.numel() * t.element_size() / (ms * 1e-3) / 1e9, 1)


def _cold_ms(fn, steps):
    """Per-sort time when a 512 MB write has just evicted the caches (L2 and
    the 256 MB last-level cache) before each sort: median and minimum."""
    import statistics
    import torch
    flush = torch.empty(1 << 27, dtype=torch.int32, device="cuda:0")
    times = []
    for _ in range(steps):
        flush.fill_(1)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e))
    del flush
    return {"ms_cold_median": round(statistics.median(times), 5), "ms_cold_min": round(min(times), 5)}


def _kernel_avgs(ctx, fn, steps):
    """The same steps again with HIP events around every kernel, on the stream
    the kernels run on: average milliseconds per kernel kind."""
    ctx.timing(True)
    ctx.kernel_times()
    for _ in range(steps):
        fn()
    times = ctx.kernel_times()
    ctx.timing(False)
    per = {}
    for kind, idx, t in times:
        per.setdefault(kind, []).append(t)
    return {k: sum(x) / len(x) for k, x in per.items()}


def sources_digest(paths=PASS_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per digit-pass launch from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration), or None when the
    summary is missing or the kernel sources have changed since it was taken."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as f:
            fields = dict(line.strip("- \n").split(": ", 1) for line in f if line.startswith("- ") and ": " in line)
        if fields.get("kernel_sources_sha256") != sources_digest():
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def calibrate_copy():
    """One plain copy of known size for the counter calibration: torch's
    device copy of a 1 GiB buffer, 1 GiB read and 1 GiB written."""
    import torch
    z = torch.zeros(1 << 28, dtype=torch.uint32, device="cuda:0")
    o = torch.empty_like(z)
    for _ in range(2):
        o.copy_(z)
    torch.cuda.synchronize()
    del z, o
    torch.cuda.empty_cache()


def _memory(width, has_values, n, segments=0, **opt):
    """Device bytes one call of the workload holds: its input and output
    buffers and the workspace the library asks for (the analogue of the
    paper's memory table)."""
    from paper_1206_3511_amd import intsort as I
    ctx = I.context(-1)   # planning context: sizes only
    kt = I.U32 if width == 4 else I.U64
    ws = ctx.workspace_size(kt, has_values, n, segments, I.make_options(**opt))
    io = n * (width + (4 if has_values else 0))
    return {"workspace_bytes": int(ws), "input_bytes": int(io), "output_bytes": int(io),
            "peak_device_bytes": int(ws + 2 * io), "workspace_bytes_per_key": round(ws / max(n, 1), 3)}


def _roofline(kernel, bytes_per_launch, avg_ms, extra=None):
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": int(bytes_per_launch),
         "avg_launch_ms": round(avg_ms, 5)}
    if extra:
        r.update(extra)
    return r


def _line(metric, value, unit, ms, steps, warmup, dtype, config, roofline=None, cpu=None, **extra):
    d = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
         "dtype": dtype, "data": "synthetic", "config": config, "roofline": roofline, "cpu_baseline": cpu}
    d.update(_step_stats())
    d.update(extra)
    return d


def _sorted_permutation(keys_h, out_h):
    """The output holds the input's bit patterns and is nondecreasing: unsigned
    keys against numpy's sort; signed keys by value; IEEE keys by their
    totalOrder rank (sign-magnitude bits mapped to a monotone unsigned)."""
    import numpy as np
    ut = np.uint32 if keys_h.dtype.itemsize == 4 else np.uint64
    if keys_h.dtype.kind == "u":
        return bool(np.array_equal(out_h, np.sort(keys_h)))
    same = np.array_equal(np.sort(out_h.view(ut)), np.sort(keys_h.view(ut)))
    if keys_h.dtype.kind == "i":
        return bool(same and np.all(out_h[1:] >= out_h[:-1]))
    b = out_h.view(ut).astype(np.uint64)
    sign = np.uint64(1) << np.uint64(8 * keys_h.dtype.itemsize - 1)
    rank = np.where(b & sign != 0, (sign - np.uint64(1)) - (b & (sign - np.uint64(1))), b | sign)
    return bool(same and np.all(rank[1:] >= rank[:-1]))


def run_plain(name, p, args):
    import numpy as np
    import torch

    import workloads
    from paper_1206_3511_amd import intsort as I

    n, algo, bits, B = p["n"], p["algo"], p["bits"], p["B"]
    kind = p.get("kind", "u32")
    print(f"bench[{name}]: generating {n} keys ({DISTS[p['dist']] if kind == 'u32' else kind})",
          file=sys.stderr, flush=True)
    if kind == "i32":
        keys_h = workloads.signed_keys(n, 32, seed=0)
    elif kind == "f32":
        keys_h = workloads.ieee_keys(n, 32, seed=0)
    else:
        keys_h = workloads.config2_keys(p["dist"], n, seed=0 if p["dist"] == 0 else None)
    keys = torch.from_numpy(keys_h).to("cuda:0")
    out = torch.empty_like(keys)
    ctx = I.context(0)
    opts = dict(algo=algo, digit_bits=bits, num_buckets=B)
    fn = lambda: I.sort(keys, out=out, **opts)  # noqa: E731
    ms = _timed(fn, args.steps, args.warmup)
    steps_ms = list(_STEPS_MS)
    value = n / (ms * 1e-3) / 1e9
    print(f"bench[{name}]: {ms:.4f} ms/sort, {value:.2f} Gkeys/s", file=sys.stderr, flush=True)
    avg = _kernel_avgs(ctx, fn, args.steps)
    # a 4 MB input stays in the 256 MB last-level cache between sorts, so
    # small sorts also report times with the caches flushed first
    cold = _cold_ms(fn, args.steps) if n * 4 <= (1 << 26) else {}
    copy_gbs = _copy_ceiling(keys) if name == "uniform_u32_100M_radix_r8" else None
    _STEPS_MS[:] = steps_ms
    w = 4
    if algo == "radix":
        passes = -(-32 // bits)
        per_pass = 2 * n * w
        total = n * w + passes * per_pass
        kname = "k_chunk_count + k_chunk_scan + k_chunk_sort (one 11-bit digit pass)" if bits == 11 else \
            "k_onesweep (one digit pass)"
        roof = _roofline(kname, per_pass, avg.get("pass", float("nan")),
                         {"traffic": measured_traffic() if name == "uniform_u32_100M_radix_r8" else None,
                          "copy_ceiling_gbs": copy_gbs,
                          "frac_of_copy": (round(per_pass / (avg.get("pass", float("nan")) * 1e-3) / 1e9 / copy_gbs, 4)
                                           if copy_gbs else None),
                          "kernel_avg_ms": {k: round(x, 5) for k, x in avg.items()},
                          "sort_level_frac": round(total / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "algorithmic_bytes_per_sort": total})
    else:
        per_pass = 2 * n * w
        roof = _roofline("k_onesweep<BucketDigit> (one bucket-scatter pass)", per_pass,
                         avg.get("bucket_scatter", float("nan")),
                         {"kernel_avg_ms": {k: round(x, 5) for k, x in avg.items()}})
    ok = _sorted_permutation(keys_h, out.cpu().numpy())
    cpu = None
    if not args.no_cpu_baseline and name == "uniform_u32_100M_radix_r8":
        cpu = cpu_baseline(keys_h, algo, bits, B, args)
    tname = {"u32": "uint32", "i32": "int32", "f32": "float32"}[kind]
    metric = "Gkeys/s at 100M uint32 (LSD radix, 8-bit digits)" if name == "uniform_u32_100M_radix_r8" else \
        f"Gkeys/s ({algo}, {n} {tname} keys)"
    mem = _memory(4, False, n, algo=algo, digit_bits=bits, num_buckets=B)
    return _line(metric, value, "Gkeys/s", ms, args.steps, args.warmup, kind,
                 {"workload": name, "n": n, "distribution": DISTS[p["dist"]] if kind == "u32" else kind,
                  "algo": algo, "digit_bits": bits, "num_buckets": B or None}, roof, cpu,
                 output_matches_library_sort=ok, memory=mem, **cold)


# section 3.2, Table 1 of the paper: seconds on its i5 laptop, one thread, by
# (case, n) for RADIX sort and bucket sort; context for the case lines only
PAPER_TABLE1 = {
    "radix": {1: (1.78, 17.66, 176.84), 2: (1.88, 18.93, 174.85), 3: (1.86, 17.69, 178.68),
              4: (1.05, 11.10, 105.31), 5: (2.45, 24.56, 246.28), 6: (1.77, 17.66, 176.65)},
    "bucket": {1: (0.74, 5.84, 45.92), 2: (0.61, 4.14, 26.83), 3: (0.61, 4.12, 28.27),
               4: (0.31, 3.00, 31.54), 5: (0.78, 8.54, 97.43), 6: (0.61, 5.18, 41.06)},
}


def run_paper(name, p, args):
    """One of the paper's six input cases at one of its three sizes: radix
    sort (8-bit digits) or bucket sort with the paper's own map, B = n
    buckets over the declared range [0, M]."""
    import numpy as np
    import torch

    import workloads
    from paper_1206_3511_amd import intsort as I

    case, n, algo = p["case"], p["n"], p["algo"]
    print(f"bench[{name}]: generating case {case}, n={n}", file=sys.stderr, flush=True)
    keys_h, M = workloads.paper_case(case, n)
    keys = torch.from_numpy(keys_h).to("cuda:0")
    out = torch.empty_like(keys)
    ctx = I.context(0)
    opts = dict(algo="radix", digit_bits=8) if algo == "radix" else dict(algo="bucket", num_buckets=n, key_bound=M)
    fn = lambda: I.sort(keys, out=out, **opts)  # noqa: E731
    steps = max(2, args.steps // 4)
    ms = _timed(fn, steps, 1)
    value = n / (ms * 1e-3) / 1e9
    avg = _kernel_avgs(ctx, fn, steps)
    kind = "pass" if algo == "radix" else "bucket_scatter"
    roof = _roofline("k_onesweep (one pass)" if algo == "radix" else "k_onesweep<BucketDigit> (one scatter pass)",
                     2 * n * 4, avg.get(kind, float("nan")), {"kernel_avg_ms": {k: round(x, 5) for k, x in avg.items()}})
    ok = _sorted_permutation(keys_h, out.cpu().numpy())
    sec = PAPER_TABLE1[algo][case][{10**6: 0, 10**7: 1, 10**8: 2}[n]]
    return _line(f"Gkeys/s (paper case {case}, {algo})", value, "Gkeys/s", ms, steps, 1, "u32",
                 {"workload": name, "case": case, "n": n, "M": M, "algo": algo,
                  "buckets": n if algo == "bucket" else None, "declared_range": [0, M] if algo == "bucket" else None},
                 roof, None, output_matches_library_sort=ok,
                 paper={"seconds": sec, "Gkeys_per_s": round(n / sec / 1e9, 7),
                        "machine": "Intel i5 laptop, one thread (section 3.1)"},
                 memory=_memory(4, False, n, **opts))


def cpu_baseline(keys_h, algo, bits, B, args):
    import oracle

    n = keys_h.shape[0]
    m = min(args.cpu_sample, n) if args.cpu_sample > 0 else n
    sample = keys_h[:m].copy()
    print(f"bench: CPU oracle on {m} keys", file=sys.stderr, flush=True)
    runs, spent, best = 0, 0.0, float("inf")
    # one core, the first this process may use, for the whole timing
    try:
        old_aff = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(old_aff)})
    except (AttributeError, OSError):
        old_aff = None
    while runs < 1 or (spent < args.cpu_seconds and runs < 20):
        t0 = time.perf_counter()
        if algo == "radix":
            oracle.radix_lsd(sample, r=bits)
        else:
            oracle.bucket(sample, num_buckets=B or 1024)
        dt = time.perf_counter() - t0
        spent += dt
        best = min(best, dt)
        runs += 1
    if old_aff is not None:
        os.sched_setaffinity(0, old_aff)
    per = spent / runs
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": round(m / per / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "host_cores": os.cpu_count(),
            "sample": f"{'all' if m == n else 'first'} {m} keys of the same input, single-threaded oracle "
                      f"{algo} sort repeated {runs} times ({spent:.1f} s, mean {per:.3f} s, best {best:.3f} s)"}


def run_pairs(name, p, args):
    import numpy as np
    import torch

    import workloads
    from paper_1206_3511_amd import intsort as I

    n, algo, bits, B = p["n"], p["algo"], p["bits"], p["B"]
    print(f"bench[{name}]: generating", file=sys.stderr, flush=True)
    kh, vh = workloads.config3_pairs(p["variant"], n)
    k = torch.from_numpy(kh).to("cuda:0")
    v = torch.from_numpy(vh).to("cuda:0")
    ok_, ov_ = torch.empty_like(k), torch.empty_like(v)
    ctx = I.context(0)
    fn = lambda: I.sort_pairs(k, v, algo=algo, digit_bits=bits, num_buckets=B, out_keys=ok_, out_vals=ov_)  # noqa
    steps = max(1, args.steps // 4)
    ms = _timed(fn, steps, 1)
    value = n / (ms * 1e-3) / 1e9
    avg = _kernel_avgs(ctx, fn, steps)
    kind = "pass" if algo == "radix" else "bucket_scatter"
    kname = ("k_chunk_count + k_chunk_scan + k_chunk_sort (one 11-bit pass, pairs)" if algo == "radix" and bits == 11
             else f"k_onesweep (one pass, pairs, {algo})")
    roof = _roofline(kname, 2 * n * 12, avg.get(kind, float("nan")),
                     {"kernel_avg_ms": {kk: round(x, 5) for kk, x in avg.items()}})
    order = np.argsort(kh, kind="stable")
    good = bool(np.array_equal(ok_.cpu().numpy(), kh[order]) and np.array_equal(ov_.cpu().numpy(), vh[order]))
    return _line(f"Gkeys/s ({algo} pairs, 100M uint64 keys + uint32 payload)", value, "Gkeys/s", ms, steps, 1,
                 "u64+u32", {"workload": name, "n": n, "variant": p["variant"], "algo": algo, "digit_bits": bits,
                             "num_buckets": B or None}, roof, None, output_matches_stable_library_sort=good,
                 memory=_memory(8, True, n, algo=algo, digit_bits=bits, num_buckets=B))


def run_batched(name, p, args):
    import numpy as np
    import torch

    import workloads
    from paper_1206_3511_amd import intsort as I

    print(f"bench[{name}]: generating 10,000 arrays", file=sys.stderr, flush=True)
    keys, offsets = workloads.segmented_keys()
    N = keys.size
    k = torch.from_numpy(keys).to("cuda:0")
    out = torch.empty_like(k)
    offs = torch.from_numpy(offsets.view(np.int64)).to("cuda:0")
    ctx = I.context(0)
    from paper_1206_3511_amd import autotune

    cut = autotune.tuned_options("segmented", 4, N)
    bits = autotune.tuned_options("segmented_bits", 4, N)
    choice = {**cut, **bits}
    tuned_now = not (cut and bits)
    if tuned_now:
        print(f"bench[{name}]: autotuning the LDS cutoff and digit width", file=sys.stderr, flush=True)
        choice = autotune.tune_segmented(k, offs)
    fn = lambda: I.segmented_sort(k, offs, out_keys=out, **choice)  # noqa: E731
    steps = max(1, args.steps // 4)
    ms_stream = _timed(fn, steps, 1)
    avg = _kernel_avgs(ctx, fn, steps)
    ms, launch = ms_stream, "one launch sequence per batch (no graph: profiling run)"
    steps_ms = list(_STEPS_MS)
    if not args.profile_light:
        # the same calls recorded once into a HIP graph and replayed: one
        # graph launch per batch
        side = torch.cuda.Stream()
        graph = I.capture(fn, side)
        with torch.cuda.stream(side):
            ms = _timed(lambda: graph.launch(side), steps, 1)
        steps_ms = list(_STEPS_MS)
        launch = "one HIP graph replay per batch"
    # the first 2^20 outputs against numpy's sort of the arrays they come from
    head, j = [], 0
    while sum(a.size for a in head) < (1 << 20) and j < len(offsets) - 1:
        head.append(np.sort(keys[int(offsets[j]):int(offsets[j + 1])]))
        j += 1
    ref = np.concatenate(head)[:1 << 20]
    graph_ok = bool(np.array_equal(out[:ref.size].cpu().numpy(), ref))
    if not args.profile_light:
        graph.close()
    value = N / (ms * 1e-3) / 1e9
    ms_loop = None
    if not args.profile_light:
        # the plain path: every array in its own buffer, one sort call each
        arrs = [k[int(offsets[j]):int(offsets[j + 1])].clone() for j in range(len(offsets) - 1)]
        outs = [torch.empty_like(a) for a in arrs]

        def loop():
            for a, b in zip(arrs, outs):
                I.sort(a, out=b)
        ms_loop = _timed(loop, 1, 1)
        del arrs, outs
    _STEPS_MS[:] = steps_ms
    # what the pass launches move: the arrays longer than the LDS cutoff,
    # each in the passes whose digit is not constant inside it (an array
    # skips the others), averaged over the 4 pass launches of a sort
    cut = int(choice.get("lds_cutoff") or SEG_LDS_MAX_U32)
    moved = 0
    for j in np.nonzero(np.diff(offsets) > cut)[0]:
        seg = keys[int(offsets[j]):int(offsets[j + 1])]
        diff = int(np.bitwise_or.reduce(seg ^ seg[0]))
        moved += seg.size * sum(1 for p in range(4) if (diff >> (8 * p)) & 255)
    roof = _roofline("k_onesweep<SegTiles> (one digit pass of the arrays above the LDS cutoff)", 2 * 4 * moved / 4,
                     avg.get("pass", float("nan")), {"kernel_avg_ms": {kk: round(x, 5) for kk, x in avg.items()},
                                                     "keys_moved_per_sort": int(moved)})
    extra = {}
    if ms_loop is not None:
        extra = {"per_array_loop": {"value": round(N / (ms_loop * 1e-3) / 1e9, 3), "ms": round(ms_loop, 3)},
                 "speedup_vs_per_array_loop": round(ms_loop / ms, 2)}
    return _line("Gkeys/s (batched segmented sort of 10,000 uint32 arrays)", value, "Gkeys/s", ms, steps, 1, "u32",
                 {"workload": name, "arrays": len(offsets) - 1, "keys": int(N), "sizes": "log-uniform [16, 2^20)",
                  "tuned": choice, "tuned_in_this_run": tuned_now, "launch": launch},
                 roof, None, **extra,
                 stream_launches={"value": round(N / (ms_stream * 1e-3) / 1e9, 3), "ms": round(ms_stream, 5)},
                 graph_output_matches_per_array_sort=graph_ok,
                 memory=_memory(4, False, int(N), len(offsets) - 1, **choice))


def serve_trace(I, pool, out_cap_bytes, trace, mode, sample_every=0):
    """Replays the trace through a server.  Requests arrive at their trace
    times (open loop); each gets an output tensor of its own size, and a
    request that would take the output memory in flight past `out_cap_bytes`
    waits until completions free enough (that wait counts in its latency,
    which runs from arrival to the completion the driver observes).
    Returns (throughput Gkeys/s, p50 s, p99 s, requests, keys, samples)."""
    import numpy as np
    import torch

    t_arr, wid, nn, dd = trace
    max_batch, slots = (64, 2) if mode == "batched" else (1, 1)
    srv = I.Server(0, budget_bytes=64 << 30, max_batch=max_batch, slots=slots)
    inflight = 0
    lat, keys_done, live, samples = [], 0, {}, []
    R = len(t_arr)
    i = 0
    t0 = time.perf_counter()
    first = last = None
    while i < R or live:
        now = time.perf_counter() - t0
        while i < R and t_arr[i] <= now:
            n = int(nn[i])
            nbytes = n * int(wid[i])
            if live and inflight + nbytes > out_cap_bytes:
                break
            src = pool[(int(wid[i]), int(dd[i]))][:n]
            out = torch.empty_like(src)
            inflight += nbytes
            tk = srv.submit(src, out)
            live[tk] = (i, nbytes, out)
            if first is None:
                first = time.perf_counter()
            i += 1
        for tk, _ in srv.completed():
            idx, nbytes, out = live.pop(tk)
            done = time.perf_counter()
            lat.append(done - (t0 + t_arr[idx]))
            keys_done += int(nn[idx])
            if sample_every and idx % sample_every == 0 and len(samples) < 40:
                samples.append((idx, out))
            inflight -= nbytes
            last = done
        time.sleep(0.0001)
    srv.drain()
    srv.close()
    lat = np.array(lat)
    span = (last - first) if (first and last) else float("nan")
    return keys_done / span / 1e9, float(np.percentile(lat, 50)), float(np.percentile(lat, 99)), len(lat), \
        keys_done, samples


def run_serving(name, p, args):
    import numpy as np
    import torch

    import oracle
    import workloads
    from paper_1206_3511_amd import intsort as I

    seconds = args.serve_seconds
    trace = workloads.serving_trace(rate=2000.0, seconds=seconds)
    print(f"bench[{name}]: {len(trace[0])} requests over {seconds} s; building device pool", file=sys.stderr,
          flush=True)
    pool = {}
    for wdt in (4, 8):
        for d in range(7):
            pool[(wdt, d)] = workloads.device_keys(d, 1 << 26, 7000 + 10 * d + wdt, wdt, "cuda:0")
    torch.cuda.synchronize()
    out_cap = int(args.serve_out_gb * (1 << 30))
    res = {}
    for mode in ("batched", "plain"):
        print(f"bench[{name}]: {mode}", file=sys.stderr, flush=True)
        thr, p50, p99, cnt, keys, samples = serve_trace(I, pool, out_cap, trace, mode,
                                                        sample_every=100 if mode == "batched" else 0)
        print(f"bench[{name}]: {mode}: {thr:.2f} Gkeys/s p50 {p50 * 1e3:.3f} ms p99 {p99 * 1e3:.3f} ms",
              file=sys.stderr, flush=True)
        res[mode] = {"gkeys_per_s": round(thr, 3), "p50_ms": round(p50 * 1e3, 3), "p99_ms": round(p99 * 1e3, 3),
                     "requests": cnt, "keys": keys}
        if mode == "batched":
            bad = 0
            for idx, out in samples[:40]:
                src = pool[(int(trace[1][idx]), int(trace[3][idx]))][: int(trace[2][idx])]
                got = out.cpu().numpy()
                alone = I.sort(src).cpu().numpy()
                ref = oracle.radix_lsd(src.cpu().numpy()).keys
                bad += int(not (np.array_equal(got, ref) and got.tobytes() == alone.tobytes()))
            res["checked_samples"] = min(40, len(samples))
            res["sample_mismatches"] = bad
    b = res["batched"]
    return _line("Gkeys/s served (Poisson 2000 req/s, uint32/uint64, 1K-64M keys)", b["gkeys_per_s"], "Gkeys/s",
                 float("nan"), 0, 0, "u32/u64",
                 {"workload": name, "rate_per_s": 2000, "seconds": seconds, "budget_gb": 64, "max_batch": 64,
                  "slots": 2, "output_cap_gb": args.serve_out_gb}, None, None, serving=res,
                 p50_ms=b["p50_ms"], p99_ms=b["p99_ms"], plain_path=res["plain"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform_u32_100M_radix_r8",
                    help="one of: " + ", ".join(sorted(WORKLOADS)) + ", all, or paper_suite (the 36 case lines)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="keys of the same input that the CPU oracle sorts (0 = all of them)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the CPU oracle sort until this much time has passed")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the serving trace")
    ap.add_argument("--serve-out-gb", type=float, default=64.0,
                    help="serving trace: output memory the requests in flight may hold")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB plain copy (for scaling hardware byte counters)")
    ap.add_argument("--profile-light", action="store_true",
                    help="batched workload: leave out the graph replay and the one-call-per-array comparison "
                         "(for profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline run: leave out the batched and serving results it appends")
    ap.add_argument("--extras-serve-seconds", type=float, default=20.0,
                    help="headline run: length of the serving trace whose results it appends")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "all":
        names = sorted(WORKLOADS)
    elif args.workload == "paper_suite":
        names = [k for k in WORKLOADS if k.startswith("paper_case")]
    else:
        names = [args.workload]
    if args.calibrate_copy:
        calibrate_copy()
    for name in names:
        if name not in WORKLOADS:
            print(f"unknown workload {name}", file=sys.stderr)
            sys.exit(2)
        kind, p = WORKLOADS[name]
        fn = {"plain": run_plain, "pairs": run_pairs, "batched": run_batched, "serving": run_serving,
              "paper": run_paper}[kind]
        _STEPS_MS.clear()
        line = fn(name, p, args)
        import torch
        torch.cuda.empty_cache()
        if name == HEADLINE and len(names) == 1 and not args.no_extras:
            line.update(headline_extras(args))
        print(json.dumps(line), flush=True)
        torch.cuda.empty_cache()


def headline_extras(args):
    """The metric's other halves, appended to the headline line: the batched
    segmented sort of 10,000 arrays against one call per array, and the
    serving loop (continuous batching against one request per launch) on a
    shorter trace.  A failure is reported in the line, not raised."""
    import copy

    import torch
    out = {}
    steps_ms = list(_STEPS_MS)
    try:
        a = copy.copy(args)
        a.steps = 8
        r = run_batched("config4_batched_10k", {}, a)
        out["config4_batched"] = {
            "gkeys_per_s": r["value"], "ms_per_batch": r["ms_per_step"], "arrays": r["config"]["arrays"],
            "keys": r["config"]["keys"], "tuned": r["config"]["tuned"],
            "per_array_loop_gkeys_per_s": r["per_array_loop"]["value"],
            "speedup_vs_per_array_loop": r["speedup_vs_per_array_loop"],
            "output_matches_per_array_sort": r["graph_output_matches_per_array_sort"]}
    except Exception as e:   # noqa: BLE001
        out["config4_batched"] = {"error": f"{type(e).__name__}: {e}"}
    torch.cuda.empty_cache()
    try:
        a = copy.copy(args)
        a.serve_seconds = args.extras_serve_seconds
        r = run_serving("config5_serving", {}, a)
        sv = r["serving"]
        out["config5_serving"] = {
            "trace_seconds": a.serve_seconds, "rate_per_s": 2000,
            "batched": sv["batched"], "plain": sv["plain"],
            "checked_samples": sv.get("checked_samples"), "sample_mismatches": sv.get("sample_mismatches")}
    except Exception as e:   # noqa: BLE001
        out["config5_serving"] = {"error": f"{type(e).__name__}: {e}"}
    _STEPS_MS[:] = steps_ms
    return out


if __name__ == "__main__":
    main()
