"""Benchmark of the MI355X integer sort.

One step = one complete sort (every kernel of the method) of one array that
is already resident in HBM, out of place from a pristine input.  The default
workload is the headline: 100,000,000 uint32 keys drawn uniformly from
[0, 2^32) (seed 0), LSD radix sort with 8-bit digits (4 passes).

Prints one JSON line with the throughput (Gkeys/s), the roofline figure of the
dominant kernel (the digit pass), and the single-threaded CPU oracle timed on
a bounded sample of the same input.
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

WORKLOADS = {
    # name: (distribution, n, key dtype, algo, digit bits)
    "uniform_u32_100M_radix_r8": ("uniform", 100_000_000, "u32", "radix", 8),
    "uniform_u32_100M_bucket": ("uniform", 100_000_000, "u32", "bucket", 8),
    "uniform_u32_1M_radix_r8": ("uniform", 1_000_000, "u32", "radix", 8),
}


def algorithmic_bytes(n: int, w: int, v: int, passes: int) -> dict:
    """Irreducible HBM traffic of LSD radix with a one-read histogram:
    the histogram reads every key once; every pass reads and writes every key
    (and value) once."""
    per_pass = 2 * n * (w + v)
    return {"histogram": n * w, "pass": per_pass, "total": n * w + passes * per_pass}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform_u32_100M_radix_r8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="keys of the same input that the CPU oracle sorts (0 = all of them)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the CPU oracle sort until this much time has passed")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1206_3511_amd import intsort as I

    dist, n, kdt, algo, bits = WORKLOADS[args.workload]
    assert kdt == "u32"
    w, v = 4, 0
    passes = -(-32 // bits)
    print(f"bench: generating {n} keys ({dist}, seed 0)", file=sys.stderr, flush=True)
    keys_h = workloads.config2_keys(dist, n, seed=0)
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(keys_h).to(dev)
    out = torch.empty_like(keys)
    ctx = I.context(0)
    opts = dict(algo=algo, digit_bits=bits)

    print("bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        I.sort(keys, out=out, **opts)
    torch.cuda.synchronize()

    # ---- timed region: K whole sorts, no per-kernel events
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        I.sort(keys, out=out, **opts)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / args.steps
    value = n / (ms * 1e-3) / 1e9
    print(f"bench: {ms:.4f} ms/sort, {value:.2f} Gkeys/s", file=sys.stderr, flush=True)

    # ---- the same K sorts again with HIP events around every kernel, on the
    # stream the kernels run on: average duration of each kernel kind
    ctx.timing(True)
    ctx.kernel_times()
    for _ in range(args.steps):
        I.sort(keys, out=out, **opts)
    times = ctx.kernel_times()
    ctx.timing(False)
    per_kind: dict[str, list[float]] = {}
    for kind, idx, t in times:
        per_kind.setdefault(kind, []).append(t)
    avg = {k: sum(x) / len(x) for k, x in per_kind.items()}
    ab = algorithmic_bytes(n, w, v, passes)
    pass_ms = avg.get("pass", float("nan"))
    achieved = ab["pass"] / (pass_ms * 1e-3) / 1e9
    roofline = {
        "bound": "hbm",
        "kernel": "k_onesweep (one digit pass)",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "bytes_per_launch": ab["pass"],
        "avg_launch_ms": round(pass_ms, 5),
        "kernel_avg_ms": {k: round(x, 5) for k, x in avg.items()},
        "sort_level_frac": round(ab["total"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }

    # correctness of the timed output against a library sort of the same keys
    ok = bool(np.array_equal(out.cpu().numpy(), np.sort(keys_h)))

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        m = min(args.cpu_sample, n) if args.cpu_sample > 0 else n
        sample = keys_h[:m].copy()
        print(f"bench: CPU oracle on {m} keys", file=sys.stderr, flush=True)
        runs, spent, best = 0, 0.0, float("inf")
        while runs < 1 or (spent < args.cpu_seconds and runs < 20):
            t0 = time.perf_counter()
            if algo == "radix":
                oracle.radix_lsd(sample, r=bits)
            else:
                oracle.bucket(sample, num_buckets=1024)
            dt = time.perf_counter() - t0
            spent += dt
            best = min(best, dt)
            runs += 1
        per = spent / runs
        cpu = {"value": round(m / per / 1e9, 6), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"{'all' if m == n else 'first'} {m} keys of the same input, single-threaded oracle "
                         f"{algo} sort repeated {runs} times ({spent:.1f} s, mean {per:.3f} s, best {best:.3f} s)"}

    line = {
        "metric": "Gkeys/s at 100M uint32 (LSD radix, 8-bit digits)" if n == 100_000_000 else "Gkeys/s",
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "distribution": dist, "seed": 0, "algo": algo,
                   "digit_bits": bits, "passes": passes},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "output_matches_library_sort": ok,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
