"""Writes tests/golden/input_checksums.json: the 64-bit checksums of the
first 2^16 keys of every seeded input distribution.  It calls only the input
generator (workloads.py) and never the GPU library; rerun it only when the
generator's definition changes on purpose."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import workloads as w  # noqa: E402


def main():
    out = {"n": 1 << 16, "config2": {}, "config3": {}}
    for d, name in enumerate(w.DISTRIBUTIONS):
        out["config2"][name] = hex(w.checksum(w.config2_keys(d, 1 << 16)))
    for v in ("full", "b40"):
        k, _ = w.config3_pairs(v, 1 << 16)
        out["config3"][v] = hex(w.checksum(k))
    out["paper_cases"] = {str(c): hex(w.checksum(w.paper_case(c, 1 << 16)[0])) for c in range(1, 7)}
    out["signed_ieee"] = {
        "int32": hex(w.checksum(w.signed_keys(1 << 16, 32, seed=1))),
        "int64": hex(w.checksum(w.signed_keys(1 << 16, 64, seed=1))),
        "int32_b12": hex(w.checksum(w.signed_keys(1 << 16, 32, seed=1, spread_bits=12))),
        "float32": hex(w.checksum(w.ieee_keys(1 << 16, 32, seed=1))),
        "float64": hex(w.checksum(w.ieee_keys(1 << 16, 64, seed=1))),
    }
    sizes, dists = w.segment_plan(64)
    out["segment_plan_64"] = {"sizes": [int(x) for x in sizes], "dists": [int(x) for x in dists]}
    with open(os.path.join(HERE, "input_checksums.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
