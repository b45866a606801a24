"""bench.py's command-line contract on the CPU: it measures one GPU, so a
request for more exits with status 2 and says so before touching a device,
and every workload name it lists is one it accepts."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def _bench(*args, timeout=120):
    return subprocess.run([sys.executable, str(ROOT / "bench.py"), *args], capture_output=True, text=True,
                          timeout=timeout, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_workload_names():
    sys.path.insert(0, str(ROOT))
    import bench
    names = set(bench.WORKLOADS)
    assert "uniform_u32_100M_radix_r8" in names and "config4_batched_10k" in names
    assert {f"paper_case{c}_n1e{e}_{a}" for c in range(1, 7) for e in (6, 7, 8) for a in ("radix", "bucket")} <= names
    r = _bench("--help")
    assert r.returncode == 0 and "paper_suite" in r.stdout
