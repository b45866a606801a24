"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers in tests/sanitize/ are built with both sanitizers and run here:

* oracle_check.c links the C oracle and runs every entry point on seeded
  inputs (radix with 1- to 16-bit digits, bucket sort with 1 to n+1 buckets,
  the ordered key types, segmented sorts, argument errors); leaks fail too.
* abi_check.cpp links the library's host code (every source of the shared
  library, the host side built with the sanitizers, the device side as
  usual) and drives a planning context (device -1): option parsing,
  workspace sizing for every key type, algorithm and digit width, the tuning
  table reader on good, malformed and missing files, and the argument checks
  of every entry point.  No kernel runs.

Any sanitizer report aborts the driver (-fno-sanitize-recover), so the test
asserts a zero exit status.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1206_3511_amd" / "csrc"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
# hipcc applies each -fsanitize to the host pass only when -Xarch_host precedes it
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(map(str, cmd))}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.timeout(300)
def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = tmp_path / "oracle_check"
    _run([gcc, "-O1", "-g", "-std=c11", "-Wall", "-Wextra", *SAN,
          str(ROOT / "tests/sanitize/oracle_check.c"), str(ROOT / "oracle/oracle.c"), "-o", str(exe)])
    r = _run([str(exe)], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"}, timeout=240)
    assert "passed" in r.stdout


@pytest.mark.timeout(900)
def test_abi_host_code_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("hipcc or clang++ not found")
    sources = sorted(list(CSRC.glob("*.hip")) + list(CSRC.glob("*.cpp")))
    assert sources, "no library sources"
    common = ["-O1", "-g", "-std=c++17", "-fPIC", f"-I{ROOT / 'include'}", f"-I{CSRC}"]

    def compile_one(src):
        obj = tmp_path / (src.name + ".o")
        _run([HIPCC, "--offload-arch=gfx950", *common, *HOST_SAN,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-c", str(src), "-o", str(obj)])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
        objs = list(pool.map(compile_one, sources))
    drv = tmp_path / "abi_check.o"
    _run([CLANGXX, *common, *SAN, "-c", str(ROOT / "tests/sanitize/abi_check.cpp"), "-o", str(drv)])
    exe = tmp_path / "abi_check"
    _run([HIPCC, "--offload-arch=gfx950", *HOST_SAN, str(drv), *map(str, objs), "-o", str(exe)])
    # the HIP runtime keeps process-lifetime allocations: leak reports are off
    env = {**os.environ, "ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1"}
    r = _run([str(exe), str(tmp_path / "tune.tsv")], env=env, timeout=240)
    assert "abi checks passed" in r.stdout
