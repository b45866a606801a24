"""The bucket index of bucket sort, checked on the host (no GPU): the
library's make_bucket_map / bucket_of (csrc/bucket_map.hpp, host and device
functions, the same source the kernels compile) against exact 128-bit
arithmetic, exhaustively for every range and bucket count up to 300 and at
sampled bucket boundaries up to R = 2^64 (tests/sanitize/bucket_index_check.cpp)."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.timeout(300)
def test_bucket_index_against_128_bit_arithmetic(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    exe = tmp_path / "bucket_index_check"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", f"-I{ROOT / 'include'}",
                        f"-I{ROOT / 'paper_1206_3511_amd' / 'csrc'}", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", str(ROOT / "tests/sanitize/bucket_index_check.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-3000:]
    assert r.stdout.startswith("0 of ")
