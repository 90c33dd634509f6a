"""Host-side check of the exact fixed-point cell sums of the HIP path
(to_fixed, the velocity range check and the bounds that keep every 64-bit
sum from wrapping), compiled from the library's own header and run on the
CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_to_fixed_truncates_and_range_bounds_the_sums(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fixed_point_check")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_2212_11878_amd", "csrc"),
                    os.path.join(ROOT, "tests", "fixed_point_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
