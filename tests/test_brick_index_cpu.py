"""Host-side check of the brick-binning index arithmetic the HIP kernels
use (compiled from the library's own header, run on the CPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_brick_tiling_groups_and_bucket_layout(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "brick_index_check")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-std=c++17",
                    "-I", os.path.join(ROOT, "paper_2212_11878_amd", "csrc"),
                    os.path.join(ROOT, "tests", "brick_index_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
