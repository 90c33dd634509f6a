"""The C ABI used from a plain C program (no Python, no PyTorch): default
context (the library's own hipMalloc and stream), status codes, a Maxwell
box stepped and observed, state round trip, profiling, release."""
import subprocess

import pytest

from test_abi_cpu import _build_c_client

pytestmark = pytest.mark.gpu


def test_c_client_runs(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    exe = _build_c_client(tmp_path)
    print("[case] c client", flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("ok"), (out.returncode, out.stdout, out.stderr)
