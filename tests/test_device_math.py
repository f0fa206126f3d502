"""The kernels' integer helpers, compiled for the host by hipcc and checked
against 128-bit integer arithmetic and Philox known answers (CPU only)."""
import os
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2408_06213_amd", "csrc")


def test_device_helpers_on_host(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not installed")
    exe = tmp_path / "device_math_check"
    src = os.path.join(ROOT, "tests", "native", "device_math_check.cpp")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
                    "-I", CSRC, src, "-o", str(exe)], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
