"""The register DFTs of the compile-time FFT plans (paper_1605_02060_amd/csrc/dft.h),
built for the host and checked length by length against a direct DFT in double
precision (tests/dft_host_check.cpp).  No GPU needed."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_register_dfts_match_a_direct_dft(tmp_path):
    exe = tmp_path / "dft_host_check"
    cmd = [HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_1605_02060_amd", "csrc"),
           os.path.join(ROOT, "tests", "dft_host_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    print(out.stdout)
    assert out.returncode == 0, out.stdout
    assert "R= 9" in out.stdout and "R=35" in out.stdout
