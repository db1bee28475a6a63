"""The host side of the C ABI under AddressSanitizer (CPU only): argument
validation, pyramid geometry, workspace layout and sizing, tunables, status
strings and the profiling record, driven by tests/host_abi_checks.cpp against
every library source built with ASan on its host code."""

import os
import subprocess

from paper_1605_02060_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_abi_paths_under_address_sanitizer(tmp_path):
    exe = B.build_host_asan(str(tmp_path), os.path.join(HERE, "host_abi_checks.cpp"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "host ABI checks passed" in r.stdout
