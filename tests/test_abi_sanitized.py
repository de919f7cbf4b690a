"""The C ABI's host code under AddressSanitizer and UBSan (CPU only, no GPU).

Builds libsoftshadow's sources together with tests/abi_driver.c, sanitizers on
the host side only (device code is built as usual), and runs the driver: every
entry point with arguments its validation must reject, and the layout helpers
over many shapes.  A sanitizer report or an unexpected status fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_under_sanitizers(tmp_path):
    import glob
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2005_06671_amd", "csrc", "*.hip")))
    exe = str(tmp_path / "abi_driver")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument",
           "-o", exe, "-x", "c++", os.path.join(ROOT, "tests", "abi_driver.c"), "-x", "hip"] + srcs
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    out = run.stdout + run.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert run.returncode == 0 and "ok" in run.stdout, out[-4000:]
