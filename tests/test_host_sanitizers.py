"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the FP64 oracle driven through every entry point on small grids (uneven and
missing layers, a periodic pair of axes, the smallest axis the stencil
allows), and the band-tiling brute force of the shared geometry header.
Any invalid access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    src = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", exe, src, "-lm"], check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr[-2000:]


def test_band_tiling_under_asan_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "band_tiling_sanitize")
    src = os.path.join(ROOT, "tests", "band_tiling_check.cpp")
    inc = os.path.join(ROOT, "paper_2606_06910_amd", "csrc")
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-I", inc, "-o", exe, src], check=True, capture_output=True)
    out = subprocess.run([exe, "300"], capture_output=True, text=True, timeout=300, env=ENV)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr[-2000:]
