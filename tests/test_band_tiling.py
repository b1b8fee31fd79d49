"""The band kernel's tiling and the layer-memory ownership its fused path
relies on, checked by brute force on random grids (host code only: the tile
geometry functions of csrc/fdtd_dev.hpp, compiled with hipcc for the host)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_band_tiling_brute_force(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "band_tiling_check")
    src = os.path.join(ROOT, "tests", "band_tiling_check.cpp")
    inc = os.path.join(ROOT, "paper_2606_06910_amd", "csrc")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", inc, "-o", exe, src], check=True, capture_output=True)
    out = subprocess.run([exe, "2000"], check=False, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
    fused = int(out.stdout.split()[2])
    assert fused > 1000   # most random geometries take the fused path
