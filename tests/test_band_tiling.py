"""The band kernel's tiling and the layer-memory ownership its fused path
relies on, checked by brute force on random grids (host code only: the tile
geometry functions of csrc/fdtd_dev.hpp, compiled with hipcc for the host)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not (os.path.exists(hipcc) or shutil.which(hipcc)):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "band_tiling_check")
    src = os.path.join(ROOT, "tests", "band_tiling_check.cpp")
    inc = os.path.join(ROOT, "paper_2606_06910_amd", "csrc")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-I", inc, "-o", exe, src], check=True, capture_output=True)
    return exe


def test_band_tiling_brute_force(tmp_path):
    exe = _build(tmp_path)
    out = subprocess.run([exe, "2000"], check=False, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0 and out.stdout.startswith("ok"), out.stdout + out.stderr
    fused = int(out.stdout.split()[2])
    assert fused > 1000   # most random geometries take the fused path


def test_bench_x_range_matches_the_library(tmp_path):
    """bench.py's algorithmic byte counts take the z-march's x range from its
    own restatement of the library's whole-tile rule (band_range_x); the two
    must agree, or the roofline would price points the kernel does not update."""
    import bench

    exe = _build(tmp_path)
    cases = [(n, lo, hi) for n in (9, 40, 63, 64, 65, 96, 100, 131, 200, 288, 512, 768, 1024)
             for lo in (0, 3, 15, 20, 28, 40) for hi in (0, 5, 15, 20, 28) if lo + hi + 8 <= n]
    inp = "".join("%d %d %d\n" % c for c in cases)
    out = subprocess.run([exe, "ranges"], input=inp, check=True, capture_output=True, text=True, timeout=60)
    got = [tuple(int(v) for v in line.split()) for line in out.stdout.splitlines()]
    assert got == [bench.x_range(*c) for c in cases]
