"""CPU checks of the byte and point counts bench.py turns into roofline figures."""
import itertools

import numpy as np
import pytest

import bench


def _in_band(c, n, lo, hi):
    return (lo > 0 and c < lo + 4) or (hi > 0 and c >= n - hi - 4)


def _in_xbox(x, n, lo, hi):
    # x band boxes one 32-point tile wide where the band fits one: the low box
    # [0, 32), the high box from max(32 * floor((n - hi - 4) / 32), n - 32)
    if _in_band(x, n, lo, hi):
        return True
    a = 32 if lo > 0 and lo + 4 <= 32 else (lo + 4 if lo > 0 else 0)
    b0 = n - hi - 4 if hi > 0 else n
    b = max(b0 // 32 * 32, n - 32) if hi > 0 and hi + 4 <= 32 else b0
    if a > b:
        return False
    return x < a or x >= b


@pytest.mark.parametrize("n,cpml", [((30, 25, 20), (3, 5, 0, 2, 4, 4)), ((40, 36, 33), (20, 0, 0, 0, 0, 12)),
                                    ((9, 9, 9), (4, 4, 4, 4, 4, 4)), ((16, 17, 18), (0,) * 6),
                                    ((100, 12, 10), (20, 20, 2, 2, 2, 2)), ((131, 10, 9), (15, 15, 0, 3, 3, 0)),
                                    ((70, 8, 8), (15, 20, 0, 0, 0, 0))])
def test_band_split_matches_brute_force(n, cpml):
    band = 0
    for x, y, z in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        if (_in_xbox(x, n[0], cpml[0], cpml[1]) or _in_band(y, n[1], cpml[2], cpml[3])
                or _in_band(z, n[2], cpml[4], cpml[5])):
            band += 1
    inner, b = bench.band_split(n, cpml)
    assert b == band and inner + b == int(np.prod(n))


def test_slab_points_counts_layer_points_per_axis():
    n, cpml = (20, 30, 40), (2, 3, 0, 5, 7, 0)
    expect = (2 + 3) * 30 * 40 + 5 * 20 * 40 + 7 * 20 * 30
    assert bench.slab_points(n, cpml) == expect


def test_interior_bytes_are_16_per_point():
    n, cpml = (128, 96, 64), (20,) * 6
    # x: [32, 96) (the band boxes one tile wide each); y, z: [24, n - 24)
    assert bench.interior_kernel_bytes(n, cpml) == 16 * (96 - 32) * (96 - 48) * (64 - 48)


def test_measured_traffic_needs_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "c.txt"
    f.write_text("grid: 8x8x8\ntile_ry: 2\nsources_sha256: %s\nfetch_kib_per_launch: 10\n"
                 "write_kib_per_launch: 5\nfetch_factor: 2\nwrite_factor: 1\n" % bench.sources_digest())
    monkeypatch.setattr(bench, "COUNTERS", str(f))
    assert bench.measured_traffic((8, 8, 8), (2, 2, 1)) == 10 * 1024 * 2 + 5 * 1024
    assert bench.measured_traffic((8, 8, 9), (2, 2, 1)) is None
    assert bench.measured_traffic((8, 8, 8), (2, 1, 1)) is None
    assert bench.measured_traffic((8, 8, 8), (2, 2, 1, 2)) is None      # counters of one-column tiles
    assert bench.measured_traffic((8, 8, 8), (2, 2, 1, 1)) == 10 * 1024 * 2 + 5 * 1024
    f.write_text(f.read_text().replace(bench.sources_digest(), "0" * 64))
    assert bench.measured_traffic((8, 8, 8), (2, 2, 1)) is None


@pytest.mark.parametrize("every,G", [(1, 1), (7, 7), (16, 16), (17, 9), (25, 13), (120, 15)])
def test_adjoint_step_bytes_without_layers(every, G):
    # no layers: forward step 16 B, increment 12 B, pass 3 16 B, gradient pass 8 + 16 / G B per point
    n = (10, 12, 14)
    N = 10 * 12 * 14
    assert bench.adjoint_step_bytes(n, (0,) * 6, every) == pytest.approx(N * (16 + 12 + 16 + 8 + 16 / G))
