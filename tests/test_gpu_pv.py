"""First-order pressure-velocity path (include/fdtd_pv.h) on the GPU against
its FP64 oracle (oracle/pv_oracle.py), through the C ABI.

Bar (written here): FP32 fields against the FP64 oracle, relative L2 <= 1e-5
on receiver traces and pressure snapshots.  At the paper's smallest
throughput grid (320^3, lambda = 0.05, 20-cell layers, 64 steps) a property
that holds at any size: a mirror-symmetric pulse between mirrored layers
stays exactly mirror-symmetric on every axis (the central difference changes
sign exactly under reflection, and the profiles are mirror images).
"""
import numpy as np
import pytest

import synth
from helpers import rel_l2
from oracle import pv_oracle as P

pytestmark = pytest.mark.gpu


def _coords(n):
    z, y, x = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return x, y, z


def _gpu(n, cpml, lam, nt, src=None, wav=None, rec=None, p0=None, snap_every=0, variant=0):
    import torch

    from paper_2606_06910_amd import PVPropagator

    s = PVPropagator(n, cpml, lam, variant=variant)
    if p0 is not None:
        s.set_pressure(torch.from_numpy(p0.astype(np.float32)))
    if src is not None:
        s.set_source(src, torch.from_numpy(wav.astype(np.float32)))
    tr = s.record(rec, nt) if rec is not None else None
    snaps = []
    done = 0
    while done < nt:
        k = min(snap_every or nt, nt - done)
        s.step(k)
        done += k
        if snap_every and k == snap_every:
            snaps.append(s.get_pressure().cpu().double().numpy())
    p = s.get_pressure().cpu().double().numpy()
    torch.cuda.synchronize()
    out = (None if tr is None else tr.cpu().double().numpy(), np.array(snaps), p)
    s.close()
    return out


CASES = {
    # uneven layers, Ricker source, receivers everywhere (some inside layers)
    "uneven": dict(n=(40, 36, 32), cpml=(6, 5, 4, 7, 3, 5), lam=0.3, nt=120, src=(17, 15, 14), f0=0.08),
    # several 64-point x tiles, faces without layers
    "wide": dict(n=(150, 22, 20), cpml=(9, 0, 0, 6, 5, 0), lam=0.25, nt=90, src=(40, 11, 9), f0=0.08),
    # the paper's scaling parameter
    "paper_lambda": dict(n=(44, 40, 36), cpml=(10,) * 6, lam=0.05, nt=300, src=(22, 20, 18), f0=0.2),
}


@pytest.mark.parametrize("variant", [1, 2])
@pytest.mark.parametrize("name", sorted(CASES))
def test_pv_matches_oracle(name, variant):
    c = CASES[name]
    rng = np.random.default_rng(7)
    n = c["n"]
    rec = np.stack([rng.integers(0, n[0], 12), rng.integers(0, n[1], 12), rng.integers(0, n[2], 12)], 1)
    rec = rec.astype(np.int32)
    wav = synth.ricker(c["nt"], c["lam"], c["f0"])         # time in units of h / c (wavelength 1 / f0 cells)
    ref = P.forward(n, c["cpml"], c["lam"], c["nt"], c["src"], wav, rec, snap_every=30)
    tr, snaps, p = _gpu(n, c["cpml"], c["lam"], c["nt"], c["src"], wav, rec, snap_every=30, variant=variant)
    e_tr, e_st, e_p = rel_l2(tr, ref["traces"]), rel_l2(snaps, ref["snaps"]), rel_l2(p, ref["p"])
    print("%s/%d: traces %.3e  snapshots %.3e  final p %.3e" % (name, variant, e_tr, e_st, e_p), flush=True)
    assert e_tr <= 1e-5 and e_st <= 1e-5 and e_p <= 1e-5


def test_pv_corner_source_and_receivers():
    """Source one node from a corner, inside the layers of all three axes;
    receivers on the grid's corners and faces; both variants."""
    n = (33, 29, 27)
    rec = np.array([[0, 0, 0], [32, 28, 26], [0, 28, 0], [32, 0, 26], [16, 0, 13], [16, 14, 0], [32, 14, 13],
                    [1, 1, 1], [5, 5, 5]], np.int32)
    wav = synth.ricker(90, 0.3, 0.1)
    ref = P.forward(n, (4,) * 6, 0.3, 90, (1, 1, 1), wav, rec, snap_every=30)
    for variant in (1, 2):
        tr, snaps, p = _gpu(n, (4,) * 6, 0.3, 90, (1, 1, 1), wav, rec, snap_every=30, variant=variant)
        assert rel_l2(tr, ref["traces"]) <= 1e-5 and rel_l2(snaps, ref["snaps"]) <= 1e-5, variant


@pytest.mark.parametrize("n,cpml", [((70, 45, 38), (5, 7, 3, 6, 8, 4)),     # ragged x, y tiles; two z chunks
                                    ((33, 29, 97), (0, 9, 6, 0, 0, 7)),     # one partial x tile; 4 z chunks
                                    ((130, 17, 31), (12, 12, 0, 0, 6, 6))])  # three x tiles, one y tile
def test_pv_variants_bitwise(n, cpml):
    """The z-marching stages sum every tap in the order of the one-thread-per-
    point stages, so both give the same bits (traces, snapshots, final p)."""
    rng = np.random.default_rng(11)
    rec = np.stack([rng.integers(0, n[0], 10), rng.integers(0, n[1], 10), rng.integers(0, n[2], 10)], 1)
    wav = synth.ricker(100, 0.3, 0.08)
    src = (n[0] // 3, n[1] // 2, n[2] // 2)
    a = _gpu(n, cpml, 0.3, 100, src, wav, rec.astype(np.int32), snap_every=25, variant=1)
    b = _gpu(n, cpml, 0.3, 100, src, wav, rec.astype(np.int32), snap_every=25, variant=2)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_pv_initial_pressure_matches_oracle():
    """Initial pulse, no source: set_pressure and the free evolution."""
    n = (36, 34, 30)
    x, y, z = _coords(n)
    p0 = np.exp(-((x - 14.2) ** 2 + (y - 17.5) ** 2 + (z - 12.3) ** 2) / 8.0)
    ref = P.forward(n, (0, 8, 6, 0, 0, 5), 0.3, 80, p0=p0, snap_every=20)
    _, snaps, p = _gpu(n, (0, 8, 6, 0, 0, 5), 0.3, 80, p0=p0, snap_every=20)
    assert rel_l2(snaps, ref["snaps"]) <= 1e-5 and rel_l2(p, ref["p"]) <= 1e-5


@pytest.mark.parametrize("N,variant", [(320, 1), (320, 2), (544, 0)])
def test_pv_paper_grid_mirror_symmetry(N, variant):
    """Paper grids (20-cell layers, lambda = 0.05, 64 steps) in the launch
    configuration the benchmark times (544^3: the automatic choice is the
    z-march), and 320^3 with both variants."""
    import torch

    from paper_2606_06910_amd import PVPropagator

    s = PVPropagator((N, N, N), (20,) * 6, 0.05, variant=variant)
    g = torch.arange(N, device="cuda", dtype=torch.float32) - (N - 1) / 2.0
    s.set_pressure(torch.exp(-(g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2) / 30.0))
    s.step(64)
    p = s.get_pressure()
    torch.cuda.synchronize()
    s.close()
    assert float(p.abs().max()) > 1e-3
    for ax in range(3):
        assert torch.equal(p, torch.flip(p, dims=(ax,))), ax
