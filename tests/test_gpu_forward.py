"""GPU parity of the forward hot path against the FP64 oracle (through the C ABI).

Bar (written here): FP32 fields match the oracle to relative L2 <= 1e-5 on
receiver traces and on space-time snapshots (all snapshot samples taken
together); the final field alone is ill-conditioned once the wave has been
absorbed, so it is only used while still energetic.  Kernel variants with the
same per-point arithmetic must agree bit for bit.
"""
import numpy as np
import pytest

import synth
from helpers import band_masks, per_receiver_rel_l2, rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5
NAIVE, ZMARCH = 1, 2


@pytest.fixture(scope="module")
def plain64_ref():
    w = synth.plain64()
    print("oracle: plain64 64^3 x %d steps" % w.nt, flush=True)
    return w, run_oracle(w, snap_every=10)


@pytest.mark.parametrize("variant", [NAIVE, ZMARCH])
def test_plain64_matches_oracle(plain64_ref, variant):
    w, ref = plain64_ref
    tr, snaps, fin = run_gpu(w, snap_every=10, variant=variant)
    e_tr = rel_l2(tr, ref["traces"])
    e_st = rel_l2(snaps, ref["snaps"])
    _, union = band_masks(w.n, w.cpml)
    e_band = rel_l2(snaps[:, union], ref["snaps"][:, union])
    per = per_receiver_rel_l2(tr, ref["traces"])
    print("plain64 variant %d: traces %.3e  space-time %.3e  band %.3e  per-receiver max %.3e over %d" %
          (variant, e_tr, e_st, e_band, per.max(), per.size), flush=True)
    assert e_tr <= TOL
    assert e_st <= TOL
    assert e_band <= TOL
    assert per.max() <= TOL


def test_plain64_variants_bitwise(plain64_ref):
    w, _ = plain64_ref
    a = run_gpu(w, snap_every=10, variant=NAIVE)
    b = run_gpu(w, snap_every=10, variant=ZMARCH)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def _ragged(n, h, cpml, nt, seed, nrec=12, src=None):
    """Random model; receivers within 6 cells of the source (so that every
    trace carries signal within the short runs) plus two anywhere."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    v = 1800.0 + 800.0 * rng.uniform(size=(nz, ny, nx))
    dt = synth.dt_from_courant(v.max(), h) * 0.9
    if src is None:
        src = (nx // 3, ny // 2 + 1, nz // 2 - 1)
    near = np.array(src)[None, :] + rng.integers(-6, 7, size=(nrec - 2, 3))
    far = np.stack([rng.integers(0, nx, 2), rng.integers(0, ny, 2), rng.integers(0, nz, 2)], 1)
    rec = np.clip(np.concatenate([near, far]), 0, np.array(n) - 1)
    return synth.Workload("ragged", tuple(n), tuple(h), dt, nt, tuple(cpml), v,
                          np.array([src], np.int32), synth.ricker(nt, dt, 30.0), rec.astype(np.int32))


CASES = {
    # several x/y tiles with a ragged tail, uneven layers, uneven spacing
    "ragged": dict(n=(70, 45, 38), h=(10.0, 12.0, 9.0), cpml=(5, 7, 3, 6, 8, 4), nt=80, seed=1),
    # several z chunks and y tiles, source inside a layer band
    "zchunks": dict(n=(100, 70, 150), h=(10.0, 10.0, 10.0), cpml=(10, 10, 10, 10, 10, 10), nt=40, seed=2,
                    src=(6, 35, 75)),
    # no absorbing layer at all (pure Dirichlet box)
    "nolayer": dict(n=(33, 29, 41), h=(8.0, 8.0, 8.0), cpml=(0,) * 6, nt=60, seed=3),
    # layers on some faces only
    "someface": dict(n=(48, 40, 36), h=(10.0, 10.0, 10.0), cpml=(0, 9, 6, 0, 0, 7), nt=60, seed=4),
    # smallest grid the stencil allows, with the widest layer it allows
    "tiny": dict(n=(9, 9, 9), h=(10.0, 10.0, 10.0), cpml=(4,) * 6, nt=30, seed=5, src=(4, 4, 4)),
    # x layers wider than a band tile row (28 + 4 > 32 on the low face): the band
    # kernel reads psi_x from the psi pass instead of advancing it itself
    "widex": dict(n=(80, 36, 40), h=(10.0, 10.0, 10.0), cpml=(30, 12, 5, 4, 6, 5), nt=50, seed=6),
    # z layers whose bands read each other's layer points (nz < Llo + Lhi + 8)
    "nearz": dict(n=(40, 30, 20), h=(10.0, 10.0, 10.0), cpml=(5, 6, 4, 4, 6, 7), nt=50, seed=7, src=(20, 15, 10)),
    # high x band straddling a 32-column boundary (its own tile row), x-only layers
    "xcut": dict(n=(75, 33, 30), h=(10.0, 10.0, 10.0), cpml=(9, 13, 0, 0, 0, 0), nt=60, seed=8),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_cases_match_oracle_and_variants_agree(name):
    c = dict(CASES[name])
    w = _ragged(c.pop("n"), c.pop("h"), c.pop("cpml"), c.pop("nt"), c.pop("seed"), src=c.pop("src", None))
    print("case %s n=%s" % (name, w.n), flush=True)
    ref = run_oracle(w, snap_every=10)
    z = run_gpu(w, snap_every=10, variant=ZMARCH)
    n = run_gpu(w, snap_every=10, variant=NAIVE)
    assert rel_l2(z[0], ref["traces"]) <= TOL
    assert rel_l2(z[1], ref["snaps"]) <= TOL
    # beside the global norms: each receiver that the wave has reached, and the
    # snapshot samples on the band points alone (the layers hold a small share
    # of the norm, so an error there could hide in the global figure)
    per = per_receiver_rel_l2(z[0], ref["traces"])
    msg = "case %s: per-receiver max %.2e over %d" % (name, per.max(), per.size)
    _, union = band_masks(w.n, w.cpml)
    if union.any():
        e_band = rel_l2(z[1][:, union], ref["snaps"][:, union])
        msg += "  band snapshots %.2e" % e_band
        assert e_band <= TOL, (name, e_band)
    print(msg, flush=True)
    assert per.max() <= TOL, (name, per.max())
    assert np.array_equal(z[0], n[0]) and np.array_equal(z[1], n[1]) and np.array_equal(z[2], n[2])


@pytest.mark.parametrize("ry,zc,cols", [(1, 16, 1), (2, 32, 1), (4, 64, 1), (1, 128, 1), (4, 16, 1), (2, 4096, 1),
                                        (8, 32, 1), (8, 4096, 1), (1, 16, 2), (2, 32, 2), (4, 64, 2), (2, 4096, 2),
                                        (1, 4096, 2)])
def test_zmarch_plans_bitwise_equal_naive(ry, zc, cols):
    """Every tile shape (64 or 128 wide: one or two x points per lane) and
    z-chunk plan gives the naive kernel's bits (several x/y tiles with ragged
    tails, several z chunks, source inside a layer)."""
    w = _ragged((100, 70, 150), (10.0, 10.0, 10.0), (10,) * 6, 30, 2, src=(6, 35, 75))
    a = run_gpu(w, variant=NAIVE)
    b = run_gpu(w, plan=(ZMARCH, ry, zc, 1, cols))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_variant_switched_by_plan():
    """A context created for one variant and switched to the other by
    fdtd_set_plan (naive <-> z-march: whether the band kernel advances the x
    and z layer memory itself changes with it) gives that variant's bits."""
    w = _ragged((70, 45, 38), (10.0, 12.0, 9.0), (5, 7, 3, 6, 8, 4), 40, 1)
    naive = run_gpu(w, variant=NAIVE)
    zm = run_gpu(w, variant=ZMARCH)
    to_naive = run_gpu(w, variant=ZMARCH, plan=(NAIVE, 2, 64, 1, 1))
    to_zm = run_gpu(w, variant=NAIVE, plan=(ZMARCH, 4, 64, 1, 1))
    for got in (to_naive, to_zm):
        assert np.array_equal(got[0], naive[0]) and np.array_equal(got[2], naive[2])
    assert np.array_equal(zm[2], naive[2])


@pytest.mark.parametrize("storage", [1, 2])
@pytest.mark.parametrize("name", ["ragged", "xcut", "zchunks"])
def test_two_column_plan_16bit_bitwise(storage, name):
    """16-bit storage: the two-column z-march (4-byte pair loads) gives the
    one-column kernel's bits."""
    c = dict(CASES[name])
    w = _ragged(c.pop("n"), c.pop("h"), c.pop("cpml"), c.pop("nt"), c.pop("seed"), src=c.pop("src", None))
    a = run_gpu(w, plan=(ZMARCH, 2, 64, 1, 1), storage=storage)
    b = run_gpu(w, plan=(ZMARCH, 2, 64, 1, 2), storage=storage)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_graph_replay_matches_eager():
    """A captured time loop, replayed from reset several times, gives the
    eager bits every time."""
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    w = _ragged((40, 36, 44), (10.0, 10.0, 10.0), (6,) * 6, 50, 7)
    eager = run_gpu(w, variant=ZMARCH)
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, variant=2)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)))
    p.set_receivers(0, w.rec)
    tr = p.record(0, w.nt)
    for rep in range(3):
        p.reset()
        tr.zero_()
        p.step(w.nt, graph=True)
        torch.cuda.synchronize()
        assert np.array_equal(tr.cpu().double().numpy(), eager[0]), rep
        assert np.array_equal(p.get_field(0).cpu().double().numpy(), eager[2]), rep
        _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
    p.close()


def test_run_twice_is_deterministic():
    w = _ragged((50, 40, 30), (10.0, 10.0, 10.0), (5,) * 6, 40, 8)
    a = run_gpu(w, variant=ZMARCH)
    b = run_gpu(w, variant=ZMARCH)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_error_paths():
    import torch

    from paper_2606_06910_amd import FDTDError, FDTDValueError, Propagator, Shot

    w = _ragged((24, 24, 24), (10.0, 10.0, 10.0), (4,) * 6, 10, 9)
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml)])
    with pytest.raises(FDTDError):        # no velocity yet
        p.step(1)
    with pytest.raises(FDTDValueError):   # non-positive velocity
        p.set_velocity(0, torch.zeros(w.v.shape, device="cuda"))
    with pytest.raises(FDTDValueError):   # receiver outside the grid
        p.set_receivers(0, [[0, 0, 24]])
    with pytest.raises(FDTDValueError):   # source outside the grid
        p.inject_source(0, (-1, 0, 0), torch.ones(10))
    p.close()
    unstable = Shot(n=w.n, h=w.h, dt=2.1 * 10.0 / (2600.0 * np.sqrt(3 * 6.50159)), cpml=w.cpml)
    q = Propagator([unstable])
    with pytest.raises(FDTDValueError, match="EUNSTABLE"):
        q.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    q.close()


@pytest.mark.parametrize("graph", [False, True])
def test_nan_sentinel(graph):
    """A NaN set into u^n from the host: stepping on without the sentinel raises
    nothing; with a scan every 5 steps the next call that scans reports
    ENONFINITE (eager: after the scan step; graph: after the launch); after
    fdtd_reset the flag is clear and a clean run steps on."""
    import torch

    from paper_2606_06910_amd import FDTDError, Propagator, Shot

    w = _ragged((24, 24, 24), (10.0, 10.0, 10.0), (4,) * 6, 10, 9)
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.step(3)
    f = torch.zeros(w.v.shape, device="cuda")
    f[12, 12, 12] = float("nan")
    p.set_field(0, 0, f)
    p.step(4, graph=graph)            # sentinel off
    p.set_sentinel(5)
    p.step(2, graph=False)            # steps 8, 9: no scan yet
    with pytest.raises(FDTDError, match="ENONFINITE"):
        p.step(5, graph=graph)
    p.reset()
    p.set_sentinel(5)
    p.step(10, graph=graph)
    p.close()


@pytest.mark.parametrize("n", [(512, 512, 512)])
def test_full_size_variants_bitwise_and_crop_oracle(n):
    """Full layered 512^3 shape, 50 steps: naive and z-march agree bit for bit;
    near the source (wave still far from every face) the traces match the
    oracle run on a crop of the same model."""
    import torch

    w = synth.layered(n_xyz=n, nt=50)
    a = run_gpu(w, variant=ZMARCH)
    b = run_gpu(w, variant=NAIVE)
    assert np.array_equal(a[2], b[2])
    # crop: 72^3 box around the source, same model values, zero Dirichlet faces
    c = 36
    sx, sy, sz = [int(x) for x in w.src[0]]
    crop_v = w.v[sz - c:sz + c, sy - c:sy + c, sx - c:sx + c]
    rng = np.random.default_rng(3)
    rec = np.stack([c + rng.integers(-8, 9, 12), c + rng.integers(-8, 9, 12), c + rng.integers(-8, 9, 12)], 1)
    wc = synth.Workload("crop", (2 * c,) * 3, w.h, w.dt, w.nt, (0,) * 6, crop_v, np.array([[c, c, c]], np.int32),
                        w.wavelet, rec.astype(np.int32))
    from oracle import oracle as O

    g = O.Grid(n=wc.n, h=wc.h, dt=wc.dt, cpml=(0,) * 6, vref=1.0)
    ref = O.forward(g, crop_v.astype(np.float32).astype(np.float64), w.nt, wc.src, wc.wavelet, wc.rec)
    full_rec = rec + np.array([sx - c, sy - c, sz - c])
    w2 = synth.Workload("full", w.n, w.h, w.dt, w.nt, w.cpml, w.v, w.src, w.wavelet, full_rec.astype(np.int32))
    tr = run_gpu(w2, variant=ZMARCH)[0]
    assert rel_l2(tr, ref["traces"]) <= TOL
