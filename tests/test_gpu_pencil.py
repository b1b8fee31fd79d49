"""One GPU's pencil-yz share: ghost faces on +-y and +-z filled by the on-device
pack/unpack loopback (the opposite face: y and z periodic), CPML only on the
physical +-x faces.

Bar (written here): with ghost depth 4 s exchanged every s steps, s = 2 and
s = 4 give the s = 1 bits exactly (the paper's enlarged-ghost correctness
table reports zero difference); s = 1 matches the oracle with periodic y, z
to relative L2 <= 1e-5 on traces and space-time snapshots.
"""
import numpy as np
import pytest

import synth
from helpers import rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def _pencil(n, nt, seed=1002, L=10):
    w = synth.pencil(nt=nt, seed=seed, n_xyz=n, L=L)
    rng = np.random.default_rng(seed + 7)
    nx, ny, nz = n
    # receivers anywhere, including rows next to the periodic seams
    rec = np.stack([rng.integers(0, nx, 16), rng.integers(0, ny, 16), rng.integers(0, nz, 16)], 1)
    rec[:4, 1] = [0, 1, ny - 1, ny - 2]
    rec[4:8, 2] = [0, 2, nz - 1, nz - 3]
    w.rec = rec.astype(np.int32)
    # source near a seam so waves cross it
    w.src = np.array([[nx // 2, 3, nz - 4]], np.int32)
    return w


@pytest.fixture(scope="module")
def small_pencil():
    w = _pencil((96, 40, 48), 60)
    print("oracle: periodic pencil %s" % (w.n,), flush=True)
    return w, run_oracle(w, snap_every=10)


def test_pencil_s1_matches_periodic_oracle(small_pencil):
    w, ref = small_pencil
    tr, snaps, _ = run_gpu(w, snap_every=10, exchange_every=1)
    assert rel_l2(tr, ref["traces"]) <= 1e-5
    assert rel_l2(snaps, ref["snaps"]) <= 1e-5


@pytest.mark.parametrize("s", [2, 4])
def test_enlarged_ghosts_bitwise_equal(small_pencil, s):
    w, _ = small_pencil
    a = run_gpu(w, snap_every=4, exchange_every=1)
    b = run_gpu(w, snap_every=4, exchange_every=s)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


def test_pencil_fp16_matches_periodic_oracle(small_pencil):
    """16-bit storage through the exchange (2-byte elements), at the 16-bit
    storage bar on the space-time snapshots (measured 3.5e-4).  A wrong ghost
    would put O(1) errors on the waves crossing the seams.  The traces of this
    short run mostly hold first arrivals, where 16-bit storage is least
    accurate: 2.7e-2 here and 3.2e-2 on the same grid with Dirichlet y and z
    faces, so that error is the storage's, not the exchange's; they are held
    to 1e-1."""
    w, ref = small_pencil
    tr, snaps, _ = run_gpu(w, snap_every=10, exchange_every=1, storage=1)
    e_tr, e_st = rel_l2(tr, ref["traces"]), rel_l2(snaps, ref["snaps"])
    print("FP16 pencil: traces %.3e  space-time %.3e" % (e_tr, e_st), flush=True)
    assert e_st <= 1e-2
    assert e_tr <= 1e-1


@pytest.mark.parametrize("s", [2, 4])
def test_enlarged_ghosts_bitwise_equal_fp16(small_pencil, s):
    w, _ = small_pencil
    a = run_gpu(w, snap_every=4, exchange_every=1, storage=1)
    b = run_gpu(w, snap_every=4, exchange_every=s, storage=1)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])


@pytest.mark.parametrize("s", [2, 4])
def test_enlarged_ghosts_naive_variant(small_pencil, s):
    """The naive kernel handles the extended ghost boxes the same way."""
    w, _ = small_pencil
    a = run_gpu(w, nt=20, exchange_every=1, variant=2)
    b = run_gpu(w, nt=20, exchange_every=s, variant=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_full_pencil_shape_s4_equals_s1():
    """Full 1024 x 384 x 384 share, 20-cell layers on +-x, 24 steps."""
    w = _pencil((1024, 384, 384), 24, L=20)
    a = run_gpu(w, exchange_every=1)
    b = run_gpu(w, exchange_every=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])
