"""Temporal blocking: K = 2 and K = 4 leapfrog steps per interior launch
(the shell outside each shrinking interior box advanced level by level).

Bar (written here): bit-for-bit equal to the single-step z-march kernel
(same per-point arithmetic), for step counts that are and are not multiples
of K, eagerly and from a captured graph, with receivers inside and outside
the interior box and the source inside it; and therefore within the forward
tolerance of the oracle (checked once here as well).
"""
import numpy as np
import pytest

import synth
from helpers import rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

ZMARCH, TBLOCK = 2, 3


def _case(n=(96, 88, 80), L=10, nt=30, seed=31):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    v = synth.layered_model((nz, ny, nx), rng, nlayers=(4, 6), smooth_sigma=2.0)
    dt = synth.dt_from_courant(v.max(), (10.0,) * 3)
    src = np.array([[nx // 2 + 1, ny // 2 - 2, nz // 2 + 3]], np.int32)
    near = src + rng.integers(-7, 8, size=(10, 3))
    shell = np.array([[2, ny // 2, nz // 2], [nx // 2, 3, nz // 2], [nx // 2, ny // 2, nz - 3], [15, 16, 17]])
    rec = np.clip(np.concatenate([near, shell]), 0, np.array(n) - 1).astype(np.int32)
    return synth.Workload("tb", tuple(n), (10.0,) * 3, dt, nt, (L,) * 6, v, src,
                          synth.ricker(nt, dt, 30.0), rec)


@pytest.mark.parametrize("K", [2, 4])
@pytest.mark.parametrize("nt", [24, 31])
@pytest.mark.parametrize("graph", [False, True])
def test_tblock_bitwise_equals_zmarch(K, nt, graph):
    w = _case(nt=nt)
    a = run_gpu(w, variant=ZMARCH)
    b = run_gpu(w, variant=TBLOCK, tblock_k=K, graph=graph)
    assert np.array_equal(a[0], b[0]), "traces"
    assert np.array_equal(a[2], b[2]), "final field"


@pytest.mark.parametrize("K", [2, 4])
def test_tblock_matches_oracle(K):
    w = _case(nt=40)
    ref = run_oracle(w, snap_every=8)
    tr, snaps, _ = run_gpu(w, snap_every=8, variant=TBLOCK, tblock_k=K)
    assert rel_l2(tr, ref["traces"]) <= 1e-5
    assert rel_l2(snaps, ref["snaps"]) <= 1e-5


def test_tblock_without_layers_and_small_interior():
    """No layers (B is the whole grid) and a grid whose interior box is too small
    for K = 4 tiles (then every step is a single step)."""
    for n, L in (((72, 64, 56), 0), ((48, 44, 40), 12)):
        w = _case(n=n, L=L, nt=20)
        a = run_gpu(w, variant=ZMARCH)
        b = run_gpu(w, variant=TBLOCK, tblock_k=4)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2]), n


def test_tblock_full_size():
    w = synth.layered(n_xyz=(512, 512, 512), nt=12)
    a = run_gpu(w, variant=ZMARCH)
    b = run_gpu(w, variant=TBLOCK, tblock_k=2)
    assert np.array_equal(a[2], b[2])
