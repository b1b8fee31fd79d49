"""GPU parity at the full workload sizes with signal in every layer.

A run from a point source at the centre of a 512^3 grid never reaches the
absorbing layers within the few steps the oracle can afford there, so here
both time levels start from a seeded random field over the whole grid,
layers included.  Every band point then carries signal from the first step,
and the layer memory (psi, zeta) is exercised at the full-size strides, plane
counts and launch configuration of the timed runs (default plan).

Bar (written here): after the stated steps, relative L2 <= 1e-5 against the
FP64 oracle on the whole field, on the band points alone (layer plus the
4-cell margin whose stencils read layer memory) and on the band of each of
the six faces separately, for u^n and u^{n-1}; the pencil share with ghost
faces at s = 1 and s = 4 against the oracle with periodic y and z, and s = 4
bit-equal to s = 1.  Temporal blocking is held bit-equal to the z-march from
the same state.
"""
import numpy as np
import pytest

import synth
from helpers import band_masks, rel_l2
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _state(shape_zyx, seed):
    """Two seeded time levels: white noise (every wavenumber present, so the
    layer terms are O(1) parts of each update) over the whole grid."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=shape_zyx).astype(np.float32)
    um1 = (0.5 * u + 0.5 * rng.uniform(-1.0, 1.0, size=shape_zyx)).astype(np.float32)
    return u, um1


def _run_gpu_state(n, h, dt, cpml, v, u0, um1, nt, plan=None, **shot_kw):
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    p = Propagator([Shot(n=n, h=h, dt=dt, cpml=cpml, **shot_kw)])
    if plan is not None:
        p.set_plan(0, *plan)
    p.set_velocity(0, torch.from_numpy(v.astype(np.float32)).cuda())
    p.set_field(0, 0, torch.from_numpy(u0).cuda())
    p.set_field(0, 1, torch.from_numpy(um1).cuda())
    plan = p.plan(0)
    p.step(nt)
    un = p.get_field(0, 0).cpu().numpy()
    unm1 = p.get_field(0, 1).cpu().numpy()
    p.close()
    return un, unm1, plan


def _run_oracle_state(n, h, dt, cpml, v, u0, um1, nt, periodic=(0, 0, 0)):
    vv = v.astype(np.float32).astype(np.float64)
    g = O.Grid(n=n, h=h, dt=dt, cpml=cpml, periodic=periodic, vref=float(vv.max()))
    st = O.State.zeros(g)
    st.u[...] = u0
    st.um1[...] = um1
    out = O.forward(g, vv, nt, state=st)
    return out["state"].u, out["state"].um1


def _check(name, got, ref, masks, union):
    errs = {"all": rel_l2(got, ref), "band": rel_l2(got[union], ref[union]),
            "inner": rel_l2(got[~union], ref[~union])}
    for k, m in masks.items():
        errs[k] = rel_l2(got[m], ref[m])
    print("%s: %s" % (name, "  ".join("%s %.2e" % kv for kv in errs.items())), flush=True)
    for k, e in errs.items():
        assert e <= TOL, (name, k, e)


def test_layered512_state_in_layers_matches_oracle():
    """512^3, 20-cell layers on every face, default plan (z-march, band kernel
    advancing psi_x and psi_z, psi_y pass), 6 steps from a noise state."""
    w = synth.layered(n_xyz=(512, 512, 512), nt=6)
    u0, um1 = _state(w.v.shape, 2024)
    nt = 6
    print("layered512: GPU, %d steps from a noise state" % nt, flush=True)
    un, unm1, plan = _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, nt)
    assert plan[0] == 2, plan          # the z-march path the timed runs use
    print("layered512: oracle", flush=True)
    ru, rum1 = _run_oracle_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, nt)
    masks, union = band_masks(w.n, w.cpml)
    _check("512^3 u^n", un, ru, masks, union)
    _check("512^3 u^{n-1}", unm1, rum1, masks, union)


@pytest.fixture(scope="module")
def pencil_case():
    """The 1024 x 384 x 384 pencil share (layers on +-x only; y and z are
    ghost faces filled by the loopback exchange), 8 steps from a noise state,
    and the periodic-y/z oracle run."""
    w = synth.pencil(nt=8)
    u0, um1 = _state(w.v.shape, 2025)
    print("pencil: oracle (periodic y, z), 8 steps", flush=True)
    ref = _run_oracle_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8, periodic=(0, 1, 1))
    return w, u0, um1, ref


@pytest.fixture(scope="module")
def pencil_s1(pencil_case):
    w, u0, um1, _ = pencil_case
    return _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8, face=(0, 0, 1, 1, 1, 1), exchange_every=1)


@pytest.mark.parametrize("s", [1, 4])
def test_pencil_state_in_layers_matches_periodic_oracle(pencil_case, pencil_s1, s):
    w, u0, um1, (ru, rum1) = pencil_case
    if s == 1:
        un, unm1, _ = pencil_s1
    else:
        un, unm1, _ = _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8, face=(0, 0, 1, 1, 1, 1),
                                     exchange_every=s)
        assert np.array_equal(un, pencil_s1[0]) and np.array_equal(unm1, pencil_s1[1]), "s=%d vs s=1" % s
    masks, union = band_masks(w.n, w.cpml)
    _check("pencil s=%d u^n" % s, un, ru, masks, union)
    _check("pencil s=%d u^{n-1}" % s, unm1, rum1, masks, union)


def test_two_column_plan_full_size_state_in_layers():
    """The two-column z-march (128-wide tiles) at 512^3 from a noise state:
    the default plan's bits after 8 steps."""
    w = synth.layered(n_xyz=(512, 512, 512), nt=8)
    u0, um1 = _state(w.v.shape, 2027)
    a = _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8)
    b = _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8, plan=(2, 2, 4096, 1, 2))
    assert b[2][3] == 2 and a[2][3] == 1, (a[2], b[2])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("K", [2, 4])
def test_tblock_full_size_state_in_layers(K):
    """Temporal blocking at 512^3 from a noise state (the shell carries signal
    at every level): the z-march's bits after 8 steps."""
    w = synth.layered(n_xyz=(512, 512, 512), nt=8)
    u0, um1 = _state(w.v.shape, 2026)
    a = _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8, variant=2)
    b = _run_gpu_state(w.n, w.h, w.dt, w.cpml, w.v, u0, um1, 8, variant=3, tblock_k=K)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
