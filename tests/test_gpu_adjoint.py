"""GPU adjoint and velocity gradient against the FP64 oracle (through the C ABI).

Bar (written here): GPU gradient vs the oracle's gradient, relative L2 <= 1e-4
(FP32 fields, FP64 accumulation); the checkpoint interval does not change the
result (bitwise: segment recomputation replays identical forward bits).
"""
import numpy as np
import pytest

import synth
from helpers import oracle_grid, rel_l2, v32

pytestmark = pytest.mark.gpu


def _problem(n=(40, 36, 32), L=6, nt=120, seed=21, nrec=10, cpml=None):
    rng = np.random.default_rng(seed)
    cpml = (L,) * 6 if cpml is None else tuple(cpml)
    nx, ny, nz = n
    vt = synth.layered_model((nz, ny, nx), rng, nlayers=(3, 5), smooth_sigma=2.0)
    v0 = vt * (1.0 + 0.03 * synth.smooth_field((nz, ny, nx), rng, sigma=3.0))
    dt = synth.dt_from_courant(max(vt.max(), v0.max()), (10.0,) * 3)
    rec = synth.receivers_on_plane(n, L, nrec, rng)
    src = np.array([[nx // 2, ny // 2, nz // 2]], np.int32)
    w = synth.Workload("adj", tuple(n), (10.0,) * 3, dt, nt, cpml, v0, src, synth.ricker(nt, dt, 25.0), rec)
    return w, vt


def _gpu_grad(w, dobs, every, storage=0):
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    vref = float(v32(w).max())
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, v_ref=vref, storage=storage, variant=2)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)))
    p.set_receivers(0, w.rec)
    p.set_checkpointing(0, every, w.nt)
    tr = p.record(0, w.nt)
    p.step(w.nt)
    torch.cuda.synchronize()
    d = tr.cpu().double().numpy()
    resid = torch.from_numpy((d - dobs).astype(np.float32))
    g = p.adjoint(0, w.nt, resid).cpu().numpy()
    p.close()
    return d, g


@pytest.fixture(scope="module")
def adj_case():
    from oracle import oracle as O

    w, vt = _problem()
    g = oracle_grid(w)
    wt = synth.Workload("t", w.n, w.h, w.dt, w.nt, w.cpml, vt, w.src, w.wavelet, w.rec)
    dobs = O.forward(g, v32(wt), w.nt, w.src, w.wavelet, w.rec)["traces"]
    fwd = O.forward(g, v32(w), w.nt, w.src, w.wavelet, w.rec, keep_lapf=True)
    gref = O.gradient(g, v32(w), w.nt, w.src, w.wavelet, w.rec, fwd["traces"] - dobs, fwd=fwd)
    return w, dobs, fwd["traces"], gref


def test_gradient_matches_oracle(adj_case):
    w, dobs, tr_ref, gref = adj_case
    d, g = _gpu_grad(w, dobs, every=25)
    assert rel_l2(d, tr_ref) <= 1e-5
    e = rel_l2(g, gref)
    print("gradient rel-L2 vs oracle: %.3e" % e, flush=True)
    assert e <= 1e-4


def test_gradient_independent_of_checkpoint_interval(adj_case):
    # the interval also sets the gradient pass's step count G (<= 16, a segment
    # split evenly) and the mu ring of G + 1 levels: 1 -> a ring of 2 (pass 3
    # writes mu^n where it read mu^{n+2}), 2 -> 3, 7 -> 8, 17 -> two passes of 9
    # and 8 steps, 25 -> 13 and 12, 120 -> 15
    w, dobs, _, _ = adj_case
    _, g1 = _gpu_grad(w, dobs, every=25)
    for every in (1, 2, 7, 17, 120):
        _, g2 = _gpu_grad(w, dobs, every=every)
        assert np.array_equal(g1, g2), every


def test_shorter_sweep_keeps_the_later_checkpoints(adj_case):
    """A sweep over the first segment only, before the full one, leaves the full
    gradient bit for bit as it is alone: a short sweep places nothing over the
    checkpoints it does not use."""
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    w, dobs, _, _ = adj_case
    _, g_alone = _gpu_grad(w, dobs, every=25)
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, v_ref=float(v32(w).max()), variant=2)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)))
    p.set_receivers(0, w.rec)
    p.set_checkpointing(0, 25, w.nt)
    tr = p.record(0, w.nt)
    p.step(w.nt)
    torch.cuda.synchronize()
    resid = torch.from_numpy((tr.cpu().double().numpy() - dobs).astype(np.float32))
    p.adjoint(0, 25, resid[:25].contiguous())
    g = p.adjoint(0, w.nt, resid).cpu().numpy()
    p.close()
    assert np.array_equal(g, g_alone)


def test_autograd_function(adj_case):
    import torch

    from paper_2606_06910_amd import Shot
    from paper_2606_06910_amd.autograd import simulate

    w, dobs, _, gref = adj_case
    v = torch.from_numpy(w.v.astype(np.float32)).cuda().requires_grad_(True)
    shot = Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, v_ref=float(v32(w).max()), variant=2)
    tr = simulate(v, shot, torch.from_numpy(w.wavelet.astype(np.float32)), w.src[0], w.rec, w.nt, every=25)
    J = 0.5 * ((tr.double() - torch.from_numpy(dobs).cuda()) ** 2).sum()
    J.backward()
    assert rel_l2(v.grad.double().cpu().numpy(), gref) <= 1e-4


def test_gradient_wide_uneven_layers():
    """Several 64-point x tiles, of which the middle ones do not meet the x
    band, layers of different widths on each face and faces without layers."""
    from oracle import oracle as O

    w, vt = _problem(n=(150, 26, 24), L=5, nt=160, seed=23, nrec=8, cpml=(7, 5, 0, 6, 4, 0))
    # source beside the low x layer; receivers inside the x, y and z layers and in the open,
    # so that each band holds a large part of the gradient (about half of its norm or more)
    src = np.array([[14, 13, 12]], np.int32)
    rec = np.array([[3, 13, 12], [5, 22, 12], [8, 13, 2], [40, 4, 12], [60, 13, 20], [100, 13, 12],
                    [146, 13, 12], [14, 24, 1]], np.int32)
    w = synth.Workload("adj", w.n, w.h, w.dt, w.nt, w.cpml, w.v, src, w.wavelet, rec)
    g = oracle_grid(w)
    wt = synth.Workload("t", w.n, w.h, w.dt, w.nt, w.cpml, vt, w.src, w.wavelet, w.rec)
    dobs = O.forward(g, v32(wt), w.nt, w.src, w.wavelet, w.rec)["traces"]
    fwd = O.forward(g, v32(w), w.nt, w.src, w.wavelet, w.rec, keep_lapf=True)
    gref = O.gradient(g, v32(w), w.nt, w.src, w.wavelet, w.rec, fwd["traces"] - dobs, fwd=fwd)
    d, gg = _gpu_grad(w, dobs, every=16)
    assert rel_l2(d, fwd["traces"]) <= 1e-5
    e = rel_l2(gg, gref)
    print("gradient rel-L2 vs oracle (wide, uneven layers): %.3e" % e, flush=True)
    assert e <= 1e-4
    # the same bar on each axis's band (layer plus 4 cells) on its own
    z, y, x = np.meshgrid(np.arange(24), np.arange(26), np.arange(150), indexing="ij")
    for name, m in (("x", (x < 7 + 4) | (x >= 150 - 5 - 4)), ("y", y >= 26 - 6 - 4), ("z", z < 4 + 4)):
        eb = rel_l2(gg[m], gref[m])
        print("  %s band: %.3e" % (name, eb), flush=True)
        assert eb <= 1e-4


def test_adjoint_state_errors():
    import torch

    from paper_2606_06910_amd import FDTDError, Propagator, Shot

    w, _ = _problem(n=(20, 20, 20), L=4, nt=10)
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.set_receivers(0, w.rec)
    with pytest.raises(FDTDError):          # no checkpointing registered
        p.adjoint(0, 10, torch.zeros(10, len(w.rec)))
    p.set_checkpointing(0, 5, 10)
    with pytest.raises(FDTDError):          # forward not run yet
        p.adjoint(0, 10, torch.zeros(10, len(w.rec)))
    p.close()
    # batched sweep: every shot needs checkpointing, all with one interval
    q = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml)] * 2)
    for k in range(2):
        q.set_velocity(k, torch.from_numpy(w.v.astype(np.float32)).cuda())
        q.set_receivers(k, w.rec)
    q.set_checkpointing(0, 5, 10)
    q.step(10)
    r = [torch.zeros(10, len(w.rec)) for _ in range(2)]
    with pytest.raises(FDTDError, match="ESTATE"):       # shot 1 has no checkpointing
        q.adjoint_all(10, r)
    q.set_checkpointing(1, 2, 10)
    with pytest.raises(FDTDError, match="EINVAL"):       # two intervals
        q.adjoint_all(10, r)
    q.close()
