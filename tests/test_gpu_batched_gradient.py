"""The batched forward + adjoint workload on its smallest shot (121 x 133 x 122,
15-cell layers, layered model, 64 receivers on an interior plane, 600 steps,
checkpoints every 25 steps), advanced in a batched context together with the
next smallest shot: traces and FP64 velocity gradient against the FP64
oracle's; the next shot's gradient, taken after the first one's in the same
context, equals that shot's gradient run alone bit for bit, and the batched
sweep over both shots gives both gradients bit for bit.

Bar (written here): traces within relative L2 1e-5, gradient within 1e-4 (the
adjoint tests' bar) on the whole grid and on each axis's band; the residual
(the misfit's adjoint source) is the oracle's, passed to both sides.
"""
import numpy as np
import pytest

import synth
from helpers import band_masks, rel_l2

pytestmark = pytest.mark.gpu

K, EVERY = 600, 25


def test_smallest_batched_shot_gradient_matches_oracle():
    import torch

    from oracle import oracle as O
    from paper_2606_06910_amd import Propagator, Shot

    shapes = synth.batch_shapes(24)
    order = sorted(range(24), key=lambda i: np.prod(shapes[i]))[:2]
    data = [synth.batch_shot(i, shapes[i], nt=K) for i in order]
    wt, v0 = data[0]
    assert tuple(wt.n) == (121, 133, 122) and wt.rec.shape == (64, 3)
    vref = [float(max(w.v.astype(np.float32).max(), v.astype(np.float32).max())) for w, v in data]
    f32 = lambda a: a.astype(np.float32).astype(np.float64)   # noqa: E731
    print("oracle: observed and inversion runs, gradient (%s, %d steps)" % (wt.n, K), flush=True)
    g = O.Grid(n=wt.n, h=wt.h, dt=wt.dt, cpml=wt.cpml, vref=vref[0])
    wav = f32(wt.wavelet)
    dobs = O.forward(g, f32(wt.v), K, wt.src, wav, wt.rec)["traces"]
    fwd = O.forward(g, f32(v0), K, wt.src, wav, wt.rec, keep_lapf=True)
    resid = fwd["traces"] - dobs
    gref = O.gradient(g, f32(v0), K, wt.src, wav, wt.rec, resid, fwd=fwd)
    del fwd
    print("GPU: batched context of %d shots" % len(data), flush=True)
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, v_ref=vr) for (w, _), vr in zip(data, vref)])
    trs = []
    for k, (w, v) in enumerate(data):
        p.set_velocity(k, torch.from_numpy(v.astype(np.float32)).cuda())
        p.inject_source(k, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
        p.set_receivers(k, w.rec)
        p.set_checkpointing(k, EVERY, K)
        trs.append(p.record(k, K))
    p.step(K)
    torch.cuda.synchronize()
    tr = trs[0].cpu().double().numpy()
    gg = p.adjoint(0, K, torch.from_numpy(resid.astype(np.float32))).cpu().numpy()
    # the second shot's gradient after the first one's, in the same context, is the
    # gradient of that shot run alone (same residual)
    r1 = torch.randn(K, 64, generator=torch.Generator().manual_seed(7)) * 1e-3
    g1 = p.adjoint(1, K, r1).cpu().numpy()
    ga = [g.cpu().numpy() for g in p.adjoint_all(K, [torch.from_numpy(resid.astype(np.float32)), r1])]
    p.close()
    assert np.array_equal(ga[0], gg) and np.array_equal(ga[1], g1), "batched sweep differs from the single sweeps"
    (w1, v1), vr1 = data[1], vref[1]
    q = Propagator([Shot(n=w1.n, h=w1.h, dt=w1.dt, cpml=w1.cpml, v_ref=vr1)])
    q.set_velocity(0, torch.from_numpy(v1.astype(np.float32)).cuda())
    q.inject_source(0, w1.src[0], torch.from_numpy(w1.wavelet.astype(np.float32)).cuda())
    q.set_receivers(0, w1.rec)
    q.set_checkpointing(0, EVERY, K)
    q.record(0, K)
    q.step(K)
    g1_alone = q.adjoint(0, K, r1).cpu().numpy()
    q.close()
    assert np.array_equal(g1, g1_alone), "second shot's gradient in the batch differs from the shot alone"

    e_tr, e_g = rel_l2(tr, dobs + resid), rel_l2(gg, gref)
    masks, _ = band_masks(wt.n, wt.cpml)
    per_band = {k: rel_l2(gg[m], gref[m]) for k, m in masks.items()}
    print("traces %.2e  gradient %.2e  bands %s" % (e_tr, e_g, "  ".join("%s %.2e" % kv for kv in per_band.items())),
          flush=True)
    assert e_tr <= 1e-5
    assert e_g <= 1e-4
    for k, e in per_band.items():
        assert e <= 1e-4, (k, e)
