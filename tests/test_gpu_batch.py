"""Batched shots in one context (grouped z-march launches, one band launch over
every shot's tiles, pre-passes over all shots, a mixed naive / z-march batch,
the HIP-graph time loop, the autotuner) reproduce each shot's single-shot run
bit for bit: a shot's points see the same arithmetic whatever else shares the
launch.  Every shot of a batch is also held to the FP64 oracle directly
(relative L2 <= 1e-5 on its traces and final field), and so is a batch shaped
like the batched workload (uneven grids, 15-cell layers on every face,
layered models, 64 receivers on an interior plane) at reduced size and step
count.
"""
import numpy as np
import pytest

import synth
from helpers import per_receiver_rel_l2, rel_l2

pytestmark = pytest.mark.gpu

NAIVE, ZMARCH = 1, 2

# shapes, spacings, layers: ragged tiles, uneven layers, no layer at all, and
# one whose layers are too wide for the band kernel to advance x memory itself
SHOTS = [
    dict(n=(70, 45, 38), h=(10.0, 12.0, 9.0), cpml=(5, 7, 3, 6, 8, 4), seed=11),
    dict(n=(48, 40, 36), h=(10.0, 10.0, 10.0), cpml=(0, 9, 6, 0, 0, 7), seed=12),
    dict(n=(33, 29, 41), h=(8.0, 8.0, 8.0), cpml=(0,) * 6, seed=13),
    dict(n=(80, 36, 40), h=(10.0, 10.0, 10.0), cpml=(30, 12, 5, 4, 6, 5), seed=14),
    dict(n=(56, 52, 60), h=(10.0, 10.0, 10.0), cpml=(10,) * 6, seed=15),
]
NT = 40


def _workload(c):
    rng = np.random.default_rng(c["seed"])
    nx, ny, nz = c["n"]
    v = 1800.0 + 800.0 * rng.uniform(size=(nz, ny, nx))
    dt = synth.dt_from_courant(3000.0, c["h"]) * 0.9      # one dt that is stable for every shot
    src = (nx // 3, ny // 2, nz // 2)
    # six receivers within 5 cells of the source (reached within the run), four anywhere
    near = np.array(src)[None, :] + rng.integers(-5, 6, size=(6, 3))
    far = np.stack([rng.integers(0, nx, 4), rng.integers(0, ny, 4), rng.integers(0, nz, 4)], 1)
    rec = np.clip(np.concatenate([near, far]), 0, np.array(c["n"]) - 1)
    return v, dt, src, synth.ricker(NT, dt, 45.0), rec.astype(np.int32)


def _run(indices, variants, graph=False, autotune=False, plans=None, tmp_path=None):
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    shots, data = [], []
    for i, var in zip(indices, variants):
        c = SHOTS[i]
        v, dt, src, wav, rec = _workload(c)
        shots.append(Shot(n=c["n"], h=c["h"], dt=dt, cpml=c["cpml"], variant=var))
        data.append((v, src, wav, rec))
    p = Propagator(shots)
    trs = []
    for k, (v, src, wav, rec) in enumerate(data):
        p.set_velocity(k, torch.from_numpy(v.astype(np.float32)).cuda())
        p.inject_source(k, src, torch.from_numpy(wav.astype(np.float32)).cuda())
        p.set_receivers(k, rec)
        trs.append(p.record(k, NT))
    if plans is not None:
        for k, pl in enumerate(plans):
            p.set_plan(k, *pl)
    if autotune:
        p.autotune(str(tmp_path / "tune.json"))
        p.reset()
        print("autotuned plans (variant, tile_ry, tblock_k, tile_cols):", [p.plan(k) for k in range(len(shots))],
              flush=True)
    p.step(NT, graph=graph)
    torch.cuda.synchronize()
    out = [(trs[k].cpu().numpy().copy(), p.get_field(k).cpu().numpy().copy()) for k in range(len(shots))]
    p.close()
    return out


@pytest.fixture(scope="module")
def singles():
    """Each shot alone, z-march (the arithmetic does not depend on the plan)."""
    return [_run([i], [ZMARCH])[0] for i in range(len(SHOTS))]


def _assert_same(got, ref):
    for k, ((tr, u), (tr0, u0)) in enumerate(zip(got, ref)):
        assert np.array_equal(tr, tr0), "shot %d traces differ" % k
        assert np.array_equal(u, u0), "shot %d field differs" % k


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_shots(singles, graph):
    got = _run(range(len(SHOTS)), [ZMARCH] * len(SHOTS), graph=graph)
    _assert_same(got, singles)


def test_mixed_naive_and_zmarch_batch(singles):
    """Naive shots read every psi from the pre-passes while the others advance
    x and z layer memory in the band kernel; both kinds in one batch."""
    variants = [NAIVE, ZMARCH, NAIVE, ZMARCH, ZMARCH]
    got = _run(range(len(SHOTS)), variants)
    _assert_same(got, singles)


def test_batch_with_distinct_plans(singles):
    """Shots with different z-march plans run as separate grouped launches."""
    plans = [(ZMARCH, 1, 32, 1), (ZMARCH, 2, 64, 1), (ZMARCH, 4, 4096, 1), (ZMARCH, 8, 32, 1), (ZMARCH, 1, 16, 1)]
    got = _run(range(len(SHOTS)), [ZMARCH] * len(SHOTS), graph=True, plans=plans)
    _assert_same(got, singles)


def test_autotuned_batch(singles, tmp_path):
    got = _run(range(len(SHOTS)), [ZMARCH] * len(SHOTS), autotune=True, tmp_path=tmp_path)
    _assert_same(got, singles)


def _oracle(n, h, dt, cpml, v, src, wav, rec, nt):
    from oracle import oracle as O

    vv = v.astype(np.float32).astype(np.float64)
    g = O.Grid(n=n, h=h, dt=dt, cpml=cpml, vref=float(vv.max()))
    out = O.forward(g, vv, nt, np.array([src]), wav.astype(np.float32).astype(np.float64), rec)
    return out["traces"], out["state"].u


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(graph):
    """Each of the five shots of one batched context (graph replay or eager)
    against its own FP64 oracle run."""
    got = _run(range(len(SHOTS)), [ZMARCH] * len(SHOTS), graph=graph)
    for k, c in enumerate(SHOTS):
        v, dt, src, wav, rec = _workload(c)
        rtr, ru = _oracle(c["n"], c["h"], dt, c["cpml"], v, src, wav, rec, NT)
        e_tr, e_u = rel_l2(got[k][0], rtr), rel_l2(got[k][1], ru)
        per = per_receiver_rel_l2(got[k][0], rtr)
        print("shot %d %s: traces %.2e  field %.2e  per-receiver max %.2e over %d" %
              (k, c["n"], e_tr, e_u, per.max(), per.size), flush=True)
        assert e_tr <= 1e-5 and e_u <= 1e-5, (k, e_tr, e_u)
        assert per.max() <= 1e-5, (k, per.max())


# batched-workload shape at reduced size: each axis in [64, 96], 15-cell layers,
# layered models, 64 receivers on a seeded interior plane; a 40 Hz Ricker so that
# the short run carries the whole pulse to the receivers
C4_SHAPES = [(72, 64, 80), (96, 66, 70), (64, 90, 68), (81, 77, 93)]
C4_NT = 180


def test_batched_workload_shapes_match_oracle():
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    ws = [synth.batch_shot(i, shp, nt=C4_NT, f0=40.0)[0] for i, shp in enumerate(C4_SHAPES)]
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml) for w in ws])
    trs = []
    for k, w in enumerate(ws):
        p.set_velocity(k, torch.from_numpy(w.v.astype(np.float32)).cuda())
        p.inject_source(k, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
        p.set_receivers(k, w.rec)
        trs.append(p.record(k, C4_NT))
    p.step(C4_NT, graph=True)
    torch.cuda.synchronize()
    got = [(trs[k].cpu().numpy().copy(), p.get_field(k).cpu().numpy().copy()) for k in range(len(ws))]
    p.close()
    for k, w in enumerate(ws):
        assert w.rec.shape == (64, 3) and w.cpml == (15,) * 6
        rtr, ru = _oracle(w.n, w.h, w.dt, w.cpml, w.v, w.src[0], w.wavelet, w.rec, C4_NT)
        e_tr, e_u = rel_l2(got[k][0], rtr), rel_l2(got[k][1], ru)
        per = per_receiver_rel_l2(got[k][0], rtr)
        reach = np.abs(rtr).max() / np.abs(ru).max()
        print("c4-like shot %d %s: traces %.2e  field %.2e  per-receiver max %.2e over %d  (trace/field peak %.2e)" %
              (k, w.n, e_tr, e_u, per.max(), per.size, reach), flush=True)
        assert reach >= 1e-2, "the receivers see too little of the wave for a trace comparison"
        assert e_tr <= 1e-5 and e_u <= 1e-5, (k, e_tr, e_u)
        assert per.max() <= 1e-5, (k, per.max())
