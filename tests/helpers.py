"""Shared test helpers: run a workload through the GPU library or the oracle."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def v32(w):
    """The velocity as the GPU sees it (float32), back in float64 for the oracle."""
    return w.v.astype(np.float32).astype(np.float64)


def oracle_grid(w, **kw):
    v = v32(w)
    return O.Grid(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, periodic=w.periodic, vref=float(v.max()), **kw)


def run_oracle(w, nt=None, snap_every=0):
    nt = w.nt if nt is None else nt
    g = oracle_grid(w)
    out = O.forward(g, v32(w), nt, w.src, w.wavelet, w.rec, snap_every=snap_every)
    return out


def band_masks(n, cpml):
    """Masks (nz, ny, nx) of the band points of each face with a layer (the
    layer plus the 4-cell margin whose stencils read layer memory), keyed
    '-x', '+x', ..., and their union."""
    nx, ny, nz = [int(x) for x in n]
    shape = (nz, ny, nx)
    masks = {}
    for d in range(3):
        c = np.arange(int(n[d]))
        for side in (0, 1):
            L = int(cpml[2 * d + side])
            if L <= 0:
                continue
            sel = c < L + 4 if side == 0 else c >= int(n[d]) - L - 4
            bshape = [1, 1, 1]
            bshape[2 - d] = int(n[d])
            masks["-+"[side] + "xyz"[d]] = np.broadcast_to(sel.reshape(bshape), shape)
    union = np.zeros(shape, bool)
    for m in masks.values():
        union |= m
    return masks, union


def per_receiver_rel_l2(got, ref, floor=1e-2):
    """Relative L2 error of each receiver's trace, over the receivers whose
    reference trace norm is at least ``floor`` times the largest one (a trace
    the wave has barely reached is all rounding)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    nr = np.linalg.norm(ref, axis=0)
    keep = nr >= floor * nr.max()
    return np.linalg.norm(got - ref, axis=0)[keep] / nr[keep]


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def run_gpu(w, nt=None, snap_every=0, graph=False, plan=None, **shot_kw):
    """Forward run on cuda:0.  Returns (traces, snaps, final u^n) as numpy float64.
    The variant defaults to the z-march (the automatic choice would run the
    naive kernel on the small test grids)."""
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    shot_kw.setdefault("variant", 2)
    nt = w.nt if nt is None else nt
    face = shot_kw.pop("face", None)
    if face is None:
        face = [0, 0, 1 if w.periodic[1] else 0, 1 if w.periodic[1] else 0,
                1 if w.periodic[2] else 0, 1 if w.periodic[2] else 0]
    shot = Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, face=face, **shot_kw)
    p = Propagator([shot])
    if plan is not None:
        p.set_plan(0, *plan)
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)))
    p.set_receivers(0, w.rec)
    tr = p.record(0, nt)
    snaps = []
    if snap_every:
        done = 0
        while done < nt:
            k = min(snap_every, nt - done)
            p.step(k, graph=graph)
            done += k
            if k == snap_every:
                snaps.append(p.get_field(0).cpu().double().numpy())
    else:
        p.step(nt, graph=graph)
    fin = p.get_field(0).cpu().double().numpy()
    torch.cuda.synchronize()
    out = tr.cpu().double().numpy(), (np.array(snaps) if snaps else None), fin
    p.close()
    return out
