"""Seeded synthetic inputs for the FDTD + CPML workloads.

This module holds input generation only: velocity models, time steps from
the Courant number, Ricker wavelet samples, source and receiver positions.
It contains none of the method's arithmetic (no stencil, no CPML, no time
stepping) and is used alike by the oracle-side tests and the GPU path.

Workload recipes (the paper runs on synthetic grids only; no dataset):
  plain64     64^3, 10-cell CPML on six faces, h = 10 m, v = 2000 (1 + 0.05 U[-1,1)),
              Ricker 15 Hz at the centre, 200 steps, 16 receivers on one seeded
              interior z-plane.
  layered512  512^3, 20-cell CPML, 8-12 horizontal layers at 1500-4500 m/s,
              Gaussian-smoothed (sigma 5 cells), Ricker 10 Hz at the centre,
              1000 steps.
  pencil      1024 x 384 x 384 owned block, layered model, CPML only on +-x,
              y and z periodic through the ghost loopback, 800 steps.
  blob768     768^3, 1500 m/s background + 6-10 Gaussian blobs up to +3500,
              clipped to [1500, 5000], 20-cell CPML, Ricker 12 Hz, 1500 steps.
  batch24     24 shots, each axis uniform in [96, 288], 15-cell CPML, layered
              models, 600 steps, 64 receivers each; observed data from the
              true model, inversion model perturbed by a smooth 3 % field.

dt always comes from the multi-dimensional Courant number
C = vmax dt sqrt(3) / h = 0.5.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

COURANT = 0.5


def seed_for(config: int) -> int:
    return 1000 + int(config)


def dt_from_courant(vmax: float, h: Sequence[float], courant: float = COURANT) -> float:
    """dt with vmax dt sqrt(sum 1/h_d^2) = courant (sqrt(3)/h for equal spacing)."""
    s = math.sqrt(sum(1.0 / (float(x) * float(x)) for x in h))
    return courant / (float(vmax) * s)


def ricker(nt: int, dt: float, f0: float, t0: Optional[float] = None, amp: float = 1.0) -> np.ndarray:
    """amp * (1 - 2 a^2) exp(-a^2), a = pi f0 (t - t0), sampled at t_n = n dt (FP64)."""
    if t0 is None:
        t0 = 1.5 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = math.pi * f0 * (t - t0)
    return amp * (1.0 - 2.0 * a * a) * np.exp(-a * a)


def uniform_perturbed(shape_zyx, v0: float, frac: float, rng: np.random.Generator) -> np.ndarray:
    return v0 * (1.0 + frac * rng.uniform(-1.0, 1.0, size=shape_zyx))


def _gauss_kernel1d(sigma: float, truncate: float = 4.0) -> np.ndarray:
    rad = int(truncate * sigma + 0.5)
    x = np.arange(-rad, rad + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _smooth1d_reflect(p: np.ndarray, sigma: float) -> np.ndarray:
    k = _gauss_kernel1d(sigma)
    rad = (k.size - 1) // 2
    pp = np.pad(p, rad, mode="symmetric")
    return np.convolve(pp, k, mode="valid")


def layered_profile(nz: int, rng: np.random.Generator, nlayers=(8, 12), vrange=(1500.0, 4500.0),
                    smooth_sigma: float = 5.0) -> np.ndarray:
    """1-D velocity profile along z: seeded layer count, interface depths and speeds,
    smoothed with a Gaussian (sigma in cells, reflect padding)."""
    K = int(rng.integers(nlayers[0], nlayers[1] + 1))
    cuts = np.sort(rng.choice(np.arange(1, nz), size=K - 1, replace=False))
    speeds = rng.uniform(vrange[0], vrange[1], size=K)
    prof = np.empty(nz)
    edges = np.concatenate([[0], cuts, [nz]])
    for i in range(K):
        prof[edges[i]:edges[i + 1]] = speeds[i]
    return _smooth1d_reflect(prof, smooth_sigma)


def layered_model(shape_zyx, rng: np.random.Generator, **kw) -> np.ndarray:
    nz, ny, nx = shape_zyx
    p = layered_profile(nz, rng, **kw)
    return np.broadcast_to(p[:, None, None], (nz, ny, nx)).copy()


@dataclass
class Blobs:
    centers: np.ndarray   # (K, 3) in cells, (x, y, z)
    radii: np.ndarray     # (K,) in cells (Gaussian sigma)
    amps: np.ndarray      # (K,)
    background: float = 1500.0
    vmin: float = 1500.0
    vmax: float = 5000.0


def blob_params(n_xyz, rng: np.random.Generator, kmin=6, kmax=10, amp_max=3500.0) -> Blobs:
    K = int(rng.integers(kmin, kmax + 1))
    n = np.asarray(n_xyz, dtype=np.float64)
    centers = rng.uniform(0.0, 1.0, size=(K, 3)) * n
    radii = rng.uniform(0.05, 0.20, size=K) * float(n.min())
    amps = rng.uniform(0.3, 1.0, size=K) * amp_max
    return Blobs(centers, radii, amps)


def blob_model(n_xyz, blobs: Blobs, origin=(0, 0, 0), sub_xyz=None) -> np.ndarray:
    """Velocity of the blob model on the box [origin, origin + sub) of the full grid."""
    if sub_xyz is None:
        sub_xyz = n_xyz
    sx, sy, sz = [int(s) for s in sub_xyz]
    ox, oy, oz = [int(o) for o in origin]
    v = np.full((sz, sy, sx), blobs.background, dtype=np.float64)
    xs = np.arange(ox, ox + sx, dtype=np.float64)
    ys = np.arange(oy, oy + sy, dtype=np.float64)
    zs = np.arange(oz, oz + sz, dtype=np.float64)
    for c, r, a in zip(blobs.centers, blobs.radii, blobs.amps):
        gx = np.exp(-0.5 * ((xs - c[0]) / r) ** 2)
        gy = np.exp(-0.5 * ((ys - c[1]) / r) ** 2)
        gz = np.exp(-0.5 * ((zs - c[2]) / r) ** 2)
        v += a * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    np.clip(v, blobs.vmin, blobs.vmax, out=v)
    return v


def blob_model_torch(n_xyz, blobs: Blobs, device="cuda"):
    """blob_model evaluated with torch on a device (float32), for large grids."""
    import torch

    nx, ny, nz = [int(x) for x in n_xyz]
    xs = torch.arange(nx, dtype=torch.float64, device=device)
    ys = torch.arange(ny, dtype=torch.float64, device=device)
    zs = torch.arange(nz, dtype=torch.float64, device=device)
    v = torch.full((nz, ny, nx), float(blobs.background), dtype=torch.float32, device=device)
    for c, r, a in zip(blobs.centers, blobs.radii, blobs.amps):
        gx = torch.exp(-0.5 * ((xs - float(c[0])) / float(r)) ** 2).float()
        gy = torch.exp(-0.5 * ((ys - float(c[1])) / float(r)) ** 2).float()
        gz = torch.exp(-0.5 * ((zs - float(c[2])) / float(r)) ** 2).float()
        v += float(a) * (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    return v.clamp_(float(blobs.vmin), float(blobs.vmax))


def smooth_field(shape_zyx, rng: np.random.Generator, sigma: float = 8.0) -> np.ndarray:
    """Seeded smooth random field with max |G| = 1 (separable Gaussian blur of noise)."""
    from scipy.ndimage import gaussian_filter

    g = gaussian_filter(rng.standard_normal(shape_zyx), sigma, mode="reflect", truncate=4.0)
    return g / np.abs(g).max()


def receivers_on_plane(n_xyz, L: int, count: int, rng: np.random.Generator) -> np.ndarray:
    """count distinct (i, j, k) with k a seeded interior plane and (i, j) seeded interior."""
    nx, ny, nz = [int(x) for x in n_xyz]
    k = int(rng.integers(L, nz - L))
    cells = rng.choice((nx - 2 * L) * (ny - 2 * L), size=count, replace=False)
    i = L + cells % (nx - 2 * L)
    j = L + cells // (nx - 2 * L)
    return np.stack([i, j, np.full(count, k)], axis=1).astype(np.int32)


@dataclass
class Workload:
    name: str
    n: Tuple[int, int, int]            # (nx, ny, nz)
    h: Tuple[float, float, float]
    dt: float
    nt: int
    cpml: Tuple[int, ...]              # six faces
    v: np.ndarray                      # (nz, ny, nx) FP64
    src: np.ndarray                    # (1, 3) int32
    wavelet: np.ndarray                # (nt,) FP64, amplitude applied
    rec: np.ndarray                    # (nrec, 3) int32
    periodic: Tuple[int, int, int] = (0, 0, 0)
    f0: float = 10.0
    extra: dict = field(default_factory=dict)

    @property
    def vmax(self) -> float:
        return float(self.v.max())

    @property
    def npts(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


def plain64(nt: int = 200, n: int = 64, L: int = 10, seed: int = 1000) -> Workload:
    rng = np.random.default_rng(seed)
    h = 10.0
    v = uniform_perturbed((n, n, n), 2000.0, 0.05, rng)
    dt = dt_from_courant(v.max(), (h, h, h))
    f0 = 15.0
    rec = receivers_on_plane((n, n, n), L, 16, rng)
    src = np.array([[n // 2, n // 2, n // 2]], dtype=np.int32)
    return Workload("plain64", (n, n, n), (h, h, h), dt, nt, (L,) * 6, v, src,
                    ricker(nt, dt, f0), rec, f0=f0)


def layered(n_xyz=(512, 512, 512), nt: int = 1000, L: int = 20, seed: int = 1001, f0: float = 10.0,
            nrec: int = 16, cpml=None, periodic=(0, 0, 0), h: float = 10.0, name="layered512") -> Workload:
    rng = np.random.default_rng(seed)
    nx, ny, nz = n_xyz
    v = layered_model((nz, ny, nx), rng)
    dt = dt_from_courant(v.max(), (h, h, h))
    if cpml is None:
        cpml = (L,) * 6
    Lr = max(cpml) if max(cpml) > 0 else 0
    rec = receivers_on_plane(n_xyz, min(Lr, min(n_xyz) // 4), nrec, rng)
    src = np.array([[nx // 2, ny // 2, nz // 2]], dtype=np.int32)
    return Workload(name, tuple(n_xyz), (h, h, h), dt, nt, tuple(cpml), v, src,
                    ricker(nt, dt, f0), rec, periodic=tuple(periodic), f0=f0)


def pencil(nt: int = 800, seed: int = 1002, n_xyz=(1024, 384, 384), L: int = 20) -> Workload:
    w = layered(n_xyz, nt=nt, L=L, seed=seed, cpml=(L, L, 0, 0, 0, 0), periodic=(0, 1, 1),
                name="pencil")
    return w


def blob(n: int = 768, nt: int = 1500, L: int = 20, seed: int = 1003, crop: Optional[int] = None,
         f0: float = 12.0, h: float = 10.0) -> Workload:
    """Gaussian-blob model on n^3; with crop=c, the central c^3 box of the same
    model (own CPML of width L, same source node relative to the crop centre)."""
    rng = np.random.default_rng(seed)
    blobs = blob_params((n, n, n), rng)
    vmax_full = float(blobs.vmax)
    if crop is None:
        v = blob_model((n, n, n), blobs)
        size = n
    else:
        o = (n - crop) // 2
        v = blob_model((n, n, n), blobs, origin=(o, o, o), sub_xyz=(crop, crop, crop))
        size = crop
    # dt from the full model's velocity ceiling so that crop and full run share dt
    dt = dt_from_courant(vmax_full, (h, h, h))
    rec = receivers_on_plane((size, size, size), L, 16, rng)
    src = np.array([[size // 2, size // 2, size // 2]], dtype=np.int32)
    return Workload("blob%d" % size, (size, size, size), (h, h, h), dt, nt, (L,) * 6, v, src,
                    ricker(nt, dt, f0), rec, f0=f0, extra=dict(blobs=blobs))


def batch_shapes(count: int = 24, lo: int = 96, hi: int = 288, seed: int = 1004) -> List[Tuple[int, int, int]]:
    rng = np.random.default_rng(seed)
    return [tuple(int(x) for x in rng.integers(lo, hi + 1, size=3)) for _ in range(count)]


def batch_shot(i: int, shape_xyz, nt: int = 600, L: int = 15, nrec: int = 64, seed: int = 1004,
               f0: float = 10.0, h: float = 10.0, perturb: float = 0.03):
    """One shot of the batched workload: (true model workload, perturbed model)."""
    rng = np.random.default_rng([seed, i])
    nx, ny, nz = shape_xyz
    vt = layered_model((nz, ny, nx), rng)
    G = smooth_field((nz, ny, nx), rng, sigma=8.0)
    v0 = vt * (1.0 + perturb * G)
    vmax = max(vt.max(), v0.max())
    dt = dt_from_courant(vmax, (h, h, h))
    rec = receivers_on_plane(shape_xyz, L, nrec, rng)
    src = np.array([[nx // 2, ny // 2, nz // 2]], dtype=np.int32)
    w = Workload("shot%d" % i, tuple(shape_xyz), (h, h, h), dt, nt, (L,) * 6, vt, src,
                 ricker(nt, dt, f0), rec, f0=f0)
    return w, v0


# ---------------------------------------------------------------------------
# layer reflection study: normal incidence on the low face of one axis
# ---------------------------------------------------------------------------
REFL_WIDTHS = (0, 8, 12, 16, 24)     # layer widths of the study (the paper's reflection table)
# Uniform 2000 m/s, h = 10 m, Ricker 12.5 Hz (16 points per wavelength at the
# peak frequency), Courant number 0.5.  The run lasts until the widest layer's
# return from its Dirichlet wall (path 24 + 2 L + 4 cells) and the pulse's
# half-width (15 cells) have passed the receiver: 91 cells of travel after the
# source peak.  Every other path back to the receiver (off a transverse face,
# the opposite face, or a transverse face and then the layer) is longer than
# 106 cells, so that nothing else it returns arrives within the run.
REFL_NT = 400
REFL_F0 = 12.5
REFL_GAP_REC = 4      # receiver: first point past the layer band (layer + 4-cell margin)
REFL_GAP_SRC = 24     # source: 24 cells from the layer's inner edge, on the same normal line
REFL_BEHIND = 46      # cells from the source to the opposite (Dirichlet) face
REFL_HALF = 56        # transverse half-width (Dirichlet transverse faces)
REFL_EXTEND = 48      # reference run: the low face moved this many cells further out, no layer


def reflection_case(axis: int, L: int, reference: bool = False, v0: float = 2000.0, f0: float = REFL_F0,
                    h: float = 10.0) -> Workload:
    """Normal-incidence reflection off the low face of `axis` with a layer of L
    cells there (no layer anywhere else).  Uniform v0; source and receivers on
    the face normal through the transverse centre; every other face is far
    enough that nothing it returns reaches the receivers within REFL_NT steps.
    reference=True: the same geometry relative to the source, with the low
    face REFL_EXTEND cells further out and no layer, so that within the run
    its traces hold the incident wave only (the layer width then only names
    which run it serves)."""
    lo = REFL_EXTEND if reference else L
    nn = lo + REFL_GAP_SRC + REFL_BEHIND
    t = 2 * REFL_HALF + 1
    n = [t, t, t]
    n[axis] = nn
    cpml = [0] * 6
    if not reference:
        cpml[2 * axis] = L
    dt = dt_from_courant(v0, (h, h, h))
    src = [REFL_HALF] * 3
    src[axis] = lo + REFL_GAP_SRC
    recs = []
    for gap in (REFL_GAP_REC, REFL_GAP_REC + 8):
        r = [REFL_HALF] * 3
        r[axis] = lo + gap
        recs.append(r)
    nx, ny, nz = n
    v = np.full((nz, ny, nx), v0)
    name = "refl_%s_%s" % ("xyz"[axis], "ref" if reference else "L%d" % L)
    return Workload(name, tuple(n), (h, h, h), dt, REFL_NT, tuple(cpml), v, np.array([src], np.int32),
                    ricker(REFL_NT, dt, f0), np.array(recs, np.int32), f0=f0)


def reflection_ratio(trace: np.ndarray, ref_trace: np.ndarray) -> float:
    """Reflected-to-incident amplitude ratio at one receiver: the peak of the
    difference from the reference run (which holds the incident wave only)
    over the peak of the reference trace."""
    d = np.asarray(trace, np.float64) - np.asarray(ref_trace, np.float64)
    return float(np.abs(d).max() / np.abs(np.asarray(ref_trace, np.float64)).max())
