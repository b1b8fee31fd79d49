"""FP64 CPU oracle for the paper's first-order pressure-velocity system with CPML.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.
Plain numpy in float64: whole-array shifts, no blocking or fusion.

Paper passages followed:
  * "First-Order Acoustic Model and Discrete Update" -- the normalised
    two-stage update: v_d^{n+1/2} = v_d^{n-1/2} - lambda delta_d p^n for each
    axis d, then p^{n+1} = p^n - lambda sum_d delta_d v_d^{n+1/2}, with the
    radius-r central operator (delta f)_i = sum_l a_l (f_{i+l} - f_{i-l})
    (unit spacing), r = 4.
  * "CPML Boundary Layers" -- inside a layer every derivative becomes
    (1/kappa) delta f + psi, with psi <- b psi + a delta f; one memory
    variable per axis for the pressure derivatives (velocity stage) and one
    per axis for the velocity derivatives (pressure stage).  b, a, 1/kappa
    come from the cubic profiles of the same section.
  * the parameter table -- lambda = 0.05, 20-cell layers, R = 1e-8,
    kappa_max = 5, alpha_max = 0.05 sigma_max.

Readings where the paper is silent (each listed in the design notes):
  * units: the coefficients are absorbed into lambda, i.e. c = h = 1 and
    dt = lambda, so b = exp(-(sigma/kappa + alpha) lambda) and
    sigma_max = -4 ln(R) / (2 L);
  * psi is updated with the current derivative before it is used (psi_v at
    step n holds delta p^n; psi_p at n+1/2 holds delta v^{n+1/2});
  * the grid is surrounded by zeros (a Dirichlet frame), or wraps on the axes
    marked periodic;
  * a point source adds lambda w^n to p at its node after the pressure stage;
    receivers record p^{n+1}.

Array convention: numpy arrays of shape (nz, ny, nx), x fastest.
Parity status: pinned by tests/test_pv_oracle_pins.py: one step with layers
of a different width on every face equals an independently assembled sparse
step matrix (Kronecker products of the 1-D derivative matrix with diagonal
b, a, 1/kappa) plus the source vector; kappa_max = 1 on a line equals a 1-D
scalar loop with its own profile; exact Fourier-mode recurrence; exact
discrete energy without layers; the stability limit; mirror symmetry; energy
loss and its fall with layer width.  The psi index and the source placement
are readings (the paper fixes neither); the matrix pins the oracle to them.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np

from oracle import oracle as O

_AXIS = {0: 2, 1: 1, 2: 0}   # grid axis d -> numpy axis of an (nz, ny, nx) array


def shift(f: np.ndarray, d: int, l: int, periodic: bool) -> np.ndarray:
    """g with g_i = f_{i+l} along grid axis d (zero outside the grid unless periodic)."""
    ax = _AXIS[d]
    if periodic:
        return np.roll(f, -l, axis=ax)
    g = np.zeros_like(f)
    n = f.shape[ax]
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if l > 0:
        src[ax], dst[ax] = slice(l, n), slice(0, n - l)
    else:
        src[ax], dst[ax] = slice(0, n + l), slice(-l, n)
    g[tuple(dst)] = f[tuple(src)]
    return g


def delta(f: np.ndarray, d: int, a: np.ndarray, periodic: bool) -> np.ndarray:
    """Central first derivative along axis d, unit spacing: sum_l a_l (f_{i+l} - f_{i-l})."""
    out = np.zeros_like(f)
    for l in range(1, len(a)):
        out += a[l] * (shift(f, d, l, periodic) - shift(f, d, -l, periodic))
    return out


class PV:
    """State and time loop of the first-order system on an (nx, ny, nz) grid."""

    def __init__(self, n: Sequence[int], cpml: Sequence[int] = (0,) * 6, lam: float = 0.05,
                 periodic: Sequence[int] = (0, 0, 0), r: int = 4, R: float = 1e-8,
                 kappa_max: float = 5.0, alpha_frac: float = 0.05):
        self.n = tuple(int(x) for x in n)
        self.lam = float(lam)
        self.periodic = tuple(bool(x) for x in periodic)
        self.a = O.weights(r)[0]                       # a_0 = 0, a_1 .. a_r
        shape = (self.n[2], self.n[1], self.n[0])
        self.p = np.zeros(shape)
        self.v = [np.zeros(shape) for _ in range(3)]
        self.psi_v = [np.zeros(shape) for _ in range(3)]
        self.psi_p = [np.zeros(shape) for _ in range(3)]
        # layer coefficients in the units above: h = 1, dt = lambda, velocity 1
        g = O.Grid(n=self.n, h=(1.0, 1.0, 1.0), dt=self.lam, r=r, periodic=tuple(int(x) for x in periodic),
                   cpml=tuple(int(x) for x in cpml), R=R, kappa_max=kappa_max, alpha_frac=alpha_frac, vref=1.0)
        self.b, self.acoef, self.kinv = [], [], []
        for d in range(3):
            pr = O.profile(g, d)
            bshape = [1, 1, 1]
            bshape[_AXIS[d]] = self.n[d]
            self.b.append(pr["b"].reshape(bshape))
            self.acoef.append(pr["a"].reshape(bshape))
            self.kinv.append(pr["kinv"].reshape(bshape))
        self.step_index = 0

    def _stretched(self, f: np.ndarray, d: int, psi: np.ndarray) -> np.ndarray:
        """(1/kappa_d) delta_d f + psi_d, psi_d advanced with the current derivative first."""
        g = delta(f, d, self.a, self.periodic[d])
        psi *= self.b[d]
        psi += self.acoef[d] * g
        return self.kinv[d] * g + psi

    def step(self, src_ijk=None, src_w: Optional[np.ndarray] = None) -> None:
        lam = self.lam
        for d in range(3):                             # pressure to velocity
            self.v[d] -= lam * self._stretched(self.p, d, self.psi_v[d])
        div = np.zeros_like(self.p)
        for d in range(3):                             # velocity to pressure
            div += self._stretched(self.v[d], d, self.psi_p[d])
        self.p -= lam * div
        if src_ijk is not None and src_w is not None and self.step_index < len(src_w):
            i, j, k = (int(x) for x in src_ijk)
            self.p[k, j, i] += lam * float(src_w[self.step_index])
        self.step_index += 1


def forward(n, cpml, lam: float, nt: int, src_ijk=None, src_w=None, rec_ijk=None, p0: Optional[np.ndarray] = None,
            periodic=(0, 0, 0), snap_every: int = 0):
    """Run nt steps from rest (or from p0 with v = 0).  Returns dict(traces
    (nt, nrec) of p^{n+1} at the receivers, snaps (list of p), p, v)."""
    s = PV(n, cpml, lam, periodic)
    if p0 is not None:
        s.p[...] = p0
    rec = None if rec_ijk is None else np.asarray(rec_ijk, dtype=np.int64).reshape(-1, 3)
    traces = np.zeros((nt, 0 if rec is None else len(rec)))
    snaps = []
    for t in range(nt):
        s.step(src_ijk, src_w)
        if rec is not None:
            traces[t] = s.p[rec[:, 2], rec[:, 1], rec[:, 0]]
        if snap_every and (t + 1) % snap_every == 0:
            snaps.append(s.p.copy())
    return dict(traces=traces, snaps=np.array(snaps), p=s.p, v=s.v)
