"""FP64 CPU oracle for the second-order acoustic FDTD + CPML step (Python side).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path:
the arithmetic lives in ``fdtd_oracle.c`` (plain double-precision loops), and
this file only marshals numpy arrays, drives the time loop and gathers
receiver traces, snapshots and the model gradient.

Paper passages followed:
  * "Model" -- the scalar wave equation implied by the first-order system,
    the radius-r central derivative operator delta^(2r), r = 4.
  * "CPML Boundary Layers" -- stretched derivative (1/kappa) delta f + psi,
    psi recursion with b = exp(-(sigma/kappa + alpha) dt),
    a = sigma (b - 1) / (kappa (sigma + kappa alpha)), cubic grading,
    sigma_max from R, kappa_max = 5, alpha_max = 0.05 sigma_max.
  * "FDTD Verification" -- periodic standing-wave MMS used by the pins.
  * the Ricker source s(t) = (1 - 2 a^2) exp(-a^2), a = pi f0 (t - t0), of
    the CPML visualisation experiment (the wavelet itself is an input).

Array convention: numpy arrays of shape (nz, ny, nx), C order (x fastest).
Parity status: every function here is pinned by a CPU test (see the tests
named test_oracle_*); nothing is "parity unpinned" except the conventions
listed in the C file's header (rho sampling, sigma_max's velocity factor,
update-then-use ordering of psi/zeta), which are choices, not computations.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "fdtd_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    import subprocess

    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC_PATH, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _OG(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("r", ctypes.c_int),
        ("periodic", ctypes.c_int * 3),
        ("cpml", ctypes.c_int * 6),
        ("R", ctypes.c_double),
        ("kappa_max", ctypes.c_double),
        ("alpha_frac", ctypes.c_double),
        ("vref", ctypes.c_double),
    ]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        dp = P(ctypes.c_double)
        og = P(_OG)
        lib.og_weights.argtypes = [ctypes.c_int, dp, dp]
        lib.og_deriv1.argtypes = [og, ctypes.c_int, dp, dp]
        lib.og_deriv2.argtypes = [og, ctypes.c_int, dp, dp]
        lib.og_laplacian.argtypes = [og, dp, dp]
        lib.og_profile.argtypes = [og, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.og_profiles_all.argtypes = [og, ctypes.c_int, dp]
        lib.og_step.argtypes = [og, dp, dp, ctypes.c_int, dp, dp, dp, dp, ctypes.c_long,
                                ctypes.c_double, dp, dp]
        lib.og_adjoint_step.argtypes = [og, dp, dp, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.og_threads.argtypes = []
        lib.og_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Grid:
    """Problem statement: grid, spacing, dt, stencil radius, faces and CPML."""

    n: Sequence[int]                     # (nx, ny, nz)
    h: Sequence[float]                   # (hx, hy, hz) metres
    dt: float
    r: int = 4
    periodic: Sequence[int] = (0, 0, 0)
    cpml: Sequence[int] = (0, 0, 0, 0, 0, 0)
    R: float = 1e-8
    kappa_max: float = 5.0
    alpha_frac: float = 0.05
    vref: float = 1.0

    def c(self) -> _OG:
        g = _OG()
        g.n[:] = [int(x) for x in self.n]
        g.h[:] = [float(x) for x in self.h]
        g.dt = float(self.dt)
        g.r = int(self.r)
        g.periodic[:] = [int(x) for x in self.periodic]
        g.cpml[:] = [int(x) for x in self.cpml]
        g.R = float(self.R)
        g.kappa_max = float(self.kappa_max)
        g.alpha_frac = float(self.alpha_frac)
        g.vref = float(self.vref)
        return g

    @property
    def shape(self):
        return (int(self.n[2]), int(self.n[1]), int(self.n[0]))

    @property
    def npts(self) -> int:
        return int(np.prod(self.shape))


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_L().og_threads())


def weights(r: int = 4):
    """(d1[0..r], d2[0..r]) central weights of order 2r (d1[0] = 0)."""
    d1 = np.zeros(r + 1)
    d2 = np.zeros(r + 1)
    if _L().og_weights(r, _p(d1), _p(d2)) != 0:
        raise ValueError("radius must be 1..4")
    return d1, d2


def deriv1(g: Grid, axis: int, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    _L().og_deriv1(ctypes.byref(g.c()), axis, _p(f), _p(out))
    return out


def deriv2(g: Grid, axis: int, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    _L().og_deriv2(ctypes.byref(g.c()), axis, _p(f), _p(out))
    return out


def laplacian(g: Grid, f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    _L().og_laplacian(ctypes.byref(g.c()), _p(f), _p(out))
    return out


def profile(g: Grid, axis: int):
    """dict(rho, b, a, kinv, dkinv) for one axis, FP64, length n[axis]."""
    n = int(g.n[axis])
    arrs = [np.zeros(n) for _ in range(5)]
    rc = _L().og_profile(ctypes.byref(g.c()), axis, *[_p(a) for a in arrs])
    if rc != 0:
        raise ValueError("invalid CPML layer for axis %d" % axis)
    return dict(zip(["rho", "b", "a", "kinv", "dkinv"], arrs))


def _profiles_block(g: Grid):
    nmax = int(max(g.n))
    prof = np.zeros(3 * 5 * nmax)
    if _L().og_profiles_all(ctypes.byref(g.c()), nmax, _p(prof)) != 0:
        raise ValueError("invalid CPML layer")
    return prof, nmax


def flat_index(g: Grid, ijk) -> np.ndarray:
    ijk = np.asarray(ijk, dtype=np.int64).reshape(-1, 3)
    nx, ny = int(g.n[0]), int(g.n[1])
    return ijk[:, 0] + nx * (ijk[:, 1] + ny * ijk[:, 2])


@dataclass
class State:
    u: np.ndarray                  # u^n          (nz, ny, nx)
    um1: np.ndarray                # u^{n-1}
    psi: np.ndarray                # (3, nz, ny, nx), zero outside each layer
    zeta: np.ndarray

    @staticmethod
    def zeros(g: Grid) -> "State":
        s = g.shape
        return State(np.zeros(s), np.zeros(s), np.zeros((3,) + s), np.zeros((3,) + s))

    def copy(self) -> "State":
        return State(self.u.copy(), self.um1.copy(), self.psi.copy(), self.zeta.copy())


class Stepper:
    """Holds the model and profiles; advances a State one step at a time."""

    def __init__(self, g: Grid, v: np.ndarray):
        self.g = g
        self.gc = g.c()
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert v.shape == g.shape, (v.shape, g.shape)
        self.v = v
        self.m = np.ascontiguousarray(v * v * (g.dt * g.dt))
        self.prof, self.nmax = _profiles_block(g)
        self.work = np.zeros(g.npts)          # grows to 7 N for the adjoint step

    def step(self, st: State, src_index: int = -1, src_amp: float = 0.0,
             lapf: Optional[np.ndarray] = None):
        lp = _p(lapf) if lapf is not None else ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
        rc = _L().og_step(ctypes.byref(self.gc), _p(self.m), _p(self.prof), self.nmax,
                          _p(st.u), _p(st.um1), _p(st.psi), _p(st.zeta),
                          int(src_index), float(src_amp), lp, _p(self.work))
        if rc != 0:
            raise RuntimeError("og_step failed (%d)" % rc)

    def adjoint_step(self, lam: np.ndarray, lamp: np.ndarray, psib: np.ndarray, zetab: np.ndarray):
        if self.work.size < 7 * self.g.npts:
            self.work = np.zeros(7 * self.g.npts)
        rc = _L().og_adjoint_step(ctypes.byref(self.gc), _p(self.m), _p(self.prof), self.nmax,
                                  _p(lam), _p(lamp), _p(psib), _p(zetab), _p(self.work))
        if rc != 0:
            raise RuntimeError("og_adjoint_step failed (%d)" % rc)


def forward(g: Grid, v: np.ndarray, nt: int, src_ijk=None, src_w=None, rec_ijk=None,
            snap_every: int = 0, state: Optional[State] = None, keep_lapf: bool = False):
    """Run nt leapfrog steps from ``state`` (zeros by default).

    src_w[n] is the source amplitude times the wavelet sampled at t_n = n dt;
    it is injected into u^{n+1} at node src_ijk as m * src_w[n] / (hx hy hz).
    traces[n, r] = u^{n+1} at receiver r.  snaps holds u^{n+1} whenever
    (n + 1) % snap_every == 0.  Returns a dict.
    """
    st = state.copy() if state is not None else State.zeros(g)
    S = Stepper(g, v)
    src_index = -1
    if src_ijk is not None:
        src_index = int(flat_index(g, src_ijk)[0])
        src_w = np.asarray(src_w, dtype=np.float64)
        assert src_w.shape[0] >= nt
    rec = flat_index(g, rec_ijk) if rec_ijk is not None else np.zeros(0, np.int64)
    traces = np.zeros((nt, rec.shape[0]))
    snaps = []
    lapf = []
    for n in range(nt):
        lf = np.zeros(g.shape) if keep_lapf else None
        amp = float(src_w[n]) if src_index >= 0 else 0.0
        S.step(st, src_index, amp, lf)
        if keep_lapf:
            lapf.append(lf)
        if rec.size:
            traces[n] = st.u.reshape(-1)[rec]
        if snap_every and (n + 1) % snap_every == 0:
            snaps.append(st.u.copy())
    out = dict(traces=traces, state=st, snaps=np.array(snaps) if snaps else None)
    if keep_lapf:
        out["lapf"] = lapf
        out["stepper"] = S
    return out


def gradient(g: Grid, v: np.ndarray, nt: int, src_ijk, src_w, rec_ijk, resid: np.ndarray,
             fwd: Optional[dict] = None):
    """dJ/dv for J with dJ/dtraces = resid (shape (nt, nrec)).

    Reverse-time sweep of the exact transposed step; the model enters only
    through m = v^2 dt^2 multiplying (Lt u^n + f^n), so
    dJ/dm = sum_n lambda^{n+1} (Lt u^n + f^n) and dJ/dv = 2 v dt^2 dJ/dm.
    """
    if fwd is None or "lapf" not in fwd:
        fwd = forward(g, v, nt, src_ijk, src_w, rec_ijk, keep_lapf=True)
    S = fwd["stepper"]
    rec = flat_index(g, rec_ijk)
    s = g.shape
    lam = np.zeros(s)
    lamp = np.zeros(s)
    psib = np.zeros((3,) + s)
    zetab = np.zeros((3,) + s)
    gm = np.zeros(s)
    resid = np.asarray(resid, dtype=np.float64)
    for n in range(nt - 1, -1, -1):
        lf = lam.reshape(-1)
        np.add.at(lf, rec, resid[n])
        gm += lam * fwd["lapf"][n]
        S.adjoint_step(lam, lamp, psib, zetab)
    return gm * 2.0 * np.asarray(v, dtype=np.float64) * g.dt * g.dt


def misfit(traces: np.ndarray, observed: np.ndarray) -> float:
    """J = 1/2 sum (d - d_obs)^2."""
    d = np.asarray(traces, np.float64) - np.asarray(observed, np.float64)
    return 0.5 * float(np.sum(d * d))
