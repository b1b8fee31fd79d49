"""Pins of the first-order pressure-velocity oracle (oracle/pv_oracle.py) to
facts fixed by the mathematics, not by its own code:

* exact Fourier-mode recurrence on a periodic grid (closed form);
* an exactly conserved discrete energy without layers (Dirichlet frame);
* mirror symmetry with mirrored layers, broken by unequal layers;
* energy loss through the layers, and less reflected energy from wider layers.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pv_oracle as P


def _grid_coords(n):
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x, y, z


@pytest.mark.parametrize("m,lam", [((1, 2, 1), 0.25), ((3, 1, 2), 0.2), ((0, 0, 1), 0.3)])
def test_fourier_mode_closed_form(m, lam):
    """p^0 = cos(k.x), v^{-1/2} = 0 on a periodic grid.  delta maps cos to
    -s sin and sin to s cos, s_d = 2 sum_l a_l sin(l k_d), so eliminating v
    gives p^{n+1} - 2 p^n + p^{n-1} = -lam^2 S^2 p^n with S^2 = sum_d s_d^2 and
    p^1 = (1 - lam^2 S^2) p^0: p^n = [cos(n t) + (cos t - 1) / sin t sin(n t)] p^0,
    cos t = 1 - lam^2 S^2 / 2."""
    n = (16, 12, 10)
    a = O.weights(4)[0]
    k = [2 * math.pi * m[d] / n[d] for d in range(3)]
    x, y, z = _grid_coords(n)
    p0 = np.cos(k[0] * x + k[1] * y + k[2] * z)
    S2 = sum((2 * sum(a[l] * math.sin(l * kd) for l in range(1, 5))) ** 2 for kd in k)
    t = math.acos(1 - lam * lam * S2 / 2)
    s = P.PV(n, (0,) * 6, lam, periodic=(1, 1, 1))
    s.p[...] = p0
    for step in range(1, 41):
        s.step()
        amp = math.cos(step * t) + (math.cos(t) - 1) / math.sin(t) * math.sin(step * t)
        assert np.max(np.abs(s.p - amp * p0)) < 1e-12, step


def test_energy_invariant_without_layers():
    """With zero padding delta_d is skew-symmetric, so E^n = |p^n|^2 +
    sum_d <v_d^{n+1/2}, v_d^{n-1/2}> is conserved exactly (E^{n+1} - E^n =
    -<p^{n+1} + p^n, p^{n+1} - p^n> + |p^{n+1}|^2 - |p^n|^2 = 0), while a pulse
    reflects off the walls many times."""
    n = (20, 16, 14)
    x, y, z = _grid_coords(n)
    p0 = np.exp(-((x - 8.3) ** 2 + (y - 7.1) ** 2 + (z - 6.4) ** 2) / 6.0)
    s = P.PV(n, (0,) * 6, 0.3)
    s.p[...] = p0
    energies = []
    for _ in range(300):
        # a step takes (p^m, v^{m-1/2}) to (p^{m+1}, v^{m+1/2}): E^m pairs the p it
        # started from with the velocities on either side of it
        pm, vm = s.p.copy(), [v.copy() for v in s.v]
        s.step()
        energies.append(float(np.sum(pm * pm)) + sum(float(np.sum(s.v[d] * vm[d])) for d in range(3)))
    e = np.array(energies)
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-12
    # and the field really moved (the pulse left its start and came back distorted)
    assert np.max(np.abs(s.p - p0)) > 0.1


def test_mirror_symmetry():
    """Mirrored layers and a pulse centred in x keep p even in x to rounding;
    unequal layers break it."""
    n = (21, 14, 12)
    x, y, z = _grid_coords(n)
    p0 = np.exp(-((x - 10.0) ** 2 + (y - 6.3) ** 2 + (z - 5.2) ** 2) / 5.0)
    for cpml, symmetric in (((6, 6, 3, 2, 2, 4), True), ((6, 5, 3, 2, 2, 4), False)):
        s = P.PV(n, cpml, 0.25)
        s.p[...] = p0
        for _ in range(60):
            s.step()
        asym = np.max(np.abs(s.p - s.p[:, :, ::-1])) / np.max(np.abs(s.p))
        if symmetric:
            assert asym < 1e-13
        else:
            assert asym > 1e-6


def _energy(s):
    return float(np.sum(s.p ** 2) + sum(np.sum(v ** 2) for v in s.v))


def test_layers_absorb_and_wider_reflects_less():
    """A pulse leaves through 10-cell layers on every face: the energy left in
    the grid falls by orders of magnitude (without layers it would stay).  The
    energy reflected back into a probe box at the centre falls as the layers
    widen from 4 to 8 to 16 cells."""
    n = (40, 40, 40)
    x, y, z = _grid_coords(n)
    p0 = np.exp(-((x - 19.5) ** 2 + (y - 19.5) ** 2 + (z - 19.5) ** 2) / 4.0)
    s = P.PV(n, (10,) * 6, 0.3)
    s.p[...] = p0
    e0 = _energy(s)
    for _ in range(400):
        s.step()
    assert _energy(s) < 1e-3 * e0

    refl = []
    for L in (4, 8, 16):
        nn = (40 + 2 * L,) * 3
        xx, yy, zz = _grid_coords(nn)
        c = (nn[0] - 1) / 2
        s = P.PV(nn, (L,) * 6, 0.3)
        s.p[...] = np.exp(-((xx - c) ** 2 + (yy - c) ** 2 + (zz - c) ** 2) / 4.0)
        # the direct pulse has left the probe box after 40 steps (12 cells at speed 1 per
        # 1/lam steps); what enters it up to step 160 came back from the walls
        b = tuple(slice(L + 16, L + 24) for _ in range(3))
        peak = 0.0
        for t in range(160):
            s.step()
            if t >= 40:
                peak = max(peak, float(np.max(np.abs(s.p[b]))))
        refl.append(peak)
    assert refl[0] > refl[1] > refl[2]


# ------------------- independent sparse-matrix assembly of one step (layers) --

def _pv_step_matrix(n, cpml, lam):
    """One step of the first-order system as a sparse matrix on the state
    [p, v_x, v_y, v_z, psi_v (3), psi_p (3)], assembled from Kronecker
    products of the 1-D first-derivative matrix (zero outside the grid) and
    diagonal b, a and 1/kappa ("CPML Boundary Layers"): the velocity stage
    (psi_v,d' = B_d psi_v,d + A_d D_d p, v_d' = v_d - lam (K_d D_d p + psi_v,d'))
    followed by the pressure stage (psi_p,d' = B_d psi_p,d + A_d D_d v_d',
    p' = p - lam sum_d (K_d D_d v_d' + psi_p,d'))."""
    import scipy.sparse as sp

    a = O.weights(4)[0]
    nn = [int(x) for x in n]
    N = nn[0] * nn[1] * nn[2]

    def D1(m):
        M = sp.lil_matrix((m, m))
        for i in range(m):
            for l in range(1, 5):
                if i + l < m:
                    M[i, i + l] += a[l]
                if i - l >= 0:
                    M[i, i - l] -= a[l]
        return M.tocsr()

    def lift(A, d):
        mats = [sp.identity(nn[2]), sp.identity(nn[1]), sp.identity(nn[0])]   # kron order z, y, x
        mats[2 - d] = A
        return sp.kron(mats[0], sp.kron(mats[1], mats[2])).tocsr()

    # profiles in the first-order units (h = 1, dt = lam, unit velocity)
    g = O.Grid(n=tuple(nn), h=(1.0, 1.0, 1.0), dt=lam, cpml=tuple(cpml), vref=1.0)
    prof = [O.profile(g, d) for d in range(3)]
    D = [lift(D1(nn[d]), d) for d in range(3)]
    B = [lift(sp.diags(prof[d]["b"]), d) for d in range(3)]
    A = [lift(sp.diags(prof[d]["a"]), d) for d in range(3)]
    K = [lift(sp.diags(prof[d]["kinv"]), d) for d in range(3)]
    I = sp.identity(N, format="csr")
    Z = None

    def blocks():
        return [[Z] * 10 for _ in range(10)]

    V = blocks()                                   # velocity stage
    V[0][0] = I
    for d in range(3):
        V[1 + d][0] = -lam * (K[d] @ D[d]) - lam * (A[d] @ D[d])
        V[1 + d][1 + d] = I
        V[1 + d][4 + d] = -lam * B[d]
        V[4 + d][0] = A[d] @ D[d]
        V[4 + d][4 + d] = B[d]
        V[7 + d][7 + d] = I
    Pm = blocks()                                  # pressure stage
    Pm[0][0] = I
    for d in range(3):
        Pm[0][1 + d] = -lam * (K[d] @ D[d]) - lam * (A[d] @ D[d])
        Pm[0][7 + d] = -lam * B[d]
        Pm[1 + d][1 + d] = I
        Pm[4 + d][4 + d] = I
        Pm[7 + d][1 + d] = A[d] @ D[d]
        Pm[7 + d][7 + d] = B[d]
    V = sp.bmat(V, format="csr")
    Pm = sp.bmat(Pm, format="csr")
    layer = [(prof[d]["rho"] > 0).astype(float) for d in range(3)]
    return (Pm @ V).tocsr(), layer


def _pv_state_vector(s):
    return np.concatenate([s.p.ravel()] + [x.ravel() for x in s.v] + [x.ravel() for x in s.psi_v] +
                          [x.ravel() for x in s.psi_p])


@pytest.mark.parametrize("lam", [0.05, 0.3])
def test_step_matches_sparse_matrix_bruteforce(lam):
    """One oracle step, from a random state with memory variables inside their
    layers, equals the independently assembled step matrix to 1e-13, on a grid
    with a different layer width on every face and a point source."""
    n, cpml = (15, 13, 12), (3, 5, 2, 4, 4, 3)
    T, layer = _pv_step_matrix(n, cpml, lam)
    rng = np.random.default_rng(17)
    s = P.PV(n, cpml, lam)
    shape = s.p.shape
    s.p[...] = rng.standard_normal(shape)
    for d in range(3):
        mask = layer[d].reshape([-1 if P._AXIS[d] == ax else 1 for ax in range(3)])
        s.v[d][...] = rng.standard_normal(shape)
        s.psi_v[d][...] = rng.standard_normal(shape) * mask
        s.psi_p[d][...] = rng.standard_normal(shape) * mask
    x = _pv_state_vector(s)
    src, w = (7, 6, 5), np.array([0.75])
    s.step(src, w)
    y = T @ x
    N = int(np.prod(n))
    y[src[0] + n[0] * (src[1] + n[1] * src[2])] += lam * 0.75     # source after the pressure stage
    got = _pv_state_vector(s)
    assert np.abs(got - y).max() <= 1e-13 * np.abs(y).max()
    # the layers really act: without the memory terms the step differs
    assert np.abs(got[:N] - (T @ np.where(np.arange(10 * N) < 4 * N, x, 0.0))[:N]).max() > 1e-3


def test_kappa_one_line_matches_scalar_loop():
    """kappa_max = 1 on a line (periodic y, z of size 1, so their derivatives
    vanish): the oracle equals a 1-D scalar loop written from the section's
    formulas, with its own profile: sigma = sigma_max rho^3, sigma_max =
    -4 ln R / (2 L), alpha = 0.05 sigma_max (1 - rho), b = exp(-(sigma +
    alpha) lam), a = sigma (b - 1) / (sigma + alpha), memory updated before
    use in each stage."""
    nx, L, lam, R = 60, 9, 0.3, 1e-8
    a = O.weights(4)[0]
    rho = np.zeros(nx)
    for i in range(nx):
        if i < L:
            rho[i] = (L - i) / L
        elif i >= nx - L:
            rho[i] = (i - (nx - 1 - L)) / L
    smax = -4.0 * math.log(R) / (2 * L)
    sig = smax * rho ** 3
    alp = 0.05 * smax * (1 - rho)
    b = np.where(rho > 0, np.exp(-(sig + alp) * lam), 0.0)
    ac = np.where(rho > 0, sig * (b - 1) / np.where(rho > 0, sig + alp, 1.0), 0.0)

    xs = np.arange(nx)
    p = np.exp(-((xs - 23.4) ** 2) / 6.0)
    v = np.zeros(nx)
    pv, pp = np.zeros(nx), np.zeros(nx)
    s = P.PV((nx, 1, 1), (L, L, 0, 0, 0, 0), lam, periodic=(0, 1, 1), kappa_max=1.0)
    s.p[0, 0, :] = p

    def dlt(f, i):
        acc = 0.0
        for l in range(1, 5):
            fp = f[i + l] if i + l < nx else 0.0
            fm = f[i - l] if i - l >= 0 else 0.0
            acc += a[l] * (fp - fm)
        return acc

    for _ in range(120):
        dp = [dlt(p, i) for i in range(nx)]
        for i in range(nx):
            pv[i] = b[i] * pv[i] + ac[i] * dp[i]
            v[i] -= lam * (dp[i] + pv[i])
        dv = [dlt(v, i) for i in range(nx)]
        for i in range(nx):
            pp[i] = b[i] * pp[i] + ac[i] * dv[i]
            p[i] -= lam * (dv[i] + pp[i])
        s.step()
    assert np.abs(s.p[0, 0] - p).max() <= 1e-13 * np.abs(p).max()
    assert np.abs(s.v[0][0, 0] - v).max() <= 1e-13 * np.abs(v).max()
    assert np.all(s.v[1] == 0) and np.all(s.v[2] == 0)


def _symbol_max():
    """max over theta of 2 sum_l a_l sin(l theta) (the first-derivative symbol)."""
    a = O.weights(4)[0]
    th = np.linspace(0.0, math.pi, 200001)
    s = 2 * sum(a[l] * np.sin(l * th) for l in range(1, 5))
    return float(s.max())


def test_stability_limit_of_the_leapfrog():
    """From the Fourier closed form above, a mode is bounded iff lam^2 S^2 <= 4;
    S^2 <= 3 s_max^2, so lam <= 2 / (sqrt(3) s_max) ~ 0.667 keeps every mode
    bounded.  On a periodic grid whose modes reach the symbol's maximum on
    every axis the oracle stays bounded just below that limit and blows up
    just above it."""
    smax = _symbol_max()
    lim = 2 / (math.sqrt(3) * smax)
    assert 0.666 < lim < 0.668
    n = (14, 14, 14)          # theta = 2 pi 5 / 14 lies near the symbol's maximum
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal((n[2], n[1], n[0]))
    a = O.weights(4)[0]
    sg = max(abs(2 * sum(a[l] * math.sin(l * 2 * math.pi * m / 14) for l in range(1, 5))) for m in range(14))
    peaks = []
    for lam in (0.995 * lim, 1.02 * 2 / (math.sqrt(3) * sg)):
        s = P.PV(n, (0,) * 6, lam, periodic=(1, 1, 1))
        s.p[...] = p0
        for _ in range(300):
            s.step()
        peaks.append(float(np.abs(s.p).max()))
    assert peaks[0] < 100 * np.abs(p0).max()
    assert peaks[1] > 1e6 * np.abs(p0).max()
