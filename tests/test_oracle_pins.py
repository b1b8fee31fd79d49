"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one part of the oracle to something other than itself:
printed values from the paper, closed forms, exact invariants, an
independently assembled sparse-matrix operator, or brute force.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_table(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([float(x) for x in line.split()])
    return rows


# ---------------------------------------------------------------- weights --

@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_oracle_weights_polynomial_exactness(r):
    """P2: D2 of order 2r is exact for monomials of degree <= 2r+1, D1 for
    degree <= 2r; one degree higher is not exact (so the test can fail).
    Monomials x^k on a unit-spaced line centred at 0, checked at the nodes whose
    stencil stays inside the line."""
    n = 2 * r + 3
    g = O.Grid(n=(n, 1, 1), h=(1.0, 1.0, 1.0), dt=1.0, r=r, periodic=(0, 1, 1))
    x = np.arange(n, dtype=np.float64) - n // 2
    interior = slice(r, n - r)
    for deg in range(0, 2 * r + 3):
        f = x ** deg
        df = deg * x ** (deg - 1) if deg >= 1 else np.zeros(n)
        d2f = deg * (deg - 1) * x ** (deg - 2) if deg >= 2 else np.zeros(n)
        F = f.reshape(1, 1, n)
        scale1 = np.abs(df[interior]).max() + 1.0
        scale2 = np.abs(d2f[interior]).max() + 1.0
        e1 = np.abs(O.deriv1(g, 0, F).ravel()[interior] - df[interior]).max() / scale1
        e2 = np.abs(O.deriv2(g, 0, F).ravel()[interior] - d2f[interior]).max() / scale2
        if deg <= 2 * r:
            assert e1 < 1e-10, (r, deg, e1)
        if deg == 2 * r + 1:
            assert e1 > 1e-3, (r, deg, e1)
        if deg <= 2 * r + 1:
            assert e2 < 1e-10, (r, deg, e2)
        if deg == 2 * r + 2:
            assert e2 > 1e-3, (r, deg, e2)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_oracle_derivatives_follow_their_axis(axis):
    """P2 per axis: a degree-8 polynomial along one axis, constant along the
    others; D1/D2 along that axis are exact at interior nodes and the other
    axes' derivatives vanish."""
    n = [14, 15, 16]
    h = [0.5, 0.7, 0.9]
    g = O.Grid(n=n, h=h, dt=1.0, r=4)
    c = np.random.default_rng(axis).uniform(-1, 1, 9)
    coord = (np.arange(n[axis]) - n[axis] / 2) * h[axis]
    shape = [1, 1, 1]
    shape[2 - axis] = n[axis]
    f1 = np.polyval(c, coord).reshape(shape)
    F = np.broadcast_to(f1, g.shape).copy()
    d1 = np.broadcast_to(np.polyval(np.polyder(c), coord).reshape(shape), g.shape)
    d2 = np.broadcast_to(np.polyval(np.polyder(c, 2), coord).reshape(shape), g.shape)
    inner = [slice(4, s - 4) for s in g.shape]
    assert np.allclose(O.deriv1(g, axis, F)[tuple(inner)], d1[tuple(inner)], rtol=1e-9, atol=1e-9)
    assert np.allclose(O.deriv2(g, axis, F)[tuple(inner)], d2[tuple(inner)], rtol=1e-9, atol=1e-8)
    for other in range(3):
        if other != axis:
            # interior along the other axis: constant there, so derivative 0
            sl = [slice(None)] * 3
            sl[2 - other] = slice(4, g.shape[2 - other] - 4)
            fs = np.abs(F).max()
            assert np.abs(O.deriv1(g, other, F)[tuple(sl)]).max() < 1e-13 * fs / h[other]
            assert np.abs(O.deriv2(g, other, F)[tuple(sl)]).max() < 1e-13 * fs / h[other] ** 2


def test_oracle_laplacian_of_constant_and_linear():
    """P2: Lap_h(const) = 0 everywhere on a periodic grid, Lap_h(linear) = 0 at
    interior nodes of a Dirichlet grid."""
    g = O.Grid(n=(12, 13, 14), h=(1.0, 2.0, 3.0), dt=1.0, periodic=(1, 1, 1))
    c = np.full(g.shape, 3.25)
    assert np.abs(O.laplacian(g, c)).max() < 1e-13
    g2 = O.Grid(n=(12, 13, 14), h=(1.0, 2.0, 3.0), dt=1.0)
    z, y, x = np.meshgrid(np.arange(14), np.arange(13), np.arange(12), indexing="ij")
    lin = 0.3 * x - 1.1 * y + 2.0 * z + 0.5
    L = O.laplacian(g2, lin)
    assert np.abs(L[4:-4, 4:-4, 4:-4]).max() < 1e-12


# ------------------------------------------------- P1: paper's printed table --

def _mms_laplacian_error(order, N, m=4):
    g = O.Grid(n=(N, N, N), h=(1.0 / N,) * 3, dt=1.0, r=order // 2, periodic=(1, 1, 1))
    x = np.arange(N) / N
    s = np.sin(2 * np.pi * m * x)
    u = s[:, None, None] * s[None, :, None] * s[None, None, :]
    exact = -3.0 * (2 * np.pi * m) ** 2 * u
    err = O.laplacian(g, u) - exact
    return (np.linalg.norm(err) / np.linalg.norm(exact), np.abs(err).max() / np.abs(exact).max())


@pytest.mark.parametrize("order,N,l2,linf", [tuple(r) for r in _read_table("t6_spatial_convergence.txt")
                                              if r[1] <= 120])
def test_oracle_laplacian_reproduces_printed_convergence(order, N, l2, linf):
    """P1: the paper's spatial-convergence table, reproduced to its 4 printed digits."""
    e2, ei = _mms_laplacian_error(int(order), int(N))
    assert abs(e2 - l2) <= 6e-4 * l2, (order, N, e2, l2)
    assert abs(ei - linf) <= 6e-4 * linf, (order, N, ei, linf)


@pytest.mark.slow
def test_oracle_laplacian_printed_convergence_N240():
    """P1 at N = 240 (order 2 and 4 to 4 digits; order 8 is at FP64 noise level)."""
    rows = [r for r in _read_table("t6_spatial_convergence.txt") if r[1] == 240]
    for order, N, l2, linf in rows:
        e2, ei = _mms_laplacian_error(int(order), int(N))
        tol = 6e-4 if order < 8 else 5e-2
        assert abs(e2 - l2) <= tol * l2, (order, e2, l2)


# --------------------------------------------- P3: exact discrete dispersion --

def _symbol(g, kvec):
    d1, d2 = O.weights(g.r)
    lam = 0.0
    for d in range(3):
        kh = kvec[d] * g.h[d]
        lam += (d2[0] + 2 * sum(d2[l] * math.cos(l * kh) for l in range(1, g.r + 1))) / g.h[d] ** 2
    return lam


def test_oracle_time_loop_exact_discrete_mode():
    """P3: a periodic eigenmode with zero initial velocity evolves as exactly
    cos(n theta) u^0 with cos(theta) = 1 + m lambda_h / 2."""
    N, mode = 16, 2
    g = O.Grid(n=(N, N, N), h=(1.0 / N,) * 3, dt=2.0e-3, periodic=(1, 1, 1))
    v = np.full(g.shape, 3.0)
    x = np.arange(N) / N
    s = np.sin(2 * np.pi * mode * x)
    u0 = s[:, None, None] * s[None, :, None] * s[None, None, :]
    k = 2 * np.pi * mode
    mlam = 9.0 * g.dt ** 2 * _symbol(g, (k, k, k))
    cth = 1.0 + 0.5 * mlam
    st = O.State.zeros(g)
    st.u[:] = u0
    st.um1[:] = cth * u0
    nt = 120
    out = O.forward(g, v, nt, state=st)
    theta = math.acos(cth)
    expect = math.cos(nt * theta) * u0
    assert np.abs(out["state"].u - expect).max() < 1e-11


def test_oracle_time_order_two():
    """P4: halving dt divides the time error by 4 (the paper's printed rate 2.00)."""
    rows = _read_table("t7_time_convergence.txt")
    paper_rates = [math.log2(rows[i][1] / rows[i + 1][1]) for i in range(len(rows) - 1)]
    assert all(abs(r - 2.0) < 0.01 for r in paper_rates)
    N, mode, c, T = 24, 1, 1.0, 0.2
    x = np.arange(N) / N
    s = np.sin(2 * np.pi * mode * x)
    u0 = s[:, None, None] * s[None, :, None] * s[None, None, :]
    om = 2 * np.pi * mode * math.sqrt(3.0) * c
    errs = []
    for dt in (2e-3, 1e-3, 5e-4):
        g = O.Grid(n=(N, N, N), h=(1.0 / N,) * 3, dt=dt, periodic=(1, 1, 1))
        st = O.State.zeros(g)
        st.u[:] = u0
        st.um1[:] = math.cos(om * dt) * u0
        nt = int(round(T / dt))
        out = O.forward(g, np.full(g.shape, c), nt, state=st)
        ex = math.cos(om * nt * dt) * u0
        errs.append(np.linalg.norm(out["state"].u - ex) / np.linalg.norm(ex))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for r in rates:
        assert abs(r - 2.0) < 0.05, (errs, rates)


# ------------------------------------------------ P5: exact energy invariant --

def test_oracle_energy_conserved_without_cpml():
    """P5: with zero Dirichlet faces, no layer and no source,
    E = sum (u^{n+1}-u^n)^2/m - sum u^{n+1} Lap_h u^n is constant."""
    n = (20, 18, 22)
    g = O.Grid(n=n, h=(10.0, 9.0, 11.0), dt=1.0e-3)
    rng = np.random.default_rng(5)
    v = 2000.0 * (1 + 0.2 * rng.uniform(-1, 1, g.shape))
    m = v * v * g.dt ** 2
    z, y, x = np.meshgrid(*[np.arange(s) for s in g.shape], indexing="ij")
    bump = np.exp(-((x - 10) ** 2 + (y - 9) ** 2 + (z - 11) ** 2) / 8.0)
    st = O.State.zeros(g)
    st.u[:] = bump
    st.um1[:] = bump
    S = O.Stepper(g, v)
    E = []
    for _ in range(150):
        un = st.u.copy()
        S.step(st)
        E.append(np.sum((st.u - un) ** 2 / m) - np.sum(st.u * O.laplacian(g, un)))
    E = np.array(E)
    assert E[0] > 0
    assert np.abs(E - E[0]).max() / E[0] < 1e-11


# ---------------------------------------- P6: FFT recurrence with a source --

def test_oracle_point_source_matches_fourier_recurrence():
    """P6: periodic homogeneous box; every Fourier mode obeys
    u_k^{n+1} = (2 + m lambda_k) u_k^n - u_k^{n-1} + m f^n s_k."""
    n = (12, 10, 14)
    h = (10.0, 12.0, 8.0)
    g = O.Grid(n=n, h=h, dt=1.2e-3, periodic=(1, 1, 1))
    vel = 1800.0
    m = vel * vel * g.dt ** 2
    nt = 80
    w = np.sin(np.arange(nt) * 0.21) * np.exp(-0.03 * np.arange(nt))
    src = np.array([[3, 7, 5]])
    out = O.forward(g, np.full(g.shape, vel), nt, src_ijk=src, src_w=w)
    nz, ny, nx = g.shape
    d1, d2 = O.weights(4)

    def sym1(nn, hh):
        k = 2 * np.pi * np.fft.fftfreq(nn)
        return (d2[0] + 2 * sum(d2[l] * np.cos(l * k) for l in range(1, 5))) / hh ** 2

    lam = sym1(nz, h[2])[:, None, None] + sym1(ny, h[1])[None, :, None] + sym1(nx, h[0])[None, None, :]
    delta = np.zeros(g.shape)
    delta[5, 7, 3] = 1.0 / (h[0] * h[1] * h[2])
    sk = np.fft.fftn(delta)
    a, b = np.zeros(g.shape, complex), np.zeros(g.shape, complex)
    for i in range(nt):
        a, b = (2 + m * lam) * a - b + m * w[i] * sk, a
    ref = np.real(np.fft.ifftn(a))
    assert np.abs(out["state"].u - ref).max() <= 1e-10 * np.abs(ref).max()


# --------------------------------------- P7: band-limited Green's function --

def test_oracle_greens_function_homogeneous():
    """P7: homogeneous medium, before boundary arrivals the trace at distance r
    is w(t - r/v) / (4 pi r) (3-D scalar wave Green's function)."""
    n = 72
    h = 5.0
    vel = 2000.0
    dt = 0.5 * h / (vel * math.sqrt(3.0))
    f0 = 20.0
    nt = 230
    t = np.arange(nt + 2) * dt
    t0 = 1.5 / f0
    a = np.pi * f0 * (t - t0)
    w = (1 - 2 * a * a) * np.exp(-a * a)
    c = n // 2
    offs = [(8, 0, 0), (0, 0, 8), (6, 6, 0)]
    rec = np.array([[c + o[0], c + o[1], c + o[2]] for o in offs])
    g = O.Grid(n=(n, n, n), h=(h, h, h), dt=dt, cpml=(12,) * 6, vref=vel)
    out = O.forward(g, np.full(g.shape, vel), nt, src_ijk=np.array([[c, c, c]]), src_w=w, rec_ijk=rec)
    for j, o in enumerate(offs):
        r = h * math.sqrt(sum(x * x for x in o))
        tt = t[1:nt + 1] - r / vel           # trace[n] = u^{n+1} = u(t_{n+1})
        aa = np.pi * f0 * (tt - t0)
        ref = (1 - 2 * aa * aa) * np.exp(-aa * aa) / (4 * np.pi * r)
        err = np.linalg.norm(out["traces"][:, j] - ref) / np.linalg.norm(ref)
        assert err < 2e-2, (o, err)


# ----------------------------------------------------- CPML profile values --

def test_oracle_profile_special_values():
    """Profile coefficients at rho = 1, 1/2 and 0 reduce to short closed forms:
    rho=1: sigma=smax, kappa=kmax, alpha=0 -> b=exp(-smax dt/kmax), a=(b-1)/kmax;
    rho=0: a=0, kinv=1, dkinv=0."""
    L, hx, v, dt, R = 10, 10.0, 2000.0, 1e-3, 1e-8
    g = O.Grid(n=(40, 30, 30), h=(hx, 10.0, 10.0), dt=dt, cpml=(L, L, 0, 0, 0, 0), vref=v, R=R)
    p = O.profile(g, 0)
    smax = 4 * v * math.log(1e8) / (2 * L * hx)          # -(q+1) v ln R / (2 L h)
    # outermost nodes
    for i in (0, 39):
        assert p["rho"][i] == 1.0
        b = math.exp(-smax * dt / 5.0)
        assert math.isclose(p["b"][i], b, rel_tol=1e-14)
        assert math.isclose(p["a"][i], (b - 1) / 5.0, rel_tol=1e-13)
        assert math.isclose(p["kinv"][i], 0.2, rel_tol=1e-15)
    # rho = 1/2 at i = 5 (low face) and i = 34 (high face)
    for i, sgn in ((5, +1), (34, -1)):
        assert p["rho"][i] == 0.5
        sig, kap, alp = smax / 8, 1 + 4 / 8, 0.05 * smax / 2
        b = math.exp(-(sig / kap + alp) * dt)
        assert math.isclose(p["b"][i], b, rel_tol=1e-14)
        assert math.isclose(p["a"][i], sig * (b - 1) / (kap * (sig + kap * alp)), rel_tol=1e-13)
        # d(1/kappa)/dx = -12 rho^2 rho'(x) / kappa^2, rho' = -+1/(L h)
        assert math.isclose(p["dkinv"][i], sgn * 12 * 0.25 / (L * hx) / kap ** 2, rel_tol=1e-13)
    # interior nodes
    for i in range(10, 30):
        assert p["rho"][i] == 0 and p["a"][i] == 0 and p["kinv"][i] == 1 and p["dkinv"][i] == 0
    # layer extent: rho > 0 exactly on the first and last L nodes
    assert list(np.nonzero(p["rho"] > 0)[0]) == list(range(10)) + list(range(30, 40))
    # a vanishes where sigma does
    assert np.all((p["a"] != 0) == (p["rho"] > 0))


def test_oracle_dkinv_matches_profile_slope():
    """The analytic d(1/kappa)/dx agrees with the slope of the sampled 1/kappa
    (central difference of the node values, O(1/L^2) agreement)."""
    L, hx = 40, 5.0
    g = O.Grid(n=(100, 9, 9), h=(hx, 5.0, 5.0), dt=1e-3, cpml=(L, L, 0, 0, 0, 0), vref=1500.0)
    p = O.profile(g, 0)
    fd = (p["kinv"][2:] - p["kinv"][:-2]) / (2 * hx)
    an = p["dkinv"][1:-1]
    sel = (p["rho"][1:-1] > 0.1) & (p["rho"][1:-1] < 0.95)
    assert np.abs(fd[sel] - an[sel]).max() < 3e-3 * np.abs(an[sel]).max()


# ------------------------------ P9: independent sparse-matrix assembly (16^3) --

def _sparse_step_matrix(g, m):
    import scipy.sparse as sp

    d1w, d2w = O.weights(4)
    nx, ny, nz = [int(x) for x in g.n]
    N = nx * ny * nz

    def D1(n, h):
        M = sp.lil_matrix((n, n))
        for i in range(n):
            for l in range(1, 5):
                if i + l < n:
                    M[i, i + l] += d1w[l] / h
                if i - l >= 0:
                    M[i, i - l] -= d1w[l] / h
        return M.tocsr()

    def D2(n, h):
        M = sp.lil_matrix((n, n))
        for i in range(n):
            M[i, i] += d2w[0] / h ** 2
            for l in range(1, 5):
                if i + l < n:
                    M[i, i + l] += d2w[l] / h ** 2
                if i - l >= 0:
                    M[i, i - l] += d2w[l] / h ** 2
        return M.tocsr()

    I = [sp.identity(nx), sp.identity(ny), sp.identity(nz)]

    def lift(A, d):
        mats = [I[2], I[1], I[0]]          # kron order: z, y, x (x fastest)
        mats[2 - d] = A
        return sp.kron(mats[0], sp.kron(mats[1], mats[2])).tocsr()

    def diag_axis(vals, d):
        return lift(sp.diags(vals), d)

    Dd1 = [lift(D1(int(g.n[d]), g.h[d]), d) for d in range(3)]
    Dd2 = [lift(D2(int(g.n[d]), g.h[d]), d) for d in range(3)]
    P = [O.profile(g, d) for d in range(3)]
    S = [diag_axis((P[d]["rho"] > 0).astype(float), d) for d in range(3)]
    A = [diag_axis(P[d]["a"], d) for d in range(3)]
    B = [diag_axis(P[d]["b"], d) for d in range(3)]
    K = [diag_axis(P[d]["kinv"], d) for d in range(3)]
    dK = [diag_axis(P[d]["dkinv"], d) for d in range(3)]
    M = sp.diags(m.ravel())
    Z = sp.csr_matrix((N, N))
    Id = sp.identity(N, format="csr")
    # state blocks: u, um1, psi_x, psi_y, psi_z, zeta_x, zeta_y, zeta_z
    # psi'_d = S_d (B_d psi_d + A_d D1_d u)
    psi_new = [[S[d] @ A[d] @ Dd1[d], Z] + [S[d] @ B[d] if e == d else Z for e in range(3)] + [Z, Z, Z]
               for d in range(3)]
    # eta_d = K_d D2_d u + dK_d D1_d u + D1_d psi'_d
    eta = []
    for d in range(3):
        row = [K[d] @ Dd2[d] + dK[d] @ Dd1[d]] + [Z] * 7
        row = [row[j] + Dd1[d] @ psi_new[d][j] for j in range(8)]
        eta.append(row)
    # zeta'_d = S_d (B_d zeta_d + A_d eta_d)
    zeta_new = []
    for d in range(3):
        row = [S[d] @ A[d] @ eta[d][j] for j in range(8)]
        row[5 + d] = row[5 + d] + S[d] @ B[d]
        zeta_new.append(row)
    # u' = 2u - um1 + M sum_d (K_d eta_d + zeta'_d)
    u_new = [2 * Id, -Id] + [Z] * 6
    for d in range(3):
        u_new = [u_new[j] + M @ (K[d] @ eta[d][j] + zeta_new[d][j]) for j in range(8)]
    rows = [u_new, [Id] + [Z] * 7] + psi_new + zeta_new
    return sp.bmat(rows, format="csr"), S


def _small_cpml_grid():
    return O.Grid(n=(16, 15, 14), h=(10.0, 12.0, 9.0), dt=1.1e-3, cpml=(3, 4, 2, 3, 4, 2), vref=2400.0)


def test_oracle_step_matches_sparse_matrix_bruteforce():
    """P9: one oracle step equals the step operator assembled independently from
    Kronecker products of 1-D D1/D2 matrices and diagonal profile matrices."""
    g = _small_cpml_grid()
    rng = np.random.default_rng(9)
    v = 2000 + 400 * rng.uniform(size=g.shape)
    m = v * v * g.dt ** 2
    T, S = _sparse_step_matrix(g, m)
    N = g.npts
    x = rng.standard_normal(8 * N)
    for d in range(3):          # memory variables live only inside each layer
        x[(2 + d) * N:(3 + d) * N] *= S[d].diagonal()
        x[(5 + d) * N:(6 + d) * N] *= S[d].diagonal()
    st = O.State(x[:N].reshape(g.shape).copy(), x[N:2 * N].reshape(g.shape).copy(),
                 x[2 * N:5 * N].reshape((3,) + g.shape).copy(), x[5 * N:].reshape((3,) + g.shape).copy())
    O.Stepper(g, v).step(st)
    y = T @ x
    got = np.concatenate([st.u.ravel(), st.um1.ravel(), st.psi.ravel(), st.zeta.ravel()])
    assert np.abs(got - y).max() <= 1e-13 * np.abs(y).max()


def test_oracle_adjoint_step_is_matrix_transpose():
    """P9 transposed: the oracle's adjoint step equals T^T applied to the
    adjoint state (leapfrog form: slot 1 carries -lambda)."""
    g = _small_cpml_grid()
    rng = np.random.default_rng(10)
    v = 2000 + 400 * rng.uniform(size=g.shape)
    m = v * v * g.dt ** 2
    T, S = _sparse_step_matrix(g, m)
    N = g.npts
    y = rng.standard_normal(8 * N)
    for d in range(3):
        y[(2 + d) * N:(3 + d) * N] *= S[d].diagonal()
        y[(5 + d) * N:(6 + d) * N] *= S[d].diagonal()
    ref = T.T @ y
    lam = y[:N].reshape(g.shape).copy()
    lamp = -y[N:2 * N].reshape(g.shape).copy()
    psib = y[2 * N:5 * N].reshape((3,) + g.shape).copy()
    zetab = y[5 * N:].reshape((3,) + g.shape).copy()
    O.Stepper(g, v).adjoint_step(lam, lamp, psib, zetab)
    got = np.concatenate([lam.ravel(), -lamp.ravel(), psib.ravel(), zetab.ravel()])
    # memory-variable adjoints outside the layers are irrelevant (masked states)
    for d in range(3):
        for blk in (2 + d, 5 + d):
            msk = S[d].diagonal()
            got[blk * N:(blk + 1) * N] *= msk
            ref[blk * N:(blk + 1) * N] *= msk
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_oracle_source_adds_m_f_at_one_node():
    """Source: u^{n+1} gains exactly m[s] A w_n / (hx hy hz) at node s."""
    g = _small_cpml_grid()
    rng = np.random.default_rng(11)
    v = 2000 + 400 * rng.uniform(size=g.shape)
    st = O.State.zeros(g)
    st.u[:] = rng.standard_normal(g.shape)
    st2 = st.copy()
    S = O.Stepper(g, v)
    S.step(st)
    S.step(st2, src_index=int(O.flat_index(g, [[5, 6, 7]])[0]), src_amp=3.5)
    d = st2.u - st.u
    expect = v[7, 6, 5] ** 2 * g.dt ** 2 * 3.5 / (10.0 * 12.0 * 9.0)
    assert math.isclose(d[7, 6, 5], expect, rel_tol=1e-12)
    d[7, 6, 5] = 0
    assert np.abs(d).max() == 0


# ------------------------------------------ P10: kappa = 1 special case --

def test_oracle_kappa_one_reduces_to_pasalic_mcgarry_1d():
    """P10: with kappa_max = 1 the layer update is the published acoustic CPML
    of Pasalic and McGarry: p_tt = v^2 (p_xx + d(psi)/dx + zeta),
    psi <- b psi + a p_x, zeta <- b zeta + a (p_xx + d(psi)/dx).
    Checked against a 1-D numpy implementation (a line with periodic y, z of size 1)."""
    nx, L, h, vel = 80, 12, 10.0, 2000.0
    dt = 0.5 * h / (vel * math.sqrt(3))
    g = O.Grid(n=(nx, 1, 1), h=(h, h, h), dt=dt, periodic=(0, 1, 1), cpml=(L, L, 0, 0, 0, 0),
               kappa_max=1.0, vref=vel)
    p = O.profile(g, 0)
    assert np.all(p["kinv"] == 1.0) and np.all(p["dkinv"] == 0.0)
    nt = 150
    w = np.exp(-((np.arange(nt) - 30) / 8.0) ** 2)
    out = O.forward(g, np.full(g.shape, vel), nt, src_ijk=np.array([[20, 0, 0]]), src_w=w)
    d1w, d2w = O.weights(4)

    def Dx(f, wts, second):
        fp = np.concatenate([np.zeros(4), f, np.zeros(4)])
        out_ = (wts[0] * f) if second else np.zeros_like(f)
        for l in range(1, 5):
            if second:
                out_ = out_ + wts[l] * (fp[4 + l:4 + l + nx] + fp[4 - l:4 - l + nx])
            else:
                out_ = out_ + wts[l] * (fp[4 + l:4 + l + nx] - fp[4 - l:4 - l + nx])
        return out_ / (h * h if second else h)

    inl = p["rho"] > 0
    u, um, psi, zeta = np.zeros(nx), np.zeros(nx), np.zeros(nx), np.zeros(nx)
    mm = vel * vel * dt * dt
    for n in range(nt):
        psi = np.where(inl, p["b"] * psi + p["a"] * Dx(u, d1w, False), 0.0)
        inner = Dx(u, d2w, True) + Dx(psi, d1w, False)
        zeta = np.where(inl, p["b"] * zeta + p["a"] * inner, 0.0)
        f = np.zeros(nx)
        f[20] = w[n] / h ** 3
        u, um = 2 * u - um + mm * (inner + zeta) + mm * f, u
    got = out["state"].u.ravel()
    assert np.abs(got - u).max() <= 1e-11 * np.abs(u).max()


# ------------------------------------------------- P8 / P11: absorption --

def _energy(S, g, u_new, u_old):
    return float(np.sum((u_new - u_old) ** 2 / S.m) - np.sum(u_new * O.laplacian(g, u_old)))


def test_oracle_cpml_energy_decays():
    """P8: after the source stops, the discrete energy (sampled every 50 steps)
    does not grow while it is above 1e-6 of its peak, and falls by orders of
    magnitude; without the layer it is conserved instead."""
    n, L, h, vel = 40, 10, 10.0, 2000.0
    dt = 0.5 * h / (vel * math.sqrt(3))
    nt = 900
    t = np.arange(nt) * dt
    f0 = 25.0
    a = np.pi * f0 * (t - 1.5 / f0)
    w = (1 - 2 * a * a) * np.exp(-a * a)
    for width in (L, 0):
        g = O.Grid(n=(n, n, n), h=(h,) * 3, dt=dt, cpml=(width,) * 6, vref=vel)
        S = O.Stepper(g, np.full(g.shape, vel))
        st = O.State.zeros(g)
        E = []
        for i in range(nt):
            uo = st.u.copy()
            S.step(st, src_index=int(O.flat_index(g, [[20, 20, 20]])[0]), src_amp=w[i])
            if i % 50 == 49:
                E.append(_energy(S, g, st.u, uo))
        E = np.array(E)
        after = E[3:]                       # source is negligible after ~2.5 t0
        if width:
            peak = E.max()
            for k in range(1, len(after)):
                if after[k - 1] > 1e-6 * peak:
                    assert after[k] <= after[k - 1] * (1 + 1e-9), (k, after)
            assert after[-1] < 1e-5 * peak
        else:
            assert np.abs(after - after[0]).max() < 1e-9 * after[0]


def test_oracle_cpml_reflection_falls_with_width():
    """P11 (qualitative, as the paper's reflection table): the reflected
    amplitude at a receiver near the face falls monotonically as the layer
    widens (normal incidence along each axis in turn)."""
    h, vel = 10.0, 2000.0
    dt = 0.5 * h / (vel * math.sqrt(3))
    nt = 400
    t = np.arange(nt) * dt
    f0 = 20.0
    a = np.pi * f0 * (t - 1.5 / f0)
    w = (1 - 2 * a * a) * np.exp(-a * a)
    for axis in range(3):
        def run(n_ax, width, src_pos, rec_pos):
            n = [1, 1, 1]
            n[axis] = n_ax
            per = [1, 1, 1]
            per[axis] = 0
            cp = [0] * 6
            cp[2 * axis] = cp[2 * axis + 1] = width
            g = O.Grid(n=n, h=(h,) * 3, dt=dt, periodic=per, cpml=cp, vref=vel)
            s = [0, 0, 0]
            s[axis] = src_pos
            r = [0, 0, 0]
            r[axis] = rec_pos
            out = O.forward(g, np.full(g.shape, vel), nt, src_ijk=np.array([s]), src_w=w,
                            rec_ijk=np.array([r]))
            return out["traces"][:, 0]
        ratios = []
        for width in (0, 6, 12, 24):
            n_ax = 200 + 2 * width
            tr = run(n_ax, width, width + 150, width + 180)
            ref = run(2000, 0, 1000 + 150, 1000 + 180)   # same offsets, faces far away
            ratios.append(np.abs(tr - ref).max() / np.abs(ref).max())
        assert ratios[0] > 0.5, ratios
        assert all(ratios[i + 1] < ratios[i] for i in range(3)), (axis, ratios)
        assert ratios[-1] < 1e-2, ratios


# -------------------------------------------- adjoint and gradient pins --

def test_oracle_gradient_matches_central_differences():
    """dJ/dv from the reverse sweep agrees with central finite differences of
    J = 1/2 |d(v) - d_obs|^2 along random smooth directions."""
    g = O.Grid(n=(24, 22, 20), h=(10.0, 10.0, 10.0), dt=0.0, cpml=(5,) * 6)
    rng = np.random.default_rng(12)
    v = 2000 + 300 * rng.uniform(size=g.shape)
    g.dt = 0.5 * 10.0 / (v.max() * 1.2 * math.sqrt(3))
    g.vref = float(v.max())
    nt = 90
    t = np.arange(nt) * g.dt
    a = np.pi * 25 * (t - 0.06)
    w = (1 - 2 * a * a) * np.exp(-a * a)
    src = np.array([[12, 11, 10]])
    rec = np.array([[6, 6, 6], [17, 15, 13], [12, 5, 14], [8, 16, 9]])
    vt = v * (1 + 0.02 * rng.uniform(-1, 1, g.shape))
    dobs = O.forward(g, vt, nt, src, w, rec)["traces"]
    fwd = O.forward(g, v, nt, src, w, rec, keep_lapf=True)
    resid = fwd["traces"] - dobs
    grad = O.gradient(g, v, nt, src, w, rec, resid, fwd=fwd)

    def J(vv):
        return O.misfit(O.forward(g, vv, nt, src, w, rec)["traces"], dobs)

    for k in range(2):
        dv = rng.standard_normal(g.shape)
        an = float(np.sum(grad * dv))
        errs = []
        for e in (1e-4, 1e-5):
            eps = e * v.mean() / np.abs(dv).max()
            fd = (J(v + eps * dv) - J(v - eps * dv)) / (2 * eps)
            errs.append(abs(fd - an) / abs(an))
        # central differences: the remaining gap is O(eps^2) truncation
        assert errs[1] < 1e-7, errs
        assert errs[1] < errs[0] / 30, errs


def test_oracle_dot_product_multistep():
    """Adjoint dot-product test over a whole run: <F x0, y> = <x0, F^T y> where F
    maps the initial u^0 to all receiver traces (linear, source off)."""
    g = _small_cpml_grid()
    rng = np.random.default_rng(13)
    v = 2000 + 400 * rng.uniform(size=g.shape)
    nt = 40
    rec = np.array([[3, 3, 3], [12, 10, 9], [8, 7, 2]])
    x0 = rng.standard_normal(g.shape)
    st = O.State.zeros(g)
    st.u[:] = x0
    tr = O.forward(g, v, nt, rec_ijk=rec, state=st)["traces"]
    y = rng.standard_normal(tr.shape)
    S = O.Stepper(g, v)
    lam, lamp = np.zeros(g.shape), np.zeros(g.shape)
    psib, zetab = np.zeros((3,) + g.shape), np.zeros((3,) + g.shape)
    idx = O.flat_index(g, rec)
    for n in range(nt - 1, -1, -1):
        np.add.at(lam.reshape(-1), idx, y[n])
        S.adjoint_step(lam, lamp, psib, zetab)
    # after the sweep lam is the adjoint of u^0 in slot 0
    lhs = float(np.sum(tr * y))
    rhs = float(np.sum(x0 * lam))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
