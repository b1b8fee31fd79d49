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
