"""The stored oracle traces of the layer reflection study
(tests/golden/cpml_reflection_oracle.npz, written by
make_cpml_reflection_reference.py from the oracle alone) hold what the
oracle computes for synth.reflection_case's inputs, and obey what the
geometry fixes independently of the layer:

* the first steps of a run (before any wave has returned from the low face)
  recomputed here with the oracle equal the stored ones;
* the three axes give the same traces (the problem is the same up to a
  relabelling of the axes: equal spacings, uniform medium);
* with no layer (zero Dirichlet face) the reflection is the wall's: close to
  the image-source ratio, direct distance over image distance (20/30), the
  wide stencil's zero frame making the discrete wall an imperfect mirror;
* the reflection falls strictly with the layer width.
"""
import os

import numpy as np

import synth
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cpml_reflection_oracle.npz")


def _ratios(d, a):
    ref = d["refl_%s_ref" % a][:, 0]
    return [synth.reflection_ratio(d["refl_%s_L%d" % (a, L)][:, 0], ref) for L in synth.REFL_WIDTHS]


def test_stored_traces_are_the_oracles():
    d = np.load(GOLDEN)
    w = synth.reflection_case(0, 8)
    nt = 160      # the incident peak has passed the first receiver; the low face's return has not arrived
    v = w.v.astype(np.float32).astype(np.float64)
    g = O.Grid(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, vref=float(v.max()))
    tr = O.forward(g, v, nt, w.src, w.wavelet.astype(np.float32).astype(np.float64), w.rec)["traces"]
    assert np.abs(tr).max() > 1e-3 * np.abs(d[w.name]).max()
    np.testing.assert_allclose(tr, d[w.name][:nt], rtol=0, atol=1e-13 * np.abs(tr).max())


def test_axes_agree_and_reflection_falls_with_width():
    d = np.load(GOLDEN)
    for L in list(synth.REFL_WIDTHS) + ["ref"]:
        key = "L%d" % L if L != "ref" else "ref"
        x, y, z = (d["refl_%s_%s" % (a, key)] for a in "xyz")
        scale = np.abs(x).max()
        assert np.abs(x - y).max() <= 1e-12 * scale and np.abs(x - z).max() <= 1e-12 * scale, key
    r = _ratios(d, "x")
    assert abs(r[0] - 20.0 / 30.0) < 0.05, r[0]
    assert all(r[i + 1] < r[i] for i in range(len(r) - 1)), r
    assert r[-1] < 1e-3 * r[0], r
