"""Write cpml_reflection_oracle.npz: the FP64 oracle's receiver traces for the
layer reflection study (normal incidence on the low face of each axis, layer
widths 0, 8, 12, 16 and 24, and one reference run per axis whose low face is
out of reach), on the inputs synth.reflection_case defines.

Calls only the oracle and the input generators.  Run from the repository root:
    python tests/golden/make_cpml_reflection_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cpml_reflection_oracle.npz")


def oracle_traces(w):
    v = w.v.astype(np.float32).astype(np.float64)
    g = O.Grid(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, vref=float(v.max()))
    wav = w.wavelet.astype(np.float32).astype(np.float64)
    return O.forward(g, v, w.nt, w.src, wav, w.rec)["traces"]


def main():
    out = {}
    for axis in range(3):
        for L in synth.REFL_WIDTHS:
            w = synth.reflection_case(axis, L)
            out[w.name] = oracle_traces(w)
            print(w.name, flush=True)
        w = synth.reflection_case(axis, 0, reference=True)
        out[w.name] = oracle_traces(w)
        print(w.name, flush=True)
    np.savez_compressed(OUT, **out)
    for axis in "xyz":
        ref = out["refl_%s_ref" % axis][:, 0]
        print(axis, " ".join("L%d %.3e" % (L, synth.reflection_ratio(out["refl_%s_L%d" % (axis, L)][:, 0], ref))
                             for L in synth.REFL_WIDTHS))


if __name__ == "__main__":
    main()
