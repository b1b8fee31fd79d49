"""Write the FP64 oracle reference for the 16-bit-storage error statement.

Workload: central 160^3 crop of the seeded 768^3 Gaussian-blob model, own
20-cell layers on all faces, Ricker 12 Hz at the crop centre, 1500 steps,
dt from the full model's velocity ceiling (Courant number 0.5).
Output (tests/golden/blob160_oracle.npz):
  traces  float64 [1500][16]   receiver traces
  planes  float32 [15][160][160] the centre z-plane every 100 steps
Calls only oracle/ and the synthetic input generators.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "blob160_oracle.npz")
NT, EVERY = 1500, 100


def main():
    w = synth.blob(crop=160, nt=NT)
    v = w.v.astype(np.float32).astype(np.float64)
    g = O.Grid(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, vref=float(v.max()))
    S = O.Stepper(g, v)
    st = O.State.zeros(g)
    src = int(O.flat_index(g, w.src)[0])
    rec = O.flat_index(g, w.rec)
    traces = np.zeros((NT, rec.size))
    planes = []
    t0 = time.time()
    for n in range(NT):
        S.step(st, src, float(w.wavelet[n]))
        traces[n] = st.u.reshape(-1)[rec]
        if (n + 1) % EVERY == 0:
            planes.append(st.u[w.n[2] // 2].astype(np.float32))
            print("step %d  %.0fs" % (n + 1, time.time() - t0), flush=True)
    np.savez_compressed(OUT, traces=traces, planes=np.array(planes), rec=w.rec, dt=w.dt, vref=float(v.max()))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
