"""Benchmark of the hot path on one MI355X.

Workload (the headline one): 512^3 grid with 20-cell CPML on all faces, seeded
layered model (8-12 layers, 1500-4500 m/s, Gaussian-smoothed), Ricker 10 Hz
at the centre, h = 10 m, dt at Courant number 0.5.  A step is one leapfrog
step of the whole grid: psi pre-pass, wavefield update (interior + layers),
source and receiver gather.  Metric: million output points per second,
nx*ny*nz*steps / time, plus the HBM roofline of the dominant kernel.

Prints one JSON line.  With --gpus above 1 it exits: this build runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, 8 TB/s


def slab_points(n, cpml):
    """Points inside each axis' layer (rho > 0), summed over the axes."""
    nx, ny, nz = n
    tot = 0
    for d, (lo, hi) in enumerate([(cpml[0], cpml[1]), (cpml[2], cpml[3]), (cpml[4], cpml[5])]):
        other = (ny * nz, nx * nz, nx * ny)[d]
        tot += (lo + hi) * other
    return tot


def update_kernel_bytes(n, cpml, field_bytes=4):
    """Algorithmic bytes of one update launch: read u^n, u^{n-1}, m and write
    u^{n+1} per point; per layer point and axis read psi, read+write zeta."""
    N = n[0] * n[1] * n[2]
    return (3 * field_bytes + 4) * N + 12 * slab_points(n, cpml)


def step_bytes(n, cpml, field_bytes=4):
    """Algorithmic bytes of a whole step (16 B/point + 16 B per layer point-axis in FP32)."""
    N = n[0] * n[1] * n[2]
    return (3 * field_bytes + 4) * N + 16 * slab_points(n, cpml)


def time_gpu(w, K, W, variant, storage=0, graph=True):
    import numpy as np
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, variant=variant, storage=storage)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
    p.set_receivers(0, w.rec)
    p.record(0, K + W + 2)
    W += W % 2
    if graph:
        p.step(K, graph=True)            # capture once (phase 0), untimed
        torch.cuda.synchronize()
        p.reset()
    p.step(W)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(p.stream)
    p.step(K, graph=graph)
    e1.record(p.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    p.check_finite()
    # per-kernel timing pass (eager; HIP events around every launch on the library's stream)
    Kt = min(K, 200)
    p.set_timing(True)
    p.step(Kt)
    upd = p.timing(0)
    psi = p.timing(1)
    rec = p.timing(2)
    p.set_timing(False)
    p.close()
    return ms, upd, psi, rec


def cpu_baseline(w, steps=2):
    """The FP64 oracle on the same workload: `steps` full steps after one untimed step."""
    import numpy as np

    from oracle import oracle as O

    v = w.v.astype(np.float32).astype(np.float64)
    g = O.Grid(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, vref=float(v.max()))
    S = O.Stepper(g, v)
    st = O.State.zeros(g)
    src = int(O.flat_index(g, w.src)[0])
    S.step(st, src, float(w.wavelet[0]))
    t0 = time.perf_counter()
    for n in range(1, steps + 1):
        S.step(st, src, float(w.wavelet[n]))
    dt = time.perf_counter() - t0
    return dict(value=round(w.npts * steps / dt / 1e6, 3), unit="Mpts/s", cores=O.threads(), kind="oracle",
                sample="%d full steps of the %dx%dx%d workload (FP64 C oracle, OpenMP), after 1 untimed step"
                % (steps, w.n[0], w.n[1], w.n[2]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variant", type=int, default=0, help="0 auto, 1 naive, 2 z-march, 3 temporal blocking")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--compare", action="store_true", help="also time the other kernel variants")
    ap.add_argument("--eager", action="store_true", help="launch every step eagerly (no HIP graph)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration run)")
    args = ap.parse_args()
    if args.copy_probe:
        import torch

        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    K, W = args.steps, args.warmup
    n = (args.n, args.n, args.n)
    w = synth.layered(n_xyz=n, nt=K + W + 2)
    print("bench: layered %s, %d+%d steps" % (str(n), W, K), file=sys.stderr, flush=True)
    ms, upd, psi, rec = time_gpu(w, K, W, args.variant, graph=not args.eager)
    N = w.npts
    value = N * K / (ms / 1e3) / 1e6
    upd_bytes = update_kernel_bytes(w.n, w.cpml)
    achieved = upd_bytes / (upd[0] / 1e3) / 1e9
    out = {
        "metric": "Mpts/s (output points/sec) + % HBM peak, FP32 vs FP16-storage at stated error",
        "value": round(value, 1),
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "layered %dx%dx%d, 20-cell CPML on 6 faces, Ricker 10 Hz, FP32 fields" % n,
                   "grid": list(n), "cpml": 20, "variant": args.variant, "graph": not args.eager},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": "k_zmarch<float> (wavefield update)",
                     "kernel_ms": round(upd[0], 5), "algorithmic_bytes_per_launch": upd_bytes},
        "step_algorithmic_gbs": round(step_bytes(w.n, w.cpml) / (ms / K / 1e3) / 1e9, 1),
        "kernel_ms": {"update": round(upd[0], 5), "psi": round(psi[0], 5), "record": round(rec[0], 5)},
    }
    if args.compare:
        var = {}
        for name, vv in (("naive", 1), ("zmarch", 2)):
            m2, u2, _, _ = time_gpu(w, min(K, 200), W, vv, graph=not args.eager)
            var[name] = round(N * min(K, 200) / (m2 / 1e3) / 1e6, 1)
        out["variants_mpts"] = var
    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
