"""Benchmark of the hot path on one MI355X.

Workload (the headline one): 512^3 grid with 20-cell CPML on all faces, seeded
layered model (8-12 layers, 1500-4500 m/s, Gaussian-smoothed), Ricker 10 Hz
at the centre, h = 10 m, dt at Courant number 0.5.  A step is one leapfrog
step of the whole grid: psi pre-pass, wavefield update (interior + layers),
source and receiver gather.  Metric: million output points per second,
nx*ny*nz*steps / time, plus the HBM roofline of the dominant kernel.

Prints one JSON line.  With --gpus above 1 it exits: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
COPY_CEILING_GBS = 5090.0   # plain 1 GiB device copy, read + write (copy_1GiB_counters.txt)
STREAM_CEILING_GBS = 5855.0  # o = a + b * c over 400 MiB FP32 arrays: the interior's 3-read 1-write mix, this
                             # library's one-shot-block kernel (--leg stream_ceiling;
                             # stream_probe_kernel_400MiB_kernel_trace.txt; torch's addcmul: 5.73 TB/s)


def slab_points_axis(n, cpml, d):
    """Points inside axis d's layers (rho_d > 0)."""
    nx, ny, nz = n
    return (cpml[2 * d] + cpml[2 * d + 1]) * (ny * nz, nx * nz, nx * ny)[d]


def slab_points(n, cpml):
    """Points inside each axis' layer (rho > 0), summed over the axes."""
    return sum(slab_points_axis(n, cpml, d) for d in range(3))


def x_range(nx, lo, hi, tile=32):
    """The z-march's x range [a, b): outside the x bands, narrowed to whole
    32-point band tiles where a band fits one (the low bound to 32, the high
    one to max(b rounded down to a multiple of 32, nx - 32)), unless that would
    make the range empty."""
    a = min(lo + 4, nx) if lo > 0 else 0
    b = max(nx - hi - 4, a) if hi > 0 else nx
    a2, b2 = a, b
    if lo > 0 and a <= tile:
        a2 = tile
    if hi > 0 and nx - b <= tile:
        b2 = max(b // tile * tile, nx - tile)
    return (a2, b2) if a2 <= b2 else (a, b)


def band_split(n, cpml):
    """(points the z-march updates, points of the band boxes): the band of an
    axis is its layer plus the 4-cell margin the psi derivative reaches, and
    along x the band boxes are widened to whole tiles (x_range)."""
    a, b = x_range(n[0], cpml[0], cpml[1])
    inner = b - a
    for d in (1, 2):
        lo, hi = cpml[2 * d], cpml[2 * d + 1]
        a = min(lo + 4, n[d]) if lo > 0 else 0
        b = max(n[d] - hi - 4, a) if hi > 0 else n[d]
        inner *= b - a
    N = n[0] * n[1] * n[2]
    return inner, N - inner


def interior_kernel_bytes(n, cpml, field_bytes=4):
    """Algorithmic bytes of one z-march launch (points outside every band):
    read u^n, u^{n-1}, m and write u^{n+1} per point."""
    return (3 * field_bytes + 4) * band_split(n, cpml)[0]


def band_kernel_bytes(n, cpml, field_bytes=4):
    """Algorithmic bytes of one band launch (layer memory of x and z advanced
    in the kernel): the four arrays per band point, a read + write of zeta per
    layer point and axis, a read + write of psi_x and psi_z, a read of psi_y."""
    sx, sy, sz = (slab_points_axis(n, cpml, d) for d in range(3))
    return (3 * field_bytes + 4) * band_split(n, cpml)[1] + 8 * (sx + sy + sz) + 8 * (sx + sz) + 4 * sy


def psi_kernel_bytes(n, cpml, field_bytes=4):
    """Algorithmic bytes of one psi pre-pass (psi_y only): per y-layer point
    read u, read and write psi_y."""
    return (field_bytes + 8) * slab_points_axis(n, cpml, 1)


def step_bytes(n, cpml, field_bytes=4):
    """Algorithmic bytes of a whole step (16 B/point + 16 B per layer point-axis in FP32)."""
    N = n[0] * n[1] * n[2]
    return (3 * field_bytes + 4) * N + 16 * slab_points(n, cpml)


def adjoint_step_bytes(n, cpml, every):
    """Algorithmic bytes of one step of an FP32 adjoint sweep: the recomputed
    forward step and its level increment (two levels read, one written); on
    each axis' layer points pass 1 (mu and zeta_b read; zeta_b, E and K
    written) and pass 2 (E and psi_b read; W and psi_b written); pass 3 on
    every point (mu^{n+1}, mu^{n+2}, m read; mu^n written); and the gradient
    pass (mu^{n+1} and one increment per step, the FP64 accumulator read and
    written once per pass of G <= 16 steps, a segment split evenly)."""
    N = n[0] * n[1] * n[2]
    passes = -(-every // 16)
    G = -(-every // passes)
    return step_bytes(n, cpml) + 12 * N + (20 + 16) * slab_points(n, cpml) + 16 * N + (8 + 16 / G) * N


def sweep_roofline(nbytes_per_step, steps, ms):
    """Whole-sweep rate: algorithmic bytes of every recomputed and reverse step
    over the sweep's wall time (the sweep's kernels overlap on two streams, so
    no single kernel's duration is taken)."""
    gbs = nbytes_per_step * steps / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "kind": "whole sweep, algorithmic bytes over wall time",
            "algorithmic_bytes_per_step": int(nbytes_per_step)}


def exchange_bytes(n, cpml, s, field_bytes=4):
    """Algorithmic bytes of one ghost exchange of the pencil share (ghost
    faces on y and z, depth g = 4 s): u^n to depth g, and for s > 1 u^{n-1}
    (16-bit: d^n) and the x layer memory (psi_x, zeta_x, FP32) to depth g - 4;
    y faces over the owned z range, z faces spanning the y ghosts; each byte
    is read and written once when packed and once when unpacked."""
    nx, ny, nz = n
    g = 4 * s
    fields = [(field_bytes, nx, g)]
    if g > 4:
        fields.append((field_bytes, nx, g - 4))
        for _ in range(2):
            for L in (cpml[0], cpml[1]):
                if L > 0:
                    fields.append((4, L, g - 4))
    payload = 0
    for e, ex, dep in fields:
        payload += 2 * dep * nz * ex * e + 2 * dep * (ny + 2 * dep) * ex * e
    return 4 * payload


def roofline(nbytes, ms, kernel, traffic=None):
    """Roofline record of one kernel from its algorithmic bytes per launch and mean duration."""
    gbs = nbytes / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic, "kernel": kernel, "kernel_ms": round(ms, 5),
            "algorithmic_bytes_per_launch": int(nbytes)}


KERNEL_CLASSES = ("update", "psi", "record", "exchange", "band", "tblock")


PLAN = None   # (variant, tile_ry, zchunk, tblock_k, tile_cols) forced on the headline runs (--plan)


def make_propagator(w, K, W, variant, storage=0, tblock_k=1, **shot_kw):
    import numpy as np
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, variant=variant, storage=storage, tblock_k=tblock_k,
                         **shot_kw)])
    if PLAN is not None and variant in (0, 2):
        p.set_plan(0, *PLAN)
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
    p.set_receivers(0, w.rec)
    p.record(0, K + W + 2)
    return p


def kernel_timing(w, K, W, variant=0, storage=0, **shot_kw):
    """Per-kernel mean durations (ms, count) from an eager pass of K steps with
    HIP events around every launch on the stream it runs on; the library runs
    the kernels of a step one after another while timing is on."""
    import torch

    p = make_propagator(w, K, W, variant, storage, **shot_kw)
    p.set_timing(True)     # warm-up launches run like the timed ones
    p.step(W)
    torch.cuda.synchronize()
    p.set_timing(True)     # clears the counters
    p.step(K)
    tm = {name: p.timing(c) for c, name in enumerate(KERNEL_CLASSES)}
    p.set_timing(False)
    plan = p.plan(0)
    p.close()
    return tm, plan


def time_gpu(w, K, W, variant, storage=0, graph=True, tblock_k=1):
    import torch

    p = make_propagator(w, K, W, variant, storage, tblock_k)
    W += (-W) % 4
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
    p.close()
    return ms


COUNTERS = os.path.join(ROOT, "profiles", "zmarch_layered512_counters.txt")
ZMARCH_SOURCES = ("paper_2606_06910_amd/csrc/kernels_step.hip", "paper_2606_06910_amd/csrc/fdtd_dev.hpp")


def sources_digest():
    """sha256 over the z-march kernel's source files (identifies the kernel the counters were taken on)."""
    import hashlib

    h = hashlib.sha256()
    for f in ZMARCH_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n, plan, path=None):
    """HBM bytes per z-march launch from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE KiB per dispatch times their copy-kernel
    calibration factors), or None when that summary is missing or was taken on
    other kernel sources, another grid or another plan."""
    path = COUNTERS if path is None else path
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("sources_sha256") != sources_digest():
            return None
        if kv.get("grid") != "%dx%dx%d" % tuple(n) or kv.get("tile_ry") != str(plan[1]) or \
                kv.get("tile_cols", "1") != str(plan[3] if len(plan) > 3 else 1):
            return None
        fetch = float(kv["fetch_kib_per_launch"]) * 1024 * float(kv["fetch_factor"])
        write = float(kv["write_kib_per_launch"]) * 1024 * float(kv["write_factor"])
        return int(round(fetch + write))
    except (OSError, KeyError, ValueError):
        return None


def precision_leg(K=200):
    """FP32 vs FP16 vs BF16 field storage on the 768^3 Gaussian-blob workload
    (Mpts/s over K steps), with the error of each storage stated against the
    stored FP64 oracle run of the central 160^3 crop (1500 steps)."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    n = 768
    rng = np.random.default_rng(1003)
    blobs = synth.blob_params((n, n, n), rng)
    dt = synth.dt_from_courant(blobs.vmax, (10.0,) * 3)
    v = synth.blob_model_torch((n, n, n), blobs)
    wav = torch.from_numpy(synth.ricker(K + 20, dt, 12.0).astype(np.float32)).cuda()
    out = {}
    for name, st in (("f32", 0), ("f16", 1), ("bf16", 2)):
        p = Propagator([Shot(n=(n, n, n), h=(10.0,) * 3, dt=dt, cpml=(20,) * 6, storage=st)])
        p.set_velocity(0, v)
        p.inject_source(0, (n // 2,) * 3, wav)
        p.step(K, graph=True)
        torch.cuda.synchronize()
        p.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(p.stream)
        p.step(K, graph=True)
        e1.record(p.stream)
        torch.cuda.synchronize()
        out[name] = {"mpts": round(n ** 3 * K / (e0.elapsed_time(e1) / 1e3) / 1e6, 1)}
        # per-kernel durations (eager, kernels one after another) and the
        # z-march's roofline: 16 B (FP32) or 12 B (16-bit: u^n, d^n in and out,
        # m in) per point outside the bands
        p.reset()
        p.set_timing(True)
        p.step(8)
        p.set_timing(True)
        p.step(40)
        tm = {kn: p.timing(c) for c, kn in enumerate(KERNEL_CLASSES)}
        p.set_timing(False)
        fb = 4 if st == 0 else 2
        per_pt = 16 if st == 0 else 12
        nb = per_pt * band_split((n, n, n), (20,) * 6)[0]
        out[name]["kernel_ms"] = {k: round(v[0], 5) for k, v in tm.items() if v[1] > 0}
        traffic = None
        if st == 1:
            traffic = measured_traffic((n, n, n), p.plan(0), os.path.join(ROOT, "profiles",
                                                                          "zmarch_f16_blob768_counters.txt"))
        out[name]["roofline"] = roofline(nb, tm["update"][0], "k_zmarch<%s> (points outside the layer bands)" %
                                         {0: "float", 1: "_Float16", 2: "__bf16"}[st], traffic)
        p.close()
    del v
    torch.cuda.empty_cache()
    # error statement: 160^3 crop, 1500 steps, vs the stored FP64 oracle traces
    ref_path = os.path.join(ROOT, "tests", "golden", "blob160_oracle.npz")
    if os.path.exists(ref_path):
        ref = np.load(ref_path)
        wc = synth.blob(crop=160, nt=1500)
        for name, st in (("f32", 0), ("f16", 1), ("bf16", 2)):
            p = Propagator([Shot(n=wc.n, h=wc.h, dt=wc.dt, cpml=wc.cpml, storage=st)])
            p.set_velocity(0, torch.from_numpy(wc.v.astype(np.float32)).cuda())
            p.inject_source(0, wc.src[0], torch.from_numpy(wc.wavelet.astype(np.float32)).cuda())
            p.set_receivers(0, wc.rec)
            tr = p.record(0, wc.nt)
            p.step(wc.nt, graph=True)
            torch.cuda.synchronize()
            d = tr.cpu().double().numpy()
            out[name]["trace_rel_l2_vs_fp64"] = float("%.3e" % (np.linalg.norm(d - ref["traces"]) /
                                                              np.linalg.norm(ref["traces"])))
            p.close()
    out["workload"] = "blob 768^3, 20-cell CPML, Ricker 12 Hz; error on the central 160^3 crop over 1500 steps"
    return out


def _timed_steps(p, steps, graph):
    """ms of `steps` steps from reset (capture, if any, untimed)."""
    import torch

    if graph:
        p.step(steps, graph=True)
        torch.cuda.synchronize()
    p.reset()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(p.stream)
    p.step(steps, graph=graph)
    e1.record(p.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def small_leg():
    """The 64^3 workload (10-cell layers, 200 steps): a few MB, launch-bound;
    Mpts/s with every step launched eagerly and with the HIP-graph time loop,
    for the automatic variant (the naive kernel at this size) and for the
    z-march."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    w = synth.plain64()
    out = {}
    for tag, variant in (("", 0), ("zmarch_", 2)):
        p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, variant=variant)])
        p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
        p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
        p.set_receivers(0, w.rec)
        p.record(0, w.nt)
        for name, graph in (("eager", False), ("graph", True)):
            ms = _timed_steps(p, w.nt, graph)
            out[tag + name + "_mpts"] = round(w.npts * w.nt / (ms / 1e3) / 1e6, 1)
        if not tag:
            out["auto_variant"] = {1: "naive", 2: "zmarch"}.get(p.plan(0)[0], str(p.plan(0)[0]))
        p.close()
    out["workload"] = "64^3, 10-cell CPML, 200 steps"
    return out


def pencil_leg(K=100):
    """One GPU's pencil-yz share: owned 1024 x 384 x 384, CPML on +-x only,
    ghost faces on y and z exchanged (loopback) every s steps with depth 4 s.
    Mpts/s of owned points for s = 1, 2, 4, the speed-up S_s over s = 1 and
    the exchange kernels' share of a step."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    w = synth.pencil(nt=K + 8)
    v = torch.from_numpy(w.v.astype(np.float32)).cuda()
    wav = torch.from_numpy(w.wavelet.astype(np.float32)).cuda()
    out = {}
    for s_ in (1, 2, 4):
        p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, face=(0, 0, 1, 1, 1, 1), exchange_every=s_)])
        p.set_velocity(0, v)
        p.inject_source(0, w.src[0], wav)
        ms = _timed_steps(p, K, True)
        p.reset()
        p.set_timing(True)
        p.step(4 * 4)
        ex = p.timing(3)
        upd = p.timing(0)
        p.set_timing(False)
        exch_ms_per_step = ex[0] * ex[1] / 16.0
        out["s%d" % s_] = {"mpts": round(w.npts * K / (ms / 1e3) / 1e6, 1),
                           "exchange_ms_per_step": round(exch_ms_per_step, 5),
                           "exchange_roofline": roofline(exchange_bytes(w.n, w.cpml, s_), ex[0],
                                                         "k_copy_jobs (pack + unpack of one exchange, 4 launches)")}
        if s_ == 1:
            out["s1"]["roofline"] = roofline(interior_kernel_bytes(w.n, w.cpml), upd[0],
                                             "k_zmarch<float> (points outside the layer bands)")
        p.close()
    for s_ in (2, 4):
        out["s%d" % s_]["S"] = round(out["s%d" % s_]["mpts"] / out["s1"]["mpts"], 3)
    out["workload"] = "owned 1024x384x384, CPML 20 on +-x, y/z ghost faces (loopback), %d steps" % K
    return out


def adjoint_leg(nshots=3, K=600, every=25):
    """Forward (with checkpoints every 25 steps) and adjoint (FP64 velocity
    gradient, segment recomputation) of the smallest shots of the 24-shot
    workload, advanced together in one batched context and swept back in one
    batched reverse sweep; and the same shots one context at a time.  Mpts/s
    of each pass over the shots' points x steps."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    shapes = synth.batch_shapes(24)
    order = sorted(range(len(shapes)), key=lambda i: np.prod(shapes[i]))[:nshots]
    data = [synth.batch_shot(i, shapes[i], nt=K) for i in order]
    npts = sum(w.npts for w, _ in data)

    def run(group):
        p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, v_ref=float(w.v.max())) for w, _ in group])
        trs = []
        for k, (w, v0) in enumerate(group):
            p.set_velocity(k, torch.from_numpy(v0.astype(np.float32)).cuda())
            p.inject_source(k, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
            p.set_receivers(k, w.rec)
            p.set_checkpointing(k, every, K)
            trs.append(p.record(k, K))
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(p.stream)
        p.step(K)
        e[1].record(p.stream)
        torch.cuda.synchronize()
        resid = [t.clone() for t in trs]

        def sweep(nt):
            if len(group) > 1:
                p.adjoint_all(nt, [r[:nt].contiguous() for r in resid])
            else:
                p.adjoint(0, nt, resid[0][:nt].contiguous())

        sweep(every)   # untimed warm-up: one segment (streams, tables and kernels loaded)
        torch.cuda.synchronize()
        e[1].record(p.stream)
        sweep(K)
        e[2].record(p.stream)
        torch.cuda.synchronize()
        p.close()
        return e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])

    fwd_ms, adj_ms = run(data)
    one_f = one_a = 0.0
    for d in data:
        f, a = run([d])
        one_f += f
        one_a += a
    nb = sum(adjoint_step_bytes(w.n, w.cpml, every) for w, _ in data)
    return {"shots": [list(shapes[i]) for i in order], "steps": K, "checkpoint_every": every,
            "forward_with_checkpoints_mpts": round(npts * K / (fwd_ms / 1e3) / 1e6, 1),
            "adjoint_mpts": round(npts * K / (adj_ms / 1e3) / 1e6, 1),
            "adjoint_roofline": sweep_roofline(nb, K, adj_ms),
            "one_context_per_shot": {"forward_with_checkpoints_mpts": round(npts * K / (one_f / 1e3) / 1e6, 1),
                                     "adjoint_mpts": round(npts * K / (one_a / 1e3) / 1e6, 1)}}


def batched_leg(K=600, nshots=24):
    """24 shots of uneven shape (each axis uniform in [96, 288]), 15-cell CPML,
    layered models: Mpts/s of all shots advanced together (one launch per kernel
    class per step, HIP-graph time loop) vs the same shots one after another."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    shapes = synth.batch_shapes(nshots)
    shots, models, wavs = [], [], []
    for i, sh in enumerate(shapes):
        rng = np.random.default_rng([1004, i])
        nx, ny, nz = sh
        vt = synth.layered_model((nz, ny, nx), rng)
        dt = synth.dt_from_courant(vt.max() * 1.03, (10.0,) * 3)
        shots.append(Shot(n=sh, h=(10.0,) * 3, dt=dt, cpml=(15,) * 6))
        models.append(torch.from_numpy(vt.astype(np.float32)).cuda())
        wavs.append(torch.from_numpy(synth.ricker(K, dt, 10.0).astype(np.float32)).cuda())
    npts = sum(a * b * c for a, b, c in shapes)

    def setup(p, idx):
        for j, i in enumerate(idx):
            p.set_velocity(j, models[i])
            nx, ny, nz = shapes[i]
            p.inject_source(j, (nx // 2, ny // 2, nz // 2), wavs[i])

    def timed(p, steps):
        p.step(steps, graph=True)
        torch.cuda.synchronize()
        p.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(p.stream)
        p.step(steps, graph=True)
        e1.record(p.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    pb = Propagator(shots)
    setup(pb, range(nshots))
    pb.autotune(os.path.join(ROOT, "paper_2606_06910_amd", "autotune_cache.json"))
    setup(pb, range(nshots))
    ms_b = timed(pb, K)
    # per-kernel durations (eager, the kernels of a step one after another) and
    # the rooflines of the z-march and the band kernel over all shots
    pb.reset()
    pb.set_timing(True)
    pb.step(8)
    pb.set_timing(True)
    pb.step(40)
    tm = {kn: pb.timing(c) for c, kn in enumerate(KERNEL_CLASSES)}
    pb.set_timing(False)
    pb.close()
    cp = (15,) * 6
    kb = {"update": sum(interior_kernel_bytes(sh, cp) for sh in shapes),
          "band": sum(band_kernel_bytes(sh, cp) for sh in shapes),
          "psi": sum(psi_kernel_bytes(sh, cp) for sh in shapes)}
    kms = {k: round(v[0], 5) for k, v in tm.items() if v[1] > 0}
    dom = max(("update", "band"), key=lambda k: kms.get(k, 0.0))
    names = {"update": "k_zmarch (points outside the layer bands, all shots)", "band": "k_band (band points, all shots)"}
    ms_s = 0.0
    for i in range(nshots):
        p = Propagator([shots[i]])
        setup(p, [i])
        ms_s += timed(p, K)
        p.close()
    return {"shots": nshots, "points": npts, "steps": K,
            "batched_mpts": round(npts * K / (ms_b / 1e3) / 1e6, 1),
            "sequential_mpts": round(npts * K / (ms_s / 1e3) / 1e6, 1),
            "kernel_ms": kms,
            "kernel_algorithmic_gbs": {k: round(kb[k] / (kms[k] / 1e3) / 1e9, 1) for k in kb if k in kms},
            "roofline": roofline(kb[dom], kms[dom], names[dom])}


def batched_fwd_adj_leg(K=600, every=25, nshots=24):
    """The batched forward + adjoint workload end to end: 24 shots (each axis
    uniform in [96, 288]), 15-cell layers, layered true models, 64 receivers on
    a seeded interior plane.  Observed data from the true models; the
    inversion models v0 = v_true (1 + 0.03 G) advance together in one batched
    context with the full state saved every 25 steps, the L2 misfit is formed,
    and every shot's FP64 velocity gradient comes from the adjoint (segments
    recomputed from the checkpoints) in one batched reverse sweep.  Mpts/s of
    the forward (with checkpoints) and of the 24 gradients, over points x
    steps."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    shapes = synth.batch_shapes(nshots)
    data = [synth.batch_shot(i, sh, nt=K) for i, sh in enumerate(shapes)]
    shots = [Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml,
                  v_ref=float(max(w.v.astype(np.float32).max(), v0.astype(np.float32).max())))
             for w, v0 in data]
    npts = sum(w.npts for w, _ in data)

    def setup(p, models):
        trs = []
        for k, ((w, _), v) in enumerate(zip(data, models)):
            p.set_velocity(k, torch.from_numpy(v.astype(np.float32)).cuda())
            p.inject_source(k, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
            p.set_receivers(k, w.rec)
            trs.append(p.record(k, K))
        return trs

    # observed data from the true models
    po = Propagator(shots)
    obs = setup(po, [w.v for w, _ in data])
    po.step(K, graph=True)
    torch.cuda.synchronize()
    obs = [t.clone() for t in obs]
    po.close()
    del po
    torch.cuda.empty_cache()
    # inversion models: batched forward with checkpoints, misfit, gradients
    p = Propagator(shots)
    trs = setup(p, [v0 for _, v0 in data])
    for k in range(nshots):
        p.set_checkpointing(k, every, K)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record(p.stream)
    p.step(K)
    e[1].record(p.stream)
    torch.cuda.synchronize()
    misfit = 0.5 * sum(float(((t.double() - o.double()) ** 2).sum()) for t, o in zip(trs, obs))
    resid = [t - o for t, o in zip(trs, obs)]
    p.adjoint_all(every, [r[:every].contiguous() for r in resid])   # untimed warm-up: one segment
    torch.cuda.synchronize()
    e[1].record(p.stream)
    grads = p.adjoint_all(K, resid)
    e[2].record(p.stream)
    torch.cuda.synchronize()
    fwd_ms, adj_ms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    gnorm = float(torch.sqrt(sum((g * g).sum() for g in grads)))
    finite = all(bool(torch.isfinite(g).all()) for g in grads)
    p.close()
    nb = sum(adjoint_step_bytes(w.n, w.cpml, every) for w, _ in data)
    return {"shots": nshots, "points": npts, "steps": K, "checkpoint_every": every, "receivers_per_shot": 64,
            "forward_with_checkpoints_mpts": round(npts * K / (fwd_ms / 1e3) / 1e6, 1),
            "gradient_mpts": round(npts * K / (adj_ms / 1e3) / 1e6, 1),
            "gradient_roofline": sweep_roofline(nb, K, adj_ms),
            "forward_s": round(fwd_ms / 1e3, 3), "gradient_s": round(adj_ms / 1e3, 3),
            "misfit": float("%.6e" % misfit), "gradient_l2": float("%.6e" % gnorm), "gradient_finite": finite}


def zmarch_instance(plan):
    """Template instance of the z-march kernel a plan (variant, tile_ry, tblock_k, tile_cols)
    launches: one column per lane, tile_ry 1, 2, 4, 8 -> k_zmarch (waves, rows per thread)
    (4, 2), (4, 4), (8, 4), (16, 4); two columns, tile_ry 1, 2, 4 -> k_zmarch2 (4, 2), (8, 2), (16, 2)."""
    if len(plan) > 3 and plan[3] == 2:
        nw, ry = {1: (4, 2), 2: (8, 2), 4: (16, 2)}.get(plan[1], (0, 0))
        return "k_zmarch2<float, %d, %d>" % (nw, ry)
    nw, ry = {1: (4, 2), 2: (4, 4), 4: (8, 4), 8: (16, 4)}.get(plan[1], (0, 0))
    return "k_zmarch<float, %d, %d>" % (nw, ry)


def cpu_baseline(w, steps=5):
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


PAPER_PV_MPTS = {320: 3289.58, 480: 2889.58, 544: 2900.14, 640: 2909.64, 800: 2920.36}   # one Quadro RTX 6000


def pv_leg(sizes=(320, 480, 544, 640, 800), K=64, W=4):
    """The paper's own first-order pressure-velocity system (two stages per
    step, six memory variables) on its single-GPU throughput grids: N^3 with
    20-cell layers on every face, lambda = 0.05, 64 steps from an initial
    pulse, FP32.  Mpts/s, and the step's algorithmic bytes over its time
    (48 B per point: p read, v read and written in the velocity stage; v read,
    p read and written in the pressure stage; plus a read and write of a
    memory variable per layer point and axis in each stage).  The paper's
    numbers for the same grids (another GPU) ride along as context."""
    import torch

    from paper_2606_06910_amd import PVPropagator

    out = {}
    for N in sizes:
        s = PVPropagator((N, N, N), (20,) * 6, 0.05)
        g = torch.arange(N, device="cuda", dtype=torch.float32) - (N - 1) / 2.0
        r2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2
        s.set_pressure(torch.exp(-r2 / 30.0))
        del g, r2
        s.step(W)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(K)
        e1.record(s.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        assert torch.isfinite(s.get_pressure()).all()
        s.close()
        del s
        torch.cuda.empty_cache()
        slab = slab_points((N, N, N), (20,) * 6)
        nbytes = 48 * N ** 3 + 16 * slab
        mpts = N ** 3 * K / (ms / 1e3) / 1e6
        out["n%d" % N] = {"mpts": round(mpts, 1), "ms_per_step": round(ms / K, 4),
                          "algorithmic_gbs": round(nbytes / (ms / K / 1e3) / 1e9, 1),
                          "paper_rtx6000_mpts": PAPER_PV_MPTS.get(N)}
    out["workload"] = "first-order p-v, N^3, 20-cell CPML on 6 faces, lambda 0.05, %d steps, FP32" % K
    return out


PAPER_REFLECTION = {0: 9.438e-1, 8: 8.049e-2, 12: 6.714e-3, 16: 5.581e-4, 24: 3.328e-5}   # first-order system, 4 GPUs


def reflection_leg():
    """Reflected-to-incident amplitude ratio of the absorbing layer against its
    width (0, 8, 12, 16, 24 cells) at normal incidence on the low face of each
    axis (synth.reflection_case: uniform 2000 m/s, Ricker 12.5 Hz, every other
    face out of reach), from the GPU path: the 18 runs (5 widths and a
    reference per axis) in one batched context.  The paper's ratios for its
    own first-order system and unstated setup ride along as context."""
    import numpy as np
    import torch

    import synth
    from paper_2606_06910_amd import Propagator, Shot

    ws = []
    for axis in range(3):
        ws += [synth.reflection_case(axis, L) for L in synth.REFL_WIDTHS]
        ws.append(synth.reflection_case(axis, 0, reference=True))
    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml) for w in ws])
    trs = []
    for k, w in enumerate(ws):
        p.set_velocity(k, torch.from_numpy(w.v.astype(np.float32)).cuda())
        p.inject_source(k, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
        p.set_receivers(k, w.rec)
        trs.append(p.record(k, w.nt))
    p.step(synth.REFL_NT, graph=True)
    torch.cuda.synchronize()
    got = {w.name: trs[k][:, 0].cpu().double().numpy() for k, w in enumerate(ws)}
    p.close()
    out = {}
    for a in "xyz":
        ref = got["refl_%s_ref" % a]
        out[a] = {"L%d" % L: float("%.4e" % synth.reflection_ratio(got["refl_%s_L%d" % (a, L)], ref))
                  for L in synth.REFL_WIDTHS}
    out["paper_first_order"] = {"L%d" % L: v for L, v in PAPER_REFLECTION.items()}
    out["workload"] = ("normal incidence on the low face of each axis, uniform 2000 m/s, h 10 m, Ricker 12.5 Hz, "
                       "receiver 4 cells past the layer band, source 24 cells from the layer, %d steps" % synth.REFL_NT)
    return out


def stream_ceiling_leg(mib=400):
    """This library's own streaming kernel (fdtd_stream_probe: o = a + b * c,
    16-byte lanes, three FP32 streams read and one written, the interior
    update's access mix) over arrays far larger than the caches: TB/s of the
    best of one-shot blocks and grid-stride loops over several grid sizes, at
    several in-flight depths (HIP events, 20 launches)."""
    import ctypes

    import torch

    from paper_2606_06910_amd import lib

    L = lib()
    n = mib * (1 << 20) // 4
    a, b, c = (torch.rand(n, device="cuda") for _ in range(3))
    o = torch.empty_like(a)
    st = torch.cuda.current_stream()
    ptr = [ctypes.c_void_p(t.data_ptr()) for t in (a, b, c, o)]
    best = None
    for blocks in (0, 1024, 2048, 4096, 8192):   # 0: one-shot blocks
        for unroll in (1, 2, 4):
            for _ in range(3):
                assert L.fdtd_stream_probe(*ptr, n, blocks, unroll, ctypes.c_void_p(st.cuda_stream)) == 0
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record(st)
            for _ in range(reps):
                L.fdtd_stream_probe(*ptr, n, blocks, unroll, ctypes.c_void_p(st.cuda_stream))
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tbs = 16 * n / (ms / 1e3) / 1e12
            if best is None or tbs > best["TB_per_s"]:
                best = {"TB_per_s": round(tbs, 3), "ms": round(ms, 4), "blocks": blocks, "unroll": unroll}
    assert torch.allclose(o, a + b * c)
    return {"kernel": "k_stream_chunk (blocks 0) / k_stream_probe (o = a + b * c, float4 lanes)",
            "bytes_per_launch": 16 * n, "best": best}


def oracle_timings_leg(full=False):
    """The FP64 oracle timed on this machine's host cores for each workload:
    the 64^3 run in full (200 steps), 10 steps at the pencil share's shape,
    the 160^3 blob crop and the smallest batched shot's forward + adjoint
    (full runs with full=True; otherwise 100 steps of each)."""
    import numpy as np

    import synth
    from oracle import oracle as O

    def grid(w, periodic=(0, 0, 0)):
        v = w.v.astype(np.float32).astype(np.float64)
        return O.Grid(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, periodic=periodic, vref=float(v.max())), v

    out = {"cores": O.threads()}
    w = synth.plain64()
    g, v = grid(w)
    t0 = time.perf_counter()
    O.forward(g, v, w.nt, w.src, w.wavelet, w.rec)
    dt = time.perf_counter() - t0
    out["plain64_full"] = {"steps": w.nt, "s": round(dt, 2), "mpts": round(w.npts * w.nt / dt / 1e6, 2)}
    w = synth.pencil(nt=11)
    g, v = grid(w, periodic=(0, 1, 1))
    S = O.Stepper(g, v)
    st = O.State.zeros(g)
    S.step(st)
    t0 = time.perf_counter()
    for _ in range(10):
        S.step(st)
    dt = time.perf_counter() - t0
    out["pencil_10_steps"] = {"steps": 10, "s": round(dt, 2), "mpts": round(w.npts * 10 / dt / 1e6, 2)}
    del S, st
    nt = 1500 if full else 100
    w = synth.blob(crop=160, nt=nt)
    g, v = grid(w)
    t0 = time.perf_counter()
    O.forward(g, v, nt, w.src, w.wavelet, w.rec)
    dt = time.perf_counter() - t0
    out["blob160_crop"] = {"steps": nt, "s": round(dt, 2), "mpts": round(w.npts * nt / dt / 1e6, 2)}
    shapes = synth.batch_shapes(24)
    i = min(range(24), key=lambda k: np.prod(shapes[k]))
    nt = 600 if full else 100
    wt, v0 = synth.batch_shot(i, shapes[i], nt=nt)
    g = O.Grid(n=wt.n, h=wt.h, dt=wt.dt, cpml=wt.cpml, vref=float(wt.v.max()))
    vv = v0.astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()
    fwd = O.forward(g, vv, nt, wt.src, wt.wavelet, wt.rec, keep_lapf=True)
    t1 = time.perf_counter()
    O.gradient(g, vv, nt, wt.src, wt.wavelet, wt.rec, fwd["traces"], fwd=fwd)
    t2 = time.perf_counter()
    out["smallest_shot_fwd_adj"] = {"shape": list(shapes[i]), "steps": nt, "forward_s": round(t1 - t0, 2),
                                    "adjoint_s": round(t2 - t1, 2),
                                    "mpts_fwd_adj": round(wt.npts * nt / (t2 - t0) / 1e6, 2)}
    out["sample"] = "full runs" if full else "100-step samples of the blob crop and the batched shot"
    return out


LEGS = {
    "cpml_reflection": lambda: reflection_leg(),
    "batched_fwd_adj_24": lambda: batched_fwd_adj_leg(),
    "stream_ceiling": lambda: stream_ceiling_leg(),
    "oracle_timings": lambda: oracle_timings_leg(full=os.environ.get("FDTD_ORACLE_FULL") == "1"),
    "storage_768": lambda: precision_leg(),
    "batched_24": lambda: batched_leg(),
    "small_64": lambda: small_leg(),
    "pencil_1024x384x384": lambda: pencil_leg(),
    "adjoint_3_smallest": lambda: adjoint_leg(),
    "pv_paper_grids": lambda: pv_leg(),
}


def run_leg(name, timeout=600):
    """One extra leg in a child process, so that a failure there cannot take
    the headline figure down with it; returns its JSON, or the failure."""
    import subprocess

    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--leg", name], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=timeout)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
    if r.returncode == 0 and lines:
        return json.loads(lines[-1])
    return {"error": "leg exited with status %d" % r.returncode, "stderr_tail": r.stderr[-400:]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variant", type=int, default=0, help="0 auto, 1 naive, 2 z-march, 3 temporal blocking")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other kernel variants (naive, temporal blocking)")
    ap.add_argument("--compare", action="store_true", help="(default; kept for old command lines)")
    ap.add_argument("--eager", action="store_true", help="launch every step eagerly (no HIP graph)")
    ap.add_argument("--no-extra", action="store_true", help="skip the 16-bit storage and batched-shot legs")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration run)")
    ap.add_argument("--stream-probe", type=int, default=0, metavar="MIB",
                    help="only time o = a + b * c over FP32 arrays of MIB MiB (3 read + 1 write streams)")
    ap.add_argument("--kernel-timing", action="store_true",
                    help="only run the per-kernel timing pass (the launches a profiler summary is taken over)")
    ap.add_argument("--workload", default="layered", choices=("layered", "blob", "pencil"),
                    help="workload of --kernel-timing: the layered N^3 grid, the Gaussian-blob N^3 grid of the "
                         "storage leg, or the 1024x384x384 pencil share")
    ap.add_argument("--storage", type=int, default=0, help="field storage of --kernel-timing: 0 FP32, 1 FP16, 2 BF16")
    ap.add_argument("--exchange-every", type=int, default=1, help="s of the pencil workload (--kernel-timing)")
    ap.add_argument("--leg", choices=sorted(LEGS), help="only run one extra leg and print its JSON")
    ap.add_argument("--plan", default="", metavar="V,RY,ZC,K,COLS",
                    help="force a kernel plan on the headline runs (fdtd_set_plan arguments)")
    ap.add_argument("--no-storage-leg", action="store_true",
                    help="skip the 768^3 FP32/FP16/BF16 storage leg")
    ap.add_argument("--storage-leg", action="store_true", help="(default; kept for old command lines)")
    args = ap.parse_args()
    if args.plan:
        global PLAN
        PLAN = tuple(int(x) for x in args.plan.split(","))
        assert len(PLAN) == 5, "--plan takes variant,tile_ry,zchunk,tblock_k,tile_cols"
    if args.leg:
        print(json.dumps(LEGS[args.leg]()), flush=True)
        return
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
    if args.stream_probe:
        import torch

        # the z-march's access mix with nothing else: three FP32 streams read,
        # one written, o = a + b * c, arrays far larger than the caches
        n = args.stream_probe * (1 << 20) // 4
        a, b, c = (torch.rand(n, device="cuda") for _ in range(3))
        o = torch.empty_like(a)
        for _ in range(3):
            torch.addcmul(a, b, c, out=o)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            torch.addcmul(a, b, c, out=o)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        print(json.dumps({"stream_probe": "o = a + b * c, FP32", "bytes_per_launch": 16 * n,
                          "ms": round(ms, 4), "TB_per_s": round(16 * n / (ms / 1e3) / 1e12, 3)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    K, W = args.steps, args.warmup
    n = (args.n, args.n, args.n)
    Kt = min(K, 200)
    if args.kernel_timing:
        kw = {}
        if args.workload == "blob":
            w = synth.blob(n=args.n, nt=Kt + W + 2)
        elif args.workload == "pencil":
            w = synth.pencil(nt=Kt + W + 2)
            kw = dict(face=(0, 0, 1, 1, 1, 1), exchange_every=args.exchange_every)
        else:
            w = synth.layered(n_xyz=n, nt=Kt + W + 2)
        print("bench: kernel timing, %s %s, storage %d" % (args.workload, str(w.n), args.storage), file=sys.stderr,
              flush=True)
        tm, plan = kernel_timing(w, Kt, W, args.variant, args.storage, **kw)
        print(json.dumps({"kernel_ms": {k: round(v[0], 5) for k, v in tm.items() if v[1] > 0},
                          "launches": {k: v[1] for k, v in tm.items() if v[1] > 0}, "plan": plan}), flush=True)
        return
    w = synth.layered(n_xyz=n, nt=K + W + 2)
    print("bench: layered %s, %d+%d steps" % (str(n), W, K), file=sys.stderr, flush=True)
    ms = time_gpu(w, K, W, args.variant, graph=not args.eager)
    tm, plan = kernel_timing(w, Kt, W, args.variant)
    N = w.npts
    value = N * K / (ms / 1e3) / 1e6
    upd = tm["update"]
    upd_bytes = interior_kernel_bytes(w.n, w.cpml)
    achieved = upd_bytes / (upd[0] / 1e3) / 1e9
    kgbs = {}
    for name, nbytes in (("update", upd_bytes), ("band", band_kernel_bytes(w.n, w.cpml)),
                         ("psi", psi_kernel_bytes(w.n, w.cpml))):
        if tm[name][1] > 0:
            kgbs[name] = round(nbytes / (tm[name][0] / 1e3) / 1e9, 1)
    traffic = measured_traffic(w.n, plan)
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
                   "grid": list(n), "cpml": 20, "variant": args.variant, "graph": not args.eager,
                   "plan": list(plan)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                     "measured_frac": (round(traffic / (upd[0] / 1e3) / 1e9 / PEAK_HBM_GBS, 4)
                                       if traffic else None),
                     "copy_ceiling_gbs": COPY_CEILING_GBS,
                     "stream_ceiling_gbs": STREAM_CEILING_GBS,
                     "kernel": "%s (update of the points outside the layer bands)" % zmarch_instance(plan),
                     "kernel_ms": round(upd[0], 5), "algorithmic_bytes_per_launch": upd_bytes},
        "step_algorithmic_gbs": round(step_bytes(w.n, w.cpml) / (ms / K / 1e3) / 1e9, 1),
        "kernel_ms": {k: round(v[0], 5) for k, v in tm.items() if v[1] > 0},
        "kernel_algorithmic_gbs": kgbs,
    }
    if not args.no_compare:
        var = {}
        Kc = min(K, 200)
        for name, vv, kk in (("naive", 1, 1), ("zmarch", 2, 1), ("tblock2", 3, 2), ("tblock4", 3, 4)):
            print("bench: compare %s" % name, file=sys.stderr, flush=True)
            m2 = time_gpu(w, Kc, W, vv, graph=not args.eager, tblock_k=kk)
            var[name] = round(N * Kc / (m2 / 1e3) / 1e6, 1)
        out["variants_mpts"] = var
    if not args.no_extra:
        torch.cuda.empty_cache()
        legs = ["batched_24", "batched_fwd_adj_24", "small_64", "pencil_1024x384x384", "adjoint_3_smallest",
                "pv_paper_grids", "cpml_reflection", "stream_ceiling"]
        if not args.no_storage_leg:
            legs.insert(0, "storage_768")
        for name in legs:
            print("bench: %s leg" % name, file=sys.stderr, flush=True)
            out[name] = run_leg(name)
    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
        if not args.no_extra:
            print("bench: oracle_timings leg", file=sys.stderr, flush=True)
            out["oracle_timings"] = run_leg("oracle_timings")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
