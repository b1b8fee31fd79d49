"""fdtd_forward_static (state in the library's fixed device array, no device
allocation) against the same forward run through fdtd_step on a caller
workspace.

Bar (written here): identical bits (same kernels, same orchestration) for
the traces and the final field, on two calls in a row on one GPU, the second
with a smaller grid than the first (the array keeps the first call's
contents, so whatever must start at zero has to be cleared), and both within
relative L2 1e-5 of the FP64 oracle.  A shot whose workspace exceeds the
array is rejected with FDTD_ENOMEM before any GPU work.
"""
import ctypes

import numpy as np
import pytest

import synth
from helpers import rel_l2, run_oracle

pytestmark = pytest.mark.gpu

ENOMEM = -4


def _workload(n, cpml, nt, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    v = 1800.0 + 900.0 * rng.uniform(size=(nz, ny, nx))
    h = (10.0, 10.0, 10.0)
    dt = synth.dt_from_courant(v.max(), h) * 0.9
    src = (nx // 2 - 3, ny // 2 + 2, nz // 2)
    near = np.array(src)[None, :] + rng.integers(-6, 7, size=(14, 3))
    rec = np.clip(near, 0, np.array(n) - 1).astype(np.int32)
    return synth.Workload("static", tuple(n), h, dt, nt, tuple(cpml), v, np.array([src], np.int32),
                          synth.ricker(nt, dt, 30.0), rec)


def _config(w, variant):
    from paper_2606_06910_amd import Shot

    return Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, variant=variant).c()


def _run_static(w, variant):
    import torch

    from paper_2606_06910_amd import lib

    L = lib()
    dev = torch.device("cuda")
    v = torch.from_numpy(w.v.astype(np.float32)).to(dev)
    wav = torch.from_numpy(w.wavelet.astype(np.float32)).to(dev)
    rec = torch.from_numpy(w.rec.astype(np.int32)).to(dev)
    tr = torch.zeros((w.nt, len(w.rec)), dtype=torch.float32, device=dev)
    u = torch.zeros(w.v.shape, dtype=torch.float32, device=dev)
    cfg = _config(w, variant)
    s = w.src[0]
    stream = torch.cuda.current_stream(dev)
    rc = L.fdtd_forward_static(ctypes.byref(cfg), ctypes.c_void_p(v.data_ptr()), int(s[0]), int(s[1]), int(s[2]),
                               ctypes.c_void_p(wav.data_ptr()), w.nt, 1.0, ctypes.c_void_p(rec.data_ptr()),
                               len(w.rec), ctypes.c_void_p(tr.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                               ctypes.c_void_p(stream.cuda_stream))
    assert rc == 0, rc
    return tr.cpu().double().numpy(), u.cpu().double().numpy()


def _run_workspace(w, variant):
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    p = Propagator([Shot(n=w.n, h=w.h, dt=w.dt, cpml=w.cpml, variant=variant)])
    p.set_velocity(0, torch.from_numpy(w.v.astype(np.float32)).cuda())
    p.inject_source(0, w.src[0], torch.from_numpy(w.wavelet.astype(np.float32)).cuda())
    p.set_receivers(0, w.rec)
    tr = p.record(0, w.nt)
    p.step(w.nt)
    u = p.get_field(0)
    torch.cuda.synchronize()
    out = tr.cpu().double().numpy(), u.cpu().double().numpy()
    p.close()
    return out


def test_static_forward_two_calls_match_workspace_path():
    # first the larger grid (z-march + band kernel), then a smaller one with
    # other layers (automatic variant: the naive kernel at this size)
    cases = [(_workload((96, 80, 72), (8, 10, 6, 9, 7, 8), 70, 41), 2),
             (_workload((44, 38, 50), (5, 4, 6, 0, 3, 7), 60, 42), 0)]
    for w, variant in cases:
        print("static forward: n=%s variant=%d" % (w.n, variant), flush=True)
        got = _run_static(w, variant)
        ref = _run_workspace(w, variant)
        assert np.array_equal(got[0], ref[0]), "traces differ"
        assert np.array_equal(got[1], ref[1]), "final field differs"
        orc = run_oracle(w)
        e_tr, e_u = rel_l2(got[0], orc["traces"]), rel_l2(got[1], orc["state"].u)
        print("  bit-equal to the workspace path; vs oracle: traces %.2e  field %.2e" % (e_tr, e_u), flush=True)
        assert e_tr <= 1e-5 and e_u <= 1e-5


def test_static_forward_rejects_a_shot_above_the_array():
    """A 400^3 shot needs more than 256 MiB of state: ENOMEM before any GPU work."""
    import torch

    from paper_2606_06910_amd import lib

    L = lib()
    w = _workload((40, 40, 40), (4,) * 6, 4, 43)
    from paper_2606_06910_amd import Shot

    cfg = Shot(n=(400, 400, 400), h=w.h, dt=w.dt, cpml=(10,) * 6).c()
    v = torch.ones(1, device="cuda")   # never read: the size check comes first
    rc = L.fdtd_forward_static(ctypes.byref(cfg), ctypes.c_void_p(v.data_ptr()), 0, 0, 0, None, 4, 1.0, None, 0,
                               None, None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == ENOMEM, rc
