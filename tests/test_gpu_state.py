"""Resume path: fdtd_save_state / fdtd_load_state.

Bar (written here): a run saved at step k and restored into a fresh context of
the same configuration continues bit for bit as the uninterrupted run (the
final field and the receiver rows after k), for a single shot with uneven
layers (z-march and band kernel: psi and zeta carry the layer state), a
16-bit-storage shot (the increment state d^n) and the pencil share with
enlarged ghosts saved at a step that is not a multiple of the exchange
interval; a blob of another configuration is rejected.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _case(n=(70, 45, 38), cpml=(5, 7, 3, 6, 8, 4), nt=60, seed=51):
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    v = 1800.0 + 800.0 * rng.uniform(size=(nz, ny, nx))
    dt = synth.dt_from_courant(v.max(), (10.0,) * 3) * 0.9
    src = (nx // 3, ny // 2, nz // 2)
    rec = np.clip(np.array(src)[None, :] + rng.integers(-6, 7, size=(10, 3)), 0, np.array(n) - 1).astype(np.int32)
    return v, dt, src, synth.ricker(nt, dt, 30.0), rec


def _prop(n, dt, cpml, v, src, wav, rec, nt, **kw):
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    p = Propagator([Shot(n=n, h=(10.0,) * 3, dt=dt, cpml=cpml, **kw)])
    p.set_velocity(0, torch.from_numpy(v.astype(np.float32)).cuda())
    p.inject_source(0, src, torch.from_numpy(wav.astype(np.float32)).cuda())
    p.set_receivers(0, rec)
    tr = p.record(0, nt)
    return p, tr


@pytest.mark.parametrize("kw,n,cpml,k", [
    (dict(variant=2), (70, 45, 38), (5, 7, 3, 6, 8, 4), 23),
    (dict(variant=2, storage=1), (70, 45, 38), (5, 7, 3, 6, 8, 4), 31),
    (dict(face=(0, 0, 1, 1, 1, 1), exchange_every=4), (64, 40, 44), (10, 10, 0, 0, 0, 0), 22),
])
def test_save_load_continues_bit_for_bit(kw, n, cpml, k):
    import torch

    nt = 60
    v, dt, src, wav, rec = _case(n=n, cpml=cpml, nt=nt)
    a, tra = _prop(n, dt, cpml, v, src, wav, rec, nt, **kw)
    a.step(k)
    blob = a.save_state()
    a.step(nt - k)
    torch.cuda.synchronize()
    ua, ta = a.get_field(0).cpu().numpy(), tra.cpu().numpy().copy()
    b, trb = _prop(n, dt, cpml, v, src, wav, rec, nt, **kw)
    b.load_state(blob)
    assert b.nstep == k
    b.step(nt - k)
    torch.cuda.synchronize()
    ub, tb = b.get_field(0).cpu().numpy(), trb.cpu().numpy()
    assert np.array_equal(ua, ub)
    assert np.array_equal(ta[k:], tb[k:])
    a.close()
    b.close()


def test_load_rejects_another_configuration():
    from paper_2606_06910_amd import FDTDValueError

    v, dt, src, wav, rec = _case()
    a, _ = _prop((70, 45, 38), dt, (5, 7, 3, 6, 8, 4), v, src, wav, rec, 10, variant=2)
    a.step(3)
    blob = a.save_state()
    v2, _, _, wav2, _ = _case(n=(60, 45, 38))
    b, _ = _prop((60, 45, 38), dt, (5, 7, 3, 6, 8, 4), v2, src, wav2, rec, 10, variant=2)
    with pytest.raises(FDTDValueError):
        b.load_state(blob)
    a.close()
    b.close()
