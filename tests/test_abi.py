"""C ABI: the library loads, exports every entry point of include/*.h, and
validates configurations on the host (no GPU work involved)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names.update(re.findall(r"\b(fdtd_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["fdtd_create", "fdtd_set_velocity", "fdtd_inject_source", "fdtd_step", "fdtd_record_receivers",
                 "fdtd_adjoint", "fdtd_pv_create", "fdtd_pv_step"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2606_06910_amd import _lib

    L = _lib.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(_lib.exported_names()) == _declared()


def _cfg(**kw):
    from paper_2606_06910_amd import Shot

    base = dict(n=(32, 30, 28), h=(10.0, 10.0, 10.0), dt=1e-3, cpml=(5,) * 6)
    base.update(kw)
    return Shot(**base).c()


def _create(cfgs):
    from paper_2606_06910_amd import _lib

    L = _lib.lib()
    arr = (_lib.ShotConfig * len(cfgs))(*cfgs)
    ctx = ctypes.c_void_p()
    rc = L.fdtd_create(arr, len(cfgs), None, ctypes.byref(ctx))
    return L, rc, ctx


@pytest.mark.parametrize("bad", [
    dict(n=(8, 30, 28)),                       # axis shorter than the stencil
    dict(h=(0.0, 10.0, 10.0)),
    dict(dt=0.0),
    dict(cpml=(16, 5, 5, 5, 5, 5)),            # layer wider than half the axis
    dict(cpml=(-1, 5, 5, 5, 5, 5)),
    dict(face=(1, 1, 0, 0, 0, 0)),             # ghost faces only on y/z
    dict(face=(0, 0, 1, 0, 0, 0)),             # ghost faces in pairs
    dict(face=(0, 0, 1, 1, 0, 0)),             # ghost faces carry no layer
    dict(face=(0, 0, 1, 1, 0, 0), cpml=(5, 5, 0, 0, 5, 5), exchange_every=3),
    dict(storage=7),
    dict(variant=9),
    dict(variant=3, tblock_k=3),
    dict(field_scale=3.0),
    # a 49 MB FP32 plane: below 64 MiB, but the band kernel's z walk (32 planes
    # + 12) from one descriptor would pass the 2^31-byte offset range
    dict(n=(3500, 3500, 20), cpml=(5,) * 6),
])
def test_create_rejects_invalid_configs(bad):
    from paper_2606_06910_amd import _lib

    L, rc, ctx = _create([_cfg(**bad)])
    assert rc == -1, (bad, rc)
    assert not ctx.value


def test_create_and_workspace_size_on_host():
    from paper_2606_06910_amd import _lib

    L, rc, ctx = _create([_cfg(), _cfg(n=(40, 41, 42))])
    assert rc == 0
    nb = ctypes.c_size_t()
    assert L.fdtd_workspace_size(ctx, ctypes.byref(nb)) == 0
    # two FP32 level buffers + m per shot dominate: at least 3 * 4 bytes per padded point
    assert nb.value > 3 * 4 * (32 * 30 * 28 + 40 * 41 * 42)
    # calls that need a workspace fail cleanly before one is bound
    assert L.fdtd_step(ctx, 1) == -3
    assert b"workspace" in L.fdtd_last_error(ctx)
    assert L.fdtd_set_sentinel(ctx, 5) == -3      # sentinel: needs a workspace too
    assert L.fdtd_set_sentinel(ctx, -1) == -1     # and a non-negative interval
    assert L.fdtd_set_sentinel(None, 5) == -1
    L.fdtd_destroy(ctx)


def test_strerror_covers_every_status():
    from paper_2606_06910_amd import _lib

    L = _lib.lib()
    for st in range(-7, 1):
        assert L.fdtd_strerror(st) and L.fdtd_strerror(st) != b"unknown status"


@pytest.mark.parametrize("n,face,s,ry", [
    ((512, 512, 512), (0,) * 6, 1, 4),              # 128 tiles of 64 x 32 (target 143)
    ((768, 768, 768), (0,) * 6, 1, 8),              # 144 tiles of 64 x 64 (64 x 32: 288 > 256)
    ((640, 640, 640), (0,) * 6, 1, 4),              # 200 tiles of 64 x 32 (target 152)
    ((384, 384, 384), (0,) * 6, 1, 4),              # 72 tiles of 64 x 32 in two z chunks
    ((1024, 384, 384), (0, 0, 1, 1, 1, 1), 1, 4),   # pencil share: 192 tiles of 64 x 32
    ((1024, 384, 384), (0, 0, 1, 1, 1, 1), 4, 4),   # with 12 ghost rows: 208 tiles of 64 x 32
    ((1024, 1024, 1024), (0,) * 6, 1, 8),           # 256 tiles of 64 x 64
])
def test_default_plan_tile_shape(n, face, s, ry):
    """The default z-march plan: about one workgroup per CU for three quarters
    of the chip times the fraction of points outside the bands (the shapes
    measured best beside the band kernel), never more workgroups than CUs."""
    cp = (20, 20, 0, 0, 0, 0) if face[2] else (20,) * 6
    L, rc, ctx = _create([_cfg(n=n, cpml=cp, face=face, exchange_every=s)])
    assert rc == 0
    v, r, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert L.fdtd_get_plan(ctx, 0, ctypes.byref(v), ctypes.byref(r), ctypes.byref(k), None) == 0
    assert (v.value, r.value, k.value) == (2, ry, 1)
    L.fdtd_destroy(ctx)


@pytest.mark.parametrize("cfgs,variants", [
    ([dict(n=(64, 64, 64))], [1]),                         # a lone small shot: naive
    ([dict(n=(160, 160, 160))], [2]),                      # above 150^3 points: z-march
    ([dict(n=(64, 64, 64)), dict(n=(64, 64, 64))], [2, 2]),   # batched shots: z-march
    ([dict(n=(64, 64, 64), variant=2)], [2]),              # an explicit choice stands
])
def test_auto_variant(cfgs, variants):
    L, rc, ctx = _create([_cfg(**c) for c in cfgs])
    assert rc == 0
    for i, want in enumerate(variants):
        v, r, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert L.fdtd_get_plan(ctx, i, ctypes.byref(v), ctypes.byref(r), ctypes.byref(k), None) == 0
        assert v.value == want
    L.fdtd_destroy(ctx)


def test_batch_default_plan():
    """Batched shots whose single-shot plans would over-subscribe the CUs get
    many small z-march workgroups (64 x 8 tiles); a pair of large shots keeps
    the single-shot shapes."""
    shapes = [(96 + 8 * i, 288 - 8 * i, 160) for i in range(24)]
    L, rc, ctx = _create([_cfg(n=n, cpml=(15,) * 6) for n in shapes])
    assert rc == 0
    v, r, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    for i in range(len(shapes)):
        assert L.fdtd_get_plan(ctx, i, ctypes.byref(v), ctypes.byref(r), ctypes.byref(k), None) == 0
        assert (v.value, r.value) == (2, 1)
    L.fdtd_destroy(ctx)
    L, rc, ctx = _create([_cfg(n=(512, 512, 256), cpml=(20,) * 6)] * 2)
    assert rc == 0
    assert L.fdtd_get_plan(ctx, 0, ctypes.byref(v), ctypes.byref(r), ctypes.byref(k), None) == 0
    assert r.value != 1
    L.fdtd_destroy(ctx)


def test_pv_create_validates_on_the_host():
    """The first-order path's context: sizes and argument checks, no GPU work."""
    from paper_2606_06910_amd import _lib

    L = _lib.lib()

    def make(n=(32, 30, 28), cpml=(5,) * 6, lam=0.05):
        c = _lib.PVConfig()
        c.n[:] = list(n)
        c.cpml[:] = list(cpml)
        c.lam = lam
        ctx = ctypes.c_void_p()
        return L.fdtd_pv_create(ctypes.byref(c), None, ctypes.byref(ctx)), ctx

    rc, ctx = make()
    assert rc == 0
    nb = ctypes.c_size_t()
    assert L.fdtd_pv_workspace_size(ctx, ctypes.byref(nb)) == 0
    assert nb.value >= 10 * (32 + 8) * (30 + 8) * (28 + 8) * 4      # ten padded fields
    assert L.fdtd_pv_step(ctx, 1) == -3                           # no workspace bound
    L.fdtd_pv_destroy(ctx)
    for kw in (dict(lam=0.0), dict(n=(8, 30, 28)), dict(n=(32, 30, 40000)),
               dict(cpml=(16, 16, 5, 5, 5, 5)), dict(cpml=(-1, 5, 5, 5, 5, 5))):
        rc, _ = make(**kw)
        assert rc == -1, kw
    # the leapfrog's limit 2 / (sqrt(3) max s) = 0.667226 (the oracle test of the
    # same limit shows growth just above it): EUNSTABLE above, accepted below
    for lam, want in ((0.69, -2), (0.8, -2), (0.6675, -2), (0.6668, 0), (0.66, 0)):
        rc, ctx = make(lam=lam)
        assert rc == want, lam
        if rc == 0:
            L.fdtd_pv_destroy(ctx)
