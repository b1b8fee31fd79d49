"""16-bit field storage (FP16 / BF16) with FP32 arithmetic.

The error against the FP64 oracle is stated by these tests (printed) and
bounded: FP16 <= 1e-2 relative L2 on traces and space-time snapshots for the
64^3 workload (the 1e-2 target), BF16 <= 1e-1 (8-bit mantissa; stated, not
claimed to meet 1e-2).  The kernel variants agree bit for bit in every storage.
"""
import numpy as np
import pytest

import synth
from helpers import rel_l2, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

F16, BF16 = 1, 2


@pytest.fixture(scope="module")
def plain64_ref():
    w = synth.plain64()
    return w, run_oracle(w, snap_every=10)


@pytest.mark.parametrize("storage,bound", [(F16, 1e-2), (BF16, 1e-1)])
def test_16bit_error_vs_oracle(plain64_ref, storage, bound):
    w, ref = plain64_ref
    tr, snaps, _ = run_gpu(w, snap_every=10, storage=storage)
    e_tr, e_st = rel_l2(tr, ref["traces"]), rel_l2(snaps, ref["snaps"])
    print("storage %d: traces %.3e  space-time %.3e" % (storage, e_tr, e_st), flush=True)
    assert e_tr <= bound and e_st <= bound


@pytest.mark.parametrize("storage", [F16, BF16])
def test_16bit_variants_bitwise(plain64_ref, storage):
    w, _ = plain64_ref
    a = run_gpu(w, nt=60, storage=storage, variant=1)
    b = run_gpu(w, nt=60, storage=storage, variant=2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_blob_crop_error_statement():
    """The 16-bit error statement of the 768^3 blob workload, measured on its
    central 160^3 crop over 1500 steps against the stored FP64 oracle run
    (tests/golden/blob160_oracle.npz, written by make_blob_crop_reference.py)."""
    import os

    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "blob160_oracle.npz"))
    w = synth.blob(crop=160, nt=1500)
    assert np.array_equal(ref["rec"], w.rec)
    out = {}
    for name, st in (("f32", 0), ("f16", F16), ("bf16", BF16)):
        tr, _, _ = run_gpu(w, storage=st)
        out[name] = rel_l2(tr, ref["traces"])
    print("blob160 x 1500 trace rel-L2: %s" % out, flush=True)
    assert out["f32"] <= 1e-5
    assert out["f16"] <= 1e-2


@pytest.mark.parametrize("storage", [F16, BF16])
def test_16bit_state_roundtrip(storage):
    """The 16-bit state is (u^n, d^n = u^n - u^{n-1}); fdtd_set_field /
    fdtd_get_field expose u^n and u^{n-1} and round-trip values that 16 bits hold."""
    import torch

    from paper_2606_06910_amd import Propagator, Shot

    n = (20, 18, 16)
    p = Propagator([Shot(n=n, h=(10.0,) * 3, dt=1e-3, storage=storage, field_scale=1.0, variant=2)])
    p.set_velocity(0, torch.full((16, 18, 20), 2000.0, device="cuda"))
    g = torch.Generator().manual_seed(1)
    # values exact in both 16-bit formats (8 significant bits), and so are their differences
    a = (torch.randint(-64, 64, (16, 18, 20), generator=g).float() / 16).cuda()
    b = a + (torch.randint(-8, 8, (16, 18, 20), generator=g).float() / 16).cuda()
    p.set_field(0, 0, a)
    p.set_field(0, 1, b)
    assert torch.equal(p.get_field(0, 0), a)
    assert torch.equal(p.get_field(0, 1), b)
    p.close()
