"""ctypes binding of libfdtd.so (the C ABI declared in include/fdtd.h and include/fdtd_pv.h).

Argument marshalling only: every step of the path runs in the library's
HIP kernels.  There is no fallback: if the library is missing or cannot be
loaded, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

FDTD_OK = 0
STATUS = {
    0: "FDTD_OK",
    -1: "FDTD_EINVAL",
    -2: "FDTD_EUNSTABLE",
    -3: "FDTD_ESTATE",
    -4: "FDTD_ENOMEM",
    -5: "FDTD_EHIP",
    -6: "FDTD_ENONFINITE",
    -7: "FDTD_EUNSUPPORTED",
}
F32, F16, BF16 = 0, 1, 2
FACE_DIRICHLET, FACE_GHOST = 0, 1
VARIANT_AUTO, VARIANT_NAIVE, VARIANT_ZMARCH, VARIANT_TBLOCK = 0, 1, 2, 3


class ShotConfig(ctypes.Structure):
    """Mirror of fdtd_shot_config."""

    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("h", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("cpml", ctypes.c_int32 * 6),
        ("face", ctypes.c_int32 * 6),
        ("exchange_every", ctypes.c_int32),
        ("R", ctypes.c_double),
        ("kappa_max", ctypes.c_double),
        ("alpha_frac", ctypes.c_double),
        ("v_ref", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("tblock_k", ctypes.c_int32),
        ("field_scale", ctypes.c_double),
    ]


class PVConfig(ctypes.Structure):
    """Mirror of fdtd_pv_config (include/fdtd_pv.h)."""

    _fields_ = [
        ("n", ctypes.c_int32 * 3),
        ("cpml", ctypes.c_int32 * 6),
        ("lam", ctypes.c_double),
        ("R", ctypes.c_double),
        ("kappa_max", ctypes.c_double),
        ("alpha_frac", ctypes.c_double),
        ("variant", ctypes.c_int32),
    ]


class FDTDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class FDTDValueError(FDTDError, ValueError):
    pass


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "fdtd_create": (ctypes.c_int, [ctypes.POINTER(ShotConfig), ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "fdtd_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "fdtd_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "fdtd_set_velocity": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "fdtd_inject_source": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          _P, ctypes.c_int32, ctypes.c_float]),
    "fdtd_set_receivers": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32]),
    "fdtd_record_receivers": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32]),
    "fdtd_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fdtd_step_graph": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fdtd_get_field": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    "fdtd_set_field": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    "fdtd_reset": (ctypes.c_int, [_P]),
    "fdtd_get_step": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "fdtd_check_finite": (ctypes.c_int, [_P]),
    "fdtd_set_sentinel": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fdtd_state_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "fdtd_save_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "fdtd_load_state": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "fdtd_adjoint_workspace_size": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "fdtd_set_checkpointing": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t]),
    "fdtd_adjoint": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P]),
    "fdtd_adjoint_batch": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "fdtd_autotune": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "fdtd_set_plan": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32]),
    "fdtd_get_plan": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "fdtd_get_scale": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "fdtd_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fdtd_get_timing": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64)]),
    "fdtd_stream_probe": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, _P]),
    "fdtd_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fdtd_last_error": (ctypes.c_char_p, [_P]),
    "fdtd_destroy": (None, [_P]),
    "fdtd_forward_static": (ctypes.c_int, [ctypes.POINTER(ShotConfig), _P, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_float, _P, ctypes.c_int32,
                                           _P, _P, _P]),
    # first-order pressure-velocity path (include/fdtd_pv.h)
    "fdtd_pv_create": (ctypes.c_int, [ctypes.POINTER(PVConfig), _P, ctypes.POINTER(_P)]),
    "fdtd_pv_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "fdtd_pv_bind_workspace": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "fdtd_pv_set_pressure": (ctypes.c_int, [_P, _P]),
    "fdtd_pv_get_pressure": (ctypes.c_int, [_P, _P]),
    "fdtd_pv_set_source": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32]),
    "fdtd_pv_set_receivers": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, ctypes.c_int32]),
    "fdtd_pv_step": (ctypes.c_int, [_P, ctypes.c_int32]),
    "fdtd_pv_last_error": (ctypes.c_char_p, [_P]),
    "fdtd_pv_destroy": (None, [_P]),
}


def lib() -> ctypes.CDLL:
    """Load libfdtd.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libfdtd.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


def check(rc: int, ctx=None) -> None:
    if rc == FDTD_OK:
        return
    L = lib()
    msg = ""
    if ctx is not None:
        m = L.fdtd_last_error(ctx)
        msg = m.decode() if m else ""
    if not msg:
        msg = L.fdtd_strerror(rc).decode()
    if rc in (-1, -2):
        raise FDTDValueError(rc, msg)
    raise FDTDError(rc, msg)
