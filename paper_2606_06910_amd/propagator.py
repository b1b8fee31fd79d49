"""Propagator: Python handle on one fdtd_ctx (one or more shots).

PyTorch provides the device memory (workspace, model, traces, ...) and the
stream; the library does all the work.  Device tensors passed in are kept
referenced here for as long as the library borrows them.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import ShotConfig, check


@dataclass
class Shot:
    """Problem statement of one shot (grid, spacing, dt, layers, faces)."""

    n: Sequence[int]
    h: Sequence[float]
    dt: float
    cpml: Sequence[int] = (0, 0, 0, 0, 0, 0)
    face: Sequence[int] = (0, 0, 0, 0, 0, 0)
    exchange_every: int = 1
    R: float = 1e-8
    kappa_max: float = 5.0
    alpha_frac: float = 0.05
    v_ref: float = 0.0
    storage: int = _lib.F32
    variant: int = _lib.VARIANT_AUTO
    tblock_k: int = 1
    field_scale: float = 0.0

    def c(self) -> ShotConfig:
        s = ShotConfig()
        s.n[:] = [int(x) for x in self.n]
        s.h[:] = [float(x) for x in self.h]
        s.dt = float(self.dt)
        s.cpml[:] = [int(x) for x in self.cpml]
        s.face[:] = [int(x) for x in self.face]
        s.exchange_every = int(self.exchange_every)
        s.R = float(self.R)
        s.kappa_max = float(self.kappa_max)
        s.alpha_frac = float(self.alpha_frac)
        s.v_ref = float(self.v_ref)
        s.storage = int(self.storage)
        s.variant = int(self.variant)
        s.tblock_k = int(self.tblock_k)
        s.field_scale = float(self.field_scale)
        return s

    @property
    def shape(self):
        return (int(self.n[2]), int(self.n[1]), int(self.n[0]))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return ctypes.c_void_p(t.data_ptr())


class Propagator:
    def __init__(self, shots: List[Shot], device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        self.L = _lib.lib()
        self.shots = list(shots)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr = (ShotConfig * len(shots))(*[s.c() for s in shots])
        ctx = ctypes.c_void_p()
        rc = self.L.fdtd_create(arr, len(shots), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        check(rc)
        self.ctx = ctx
        nb = ctypes.c_size_t()
        check(self.L.fdtd_workspace_size(self.ctx, ctypes.byref(nb)), self.ctx)
        self.ws_bytes = int(nb.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        check(self.L.fdtd_bind_workspace(self.ctx, ctypes.c_void_p(base + off), self.ws_bytes), self.ctx)
        self._keep = {}

    # -- setup ---------------------------------------------------------------
    def set_velocity(self, shot: int, v: torch.Tensor) -> None:
        v = v.to(device=self.device, dtype=torch.float32).contiguous()
        assert tuple(v.shape) == self.shots[shot].shape, (tuple(v.shape), self.shots[shot].shape)
        check(self.L.fdtd_set_velocity(self.ctx, shot, _ptr(v)), self.ctx)

    def inject_source(self, shot: int, ijk, wavelet: torch.Tensor, amplitude: float = 1.0) -> None:
        w = wavelet.to(device=self.device, dtype=torch.float32).contiguous()
        self._keep[("wav", shot)] = w
        i, j, k = [int(x) for x in ijk]
        check(self.L.fdtd_inject_source(self.ctx, shot, i, j, k, _ptr(w), int(w.numel()), float(amplitude)),
              self.ctx)

    def set_receivers(self, shot: int, rec) -> None:
        r = torch.as_tensor(rec, dtype=torch.int32).reshape(-1, 3).to(self.device).contiguous()
        self._keep[("rec", shot)] = r
        check(self.L.fdtd_set_receivers(self.ctx, shot, _ptr(r), int(r.shape[0])), self.ctx)

    def record(self, shot: int, nt: int) -> torch.Tensor:
        """Allocate and register float32 traces [nt][nrec] for one shot."""
        r = self._keep.get(("rec", shot))
        nrec = 0 if r is None else int(r.shape[0])
        tr = torch.zeros((nt, max(nrec, 1)), dtype=torch.float32, device=self.device)
        self._keep[("tr", shot)] = tr
        check(self.L.fdtd_record_receivers(self.ctx, shot, _ptr(tr), int(nt)), self.ctx)
        return tr[:, :nrec]

    # -- stepping --------------------------------------------------------------
    def step(self, n: int, graph: bool = False) -> None:
        f = self.L.fdtd_step_graph if graph else self.L.fdtd_step
        check(f(self.ctx, int(n)), self.ctx)

    def reset(self) -> None:
        check(self.L.fdtd_reset(self.ctx), self.ctx)

    @property
    def nstep(self) -> int:
        s = ctypes.c_int64()
        check(self.L.fdtd_get_step(self.ctx, ctypes.byref(s)), self.ctx)
        return int(s.value)

    def get_field(self, shot: int = 0, which: int = 0) -> torch.Tensor:
        out = torch.empty(self.shots[shot].shape, dtype=torch.float32, device=self.device)
        check(self.L.fdtd_get_field(self.ctx, shot, which, _ptr(out)), self.ctx)
        return out

    def set_field(self, shot: int, which: int, f: torch.Tensor) -> None:
        f = f.to(device=self.device, dtype=torch.float32).contiguous()
        assert tuple(f.shape) == self.shots[shot].shape
        check(self.L.fdtd_set_field(self.ctx, shot, which, _ptr(f)), self.ctx)
        self.stream.synchronize()

    def save_state(self) -> torch.Tensor:
        """The full state of every shot and the step count, as an opaque device blob."""
        nb = ctypes.c_size_t()
        check(self.L.fdtd_state_size(self.ctx, ctypes.byref(nb)), self.ctx)
        blob = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        check(self.L.fdtd_save_state(self.ctx, ctypes.c_void_p(blob.data_ptr()), int(nb.value)), self.ctx)
        return blob

    def load_state(self, blob: torch.Tensor) -> None:
        """Restore a blob from save_state of a context with the same shot configurations."""
        assert blob.is_cuda and blob.dtype == torch.uint8 and blob.is_contiguous()
        check(self.L.fdtd_load_state(self.ctx, ctypes.c_void_p(blob.data_ptr()), int(blob.numel())), self.ctx)

    def check_finite(self) -> None:
        check(self.L.fdtd_check_finite(self.ctx), self.ctx)

    def set_sentinel(self, every: int) -> None:
        """Scan for NaN/Inf every `every` steps while stepping (0: off); step raises FDTDError then."""
        check(self.L.fdtd_set_sentinel(self.ctx, int(every)), self.ctx)

    def set_plan(self, shot: int, variant: int, tile_ry: int = 2, zchunk: int = 64, tblock_k: int = 1,
                 tile_cols: int = 1) -> None:
        check(self.L.fdtd_set_plan(self.ctx, shot, variant, tile_ry, zchunk, tblock_k, tile_cols), self.ctx)

    def plan(self, shot: int = 0):
        """(variant, tile_ry, tblock_k, tile_cols) of one shot."""
        v, ry, k, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(self.L.fdtd_get_plan(self.ctx, shot, ctypes.byref(v), ctypes.byref(ry), ctypes.byref(k), ctypes.byref(c)),
              self.ctx)
        return int(v.value), int(ry.value), int(k.value), int(c.value)

    def scale(self, shot: int = 0) -> float:
        s = ctypes.c_double()
        check(self.L.fdtd_get_scale(self.ctx, shot, ctypes.byref(s)), self.ctx)
        return float(s.value)

    def autotune(self, cache_path: Optional[str] = None) -> None:
        p = cache_path.encode() if cache_path else None
        check(self.L.fdtd_autotune(self.ctx, p), self.ctx)

    def set_timing(self, enable: bool) -> None:
        check(self.L.fdtd_set_timing(self.ctx, 1 if enable else 0), self.ctx)

    def timing(self, kernel_class: int = 0):
        """(mean ms, count) of one kernel class: 0 update outside the layer bands,
        1 psi, 2 receivers, 3 exchange, 4 band update, 5 temporal block."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        check(self.L.fdtd_get_timing(self.ctx, kernel_class, ctypes.byref(ms), ctypes.byref(n)), self.ctx)
        return float(ms.value), int(n.value)

    # -- adjoint -----------------------------------------------------------------
    def adjoint_workspace_size(self, shot: int, every: int, nt: int) -> int:
        nb = ctypes.c_size_t()
        check(self.L.fdtd_adjoint_workspace_size(self.ctx, shot, every, nt, ctypes.byref(nb)), self.ctx)
        return int(nb.value)

    def set_checkpointing(self, shot: int, every: int, nt: int) -> None:
        if every <= 0:
            check(self.L.fdtd_set_checkpointing(self.ctx, shot, 0, None, 0), self.ctx)
            self._keep.pop(("adj", shot), None)
            return
        nb = self.adjoint_workspace_size(shot, every, nt)
        buf = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        self._keep[("adj", shot)] = buf
        check(self.L.fdtd_set_checkpointing(self.ctx, shot, every, ctypes.c_void_p(buf.data_ptr() + off), nb),
              self.ctx)

    def adjoint(self, shot: int, nt: int, resid: torch.Tensor) -> torch.Tensor:
        r = resid.to(device=self.device, dtype=torch.float32).contiguous()
        g = torch.empty(self.shots[shot].shape, dtype=torch.float64, device=self.device)
        check(self.L.fdtd_adjoint(self.ctx, shot, int(nt), _ptr(r), _ptr(g)), self.ctx)
        return g

    def adjoint_all(self, nt: int, resids: Sequence[torch.Tensor]) -> List[torch.Tensor]:
        """Gradients of every shot in one batched reverse sweep (one residual per shot)."""
        assert len(resids) == len(self.shots)
        rs = [r.to(device=self.device, dtype=torch.float32).contiguous() for r in resids]
        gs = [torch.empty(sh.shape, dtype=torch.float64, device=self.device) for sh in self.shots]
        RA = (ctypes.c_void_p * len(rs))(*[r.data_ptr() for r in rs])
        GA = (ctypes.c_void_p * len(gs))(*[g.data_ptr() for g in gs])
        check(self.L.fdtd_adjoint_batch(self.ctx, int(nt), RA, GA), self.ctx)
        return gs

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.stream.synchronize()
            self.L.fdtd_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
