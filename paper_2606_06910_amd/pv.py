"""Handle for the first-order pressure-velocity path (include/fdtd_pv.h).

Argument marshalling only: the library's HIP kernels do every step.  PyTorch
provides the device memory (workspace, pressure, wavelet, receivers, traces)
and the stream; device tensors passed in are kept alive by the handle while
the library borrows them.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import FDTD_OK, FDTDError, FDTDValueError, PVConfig


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class PVPropagator:
    """One grid of the first-order system: p, v_x, v_y, v_z and the layer memory."""

    def __init__(self, n: Sequence[int], cpml: Sequence[int] = (20,) * 6, lam: float = 0.05, variant: int = 0,
                 device: str = "cuda", stream: Optional[torch.cuda.Stream] = None):
        self.L = _lib.lib()
        self.n = tuple(int(x) for x in n)
        self.shape = (self.n[2], self.n[1], self.n[0])
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg = PVConfig()
        cfg.n[:] = list(self.n)
        cfg.cpml[:] = [int(x) for x in cpml]
        cfg.lam = float(lam)
        cfg.variant = int(variant)
        ctx = ctypes.c_void_p()
        self._check(self.L.fdtd_pv_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(ctx)), None)
        self.ctx = ctx
        nb = ctypes.c_size_t()
        self._check(self.L.fdtd_pv_workspace_size(self.ctx, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.ws.data_ptr()) % 256
        self._check(self.L.fdtd_pv_bind_workspace(self.ctx, ctypes.c_void_p(self.ws.data_ptr() + off),
                                                  self.ws_bytes))
        self._keep = {}

    def _check(self, rc: int, ctx="self") -> None:
        if rc == FDTD_OK:
            return
        c = self.ctx if ctx == "self" else ctx
        msg = ""
        if c is not None:
            m = self.L.fdtd_pv_last_error(c)
            msg = m.decode() if m else ""
        if not msg:
            msg = self.L.fdtd_strerror(rc).decode()
        raise (FDTDValueError if rc == -1 else FDTDError)(rc, msg)

    def set_pressure(self, p: torch.Tensor) -> None:
        p = p.to(device=self.device, dtype=torch.float32).contiguous()
        assert tuple(p.shape) == self.shape, (tuple(p.shape), self.shape)
        self._keep["p_in"] = p
        self._check(self.L.fdtd_pv_set_pressure(self.ctx, _ptr(p)))

    def get_pressure(self) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        self._check(self.L.fdtd_pv_get_pressure(self.ctx, _ptr(out)))
        return out

    def set_source(self, ijk, wavelet: torch.Tensor) -> None:
        w = wavelet.to(device=self.device, dtype=torch.float32).contiguous()
        self._keep["wav"] = w
        i, j, k = (int(x) for x in ijk)
        self._check(self.L.fdtd_pv_set_source(self.ctx, i, j, k, _ptr(w), int(w.numel())))

    def record(self, rec, nt: int) -> torch.Tensor:
        """Receivers (nrec, 3) as (i, j, k); returns the (nt, nrec) traces tensor
        the following steps fill."""
        r = torch.as_tensor(rec, dtype=torch.int32).reshape(-1, 3).to(self.device).contiguous()
        tr = torch.zeros((int(nt), r.shape[0]), dtype=torch.float32, device=self.device)
        self._keep["rec"], self._keep["traces"] = r, tr
        self._check(self.L.fdtd_pv_set_receivers(self.ctx, _ptr(r), int(r.shape[0]), _ptr(tr), int(nt)))
        return tr

    def step(self, nsteps: int) -> None:
        self._check(self.L.fdtd_pv_step(self.ctx, int(nsteps)))

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.stream.synchronize()
            self.L.fdtd_pv_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
