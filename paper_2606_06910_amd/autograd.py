"""torch.autograd.Function returning receiver traces with a velocity gradient.

Forward: one shot from rest through the library (checkpoints saved every
`every` steps).  Backward: fdtd_adjoint, the library's reverse-time sweep of
the exact transposed step with segment recomputation; it returns dJ/dv
accumulated in FP64 (cast to the dtype of v).  The layer profiles (v_ref)
and dt are parameters of the shot and are held fixed.
"""
from __future__ import annotations

from typing import Optional

import torch

from .propagator import Propagator, Shot


class FDTDFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v: torch.Tensor, prop: Propagator, shot: int, nt: int, every: int):
        prop.set_velocity(shot, v.detach())
        prop.set_checkpointing(shot, every, nt)
        traces = prop.record(shot, nt)
        prop.reset()
        prop.step(nt)
        ctx.prop, ctx.shot, ctx.nt = prop, shot, nt
        ctx.v_dtype = v.dtype
        return traces.clone()

    @staticmethod
    def backward(ctx, grad_traces: torch.Tensor):
        g = ctx.prop.adjoint(ctx.shot, ctx.nt, grad_traces.contiguous())
        return g.to(ctx.v_dtype), None, None, None, None


def simulate(v: torch.Tensor, shot: Shot, wavelet: torch.Tensor, src_ijk, rec_ijk, nt: int, every: int = 25,
             prop: Optional[Propagator] = None) -> torch.Tensor:
    """Traces [nt][nrec] of one shot for velocity v (differentiable in v).

    ``shot.v_ref`` should be set (> 0) when v changes between calls, so that
    the layer profiles stay fixed while the model is updated."""
    if prop is None:
        prop = Propagator([shot])
    prop.inject_source(0, src_ijk, wavelet)
    prop.set_receivers(0, rec_ijk)
    return FDTDFunction.apply(v, prop, 0, nt, every)
