"""Differentiable forward map (velocity, wavelet) -> receiver traces.

``FdModel.apply(v, wavelet, geom)`` runs the forward sweep of libfdwave.so;
its backward returns
  * dL/dv through the library's checkpointed adjoint-state computation
    (fd_vjp: forward checkpoints every ``geom.ckpt_every`` steps, segment
    recomputation, adjoint sweep, zero-lag imaging condition accumulated in
    FP64, dL/dm -> dL/dv = dL/dm * (-2 / v^3));
  * dL/dwavelet = F^T (dL/dd), the adjoint sweep read at the sources
    (fd_adjoint), since the traces are linear in the wavelet.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import api


@dataclass
class Geometry:
    """Everything about a shot except the two differentiable inputs."""

    h: tuple
    space_order: int
    nt: int
    dt: float
    src_idx: np.ndarray
    rec_idx: np.ndarray
    sponge: int = 0
    vref: float = 1500.0
    options: dict = field(default_factory=dict)
    ckpt_every: int = 0


class FdModel(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, wavelet, geom: Geometry):
        opts = dict(geom.options)
        out = api.forward(v.detach(), geom.h, geom.space_order, geom.nt, geom.dt, geom.src_idx,
                          wavelet.detach(), geom.rec_idx, sponge=geom.sponge, vref=geom.vref, **opts)
        ctx.save_for_backward(v.detach(), wavelet.detach())
        ctx.geom = geom
        return out["rec"]

    @staticmethod
    def backward(ctx, grad_traces):
        v, wavelet = ctx.saved_tensors
        g = ctx.geom
        y = grad_traces.contiguous().to(torch.float32)
        gv = gw = None
        opts = dict(g.options)
        if ctx.needs_input_grad[0]:
            gv = api.vjp(v, g.h, g.space_order, g.nt, g.dt, g.src_idx, wavelet, g.rec_idx, y,
                         sponge=g.sponge, vref=g.vref, ckpt_every=g.ckpt_every, **opts)
        if ctx.needs_input_grad[1]:
            gw = api.adjoint(v, g.h, g.space_order, g.nt, g.dt, g.src_idx, g.rec_idx, y,
                             sponge=g.sponge, vref=g.vref, **opts)["src"]
        return gv, gw, None


def fd_model(v, wavelet, geom: Geometry):
    """Receiver traces [nt][nr] for velocity v and source wavelet [nt][ns] (differentiable)."""
    return FdModel.apply(v, wavelet, geom)
