"""Differentiable forward map (velocity, wavelet) -> receiver traces.

``FdModel.apply(v, wavelet, geom)`` runs the forward sweep of libfdwave.so.
Reverse mode (backward) returns
  * dL/dv through the library's checkpointed adjoint-state computation
    (fd_vjp: forward checkpoints every ``geom.ckpt_every`` steps and segment
    recomputation, or the whole time axis stored, or ``"auto"``: the library
    picks one for the device's free memory; adjoint sweep, zero-lag imaging
    condition summed in FP32 over 64-step blocks into an FP64 image,
    dL/dm -> dL/dv = dL/dm * (-2 / v^3));
  * dL/dwavelet = F^T (dL/dd), the adjoint sweep read at the sources
    (fd_adjoint), since the traces are linear in the wavelet.
Forward mode (jvp, with ``torch.autograd.forward_ad`` dual tensors) returns
  * (dd/dv) dv through Born modelling (fd_born), plus
  * F dwavelet, the forward sweep driven by the wavelet's tangent.
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
    ckpt_every: int | str = 0


class FdModel(torch.autograd.Function):
    @staticmethod
    def forward(v, wavelet, geom: Geometry):
        opts = dict(geom.options)
        out = api.forward(v.detach(), geom.h, geom.space_order, geom.nt, geom.dt, geom.src_idx,
                          wavelet.detach(), geom.rec_idx, sponge=geom.sponge, vref=geom.vref, **opts)
        return out["rec"]

    @staticmethod
    def setup_context(ctx, inputs, output):
        v, wavelet, geom = inputs
        ctx.save_for_backward(v, wavelet)
        ctx.save_for_forward(v, wavelet)
        ctx.geom = geom

    @staticmethod
    def backward(ctx, grad_traces):
        v, wavelet = ctx.saved_tensors
        g = ctx.geom
        gv = gw = None
        opts = dict(g.options)
        with torch.no_grad():
            y = grad_traces.detach().contiguous().to(torch.float32)
            v, wavelet = v.detach(), wavelet.detach()
            if ctx.needs_input_grad[0]:
                gv = api.vjp(v, g.h, g.space_order, g.nt, g.dt, g.src_idx, wavelet, g.rec_idx, y,
                             sponge=g.sponge, vref=g.vref, ckpt_every=g.ckpt_every, **opts)
            if ctx.needs_input_grad[1]:
                gw = api.adjoint(v, g.h, g.space_order, g.nt, g.dt, g.src_idx, g.rec_idx, y,
                                 sponge=g.sponge, vref=g.vref, **opts)["src"]
        return gv, gw, None

    @staticmethod
    def jvp(ctx, v_t, wavelet_t, geom_t):
        v, wavelet = ctx.saved_tensors
        g = ctx.geom
        opts = dict(g.options)
        out = None
        with torch.no_grad():
            v, wavelet = v.detach(), wavelet.detach()
            if v_t is not None:
                out = api.born(v, g.h, g.space_order, g.nt, g.dt, g.src_idx, wavelet, g.rec_idx,
                               v_t.detach(), sponge=g.sponge, vref=g.vref, **opts)
            if wavelet_t is not None:
                d = api.forward(v, g.h, g.space_order, g.nt, g.dt, g.src_idx, wavelet_t.detach(), g.rec_idx,
                                sponge=g.sponge, vref=g.vref, **opts)["rec"]
                out = d if out is None else out + d
        return out


def fd_model(v, wavelet, geom: Geometry):
    """Receiver traces [nt][nr] for velocity v and source wavelet [nt][ns] (differentiable)."""
    return FdModel.apply(v, wavelet, geom)
