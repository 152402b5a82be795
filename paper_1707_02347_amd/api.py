"""Torch-facing wrappers over the C ABI: device buffers come from PyTorch, the
work runs on the current HIP stream, every step is done by libfdwave.so.

Shapes: a velocity model ``v`` is a float32 CUDA tensor of 1, 2 or 3 dims
(last axis contiguous); point indices are integer arrays [n][ndim] (float
arrays: positions between nodes, multilinear; ``Sinc(pos, r)``: windowed sinc); sample
arrays are float32 CUDA tensors [nt][n].
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

Sinc = L.Sinc  # positions with Kaiser-windowed sinc interpolation: Sinc(pos, r)


def _dev_f32(t, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.contiguous()


def _opts(variant=0, tile=(0, 0, 0), tblock=0, ckpt_every=0, flags=0):
    return L.make_options(variant, tile, tblock, ckpt_every, flags)


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _opts_storage(variant, tile, tblock, ckpt_every, flags, grid, tm, src, rec, op, mem_budget, device):
    """Options of a gradient-type call.  ckpt_every="auto" lets fd_gradient_storage
    choose between storing the whole time axis and checkpointing, for mem_budget
    bytes of workspace (default: 80 % of the device's free memory)."""
    if ckpt_every != "auto":
        if mem_budget is not None:
            raise ValueError("mem_budget applies to ckpt_every='auto' only")
        return _opts(variant, tile, tblock, ckpt_every, flags)
    o = _opts(variant, tile, tblock, 0, flags)
    budget = mem_budget
    if budget is None:
        budget = int(0.8 * torch.cuda.mem_get_info(device)[0])
    need = C.c_size_t(0)
    rc = L.fd_gradient_storage(C.byref(grid), C.byref(tm), C.byref(src.s), C.byref(rec.s), op, int(budget),
                               C.byref(o), C.byref(need))
    if rc == L.FD_EWORKSPACE and mem_budget is None:
        rc = L.FD_OK  # no explicit budget: try the smallest footprint anyway
    L._check(rc, "fd_gradient_storage")
    return o


def forward(v, h, so, nt, dt, src_idx=None, src_amp=None, rec_idx=None, u0=None, um1=None,
            sponge=0, vref=1500.0, variant=0, tile=(0, 0, 0), tblock=0, flags=0):
    """Forward sweep; returns dict(rec=[nt][nr], u=u^nt, u_prev=u^{nt-1})."""
    v = _dev_f32(v, "v")
    shape = tuple(v.shape)
    nd = len(shape)
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    amp = None if src_amp is None else _dev_f32(src_amp, "src_amp")
    src = L.Points(src_idx, amp, nd)
    rec = L.Points(rec_idx, None, nd)
    o = _opts(variant, tile, tblock, 0, flags)
    state = torch.zeros((2,) + shape, dtype=torch.float32, device=v.device)
    if u0 is not None:
        state[0].copy_(u0)
    if um1 is not None:
        state[1].copy_(um1)
    rec_out = torch.zeros((int(nt), rec.n), dtype=torch.float32, device=v.device)
    nbytes = L.fd_workspace_size(C.byref(grid), C.byref(tm), C.byref(src.s), C.byref(rec.s), C.byref(o),
                                 L.FD_OP_FORWARD)
    ws = _workspace(nbytes, v.device)
    rc = L.fd_forward(C.byref(grid), C.byref(tm), L._ptr(v), C.byref(src.s), C.byref(rec.s),
                      L._ptr(rec_out) if rec.n else None, L._ptr(state), L._ptr(ws), ws.numel(),
                      C.byref(o), L._stream(v.device))
    L._check(rc, "fd_forward")
    return {"rec": rec_out, "u": state[0], "u_prev": state[1]}


def adjoint(v, h, so, nt, dt, src_idx, rec_idx, rec_amp, sponge=0, vref=1500.0, variant=0,
            tile=(0, 0, 0), tblock=0, flags=0):
    """Adjoint sweep: traces rec_amp [nt][nr] -> F^T y at the sources [nt][ns]; also (lambda^1, lambda^2)."""
    v = _dev_f32(v, "v")
    shape = tuple(v.shape)
    nd = len(shape)
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    src = L.Points(src_idx, None, nd)
    rec = L.Points(rec_idx, _dev_f32(rec_amp, "rec_amp"), nd)
    o = _opts(variant, tile, tblock, 0, flags)
    out = torch.zeros((int(nt), src.n), dtype=torch.float32, device=v.device)
    lam = torch.zeros((2,) + shape, dtype=torch.float32, device=v.device)
    nbytes = L.fd_workspace_size(C.byref(grid), C.byref(tm), C.byref(src.s), C.byref(rec.s), C.byref(o),
                                 L.FD_OP_ADJOINT)
    ws = _workspace(nbytes, v.device)
    rc = L.fd_adjoint(C.byref(grid), C.byref(tm), L._ptr(v), C.byref(src.s), C.byref(rec.s),
                      L._ptr(out) if src.n else None, L._ptr(lam), L._ptr(ws), ws.numel(), C.byref(o),
                      L._stream(v.device))
    L._check(rc, "fd_adjoint")
    return {"src": out, "lam": lam}


def gradient(v, h, so, nt, dt, src_idx, src_amp, rec_idx, d_obs, sponge=0, vref=1500.0, variant=0,
             tile=(0, 0, 0), tblock=0, ckpt_every=0, flags=0, mem_budget=None):
    """Least-squares misfit and dJ/dv (adjoint state); returns (J, grad_v, residual).
    ckpt_every: checkpoint interval (0 = 50, >= nt = whole time axis stored, "auto" =
    chosen for mem_budget bytes of workspace)."""
    v = _dev_f32(v, "v")
    shape = tuple(v.shape)
    nd = len(shape)
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    src = L.Points(src_idx, _dev_f32(src_amp, "src_amp"), nd)
    rec = L.Points(rec_idx, _dev_f32(d_obs, "d_obs"), nd)
    o = _opts_storage(variant, tile, tblock, ckpt_every, flags, grid, tm, src, rec, L.FD_OP_GRADIENT, mem_budget,
                      v.device)
    gv = torch.zeros(shape, dtype=torch.float32, device=v.device)
    res = torch.zeros((int(nt), rec.n), dtype=torch.float32, device=v.device)
    J = C.c_double(0.0)
    nbytes = L.fd_workspace_size(C.byref(grid), C.byref(tm), C.byref(src.s), C.byref(rec.s), C.byref(o),
                                 L.FD_OP_GRADIENT)
    ws = _workspace(nbytes, v.device)
    rc = L.fd_gradient(C.byref(grid), C.byref(tm), L._ptr(v), C.byref(src.s), C.byref(rec.s), L._ptr(gv),
                       C.byref(J), L._ptr(res) if rec.n else None, L._ptr(ws), ws.numel(), C.byref(o),
                       L._stream(v.device))
    L._check(rc, "fd_gradient")
    return float(J.value), gv, res


def vjp(v, h, so, nt, dt, src_idx, src_amp, rec_idx, y, sponge=0, vref=1500.0, variant=0,
        tile=(0, 0, 0), tblock=0, ckpt_every=0, flags=0, mem_budget=None):
    """(dd/dv)^T y for trace cotangent y [nt][nr]; ckpt_every as in gradient()."""
    v = _dev_f32(v, "v")
    shape = tuple(v.shape)
    nd = len(shape)
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    src = L.Points(src_idx, _dev_f32(src_amp, "src_amp"), nd)
    rec = L.Points(rec_idx, _dev_f32(y, "y"), nd)
    o = _opts_storage(variant, tile, tblock, ckpt_every, flags, grid, tm, src, rec, L.FD_OP_VJP, mem_budget,
                      v.device)
    gv = torch.zeros(shape, dtype=torch.float32, device=v.device)
    nbytes = L.fd_workspace_size(C.byref(grid), C.byref(tm), C.byref(src.s), C.byref(rec.s), C.byref(o),
                                 L.FD_OP_VJP)
    ws = _workspace(nbytes, v.device)
    rc = L.fd_vjp(C.byref(grid), C.byref(tm), L._ptr(v), C.byref(src.s), C.byref(rec.s), L._ptr(gv),
                  L._ptr(ws), ws.numel(), C.byref(o), L._stream(v.device))
    L._check(rc, "fd_vjp")
    return gv


def born(v, h, so, nt, dt, src_idx, src_amp, rec_idx, dv, sponge=0, vref=1500.0, variant=0,
         tile=(0, 0, 0), tblock=0, flags=0):
    """Born (linearised) traces (dd/dv) dv [nt][nr] for a velocity perturbation dv."""
    v = _dev_f32(v, "v")
    shape = tuple(v.shape)
    nd = len(shape)
    dv = _dev_f32(dv, "dv")
    if tuple(dv.shape) != shape:
        raise ValueError("dv must have the shape of v")
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    src = L.Points(src_idx, _dev_f32(src_amp, "src_amp"), nd)
    rec = L.Points(rec_idx, None, nd)
    o = _opts(variant, tile, tblock, 0, flags)
    dd = torch.zeros((int(nt), rec.n), dtype=torch.float32, device=v.device)
    nbytes = L.fd_workspace_size(C.byref(grid), C.byref(tm), C.byref(src.s), C.byref(rec.s), C.byref(o),
                                 L.FD_OP_BORN)
    ws = _workspace(nbytes, v.device)
    rc = L.fd_born(C.byref(grid), C.byref(tm), L._ptr(v), L._ptr(dv), C.byref(src.s), C.byref(rec.s),
                   L._ptr(dd) if rec.n else None, L._ptr(ws), ws.numel(), C.byref(o), L._stream(v.device))
    L._check(rc, "fd_born")
    return dd


def autotune(shape, h, so, dt, device="cuda", sponge=0, vref=1500.0, nt=8, variant=0, tblock=0):
    """Run the library's autotuner for this grid; returns the chosen options as a dict."""
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    o = _opts(variant, (0, 0, 0), tblock)
    nbytes = L.fd_workspace_size(C.byref(grid), C.byref(L.make_time(8, dt)), None, None, None,
                                 L.FD_OP_FORWARD)
    ws = _workspace(nbytes, device)
    rc = L.fd_autotune(C.byref(grid), C.byref(tm), C.byref(o), L._ptr(ws), ws.numel(), L._stream(device))
    L._check(rc, "fd_autotune")
    return {"variant": o.variant, "tile": tuple(o.tile), "tblock": o.tblock}


def last_config():
    return L.fd_last_config()


def _shot_struct(sh, op, keep):
    """Fill an fd_shot from a dict (v, h, so, nt, dt, src_idx, src_amp, rec_idx, [d_obs], options)."""
    v = _dev_f32(sh["v"], "v")
    nd = v.dim()
    s = L.fd_shot()
    s.grid = L.make_grid(tuple(v.shape), sh["h"], sh["so"], sh.get("sponge", 0), sh.get("vref", 1500.0))
    s.time = L.make_time(sh["nt"], sh["dt"])
    s.v = L._ptr(v)
    src = L.Points(sh["src_idx"], _dev_f32(sh["src_amp"], "src_amp"), nd)
    d_obs = sh.get("d_obs")
    rec = L.Points(sh["rec_idx"], None if d_obs is None else _dev_f32(d_obs, "d_obs"), nd)
    s.src = src.s
    s.rec = rec.s
    out = {}
    if op == L.FD_OP_FORWARD:
        out["rec"] = torch.zeros((int(sh["nt"]), rec.n), dtype=torch.float32, device=v.device)
        s.rec_out = L._ptr(out["rec"]) if rec.n else None
    else:
        out["grad_v"] = torch.zeros(tuple(v.shape), dtype=torch.float32, device=v.device)
        s.grad_v = L._ptr(out["grad_v"])
    s.opts = _opts(**sh.get("options", {}))
    keep += [v, src, rec, out]
    return s, out


def forward_batch(shots, graph=True):
    """Forward sweeps of many shots (uneven grids / orders); returns a list of trace tensors."""
    keep, outs = [], []
    arr = (L.fd_shot * len(shots))()
    for i, sh in enumerate(shots):
        arr[i], o = _shot_struct(sh, L.FD_OP_FORWARD, keep)
        outs.append(o)
    nbytes = L.fd_batch_workspace_size(len(shots), arr, L.FD_OP_FORWARD)
    dev = shots[0]["v"].device
    ws = _workspace(nbytes, dev)
    rc = L.fd_forward_batch(len(shots), arr, L._ptr(ws), ws.numel(), L.FD_BATCH_GRAPH if graph else 0,
                            L._stream(dev))
    L._check(rc, "fd_forward_batch")
    return [o["rec"] for o in outs]


def gradient_batch(shots, graph=True):
    """Least-squares gradients of many shots; returns (misfits, list of grad_v tensors)."""
    keep, outs = [], []
    arr = (L.fd_shot * len(shots))()
    for i, sh in enumerate(shots):
        arr[i], o = _shot_struct(sh, L.FD_OP_GRADIENT, keep)
        outs.append(o)
    nbytes = L.fd_batch_workspace_size(len(shots), arr, L.FD_OP_GRADIENT)
    dev = shots[0]["v"].device
    ws = _workspace(nbytes, dev)
    rc = L.fd_gradient_batch(len(shots), arr, L._ptr(ws), ws.numel(), L.FD_BATCH_GRAPH if graph else 0,
                             L._stream(dev))
    L._check(rc, "fd_gradient_batch")
    return [float(arr[i].misfit) for i in range(len(shots))], [o["grad_v"] for o in outs]


def batch_autotune(shots):
    """Let the library's batch tuner choose one kernel per space-order class for
    the shots whose options are automatic; updates each shot's ``options`` dict
    (variant, tile, tblock) in place and returns the list of chosen options."""
    keep = []
    arr = (L.fd_shot * len(shots))()
    for i, sh in enumerate(shots):
        arr[i], _ = _shot_struct(sh, L.FD_OP_FORWARD, keep)
    nbytes = L.fd_batch_workspace_size(len(shots), arr, L.FD_OP_FORWARD)
    dev = shots[0]["v"].device
    ws = _workspace(nbytes, dev)
    rc = L.fd_batch_autotune(len(shots), arr, L._ptr(ws), ws.numel(), L._stream(dev))
    L._check(rc, "fd_batch_autotune")
    out = []
    for i, sh in enumerate(shots):
        o = arr[i].opts
        chosen = {"variant": int(o.variant), "tile": tuple(int(t) for t in o.tile), "tblock": int(o.tblock)}
        sh["options"] = dict(sh.get("options", {}), **chosen)
        out.append(chosen)
    return out
