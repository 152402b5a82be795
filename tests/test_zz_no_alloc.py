"""fd_forward_noalloc (the forward sweep with its scratch in the library's
static device array) called through the C ABI equals fd_forward with a
caller workspace, bit for bit: traces and the final state pair, on two calls
in a row, the second on a smaller grid of another space order, and a call
whose scratch would exceed the array is refused with FD_ESCRATCH."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(shape, so, nt, seed):
    v = synth.smooth_velocity(shape, seed=seed, sigma=3.0)
    dt = 0.8 * 2.0 / (float(v.max()) * np.sqrt(3 * 7.5)) * 10.0
    src = synth.centre_source(shape, depth=shape[-1] // 3)
    rec = synth.receiver_line(shape, 5, depth=shape[-1] // 3)
    amp = torch.from_numpy(synth.ricker(nt, dt, 30.0)[:, None].copy()).to(DEV)
    return v.to(DEV), dt, src, rec, amp


def _noalloc(v, h, so, nt, dt, src_idx, amp, rec_idx, u0, um1, sponge, vref, variant=0):
    shape = tuple(v.shape)
    grid = L.make_grid(shape, h, so, sponge, vref)
    tm = L.make_time(nt, dt)
    src = L.Points(src_idx, amp, len(shape))
    rec = L.Points(rec_idx, None, len(shape))
    o = L.make_options(variant)
    state = torch.stack([u0, um1]).contiguous()
    rec_out = torch.zeros((int(nt), rec.n), dtype=torch.float32, device=v.device)
    rc = L.fd_forward_noalloc(C.byref(grid), C.byref(tm), L._ptr(v), C.byref(src.s), C.byref(rec.s),
                              L._ptr(rec_out), L._ptr(state), C.byref(o), L._stream(v.device))
    L._check(rc, "fd_forward_noalloc")
    return rec_out, state


@pytest.mark.parametrize("variant", [0, L.FD_VARIANT_STREAM])
def test_noalloc_forward_equals_workspace_forward_twice(variant):
    cases = [((44, 40, 64), 8, 40, 11), ((30, 28, 36), 4, 33, 12)]  # the second smaller
    for shape, so, nt, seed in cases:
        v, dt, src, rec, amp = _case(shape, so, nt, seed)
        g = torch.Generator(device=DEV).manual_seed(seed)
        u0 = 1e-3 * torch.randn(shape, generator=g, device=DEV)
        um1 = 1e-3 * torch.randn(shape, generator=g, device=DEV)
        ref = api.forward(v, [10.0] * 3, so, nt, dt, src, amp, rec, u0=u0, um1=um1, sponge=5, vref=4500.0,
                          variant=variant)
        tr, st = _noalloc(v, [10.0] * 3, so, nt, dt, src, amp, rec, u0, um1, 5, 4500.0, variant)
        torch.cuda.synchronize()
        assert float(ref["rec"].abs().max()) > 0
        assert torch.equal(tr, ref["rec"]), shape
        assert torch.equal(st[0], ref["u"]), shape
        assert torch.equal(st[1], ref["u_prev"]), shape


def test_noalloc_refuses_a_grid_beyond_its_scratch():
    shape = (160, 160, 160)
    grid = L.make_grid(shape, [10.0] * 3, 8, 0, 1500.0)
    tm = L.make_time(4, 1e-4)
    o = L.make_options()
    assert L.fd_workspace_size(C.byref(grid), C.byref(tm), None, None, C.byref(o),
                               L.FD_OP_FORWARD) > L.FD_NOALLOC_SCRATCH_BYTES
    v = torch.full(shape, 2000.0, device=DEV)
    rc = L.fd_forward_noalloc(C.byref(grid), C.byref(tm), L._ptr(v), None, None, None, None, C.byref(o),
                              L._stream(v.device))
    assert rc == L.FD_ESCRATCH
    assert "static" in L.strerror(rc)
