"""The autograd.Function over the HIP library: gradients agree with the fused
least-squares gradient, with the oracle's vector-Jacobian product and with
finite differences."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api
from paper_1707_02347_amd.autograd import Geometry, fd_model

pytestmark = pytest.mark.gpu
DEV = "cuda"


def setup(opts=None):
    shape, so, nt = (36, 34, 40), 4, 100
    v = synth.smooth_velocity(shape, seed=3, sigma=4.0)
    dt = 0.8 * 0.5 * 10.0 / float(v.max())
    src = synth.centre_source(shape, depth=10)
    rec = synth.receiver_line(shape, 10, depth=10)
    w = synth.ricker(nt, dt, 25.0)[:, None].copy()
    geom = Geometry(h=(10.0, 10.0, 10.0), space_order=so, nt=nt, dt=dt, src_idx=src, rec_idx=rec,
                    sponge=5, vref=4500.0, options=opts or {}, ckpt_every=16)
    vtrue = synth.blob_velocity(v, amp=0.05, width_frac=1 / 8)
    prob = oracle.Problem(vtrue.numpy().astype(np.float64), geom.h, so, nt, dt, 5, 4500.0, src, rec)
    d_obs = oracle.forward(prob, amp=w.astype(np.float64))["rec"].astype(np.float32)
    return v, w, geom, d_obs


@pytest.mark.parametrize("opts", [{}, dict(variant=L.FD_VARIANT_TBLOCK, tblock=2)])
def test_autograd_velocity_gradient_equals_fused_gradient(opts):
    v, w, g, d_obs = setup(opts)
    vd = v.to(DEV).requires_grad_(True)
    wd = torch.from_numpy(w).to(DEV)
    dobs = torch.from_numpy(d_obs).to(DEV)
    d = fd_model(vd, wd, g)
    loss = 0.5 * ((d - dobs) ** 2).sum()
    loss.backward()
    J, gv, _ = api.gradient(v.to(DEV), g.h, g.space_order, g.nt, g.dt, g.src_idx, wd, g.rec_idx, dobs,
                            sponge=g.sponge, vref=g.vref, ckpt_every=g.ckpt_every, **opts)
    assert torch.equal(vd.grad, gv)
    assert abs(float(loss) - J) <= 1e-5 * J


def test_autograd_with_automatic_storage_equals_checkpointing():
    """Geometry(ckpt_every="auto"): the library picks the storage scheme for the
    free device memory; the backward pass gives the checkpointed result."""
    import dataclasses

    v, w, g, d_obs = setup()
    wd, dobs = torch.from_numpy(w).to(DEV), torch.from_numpy(d_obs).to(DEV)
    grads = []
    for geom in (g, dataclasses.replace(g, ckpt_every="auto")):
        vd = v.to(DEV).requires_grad_(True)
        loss = 0.5 * ((fd_model(vd, wd, geom) - dobs) ** 2).sum()
        loss.backward()
        grads.append(vd.grad)
    assert torch.equal(grads[0], grads[1])
    assert float(grads[0].abs().max()) > 0


def test_autograd_velocity_gradient_matches_oracle_vjp():
    v, w, g, d_obs = setup()
    vd = v.to(DEV).requires_grad_(True)
    wd = torch.from_numpy(w).to(DEV)
    rng = np.random.default_rng(0)
    y = rng.standard_normal((g.nt, len(g.rec_idx))).astype(np.float32)
    d = fd_model(vd, wd, g)
    (d * torch.from_numpy(y).to(DEV)).sum().backward()
    prob = oracle.Problem(v.numpy().astype(np.float64), g.h, g.space_order, g.nt, g.dt, g.sponge, g.vref,
                          g.src_idx, g.rec_idx)
    gref, _ = oracle.vjp(prob, w.astype(np.float64), y.astype(np.float64))
    got = vd.grad.cpu().numpy()
    err = np.linalg.norm(got - gref) / np.linalg.norm(gref)
    print(f"vjp vs oracle rel_l2 {err:.3e}")
    assert err <= 1e-5


def test_autograd_wavelet_gradient_finite_difference():
    v, w, g, d_obs = setup()
    vd = v.to(DEV)
    wd = torch.from_numpy(w).to(DEV).requires_grad_(True)
    dobs = torch.from_numpy(d_obs).to(DEV)
    loss = 0.5 * ((fd_model(vd, wd, g) - dobs) ** 2).sum()
    loss.backward()
    rng = np.random.default_rng(1)
    dw = torch.from_numpy(rng.standard_normal(w.shape).astype(np.float32)).to(DEV)
    eps = 1e-2

    def L_at(ww):
        with torch.no_grad():
            return float(0.5 * ((fd_model(vd, ww, g) - dobs) ** 2).double().sum())

    fd = (L_at(wd.detach() + eps * dw) - L_at(wd.detach() - eps * dw)) / (2 * eps)
    an = float((wd.grad.double() * dw.double()).sum())
    assert abs(fd - an) <= 1e-3 * abs(an)


def test_autograd_velocity_gradient_finite_difference():
    v, w, g, d_obs = setup()
    wd = torch.from_numpy(w).to(DEV)
    dobs = torch.from_numpy(d_obs).to(DEV)
    vd = v.to(DEV).requires_grad_(True)
    loss = 0.5 * ((fd_model(vd, wd, g) - dobs) ** 2).sum()
    loss.backward()
    rng = np.random.default_rng(2)
    dv = torch.from_numpy(synth.smooth_velocity(v.shape, seed=9, sigma=3.0).numpy() - 3000.0).to(DEV) * 0.01
    eps = 1.0

    def L_at(vv):
        with torch.no_grad():
            return float(0.5 * ((fd_model(vv, wd, g) - dobs) ** 2).double().sum())

    fd = (L_at(v.to(DEV) + eps * dv) - L_at(v.to(DEV) - eps * dv)) / (2 * eps)
    an = float((vd.grad.double() * dv.double()).sum())
    print(f"velocity FD {fd:.6e} vs adjoint {an:.6e}")
    assert abs(fd - an) <= 1e-2 * abs(an)


def _jvp(f, x, t):
    import torch.autograd.forward_ad as fwAD

    with fwAD.dual_level():
        out = fwAD.unpack_dual(f(fwAD.make_dual(x, t)))
        return out.primal, out.tangent


def test_forward_mode_velocity_tangent_is_born_modelling():
    """Forward mode (dual tensors) along dv equals fd_born, matches the oracle's
    Born traces, and pairs with the reverse-mode gradient: <J dv, y> = <dv, J^T y>."""
    v, w, g, _ = setup()
    vd = v.to(DEV)
    wd = torch.from_numpy(w).to(DEV)
    dv = (synth.smooth_velocity(tuple(v.shape), seed=31, sigma=3.0) - 3000.0).to(DEV)
    d, dd = _jvp(lambda vv: fd_model(vv, wd, g), vd, dv)
    born = api.born(vd, g.h, g.space_order, g.nt, g.dt, g.src_idx, wd, g.rec_idx, dv, sponge=g.sponge, vref=g.vref)
    assert torch.equal(dd, born)
    prob = oracle.Problem(v.numpy().astype(np.float64), g.h, g.space_order, g.nt, g.dt, g.sponge, g.vref,
                          g.src_idx, g.rec_idx)
    ref = oracle.born(prob, w.astype(np.float64), dv.cpu().numpy().astype(np.float64))
    assert np.linalg.norm(dd.cpu().numpy() - ref) <= 1e-5 * np.linalg.norm(ref)
    # cotangent: the Born traces themselves plus seeded noise at a tenth of
    # their size, so that <J dv, y> ~ |J dv|^2 is not a cancelling sum and the
    # dot test's 1e-5 bound is relative to the inner product itself
    noise = torch.randn(d.shape, generator=torch.Generator(device=DEV).manual_seed(7), device=DEV)
    y = dd.detach() + 0.1 * float(dd.double().pow(2).mean().sqrt()) * noise
    vg = vd.clone().requires_grad_(True)
    (gv,) = torch.autograd.grad((fd_model(vg, wd, g) * y).sum(), vg)
    lhs, rhs = float((dd.double() * y.double()).sum()), float((dv.double() * gv.double()).sum())
    print(f"dot test <J dv, y> {lhs:.9e} <dv, J^T y> {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_forward_mode_wavelet_tangent_is_the_forward_sweep():
    v, w, g, _ = setup()
    vd = v.to(DEV)
    wd = torch.from_numpy(w).to(DEV)
    wt = torch.from_numpy(np.ascontiguousarray(w[::-1])).to(DEV)
    _, dd = _jvp(lambda ww: fd_model(vd, ww, g), wd, wt)
    ref = api.forward(vd, g.h, g.space_order, g.nt, g.dt, g.src_idx, wt, g.rec_idx, sponge=g.sponge, vref=g.vref)
    assert torch.equal(dd, ref["rec"])
