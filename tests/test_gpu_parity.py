"""GPU parity: the HIP path against the FP64 oracle, and every compiled kernel
configuration against the untiled kernel (bit for bit).

Tolerances: forward and adjoint fields/traces within relative L2 1e-5 of the
oracle; gradients within the bound stated at each test; all GPU variants
bit-identical to the untiled FP32 kernel.
"""
import ctypes as C
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api

pytestmark = pytest.mark.gpu
DEV = "cuda"


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def stable_dt(v_max, h, so, ndim, frac=0.8):
    c = oracle.weights(so)
    S = -c[0] - 2 * sum(c[k] * (-1) ** k for k in range(1, so // 2 + 1))
    return frac * 2.0 / (v_max * math.sqrt(S * sum(1.0 / hh ** 2 for hh in h[:ndim])))


def make_case(shape, so, nt, sponge, f0=15.0, seed=1707, nsrc=1, nrec=8, depth=None):
    nd = len(shape)
    h = [10.0] * nd
    v = synth.smooth_velocity(shape, seed=seed, sigma=4.0)
    dt = stable_dt(float(v.max()), h, so, nd)
    d = depth if depth is not None else min(shape[-1] // 3, 20)
    src = synth.centre_source(shape, depth=d)
    if nsrc > 1:
        rng = np.random.default_rng(seed)
        extra = np.stack([rng.integers(0, n, nsrc - 1) for n in shape], 1).astype(np.int32)
        src = np.concatenate([src, extra], 0)
    if nd == 3:
        rec = synth.receiver_line(shape, nrec, depth=d)
    elif nd == 2:
        rec = np.stack([np.linspace(0, shape[0] - 1, nrec).astype(np.int32), np.full(nrec, d, np.int32)], 1)
    else:
        rec = np.linspace(0, shape[0] - 1, nrec).astype(np.int32)[:, None]
    amp = np.stack([synth.ricker(nt, dt, f0, delay=1.0 / f0 + 0.002 * s) for s in range(len(src))], 1)
    return dict(shape=shape, so=so, nt=nt, h=h, v=v, dt=dt, src=src, rec=rec, amp=np.ascontiguousarray(amp),
                sponge=sponge, vref=4500.0)


def oracle_forward(cs, u0=None, um1=None):
    prob = oracle.Problem(cs["v"].numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"],
                          cs["sponge"], cs["vref"], cs["src"], cs["rec"])
    return oracle.forward(prob, amp=cs["amp"].astype(np.float64), u0=u0, um1=um1)


def gpu_forward(cs, u0=None, um1=None, **opts):
    return api.forward(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
                       torch.from_numpy(cs["amp"]).to(DEV), cs["rec"], u0=u0, um1=um1,
                       sponge=cs["sponge"], vref=cs["vref"], **opts)


# every compiled configuration the forward sweep can run (variant, tile, tblock)
def configs_for(so, small_chunk=7):
    M = so // 2
    out = [dict(variant=L.FD_VARIANT_NAIVE)]
    # (tile rows, rows per thread, time levels) of every compiled configuration
    shapes = {1: [(32, 8, 1), (16, 4, 1), (32, 4, 1), (32, 16, 1), (32, 4, 2), (32, 2, 2), (32, 4, 3),
                  (32, 2, 3), (32, 4, 4), (32, 2, 4)],
              2: [(32, 8, 1), (16, 4, 1), (32, 4, 1), (32, 16, 1), (32, 4, 2), (32, 2, 2), (32, 4, 3),
                  (32, 2, 3), (32, 2, 4)],
              3: [(32, 8, 1), (32, 4, 1)],
              4: [(32, 8, 1), (16, 4, 1), (32, 16, 1), (16, 8, 1), (32, 4, 1), (32, 2, 1), (16, 2, 1),
                  (32, 4, 2), (32, 2, 2), (32, 4, 3), (32, 2, 3)],
              8: [(32, 8, 1), (16, 4, 1), (16, 8, 1), (32, 4, 1), (32, 2, 1), (32, 4, 2)]}.get(M, [(32, 8, 1), (16, 4, 1)])
    for rows, py, tb in shapes:
        var = L.FD_VARIANT_STREAM if tb == 1 else L.FD_VARIANT_TBLOCK
        out.append(dict(variant=var, tile=(0, rows, py), tblock=tb))
        out.append(dict(variant=var, tile=(small_chunk, rows, py), tblock=tb))
    return out


# ---------------------------------------------------------------- oracle parity
def test_cfg1_2d_forward_matches_oracle():
    """128^2, so 4, 100 steps, v = 1500 m/s, dt at Courant 0.5, 10 Hz Ricker at the centre."""
    shape, so, nt, h, v0 = (128, 128), 4, 100, 10.0, 1500.0
    dt = 0.5 * h / v0
    v = torch.full(shape, v0, dtype=torch.float32)
    src = np.array([[64, 64]], dtype=np.int32)
    rec = np.array([[10, 64], [64, 10], [100, 100]], dtype=np.int32)
    amp = synth.ricker(nt, dt, 10.0)[:, None].copy()
    cs = dict(shape=shape, so=so, nt=nt, h=[h, h], v=v, dt=dt, src=src, rec=rec, amp=amp, sponge=0, vref=v0)
    ref = oracle_forward(cs)
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_STREAM)):
        out = gpu_forward(cs, **opt)
        e = rel_l2(out["u"].cpu().numpy(), ref["u"])
        print(f"cfg1 {opt} rel_l2(u) = {e:.3e}")
        assert e <= 1e-5
        assert rel_l2(out["rec"].cpu().numpy(), ref["rec"]) <= 1e-5


@pytest.mark.parametrize("shape,so,nt,sponge", [((64, 60, 72), 8, 160, 10), ((48, 40, 52), 16, 100, 8),
                                                ((50, 44, 66), 4, 200, 6), ((70, 90), 8, 150, 10),
                                                ((1000,), 4, 300, 30)])
def test_forward_matches_oracle(shape, so, nt, sponge):
    cs = make_case(shape, so, nt, sponge, nsrc=2, nrec=12)
    ref = oracle_forward(cs)
    out = gpu_forward(cs)
    eu = rel_l2(out["u"].cpu().numpy(), ref["u"])
    er = rel_l2(out["rec"].cpu().numpy(), ref["rec"])
    print(f"{shape} so{so} nt{nt}: rel_l2 u {eu:.3e} rec {er:.3e} cfg {api.last_config()}")
    assert eu <= 1e-5 and er <= 1e-5


def test_paper_gaussian_initial_field_matches_oracle():
    """The paper's functional check: Gaussian first time level, no source, atol 1e-5 (Sec. 6.5)."""
    shape, so, nt = (72, 72, 72), 8, 40
    cs = make_case(shape, so, nt, 0, nsrc=1, nrec=4)
    cs["src"] = np.zeros((0, 3), np.int32)
    cs["amp"] = np.zeros((nt, 0), np.float32)
    g = synth.gaussian_field(shape, 0.4)
    ref = oracle_forward(cs, u0=g.astype(np.float64), um1=g.astype(np.float64))
    gt = torch.from_numpy(g).to(DEV)
    for tb in (1, 2, 3):
        var = L.FD_VARIANT_STREAM if tb == 1 else L.FD_VARIANT_TBLOCK
        out = gpu_forward(cs, u0=gt, um1=gt, variant=var, tblock=tb,
                          tile=(0, 32, 4) if tb > 1 else (0, 0, 0))
        u = out["u"].cpu().numpy()
        assert np.allclose(u, ref["u"], atol=1e-5, rtol=0)
        assert rel_l2(u, ref["u"]) <= 1e-5


# ---------------------------------------------------------------- variants bit-exact
@pytest.mark.parametrize("shape,so", [((37, 45, 70), 8), ((21, 9, 130), 4), ((30, 33, 65), 2),
                                      ((40, 38, 80), 16), ((26, 77), 4), ((19, 23, 41), 6),
                                      ((25, 31, 44), 10)])
def test_all_configs_bit_identical_to_untiled(shape, so):
    nt = 13
    cs = make_case(shape, so, nt, sponge=3, nsrc=3, nrec=10, depth=shape[-1] // 2)
    # duplicate source, sources on the boundary, receivers on corners
    cs["src"] = np.concatenate([cs["src"], cs["src"][:1], np.zeros((1, len(shape)), np.int32)], 0)
    cs["amp"] = np.concatenate([cs["amp"], cs["amp"][:, :1] * 0.5, cs["amp"][:, :1] * -2.0], 1)
    corners = np.array([[n - 1 for n in shape], [0] * len(shape)], np.int32)
    cs["rec"] = np.concatenate([cs["rec"], corners, cs["src"][:2]], 0)
    rng = np.random.default_rng(5)
    u0 = torch.from_numpy(rng.standard_normal(shape).astype(np.float32) * 1e-3).to(DEV)
    um1 = torch.from_numpy(rng.standard_normal(shape).astype(np.float32) * 1e-3).to(DEV)
    base = gpu_forward(cs, u0=u0, um1=um1, variant=L.FD_VARIANT_NAIVE)
    cfgs = configs_for(so)
    assert len(cfgs) >= 3
    for opt in cfgs[1:]:
        out = gpu_forward(cs, u0=u0, um1=um1, **opt)
        ok = (torch.equal(out["u"], base["u"]) and torch.equal(out["u_prev"], base["u_prev"])
              and torch.equal(out["rec"], base["rec"]))
        assert ok, f"{opt} differs: max |du| {float((out['u'] - base['u']).abs().max())}"


@pytest.mark.parametrize("shape,so", [((3, 5, 7), 8), ((1, 40, 33), 4), ((70, 1, 1), 8), ((2, 130, 3), 16),
                                      ((5, 300), 16), ((9,), 16), ((1, 1, 1), 2)])
def test_degenerate_grids_match_oracle_and_variants_agree(shape, so):
    """Grids thinner than the stencil radius and unit extents: points outside
    the grid are zero, so every configuration still matches the oracle and the
    untiled kernel."""
    cs = make_case(shape, so, 17, 0, nrec=2)
    ref = oracle_forward(cs)
    base = gpu_forward(cs, variant=L.FD_VARIANT_NAIVE)
    err = rel_l2(base["u"].cpu().numpy(), ref["u"])
    assert err <= 1e-5, err
    assert rel_l2(base["rec"].cpu().numpy(), ref["rec"]) <= 1e-5
    opts = [dict()] + (configs_for(so, small_chunk=1)[1:] if len(shape) == 3 else [])
    for opt in opts:
        out = gpu_forward(cs, **opt)
        assert torch.equal(out["u"], base["u"]) and torch.equal(out["rec"], base["rec"]), opt


def test_full_size_cfg2_tiled_equals_untiled():
    """256^3, so 8, 500 steps, smoothed random v, 15 Hz Ricker at depth 20, 20-cell sponge."""
    import bench

    cs = bench.workload("cfg2", device=DEV)
    outs = []
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), bench.launch_options("cfg2")):
        out = api.forward(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], cs["rec"],
                          sponge=cs["sponge"], vref=cs["vref"], **opt)
        outs.append(out)
    assert torch.equal(outs[0]["u"], outs[1]["u"])
    assert torch.equal(outs[0]["rec"], outs[1]["rec"])
    assert float(outs[0]["u"].abs().max()) > 0


def test_full_size_cfg3_tiled_and_time_blocked_equal_untiled():
    """512^3, so 16, 1000 steps, 40-cell sponge: the benchmark's space-tiled and
    time-blocked launch configurations reproduce the untiled sweep bit for bit."""
    import bench

    cs = bench.workload("cfg3", device=DEV)
    outs = []
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), bench.launch_options("cfg3"),
                dict(variant=L.FD_VARIANT_STREAM, tile=(128, 16, 4)),
                dict(variant=L.FD_VARIANT_TBLOCK, tblock=2)):
        out = api.forward(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], None,
                          sponge=cs["sponge"], vref=cs["vref"], **opt)
        outs.append(out["u"])
        del out
    assert float(outs[0].abs().max()) > 0
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


# Space-tiled and time-blocked configurations at 512^3 that the autotuner has
# chosen on MI355X for the benchmark's time-blocking study, and earlier picks.
STUDY_CONFIGS = {
    2: [dict(variant=L.FD_VARIANT_STREAM, tile=(256, 32, 16)), dict(variant=L.FD_VARIANT_STREAM, tile=(256, 32, 4)),
        dict(variant=L.FD_VARIANT_TBLOCK, tblock=4, tile=(74, 32, 2)),
        dict(variant=L.FD_VARIANT_TBLOCK, tblock=4, tile=(128, 32, 2))],
    4: [dict(variant=L.FD_VARIANT_STREAM, tile=(512, 16, 4)), dict(variant=L.FD_VARIANT_STREAM, tile=(256, 32, 4)),
        dict(variant=L.FD_VARIANT_TBLOCK, tblock=3, tile=(256, 32, 2)),
        dict(variant=L.FD_VARIANT_TBLOCK, tblock=3, tile=(64, 32, 2))],
    8: [dict(variant=L.FD_VARIANT_STREAM, tile=(128, 32, 4)), dict(variant=L.FD_VARIANT_STREAM, tile=(512, 16, 2)),
        dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, tile=(64, 32, 2))],
}


@pytest.mark.parametrize("so", [2, 4, 8])
def test_full_size_time_blocking_study_configs_equal_untiled(so):
    """512^3 with the space orders of the benchmark's time-blocking study and
    the configurations its tuner picks (48 steps): every one equals the untiled
    kernel bit for bit."""
    import bench

    cs = bench.workload("cfg3", device=DEV)
    nt = 48
    dt = 0.8 * bench.courant_max(so, 3) * 10.0 / 4500.0
    amp = torch.from_numpy(synth.ricker(nt, dt, 15.0)[:, None].copy()).to(DEV)
    outs = []
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), *STUDY_CONFIGS[so]):
        out = api.forward(cs["v"], cs["h"], so, nt, dt, cs["src"], amp, None, sponge=cs["sponge"],
                          vref=cs["vref"], **opt)
        outs.append(out["u"])
        del out
    assert float(outs[0].abs().max()) > 0
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


def test_full_size_cfg3_sampled_points_match_oracle():
    """512^3 so 16 at the benchmark's launch configuration: a Gaussian initial
    state advanced 6 steps, single points checked against the oracle on their
    cube of dependence (radius 6 M)."""
    import bench

    cs = bench.workload("cfg3", device=DEV)
    nt, so, M = 6, cs["so"], cs["so"] // 2
    shape = tuple(cs["v"].shape)
    g = torch.from_numpy(synth.gaussian_field(shape, 0.3)).to(DEV)
    out = api.forward(cs["v"], cs["h"], so, nt, cs["dt"], None, None, None, u0=g, um1=g,
                      **bench.launch_options("cfg3"))
    u = out["u"].cpu().numpy()
    R = nt * M
    v = cs["v"].cpu().numpy()
    gh = g.cpu().numpy()
    for p in [(256, 256, 256), (0, 511, 0), (511, 3, 300), (100, 400, 511)]:
        sl = tuple(slice(max(0, c - R), min(n, c + R + 1)) for c, n in zip(p, shape))
        loc = tuple(c - s.start for c, s in zip(p, sl))
        prob = oracle.Problem(v[sl].astype(np.float64), cs["h"], so, nt, cs["dt"])
        ref = oracle.forward(prob, u0=gh[sl].astype(np.float64), um1=gh[sl].astype(np.float64))["u"]
        assert abs(u[p] - ref[loc]) <= 1e-5 * max(abs(ref[loc]), 1e-3 * np.abs(ref).max()), p


def test_full_size_cfg4_gradient_tiled_equals_untiled():
    """256^3 so 8, 1000 steps, 256 receivers, checkpoint every 50: the gradient in
    the benchmark's launch configuration equals the untiled one bit for bit."""
    import bench

    cs = bench.workload("cfg4", device=DEV)
    vtrue = synth.blob_velocity(cs["v"], amp=0.05, width_frac=1.0 / 16.0)
    d_obs = api.forward(vtrue, cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], cs["rec"],
                        sponge=cs["sponge"], vref=cs["vref"], **bench.launch_options("cfg4"))["rec"]
    res = []
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), bench.launch_options("cfg4")):
        J, g, _ = api.gradient(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], cs["rec"],
                               d_obs, sponge=cs["sponge"], vref=cs["vref"], ckpt_every=50, **opt)
        res.append((J, g))
    assert res[0][0] == res[1][0] and res[0][0] > 0
    assert torch.equal(res[0][1], res[1][1])
    assert float(res[0][1].abs().max()) > 0


def test_full_size_sampled_points_match_oracle():
    """256^3 so 8 at the benchmark's launch configuration: a Gaussian initial state
    advanced 12 steps; single points are checked against the oracle run on the
    cube of dependence (radius 12 M) around them, exact by the finite speed of the
    stencil."""
    import bench

    cs = bench.workload("cfg2", device=DEV)
    nt, so, M = 12, cs["so"], cs["so"] // 2
    shape = tuple(cs["v"].shape)
    g = torch.from_numpy(synth.gaussian_field(shape, 0.3)).to(DEV)
    rng = np.random.default_rng(0)
    wob = torch.from_numpy(rng.standard_normal(shape).astype(np.float32) * 1e-4).to(DEV)
    u0 = (g + wob).contiguous()
    out = api.forward(cs["v"], cs["h"], so, nt, cs["dt"], None, None, None, u0=u0, um1=g,
                      **bench.launch_options("cfg2"))
    u = out["u"].cpu().numpy()
    R = nt * M
    v = cs["v"].cpu().numpy()
    u0h, gh = u0.cpu().numpy(), g.cpu().numpy()
    pts = [(128, 128, 128), (0, 0, 0), (255, 17, 200), (60, 255, 3), (200, 100, 250), (5, 130, 60)]
    for p in pts:
        sl = tuple(slice(max(0, c - R), min(n, c + R + 1)) for c, n in zip(p, shape))
        loc = tuple(c - s.start for c, s in zip(p, sl))
        prob = oracle.Problem(v[sl].astype(np.float64), cs["h"], so, nt, cs["dt"])
        ref = oracle.forward(prob, u0=u0h[sl].astype(np.float64), um1=gh[sl].astype(np.float64))["u"]
        assert abs(u[p] - ref[loc]) <= 1e-5 * max(abs(ref[loc]), 1e-3 * np.abs(ref).max()), p


# ---------------------------------------------------------------- adjoint
def adjoint_case():
    cs = make_case((48, 44, 52), 8, 150, 8, nsrc=2, nrec=16)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((cs["nt"], len(cs["rec"]))).astype(np.float32)
    return cs, y


@pytest.mark.parametrize("opt", [dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_STREAM),
                                 dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, tile=(0, 32, 4))])
def test_adjoint_dot_product_fp32(opt):
    cs, y = adjoint_case()
    d = gpu_forward(cs, **opt)["rec"].cpu().numpy().astype(np.float64)
    fty = api.adjoint(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["rec"],
                      torch.from_numpy(y).to(DEV), sponge=cs["sponge"], vref=cs["vref"], **opt)["src"]
    lhs = float((d * y).sum())
    rhs = float((cs["amp"].astype(np.float64) * fty.cpu().numpy().astype(np.float64)).sum())
    print(f"dot test {opt}: {lhs:.9e} vs {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_adjoint_matches_oracle_and_variants_agree():
    cs, y = adjoint_case()
    prob = oracle.Problem(cs["v"].numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"],
                          cs["sponge"], cs["vref"], cs["src"], cs["rec"])
    ref = oracle.adjoint(prob, y.astype(np.float64))["src"]
    outs = []
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_STREAM, tile=(9, 0, 0)),
                dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, tile=(0, 32, 4))):
        o = api.adjoint(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["rec"],
                        torch.from_numpy(y).to(DEV), sponge=cs["sponge"], vref=cs["vref"], **opt)
        outs.append(o)
        e = rel_l2(o["src"].cpu().numpy(), ref)
        print(f"adjoint {opt} rel_l2 {e:.3e}")
        assert e <= 1e-5
    for o in outs[1:]:
        assert torch.equal(o["src"], outs[0]["src"]) and torch.equal(o["lam"], outs[0]["lam"])


# ---------------------------------------------------------------- gradient
def gradient_case():
    cs = make_case((40, 36, 44), 4, 120, 6, f0=25.0, nsrc=1, nrec=12)
    vtrue = synth.blob_velocity(cs["v"], amp=0.05, width_frac=1 / 8)
    ptrue = oracle.Problem(vtrue.numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"],
                           cs["sponge"], cs["vref"], cs["src"], cs["rec"])
    d_obs = oracle.forward(ptrue, amp=cs["amp"].astype(np.float64))["rec"].astype(np.float32)
    return cs, d_obs


# gradients are required to rel-L2 1e-5 of the FP64 oracle (measured 6.7e-6 here: FP32 wavefields, and
# the residual is a 5 % difference of two traces, which amplifies their rounding)
GRAD_TOL = 1e-5


def test_gradient_matches_oracle():
    cs, d_obs = gradient_case()
    prob = oracle.Problem(cs["v"].numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"],
                          cs["sponge"], cs["vref"], cs["src"], cs["rec"])
    Jref, gref, _ = oracle.gradient(prob, cs["amp"].astype(np.float64), d_obs.astype(np.float64))
    J, gv, res = api.gradient(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
                              torch.from_numpy(cs["amp"]).to(DEV), cs["rec"], torch.from_numpy(d_obs).to(DEV),
                              sponge=cs["sponge"], vref=cs["vref"], ckpt_every=16)
    eg = rel_l2(gv.cpu().numpy(), gref)
    print(f"gradient: J {J:.9e} vs {Jref:.9e}; rel_l2(grad) {eg:.3e}")
    assert abs(J - Jref) <= 1e-4 * Jref
    assert eg <= GRAD_TOL


def test_gradient_identical_across_variants_and_checkpoint_intervals():
    cs, d_obs = gradient_case()
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
            torch.from_numpy(cs["amp"]).to(DEV), cs["rec"], torch.from_numpy(d_obs).to(DEV))
    kw = dict(sponge=cs["sponge"], vref=cs["vref"])
    J0, g0, _ = api.gradient(*args, variant=L.FD_VARIANT_NAIVE, ckpt_every=cs["nt"], **kw)
    for opt in (dict(variant=L.FD_VARIANT_NAIVE, ckpt_every=7),
                dict(variant=L.FD_VARIANT_STREAM, ckpt_every=16),
                dict(variant=L.FD_VARIANT_STREAM, ckpt_every=1),
                dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, ckpt_every=25),
                dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, ckpt_every=50, tile=(5, 0, 0))):
        J, g, _ = api.gradient(*args, **opt, **kw)
        assert J == J0
        assert torch.equal(g, g0), f"{opt}: max diff {float((g - g0).abs().max())}"


def test_vjp_equals_gradient_with_residual_cotangent():
    cs, d_obs = gradient_case()
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
            torch.from_numpy(cs["amp"]).to(DEV), cs["rec"])
    J, g, res = api.gradient(*args, torch.from_numpy(d_obs).to(DEV), sponge=cs["sponge"], vref=cs["vref"])
    g2 = api.vjp(*args, res, sponge=cs["sponge"], vref=cs["vref"])
    assert torch.equal(g, g2)


# ---------------------------------------------------------------- state, resume and errors
@pytest.mark.parametrize("opt", [dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_STREAM),
                                 dict(variant=L.FD_VARIANT_TBLOCK, tblock=3, tile=(0, 32, 4))])
def test_resume_is_bit_exact(opt):
    cs = make_case((40, 42, 66), 4, 60, 5, nsrc=2, nrec=6)
    full = gpu_forward(cs, **opt)
    a = dict(cs, nt=30, amp=np.ascontiguousarray(cs["amp"][:30]))
    b = dict(cs, nt=30, amp=np.ascontiguousarray(cs["amp"][30:]))
    first = gpu_forward(a, **opt)
    second = gpu_forward(b, u0=first["u"], um1=first["u_prev"], **opt)
    assert torch.equal(second["u"], full["u"]) and torch.equal(second["u_prev"], full["u_prev"])
    assert torch.equal(torch.cat([first["rec"], second["rec"]]), full["rec"])


def test_zero_steps_returns_initial_state():
    cs = make_case((20, 20, 20), 4, 0, 0, nsrc=1, nrec=2)
    u0 = torch.randn(20, 20, 20, device=DEV)
    out = gpu_forward(cs, u0=u0, um1=2 * u0)
    assert torch.equal(out["u"], u0) and torch.equal(out["u_prev"], 2 * u0)


def test_cfl_violation_and_bad_velocity_are_reported():
    cs = make_case((24, 24, 24), 8, 5, 0)
    with pytest.raises(L.FdError) as e:
        api.forward(cs["v"].to(DEV), cs["h"], 8, 5, cs["dt"] * 1.3, cs["src"],
                    torch.from_numpy(cs["amp"]).to(DEV), cs["rec"])
    assert e.value.code == L.FD_ECFL
    vb = cs["v"].clone()
    vb[3, 4, 5] = float("nan")
    with pytest.raises(L.FdError) as e:
        api.forward(vb.to(DEV), cs["h"], 8, 5, cs["dt"], None, None, None)
    assert e.value.code == L.FD_ENONFINITE
    vb = cs["v"].clone()
    vb[0, 0, 0] = -1.0
    with pytest.raises(L.FdError) as e:
        api.forward(vb.to(DEV), cs["h"], 8, 5, cs["dt"], None, None, None)
    assert e.value.code == L.FD_ENONFINITE
    # the check can be skipped explicitly
    api.forward(cs["v"].to(DEV), cs["h"], 8, 5, cs["dt"], None, None, None, flags=L.FD_FLAG_NO_CFL_CHECK)


def test_check_finite_flag_detects_blow_up():
    cs = make_case((24, 24, 24), 8, 300, 0, nrec=4)
    big_dt = cs["dt"] * 1.6
    amp = torch.from_numpy(synth.ricker(300, big_dt, 15.0)[:, None].copy()).to(DEV)
    with pytest.raises(L.FdError) as e:
        api.forward(cs["v"].to(DEV), cs["h"], 8, 300, big_dt, cs["src"], amp, cs["rec"],
                    flags=L.FD_FLAG_NO_CFL_CHECK | L.FD_FLAG_CHECK_FINITE)
    assert e.value.code == L.FD_ENONFINITE


@pytest.mark.parametrize("so", [4, 8])
def test_anisotropic_spacing_matches_oracle_and_variants_agree(so):
    """Unequal spacings select the per-axis Laplacian form in every kernel."""
    shape, nt = (40, 36, 70), 60
    cs = make_case(shape, so, nt, 5, nsrc=2, nrec=8)
    cs["h"] = [10.0, 12.5, 8.0]
    cs["dt"] = stable_dt(float(cs["v"].max()), cs["h"], so, 3)
    cs["amp"] = np.ascontiguousarray(np.stack([synth.ricker(nt, cs["dt"], 25.0)] * 2, 1))
    ref = oracle_forward(cs)
    base = gpu_forward(cs, variant=L.FD_VARIANT_NAIVE)
    assert rel_l2(base["u"].cpu().numpy(), ref["u"]) <= 1e-5
    for opt in (dict(variant=L.FD_VARIANT_STREAM), dict(variant=L.FD_VARIANT_STREAM, tile=(9, 32, 8)),
                dict(variant=L.FD_VARIANT_TBLOCK, tblock=2), dict(variant=L.FD_VARIANT_TBLOCK, tblock=2,
                                                                  tile=(0, 32, 4))):
        out = gpu_forward(cs, **opt)
        assert torch.equal(out["u"], base["u"]) and torch.equal(out["rec"], base["rec"]), opt


@pytest.mark.parametrize("opt", [dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_STREAM),
                                 dict(variant=L.FD_VARIANT_TBLOCK, tblock=2)])
def test_full_storage_gradient_equals_checkpointed(opt):
    """ckpt_every >= nt stores the whole time axis (no recomputation): same J,
    gradient and residual bit for bit, and the same vector-Jacobian product."""
    cs, d_obs = gradient_case()
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
            torch.from_numpy(cs["amp"]).to(DEV), cs["rec"])
    kw = dict(sponge=cs["sponge"], vref=cs["vref"], **opt)
    Jf, gf, rf = api.gradient(*args, torch.from_numpy(d_obs).to(DEV), ckpt_every=cs["nt"] + 5, **kw)
    Jc, gc, rc = api.gradient(*args, torch.from_numpy(d_obs).to(DEV), ckpt_every=13, **kw)
    assert Jf == Jc and torch.equal(gf, gc) and torch.equal(rf, rc)
    assert torch.equal(api.vjp(*args, rc, ckpt_every=cs["nt"], **kw), api.vjp(*args, rc, ckpt_every=13, **kw))


def test_auto_storage_follows_the_budget():
    """ckpt_every="auto": a budget that holds the whole time axis stores it, a
    smaller one checkpoints at the interval fd_gradient_storage reports; both
    give the fixed-interval results bit for bit."""
    cs, d_obs = gradient_case()
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
            torch.from_numpy(cs["amp"]).to(DEV), cs["rec"])
    kw = dict(sponge=cs["sponge"], vref=cs["vref"], variant=L.FD_VARIANT_STREAM)
    d = torch.from_numpy(d_obs).to(DEV)
    J0, g0, r0 = api.gradient(*args, d, ckpt_every=cs["nt"], **kw)
    grid = L.make_grid(cs["shape"], cs["h"], cs["so"], cs["sponge"], cs["vref"])
    tm = L.make_time(cs["nt"], cs["dt"])
    rec = L.Points(cs["rec"], None, len(cs["shape"]))
    full = L.fd_workspace_size(C.byref(grid), C.byref(tm), None, C.byref(rec.s),
                               C.byref(L.make_options(ckpt_every=cs["nt"])), L.FD_OP_GRADIENT)
    for budget in (None, full, full - 1):
        J, g, r = api.gradient(*args, d, ckpt_every="auto", mem_budget=budget, **kw)
        assert J == J0 and torch.equal(g, g0) and torch.equal(r, r0), budget
    with pytest.raises(L.FdError):
        api.gradient(*args, d, ckpt_every="auto", mem_budget=4096, **kw)
    assert torch.equal(api.vjp(*args, r0, ckpt_every="auto", **kw), api.vjp(*args, r0, ckpt_every=13, **kw))
