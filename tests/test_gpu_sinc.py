"""Sources and receivers with Kaiser-windowed sinc interpolation (half-width r,
(2r)^ndim nodes per point) on the GPU: forward, adjoint, gradient and Born
against the FP64 oracle (rel-L2 1e-5), every kernel configuration bit-identical
to the untiled one, nodes on the grid bit-identical to grid indices, and the
FP32 dot test.  Half-width 8 (4096 nodes per point) exceeds what a tile stages
in LDS and takes the direct walk."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api
from tests.test_gpu_offgrid import CONFIGS, offgrid_case
from tests.test_gpu_parity import GRAD_TOL, make_case, rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda"


def problem(cs, r, v=None):
    vv = cs["v"] if v is None else v
    return oracle.Problem(vv.numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["sponge"],
                          cs["vref"], cs["src"], cs["rec"], src_sinc=r, rec_sinc=r)


def gpu_fwd(cs, r, **opts):
    return api.forward(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], api.Sinc(cs["src"], r),
                       torch.from_numpy(cs["amp"]).to(DEV), api.Sinc(cs["rec"], r), sponge=cs["sponge"],
                       vref=cs["vref"], **opts)


@pytest.mark.parametrize("so,r", [(8, 4), (8, 2), (4, 3)])
def test_sinc_forward_matches_oracle_and_configs_agree(so, r):
    cs = offgrid_case(so=so, nt=70)
    print(f"case so{so} r{r} shape {cs['shape']}", flush=True)
    ref = oracle.forward(problem(cs, r), amp=cs["amp"].astype(np.float64))
    outs = [gpu_fwd(cs, r, **o) for o in CONFIGS]
    for o, out in zip(CONFIGS, outs):
        er = rel_l2(out["rec"].cpu().numpy(), ref["rec"])
        eu = rel_l2(out["u"].cpu().numpy(), ref["u"])
        print(f"so{so} r{r} {o}: traces {er:.2e} field {eu:.2e}")
        assert er <= 1e-5 and eu <= 1e-5
    for out in outs[1:]:
        assert torch.equal(out["rec"], outs[0]["rec"])
        assert torch.equal(out["u"], outs[0]["u"])


def test_sinc_2d_and_widest_window_match_oracle():
    cs = offgrid_case(shape=(120, 96), so=4, nt=100, nsrc=1, nrec=9)
    ref = oracle.forward(problem(cs, 4), amp=cs["amp"].astype(np.float64))
    out = gpu_fwd(cs, 4)
    assert rel_l2(out["rec"].cpu().numpy(), ref["rec"]) <= 1e-5
    assert rel_l2(out["u"].cpu().numpy(), ref["u"]) <= 1e-5
    # r = 8: 4096 nodes per point, more than a tile stages
    cs = offgrid_case(shape=(40, 38, 72), so=8, nt=60, nsrc=1, nrec=5)
    near = cs["src"][0] + np.array([[1.3, 0.7, 2.1], [-2.2, 1.1, 0.4], [0.5, -3.3, -1.7]])
    cs["rec"] = np.concatenate([near, cs["rec"][-3:]], 0)
    ref = oracle.forward(problem(cs, 8), amp=cs["amp"].astype(np.float64))
    outs = [gpu_fwd(cs, 8, **o) for o in CONFIGS[:3]]
    er = rel_l2(outs[0]["rec"].cpu().numpy(), ref["rec"])
    eu = rel_l2(outs[0]["u"].cpu().numpy(), ref["u"])
    print(f"r8: traces {er:.2e} field {eu:.2e}")
    assert er <= 1e-5 and eu <= 1e-5
    for out in outs[1:]:
        assert torch.equal(out["rec"], outs[0]["rec"]) and torch.equal(out["u"], outs[0]["u"])


def test_sinc_on_grid_nodes_equals_grid_indices_bitwise():
    cs = make_case((40, 42, 66), 8, 50, 5, nsrc=2, nrec=6)
    pos = dict(cs, src=cs["src"].astype(np.float64), rec=cs["rec"].astype(np.float64))
    for o in CONFIGS[:2]:
        a = api.forward(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
                        torch.from_numpy(cs["amp"]).to(DEV), cs["rec"], sponge=cs["sponge"], vref=cs["vref"], **o)
        b = gpu_fwd(pos, 4, **o)
        assert torch.equal(a["rec"], b["rec"]) and torch.equal(a["u"], b["u"])


def test_sinc_adjoint_matches_oracle_and_dot_test():
    r = 4
    cs = offgrid_case(nt=70)
    y = np.random.default_rng(19).standard_normal((cs["nt"], len(cs["rec"]))).astype(np.float32)
    ref = oracle.adjoint(problem(cs, r), y.astype(np.float64))["src"]
    outs = []
    for o in CONFIGS:
        fty = api.adjoint(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], api.Sinc(cs["src"], r),
                          api.Sinc(cs["rec"], r), torch.from_numpy(y).to(DEV), sponge=cs["sponge"],
                          vref=cs["vref"], **o)["src"]
        e = rel_l2(fty.cpu().numpy(), ref)
        print(f"sinc adjoint {o}: {e:.2e}")
        assert e <= 1e-5
        outs.append(fty)
    for f in outs[1:]:
        assert torch.equal(f, outs[0])
    d = gpu_fwd(cs, r)["rec"].cpu().numpy().astype(np.float64)
    lhs = float((d * y).sum())
    rhs = float((cs["amp"].astype(np.float64) * outs[0].cpu().numpy().astype(np.float64)).sum())
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_sinc_gradient_and_born_match_oracle():
    r = 4
    cs = make_case((40, 36, 44), 4, 100, 6, f0=25.0, nsrc=1, nrec=12)
    cs["src"] = np.array([[19.4, 17.7, 14.35]])
    cs["rec"] = synth.offgrid_receiver_line(cs["shape"], 12, depth=14.6)
    vtrue = synth.blob_velocity(cs["v"], amp=0.05, width_frac=1 / 8)
    d_obs = oracle.forward(problem(cs, r, vtrue), amp=cs["amp"].astype(np.float64))["rec"].astype(np.float32)
    Jref, gref, _ = oracle.gradient(problem(cs, r), cs["amp"].astype(np.float64), d_obs.astype(np.float64))
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], api.Sinc(cs["src"], r),
            torch.from_numpy(cs["amp"]).to(DEV), api.Sinc(cs["rec"], r), torch.from_numpy(d_obs).to(DEV))
    kw = dict(sponge=cs["sponge"], vref=cs["vref"])
    J0, g0, _ = api.gradient(*args, variant=L.FD_VARIANT_NAIVE, ckpt_every=16, **kw)
    eg = rel_l2(g0.cpu().numpy(), gref)
    print(f"sinc gradient: J {J0:.9e} vs {Jref:.9e}; rel_l2 {eg:.2e}")
    assert abs(J0 - Jref) <= 1e-4 * Jref
    assert eg <= GRAD_TOL
    for o in (dict(variant=L.FD_VARIANT_STREAM, ckpt_every=16), dict(variant=L.FD_VARIANT_STREAM, ckpt_every=100),
              dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, ckpt_every=25)):
        J, g, _ = api.gradient(*args, **o, **kw)
        assert J == J0 and torch.equal(g, g0), o
    dv = (vtrue - cs["v"]).contiguous()
    ref = oracle.born(problem(cs, r), cs["amp"].astype(np.float64), dv.numpy().astype(np.float64))
    outs = [api.born(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], api.Sinc(cs["src"], r),
                     torch.from_numpy(cs["amp"]).to(DEV), api.Sinc(cs["rec"], r), dv.to(DEV), **kw, **o)
            for o in CONFIGS[:2]]
    e = rel_l2(outs[0].cpu().numpy(), ref)
    print(f"sinc born: {e:.2e}")
    assert e <= 1e-5 and torch.equal(outs[0], outs[1])


def test_sinc_batch_equals_single_shots():
    """Batched shots whose windowed-sinc tables are too large to stage (they take
    the separate recording and untiled injection routes) next to shots whose
    tables stage: forward traces and gradients equal single calls bit for bit."""
    shots = []
    for i, (shape, so, nt, r, nrec) in enumerate([((40, 38, 44), 4, 30, 4, 9), ((36, 44, 52), 8, 25, 2, 4),
                                                   ((48, 40, 46), 16, 20, 8, 3)]):
        v = synth.smooth_velocity(shape, seed=500 + i, sigma=3.0).to(DEV)
        dt = 0.8 * 2.0 / (float(v.max()) * np.sqrt(3 * 7.5)) * 10.0
        amp = torch.from_numpy(synth.ricker(nt, dt, 30.0)[:, None].copy()).to(DEV)
        src = api.Sinc(synth.offgrid_points(shape, 1, seed=50 + i, margin=2.0), r)
        rec = api.Sinc(synth.offgrid_receiver_line(shape, nrec, depth=12.4), r)
        shots.append(dict(v=v, h=[10.0] * 3, so=so, nt=nt, dt=dt, src_idx=src, src_amp=amp, rec_idx=rec,
                          sponge=4, vref=4500.0, options={}))
    outs = api.forward_batch(shots, graph=True)
    for sh, o in zip(shots, outs):
        ref = api.forward(sh["v"], sh["h"], sh["so"], sh["nt"], sh["dt"], sh["src_idx"], sh["src_amp"], sh["rec_idx"],
                          sponge=4, vref=4500.0)["rec"]
        assert float(ref.abs().max()) > 0.0
        assert torch.equal(o, ref)
    for sh in shots:
        sh["d_obs"] = api.forward(sh["v"] * 1.02, sh["h"], sh["so"], sh["nt"], sh["dt"], sh["src_idx"],
                                  sh["src_amp"], sh["rec_idx"], sponge=4, vref=4500.0)["rec"]
        sh["options"] = dict(ckpt_every=9)
    misfits, grads = api.gradient_batch(shots, graph=True)
    for sh, J, g in zip(shots, misfits, grads):
        Jr, gr, _ = api.gradient(sh["v"], sh["h"], sh["so"], sh["nt"], sh["dt"], sh["src_idx"], sh["src_amp"],
                                 sh["rec_idx"], sh["d_obs"], sponge=4, vref=4500.0, ckpt_every=9)
        assert J == Jr and torch.equal(g, gr)


def test_sinc_1d_matches_oracle():
    cs = offgrid_case(shape=(1000,), so=4, nt=200, nsrc=2, nrec=9, sponge=30)
    near = cs["src"][0, 0] + np.array([3.3, -5.7, 20.1, 41.25])
    cs["rec"] = np.concatenate([near[:, None], cs["rec"][-3:]], 0)
    for r in (1, 8):
        ref = oracle.forward(problem(cs, r), amp=cs["amp"].astype(np.float64))
        outs = [gpu_fwd(cs, r, **o) for o in CONFIGS[:2]]
        assert rel_l2(outs[0]["rec"].cpu().numpy(), ref["rec"]) <= 1e-5
        assert rel_l2(outs[0]["u"].cpu().numpy(), ref["u"]) <= 1e-5
        assert torch.equal(outs[0]["rec"], outs[1]["rec"]) and torch.equal(outs[0]["u"], outs[1]["u"])


def test_full_size_sinc_headline_tiled_equals_untiled():
    """256^3 so 8, 500 steps, a windowed-sinc source and 256 windowed-sinc
    receivers (r = 4, 512 nodes each), in the launch configuration the
    benchmark times: the tiled sweep (receivers recorded after each pass)
    equals the untiled one bit for bit."""
    import bench

    cs = bench.offgrid(dict(bench.workload("cfg2", device=DEV), rec=synth.receiver_line((256,) * 3, 256, depth=20)))
    src, rec = api.Sinc(cs["src"], 4), api.Sinc(cs["rec"], 4)
    outs = [api.forward(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], src, cs["amp"], rec, sponge=cs["sponge"],
                        vref=cs["vref"], **opt)
            for opt in (dict(variant=L.FD_VARIANT_NAIVE), bench.launch_options("cfg2"))]
    assert torch.equal(outs[0]["rec"], outs[1]["rec"])
    assert torch.equal(outs[0]["u"], outs[1]["u"])
    assert float(outs[1]["rec"].abs().max()) > 0


def test_sinc_heavy_source_gradient_routes_equal_untiled():
    """A 4096-node source (r = 8) is injected after the tiled pass in every
    mode the gradient uses (plain checkpoint sweep, second-difference
    recomputation, and with the receivers' tables the imaging adjoint): the
    gradient equals the untiled one bit for bit, checkpointed and with the
    whole time axis stored, and matches the oracle."""
    cs = make_case((40, 36, 44), 4, 60, 6, f0=25.0, nsrc=1, nrec=12)
    cs["src"] = np.array([[19.4, 17.7, 14.35]])
    cs["rec"] = synth.offgrid_receiver_line(cs["shape"], 12, depth=14.6)
    rs, rr = 8, 2
    prob = lambda v: oracle.Problem(v.numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"],
                                    cs["sponge"], cs["vref"], cs["src"], cs["rec"], src_sinc=rs, rec_sinc=rr)
    vtrue = synth.blob_velocity(cs["v"], amp=0.05, width_frac=1 / 8)
    d_obs = oracle.forward(prob(vtrue), amp=cs["amp"].astype(np.float64))["rec"].astype(np.float32)
    Jref, gref, _ = oracle.gradient(prob(cs["v"]), cs["amp"].astype(np.float64), d_obs.astype(np.float64))
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], api.Sinc(cs["src"], rs),
            torch.from_numpy(cs["amp"]).to(DEV), api.Sinc(cs["rec"], rr), torch.from_numpy(d_obs).to(DEV))
    kw = dict(sponge=cs["sponge"], vref=cs["vref"])
    J0, g0, r0 = api.gradient(*args, variant=L.FD_VARIANT_NAIVE, ckpt_every=16, **kw)
    eg = rel_l2(g0.cpu().numpy(), gref)
    print(f"heavy-source gradient: J {J0:.9e} vs {Jref:.9e}; rel_l2 {eg:.2e}")
    assert abs(J0 - Jref) <= 1e-4 * Jref and eg <= GRAD_TOL
    for o in (dict(variant=L.FD_VARIANT_STREAM, ckpt_every=16), dict(variant=L.FD_VARIANT_STREAM, ckpt_every=60),
              dict(variant=L.FD_VARIANT_TBLOCK, tblock=2, ckpt_every=25)):
        J, g, r = api.gradient(*args, **o, **kw)
        assert J == J0 and torch.equal(g, g0) and torch.equal(r, r0), o


def test_sinc_anisotropic_spacing_forward_and_adjoint_match_oracle():
    """Unequal spacing per axis (10, 12, 9 m; the anisotropic Laplacian form):
    windowed-sinc forward traces and adjoint samples against the oracle, every
    configuration bit-identical to the untiled one."""
    from tests.test_gpu_parity import stable_dt

    r = 3
    cs = offgrid_case(shape=(44, 38, 50), so=8, nt=60)
    cs["h"] = [10.0, 12.0, 9.0]
    cs["dt"] = stable_dt(float(cs["v"].max()), cs["h"], 8, 3)
    cs["amp"] = np.ascontiguousarray(synth.ricker(cs["nt"], cs["dt"], 25.0)[:, None].repeat(len(cs["src"]), 1))
    ref = oracle.forward(problem(cs, r), amp=cs["amp"].astype(np.float64))
    outs = [gpu_fwd(cs, r, **o) for o in CONFIGS]
    assert rel_l2(outs[0]["rec"].cpu().numpy(), ref["rec"]) <= 1e-5
    assert rel_l2(outs[0]["u"].cpu().numpy(), ref["u"]) <= 1e-5
    for out in outs[1:]:
        assert torch.equal(out["rec"], outs[0]["rec"]) and torch.equal(out["u"], outs[0]["u"])
    y = np.random.default_rng(29).standard_normal((cs["nt"], len(cs["rec"]))).astype(np.float32)
    aref = oracle.adjoint(problem(cs, r), y.astype(np.float64))["src"]
    adj = [api.adjoint(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], api.Sinc(cs["src"], r),
                       api.Sinc(cs["rec"], r), torch.from_numpy(y).to(DEV), sponge=cs["sponge"], vref=cs["vref"],
                       **o)["src"] for o in CONFIGS]
    assert rel_l2(adj[0].cpu().numpy(), aref) <= 1e-5
    for f in adj[1:]:
        assert torch.equal(f, adj[0])
