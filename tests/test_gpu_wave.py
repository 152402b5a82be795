"""Two-level passes without redundant halos (FD_VARIANT_WAVE): each workgroup
computes both levels on its own (y, z) tile of the whole x axis and reads
level 1 on the ring around its tile from its neighbours, once their progress
counters show it stored.  Every case must equal the untiled kernel bit for bit
(the exchange must deliver exactly the neighbours' values, and the counters
must order every read after the write it needs); one case is also compared
with the FP64 oracle, and the full 512^3 so-8 grid with the space-tiled
kernel."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api
from tests.test_gpu_parity import make_case, rel_l2, stable_dt

pytestmark = pytest.mark.gpu
DEV = "cuda"


def run(cs, rec=None, src=None, **opts):
    return api.forward(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"],
                       cs["src"] if src is None else src, torch.from_numpy(cs["amp"]).to(DEV), rec,
                       sponge=cs["sponge"], vref=cs["vref"], **opts)


@pytest.mark.parametrize("so,shape,tile", [
    (2, (46, 41, 70), (0, 0, 0)),
    (4, (61, 83, 150), (0, 0, 0)),     # 3 x 6 tiles, ragged in y and z
    (8, (50, 70, 130), (0, 16, 4)),
    (8, (50, 70, 130), (0, 16, 2)),
    (8, (40, 38, 44), (0, 8, 2)),      # one column of tiles, ragged rows
    (8, (35, 50, 200), (0, 8, 2)),
    (4, (45, 66, 129), (0, 16, 4)),
    (6, (33, 45, 77), (0, 0, 0)),
    (12, (41, 50, 90), (0, 0, 0)),
    (16, (52, 36, 140), (0, 0, 0)),
    (2, (3, 40, 70), (0, 0, 0)),       # x extents shorter than the level lag
    (4, (7, 33, 100), (0, 16, 2)),
    (8, (9, 20, 64), (0, 8, 2)),
])
def test_wave_equals_untiled(so, shape, tile):
    print(f"wave so {so} shape {shape} tile {tile}", flush=True)
    # an odd step count: the last pass is single-level; the sponge fits every axis
    cs = make_case(shape, so, 31, min(5, min(shape) // 2))
    base = run(cs, rec=cs["rec"], variant=L.FD_VARIANT_NAIVE)
    out = run(cs, rec=cs["rec"], variant=L.FD_VARIANT_WAVE, tile=tile)
    cfg = api.last_config()
    assert cfg["variant"] == L.FD_VARIANT_WAVE and cfg["tblock"] == 2, cfg
    assert float(base["u"].abs().max()) > 0 and float(base["rec"].abs().max()) > 0
    assert torch.equal(out["u"], base["u"]) and torch.equal(out["u_prev"], base["u_prev"])
    assert torch.equal(out["rec"], base["rec"])


def test_wave_anisotropic_and_points_between_nodes():
    cs = make_case((44, 58, 100), 8, 26, 6, nsrc=5, nrec=12)
    cs["h"] = [10.0, 12.5, 10.0]
    cs["dt"] = stable_dt(float(cs["v"].max()), cs["h"], 8, 3)
    src = synth.offgrid_points(cs["shape"], 5, seed=301, margin=0.0)
    rec = synth.offgrid_points(cs["shape"], 12, seed=302, margin=0.0)
    base = run(cs, rec=rec, src=src, variant=L.FD_VARIANT_NAIVE)
    out = run(cs, rec=rec, src=src, variant=L.FD_VARIANT_WAVE)
    assert api.last_config()["variant"] == L.FD_VARIANT_WAVE
    assert torch.equal(out["u"], base["u"]) and torch.equal(out["u_prev"], base["u_prev"])
    assert torch.equal(out["rec"], base["rec"])


def test_wave_matches_oracle():
    cs = make_case((40, 52, 90), 8, 36, 5, nsrc=3, nrec=10)
    out = run(cs, rec=cs["rec"], variant=L.FD_VARIANT_WAVE)
    assert api.last_config()["variant"] == L.FD_VARIANT_WAVE
    prob = oracle.Problem(cs["v"].numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["sponge"],
                          cs["vref"], cs["src"], cs["rec"])
    ref = oracle.forward(prob, amp=cs["amp"].astype(np.float64))
    assert rel_l2(out["u"].cpu().numpy(), ref["u"]) <= 1e-5
    assert rel_l2(out["rec"].cpu().numpy(), ref["rec"]) <= 1e-5


def test_wave_adjoint_equals_untiled():
    cs = make_case((46, 60, 110), 8, 27, 5, nrec=16)
    y = torch.from_numpy(np.random.default_rng(7).standard_normal((cs["nt"], len(cs["rec"]))).astype(np.float32))
    args = (cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["rec"], y.to(DEV))
    base = api.adjoint(*args, sponge=cs["sponge"], vref=cs["vref"], variant=L.FD_VARIANT_NAIVE)
    out = api.adjoint(*args, sponge=cs["sponge"], vref=cs["vref"], variant=L.FD_VARIANT_WAVE)
    assert api.last_config()["variant"] == L.FD_VARIANT_WAVE
    assert float(base["src"].abs().max()) > 0
    assert torch.equal(out["src"], base["src"]) and torch.equal(out["lam"], base["lam"])


def test_wave_gradient_equals_space_tiled():
    """A gradient under an exchange plan: its checkpointing forward segments run
    exchange passes, the recomputation and imaging passes the other kernels;
    the checkpoints, hence the gradient, are the same bits as under the
    space-tiled plan."""
    cs = make_case((40, 52, 90), 8, 33, 5, nrec=12)
    v = cs["v"].to(DEV)
    amp = torch.from_numpy(cs["amp"]).to(DEV)
    d_obs = 1e-3 * torch.from_numpy(np.random.default_rng(3).standard_normal((cs["nt"], len(cs["rec"]))).astype(np.float32)).to(DEV)
    args = (v, cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], amp, cs["rec"], d_obs)
    ja, ga, ra = api.gradient(*args, sponge=cs["sponge"], vref=cs["vref"], variant=L.FD_VARIANT_WAVE, ckpt_every=7)
    jb, gb, rb = api.gradient(*args, sponge=cs["sponge"], vref=cs["vref"], variant=L.FD_VARIANT_STREAM, ckpt_every=7)
    assert float(gb.abs().max()) > 0
    assert ja == jb and torch.equal(ga, gb) and torch.equal(ra, rb)


def test_wave_plan_needs_every_tile_resident():
    """A grid with more tiles than the device holds at once is refused."""
    v = torch.full((8, 2048, 4096), 2000.0, device=DEV)  # 64 x 128 tiles of 64 x 16
    with pytest.raises(L.FdError) as e:
        api.forward(v, [10.0] * 3, 8, 2, 1e-4, variant=L.FD_VARIANT_WAVE)
    assert e.value.code == L.FD_EUNSUPPORTED


@pytest.mark.parametrize("so", [4, 8, 16])
def test_wave_full_size_equals_untiled(so):
    """512^3 (the time-blocking study's grid and the headline's), 48 steps:
    256 tiles of 64 x 16 (512 of 64 x 8), every one resident, in each compiled
    tile shape."""
    import bench

    print(f"wave 512^3 so {so}", flush=True)
    cs = bench.workload("cfg3", device=DEV)
    nt = 48
    dt = 0.8 * bench.courant_max(so, 3) * 10.0 / 4500.0
    amp = torch.from_numpy(synth.ricker(nt, dt, 15.0)[:, None].copy()).to(DEV)
    outs = []
    shapes = {4: [(0, 16, 4)], 8: [(0, 16, 4), (0, 8, 2)], 16: []}[so]
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_WAVE),
                *(dict(variant=L.FD_VARIANT_WAVE, tile=t) for t in shapes)):
        out = api.forward(cs["v"], cs["h"], so, nt, dt, cs["src"], amp, None, sponge=cs["sponge"],
                          vref=cs["vref"], **opt)
        if opt["variant"] == L.FD_VARIANT_WAVE:
            assert api.last_config()["variant"] == L.FD_VARIANT_WAVE
        outs.append(out["u"])
        del out
    assert float(outs[0].abs().max()) > 0
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


@pytest.mark.parametrize("so,tile", [(8, (0, 16, 2)), (8, (0, 8, 2)), (4, (0, 16, 2))])
def test_wave_long_sweep_equals_space_tiled(so, tile):
    """1000 steps at 512^3 (500 exchange passes, each with every workgroup
    publishing and polling counters some 500 times): any read of a neighbour's
    level 1 before it was stored would change bits somewhere in the field."""
    import bench

    print(f"wave 512^3 so {so} tile {tile}, 1000 steps", flush=True)
    cs = bench.workload("cfg3", device=DEV)
    nt = 1000
    dt = 0.8 * bench.courant_max(so, 3) * 10.0 / 4500.0
    amp = torch.from_numpy(synth.ricker(nt, dt, 15.0)[:, None].copy()).to(DEV)
    a = api.forward(cs["v"], cs["h"], so, nt, dt, cs["src"], amp, None, sponge=cs["sponge"], vref=cs["vref"],
                    variant=L.FD_VARIANT_WAVE, tile=tile)
    assert api.last_config()["variant"] == L.FD_VARIANT_WAVE
    b = api.forward(cs["v"], cs["h"], so, nt, dt, cs["src"], amp, None, sponge=cs["sponge"], vref=cs["vref"],
                    variant=L.FD_VARIANT_STREAM)
    assert float(b["u"].abs().max()) > 0
    assert torch.equal(a["u"], b["u"]) and torch.equal(a["u_prev"], b["u_prev"])
