"""Split (Pochoir-style trapezoid) tiles along the streamed axis, the
FD_VARIANT_SPLIT form of two-level passes: chunks compute upright trapezoids
on disjoint planes and a second, single-level phase fills the inverted
trapezoids around the chunk ends.  Every case equals the untiled kernel bit for
bit and the oracle within 1e-5; passes with receivers keep the overlapped
chunks."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api
from tests.test_gpu_parity import make_case, rel_l2

pytestmark = pytest.mark.gpu
DEV = "cuda"


def run(cs, rec=None, **opts):
    return api.forward(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
                       torch.from_numpy(cs["amp"]).to(DEV), rec, sponge=cs["sponge"], vref=cs["vref"], **opts)


@pytest.mark.parametrize("so,shape,lx", [
    (2, (46, 41, 70), 9), (4, (46, 41, 70), 11), (8, (46, 41, 70), 13),
    (8, (40, 38, 44), 13),   # last chunk of one plane, shorter than M
    (4, (61, 33, 40), 0),    # automatic chunk
    (16, (52, 36, 40), 17),
])
def test_split_equals_untiled(so, shape, lx):
    cs = make_case(shape, so, 31, 5)  # an odd step count: the last pass is single-level
    base = run(cs, variant=L.FD_VARIANT_NAIVE)
    out = run(cs, variant=L.FD_VARIANT_SPLIT, tile=(lx, 0, 0))
    cfg = api.last_config()
    assert cfg["variant"] == L.FD_VARIANT_SPLIT and cfg["tblock"] == 2, cfg
    assert float(base["u"].abs().max()) > 0
    assert torch.equal(out["u"], base["u"]) and torch.equal(out["u_prev"], base["u_prev"])


def test_split_matches_oracle_with_sources_between_nodes():
    cs = make_case((50, 40, 44), 8, 40, 6, nsrc=12, nrec=4)
    cs["src"] = synth.offgrid_points(cs["shape"], 12, seed=91, margin=1.0)
    base = run(cs, variant=L.FD_VARIANT_NAIVE)
    out = run(cs, variant=L.FD_VARIANT_SPLIT, tile=(12, 32, 4))
    assert api.last_config()["variant"] == L.FD_VARIANT_SPLIT
    assert torch.equal(out["u"], base["u"]) and torch.equal(out["u_prev"], base["u_prev"])
    prob = oracle.Problem(cs["v"].numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["sponge"],
                          cs["vref"], cs["src"], None)
    ref = oracle.forward(prob, amp=cs["amp"].astype(np.float64))
    assert rel_l2(out["u"].cpu().numpy(), ref["u"]) <= 1e-5


def test_split_with_receivers():
    """A few receivers (their entries walked in memory) keep the split form;
    more than 32 entries keep the overlapped chunks.  Both equal the untiled
    kernel."""
    for nrec, variant in ((9, L.FD_VARIANT_SPLIT), (40, L.FD_VARIANT_TBLOCK)):
        cs = make_case((46, 41, 70), 4, 30, 5, nrec=nrec)
        base = run(cs, rec=cs["rec"], variant=L.FD_VARIANT_NAIVE)
        out = run(cs, rec=cs["rec"], variant=L.FD_VARIANT_SPLIT, tile=(11, 0, 0))
        cfg = api.last_config()
        assert cfg["variant"] == variant and cfg["tblock"] == 2, (nrec, cfg)
        assert float(base["rec"].abs().max()) > 0
        assert torch.equal(out["rec"], base["rec"]) and torch.equal(out["u"], base["u"])


def test_split_shots_in_a_batch_equal_single_shots():
    """Split passes recorded into a batch: the first phases of shots of one
    order share grouped launches, and so do their second phases."""
    shots = []
    for i, (shape, so, nt) in enumerate([((44, 38, 46), 4, 25), ((40, 42, 50), 8, 21), ((50, 36, 40), 4, 24)]):
        v = synth.smooth_velocity(shape, seed=500 + i, sigma=3.0).to(DEV)
        dt = 0.8 * 2.0 / (float(v.max()) * np.sqrt(3 * 7.5)) * 10.0
        amp = torch.from_numpy(synth.ricker(nt, dt, 30.0)[:, None].copy()).to(DEV)
        shots.append(dict(v=v, h=[10.0] * 3, so=so, nt=nt, dt=dt, src_idx=synth.centre_source(shape, depth=12),
                          src_amp=amp, rec_idx=synth.receiver_line(shape, 7, depth=12), sponge=4, vref=4500.0,
                          options=dict(variant=L.FD_VARIANT_SPLIT, tile=(13, 0, 0))))
    outs = api.forward_batch(shots, graph=True)
    for sh, tr in zip(shots, outs):
        a = api.forward(sh["v"], sh["h"], sh["so"], sh["nt"], sh["dt"], sh["src_idx"], sh["src_amp"], sh["rec_idx"],
                        sponge=4, vref=4500.0, variant=L.FD_VARIANT_SPLIT, tile=(13, 0, 0))
        assert api.last_config()["variant"] == L.FD_VARIANT_SPLIT
        b = api.forward(sh["v"], sh["h"], sh["so"], sh["nt"], sh["dt"], sh["src_idx"], sh["src_amp"], sh["rec_idx"],
                        sponge=4, vref=4500.0, variant=L.FD_VARIANT_NAIVE)
        assert float(b["rec"].abs().max()) > 0
        assert torch.equal(a["rec"], b["rec"]) and torch.equal(a["u"], b["u"])
        assert torch.equal(tr, b["rec"])


@pytest.mark.parametrize("so", [2, 4])
def test_full_size_split_equals_untiled(so):
    """512^3 (the time-blocking study's grid), 48 steps."""
    import bench

    cs = bench.workload("cfg3", device=DEV)
    nt = 48
    dt = 0.8 * bench.courant_max(so, 3) * 10.0 / 4500.0
    amp = torch.from_numpy(synth.ricker(nt, dt, 15.0)[:, None].copy()).to(DEV)
    outs = []
    for opt in (dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_SPLIT, tile=(74, 32, 2)),
                dict(variant=L.FD_VARIANT_SPLIT)):
        out = api.forward(cs["v"], cs["h"], so, nt, dt, cs["src"], amp, None, sponge=cs["sponge"],
                          vref=cs["vref"], **opt)
        outs.append(out["u"])
        del out
    assert float(outs[0].abs().max()) > 0
    for o in outs[1:]:
        assert torch.equal(outs[0], o)
