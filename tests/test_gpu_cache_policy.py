"""The cache policy of the loads each point makes once per step
(FD_FLAG_LOADS_STREAM: non-temporal, FD_FLAG_LOADS_KEEP: ordinary, neither:
chosen from the fields' size) only changes the instructions' cache-policy bits:
forward sweeps (space-tiled and time-blocked), the gradient (its snapshot-saving
and imaging passes) and grouped batch launches give results identical bit for
bit to the untiled kernel and to each other."""
import numpy as np
import pytest
import torch

import synth
from paper_1707_02347_amd import _lib as L
from paper_1707_02347_amd import api

pytestmark = pytest.mark.gpu
DEV = "cuda"
POLICIES = [0, L.FD_FLAG_LOADS_STREAM, L.FD_FLAG_LOADS_KEEP]


def case(shape=(46, 41, 70), so=8, nt=26):
    v = synth.smooth_velocity(shape, seed=23, sigma=4.0)
    dt = 0.8 * 0.45 * 10.0 / float(v.max())
    src = synth.centre_source(shape, depth=9)
    rec = synth.receiver_line(shape, 11, depth=9)
    amp = torch.from_numpy(synth.ricker(nt, dt, 25.0)[:, None].copy()).to(DEV)
    return v.to(DEV), [10.0] * 3, so, nt, dt, src, rec, amp


@pytest.mark.parametrize("so,opts", [
    (8, dict(variant=L.FD_VARIANT_STREAM)),
    (4, dict(variant=L.FD_VARIANT_STREAM, tile=(16, 32, 4))),
    (4, dict(variant=L.FD_VARIANT_TBLOCK, tblock=2)),
    (2, dict(variant=L.FD_VARIANT_TBLOCK, tblock=3, tile=(0, 32, 4))),
])
def test_forward_identical_under_both_policies(so, opts):
    v, h, _, nt, dt, src, rec, amp = case(so=so)
    base = api.forward(v, h, so, nt, dt, src, amp, rec, sponge=6, vref=4500.0, variant=L.FD_VARIANT_NAIVE)
    for flags in POLICIES:
        out = api.forward(v, h, so, nt, dt, src, amp, rec, sponge=6, vref=4500.0, flags=flags, **opts)
        assert torch.equal(out["rec"], base["rec"]), flags
        assert torch.equal(out["u"], base["u"]), flags
        assert torch.equal(out["u_prev"], base["u_prev"]), flags


def test_gradient_identical_under_both_policies():
    v, h, so, nt, dt, src, rec, amp = case(so=8, nt=30)
    d_obs = api.forward(v * 1.03, h, so, nt, dt, src, amp, rec, sponge=6, vref=4500.0)["rec"]
    ref = None
    for flags in POLICIES:
        J, g, res = api.gradient(v, h, so, nt, dt, src, amp, rec, d_obs, sponge=6, vref=4500.0,
                                 variant=L.FD_VARIANT_STREAM, ckpt_every=7, flags=flags)
        if ref is None:
            ref = (J, g, res)
            assert float(g.abs().max()) > 0.0
            continue
        assert J == ref[0], flags
        assert torch.equal(g, ref[1]), flags
        assert torch.equal(res, ref[2]), flags


def test_batch_identical_under_both_policies():
    shapes = [((40, 38, 44), 4, 24), ((36, 44, 52), 8, 21), ((48, 40, 46), 16, 18)]
    shots = []
    for i, (shape, so, nt) in enumerate(shapes):
        v = synth.smooth_velocity(shape, seed=300 + i, sigma=3.0).to(DEV)
        dt = 0.8 * 2.0 / (float(v.max()) * np.sqrt(3 * 7.5)) * 10.0
        amp = torch.from_numpy(synth.ricker(nt, dt, 30.0)[:, None].copy()).to(DEV)
        shots.append(dict(v=v, h=[10.0] * 3, so=so, nt=nt, dt=dt, src_idx=synth.centre_source(shape, depth=12),
                          src_amp=amp, rec_idx=synth.receiver_line(shape, 9, depth=12), sponge=4,
                          vref=4500.0, options={}))
    ref = None
    for flags in POLICIES:
        for sh in shots:
            sh["options"] = dict(flags=flags)
        outs = api.forward_batch(shots, graph=True)
        if ref is None:
            ref = [o.clone() for o in outs]
            for sh, o in zip(shots, outs):
                single = api.forward(sh["v"], sh["h"], sh["so"], sh["nt"], sh["dt"], sh["src_idx"], sh["src_amp"],
                                     sh["rec_idx"], sponge=4, vref=4500.0)["rec"]
                assert torch.equal(o, single)
            continue
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), flags
