"""Born (linearised) modelling on the GPU: traces against the FP64 oracle
(rel-L2 1e-5), every kernel configuration bit-identical to the untiled one
(the tiled runs take the fused one-pass kernel for space orders up to 8 and
two passes per step for so 16), and the FP32 dot test against the
vector-Jacobian product (its transpose)."""
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
CONFIGS = [dict(variant=L.FD_VARIANT_NAIVE), dict(variant=L.FD_VARIANT_STREAM),
           dict(variant=L.FD_VARIANT_STREAM, tile=(9, 0, 0)), dict(variant=L.FD_VARIANT_TBLOCK, tblock=2)]


def born_case(shape=(44, 40, 52), so=8, nt=90, offgrid=False):
    cs = make_case(shape, so, nt, 6, f0=25.0, nsrc=1, nrec=10)
    if offgrid:
        cs["src"] = cs["src"].astype(np.float64) + np.array([[0.37, -0.41, 0.25]])
        cs["rec"] = synth.offgrid_receiver_line(shape, 10, depth=float(cs["rec"][0, -1]) + 0.3)
    dv = (synth.smooth_velocity(shape, seed=77, sigma=3.0) - 3000.0).float()
    return cs, dv


def gpu_born(cs, dv, **opt):
    return api.born(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
                    torch.from_numpy(cs["amp"]).to(DEV), cs["rec"], dv.to(DEV), sponge=cs["sponge"],
                    vref=cs["vref"], **opt)


@pytest.mark.parametrize("so,offgrid", [(4, False), (8, False), (8, True), (16, False)])
def test_born_matches_oracle_and_configs_agree(so, offgrid):
    cs, dv = born_case(so=so, offgrid=offgrid)
    prob = oracle.Problem(cs["v"].numpy().astype(np.float64), cs["h"], cs["so"], cs["nt"], cs["dt"],
                          cs["sponge"], cs["vref"], cs["src"], cs["rec"])
    ref = oracle.born(prob, cs["amp"].astype(np.float64), dv.numpy().astype(np.float64))
    outs = [gpu_born(cs, dv, **o) for o in CONFIGS]
    e = rel_l2(outs[0].cpu().numpy(), ref)
    print(f"born so{so} offgrid={offgrid}: rel_l2 {e:.2e}")
    assert np.linalg.norm(ref) > 0
    assert e <= 1e-5
    for o, out in zip(CONFIGS[1:], outs[1:]):
        assert torch.equal(out, outs[0]), o


def test_born_dot_test_against_vjp():
    """<J dv, y> = <dv, J^T y> with both sides computed on the GPU in FP32."""
    cs, dv = born_case(offgrid=True)
    y = np.random.default_rng(21).standard_normal((cs["nt"], len(cs["rec"]))).astype(np.float32)
    dd = gpu_born(cs, dv).cpu().numpy().astype(np.float64)
    gv = api.vjp(cs["v"].to(DEV), cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"],
                 torch.from_numpy(cs["amp"]).to(DEV), cs["rec"], torch.from_numpy(y).to(DEV),
                 sponge=cs["sponge"], vref=cs["vref"]).cpu().numpy().astype(np.float64)
    lhs = float((dd * y).sum())
    rhs = float((dv.numpy().astype(np.float64) * gv).sum())
    print(f"born dot test: {lhs:.9e} vs {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_born_zero_perturbation_gives_zero_traces():
    cs, dv = born_case(nt=30)
    out = gpu_born(cs, torch.zeros_like(dv))
    assert float(out.abs().max()) == 0.0
