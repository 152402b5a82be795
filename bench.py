"""Benchmark of the acoustic FD sweep on one MI355X.

One "step" of this benchmark is one whole forward sweep of the headline
workload: 3-D 256^3 grid, space order 8, 500 time steps, smoothed random
velocity (seed 1707, sigma 8 cells, 1.5-4.5 km/s), 15 Hz Ricker source at
depth 20, 20-cell sponge, time-tiled kernel, all inputs resident in HBM.
``value`` is GPts/s = N^3 * nt / t_sweep.  Next to it the line reports the
untiled and space-tiled kernels on the same workload, the 512^3 space-order-16
sweep (tiled vs untiled), FWI gradients/s (256^3, 1000 steps, 256 receivers,
checkpoint every 50), the batched shots, the dominant kernel's HBM roofline
and the FP64 oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--no-oracle]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)

METRIC = "GPts/s + % HBM roofline, tiled vs untiled; FWI gradients/s at rel err 1e-5"
HBM_PEAK_GBS = 8000.0


def _weights(so):
    M = so // 2
    c = [0.0] * (M + 1)
    for k in range(1, M + 1):
        r = 1.0
        for j in range(1, k + 1):
            r *= (M - k + j) / (M + j)
        c[k] = 2.0 * (1 if k % 2 else -1) * r / (k * k)
    c[0] = -2.0 * sum(c[1:])
    return c


def courant_max(so, ndim):
    """Largest stable v dt / h of the leapfrog star stencil (equal spacing)."""
    c = _weights(so)
    S = -c[0] - 2 * sum(c[k] * (-1) ** k for k in range(1, so // 2 + 1))
    return 2.0 / math.sqrt(ndim * S)


def workload(name, device="cuda"):
    """Synthetic workloads (recipes in the design doc).  Returns a dict of device inputs."""
    import torch

    import synth

    if name == "cfg1":
        shape, so, nt, h, v0 = (128, 128), 4, 100, 10.0, 1500.0
        dt = 0.5 * h / v0
        v = torch.full(shape, v0, dtype=torch.float32, device=device)
        amp = synth.ricker(nt, dt, 10.0)[:, None].copy()
        return dict(name=name, v=v, h=[h, h], so=so, nt=nt, dt=dt, src=np.array([[64, 64]], np.int32),
                    amp=torch.from_numpy(amp).to(device), rec=None, sponge=0, vref=v0)
    if name in ("cfg2", "cfg4"):
        n, so, L, nt = 256, 8, 20, (500 if name == "cfg2" else 1000)
    elif name == "cfg3":
        n, so, L, nt = 512, 16, 40, 1000
    else:
        raise ValueError(name)
    shape = (n, n, n)
    h = 10.0
    v = synth.smooth_velocity(shape, seed=1707, sigma=8.0, device=device)
    dt = 0.8 * courant_max(so, 3) * h / 4500.0
    amp = synth.ricker(nt, dt, 15.0)[:, None].copy()
    src = synth.centre_source(shape, depth=20)
    rec = synth.receiver_line(shape, 256, depth=20) if name == "cfg4" else None
    return dict(name=name, v=v, h=[h, h, h], so=so, nt=nt, dt=dt, src=src,
                amp=torch.from_numpy(amp).to(device), rec=rec, sponge=L, vref=4500.0)


# Launch configuration of each workload's time-tiled sweep (chosen by the
# library's autotuner on MI355X).
TUNED = {
    "cfg2": dict(variant=3, tile=(0, 32, 8), tblock=2),
    "cfg3": dict(variant=3, tile=(0, 32, 4), tblock=2),
    "cfg4": dict(variant=3, tile=(0, 32, 8), tblock=2),
}


def launch_options(name):
    return dict(TUNED.get(name, dict(variant=2)))


def _sweep(cs, opts, nt=None):
    from paper_1707_02347_amd import api

    return api.forward(cs["v"], cs["h"], cs["so"], cs["nt"] if nt is None else nt, cs["dt"], cs["src"],
                       cs["amp"] if nt is None else cs["amp"][: max(nt, 0)].contiguous(), cs["rec"],
                       sponge=cs["sponge"], vref=cs["vref"], **opts)


def time_sweeps(cs, opts, steps, warmup):
    """Median/mean/std ms of whole sweeps, bracketed by synchronisations, HIP events."""
    import torch

    for _ in range(warmup):
        _sweep(cs, opts)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _sweep(cs, opts)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    t = np.array(times)
    return float(np.median(t)), float(t.mean()), float(t.std())


def setup_ms(cs, opts, reps=3):
    """Time of a zero-step call (validation, q, tables): subtracted to get kernel time."""
    import torch

    best = 1e30
    for _ in range(reps):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _sweep(cs, opts, nt=0)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def oracle_baseline(cs, budget_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload (a few full-size steps)."""
    import oracle

    v = cs["v"].cpu().numpy().astype(np.float64)
    amp = cs["amp"].cpu().numpy().astype(np.float64)
    npts = v.size

    def run(steps):
        prob = oracle.Problem(v, cs["h"], cs["so"], steps, cs["dt"], cs["sponge"], cs["vref"], cs["src"], None)
        t0 = time.perf_counter()
        oracle.forward(prob, amp=amp[:steps])
        return time.perf_counter() - t0

    t1 = run(1)
    steps = int(max(2, min(200, budget_s / max(t1, 1e-3))))
    t = run(steps)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": npts * steps / t / 1e9, "unit": "GPts/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} of {cs['nt']} steps of {cs['name']} at full size ({npts} points), FP64",
            "seconds": round(t, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-oracle", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        return 2

    import torch

    from paper_1707_02347_amd import api

    dev = "cuda"
    cs = workload("cfg2", dev)
    npts = int(np.prod(cs["v"].shape))
    tiled = launch_options("cfg2")
    variants = {"untiled": dict(variant=1), "space_tiled": dict(variant=2), "time_tiled": tiled}
    res = {}
    for k, o in variants.items():
        med, mean, std = time_sweeps(cs, o, args.steps if k == "time_tiled" else max(2, args.steps // 2),
                                     args.warmup)
        res[k] = dict(ms=med, mean_ms=mean, std_ms=std, gpts=npts * cs["nt"] / (med * 1e-3) / 1e9)
    cfg_used = api.last_config()
    api.forward(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], None,
                sponge=cs["sponge"], vref=cs["vref"], **tiled)
    cfg_used = api.last_config()

    # roofline of the dominant kernel (the time-blocked sweep kernel)
    T = cfg_used["tblock"]
    setup = setup_ms(cs, tiled)
    launches = cs["nt"] // T + (cs["nt"] % T)
    kern_ms = max(res["time_tiled"]["ms"] - setup, 1e-6) / launches
    bytes_per_launch = (20 if T >= 2 else 16) * npts
    achieved = bytes_per_launch / (kern_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"k_stream M=4 T={T}", "avg_launch_us": round(kern_ms * 1e3, 2),
            "bytes_per_launch": bytes_per_launch}
    line = {
        "metric": METRIC,
        "value": round(res["time_tiled"]["gpts"], 2),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["time_tiled"]["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cfg2: 3-D 256^3, space order 8, 500 steps, smoothed random v "
                               "(seed 1707, sigma 8, 1.5-4.5 km/s), 15 Hz Ricker at depth 20, 20-cell "
                               "sponge, time-tiled", "launch": cfg_used, "parallelism": "single GPU"},
        "roofline": roof,
        "bw_equiv_frac_16B": round(res["time_tiled"]["gpts"] * 16 / HBM_PEAK_GBS, 4),
        "variants_gpts": {k: round(v["gpts"], 2) for k, v in res.items()},
        "variants_ms": {k: [round(v["ms"], 3), round(v["mean_ms"], 3), round(v["std_ms"], 3)]
                        for k, v in res.items()},
    }
    if not args.no_oracle:
        line["cpu_baseline"] = oracle_baseline(cs)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
