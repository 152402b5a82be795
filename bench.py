"""Benchmark of the acoustic FD sweep on one MI355X.

One "step" of this benchmark is one whole forward sweep of the large
workload: 3-D 512^3 grid, space order 16, 1000 time steps, smoothed random
velocity (seed 1707, sigma 8 cells, 1.5-4.5 km/s), 15 Hz Ricker source at
depth 20, 40-cell sponge, tiled kernel, all inputs resident in HBM.  Its three
512 MiB fields are far beyond the 256 MB Infinity Cache, so the sweep is bound
by HBM.  ``value`` is GPts/s = 512^3 * 1000 / t_sweep.  Next to it the line
reports the untiled and time-blocked kernels on the same workload, the tiled
adjoint sweep, the 256^3 space-order-8 sweep (three 64 MiB fields: resident in
the Infinity Cache, reported as such), FWI gradients/s (256^3, 1000 steps,
256 receivers, checkpoint every 50), the batched shots, the dominant kernel's
HBM roofline and the FP64 oracle timed on the host cores.

Kernel configurations come from the library's autotuner (fd_autotune): its
choices for these workloads, made on an MI355X with ``--retune``, are kept in
paper_1707_02347_amd/autotune_gfx950.txt, which the library reads as its tuning
cache (FD_AUTOTUNE_CACHE); every sweep below asks for the automatic
configuration and records the one that ran.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick] [--no-oracle] [--retune PATH]
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
TUNE_CACHE = os.path.join(HERE, "paper_1707_02347_amd", "autotune_gfx950.txt")

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
    """Seeded synthetic workloads (generators in synth/).  Returns a dict of device inputs."""
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


AUTO = dict(variant=0)  # the autotuner's cached choice for the grid (space-tiled default if none)
T2 = dict(variant=3, tblock=2)  # time-blocked, two levels per pass, default tile


def launch_options(name):
    """Options of a workload's tiled sweep: automatic, i.e. the autotuner's choice."""
    return dict(AUTO)


def retune(path):
    """Run fd_autotune on every workload shape of this benchmark and write the
    choices to ``path`` (the library appends each choice to FD_AUTOTUNE_CACHE)."""
    import torch

    from paper_1707_02347_amd import api

    if os.path.exists(path):
        os.remove(path)
    os.environ["FD_AUTOTUNE_CACHE"] = path
    dt_of = lambda so: 0.8 * courant_max(so, 3) * 10.0 / 4500.0  # the workloads' time step
    # the single-shot workloads (the 256^3 grid serves the sweep, gradient, Born
    # and off-grid rates); batches are tuned per space-order class by
    # fd_batch_autotune instead, since shots tuned one by one would split the
    # grouped launches
    shapes = {((512,) * 3, 16): (dt_of(16), 40), ((256,) * 3, 8): (dt_of(8), 20)}
    out = {}
    for (shape, so), (dt, sponge) in shapes.items():
        t0 = time.perf_counter()
        o = api.autotune(shape, [10.0] * 3, so, dt, sponge=sponge, vref=4500.0, nt=32)
        out[f"{shape[0]}^3 so{so}"] = dict(o, seconds=round(time.perf_counter() - t0, 2))
        print(f"# tuned {shape} so{so}: {o}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    return out


def kernel_source_hash():
    """Hash of the sources the k_stream kernels compile from (their counter
    data is only valid for these); the exchange kernels' fd_wave.h is not
    among them."""
    import hashlib

    h = hashlib.sha1()
    for f in ("fd_stream.h", "fd_internal.h", "fd_stream_configs.h", "fd_stream_entry.h"):
        h.update(open(os.path.join(HERE, "paper_1707_02347_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:12]


def profiled_traffic(profile, kernel):
    """HBM bytes per launch of ``kernel`` from a committed rocprofv3 counter
    summary under profiles/, if it was taken with the current kernel source
    and for that kernel configuration (else None)."""
    path = os.path.join(HERE, "profiles", profile)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash() or kv.get("kernel") != kernel:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_name(cfg, so):
    """Template name of the sweep kernel a configuration (fd_last_config) runs."""
    PY = int(cfg["tile"][2])
    NW = int(cfg["tile"][1]) // max(PY, 1)
    return f"k_stream<M={so // 2},T={int(cfg['tblock'])},PY={PY},NW={NW}>"


def _sweep(cs, opts, nt=None):
    from paper_1707_02347_amd import api

    n = cs["nt"] if nt is None else nt
    return api.forward(cs["v"], cs["h"], cs["so"], n, cs["dt"], cs["src"], cs["amp"][: max(n, 0)].contiguous(),
                       cs["rec"], sponge=cs["sponge"], vref=cs["vref"], **opts)


def _timed(fn, reps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    torch.cuda.synchronize()
    t = np.array(times)
    return float(np.median(t)), float(t.mean()), float(t.std())


def streaming_ceiling(field_mib, reps=30):
    """Rate of a plain elementwise kernel with the sweep's access pattern --
    three arrays read, one written in place over one of them
    (b = a + b * c) -- on fields of the given size: the practical memory
    ceiling for that footprint (the 256 MB Infinity Cache holds three
    64 MiB fields, not three 512 MiB ones).  Returns TB/s of counted bytes."""
    import torch

    n = field_mib * 2 ** 20 // 4
    a = torch.ones(n, device="cuda")
    b = torch.ones(n, device="cuda")
    c = torch.full((n,), 0.5, device="cuda")
    for _ in range(3):
        torch.addcmul(a, b, c, out=b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.addcmul(a, b, c, out=b)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    del a, b, c
    torch.cuda.empty_cache()
    return round(4 * n * 4 / t / 1e12, 2)


def time_sweeps(cs, opts, steps, warmup):
    """Median / mean / std ms of whole sweeps (HIP events on the launch stream)."""
    return _timed(lambda: _sweep(cs, opts), steps, warmup)


def adjoint_case(cs, nrec=256):
    """The adjoint sweep of a workload: residual traces injected at ``nrec``
    receivers on a line at depth 20 (seeded synthetic traces), the result
    recorded at the source."""
    import torch

    import synth

    rec = synth.receiver_line(cs["v"].shape, nrec, depth=20)
    g = torch.Generator(device=cs["v"].device).manual_seed(2347)
    res = torch.randn((cs["nt"], nrec), generator=g, device=cs["v"].device) * cs["amp"].abs().max()
    return rec, res


def _adjoint(cs, rec, res, opts, nt=None):
    from paper_1707_02347_amd import api

    n = cs["nt"] if nt is None else nt
    return api.adjoint(cs["v"], cs["h"], cs["so"], n, cs["dt"], cs["src"], rec, res[: max(n, 0)].contiguous(),
                       sponge=cs["sponge"], vref=cs["vref"], **opts)


def roofline_of(sweep_ms, setup, launches, npts, bytes_per_point, kernel, profile=None):
    """Roofline block of a sweep's dominant kernel: its average launch time
    (sweep minus a zero-step call with the same set-up, over the launches) and
    the algorithmic bytes per launch."""
    kern_ms = max(sweep_ms - setup, 1e-6) / launches
    bpl = bytes_per_point * npts
    achieved = bpl / (kern_ms * 1e-3) / 1e9
    traffic = profiled_traffic(profile, kernel) if profile else None
    # traffic: counted HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, copy
    # calibrated), beside the algorithmic bytes per launch
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_over_algorithmic": round(traffic / bpl, 3) if traffic else None,
            "kernel": kernel, "avg_launch_us": round(kern_ms * 1e3, 2), "launches": launches,
            "bytes_per_launch": bpl, "bytes_per_point": bytes_per_point}


def time_block(fn, steps, warmup):
    """ms per step of exactly ``steps`` calls timed as one block: synchronize,
    then HIP events on the launch stream and the host clock around the block,
    synchronize again.  Returns (event ms per step, wall ms per step)."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def setup_ms(cs, opts, reps=3):
    """Time of a zero-step call (validation, q, tables): subtracted to get kernel time."""
    return _timed(lambda: _sweep(cs, opts, nt=0), reps, 1)[0]


def oracle_baseline(cs, budget_s=20.0):
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

    import ctypes

    gomp = ctypes.CDLL("libgomp.so.1")  # the OpenMP runtime the oracle is built with
    cores = int(gomp.omp_get_max_threads())
    t3 = run(3) / 3.0
    steps = int(max(2, min(500, budget_s / max(t3, 1e-3))))
    t = run(steps)
    out = {"value": round(npts * steps / t / 1e9, 4), "unit": "GPts/s", "cores": cores, "kind": "oracle",
           "sample": f"{steps} of the {cs['nt']} steps of {cs['name']} at full size ({npts} points), FP64",
           "seconds": round(t, 3)}
    # the same loop nest on one core (a bounded sample of a few steps)
    gomp.omp_set_num_threads(1)
    try:
        t1 = run(1)
        steps1 = int(max(1, min(20, 0.3 * budget_s / max(t1, 1e-3))))
        ts = run(steps1) if steps1 > 1 else t1
    finally:
        gomp.omp_set_num_threads(cores)
    out["one_core"] = {"value": round(npts * steps1 / ts / 1e9, 4), "steps": steps1, "seconds": round(ts, 3)}
    return out


# Time-blocking study on the HBM-bound 512^3 grid of the so-16 workload, for
# space orders 2 / 4 / 8: the autotuner's best space-tiled (T = 1) and best
# time-blocked (T >= 2) configurations, each timed on whole 48-step sweeps.
# The configurations the profiling runs use (--kernel-only tblock-so8) are the
# so-8 choices tuned on MI355X: space-tiled, overlapped two-level, and
# two-level without redundant halos (neighbour exchange).
TIME_BLOCKING = {
    8: (dict(variant=2, tile=(256, 32, 8)), dict(variant=3, tblock=2, tile=(64, 32, 2)),
        dict(variant=5, tile=(0, 16, 2))),
}


def time_blocking_study(nt=48):
    """512^3, sponge 40, space orders 2 / 4 / 8: GPts/s of the tuner's best
    T = 1, best overlapped T >= 2 and best two-level exchange (no redundant
    halo) configuration (sweep minus set-up), with the choices; gain is the
    better time-blocked form over T = 1."""
    import torch

    import synth
    from paper_1707_02347_amd import api

    import tempfile

    base = workload("cfg3")
    out = {}
    # the study's own choices go to a scratch cache file, not the committed one
    saved = os.environ.get("FD_AUTOTUNE_CACHE")
    os.environ["FD_AUTOTUNE_CACHE"] = os.path.join(tempfile.gettempdir(), "fdwave_tb_study_tune.txt")
    for so in (2, 4, 8):
        cs = dict(base)
        cs["so"] = so
        cs["nt"] = nt
        cs["dt"] = 0.8 * courant_max(so, 3) * 10.0 / 4500.0
        cs["amp"] = torch.from_numpy(synth.ricker(nt, cs["dt"], 15.0)[:, None].copy()).to(base["v"].device)
        npts = int(np.prod(cs["v"].shape))
        r = {}
        # time-blocked: overlapped tiles (T = 2..4) and two-level passes
        # without redundant halos, each tuned on its own
        for name, variant in (("space_tiled", 2), ("time_blocked", 3), ("time_blocked_exchange", 5)):
            o = api.autotune(tuple(cs["v"].shape), cs["h"], so, cs["dt"], sponge=cs["sponge"], vref=cs["vref"],
                             nt=24, variant=variant)
            med, _, _ = time_sweeps(cs, o, 3, 1)
            ms = max(med - setup_ms(cs, o), 1e-6)
            r[name] = dict(o, gpts=round(npts * nt / (ms * 1e-3) / 1e9, 1))
        best = max(r["time_blocked"]["gpts"], r["time_blocked_exchange"]["gpts"])
        r["gain"] = round(best / r["space_tiled"]["gpts"] - 1.0, 3)
        out[f"so{so}"] = r
    if saved is None:
        os.environ.pop("FD_AUTOTUNE_CACHE", None)
    else:
        os.environ["FD_AUTOTUNE_CACHE"] = saved
    del base
    torch.cuda.empty_cache()
    return out


def offgrid(cs):
    """The same workload with its source and receivers moved between grid nodes
    (multilinear interpolation): source +0.37 / -0.39 / +0.45 cells off its node,
    receivers on a line at fractional x, y + 0.29 and depth 20.37."""
    import synth

    out = dict(cs)
    out["src"] = cs["src"].astype(np.float64) + np.array([[0.37, -0.39, 0.45]])
    nrec = 256 if cs["rec"] is None else len(cs["rec"])
    out["rec"] = synth.offgrid_receiver_line(cs["v"].shape, nrec, depth=20.37)
    return out


def offgrid_rates(cs):
    """cfg2 sweep with 256 receivers, on grid nodes and between them (GPts/s):
    multilinear (8 nodes per point) and Kaiser-windowed sinc of half-width 4
    (512 nodes per point)."""
    import synth
    from paper_1707_02347_amd import api

    on = dict(cs, rec=synth.receiver_line(cs["v"].shape, 256, depth=20))
    off = offgrid(on)
    sinc = dict(off, src=api.Sinc(off["src"], 4), rec=api.Sinc(off["rec"], 4))
    npts = int(np.prod(cs["v"].shape))
    out = {}
    for name, c in (("on_grid_256rec", on), ("off_grid_256rec", off), ("sinc4_256rec", sinc)):
        med, _, _ = time_sweeps(c, launch_options("cfg2"), 3, 1)
        out[name] = round(npts * c["nt"] / ((med - setup_ms(c, launch_options("cfg2"))) * 1e-3) / 1e9, 2)
    return out


def born_rate(reps=2, warmup=1):
    """Born modelling on the headline grid (256^3 so 8, 500 steps, 256 receivers):
    GPts/s of the linearised operator (one point-step advances the background
    and the perturbation wavefield)."""
    import synth
    from paper_1707_02347_amd import api

    cs = workload("cfg2")
    rec = synth.receiver_line(cs["v"].shape, 256, depth=20)
    dv = 0.05 * cs["v"] * synth.blob_velocity(cs["v"], amp=1.0, width_frac=1.0 / 16.0).sub(cs["v"]).div(cs["v"])
    run = lambda: api.born(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], rec, dv,
                           sponge=cs["sponge"], vref=cs["vref"], **launch_options("cfg2"))
    med, _, _ = _timed(run, reps, warmup)
    npts = int(np.prod(cs["v"].shape))
    return {"gpts": round(npts * cs["nt"] / (med * 1e-3) / 1e9, 2), "ms": round(med, 1),
            "config": "256^3 so8, 500 steps, 256 receivers, dv = 5 % Gaussian blob of width N/16"}


def gradient_rate(reps=2, warmup=1, off_grid=False, ckpt_every=50, sinc=0):
    """cfg4: FWI gradients/s (256^3, so 8, 1000 steps, 256 receivers, checkpoint every 50);
    off_grid: points between nodes (multilinear, or windowed sinc of half-width ``sinc``)."""
    import torch

    import synth
    from paper_1707_02347_amd import api

    cs = workload("cfg4")
    if off_grid:
        cs = offgrid(cs)
        if sinc:
            cs = dict(cs, src=api.Sinc(cs["src"], sinc), rec=api.Sinc(cs["rec"], sinc))
    vtrue = synth.blob_velocity(cs["v"], amp=0.05, width_frac=1.0 / 16.0)
    d_obs = api.forward(vtrue, cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"], cs["rec"],
                        sponge=cs["sponge"], vref=cs["vref"], **launch_options("cfg4"))["rec"]
    out = {}

    def run():
        out["J"], out["g"], _ = api.gradient(cs["v"], cs["h"], cs["so"], cs["nt"], cs["dt"], cs["src"], cs["amp"],
                                             cs["rec"], d_obs, sponge=cs["sponge"], vref=cs["vref"], ckpt_every=ckpt_every,
                                             **launch_options("cfg4"))

    med, mean, std = _timed(run, reps, warmup)
    del d_obs
    torch.cuda.empty_cache()
    return {"gradients_per_s": round(1000.0 / med, 3), "ms": round(med, 1), "misfit": out["J"],
            "config": "cfg4: 256^3 so8, 1000 steps, 256 receivers, d_obs from a +5% Gaussian blob, checkpoint 50"}


def batch_shots(device="cuda"):
    """cfg5: 32 seeded shots, cubic N in [128, 320], space orders {4, 8, 16}, nt in [500, 1000]."""
    import torch

    import synth

    shots = []
    for sh in synth.shot_batch(32, seed=2347):
        n, so, nt = sh["n"], sh["so"], sh["nt"]
        shape = (n, n, n)
        v = synth.smooth_velocity(shape, seed=sh["vseed"], sigma=8.0, device=device)
        dt = 0.8 * courant_max(so, 3) * 10.0 / 4500.0
        amp = torch.from_numpy(synth.ricker(nt, dt, 15.0)[:, None].copy()).to(device)
        shots.append(dict(v=v, h=[10.0] * 3, so=so, nt=nt, dt=dt, src_idx=synth.centre_source(shape, depth=20),
                          src_amp=amp, rec_idx=synth.receiver_line(shape, 128, depth=20), sponge=20, vref=4500.0,
                          options=dict(launch_options("cfg5"), ckpt_every=50)))
    return shots


def batch_rates():
    """Batched forward and gradients of cfg5 vs the same shots one by one with the untiled kernel."""
    import torch

    import synth
    from paper_1707_02347_amd import api

    shots = batch_shots()
    pts = sum(float(np.prod(s["v"].shape)) * s["nt"] for s in shots)
    res = {}
    # the planner's default tile for every shot, then the batch tuner's choice
    # (one kernel per space-order class, timed on the class's grouped launches)
    dflt = [dict(s, options=dict(s["options"], variant=2)) for s in shots]
    med_d, _, _ = _timed(lambda: api.forward_batch(dflt, graph=True), 1, 1)
    res["forward_batched_default_tile_gpts"] = round(pts / (med_d * 1e-3) / 1e9, 2)
    del dflt
    t0 = time.perf_counter()
    chosen = api.batch_autotune(shots)
    res["batch_autotune_s"] = round(time.perf_counter() - t0, 2)
    res["batch_autotune_choice"] = {f"so{s['so']}": c for s, c in zip(shots, chosen)}
    med, _, _ = _timed(lambda: api.forward_batch(shots, graph=True), 1, 1)
    res["forward_batched_gpts"] = round(pts / (med * 1e-3) / 1e9, 2)

    def sequential_untiled():
        for s in shots:
            api.forward(s["v"], s["h"], s["so"], s["nt"], s["dt"], s["src_idx"], s["src_amp"], s["rec_idx"],
                        sponge=s["sponge"], vref=s["vref"], variant=1)

    med_u, _, _ = _timed(sequential_untiled, 1, 0)
    res["forward_sequential_untiled_gpts"] = round(pts / (med_u * 1e-3) / 1e9, 2)
    # observed data from a perturbed model, then all 32 gradients in one batch
    traces = api.forward_batch([dict(s, v=synth.blob_velocity(s["v"], 0.05, 1.0 / 16.0)) for s in shots])
    for s, d in zip(shots, traces):
        s["d_obs"] = d
    t0 = time.perf_counter()
    misfits, grads = api.gradient_batch(shots, graph=True)
    torch.cuda.synchronize()
    tg = time.perf_counter() - t0
    res["gradients_batched_per_s"] = round(len(shots) / tg, 3)
    res["gradient_batch_s"] = round(tg, 2)
    res["shots"] = len(shots)
    res["point_steps"] = pts
    del grads, traces
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--retune", metavar="PATH", default=None,
                    help="run the autotuner on every workload shape and write its choices to PATH")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only a plain 1 GiB device copy (calibrates the HBM byte counters)")
    ap.add_argument("--kernel-only", choices=["cfg3", "cfg3-adjoint", "cfg2", "tblock-so8", "born", "sinc", "batch",
                                              "gradient"],
                    default=None,
                    help="only short runs of one workload, for profiling: cfg3 (512^3 so 16, whole "
                         "sweeps), cfg3-adjoint (its adjoint, whole sweeps), cfg2 (256^3 so 8, whole "
                         "sweeps), tblock-so8 (512^3 so 8: T = 1, overlapped T = 2, exchange T = 2), born (Born modelling "
                         "on the 256^3 grid, 256 receivers), sinc (the 256^3 sweep with windowed-sinc "
                         "points, r = 4), batch (the 32-shot forward batch) or gradient (the 256^3 so-8 "
                         "gradient, 200 steps, checkpoints every 50)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        return 2
    if args.retune:
        print(json.dumps({"retuned": retune(args.retune), "cache": args.retune}), flush=True)
        return 0
    # the autotuner's cached choices: automatic plans of these grids take them
    os.environ.setdefault("FD_AUTOTUNE_CACHE", TUNE_CACHE)

    import torch

    from paper_1707_02347_amd import api

    if args.copy_probe:
        n = 256 * 1024 * 1024
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        ms = _timed(lambda: y.copy_(x), 5, 2)[0]
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "copy_gbs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}), flush=True)
        return 0
    if args.kernel_only:
        return kernel_only(args)

    # ---------------------------------------------------------------- headline: 512^3 so 16
    print("# cfg3 512^3 so16 nt1000", file=sys.stderr, flush=True)
    c3 = workload("cfg3")
    n3 = int(np.prod(c3["v"].shape))
    tiled = launch_options("cfg3")
    ev, wall = time_block(lambda: _sweep(c3, tiled), args.steps, args.warmup)
    med, mean, std = time_sweeps(c3, tiled, 3, 0)
    _sweep(c3, tiled, nt=4)
    cfg3_used = api.last_config()
    setup3 = setup_ms(c3, tiled)
    T = int(cfg3_used["tblock"])
    launches = c3["nt"] // T + c3["nt"] % T
    kname = kernel_name(cfg3_used, c3["so"])
    roof = roofline_of(ev, setup3, launches, n3, 16 if T == 1 else 20, kname,
                       profile="k_stream_512cube_so16_counters.txt")
    roof["streaming_ceiling_tbs_512mib_fields"] = streaming_ceiling(512, reps=10)
    roof["frac_of_streaming_ceiling"] = round(roof["achieved"] / (roof["streaming_ceiling_tbs_512mib_fields"] * 1000.0), 4)
    gpts = n3 * c3["nt"] / (ev * 1e-3) / 1e9
    variants = {"tiled": round(gpts, 2)}
    for k, o in (("time_tiled_T2", T2), ("untiled", dict(variant=1))):
        m, _, _ = time_sweeps(c3, o, 1, 1)
        variants[k] = round(n3 * c3["nt"] / (m * 1e-3) / 1e9, 2)
    line = {
        "metric": METRIC,
        "value": round(gpts, 2),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ev, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cfg3: 3-D 512^3, space order 16, 1000 steps, smoothed random v (seed 1707, "
                               "sigma 8 cells, 1.5-4.5 km/s), 15 Hz Ricker at depth 20, 40-cell sponge; one "
                               "step = one whole 1000-step sweep; tiled kernel from the autotuner's cached "
                               "choice (untiled and time-blocked T = 2 reported beside)",
                   "launch": cfg3_used, "parallelism": "single GPU"},
        "roofline": roof,
        "bw_equiv_frac_16B": round(gpts * 16 / HBM_PEAK_GBS, 4),
        # the same at the 20 B per point a Devito-style count gives (it also
        # streams m and damp; this build derives damp from 1-D profiles)
        "bw_equiv_frac_20B": round(gpts * 20 / HBM_PEAK_GBS, 4),
        "variants_gpts": variants,
        "wall_ms_per_step": round(wall, 3),
        "ms_block_median_std": [round(ev, 3), round(med, 3), round(std, 3)],
    }
    # ---------------------------------------------------------------- the tiled adjoint sweep
    print("# adjoint sweeps", file=sys.stderr, flush=True)
    adj = {}
    rec3, res3 = adjoint_case(c3)
    am, _, _ = _timed(lambda: _adjoint(c3, rec3, res3, tiled), 2, 1)
    _adjoint(c3, rec3, res3, tiled, nt=4)
    acfg = api.last_config()
    asetup = _timed(lambda: _adjoint(c3, rec3, res3, tiled, nt=0), 3, 1)[0]
    ar = roofline_of(am, asetup, c3["nt"] // int(acfg["tblock"]) + c3["nt"] % int(acfg["tblock"]), n3, 16,
                     kernel_name(acfg, c3["so"]), profile="k_stream_512cube_so16_adjoint_counters.txt")
    adj["cfg3"] = {"gpts": round(n3 * c3["nt"] / (am * 1e-3) / 1e9, 2), "ms": round(am, 2), "launch": acfg,
                   "roofline": ar, "config": "cfg3 grid; residual traces injected at 256 receivers (depth 20), "
                                             "result recorded at the source"}
    del rec3, res3, c3
    torch.cuda.empty_cache()
    # ---------------------------------------------------------------- 256^3 so 8 (cache-resident)
    print("# cfg2 256^3 so8 nt500 (cache-resident)", file=sys.stderr, flush=True)
    cs = workload("cfg2")
    npts = int(np.prod(cs["v"].shape))
    c2 = {}
    for k, o in (("tiled", launch_options("cfg2")), ("untiled", dict(variant=1)), ("time_tiled_T2", T2)):
        e2, _ = time_block(lambda: _sweep(cs, o), max(3, args.steps // 2), 1)
        c2[k] = round(npts * cs["nt"] / (e2 * 1e-3) / 1e9, 2)
        if k == "tiled":
            ev2 = e2
    _sweep(cs, launch_options("cfg2"), nt=4)
    cfg2_used = api.last_config()
    r2 = roofline_of(ev2, setup_ms(cs, launch_options("cfg2")), cs["nt"] // int(cfg2_used["tblock"]) +
                     cs["nt"] % int(cfg2_used["tblock"]), npts, 16, kernel_name(cfg2_used, cs["so"]),
                     profile="k_stream_cfg2_counters.txt")
    r2["streaming_ceiling_tbs_64mib_fields"] = streaming_ceiling(64)
    line["cfg2_cache_resident"] = {
        "gpts": c2, "launch": cfg2_used, "roofline": r2,
        "note": "256^3 so 8, 500 steps: three 64 MiB fields stay in the 256 MB Infinity Cache between steps, "
                "so this rate is not bound by HBM"}
    rec2, res2 = adjoint_case(cs)
    am2, _, _ = _timed(lambda: _adjoint(cs, rec2, res2, launch_options("cfg2")), 3, 1)
    adj["cfg2_cache_resident"] = {"gpts": round(npts * cs["nt"] / (am2 * 1e-3) / 1e9, 2), "ms": round(am2, 2)}
    del rec2, res2
    line["adjoint"] = adj
    if not args.quick:
        print("# time blocking at 512^3", file=sys.stderr, flush=True)
        line["time_blocking_512cube_gpts"] = time_blocking_study()
        print("# cfg4", file=sys.stderr, flush=True)
        line["cfg4_fwi_gradient"] = gradient_rate()
        print("# off-grid points", file=sys.stderr, flush=True)
        og = offgrid_rates(cs)
        g = gradient_rate(off_grid=True)
        og["cfg4_off_grid_gradients_per_s"] = g["gradients_per_s"]
        og["cfg4_sinc4_gradients_per_s"] = gradient_rate(reps=1, off_grid=True, sinc=4)["gradients_per_s"]
        line["off_grid_points"] = og
        # the whole time axis stored (1000 second differences, 64 GB) instead of
        # checkpoints every 50 steps: no recomputation sweep
        line["cfg4_full_storage_gradients_per_s"] = gradient_rate(ckpt_every=1000)["gradients_per_s"]
        print("# Born modelling", file=sys.stderr, flush=True)
        line["born_modelling"] = born_rate()
        print("# cfg5", file=sys.stderr, flush=True)
        try:
            line["cfg5_batched"] = batch_rates()
        except Exception as e:  # report, do not lose the line
            line["cfg5_batched"] = {"error": f"{type(e).__name__}: {e}"}
        torch.cuda.empty_cache()
    del cs
    torch.cuda.empty_cache()
    if not args.no_oracle:
        print("# oracle baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = oracle_baseline(workload("cfg3"), budget_s=15.0)
    print(json.dumps(line), flush=True)
    return 0


def kernel_only(args):
    """Short runs of one workload for profiling (kernel trace or counters)."""
    import torch

    import synth
    from paper_1707_02347_amd import api

    n = args.warmup + args.steps
    what = args.kernel_only
    if what == "batch":
        # the planner's default tile for every shot (the profiles of the grouped
        # kernels; the benchmark's tuned batch differs only in its tile choice)
        shots = [dict(s, options=dict(s["options"], variant=2)) for s in batch_shots()]
        for _ in range(n):
            api.forward_batch(shots, graph=True)
    elif what == "sinc":
        cs = offgrid(dict(workload("cfg2"), rec=synth.receiver_line((256,) * 3, 256, depth=20)))
        cs = dict(cs, src=api.Sinc(cs["src"], 4), rec=api.Sinc(cs["rec"], 4))
        for _ in range(n):
            _sweep(cs, launch_options("cfg2"), nt=20)
    elif what == "born":
        cs = workload("cfg2")
        rec = synth.receiver_line(cs["v"].shape, 256, depth=20)
        dv = 0.05 * (synth.blob_velocity(cs["v"], amp=1.0, width_frac=1.0 / 16.0) - cs["v"])
        for _ in range(n):
            api.born(cs["v"], cs["h"], cs["so"], 20, cs["dt"], cs["src"], cs["amp"][:20].contiguous(), rec, dv,
                     sponge=cs["sponge"], vref=cs["vref"], **launch_options("cfg2"))
    elif what == "cfg2":
        cs = workload("cfg2")
        for _ in range(n):
            _sweep(cs, launch_options("cfg2"))
    elif what == "gradient":
        # the gradient workload's kernels (checkpointed forward, recomputation
        # saving second differences, adjoint with imaging, image flushes) over
        # 200 steps; the residual's values do not change the kernels' cost
        cs = workload("cfg4")
        nt = 200
        g = torch.Generator(device="cuda").manual_seed(4)
        d_obs = 1e-3 * torch.randn((nt, len(cs["rec"])), generator=g, device="cuda")
        for _ in range(n):
            api.gradient(cs["v"], cs["h"], cs["so"], nt, cs["dt"], cs["src"], cs["amp"][:nt].contiguous(), cs["rec"],
                         d_obs, sponge=cs["sponge"], vref=cs["vref"], ckpt_every=50, **launch_options("cfg4"))
    elif what == "cfg3-adjoint":
        cs = workload("cfg3")
        rec, res = adjoint_case(cs)
        for _ in range(n):
            _adjoint(cs, rec, res, launch_options("cfg3"))
    else:
        cs = workload("cfg3")
        opts = [launch_options("cfg3")]
        if what == "tblock-so8":
            cs["so"] = 8
            cs["dt"] = 0.8 * courant_max(8, 3) * 10.0 / 4500.0
            cs["amp"] = torch.from_numpy(synth.ricker(cs["nt"], cs["dt"], 15.0)[:, None].copy()).to("cuda")
            opts = list(TIME_BLOCKING[8])
        # whole sweeps for the headline kernel (a launch's time varies along the
        # sweep, so only the whole sweep's average compares with the benchmark)
        steps = cs["nt"] if what == "cfg3" else 20
        for o in opts:
            for _ in range(n):
                _sweep(cs, o, nt=steps)
    torch.cuda.synchronize()
    launch = "default tile per shot" if what == "batch" else api.last_config()
    print(json.dumps({"profiled": what, "runs": n, "launch": launch}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
