"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only *generates inputs*: velocity models, source wavelets, acquisition
geometry and initial fields.  It holds none of the finite-difference method's
arithmetic (no stencil weights, no update, no sponge, no adjoint), so that the
oracle and the product path can both consume its output without sharing any of
the method's code.

Recipes (every one seeded and deterministic):

* ``smooth_velocity``: i.i.d. uniform [0, 1) per cell from numpy's PCG64
  ``default_rng(seed)``, smoothed by a separable Gaussian (sigma in cells,
  truncated at 4 sigma, half-sample-symmetric "reflect" boundary) in float64,
  then min-max mapped onto [vmin, vmax] m/s and rounded to float32.  This is the
  "smoothed random velocity" workload family (1.5-4.5 km/s).
* ``blob_velocity``: v0 * (1 + a * exp(-|x - c|^2 / (2 w^2))) with c the grid
  centre, the perturbed "true" model used to synthesise observed data.
* ``ricker``: the textbook Ricker wavelet (1 - 2 pi^2 f^2 tau^2) exp(-pi^2 f^2 tau^2),
  tau = t - 1/f, sampled at t = n * dt.
* ``gaussian_field``: the smooth Gaussian initial wavefield used in the paper's
  functional-correctness runs (Sec. 6.5): an isotropic normal density with
  mean 0 and sigma 0.4 per axis evaluated on a [-1, 1]^d lattice.
* ``shot_batch``: a seeded list of uneven shots (cubic N in [128, 320], space
  order in {4, 8, 16}, nt in [500, 1000]).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "smooth_velocity",
    "blob_velocity",
    "ricker",
    "gaussian_field",
    "centre_source",
    "receiver_line",
    "shot_batch",
    "uniform_random_field",
]


def _gauss_taps(sigma: float, truncate: float = 4.0) -> np.ndarray:
    radius = int(truncate * sigma + 0.5)
    j = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-0.5 * (j / sigma) ** 2)
    return w / w.sum()


def _smooth_axis(t, axis: int, taps: np.ndarray):
    """Separable 1-D Gaussian along ``axis`` with half-sample-symmetric padding."""
    import torch

    n = t.shape[axis]
    r = (len(taps) - 1) // 2
    j = np.arange(-r, n + r)
    # reflect about the half-sample edge: ... c b a | a b c ... | c b a ...
    period = 2 * n
    j = np.mod(j, period)
    j = np.where(j >= n, period - 1 - j, j)
    idx = torch.as_tensor(j, device=t.device, dtype=torch.long)
    padded = torch.index_select(t, axis, idx)
    out = torch.zeros_like(t)
    for k, w in enumerate(taps):
        out += float(w) * padded.narrow(axis, k, n)
    return out


def uniform_random_field(shape, seed: int = 1707) -> np.ndarray:
    """i.i.d. uniform [0, 1) float64 values from PCG64 ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.random(tuple(int(s) for s in shape), dtype=np.float64)


def smooth_velocity(shape, seed: int = 1707, sigma: float = 8.0, vmin: float = 1500.0,
                    vmax: float = 4500.0, device: str = "cpu"):
    """Smoothed random velocity model (float32 torch tensor on ``device``), m/s."""
    import torch

    base = torch.from_numpy(uniform_random_field(shape, seed)).to(device)
    taps = _gauss_taps(sigma)
    f = base
    for ax in range(base.dim()):
        if base.shape[ax] > 1:
            f = _smooth_axis(f, ax, taps)
    lo, hi = f.min(), f.max()
    span = hi - lo
    if float(span) == 0.0:
        f = torch.full_like(f, 0.5 * (vmin + vmax))
    else:
        f = vmin + (f - lo) * ((vmax - vmin) / span)
    return f.to(torch.float32).contiguous()


def blob_velocity(v0, amp: float = 0.05, width_frac: float = 1.0 / 16.0):
    """``v0 * (1 + amp * exp(-|x - c|^2 / (2 w^2)))``, w = width_frac * N (per axis)."""
    import torch

    shape = v0.shape
    dev = v0.device
    r2 = torch.zeros(shape, dtype=torch.float64, device=dev)
    for ax, n in enumerate(shape):
        w = max(width_frac * n, 1.0)
        c = 0.5 * (n - 1)
        coord = (torch.arange(n, dtype=torch.float64, device=dev) - c) / w
        view = [1] * len(shape)
        view[ax] = n
        r2 = r2 + (coord ** 2).view(view)
    out = v0.to(torch.float64) * (1.0 + amp * torch.exp(-0.5 * r2))
    return out.to(torch.float32).contiguous()


def ricker(nt: int, dt: float, f0: float, delay: float | None = None) -> np.ndarray:
    """Ricker wavelet sampled at t = n*dt, n = 0..nt-1, as float32."""
    t0 = (1.0 / f0) if delay is None else delay
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def gaussian_field(shape, sigma: float = 0.4) -> np.ndarray:
    """Isotropic normal density (mean 0, std ``sigma`` per axis) on a [-1, 1]^d lattice, float32."""
    d = len(shape)
    grids = np.meshgrid(*[np.linspace(-1.0, 1.0, int(n)) for n in shape], indexing="ij")
    r2 = sum(g * g for g in grids)
    norm = (2.0 * math.pi * sigma * sigma) ** (-0.5 * d)
    return (norm * np.exp(-0.5 * r2 / (sigma * sigma))).astype(np.float32)


def centre_source(shape, depth: int | None = None) -> np.ndarray:
    """One source at the grid centre; with ``depth`` the last (contiguous) axis index is set to it."""
    idx = [int(n) // 2 for n in shape]
    if depth is not None:
        idx[-1] = int(depth)
    return np.asarray([idx], dtype=np.int32)


def receiver_line(shape, nrec: int, depth: int = 20, cross: int | None = None) -> np.ndarray:
    """``nrec`` receivers evenly spaced along axis 0, at axis-1 index ``cross`` and depth ``depth``."""
    n0 = int(shape[0])
    xs = np.floor(np.arange(nrec, dtype=np.float64) * n0 / nrec).astype(np.int64)
    xs = np.clip(xs, 0, n0 - 1)
    out = np.zeros((nrec, len(shape)), dtype=np.int32)
    out[:, 0] = xs
    if len(shape) == 3:
        out[:, 1] = int(shape[1]) // 2 if cross is None else int(cross)
    out[:, -1] = int(depth)
    return out


def offgrid_points(shape, npts: int, seed: int = 1707, margin: float = 0.0) -> np.ndarray:
    """``npts`` seeded positions in grid-index units (float64, [npts][ndim]), each
    coordinate uniform in [margin, n_a - 1 - margin]: points between grid nodes."""
    rng = np.random.default_rng(seed)
    lo = np.full(len(shape), float(margin))
    hi = np.array([float(n) - 1.0 - margin for n in shape])
    return lo + (hi - lo) * rng.random((npts, len(shape)))


def offgrid_receiver_line(shape, nrec: int, depth: float = 20.37, cross: float | None = None) -> np.ndarray:
    """``nrec`` receivers evenly spaced along axis 0 between nodes (float64
    positions), at axis-1 position ``cross`` (default: the middle plus 0.29 cell)
    and depth ``depth`` along the last axis."""
    n0 = float(shape[0])
    out = np.zeros((nrec, len(shape)), dtype=np.float64)
    out[:, 0] = 0.45 + np.arange(nrec, dtype=np.float64) * (n0 - 1.9) / max(nrec, 1)
    if len(shape) == 3:
        out[:, 1] = float(shape[1]) / 2.0 + 0.29 if cross is None else float(cross)
    out[:, -1] = float(depth)
    return out


def shot_batch(nshots: int = 32, seed: int = 2347, nmin: int = 128, nmax: int = 320,
               orders=(4, 8, 16), ntmin: int = 500, ntmax: int = 1000):
    """Seeded uneven shot list: dicts with keys ``n`` (cubic side), ``so``, ``nt``, ``vseed``."""
    rng = np.random.default_rng(seed)
    shots = []
    for s in range(nshots):
        n = int(rng.integers(nmin, nmax + 1))
        so = int(orders[int(rng.integers(0, len(orders)))])
        nt = int(rng.integers(ntmin, ntmax + 1))
        shots.append({"n": n, "so": so, "nt": nt, "vseed": int(seed * 1000 + s)})
    return shots
