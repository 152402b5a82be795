"""Legality of the time-tiled schedule (paper Secs. 5.2-5.5), checked on the CPU.

The paper tiles the skewed iteration space of the leapfrog update with the
CLooG constraint system of its Sec. 5.5 figure: time tiles of 8 levels, x and y
tiles of 16 in the skewed coordinates x + s t, y + s t (skew s = 4 for the
space-order-8 stencil), z untiled, and the scattering order
(tt, xx, yy, t, x, y, z); the time levels live in a modulo-8 buffer.

These tests enumerate that iteration domain from the constraints (not from the
generated loop nest), order it by the scattering function, and check

* every point of the untiled domain is visited exactly once;
* every flow dependence (u^{t+1}(p) needs u^t(p + k e_a), |k| <= M, and
  u^{t-1}(p)) is produced before it is read;
* every slot of the modulo buffer is read before it is overwritten;
* with a skew smaller than the stencil radius M the order is illegal (the
  reading that the skew equals the largest dependence distance, M = so/2);
* executing the updates in the tiled order with the modulo buffer gives the
  untiled result bit for bit (tiling only reorders legal computations).
"""
import itertools

import numpy as np
import pytest


def tiled_order(nt, n, s, ts, tts):
    """Iterations (t, x, y, z) of the update domain 1 <= t <= nt, 0 <= x, y, z < n,
    sorted by the scattering (tt, xx, yy, t, x+st, y+st, z+st) of the paper's
    tiling with skew s, spatial tile ts and time tile tts."""
    t, x, y, z = np.meshgrid(np.arange(1, nt + 1), np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    t, x, y, z = (a.ravel() for a in (t, x, y, z))
    xs, ys, zs = x + s * t, y + s * t, z + s * t
    tt, xx, yy = t // tts, xs // ts, ys // ts
    keys = [zs, ys, xs, t, yy, xx, tt]   # np.lexsort: last key is the primary one
    order = np.lexsort(keys)
    rank = np.empty((nt + 1, n, n, n), dtype=np.int64)
    rank[:] = -1
    rank[t[order], x[order], y[order], z[order]] = np.arange(order.size)
    return rank


def violations(rank, M, buf):
    """Count dependences executed out of order: flow dependences of the leapfrog
    star stencil of radius M, and (for a modulo buffer of `buf` levels) reads of
    a slot that happen after the write that overwrites it."""
    nt = rank.shape[0] - 1
    n = rank.shape[1]
    bad = 0
    for t in range(1, nt + 1):
        cons = rank[t]
        # flow: u^t (written by iteration t - 1) at distance <= M on every axis
        if t - 1 >= 1:
            prod = rank[t - 1]
            for ax in range(3):
                for k in range(-M, M + 1):
                    sl_c = [slice(None)] * 3
                    sl_p = [slice(None)] * 3
                    if k >= 0:
                        sl_c[ax] = slice(0, n - k)
                        sl_p[ax] = slice(k, n)
                    else:
                        sl_c[ax] = slice(-k, n)
                        sl_p[ax] = slice(0, n + k)
                    bad += int(np.sum(prod[tuple(sl_p)] > cons[tuple(sl_c)]))
        # flow: u^{t-1} (written by iteration t - 2) at the same point
        if t - 2 >= 1:
            bad += int(np.sum(rank[t - 2] > cons))
        # anti: iteration t writes u^{t+1} into the slot of u^{t+1-buf}, which is
        # read by iteration t+1-buf (stencil) and t+2-buf (centre)
        r1 = t + 1 - buf
        if r1 >= 1:
            reader = rank[r1]
            for ax in range(3):
                for k in range(-M, M + 1):
                    sl_c = [slice(None)] * 3
                    sl_r = [slice(None)] * 3
                    if k >= 0:
                        sl_c[ax] = slice(0, n - k)
                        sl_r[ax] = slice(k, n)
                    else:
                        sl_c[ax] = slice(-k, n)
                        sl_r[ax] = slice(0, n + k)
                    bad += int(np.sum(reader[tuple(sl_r)] > cons[tuple(sl_c)]))
        r2 = t + 2 - buf
        if 1 <= r2 <= nt:
            bad += int(np.sum(rank[r2] > cons))
    return bad


def test_paper_tiling_visits_every_point_once():
    nt, n = 9, 12
    rank = tiled_order(nt, n, s=4, ts=16, tts=8)
    r = rank[1:].ravel()
    assert np.all(r >= 0)
    assert np.array_equal(np.sort(r), np.arange(r.size))


@pytest.mark.parametrize("M,ts,tts,buf", [(4, 16, 8, 8), (2, 8, 4, 4), (1, 4, 4, 4), (4, 8, 4, 8)])
def test_skew_by_radius_is_legal(M, ts, tts, buf):
    rank = tiled_order(nt=10, n=14, s=M, ts=ts, tts=tts)
    assert violations(rank, M, buf) == 0


@pytest.mark.parametrize("M,ts,tts", [(4, 16, 8), (2, 8, 4)])
def test_skew_below_radius_is_illegal(M, ts, tts):
    rank = tiled_order(nt=10, n=14, s=M - 1, ts=ts, tts=tts)
    assert violations(rank, M, buf=tts) > 0


def test_unskewed_time_tiles_are_illegal():
    rank = tiled_order(nt=8, n=12, s=0, ts=4, tts=4)
    assert violations(rank, 1, buf=4) > 0


def test_untiled_order_is_legal_with_three_buffers():
    # time tile 1, one spatial tile: the plain loop nest with the 3-level buffer
    rank = tiled_order(nt=8, n=8, s=0, ts=1000, tts=1)
    assert violations(rank, 4, buf=3) == 0


@pytest.mark.parametrize("s", [2, 1])
def test_tiled_execution_with_modulo_buffer_matches_untiled(s):
    """Run the leapfrog update in the tiled order, storing levels in a modulo-8
    buffer, and compare with the plain time loop: identical bits with the skew
    equal to the radius (2), different results with a smaller skew."""
    nt, n, M, ts, tts, buf = 10, 10, 2, 8, 8, 8
    rng = np.random.default_rng(5)
    w = np.array([-2.5, 4.0 / 3.0, -1.0 / 12.0])  # so-4 weights (c_0, c_1, c_2)
    q = 0.05 + 0.01 * rng.random((n, n, n))
    u0 = rng.standard_normal((n, n, n))
    um = rng.standard_normal((n, n, n))

    def upd(cur, prev, x, y, z):
        def at(a, i, j, k):
            return a[i, j, k] if 0 <= i < n and 0 <= j < n and 0 <= k < n else 0.0

        lap = 3 * w[0] * cur[x, y, z]
        for k in range(1, M + 1):
            lap += w[k] * (at(cur, x - k, y, z) + at(cur, x + k, y, z))
            lap += w[k] * (at(cur, x, y - k, z) + at(cur, x, y + k, z))
            lap += w[k] * (at(cur, x, y, z - k) + at(cur, x, y, z + k))
        return 2.0 * cur[x, y, z] - prev[x, y, z] + q[x, y, z] * lap

    # untiled: u^{t+1} from u^t, u^{t-1}, iteration t = 1..nt produces level t+1
    lev = {0: um.copy(), 1: u0.copy()}
    for t in range(1, nt + 1):
        nxt = np.empty_like(u0)
        for x, y, z in itertools.product(range(n), repeat=3):
            nxt[x, y, z] = upd(lev[t], lev[t - 1], x, y, z)
        lev[t + 1] = nxt
    # tiled order, modulo buffer
    B = np.zeros((buf, n, n, n))
    B[0 % buf] = um
    B[1 % buf] = u0
    rank = tiled_order(nt, n, s, ts, tts)
    flat = np.argsort(rank[1:].ravel())
    tt_, xx_, yy_, zz_ = np.unravel_index(flat, (nt, n, n, n))
    for t, x, y, z in zip(tt_ + 1, xx_, yy_, zz_):
        B[(t + 1) % buf, x, y, z] = upd(B[t % buf], B[(t - 1) % buf], x, y, z)
    same = np.array_equal(B[(nt + 1) % buf], lev[nt + 1]) and np.array_equal(B[nt % buf], lev[nt])
    assert same == (s >= M)
