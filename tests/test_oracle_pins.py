"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own update: each compares it with an
independent derivation (Taylor moment conditions solved exactly, a dense
Kronecker-sum Laplacian, the whole space-time system solved as one dense linear
system, complex-step differentiation), a closed form (polynomial exactness,
the discrete dispersion relation), an invariant (discrete energy balance,
symmetry) or a value the paper prints (the order-8 FP32 constants).
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- independent helpers
def taylor_weights(M):
    """Exact weights of the symmetric 2M-order second-derivative stencil from the
    Taylor moment conditions sum_k c_|k| k^p = 2 [p == 2], p = 0, 2, ..., 2M."""
    n = M + 1
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for j in range(n):  # moment p = 2j
        A[j][0] = Fraction(1 if j == 0 else 0)
        for k in range(1, M + 1):
            A[j][k] = Fraction(2 * k ** (2 * j))
        b[j] = Fraction(2 if j == 1 else 0)
    for col in range(n):  # exact Gauss-Jordan
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] -= f * b[col]
    return [b[i] / A[i][i] for i in range(n)]


def dense_lap(shape, h, so):
    """Dense Dirichlet star Laplacian as a Kronecker sum of 1-D band matrices."""
    c = [float(x) for x in taylor_weights(so // 2)]
    M = so // 2
    mats = []
    for n in shape:
        D = np.zeros((n, n))
        for i in range(n):
            for k in range(-M, M + 1):
                if 0 <= i + k < n:
                    D[i, i + k] = c[abs(k)]
        mats.append(D)
    N = int(np.prod(shape))
    L = np.zeros((N, N))
    for a in range(len(shape)):
        term = np.array([[1.0]])
        for b_ in range(len(shape)):
            term = np.kron(term, mats[b_] / h[a] ** 2 if b_ == a else np.eye(shape[b_]))
        L += term
    return L


def sponge_reading(shape, h, L, vref):
    """Separable quadratic sponge of the adopted reading, evaluated directly."""
    out = np.zeros(shape)
    for a, n in enumerate(shape):
        i = np.arange(n)
        delta = np.where(i < L, L - i, np.where(i > n - 1 - L, i - (n - 1 - L), 0)).astype(float)
        d = 1.5 * math.log(1000.0) / (vref * L * h[a]) * (delta / L) ** 2 if L > 0 else 0 * delta
        view = [1] * len(shape)
        view[a] = n
        out = out + d.reshape(view)
    return out


def flat_index(shape, idx):
    return int(np.ravel_multi_index(tuple(int(x) for x in idx), shape))


# ---------------------------------------------------------------- weights
@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_weights_match_taylor_derivation(so):
    exact = taylor_weights(so // 2)
    got = oracle.weights(so)
    for e, g in zip(exact, got):
        assert abs(float(e) - g) <= 1e-15 * max(1.0, abs(float(e)))


def test_weights_known_rationals():
    assert taylor_weights(2) == [Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)]
    assert taylor_weights(4) == [Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5),
                                 Fraction(8, 315), Fraction(-1, 560)]
    assert taylor_weights(8)[0] == Fraction(-1077749, 352800)
    assert taylor_weights(8)[8] == Fraction(-1, 411840)


def test_weights_reproduce_paper_printed_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_so8_constants.json")))
    c = oracle.weights(g["space_order"])
    scale = 2.0 * g["dt"] ** 2 / g["h"] ** 2
    for k, printed in g["printed_neighbour"].items():
        val = scale * c[int(k)]
        assert abs(val - printed) <= 1e-6 * abs(printed), (k, val, printed)
    centre = 3 * scale * c[0]
    assert abs(centre - g["printed_centre"]) <= 1e-6 * abs(g["printed_centre"])


# ---------------------------------------------------------------- Laplacian
def _poly_case(ndim, so, degree, seed):
    rng = np.random.default_rng(seed)
    M = so // 2
    n = [2 * M + 5 + a for a in range(ndim)]
    h = [0.07 + 0.02 * a for a in range(ndim)]
    coords = [(np.arange(n[a]) - 0.5 * (n[a] - 1)) * h[a] for a in range(ndim)]
    polys = [np.polynomial.Polynomial(rng.uniform(-1, 1, degree + 1)) for _ in range(ndim)]
    grids = np.meshgrid(*coords, indexing="ij")
    vals = [polys[a](grids[a]) for a in range(ndim)]
    d2 = [polys[a].deriv(2)(grids[a]) for a in range(ndim)]
    u = np.prod(vals, axis=0)
    lap = sum(d2[a] * np.prod([vals[b] for b in range(ndim) if b != a], axis=0) for a in range(ndim))
    inner = tuple(slice(M, n[a] - M) for a in range(ndim))
    return u, lap, h, inner, polys, grids


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("so", [2, 4, 8, 16])
def test_laplacian_exact_on_polynomials(ndim, so):
    u, lap, h, inner, _, _ = _poly_case(ndim, so, so + 1, 17 * so + ndim)
    got = oracle.laplacian(u, h, so)
    err = np.abs(got[inner] - lap[inner]).max()
    assert err <= 1e-8 * np.abs(lap[inner]).max(), err


@pytest.mark.parametrize("so", [2, 4, 8, 16])
def test_laplacian_leading_error_term(so):
    """For u = x^(so+2) the truncation error is 2 h^so sum_k c_k k^(so+2) exactly."""
    M = so // 2
    n, h = 4 * M + 3, 0.5
    x = (np.arange(n) - (n - 1) / 2) * h
    u = x ** (so + 2)
    exact_d2 = (so + 2) * (so + 1) * x ** so
    c = taylor_weights(M)
    e = 2 * sum(c[k] * Fraction(k) ** (so + 2) for k in range(1, M + 1)) * Fraction(h) ** so
    got = oracle.laplacian(u, [h], so)
    inner = slice(M, n - M)
    assert float(e) != 0.0
    # rounding allowance per point: a few ulps of the largest |u| inside the stencil window
    csum = float(sum(abs(x) for x in c)) * 2
    win = np.array([np.abs(u[max(0, i - M):i + M + 1]).max() for i in range(n)])
    allow = 1e-9 * abs(float(e)) + 64 * np.finfo(float).eps * csum * win / h ** 2
    err = np.abs((got - exact_d2) - float(e))
    assert (err[inner] <= allow[inner]).all()
    assert err[n // 2] <= 1e-9 * abs(float(e))


@pytest.mark.parametrize("shape,so", [((7,), 2), ((9, 6), 4), ((6, 5, 7), 8), ((5, 6, 4), 2)])
def test_laplacian_matches_dense_kronecker_sum(shape, so):
    rng = np.random.default_rng(3)
    h = [1.0 + 0.25 * a for a in range(len(shape))]
    u = rng.standard_normal(shape)
    L = dense_lap(shape, h, so)
    np.testing.assert_allclose(oracle.laplacian(u, h, so).ravel(), L @ u.ravel(), rtol=0, atol=1e-12)


# ---------------------------------------------------------------- dispersion (stencil + update)
@pytest.mark.parametrize("shape,so,steps", [((220,), 8, 12), ((70, 64), 4, 9), ((44, 40, 42), 8, 3),
                                            ((56, 48), 16, 2)])
def test_plane_wave_follows_discrete_dispersion(shape, so, steps):
    ndim = len(shape)
    M = so // 2
    h = [10.0 * (1 + 0.1 * a) for a in range(ndim)]
    v = 2000.0
    c = [float(x) for x in taylor_weights(M)]
    kappa = [2 * math.pi / (9.5 * h[a]) * (1 + 0.3 * a) for a in range(ndim)]
    sig = sum((-c[0] - 2 * sum(c[k] * math.cos(k * kappa[a] * h[a]) for k in range(1, M + 1))) / h[a] ** 2
              for a in range(ndim))
    sig_max = sum((-c[0] - 2 * sum(c[k] * (-1) ** k for k in range(1, M + 1))) / h[a] ** 2
                  for a in range(ndim))
    dt = 0.9 * 2.0 / (v * math.sqrt(sig_max))  # inside the leapfrog stability limit
    omega = 2.0 / dt * math.asin(v * dt / 2.0 * math.sqrt(sig))
    grids = np.meshgrid(*[np.arange(n) * h[a] for a, n in enumerate(shape)], indexing="ij")
    phase = sum(kappa[a] * grids[a] for a in range(ndim))
    prob = oracle.Problem(np.full(shape, v), h, so, steps, dt)
    out = oracle.forward(prob, u0=np.cos(phase), um1=np.cos(phase + omega * dt))
    exact = np.cos(phase - omega * steps * dt)
    reach = steps * M
    inner = tuple(slice(reach, n - reach) for n in shape)
    assert out["u"][inner].size > 0
    np.testing.assert_allclose(out["u"][inner], exact[inner], rtol=0, atol=1e-11)


# ---------------------------------------------------------------- energy
def _energy_series(hist, L, m, damp, dt):
    """E^{n+1/2} = <m du, du>/dt^2 - <u^{n+1}, L u^n> and the damping loss per step."""
    U = hist.reshape(hist.shape[0], -1)
    LU = U @ L.T
    du = U[1:] - U[:-1]
    E = (du * du * m).sum(1) / dt ** 2 - (U[1:] * LU[:-1]).sum(1)
    loss = ((U[2:] - U[:-2]) ** 2 * damp).sum(1) / (2 * dt)
    return E, loss


@pytest.mark.parametrize("shape,so,steps", [((13, 12, 14), 8, 400), ((40, 36), 4, 1500), ((60,), 16, 800)])
def test_energy_conserved_with_dirichlet_and_variable_m(shape, so, steps):
    ndim = len(shape)
    h = [10.0 + a for a in range(ndim)]
    v = synth.smooth_velocity(shape, seed=11, sigma=2.0).numpy().astype(np.float64)
    dt = 0.5 * min(h) / v.max() * 0.7
    g = synth.gaussian_field(shape, sigma=0.25).astype(np.float64)
    prob = oracle.Problem(v, h, so, steps, dt)
    out = oracle.forward(prob, u0=g, um1=0.9 * g, history=True)
    L = dense_lap(shape, h, so)
    E, _ = _energy_series(out["hist"], L, (1 / v ** 2).ravel(), np.zeros(v.size), dt)
    assert np.abs(E - E[0]).max() <= 1e-10 * np.abs(E).max()


def test_energy_balance_with_sponge():
    shape, so, steps = (16, 15, 17), 4, 300
    h = [10.0, 10.0, 10.0]
    v = synth.smooth_velocity(shape, seed=5, sigma=2.0).numpy().astype(np.float64)
    dt = 0.5 * 10.0 / v.max() * 0.8
    g = synth.gaussian_field(shape, sigma=0.3).astype(np.float64)
    prob = oracle.Problem(v, h, so, steps, dt, sponge=5, vref=4500.0)
    out = oracle.forward(prob, u0=g, um1=g, history=True)
    damp = sponge_reading(shape, h, 5, 4500.0)
    np.testing.assert_allclose(oracle.damp(prob), damp, rtol=1e-14, atol=0)
    L = dense_lap(shape, h, so)
    E, loss = _energy_series(out["hist"], L, (1 / v ** 2).ravel(), damp.ravel(), dt)
    bal = E[1:] - E[:-1] + loss
    assert np.abs(bal).max() <= 1e-9 * np.abs(E).max()
    assert (np.diff(E) <= 1e-9 * np.abs(E).max()).all()
    assert E[-1] < 0.9 * E[0]


def test_sponge_reading_hand_values():
    shape, h, L, vref = (50,), [10.0], 20, 4500.0
    prob = oracle.Problem(np.full(shape, 3000.0), h, 4, 1, 1e-3, sponge=L, vref=vref)
    d = oracle.damp(prob)
    # 1.5 ln(1000) vref / (L h) = 233.1367 1/s, divided by vref^2 (s/m^2 like m)
    d0 = 233.1367407 / 4500.0 ** 2
    assert abs(d0 - 1.5 * math.log(1000.0) / (4500.0 * 20 * 10.0)) < 1e-9 * d0
    assert d[0] == pytest.approx(d0, rel=1e-7)
    assert d[49] == pytest.approx(d0, rel=1e-7)
    assert d[19] == pytest.approx(d0 / 400.0, rel=1e-7)
    assert d[20] == 0.0 and d[29] == 0.0 and d[25] == 0.0
    assert d[30] == pytest.approx(d0 / 400.0, rel=1e-7)


# ---------------------------------------------------------------- textbook special case
def test_paper_1d_kernel_with_corrected_sign():
    """so=2, 1-D, constant v, no damping reduces to u+ = 2u - u- + C^2 (u_{i+1} - 2u_i + u_{i-1})."""
    n, steps, v, h, dt = 31, 25, 1500.0, 10.0, 0.004
    C2 = (v * dt / h) ** 2
    rng = np.random.default_rng(0)
    u0 = rng.standard_normal(n)
    um = rng.standard_normal(n)
    a, b = u0.copy(), um.copy()
    for _ in range(steps):
        pad = np.concatenate([[0.0], a, [0.0]])
        new = 2 * a - b + C2 * (pad[2:] - 2 * pad[1:-1] + pad[:-2])
        a, b = new, a
    out = oracle.forward(oracle.Problem(np.full(n, v), [h], 2, steps, dt), u0=u0, um1=um)
    np.testing.assert_allclose(out["u"], a, rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["u_prev"], b, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- whole recurrence as one linear system
def _space_time_system(shape, h, so, nt, dt, v, damp, src, rec):
    N = int(np.prod(shape))
    L = dense_lap(shape, h, so)
    m = 1.0 / v.ravel() ** 2
    A = np.diag(2 * m + dt * damp.ravel())
    B = 4 * np.diag(m) + 2 * dt * dt * L
    Cm = np.diag(dt * damp.ravel() - 2 * m)
    big = np.zeros((nt * N, nt * N), dtype=np.result_type(v, 1.0))
    for k in range(nt):
        big[k * N:(k + 1) * N, k * N:(k + 1) * N] = A
        if k >= 1:
            big[k * N:(k + 1) * N, (k - 1) * N:k * N] = -B
        if k >= 2:
            big[k * N:(k + 1) * N, (k - 2) * N:(k - 1) * N] = -Cm
    S = np.zeros((nt * N, nt * len(src)))
    for k in range(nt):
        for s, idx in enumerate(src):
            S[k * N + flat_index(shape, idx), k * len(src) + s] += 2 * dt * dt
    P = np.zeros((nt * len(rec), nt * N))
    for k in range(nt):
        for r, idx in enumerate(rec):
            P[k * len(rec) + r, k * N + flat_index(shape, idx)] = 1.0
    return big, S, P


CASES = [
    ((7,), 2, 6, 0),
    ((6, 7), 4, 5, 2),
    ((5, 4, 6), 4, 4, 1),
    ((6, 6, 6), 8, 3, 2),
]


@pytest.mark.parametrize("shape,so,nt,L", CASES)
def test_forward_and_adjoint_equal_dense_space_time_solve(shape, so, nt, L):
    rng = np.random.default_rng(len(shape) * 100 + so)
    ndim = len(shape)
    h = [10.0 + 2 * a for a in range(ndim)]
    v = rng.uniform(1500, 3000, shape)
    dt = 0.3 * min(h) / v.max()
    src = np.array([[n // 2 for n in shape], [0] * ndim, [n // 2 for n in shape]], dtype=np.int32)
    rec = np.array([[n - 1 - a for a, n in enumerate(shape)], [n // 3 for n in shape],
                    [n // 2 for n in shape]], dtype=np.int32)
    prob = oracle.Problem(v, h, so, nt, dt, sponge=L, vref=4000.0, src=src, rec=rec)
    damp = sponge_reading(shape, h, L, 4000.0)
    big, S, P = _space_time_system(shape, h, so, nt, dt, v, damp, src, rec)
    w = rng.standard_normal((nt, len(src)))
    U = np.linalg.solve(big, S @ w.ravel())
    out = oracle.forward(prob, amp=w, history=True)
    N = int(np.prod(shape))
    np.testing.assert_allclose(out["u"].ravel(), U[(nt - 1) * N:], rtol=0, atol=1e-13 * np.abs(U).max())
    np.testing.assert_allclose(out["rec"].ravel(), P @ U, rtol=0, atol=1e-13 * np.abs(U).max())
    F = P @ np.linalg.solve(big, S)
    y = rng.standard_normal((nt, len(rec)))
    adj = oracle.adjoint(prob, y)["src"]
    np.testing.assert_allclose(adj.ravel(), F.T @ y.ravel(), rtol=0, atol=1e-12 * np.abs(F.T @ y.ravel()).max())


@pytest.mark.parametrize("shape,so,nt,L", [((6, 5), 4, 6, 1), ((4, 4, 5), 2, 5, 1)])
def test_gradient_equals_complex_step_of_dense_system(shape, so, nt, L):
    rng = np.random.default_rng(7)
    ndim = len(shape)
    h = [10.0] * ndim
    v = rng.uniform(1500, 3000, shape)
    dt = 0.3 * min(h) / v.max()
    src = np.array([[n // 2 for n in shape]], dtype=np.int32)
    rec = np.array([[0] * ndim, [n - 1 for n in shape], [1] * ndim], dtype=np.int32)
    damp = sponge_reading(shape, h, L, 4000.0)
    w = rng.standard_normal((nt, 1))
    d_obs = rng.standard_normal((nt, len(rec))) * 1e-6
    prob = oracle.Problem(v, h, so, nt, dt, sponge=L, vref=4000.0, src=src, rec=rec)
    J, gv, gm = oracle.gradient(prob, w, d_obs)

    def J_of_m(m):
        vv = 1.0 / np.sqrt(m.astype(complex))
        big, S, P = _space_time_system(shape, h, so, nt, dt, vv, damp, src, rec)
        r = P @ np.linalg.solve(big, S @ w.ravel()) - d_obs.ravel()
        return 0.5 * np.sum(r * r)

    m0 = 1.0 / v ** 2
    assert abs(J_of_m(m0).real - J) <= 1e-12 * J
    eps = 1e-30
    cs = np.zeros(m0.size)
    for i in range(m0.size):
        mm = m0.astype(complex).ravel()
        mm[i] += 1j * eps
        cs[i] = J_of_m(mm.reshape(shape)).imag / eps
    np.testing.assert_allclose(gm.ravel(), cs, rtol=0, atol=1e-10 * np.abs(cs).max())
    np.testing.assert_allclose(gv, gm * (-2.0 / v ** 3), rtol=1e-14)


# ---------------------------------------------------------------- larger-size invariants
def _medium_problem(nt=60, n=(20, 18, 22), so=8, L=5):
    v = synth.smooth_velocity(n, seed=1707, sigma=3.0).numpy().astype(np.float64)
    h = [10.0, 10.0, 10.0]
    dt = 0.8 * 0.4529 * 10.0 / v.max()
    src = synth.centre_source(n, depth=6)
    rec = synth.receiver_line(n, 12, depth=6)
    prob = oracle.Problem(v, h, so, nt, dt, sponge=L, vref=4500.0, src=src, rec=rec)
    w = synth.ricker(nt, dt, 60.0).astype(np.float64)[:, None]
    return prob, v, w


def test_dot_product_fp64():
    prob, _, w = _medium_problem()
    rng = np.random.default_rng(1)
    y = rng.standard_normal((prob.nt, len(prob.rec)))
    d = oracle.forward(prob, amp=w)["rec"]
    fty = oracle.adjoint(prob, y)["src"]
    lhs, rhs = float((d * y).sum()), float((w * fty).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_gradient_central_finite_difference_fp64():
    prob, v, w = _medium_problem(nt=50)
    rng = np.random.default_rng(2)
    vtrue = synth.blob_velocity(__import__("torch").from_numpy(v.astype(np.float32))).numpy().astype(np.float64)
    ptrue = oracle.Problem(vtrue, prob.h, prob.so, prob.nt, prob.dt, prob.sponge, prob.vref, prob.src, prob.rec)
    d_obs = oracle.forward(ptrue, amp=w)["rec"]
    J, gv, _ = oracle.gradient(prob, w, d_obs)
    dv = rng.standard_normal(v.shape) * 10.0
    eps = 1e-3

    def J_at(vv):
        p = oracle.Problem(vv, prob.h, prob.so, prob.nt, prob.dt, prob.sponge, prob.vref, prob.src, prob.rec)
        r = oracle.forward(p, amp=w)["rec"] - d_obs
        return 0.5 * float((r * r).sum())

    fd = (J_at(v + eps * dv) - J_at(v - eps * dv)) / (2 * eps)
    an = float((gv * dv).sum())
    assert abs(fd - an) <= 1e-7 * abs(an)


def test_point_source_solution_has_cube_symmetry():
    n, so, nt = 17, 8, 30
    v = np.full((n, n, n), 2500.0)
    src = np.array([[8, 8, 8]], dtype=np.int32)
    dt = 0.8 * 0.4529 * 10.0 / 2500.0
    prob = oracle.Problem(v, [10.0] * 3, so, nt, dt, sponge=3, vref=2500.0, src=src)
    w = synth.ricker(nt, dt, 80.0).astype(np.float64)[:, None]
    u = oracle.forward(prob, amp=w)["u"]
    assert np.abs(u).max() > 0
    for perm in itertools.permutations(range(3)):
        np.testing.assert_allclose(np.transpose(u, perm), u, rtol=0, atol=1e-14 * np.abs(u).max())
    for ax in range(3):
        np.testing.assert_allclose(np.flip(u, ax), u, rtol=0, atol=1e-14 * np.abs(u).max())


def test_first_step_injection_and_receiver_sampling():
    shape, so, nt = (9, 8, 10), 4, 3
    v = np.random.default_rng(4).uniform(1500, 4000, shape)
    h = [10.0, 12.0, 9.0]
    dt = 1e-3
    src = np.array([[1, 2, 3], [4, 4, 4]], dtype=np.int32)
    rec = np.array([[1, 2, 3], [4, 4, 5], [8, 7, 9]], dtype=np.int32)
    prob = oracle.Problem(v, h, so, nt, dt, sponge=2, vref=3000.0, src=src, rec=rec)
    w = np.array([[1.5, -0.5], [0.25, 2.0], [0.0, 1.0]])
    out = oracle.forward(prob, amp=w, history=True)
    damp = sponge_reading(shape, h, 2, 3000.0)
    u1 = out["hist"][2]
    expect = np.zeros(shape)
    for s, idx in enumerate(src):
        t = tuple(idx)
        expect[t] = 2 * dt * dt * w[0, s] / (dt * damp[t] + 2.0 / v[t] ** 2)
    np.testing.assert_allclose(u1, expect, rtol=1e-15, atol=0)
    for n in range(nt):
        for r, idx in enumerate(rec):
            assert out["rec"][n, r] == out["hist"][n + 2][tuple(idx)]


# ---------------------------------------------------------------- points off the grid
# A point between nodes acts through multilinear interpolation (the reading
# adopted for the paper's unspecified source/receiver operators): a receiver
# reads P u, a source adds A^{-1} 2 dt^2 P^T w.  The pins below use what
# interpolation fixes on its own: it reproduces multilinear functions, its
# weights sum to one and have their centre at the point, integer positions are
# the grid indices, and forward and adjoint stay transposes.
OFFGRID_REC = np.array([[4.25, 5.5, 6.75], [3.0, 7.125, 5.0], [6.5, 4.0, 4.0], [5.875, 2.0625, 8.5]])


def _multilinear(x, y, z):
    return 1.0 + 0.3 * x - 0.2 * y + 0.1 * z + 0.05 * x * y - 0.02 * y * z + 0.01 * x * z + 0.003 * x * y * z


@pytest.mark.parametrize("so", [2, 4])
def test_offgrid_receivers_read_multilinear_fields_exactly(so):
    """u^0 = u^-1 = P with P multilinear: every stencil row sums to zero and P is
    linear along each axis, so L_h P = 0 wherever the stencil stays on the grid and
    u^1 = P there; interpolation then returns P at any point of such a cell."""
    shape = (11, 12, 13)
    X = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    P = _multilinear(*X)
    prob = oracle.Problem(np.full(shape, 2000.0), [10.0, 12.0, 9.0], so, 1, 1e-3, rec=OFFGRID_REC)
    out = oracle.forward(prob, u0=P, um1=P)
    expect = np.array([_multilinear(*p) for p in OFFGRID_REC])
    np.testing.assert_allclose(out["rec"][0], expect, rtol=1e-13, atol=0)


@pytest.mark.parametrize("pos", [(4.25, 5.5, 6.75), (0.0, 11.0, 3.4), (10.0, 0.6, 12.0), (7.0, 3.0, 2.0)])
def test_offgrid_source_spreads_unit_mass_at_its_position(pos):
    """From rest, one step with constant m and no sponge leaves dt^2 v^2 a times
    the interpolation weights: nonnegative, summing to one, centred on the point
    and confined to the nodes of its cell."""
    shape, v, dt, a = (11, 12, 13), 2000.0, 1e-3, 1.7
    prob = oracle.Problem(np.full(shape, v), [10.0] * 3, 4, 1, dt, src=np.array([pos]))
    u1 = oracle.forward(prob, amp=np.array([[a]]))["u"]
    mass = dt * dt * v * v * a
    assert abs(u1.sum() - mass) <= 1e-14 * mass
    assert u1.min() >= 0.0
    X = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    for ax in range(3):
        assert abs(float((u1 * X[ax]).sum()) / float(u1.sum()) - pos[ax]) <= 1e-12
    support = np.argwhere(u1 != 0.0)
    assert np.all(np.abs(support - np.array(pos)) < 1.0)
    assert len(support) <= 8


def test_integer_positions_equal_grid_indices():
    shape, so, nt = (9, 8, 10), 4, 12
    v = np.random.default_rng(5).uniform(1500, 4000, shape)
    h, dt = [10.0, 12.0, 9.0], 1e-3
    src = np.array([[1, 2, 3], [4, 4, 4]], dtype=np.int32)
    rec = np.array([[1, 2, 3], [4, 4, 5], [8, 7, 9], [0, 0, 0]], dtype=np.int32)
    w = np.random.default_rng(6).standard_normal((nt, 2))
    y = np.random.default_rng(7).standard_normal((nt, 4))
    a = oracle.Problem(v, h, so, nt, dt, sponge=2, vref=3000.0, src=src, rec=rec)
    b = oracle.Problem(v, h, so, nt, dt, sponge=2, vref=3000.0, src=src.astype(np.float64),
                       rec=rec.astype(np.float64))
    fa, fb = oracle.forward(a, amp=w), oracle.forward(b, amp=w)
    np.testing.assert_array_equal(fa["rec"], fb["rec"])
    np.testing.assert_array_equal(fa["u"], fb["u"])
    np.testing.assert_array_equal(oracle.adjoint(a, y)["src"], oracle.adjoint(b, y)["src"])


@pytest.mark.parametrize("shape", [(20, 18, 22), (40, 36)])
def test_offgrid_dot_product_fp64(shape):
    nt, so = 40, 8
    v = synth.smooth_velocity(shape, seed=1709, sigma=3.0).numpy().astype(np.float64)
    h = [10.0, 12.0, 9.0][:len(shape)]
    dt = 0.8 * 0.4529 * 9.0 / v.max()
    src = synth.offgrid_points(shape, 3, seed=11)
    rec = synth.offgrid_points(shape, 7, seed=12)
    prob = oracle.Problem(v, h, so, nt, dt, sponge=4, vref=4500.0, src=src, rec=rec)
    rng = np.random.default_rng(3)
    w = rng.standard_normal((nt, 3))
    y = rng.standard_normal((nt, 7))
    d = oracle.forward(prob, amp=w)["rec"]
    fty = oracle.adjoint(prob, y)["src"]
    lhs, rhs = float((d * y).sum()), float((w * fty).sum())
    assert abs(lhs) > 0
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_offgrid_gradient_central_finite_difference_fp64():
    n, nt, so = (20, 18, 22), 50, 8
    v = synth.smooth_velocity(n, seed=1707, sigma=3.0).numpy().astype(np.float64)
    dt = 0.8 * 0.4529 * 10.0 / v.max()
    src = np.array([[9.6, 8.3, 6.45]])
    rec = synth.offgrid_receiver_line(n, 9, depth=6.7)
    w = synth.ricker(nt, dt, 60.0).astype(np.float64)[:, None]
    mk = lambda vv: oracle.Problem(vv, [10.0] * 3, so, nt, dt, sponge=5, vref=4500.0, src=src, rec=rec)
    vtrue = synth.blob_velocity(__import__("torch").from_numpy(v.astype(np.float32))).numpy().astype(np.float64)
    d_obs = oracle.forward(mk(vtrue), amp=w)["rec"]
    J, gv, _ = oracle.gradient(mk(v), w, d_obs)
    dv = np.random.default_rng(8).standard_normal(v.shape) * 10.0
    eps = 1e-3

    def J_at(vv):
        r = oracle.forward(mk(vv), amp=w)["rec"] - d_obs
        return 0.5 * float((r * r).sum())

    fd = (J_at(v + eps * dv) - J_at(v - eps * dv)) / (2 * eps)
    an = float((gv * dv).sum())
    assert abs(fd - an) <= 1e-7 * abs(an)


# ---------------------------------------------------------------- Born modelling
def _born_problem(shape=(20, 18, 22), nt=50, offgrid=False):
    v = synth.smooth_velocity(shape, seed=1711, sigma=3.0).numpy().astype(np.float64)
    dt = 0.8 * 0.4529 * 10.0 / v.max()
    src = np.array([[9.6, 8.3, 6.45]]) if offgrid else synth.centre_source(shape, depth=6)
    rec = synth.offgrid_receiver_line(shape, 9, depth=6.7) if offgrid else synth.receiver_line(shape, 9, depth=6)
    w = synth.ricker(nt, dt, 60.0).astype(np.float64)[:, None]
    mk = lambda vv: oracle.Problem(vv, [10.0] * 3, 8, nt, dt, sponge=5, vref=4500.0, src=src, rec=rec)
    dv = synth.smooth_velocity(shape, seed=1712, sigma=2.0).numpy().astype(np.float64) - 3000.0
    return v, w, dv, mk


@pytest.mark.parametrize("offgrid", [False, True])
def test_born_is_the_derivative_of_the_forward_map(offgrid):
    """Central difference of the traces along dv: agrees with Born to O(eps^2)."""
    v, w, dv, mk = _born_problem(offgrid=offgrid)
    dd = oracle.born(mk(v), w, dv)
    eps = 1e-4
    fd = (oracle.forward(mk(v + eps * dv), amp=w)["rec"] - oracle.forward(mk(v - eps * dv), amp=w)["rec"]) / (2 * eps)
    assert np.linalg.norm(dd) > 0
    assert np.linalg.norm(fd - dd) <= 1e-7 * np.linalg.norm(dd)


def test_born_is_the_transpose_of_the_vector_jacobian_product():
    """<J dv, y> = <dv, J^T y>, J^T y from the adjoint-state gradient (itself pinned)."""
    v, w, dv, mk = _born_problem(offgrid=True)
    prob = mk(v)
    y = np.random.default_rng(14).standard_normal((prob.nt, len(prob.rec)))
    lhs = float((oracle.born(prob, w, dv) * y).sum())
    gv, _ = oracle.vjp(prob, w, y)
    rhs = float((dv * gv).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


# ---------------------------------------------------------------- windowed-sinc points
# Window shape per half-width r: the documented choice (the b that minimises the
# largest error of interpolating cos(k x + phase), k h <= pi/2, on the sampling below).
KAISER_B = {1: 1.3, 2: 2.9, 3: 4.5, 4: 6.3, 5: 7.9, 6: 9.4, 7: 10.9, 8: 12.6}


def ksinc_numpy(f, r, b):
    """1-D Kaiser-windowed sinc weights of the nodes -r+1..r around x = f, from
    numpy's sinc and scipy's I0 (library routines)."""
    from scipy.special import i0
    d = np.arange(-r + 1, r + 1) - f
    return np.sinc(d) * i0(b * np.sqrt(np.clip(1.0 - (d / r) ** 2, 0.0, None))) / i0(b)


def band_error(r, b):
    worst = 0.0
    kh = np.linspace(0.0, np.pi / 2, 31)[:, None]
    for f in np.linspace(0.0, 1.0, 41)[:-1]:
        w = ksinc_numpy(f, r, b)
        k = np.arange(-r + 1, r + 1)[None, :]
        for ph in (0.0, 0.7, 1.9):
            worst = max(worst, float(np.abs(np.cos(kh * k + ph) @ w - np.cos(kh[:, 0] * f + ph)).max()))
    return worst


@pytest.mark.parametrize("r", range(1, 9))
def test_sinc_weights_are_the_kaiser_windowed_sinc(r):
    """1-D weights equal numpy sinc x scipy I0 window (1e-13), and b(r) is a
    local minimum of the band error within +-0.1."""
    for x in (10.0, 10.3, 10.5, 10.999, 17.25):
        idx, w = oracle.point_weights((40,), (x,), sinc=r)
        ref = ksinc_numpy(x - np.floor(x), r, KAISER_B[r])
        nodes = np.floor(x) + np.arange(-r + 1, r + 1)
        keep = np.abs(ref) > 1e-14  # numpy's sinc is ~1e-17, not 0, at the nonzero integers
        np.testing.assert_array_equal(idx, nodes[keep].astype(np.int64))
        np.testing.assert_allclose(w, ref[keep], rtol=1e-13, atol=1e-15)
    b = KAISER_B[r]
    e = band_error(r, b)
    assert e <= band_error(r, b - 0.1) and e <= band_error(r, b + 0.1)


@pytest.mark.parametrize("r", [1, 2, 4, 8])
def test_sinc_at_grid_nodes_is_the_node_itself(r):
    """sinc vanishes at the nonzero integers: a position on a node keeps that
    node alone with weight exactly 1, also next to the boundary."""
    shape = (30, 20, 25)
    for pos in ((5.0, 6.0, 7.0), (0.0, 0.0, 0.0), (29.0, 19.0, 24.0), (1.0, 18.0, 12.0)):
        idx, w = oracle.point_weights(shape, pos, sinc=r)
        flat = (int(pos[0]) * shape[1] + int(pos[1])) * shape[2] + int(pos[2])
        assert idx.tolist() == [flat] and w.tolist() == [1.0]


@pytest.mark.parametrize("r", [2, 4])
def test_sinc_weights_are_separable_mirror_symmetric_and_clipped(r):
    shape = (24, 26, 28)
    pos = np.array([11.3, 12.75, 13.5])
    idx, w = oracle.point_weights(shape, pos, sinc=r)
    per = [oracle.point_weights((n,), (p,), sinc=r) for n, p in zip(shape, pos)]
    full = {}
    for (i0, w0), (i1, w1), (i2, w2) in itertools.product(*[list(zip(*p)) for p in per]):
        full[(i0 * shape[1] + i1) * shape[2] + i2] = w0 * w1 * w2
    assert sorted(full) == sorted(idx.tolist())
    np.testing.assert_allclose([full[i] for i in idx.tolist()], w, rtol=1e-14)
    # mirror: the weights at i + f, read backwards, are those at j + (1 - f)
    for f in (0.2, 0.5, 0.83):
        _, a = oracle.point_weights((40,), (15.0 + f,), sinc=r)
        _, b = oracle.point_weights((40,), (20.0 + (1.0 - f),), sinc=r)
        np.testing.assert_allclose(a, b[::-1], rtol=1e-12, atol=1e-15)  # f and 1 - f round apart
    # near a boundary the nodes outside the grid drop out, the others are unchanged
    ia, wa = oracle.point_weights((40,), (1.3,), sinc=r)
    ib, wb = oracle.point_weights((40,), (21.3,), sinc=r)
    assert ia[0] == 0 and len(ia) == len(ib) - (r - 2)
    np.testing.assert_allclose(wa, wb[len(ib) - len(ia):], rtol=1e-12)


@pytest.mark.parametrize("r,bound", [(4, 3 * 1.2e-3), (8, 3 * 2e-6)])
def test_sinc_receiver_reads_band_limited_waves(r, bound):
    """A 3-D plane wave of at least four points per wavelength on every axis is
    read at a point between nodes to the 1-D band error, compounded per axis."""
    shape = (30, 30, 30)
    X = np.stack(np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij"), -1)
    rng = np.random.default_rng(8)
    for _ in range(6):
        k = rng.uniform(-np.pi / 2, np.pi / 2, 3)
        ph = rng.uniform(0, 2 * np.pi)
        field = np.cos(X @ k + ph).ravel()
        pos = rng.uniform(12.0, 17.0, 3)
        idx, w = oracle.point_weights(shape, pos, sinc=r)
        assert len(idx) == (2 * r) ** 3
        assert abs(float(w @ field[idx]) - np.cos(pos @ k + ph)) <= bound


@pytest.mark.parametrize("shape", [(20, 18, 22), (40, 36)])
def test_sinc_dot_product_and_node_positions_fp64(shape):
    """The windowed-sinc source and receiver operators are exact transposes
    (FP64 dot test), and on grid nodes they reduce to plain grid indices."""
    nt, so, r = 40, 8, 3
    v = synth.smooth_velocity(shape, seed=1709, sigma=3.0).numpy().astype(np.float64)
    h = [10.0, 12.0, 9.0][:len(shape)]
    dt = 0.8 * 0.4529 * 9.0 / v.max()
    src = synth.offgrid_points(shape, 3, seed=21)
    rec = np.concatenate([synth.offgrid_points(shape, 6, seed=22), np.zeros((1, len(shape)))], 0)
    prob = oracle.Problem(v, h, so, nt, dt, sponge=4, vref=4500.0, src=src, rec=rec, src_sinc=r, rec_sinc=r)
    rng = np.random.default_rng(4)
    w = rng.standard_normal((nt, 3))
    y = rng.standard_normal((nt, 7))
    d = oracle.forward(prob, amp=w)["rec"]
    fty = oracle.adjoint(prob, y)["src"]
    lhs, rhs = float((d * y).sum()), float((w * fty).sum())
    assert abs(lhs) > 0
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))
    # differs from multilinear interpolation at the same positions
    lin = oracle.forward(oracle.Problem(v, h, so, nt, dt, sponge=4, vref=4500.0, src=src, rec=rec), amp=w)["rec"]
    assert np.abs(lin - d).max() > 1e-3 * np.abs(d).max()
    nodes = np.round(src).astype(np.int32), np.round(rec).astype(np.int32)
    a = oracle.Problem(v, h, so, nt, dt, sponge=4, vref=4500.0, src=nodes[0], rec=nodes[1])
    b = oracle.Problem(v, h, so, nt, dt, sponge=4, vref=4500.0, src=nodes[0].astype(np.float64),
                       rec=nodes[1].astype(np.float64), src_sinc=r, rec_sinc=r)
    np.testing.assert_array_equal(oracle.forward(a, amp=w)["rec"], oracle.forward(b, amp=w)["rec"])
