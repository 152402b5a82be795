"""FP64 CPU oracle for the acoustic finite-difference sweep -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``fdoracle.c`` (plain C, FP64,
an untiled loop nest with one OpenMP parallel-for on the outer axis) with
ctypes and shares no code with the HIP library: it does not import
``paper_1707_02347_amd`` and that package does not import it.

Every array crossing this wrapper is a float64 numpy array in C order with the
last axis contiguous.  The functions follow the paper's damped leapfrog update
(Sec. 6.3.1, Fig. "acoustic_devito") and the readings stated in ``fdoracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdoracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile ``fdoracle.c`` into ``liboracle.so`` with gcc (FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("so", C.c_int32),
        ("n", C.c_int64 * 3),
        ("h", C.c_double * 3),
        ("nt", C.c_int64),
        ("dt", C.c_double),
        ("sponge", C.c_int32),
        ("pad0", C.c_int32),
        ("vref", C.c_double),
        ("v", C.POINTER(C.c_double)),
        ("ns", C.c_int32),
        ("nr", C.c_int32),
        ("src", C.POINTER(C.c_int32)),
        ("rec", C.POINTER(C.c_int32)),
        ("spos", C.POINTER(C.c_double)),
        ("rpos", C.POINTER(C.c_double)),
        ("ssinc", C.c_int32),
        ("rsinc", C.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        D = C.POINTER(C.c_double)
        lib.or_weights.argtypes = [C.c_int, D]
        lib.or_laplacian.argtypes = [C.c_int, C.POINTER(C.c_int64), D, C.c_int, D, D]
        lib.or_damp.argtypes = [P, D]
        lib.or_forward.argtypes = [P, D, D, D, D, D]
        lib.or_adjoint.argtypes = [P, D, D, D]
        lib.or_vjp.argtypes = [P, D, D, D, D]
        lib.or_gradient.argtypes = [P, D, D, D, D, D]
        lib.or_born.argtypes = [P, D, D, D]
        lib.or_point_weights.argtypes = [P, D, C.c_int, C.POINTER(C.c_int64), D, C.c_int]
        for f in ("or_weights", "or_laplacian", "or_damp", "or_forward", "or_adjoint",
                  "or_vjp", "or_gradient", "or_born", "or_point_weights"):
            getattr(lib, f).restype = C.c_int
        _lib = lib
    return _lib


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


class Problem:
    """Problem description mirrored into the C struct (keeps its arrays alive)."""

    def __init__(self, v, h, so, nt, dt, sponge=0, vref=1500.0, src=None, rec=None, src_sinc=0, rec_sinc=0):
        v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
        self.v = v
        self.shape = v.shape
        self.ndim = v.ndim
        hh = np.broadcast_to(np.asarray(h, dtype=np.float64), (self.ndim,))
        self.h = tuple(float(x) for x in hh)
        self.so, self.nt, self.dt = int(so), int(nt), float(dt)
        self.sponge, self.vref = int(sponge), float(vref)
        # integer arrays are grid indices; floating-point arrays are positions in
        # grid-index units (off the grid: multilinear interpolation, or with
        # src_sinc / rec_sinc = r > 0 Kaiser-windowed sinc of half-width r)
        self.src, self.spos = self._points(src)
        self.rec, self.rpos = self._points(rec)
        s = _Problem()
        s.ndim, s.so = self.ndim, self.so
        for a in range(3):
            s.n[a] = self.shape[a] if a < self.ndim else 1
            s.h[a] = self.h[a] if a < self.ndim else 1.0
        s.nt, s.dt, s.sponge, s.vref = self.nt, self.dt, self.sponge, self.vref
        s.v = _dptr(self.v)
        s.ns, s.nr = len(self.src), len(self.rec)
        s.src = self.src.ctypes.data_as(C.POINTER(C.c_int32))
        s.rec = self.rec.ctypes.data_as(C.POINTER(C.c_int32))
        s.spos = None if self.spos is None else _dptr(self.spos)
        s.rpos = None if self.rpos is None else _dptr(self.rpos)
        s.ssinc, s.rsinc = int(src_sinc), int(rec_sinc)
        self._s = s

    def _points(self, pts):
        if pts is None:
            return np.zeros((0, self.ndim), dtype=np.int32), None
        a = np.asarray(pts)
        if np.issubdtype(a.dtype, np.floating):
            pos = np.ascontiguousarray(a, dtype=np.float64).reshape(-1, self.ndim)
            return np.zeros((len(pos), self.ndim), dtype=np.int32), pos
        return np.ascontiguousarray(a, dtype=np.int32).reshape(-1, self.ndim), None

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def ref(self):
        return C.byref(self._s)


def weights(so: int) -> np.ndarray:
    """Closed-form central second-derivative weights c_0..c_M for order so (FP64)."""
    c = np.zeros(so // 2 + 1, dtype=np.float64)
    _check(_load().or_weights(int(so), _dptr(c)), "weights")
    return c


def laplacian(u, h, so) -> np.ndarray:
    """Star Laplacian L_h u with u = 0 outside the grid (FP64)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = (C.c_int64 * 3)(*[int(x) for x in u.shape])
    hh = np.ascontiguousarray(np.broadcast_to(np.asarray(h, dtype=np.float64), (u.ndim,)))
    out = np.empty_like(u)
    _check(_load().or_laplacian(u.ndim, n, _dptr(hh), int(so), _dptr(u), _dptr(out)), "laplacian")
    return out


def damp(prob: Problem) -> np.ndarray:
    out = np.empty(prob.shape, dtype=np.float64)
    _check(_load().or_damp(prob.ref(), _dptr(out)), "damp")
    return out


def forward(prob: Problem, amp=None, u0=None, um1=None, history=False):
    """Forward sweep. Returns dict with u (u^nt), u_prev (u^{nt-1}), rec [nt][nr], hist."""
    N = prob.npts
    uc = np.zeros(prob.shape) if u0 is None else np.array(u0, dtype=np.float64, order="C", copy=True)
    up = np.zeros(prob.shape) if um1 is None else np.array(um1, dtype=np.float64, order="C", copy=True)
    a = None
    if amp is not None and len(prob.src):
        a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64).reshape(prob.nt, len(prob.src)))
    rec = np.zeros((prob.nt, len(prob.rec)), dtype=np.float64)
    hist = np.zeros((prob.nt + 2,) + prob.shape) if history else None
    rc = _load().or_forward(prob.ref(), _dptr(a), _dptr(rec), _dptr(uc), _dptr(up), _dptr(hist))
    _check(rc, "forward")
    assert uc.size == N
    return {"u": uc, "u_prev": up, "rec": rec, "hist": hist}


def adjoint(prob: Problem, y, history=False):
    """Adjoint sweep: y [nt][nr] injected at receivers -> [nt][ns] at sources (F^T y)."""
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(prob.nt, len(prob.rec)))
    out = np.zeros((prob.nt, len(prob.src)), dtype=np.float64)
    hist = np.zeros((prob.nt + 2,) + prob.shape) if history else None
    _check(_load().or_adjoint(prob.ref(), _dptr(y), _dptr(out), _dptr(hist)), "adjoint")
    return {"src": out, "hist": hist}


def vjp(prob: Problem, amp, y):
    """(grad_v, grad_m) of <d(v), y> for trace cotangent y, zero initial state."""
    a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64).reshape(prob.nt, len(prob.src)))
    y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(prob.nt, len(prob.rec)))
    gv = np.zeros(prob.shape)
    gm = np.zeros(prob.shape)
    _check(_load().or_vjp(prob.ref(), _dptr(a), _dptr(y), _dptr(gv), _dptr(gm)), "vjp")
    return gv, gm


def born(prob: Problem, amp, dv):
    """Born (linearised) traces [nt][nr] for a velocity perturbation dv, zero initial state."""
    a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64).reshape(prob.nt, len(prob.src)))
    dv = np.ascontiguousarray(np.asarray(dv, dtype=np.float64).reshape(prob.shape))
    dd = np.zeros((prob.nt, len(prob.rec)), dtype=np.float64)
    _check(_load().or_born(prob.ref(), _dptr(a), _dptr(dv), _dptr(dd)), "born")
    return dd


def gradient(prob: Problem, amp, d_obs):
    """(misfit J, grad_v, grad_m) for J = 1/2 sum (d - d_obs)^2."""
    a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64).reshape(prob.nt, len(prob.src)))
    d = np.ascontiguousarray(np.asarray(d_obs, dtype=np.float64).reshape(prob.nt, len(prob.rec)))
    gv = np.zeros(prob.shape)
    gm = np.zeros(prob.shape)
    J = C.c_double(0.0)
    _check(_load().or_gradient(prob.ref(), _dptr(a), _dptr(d), _dptr(gv), _dptr(gm), C.byref(J)), "gradient")
    return float(J.value), gv, gm


def point_weights(shape, pos, sinc=0):
    """Flat node indices and weights of one point at position ``pos`` (grid-index
    units) on a grid of ``shape``: multilinear (sinc=0) or Kaiser-windowed sinc
    of half-width ``sinc``."""
    nd = len(shape)
    prob = Problem(np.ones(shape), [1.0] * nd, 2, 0, 1.0)
    cap = 4096
    idx = np.zeros(cap, dtype=np.int64)
    w = np.zeros(cap, dtype=np.float64)
    p = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(nd))
    n = _load().or_point_weights(prob.ref(), _dptr(p), int(sinc), idx.ctypes.data_as(C.POINTER(C.c_int64)),
                                 _dptr(w), cap)
    if n < 0:
        raise ValueError(f"oracle point_weights failed with code {n}")
    return idx[:n].copy(), w[:n].copy()
