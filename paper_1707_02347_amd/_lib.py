"""ctypes binding of libfdwave.so (include/fdwave.h).

The functions named ``fd_*`` mirror the C entry points one to one and only
marshal arguments; every step of the sweep runs in the HIP kernels of the
library.  There is no fallback: if the shared library is missing or does not
load, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_PKG, "libfdwave.so")

FD_OK = 0
FD_EINVAL = -1
FD_ECFL = -2
FD_EDOM = -3
FD_EWORKSPACE = -4
FD_ENOMEM = -5
FD_EHIP = -6
FD_ENONFINITE = -7
FD_EUNSUPPORTED = -8
FD_ESCRATCH = -9
FD_ESYNC = -10

FD_NOALLOC_SCRATCH_BYTES = 64 << 20

FD_VARIANT_AUTO = 0
FD_VARIANT_NAIVE = 1
FD_VARIANT_STREAM = 2
FD_VARIANT_TBLOCK = 3
FD_VARIANT_SPLIT = 4
FD_VARIANT_WAVE = 5

FD_FLAG_NO_CFL_CHECK = 1
FD_FLAG_CHECK_FINITE = 2
FD_FLAG_NO_XCD_REMAP = 4
FD_FLAG_NO_X_ALTERNATE = 8
FD_FLAG_LOADS_STREAM = 16
FD_FLAG_LOADS_KEEP = 32

FD_OP_FORWARD = 0
FD_OP_ADJOINT = 1
FD_OP_GRADIENT = 2
FD_OP_VJP = 3
FD_OP_BORN = 4

FD_BATCH_GRAPH = 1


class fd_grid(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("space_order", C.c_int32),
        ("n", C.c_int64 * 3),
        ("h", C.c_double * 3),
        ("sponge", C.c_int32),
        ("reserved", C.c_int32),
        ("sponge_vref", C.c_double),
    ]


class fd_time(C.Structure):
    _fields_ = [("nt", C.c_int64), ("dt", C.c_double)]


class fd_points(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("interp", C.c_int32),
        ("idx", C.POINTER(C.c_int32)),
        ("amp", C.c_void_p),
        ("pos", C.POINTER(C.c_double)),
    ]


class fd_options(C.Structure):
    _fields_ = [
        ("variant", C.c_int32),
        ("tile", C.c_int32 * 3),
        ("tblock", C.c_int32),
        ("ckpt_every", C.c_int32),
        ("flags", C.c_uint32),
        ("reserved", C.c_int32),
    ]


class fd_shot(C.Structure):
    _fields_ = [
        ("grid", fd_grid),
        ("time", fd_time),
        ("v", C.c_void_p),
        ("src", fd_points),
        ("rec", fd_points),
        ("rec_out", C.c_void_p),
        ("grad_v", C.c_void_p),
        ("misfit", C.c_double),
        ("opts", fd_options),
    ]


class FdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


_lib = None

SYMBOLS = {
    "fd_workspace_size": (C.c_size_t, [C.POINTER(fd_grid), C.POINTER(fd_time), C.POINTER(fd_points),
                                       C.POINTER(fd_points), C.POINTER(fd_options), C.c_int]),
    "fd_gradient_storage": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.POINTER(fd_points),
                                      C.POINTER(fd_points), C.c_int, C.c_size_t, C.POINTER(fd_options),
                                      C.POINTER(C.c_size_t)]),
    "fd_forward": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.c_void_p, C.POINTER(fd_points),
                             C.POINTER(fd_points), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                             C.POINTER(fd_options), C.c_void_p]),
    "fd_forward_noalloc": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.c_void_p, C.POINTER(fd_points),
                                     C.POINTER(fd_points), C.c_void_p, C.c_void_p, C.POINTER(fd_options),
                                     C.c_void_p]),
    "fd_adjoint": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.c_void_p, C.POINTER(fd_points),
                             C.POINTER(fd_points), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                             C.POINTER(fd_options), C.c_void_p]),
    "fd_gradient": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.c_void_p, C.POINTER(fd_points),
                              C.POINTER(fd_points), C.c_void_p, C.POINTER(C.c_double), C.c_void_p,
                              C.c_void_p, C.c_size_t, C.POINTER(fd_options), C.c_void_p]),
    "fd_vjp": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.c_void_p, C.POINTER(fd_points),
                         C.POINTER(fd_points), C.c_void_p, C.c_void_p, C.c_size_t,
                         C.POINTER(fd_options), C.c_void_p]),
    "fd_born": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.c_void_p, C.c_void_p, C.POINTER(fd_points),
                          C.POINTER(fd_points), C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(fd_options),
                          C.c_void_p]),
    "fd_autotune": (C.c_int, [C.POINTER(fd_grid), C.POINTER(fd_time), C.POINTER(fd_options), C.c_void_p,
                              C.c_size_t, C.c_void_p]),
    "fd_batch_workspace_size": (C.c_size_t, [C.c_int, C.POINTER(fd_shot), C.c_int]),
    "fd_forward_batch": (C.c_int, [C.c_int, C.POINTER(fd_shot), C.c_void_p, C.c_size_t, C.c_uint32,
                                   C.c_void_p]),
    "fd_gradient_batch": (C.c_int, [C.c_int, C.POINTER(fd_shot), C.c_void_p, C.c_size_t, C.c_uint32,
                                    C.c_void_p]),
    "fd_batch_autotune": (C.c_int, [C.c_int, C.POINTER(fd_shot), C.c_void_p, C.c_size_t, C.c_void_p]),
    "fd_strerror": (C.c_char_p, [C.c_int]),
    "fd_version": (C.c_int, []),
    "fd_last_config": (C.c_int, [C.POINTER(fd_options)]),
}


def load():
    """Load libfdwave.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = C.CDLL(LIBPATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().fd_strerror(int(code)).decode()


def _check(rc: int, where: str):
    if rc != FD_OK:
        raise FdError(rc, where)


# ------------------------------------------------------------------ thin mirrors of the C ABI
def fd_workspace_size(grid, time, src, rec, opts, op):
    return load().fd_workspace_size(grid, time, src, rec, opts, op)


def fd_gradient_storage(grid, time, src, rec, op, budget, inout, ws_bytes):
    return load().fd_gradient_storage(grid, time, src, rec, op, budget, inout, ws_bytes)


def fd_forward(grid, time, v, src, rec, rec_out, u_state, workspace, ws_bytes, opts, stream):
    return load().fd_forward(grid, time, v, src, rec, rec_out, u_state, workspace, ws_bytes, opts, stream)


def fd_forward_noalloc(grid, time, v, src, rec, rec_out, u_state, opts, stream):
    return load().fd_forward_noalloc(grid, time, v, src, rec, rec_out, u_state, opts, stream)


def fd_adjoint(grid, time, v, src, rec, src_out, lam_state, workspace, ws_bytes, opts, stream):
    return load().fd_adjoint(grid, time, v, src, rec, src_out, lam_state, workspace, ws_bytes, opts, stream)


def fd_gradient(grid, time, v, src, rec, grad_v, misfit, residual, workspace, ws_bytes, opts, stream):
    return load().fd_gradient(grid, time, v, src, rec, grad_v, misfit, residual, workspace, ws_bytes, opts,
                              stream)


def fd_vjp(grid, time, v, src, rec, grad_v, workspace, ws_bytes, opts, stream):
    return load().fd_vjp(grid, time, v, src, rec, grad_v, workspace, ws_bytes, opts, stream)


def fd_born(grid, time, v, dv, src, rec, rec_out, workspace, ws_bytes, opts, stream):
    return load().fd_born(grid, time, v, dv, src, rec, rec_out, workspace, ws_bytes, opts, stream)


def fd_autotune(grid, time, inout, workspace, ws_bytes, stream):
    return load().fd_autotune(grid, time, inout, workspace, ws_bytes, stream)


def fd_batch_workspace_size(nshots, shots, op):
    return load().fd_batch_workspace_size(nshots, shots, op)


def fd_forward_batch(nshots, shots, workspace, ws_bytes, flags, stream):
    return load().fd_forward_batch(nshots, shots, workspace, ws_bytes, flags, stream)


def fd_gradient_batch(nshots, shots, workspace, ws_bytes, flags, stream):
    return load().fd_gradient_batch(nshots, shots, workspace, ws_bytes, flags, stream)


def fd_batch_autotune(nshots, shots, workspace, ws_bytes, stream):
    return load().fd_batch_autotune(nshots, shots, workspace, ws_bytes, stream)


def fd_version():
    return load().fd_version()


def fd_last_config():
    o = fd_options()
    _check(load().fd_last_config(C.byref(o)), "fd_last_config")
    return {"variant": o.variant, "tile": tuple(o.tile), "tblock": o.tblock}


# ------------------------------------------------------------------ descriptor builders
def make_grid(shape, h, so, sponge=0, vref=1500.0):
    g = fd_grid()
    g.ndim = len(shape)
    g.space_order = int(so)
    hh = np.broadcast_to(np.asarray(h, dtype=np.float64), (len(shape),))
    for a in range(3):
        g.n[a] = int(shape[a]) if a < len(shape) else 0
        g.h[a] = float(hh[a]) if a < len(shape) else 0.0
    g.sponge = int(sponge)
    g.reserved = 0
    g.sponge_vref = float(vref)
    return g


def make_time(nt, dt):
    t = fd_time()
    t.nt = int(nt)
    t.dt = float(dt)
    return t


class Sinc:
    """Positions (grid-index units) that act through Kaiser-windowed sinc
    interpolation of half-width r (2r nodes per axis) instead of multilinear."""

    def __init__(self, pos, r=4):
        self.pos = np.asarray(pos, dtype=np.float64)
        self.r = int(r)


class Points:
    """fd_points with its host array kept alive: integer arrays are grid
    indices, floating-point arrays positions in grid-index units (points between
    nodes, multilinear interpolation), a Sinc positions with windowed-sinc
    interpolation."""

    def __init__(self, idx=None, amp=None, ndim=3):
        self.pos = None
        interp = 0
        if isinstance(idx, Sinc):
            idx, interp = idx.pos, idx.r
        if idx is None:
            self.idx = np.zeros((0, ndim), dtype=np.int32)
        elif np.issubdtype(np.asarray(idx).dtype, np.floating):
            self.pos = np.ascontiguousarray(np.asarray(idx, dtype=np.float64).reshape(-1, ndim))
            self.idx = np.zeros((len(self.pos), ndim), dtype=np.int32)
        else:
            self.idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1, ndim))
        self.amp = amp
        s = fd_points()
        s.n = len(self.idx)
        s.interp = interp
        if self.pos is not None:
            s.idx = None
            s.pos = self.pos.ctypes.data_as(C.POINTER(C.c_double)) if len(self.pos) else None
        else:
            s.idx = self.idx.ctypes.data_as(C.POINTER(C.c_int32)) if len(self.idx) else None
            s.pos = None
        s.amp = _ptr(amp)
        self.s = s

    @property
    def n(self):
        return int(self.s.n)


def make_options(variant=0, tile=(0, 0, 0), tblock=0, ckpt_every=0, flags=0):
    o = fd_options()
    o.variant = int(variant)
    for i in range(3):
        o.tile[i] = int(tile[i])
    o.tblock = int(tblock)
    o.ckpt_every = int(ckpt_every)
    o.flags = int(flags)
    o.reserved = 0
    return o


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(dev=None):
    import torch

    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
