"""CPU oracle of the iterative solvers (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps liboracle.so (plain C, oracle.c) with numpy
arrays and shares no code with the GPU library.

Every function returns new arrays and leaves its inputs untouched.  The
``dtype`` argument picks the float32 or the float64 instantiation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = C.CDLL(_build.LIB)
        _setup(_lib)
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _setup(L):
    L.or_abi_version.restype = C.c_int
    for sfx in ("f32", "f64"):
        f = getattr(L, "or_heat2d_" + sfx)
        f.argtypes = [C.c_void_p, C.c_void_p, C.c_long, C.c_long] + [C.c_double] * 5 + [C.c_long, C.c_void_p]
        f.restype = C.c_int
        f = getattr(L, "or_heat3d_" + sfx)
        f.argtypes = [C.c_void_p, C.c_void_p, C.c_long, C.c_long, C.c_long] + [C.c_double] * 5 + [C.c_long, C.c_void_p]
        f.restype = C.c_int
        f = getattr(L, "or_skeleton_" + sfx)
        f.argtypes = [C.c_void_p, C.c_long, C.c_void_p, C.c_void_p, C.c_int, C.c_long, C.c_void_p]
        f.restype = C.c_int
        f = getattr(L, "or_fdtd_" + sfx)
        f.argtypes = [C.c_void_p] * 6 + [C.c_long, C.c_double, C.c_void_p, C.c_void_p, C.c_long, C.c_long, C.c_void_p]
        f.restype = C.c_int
    L.or_fdtd_pulse.argtypes = [C.c_double, C.c_double, C.c_long, C.c_void_p, C.c_void_p]
    L.or_fdtd_pulse.restype = None
    L.or_set_threads.argtypes = [C.c_int]
    L.or_set_threads.restype = None
    L.or_get_threads.restype = C.c_int


def set_threads(n):
    """Threads of the oracle's loops over independent rows, planes and
    elements (the results are the same bits for every count)."""
    lib().or_set_threads(int(n))


def get_threads():
    return int(lib().or_get_threads())


class threads:
    """Context manager: run the oracle with n threads, then restore."""

    def __init__(self, n):
        self.n = int(n)

    def __enter__(self):
        self.old = get_threads()
        set_threads(self.n)
        return self

    def __exit__(self, *exc):
        set_threads(self.old)
        return False


def _sfx(dtype):
    dt = np.dtype(dtype)
    if dt == np.float32:
        return "f32", np.float32
    if dt == np.float64:
        return "f64", np.float64
    raise ValueError("dtype must be float32 or float64")


HEAT_COEFFS = dict(c=1e-3, Rx=1.0, Ry=1.0, Rz=10.0, Tamb=300.0)


def heat2d(T0, P, nsteps, c=1e-3, Rx=1.0, Ry=1.0, Rz=10.0, Tamb=300.0, dtype=np.float64):
    """T after nsteps explicit 2D thermal steps (clamped neighbours)."""
    sfx, dt = _sfx(dtype)
    T0 = np.ascontiguousarray(T0, dtype=dt)
    P = np.ascontiguousarray(P, dtype=dt)
    ny, nx = T0.shape
    assert P.shape == (ny, nx)
    out = np.empty_like(T0)
    rc = getattr(lib(), "or_heat2d_" + sfx)(_ptr(T0), _ptr(P), ny, nx, c, Rx, Ry, Rz, Tamb, int(nsteps), _ptr(out))
    if rc:
        raise MemoryError("oracle heat2d")
    return out


def heat3d(T0, P, nsteps, c=1e-3, Rx=1.0, Ry=1.0, Rz=10.0, Tamb=300.0, dtype=np.float64):
    """T after nsteps layered 3D steps.  P is dense [nz][ny][nx] or one
    [ny][nx] plane (then layer 0 gets it and the other layers get zero)."""
    sfx, dt = _sfx(dtype)
    T0 = np.ascontiguousarray(T0, dtype=dt)
    nz, ny, nx = T0.shape
    P = np.asarray(P, dtype=dt)
    if P.shape == (ny, nx):
        Pd = np.zeros_like(T0)
        Pd[0] = P
        P = Pd
    P = np.ascontiguousarray(P)
    assert P.shape == T0.shape
    out = np.empty_like(T0)
    rc = getattr(lib(), "or_heat3d_" + sfx)(_ptr(T0), _ptr(P), nz, ny, nx, c, Rx, Ry, Rz, Tamb, int(nsteps), _ptr(out))
    if rc:
        raise MemoryError("oracle heat3d")
    return out


def skeleton(x0, a, b, iters, dtype=np.float64):
    """x after iters iterations of the chain x <- a_k*x + b_k, k = 1..K."""
    sfx, dt = _sfx(dtype)
    x0 = np.ascontiguousarray(x0, dtype=dt)
    a = np.ascontiguousarray(a, dtype=dt)
    b = np.ascontiguousarray(b, dtype=dt)
    assert a.shape == b.shape and a.ndim == 1
    out = np.empty_like(x0)
    getattr(lib(), "or_skeleton_" + sfx)(_ptr(x0), x0.size, _ptr(a), _ptr(b), a.size, int(iters), _ptr(out))
    return out


def fdtd_pulse(count, width=20.0, delay=80.0):
    """(g64, g32): soft-source amplitudes exp(-((n-delay)/width)^2), n < count."""
    g64 = np.empty(count, np.float64)
    g32 = np.empty(count, np.float32)
    lib().or_fdtd_pulse(float(delay), float(width), int(count), _ptr(g64), _ptr(g32))
    return g64, g32


FDTD_FIELDS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def fdtd_zero_fields(N, dtype=np.float64):
    M = N + 1
    return {k: np.zeros((M, M, M), dtype=dtype) for k in FDTD_FIELDS}


def fdtd(fields, N, nsteps, dt=0.5, src=None, g=None, n_start=0, dtype=np.float64):
    """Advance the Yee fields (dict of (N+1)^3 arrays indexed [k][j][i]) by
    nsteps steps from absolute step n_start.  Returns (new_fields, probe).
    g: per-absolute-step source amplitudes (length >= n_start+nsteps) or None.
    """
    sfx, dtp = _sfx(dtype)
    M = N + 1
    f = {k: np.ascontiguousarray(np.array(fields[k], dtype=dtp, copy=True)) for k in FDTD_FIELDS}
    for k in FDTD_FIELDS:
        assert f[k].shape == (M, M, M)
    probe = np.zeros(max(nsteps, 1), dtype=dtp)
    src_arr = np.asarray(src if src is not None else (0, 0, 0), dtype=np.int64)
    gp = None
    if g is not None:
        g = np.ascontiguousarray(g, dtype=dtp)
        assert g.size >= n_start + nsteps
        gp = _ptr(g)
    getattr(lib(), "or_fdtd_" + sfx)(*[_ptr(f[k]) for k in FDTD_FIELDS], N, float(dt),
                                     _ptr(src_arr), gp, int(n_start), int(nsteps),
                                     _ptr(probe) if src is not None else None)
    return f, probe[:nsteps]


# ---------------------------------------------------------------------------
# Learned k-step surrogate (surrogate.c): forward, loss gradient, Adam.
# ---------------------------------------------------------------------------
SG_NW = 19393


def _setup_sg(L):
    L.or_sg_nweights.restype = C.c_int
    L.or_bf16_round.argtypes = [C.c_double]
    L.or_bf16_round.restype = C.c_double
    L.or_sg_conv3x3.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_long, C.c_long,
                                C.c_void_p]
    L.or_sg_conv3x3.restype = None
    L.or_sg_conv3x3_adjoint_input.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_long, C.c_long,
                                              C.c_void_p]
    L.or_sg_conv3x3_adjoint_input.restype = None
    L.or_sg_conv3x3_adjoint_weights.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_long,
                                                C.c_long, C.c_void_p, C.c_void_p]
    L.or_sg_conv3x3_adjoint_weights.restype = None
    L.or_bf16_round_n.argtypes = [C.c_void_p, C.c_long, C.c_void_p]
    L.or_bf16_round_n.restype = None
    L.or_sg_gelu.argtypes = [C.c_void_p, C.c_long, C.c_void_p, C.c_void_p]
    L.or_sg_gelu.restype = None
    L.or_sg_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_long, C.c_long, C.c_int, C.c_void_p]
    L.or_sg_forward.restype = C.c_int
    L.or_sg_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_long, C.c_long,
                                  C.c_double, C.c_int, C.c_void_p, C.c_void_p]
    L.or_sg_loss_grad.restype = C.c_int
    L.or_adam.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_long, C.c_long, C.c_double,
                          C.c_double, C.c_double, C.c_double]
    L.or_adam.restype = None


_sg_ready = False


def _sg():
    global _sg_ready
    L = lib()
    if not _sg_ready:
        _setup_sg(L)
        _sg_ready = True
    return L


def bf16_round(v):
    """Round each value to the nearest bf16 (ties to even), in float64."""
    L = _sg()
    a = np.asarray(v, dtype=np.float64)
    if not a.ndim:
        return L.or_bf16_round(float(a))
    a = np.ascontiguousarray(a)
    out = np.empty_like(a)
    L.or_bf16_round_n(_ptr(a), a.size, _ptr(out))
    return out


def sg_conv3x3(W, b, x):
    """One 3x3 convolution with replicate padding: W[co][ci][3][3], b[co]
    (or None), x[ci][H][W] -> [co][H][W], float64."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    co, ci = W.shape[:2]
    _, H, Wd = x.shape
    out = np.empty((co, H, Wd), np.float64)
    bp = None
    if b is not None:
        b = np.ascontiguousarray(b, dtype=np.float64)
        bp = _ptr(b)
    _sg().or_sg_conv3x3(_ptr(W), bp, _ptr(x), ci, co, H, Wd, _ptr(out))
    return out


def sg_gelu(z):
    """(GELU(z), GELU'(z)) elementwise, exact erf form, float64."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = np.empty_like(z)
    dout = np.empty_like(z)
    _sg().or_sg_gelu(_ptr(z), z.size, _ptr(out), _ptr(dout))
    return out, dout


def sg_conv3x3_adjoint_input(W, g):
    """Adjoint of sg_conv3x3 in its input: W[co][ci][3][3], g[co][H][W] ->
    din[ci][H][W] = sum over (co, tap, pixel p) with clamp(p + tap) = q of
    W[co][ci][tap] g[co][p], float64."""
    W = np.ascontiguousarray(W, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    co, ci = W.shape[:2]
    assert g.shape[0] == co
    _, H, Wd = g.shape
    out = np.empty((ci, H, Wd), np.float64)
    _sg().or_sg_conv3x3_adjoint_input(_ptr(W), _ptr(g), ci, co, H, Wd, _ptr(out))
    return out


def sg_conv3x3_adjoint_weights(x, g, gb=None):
    """Adjoint of sg_conv3x3 in its weights and bias: x[ci][H][W] (the
    layer input), g[co][H][W] (gradient of its output; gb, default g, is
    the one summed into the bias) -> (dW[co][ci][3][3], db[co]), float64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    gb = g if gb is None else np.ascontiguousarray(gb, dtype=np.float64)
    ci, H, Wd = x.shape
    co = g.shape[0]
    assert g.shape == (co, H, Wd) and gb.shape == g.shape
    dW = np.zeros((co, ci, 3, 3), np.float64)
    db = np.zeros(co, np.float64)
    _sg().or_sg_conv3x3_adjoint_weights(_ptr(x), _ptr(g), _ptr(gb), ci, co, H, Wd, _ptr(dW), _ptr(db))
    return dW, db


def sg_forward(w, T0, P, round_bf16=True):
    """Network output y (normalised increment) for one field, float64."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert w.size == SG_NW
    T0 = np.ascontiguousarray(T0, dtype=np.float32)
    P = np.ascontiguousarray(P, dtype=np.float32)
    H, Wd = T0.shape
    y = np.empty((H, Wd), np.float64)
    if _sg().or_sg_forward(_ptr(w), _ptr(T0), _ptr(P), H, Wd, int(round_bf16), _ptr(y)):
        raise MemoryError("oracle sg_forward")
    return y


def sg_loss_grad(w, T0, P, target, norm=None, round_bf16=True):
    """(loss, grad) of sum (y - target)^2 / norm for one field (norm
    defaults to its pixel count)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    T0 = np.ascontiguousarray(T0, dtype=np.float32)
    P = np.ascontiguousarray(P, dtype=np.float32)
    target = np.ascontiguousarray(target, dtype=np.float64)
    H, Wd = T0.shape
    norm = float(H * Wd if norm is None else norm)
    g = np.zeros(SG_NW, np.float64)
    loss = np.zeros(1, np.float64)
    if _sg().or_sg_loss_grad(_ptr(w), _ptr(T0), _ptr(P), _ptr(target), H, Wd, norm, int(round_bf16), _ptr(g),
                             _ptr(loss)):
        raise MemoryError("oracle sg_loss_grad")
    return float(loss[0]), g


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays w, m, v."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    _sg().or_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.size, int(step), lr, b1, b2, eps)
