"""Python binding of libkbatch (include/kb.h): iteration-batched graph
execution of iterative solvers on one MI355X.

Argument marshalling only: every step of the solvers and of the batching
method runs in the HIP library.  PyTorch provides the device workspace and
the stream.  The library must be built (``python -m paper_2501_09398_amd.build``
or ``__graft_entry__.build()``); importing the binding without it raises.

torch is imported before the library is loaded so that both use the one
HIP runtime that torch brings (the library's libamdhip64 dependency then
resolves to the copy already in the process).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkbatch.so")

# problems
HEAT2D, HEAT3D, SKELETON, FDTD3D, HEAT2D_MULTI, HEAT2D_SURROGATE = 1, 2, 3, 4, 5, 6
# fields
F_T, F_P, F_X, F_A, F_B = 1, 2, 3, 4, 5
F_EX, F_EY, F_EZ, F_HX, F_HY, F_HZ, F_PROBE, F_STEP = 10, 11, 12, 13, 14, 15, 16, 17
F_W, F_SGSTATS, F_RESID = 20, 21, 22
F_REDLOG, F_REDCOUNT = 23, 24
# the surrogate's training tape (read only)
F_SG_X, F_SG_A1, F_SG_A2, F_SG_A3, F_SG_Z1, F_SG_Z2, F_SG_Z3 = 30, 31, 32, 33, 34, 35, 36
F_SG_Y, F_SG_TGT, F_SG_G4, F_SG_G1, F_SG_G2, F_SG_G3, F_SG_GRAD = 37, 38, 39, 40, 41, 42, 43
SG_NW = 19393
FDTD_FIELDS = {"Ex": F_EX, "Ey": F_EY, "Ez": F_EZ, "Hx": F_HX, "Hy": F_HY, "Hz": F_HZ}
# options
OPT_BUILDER, OPT_TILE, OPT_TDEPTH, OPT_GRAPH_CACHE, OPT_MAX_NODES, OPT_REDUCE_EVERY = 1, 2, 3, 4, 5, 6
OPT_GRAPH_UPDATE = 7
OPT_PERSISTENT = 8
OPT_SPIN_LIMIT = 9
# status
OK, EINVAL, ENOMEM, EHIP, ESTATE, WFALLBACK = 0, -1, -2, -3, -4, 1


class KBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libkbatch error {code}: {msg}")
        self.code = code


class Timing(C.Structure):
    _fields_ = [("t_create_s", C.c_double), ("t_exec_s", C.c_double),
                ("n_graph_launches", C.c_int64), ("n_nodes", C.c_int64),
                ("n_peeled", C.c_int64), ("n_kernel_launches", C.c_int64),
                ("n_graphs_built", C.c_int64), ("graph_mem_bytes", C.c_int64),
                ("t_update_s", C.c_double), ("n_graphs_updated", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded libkbatch.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2501_09398_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
        L.kb_workspace_bytes.argtypes = [C.c_int, i64p, C.c_int]
        L.kb_workspace_bytes.restype = C.c_size_t
        L.kb_create.argtypes = [C.c_int, i64p, C.c_int, C.POINTER(C.c_double), C.c_int, C.c_uint64,
                                vp, C.c_size_t, vp, C.POINTER(vp)]
        L.kb_create.restype = C.c_int
        L.kb_set_option.argtypes = [vp, C.c_int, C.c_int64]
        L.kb_set_option.restype = C.c_int
        L.kb_run.argtypes = [vp, C.c_int64, C.c_int64]
        L.kb_run.restype = C.c_int
        L.kb_reduce_noalloc.argtypes = [C.POINTER(vp), C.c_int, C.c_int64, C.c_int, vp, vp]
        L.kb_reduce_noalloc.restype = C.c_int
        L.kb_read.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.kb_read.restype = C.c_int
        L.kb_write.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.kb_write.restype = C.c_int
        L.kb_reduce.argtypes = [vp, C.POINTER(C.c_double), C.c_int]
        L.kb_reduce.restype = C.c_int
        L.kb_last_timing.argtypes = [vp, C.POINTER(Timing)]
        L.kb_last_timing.restype = C.c_int
        fp = C.POINTER(C.c_float)
        L.kb_sg_loss_grad.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, C.c_int, C.c_int,
                                      C.POINTER(C.c_double), fp]
        L.kb_sg_loss_grad.restype = C.c_int
        L.kb_sg_train_step.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, C.c_int, C.c_int,
                                       C.c_double, C.POINTER(C.c_double)]
        L.kb_sg_train_step.restype = C.c_int
        L.kb_kernels_per_iter.argtypes = [vp]
        L.kb_kernels_per_iter.restype = C.c_int
        L.kb_destroy.argtypes = [vp]
        L.kb_destroy.restype = C.c_int
        L.kb_last_error.argtypes = []
        L.kb_last_error.restype = C.c_char_p
        L.kb_abi_version.restype = C.c_int
        L.kb_stream_probe.argtypes = [C.c_int, C.c_int, C.c_int64, vp, C.c_size_t, vp, C.c_int,
                                      C.POINTER(C.c_double)]
        L.kb_stream_probe.restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise KBError(rc, lib().kb_last_error().decode())
    return rc


def _shape_arr(shape):
    shape = [int(s) for s in shape]
    return (C.c_int64 * max(1, len(shape)))(*shape), len(shape)


def workspace_bytes(problem, shape):
    arr, nd = _shape_arr(shape)
    return int(lib().kb_workspace_bytes(problem, arr, nd))


def reduce_noalloc(arrays, square=False, out=None, stream=None):
    """kb_reduce_noalloc: deterministic sum (or sum of squares) over 1..6
    contiguous float32 device tensors of equal size into a float64 device
    tensor of one element (`out`, a new one unless given), enqueued on
    `stream` (torch's current stream by default); the library's static
    scratch holds the partials, nothing is allocated by the call."""
    arrays = list(arrays)
    n = arrays[0].numel()
    for a in arrays:
        assert a.is_cuda and a.dtype == torch.float32 and a.is_contiguous() and a.numel() == n
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=arrays[0].device)
    s = stream if stream is not None else torch.cuda.current_stream(arrays[0].device)
    ptrs = (C.c_void_p * len(arrays))(*[a.data_ptr() for a in arrays])
    with torch.cuda.device(arrays[0].device):
        _check(lib().kb_reduce_noalloc(ptrs, len(arrays), n, int(bool(square)), C.c_void_p(out.data_ptr()),
                                       C.c_void_p(s.cuda_stream)))
    return out


def stream_probe(nin, nout, n, reps=10, device=0):
    """kb_stream_probe: mean seconds per launch of a kernel reading nin and
    writing nout arrays of n floats (the attainable DRAM throughput of that
    stream mix).  The workspace is a torch uint8 tensor on the device."""
    lib()
    dev = torch.device("cuda", device)
    with torch.cuda.device(dev):
        nbytes = (nin + nout) * int(n) * 4
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (ws.data_ptr() + 255) // 256 * 256
        stream = torch.cuda.current_stream(dev)
        sec = C.c_double()
        _check(lib().kb_stream_probe(int(nin), int(nout), int(n), C.c_void_p(aligned), nbytes,
                                     C.c_void_p(stream.cuda_stream), int(reps), C.byref(sec)))
        del ws
    return sec.value


class Problem:
    """One problem instance (kb_create ... kb_destroy).

    The workspace is a torch uint8 tensor on the device; the stream is a
    torch.cuda.Stream (a new one unless given).  Methods mirror the C ABI.
    """

    def __init__(self, problem, shape, coeffs=(), seed=0, device=0, stream=None):
        lib()
        self.problem = problem
        self.shape = tuple(int(s) for s in shape)
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self._h = C.c_void_p()
        self._sg_m = 0                     # pixels of the last training batch (tape fields)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
            nbytes = workspace_bytes(problem, shape)
            if nbytes == 0:
                raise KBError(EINVAL, f"invalid problem {problem} / shape {shape}")
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            arr, nd = _shape_arr(shape)
            co = [float(c) for c in coeffs]
            carr = (C.c_double * max(1, len(co)))(*co)
            torch.cuda.synchronize(self.device)
            _check(lib().kb_create(problem, arr, nd, carr, len(co), C.c_uint64(int(seed) & (2**64 - 1)),
                                   C.c_void_p(aligned), nbytes, C.c_void_p(self.stream.cuda_stream),
                                   C.byref(self._h)))

    # -- C ABI mirrors --------------------------------------------------------
    def set_option(self, option, value):
        _check(lib().kb_set_option(self._h, option, int(value)))

    def run(self, n_steps, batch_b=0):
        """Advance n_steps; batch_b = 0 per launch, >= 1 graph batches.
        Returns the status (0, or WFALLBACK if a graph build failed)."""
        return _check(lib().kb_run(self._h, int(n_steps), int(batch_b)))

    def last_timing(self):
        t = Timing()
        _check(lib().kb_last_timing(self._h, C.byref(t)))
        return t.as_dict()

    def kernels_per_iter(self):
        return _check(lib().kb_kernels_per_iter(self._h))

    def reduce(self):
        out = (C.c_double * 2)()
        _check(lib().kb_reduce(self._h, out, 2))
        return [out[0], out[1]] if self.problem == FDTD3D else [out[0]]

    def field_shape(self, field):
        p, s = self.problem, self.shape
        if field in (F_EX, F_EY, F_EZ, F_HX, F_HY, F_HZ):
            M = s[0] + 1
            return (M, M, M), np.float32
        if field == F_PROBE:
            return ((s[1] if len(s) > 1 else 16384),), np.float32
        if field == F_STEP:
            return (1,), np.int64
        if field == F_W:
            return (SG_NW,), np.float32
        if field == F_SGSTATS:
            return (2,), np.int64
        if field == F_RESID:
            return (4096,), np.float64
        if field == F_REDLOG:
            return (4096, 4), np.float64
        if field == F_REDCOUNT:
            return (1,), np.int64
        if F_SG_X <= field <= F_SG_GRAD:
            m = self._sg_m
            if field == F_SG_X:
                return (m, 2), np.uint16
            if field in (F_SG_A1, F_SG_A2, F_SG_A3):
                return (m, 32), np.uint16
            if field in (F_SG_Z1, F_SG_Z2, F_SG_Z3, F_SG_G1, F_SG_G2, F_SG_G3):
                return (m, 32), np.float32
            if field == F_SG_GRAD:
                return (SG_NW,), np.float32
            return (m,), np.float32
        if field in (F_A, F_B):
            return (self.kernels_per_iter(),), np.float32
        if field == F_X:
            return (s[0],), np.float32
        if p in (HEAT2D, HEAT2D_SURROGATE):
            return (s[0], s[1]), np.float32
        if p == HEAT3D:
            return ((s[0], s[1], s[2]) if field == F_T else (s[1], s[2])), np.float32
        if p == HEAT2D_MULTI:
            return (sum(s[1 + 2 * g] * s[2 + 2 * g] for g in range(s[0])),), np.float32
        raise KBError(EINVAL, f"unknown field {field}")

    def reduction_log(self):
        """Entries of the in-chain reduction log (KB_OPT_REDUCE_EVERY):
        array [count][4] of {step, value, second value, 0}."""
        n = int(self.read(F_REDCOUNT)[0])
        return self.read(F_REDLOG)[:min(n, 4096)]

    def read(self, field):
        """Copy a field to a new host numpy array (synchronises the stream)."""
        shp, dt = self.field_shape(field)
        out = np.empty(shp, dtype=dt)
        _check(lib().kb_read(self._h, field, out.ctypes.data_as(C.c_void_p), out.nbytes, 0))
        return out

    def _after_torch(self):
        """Order the problem's stream after the work torch has queued so
        far (device tensors handed to the library may still be in flight on
        torch's current stream)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def read_device(self, field, out: torch.Tensor):
        """Copy a field into a contiguous device tensor of the same byte size
        (synchronous: the copy is complete on return)."""
        assert out.is_cuda and out.is_contiguous()
        self._after_torch()
        _check(lib().kb_read(self._h, field, C.c_void_p(out.data_ptr()), out.numel() * out.element_size(), 1))
        return out

    def write_device(self, field, src: torch.Tensor):
        """Copy a contiguous device tensor of the field's byte size into a
        field (synchronous; torch's queued work is finished first)."""
        shp, dt = self.field_shape(field)
        assert src.is_cuda and src.is_contiguous()
        if src.numel() * src.element_size() != int(np.prod(shp)) * np.dtype(dt).itemsize:
            raise KBError(EINVAL, f"field {field} needs {int(np.prod(shp)) * np.dtype(dt).itemsize} bytes")
        torch.cuda.synchronize(self.device)
        _check(lib().kb_write(self._h, field, C.c_void_p(src.data_ptr()), src.numel() * src.element_size(), 1))

    def write(self, field, values):
        shp, dt = self.field_shape(field)
        arr = np.ascontiguousarray(values, dtype=dt)
        if arr.size != int(np.prod(shp)):
            raise KBError(EINVAL, f"field {field} needs {np.prod(shp)} values, got {arr.size}")
        _check(lib().kb_write(self._h, field, arr.ctypes.data_as(C.c_void_p), arr.nbytes, 0))

    # -- surrogate training (KB_HEAT2D_SURROGATE) ------------------------------
    @staticmethod
    def _fields(T0, P, T16):
        for t in (T0, P, T16):
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous() and t.dim() == 3
        assert T0.shape == P.shape == T16.shape
        return T0.shape

    def sg_loss_grad(self, T0, P, T16, crops, crop):
        """(loss, gradient[19393]) on the crops (int array [n][3]: field,
        y0, x0) of device fields T0, P, T16 ([nfield][H][W] float32)."""
        nf, H, W = self._fields(T0, P, T16)
        cr = np.ascontiguousarray(crops, dtype=np.int32)
        loss = C.c_double()
        grad = np.empty(SG_NW, np.float32)
        self._after_torch()
        _check(lib().kb_sg_loss_grad(self._h, C.c_void_p(T0.data_ptr()), C.c_void_p(P.data_ptr()),
                                     C.c_void_p(T16.data_ptr()), nf, H, W, cr.ctypes.data_as(C.c_void_p),
                                     cr.shape[0], int(crop), C.byref(loss),
                                     grad.ctypes.data_as(C.POINTER(C.c_float))))
        self._sg_m = cr.shape[0] * int(crop) ** 2
        return loss.value, grad

    def sg_train_step(self, T0, P, T16, crops, crop, lr):
        """One Adam step on the crops; returns the batch loss before it."""
        nf, H, W = self._fields(T0, P, T16)
        cr = np.ascontiguousarray(crops, dtype=np.int32)
        loss = C.c_double()
        self._after_torch()
        _check(lib().kb_sg_train_step(self._h, C.c_void_p(T0.data_ptr()), C.c_void_p(P.data_ptr()),
                                      C.c_void_p(T16.data_ptr()), nf, H, W, cr.ctypes.data_as(C.c_void_p),
                                      cr.shape[0], int(crop), float(lr), C.byref(loss)))
        self._sg_m = cr.shape[0] * int(crop) ** 2
        return loss.value

    def destroy(self):
        if self._h:
            rc = lib().kb_destroy(self._h)
            self._h = C.c_void_p()
            _check(rc)

    close = destroy

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            if self._h:
                lib().kb_destroy(self._h)
                self._h = C.c_void_p()
        except Exception:
            pass


def create(problem, shape, coeffs=(), seed=0, device=0, stream=None):
    return Problem(problem, shape, coeffs, seed, device, stream)


HEAT_COEFFS = (1e-3, 1.0, 1.0, 10.0, 300.0)   # c, Rx, Ry, Rz, Tamb
FDTD_COEFFS = (0.5, 20.0, 80.0)               # courant, pulse width, delay
