"""Thin ctypes binding of ``libadi.so`` (the C ABI of include/adi.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the stream.  The
binding raises if the library is not built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadi.so")

CFD, MFD = 0, 1
FP32, FP64, FP32C = 0, 1, 2

STATUS = {0: "ADI_OK", -1: "ADI_EINVAL", -2: "ADI_ENOMEM", -3: "ADI_EDEVICE",
          -4: "ADI_EBUSY", -5: "ADI_ENOTREADY", -6: "ADI_ENUMERIC"}

EXPORTS = ("adi_status_string", "adi_last_error", "adi_params_init", "adi_create",
           "adi_workspace_size", "adi_bind", "adi_run", "adi_step", "adi_sync",
           "adi_get_step", "adi_set_step", "adi_destroy",
           "adi_batch_create", "adi_batch_run", "adi_batch_sync", "adi_batch_launches",
           "adi_batch_destroy")

BATCH_GRAPH = 1


class AdiParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("method", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("order", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("sweeps", ctypes.c_int32), ("src_i", ctypes.c_int32), ("src_j", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
        ("c_max", ctypes.c_double), ("kappa0", ctypes.c_double), ("rinv0", ctypes.c_double),
        ("src_f0", ctypes.c_double), ("src_t0", ctypes.c_double), ("src_amp", ctypes.c_double),
    ]


class AdiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libadi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_2006_07583_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        L.adi_status_string.argtypes = [ctypes.c_int]
        L.adi_status_string.restype = ctypes.c_char_p
        L.adi_last_error.argtypes = []
        L.adi_last_error.restype = ctypes.c_char_p
        L.adi_params_init.argtypes = [ctypes.POINTER(AdiParams)]
        L.adi_create.argtypes = [ctypes.POINTER(AdiParams), vp, ctypes.POINTER(vp)]
        L.adi_workspace_size.argtypes = [ctypes.POINTER(AdiParams), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.adi_bind.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64), vp, ctypes.c_size_t]
        L.adi_run.argtypes = [vp, i64]
        L.adi_step.argtypes = [vp]
        L.adi_sync.argtypes = [vp]
        L.adi_get_step.argtypes = [vp, ctypes.POINTER(i64)]
        L.adi_set_step.argtypes = [vp, i64]
        L.adi_destroy.argtypes = [vp]
        L.adi_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_int, ctypes.POINTER(vp)]
        L.adi_batch_run.argtypes = [vp, i64]
        L.adi_batch_sync.argtypes = [vp]
        L.adi_batch_launches.argtypes = [vp, ctypes.POINTER(i64)]
        L.adi_batch_destroy.argtypes = [vp]
        for name in EXPORTS[2:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise AdiError(rc, lib().adi_last_error().decode())


def make_params(method, dtype, nx, ny, h, dt, c_max, sweeps=6, src=None, t0=0.0,
                kappa0=1.0, rinv0=1.0, order=0) -> AdiParams:
    p = AdiParams()
    _check(lib().adi_params_init(ctypes.byref(p)))
    p.method, p.dtype, p.order, p.nx, p.ny, p.sweeps = method, dtype, order, nx, ny, sweeps
    p.h, p.dt, p.t0, p.c_max, p.kappa0, p.rinv0 = h, dt, t0, c_max, kappa0, rinv0
    if src is not None:
        p.src_i, p.src_j = int(src["i"]), int(src["j"])
        p.src_f0, p.src_t0, p.src_amp = src["f0"], src["t0"], src.get("amp", 1.0)
    return p


def workspace_size(params: AdiParams, has_K=False, has_Rv=False, has_Rw=False) -> int:
    n = ctypes.c_size_t()
    _check(lib().adi_workspace_size(ctypes.byref(params), int(has_K), int(has_Rv), int(has_Rw),
                                    ctypes.byref(n)))
    return n.value


def _dptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Problem:
    """One ADI problem: ``adi_create`` + ``adi_bind`` on torch device tensors.

    U, V, W are updated in place by :meth:`run`; K, Rv, Rw are read at bind.
    Rows of every tensor must be contiguous (row stride = leading dimension).
    """

    def __init__(self, params: AdiParams, stream=None):
        import torch
        self.params = params
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self._h = ctypes.c_void_p()
        _check(lib().adi_create(ctypes.byref(params), ctypes.c_void_p(stream.cuda_stream),
                                ctypes.byref(self._h)))
        self._keep = ()

    def bind(self, U, V, W, K=None, Rv=None, Rw=None, workspace=None):
        arrs = (U, V, W, K, Rv, Rw)
        ld = (ctypes.c_int64 * 6)()
        for i, t in enumerate(arrs):
            if t is not None:
                if t.dim() != 2 or t.stride(1) != 1:
                    raise ValueError("arrays must be 2-D with contiguous rows")
                ld[i] = t.stride(0)
        ws_ptr, ws_bytes = None, 0
        if workspace is not None:
            ws_ptr, ws_bytes = ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()
        _check(lib().adi_bind(self._h, *[_dptr(t) for t in arrs], ld, ws_ptr, ws_bytes))
        self._keep = (U, V, W, workspace)
        return self

    def run(self, nsteps: int):
        _check(lib().adi_run(self._h, int(nsteps)))

    def step(self):
        _check(lib().adi_step(self._h))

    def sync(self):
        _check(lib().adi_sync(self._h))

    @property
    def step_index(self) -> int:
        m = ctypes.c_int64()
        _check(lib().adi_get_step(self._h, ctypes.byref(m)))
        return m.value

    @step_index.setter
    def step_index(self, m: int):
        _check(lib().adi_set_step(self._h, int(m)))

    def close(self):
        if self._h:
            lib().adi_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = ()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several bound :class:`Problem` objects advanced together
    (``adi_batch_*``): one grouped launch per kernel variant and half-step."""

    def __init__(self, problems, stream=None, graph=False):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self._problems = list(problems)
        arr = (ctypes.c_void_p * len(self._problems))(*[p._h.value for p in self._problems])
        self._h = ctypes.c_void_p()
        _check(lib().adi_batch_create(arr, len(self._problems), ctypes.c_void_p(stream.cuda_stream),
                                      BATCH_GRAPH if graph else 0, ctypes.byref(self._h)))

    def run(self, nsteps: int):
        _check(lib().adi_batch_run(self._h, int(nsteps)))

    def sync(self):
        _check(lib().adi_batch_sync(self._h))

    @property
    def launches(self) -> int:
        n = ctypes.c_int64()
        _check(lib().adi_batch_launches(self._h, ctypes.byref(n)))
        return n.value

    def close(self):
        if self._h:
            lib().adi_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
