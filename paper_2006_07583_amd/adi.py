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
           "adi_workspace_size", "adi_bind", "adi_run", "adi_step", "adi_sync", "adi_get_state",
           "adi_get_step", "adi_set_step", "adi_run_noalloc", "adi_set_check", "adi_check_stats",
           "adi_autotune", "adi_get_plan", "adi_set_plan", "adi_set_graph",
           "adi_set_forcing", "adi_set_boundary", "adi_set_damping",
           "adi_set_tolerance", "adi_sweep_stats", "adi_destroy",
           "adi_batch_create", "adi_batch_run", "adi_batch_sync", "adi_batch_launches",
           "adi_batch_destroy",
           "adi_server_params_init", "adi_server_create", "adi_submit", "adi_poll", "adi_wait", "adi_fetch",
           "adi_request_times", "adi_server_get_stats", "adi_server_destroy", "adi_stream_ceiling")

BATCH_GRAPH = 1
BATCH_ONE_STREAM = 2
WALL_X0, WALL_X1, WALL_Y0, WALL_Y1 = 1, 2, 4, 8
REQUEST_HOLD = 1


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


class AdiSignal(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("f0", ctypes.c_double),
                ("t0", ctypes.c_double), ("amp", ctypes.c_double)]


SIGNAL_RICKER, SIGNAL_COS = 1, 2

KERNEL_SINGLE, KERNEL_WAVE, KERNEL_DIRECT = 1, 3, 4


class AdiPlanInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("kernel", "lines", "slots", "windows", "window", "margin",
                                              "lines_per_group", "workgroups", "tile_shape", "tile_order",
                                              "tuned")] + [("reserved", ctypes.c_int32 * 5)]


def _signal(g):
    s = AdiSignal()
    s.kind, s.f0, s.t0, s.amp = int(g["kind"]), float(g["f0"]), float(g.get("t0", 0.0)), float(g.get("amp", 1.0))
    return s


class AdiServerParams(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_active", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_uint64)]


class AdiRequest(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_int32), ("params", AdiParams),
                ("nsteps", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("V", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("K", ctypes.c_void_p), ("Rv", ctypes.c_void_p), ("Rw", ctypes.c_void_p),
                ("ld", ctypes.c_int64 * 6)]


class AdiServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("active", ctypes.c_int64), ("done", ctypes.c_int64),
                ("peak_active", ctypes.c_int64), ("ticks", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("arena_used", ctypes.c_uint64)]


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
        L.adi_get_state.argtypes = [vp, vp, vp, vp]
        L.adi_set_check.argtypes = [vp, i64, ctypes.c_double]
        L.adi_set_forcing.argtypes = [vp, vp, i64, ctypes.POINTER(AdiSignal)]
        L.adi_set_boundary.argtypes = [vp, ctypes.POINTER(AdiSignal)]
        L.adi_set_damping.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.adi_check_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.adi_autotune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.adi_get_plan.argtypes = [vp, ctypes.c_int, ctypes.POINTER(AdiPlanInfo)]
        L.adi_set_plan.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.adi_set_graph.argtypes = [vp, ctypes.c_int]
        L.adi_stream_ceiling.argtypes = [ctypes.c_int, vp, vp, vp, vp, vp, i64, vp]
        L.adi_run_noalloc.argtypes = [ctypes.POINTER(AdiParams), vp, vp, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(i64), i64]
        L.adi_get_step.argtypes = [vp, ctypes.POINTER(i64)]
        L.adi_set_step.argtypes = [vp, i64]
        L.adi_set_tolerance.argtypes = [vp, ctypes.c_double, ctypes.c_int]
        L.adi_sweep_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.adi_destroy.argtypes = [vp]
        L.adi_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp, ctypes.c_int, ctypes.POINTER(vp)]
        L.adi_batch_run.argtypes = [vp, i64]
        L.adi_batch_sync.argtypes = [vp]
        L.adi_batch_launches.argtypes = [vp, ctypes.POINTER(i64)]
        L.adi_batch_destroy.argtypes = [vp]
        L.adi_server_params_init.argtypes = [ctypes.POINTER(AdiServerParams)]
        L.adi_server_create.argtypes = [ctypes.POINTER(AdiServerParams), ctypes.POINTER(vp)]
        L.adi_submit.argtypes = [vp, ctypes.POINTER(AdiRequest), ctypes.POINTER(ctypes.c_uint64)]
        L.adi_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
        L.adi_wait.argtypes = [vp, ctypes.c_uint64]
        L.adi_fetch.argtypes = [vp, ctypes.c_uint64, vp, vp, vp]
        dp = ctypes.POINTER(ctypes.c_double)
        L.adi_request_times.argtypes = [vp, ctypes.c_uint64, dp, dp, dp]
        L.adi_server_get_stats.argtypes = [vp, ctypes.POINTER(AdiServerStats)]
        L.adi_server_destroy.argtypes = [vp]
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


def run_noalloc(params: AdiParams, U, V, W, K=None, Rv=None, Rw=None, nsteps=1, stream=None):
    """adi_run_noalloc: nsteps steps of the problem on torch device tensors
    (U, V, W updated in place, asynchronously on `stream`) with the library's
    static workspace: no device allocation."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    ld = (ctypes.c_int64 * 6)()
    for i, t in enumerate((U, V, W, K, Rv, Rw)):
        if t is not None:
            if t.dim() != 2 or t.stride(1) != 1:
                raise ValueError("arrays must be 2-D with contiguous rows")
            ld[i] = t.stride(0)
    _check(lib().adi_run_noalloc(ctypes.byref(params), ctypes.c_void_p(stream.cuda_stream),
                                 *[_dptr(t) for t in (U, V, W, K, Rv, Rw)], ld, int(nsteps)))


class Problem:
    """One ADI problem: ``adi_create`` + ``adi_bind`` on torch device tensors.

    U, V, W hold the initial state; :meth:`run` keeps the state in the
    library's workspace and :meth:`get_state` writes it out (into U, V, W by
    default).  K, Rv, Rw are read at bind.  Rows of every tensor must be
    contiguous (row stride = leading dimension).
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

    def set_forcing(self, F, signal) -> "Problem":
        """adi_set_forcing (before bind): f = F(x, y) s(t), F a device tensor
        shaped like U, signal a dict (kind 1 Ricker / 2 cosine, f0, t0, amp);
        F None removes it."""
        if F is None:
            _check(lib().adi_set_forcing(self._h, None, 0, None))
            self._force = None
            return self
        if F.dim() != 2 or F.stride(1) != 1:
            raise ValueError("F must be 2-D with contiguous rows")
        s = _signal(signal)
        _check(lib().adi_set_forcing(self._h, _dptr(F), F.stride(0), ctypes.byref(s)))
        self._force = F
        return self

    def set_damping(self, d0: float, width: float, walls: int) -> "Problem":
        """adi_set_damping: absorbing layers of rate d0 (1 - dist/width)^2
        along the walls in the mask (WALL_*); d0 = 0 switches them off."""
        _check(lib().adi_set_damping(self._h, float(d0), float(width), int(walls)))
        return self

    def set_boundary(self, signal) -> "Problem":
        """adi_set_boundary (before bind): wall pressure = (U's wall entries
        at bind) x s(t); None restores homogeneous walls."""
        s = None if signal is None else _signal(signal)
        _check(lib().adi_set_boundary(self._h, None if s is None else ctypes.byref(s)))
        return self

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

    def get_state(self, U=None, V=None, W=None):
        """adi_get_state: write the current state into U, V, W (tensors laid
        out like the bound ones; None = the bound tensor) and wait for it."""
        for t, b in zip((U, V, W), self._keep[:3]):
            if t is not None and (t.shape != b.shape or t.stride() != b.stride() or t.dtype != b.dtype):
                raise ValueError("get_state targets must match the bound arrays' shape, strides and dtype")
        _check(lib().adi_get_state(self._h, _dptr(U), _dptr(V), _dptr(W)))

    @property
    def step_index(self) -> int:
        m = ctypes.c_int64()
        _check(lib().adi_get_step(self._h, ctypes.byref(m)))
        return m.value

    @step_index.setter
    def step_index(self, m: int):
        _check(lib().adi_set_step(self._h, int(m)))

    def set_check(self, every: int, max_abs: float = 0.0) -> "Problem":
        """adi_set_check: device-side health check every `every` steps
        (0 = off); sync and get_state raise ADI_ENUMERIC when it trips."""
        _check(lib().adi_set_check(self._h, int(every), float(max_abs)))
        return self

    def check_stats(self):
        """(largest magnitude seen, non-finite seen) of the health check."""
        m, nf = ctypes.c_double(), ctypes.c_int()
        _check(lib().adi_check_stats(self._h, ctypes.byref(m), ctypes.byref(nf)))
        return m.value, bool(nf.value)

    def autotune(self, reps: int = 0):
        """Time the launch choices of both directions' line passes and keep
        the fastest (adi_autotune); returns the chosen pass times (us) of
        the x and y passes."""
        us = (ctypes.c_double * 2)()
        _check(lib().adi_autotune(self._h, int(reps), us))
        return us[0], us[1]

    def plan(self, direction: int) -> dict:
        """The launch plan of the x (0) or y (1) lines (adi_get_plan)."""
        info = AdiPlanInfo()
        _check(lib().adi_get_plan(self._h, int(direction), ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in AdiPlanInfo._fields_ if k != "reserved"}

    def set_graph(self, on: bool = True) -> "Problem":
        """Graph replay of :meth:`run` (adi_set_graph)."""
        _check(lib().adi_set_graph(self._h, 1 if on else 0))
        return self

    def set_plan(self, direction: int, choice: int) -> "Problem":
        """Pin the tile shape / tile order of one direction (adi_set_plan)."""
        _check(lib().adi_set_plan(self._h, int(direction), int(choice)))
        return self

    def set_tolerance(self, eps: float, min_sweeps: int = 2) -> "Problem":
        """Tolerance-tested stages (adi_set_tolerance); eps = 0 restores the
        fixed sweep count."""
        _check(lib().adi_set_tolerance(self._h, float(eps), int(min_sweeps)))
        return self

    def sweep_stats(self):
        """(passes, sweeps) of the tolerance-tested passes since set_tolerance."""
        p, s = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().adi_sweep_stats(self._h, ctypes.byref(p), ctypes.byref(s)))
        return p.value, s.value

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


def stream_ceiling(a, b, c, x, y, stream=None):
    """Queue the streaming reference kernel (adi_stream_ceiling) on torch
    device tensors of one dtype and length: x = a - c b, y = b - a."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    dt = {torch.float32: FP32, torch.float64: FP64}[a.dtype]
    ts = (a, b, c, x, y)
    if any(t.dtype != a.dtype or t.numel() != a.numel() or not t.is_contiguous() for t in ts):
        raise ValueError("five contiguous tensors of one dtype and length")
    _check(lib().adi_stream_ceiling(dt, *[ctypes.c_void_p(t.data_ptr()) for t in ts], a.numel(),
                                    ctypes.c_void_p(stream.cuda_stream)))


class Batch:
    """Several bound :class:`Problem` objects advanced together
    (``adi_batch_*``): one grouped launch per kernel variant and half-step."""

    def __init__(self, problems, stream=None, graph=False, one_stream=False):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        self._problems = list(problems)
        arr = (ctypes.c_void_p * len(self._problems))(*[p._h.value for p in self._problems])
        self._h = ctypes.c_void_p()
        _check(lib().adi_batch_create(arr, len(self._problems), ctypes.c_void_p(stream.cuda_stream),
                                      (BATCH_GRAPH if graph else 0) | (BATCH_ONE_STREAM if one_stream else 0),
                                      ctypes.byref(self._h)))

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


class Server:
    """Served problems (``adi_server_*``): requests with host (numpy) arrays,
    results written back into those arrays; one grouped step of every
    admitted problem per tick, device memory from a fixed arena."""

    def __init__(self, hbm_budget_bytes=16 << 30, max_active=256):
        p = AdiServerParams()
        _check(lib().adi_server_params_init(ctypes.byref(p)))
        p.hbm_budget_bytes, p.max_active = int(hbm_budget_bytes), int(max_active)
        self._h = ctypes.c_void_p()
        _check(lib().adi_server_create(ctypes.byref(p), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, params: AdiParams, U, V, W, K=None, Rv=None, Rw=None, nsteps=1, hold=False) -> int:
        """Queue a request; U, V, W (numpy, C-ordered rows, the params' dtype)
        receive the result (with hold=True they are inputs only and the
        result waits on the device for :meth:`fetch`).  The arrays are kept
        referenced until done."""
        import numpy as np
        want = np.float64 if params.dtype == FP64 else np.float32
        r = AdiRequest()
        r.struct_size = ctypes.sizeof(AdiRequest)
        r.flags = REQUEST_HOLD if hold else 0
        r.params = params
        r.nsteps = int(nsteps)
        arrs = (U, V, W, K, Rv, Rw)
        for i, (name, a) in enumerate(zip(("U", "V", "W", "K", "Rv", "Rw"), arrs)):
            if a is None:
                continue
            if a.dtype != want or a.ndim != 2 or a.strides[1] != a.itemsize:
                raise ValueError(f"{name}: 2-D {want.__name__} array with contiguous rows required")
            setattr(r, name, a.ctypes.data)
            r.ld[i] = a.strides[0] // a.itemsize
        t = ctypes.c_uint64()
        _check(lib().adi_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = arrs
        return t.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int()
        _check(lib().adi_poll(self._h, int(ticket), ctypes.byref(st)))
        return st.value

    def wait(self, ticket: int):
        _check(lib().adi_wait(self._h, int(ticket)))
        self._keep.pop(int(ticket), None)

    def fetch(self, ticket: int, U, V, W):
        """adi_fetch: wait for the request and copy its result into the numpy
        arrays U, V, W (laid out like the request's arrays)."""
        keep = self._keep.get(int(ticket))
        if keep is not None:
            for a, b in zip((U, V, W), keep[:3]):
                if a is not None and (a.shape != b.shape or a.strides != b.strides or a.dtype != b.dtype):
                    raise ValueError("fetch targets must match the request's arrays")
        ptr = lambda a: None if a is None else ctypes.c_void_p(a.ctypes.data)
        _check(lib().adi_fetch(self._h, int(ticket), ptr(U), ptr(V), ptr(W)))
        self._keep.pop(int(ticket), None)

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().adi_request_times(self._h, int(ticket), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def stats(self) -> dict:
        st = AdiServerStats()
        _check(lib().adi_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in AdiServerStats._fields_}

    def close(self):
        if self._h:
            lib().adi_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
