"""ctypes front end of the FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE: the plain, slow reference implementation of the
Peaceman-Rachford ADI step (Section 2, Algorithms 1-4, Appendices A-C of
arXiv 2006.07583).  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
GPU library.

Array conventions (row = y index j, column = x index i), float64, C order:

=====  =======================  =======================
array  CFD                      MFD
=====  =======================  =======================
U, K   (ny+1, nx+1)             (ny+2, nx+2)
V, Rv  (ny+1, nx+1)             (ny+2, nx+1)
W, Rw  (ny+1, nx+1)             (ny+1, nx+2)
=====  =======================  =======================
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFD = 0
MFD = 1


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("method", ctypes.c_int32), ("order", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("sweeps", ctypes.c_int32), ("src_i", ctypes.c_int32),
        ("src_j", ctypes.c_int32), ("threads", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
        ("src_f0", ctypes.c_double), ("src_t0", ctypes.c_double),
        ("src_amp", ctypes.c_double),
        ("kappa0", ctypes.c_double), ("rinv0", ctypes.c_double),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_run.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, ctypes.c_int64]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_run_eps.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]
        lib.oracle_run_eps.restype = ctypes.c_int
        lib.oracle_run_direct.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, ctypes.c_int64]
        lib.oracle_run_direct.restype = ctypes.c_int
        sp = ctypes.POINTER(_Signal)
        lib.oracle_run_forced.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, ctypes.c_int64, dp, sp,
                                          sp]
        lib.oracle_run_forced.restype = ctypes.c_int
        lib.oracle_run_damped.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, dp, dp, dp, ctypes.c_int64, dp]
        lib.oracle_run_damped.restype = ctypes.c_int
        lib.oracle_source.argtypes = [ctypes.POINTER(_Params), ctypes.c_double]
        lib.oracle_source.restype = ctypes.c_double
        for name in ("oracle_cfd_d", "oracle_cfd_dbar", "oracle_mfd_g", "oracle_mfd_d"):
            fn = getattr(lib, name)
            fn.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
            fn.restype = ctypes.c_int
        lib.oracle_cfd_matrices.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp, dp, dp]
        lib.oracle_cfd_matrices.restype = ctypes.c_int
        lib.oracle_mfd_matrices.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        lib.oracle_mfd_matrices.restype = ctypes.c_int
        lib.oracle_cfd_pivots.argtypes = [ctypes.c_int, dp, dp]
        lib.oracle_cfd_pivots.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape, name):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"{name}: shape {a.shape}, expected {tuple(shape)}")
    return a


def shapes(method: int, nx: int, ny: int) -> dict:
    """Array shapes of one problem (see module docstring)."""
    if method == CFD:
        s = (ny + 1, nx + 1)
        return {"U": s, "K": s, "V": s, "Rv": s, "W": s, "Rw": s}
    return {"U": (ny + 2, nx + 2), "K": (ny + 2, nx + 2),
            "V": (ny + 2, nx + 1), "Rv": (ny + 2, nx + 1),
            "W": (ny + 1, nx + 2), "Rw": (ny + 1, nx + 2)}


def make_params(method, nx, ny, h, dt, sweeps=6, order=0, src=None, t0=0.0,
                kappa0=1.0, rinv0=1.0, threads=0) -> _Params:
    p = _Params()
    p.method, p.order, p.nx, p.ny, p.sweeps = method, order, nx, ny, sweeps
    p.threads = threads
    p.h, p.dt, p.t0 = h, dt, t0
    p.kappa0, p.rinv0 = kappa0, rinv0
    if src is None:
        p.src_i = p.src_j = -1
    else:
        p.src_i, p.src_j = int(src["i"]), int(src["j"])
        p.src_f0, p.src_t0, p.src_amp = src["f0"], src["t0"], src.get("amp", 1.0)
    return p


def run(method, U, V, W, *, h, dt, nsteps, sweeps=6, K=None, Rv=None, Rw=None,
        order=0, src=None, t0=0.0, kappa0=1.0, rinv0=1.0, threads=0):
    """Advance copies of (U, V, W) by ``nsteps`` PR-ADI steps; returns them.

    ``src`` is None or a dict with keys i, j (pressure index), f0, t0, amp of
    the Ricker point source.  ``threads`` <= 0 uses the OpenMP default.
    """
    ny = U.shape[0] - (1 if method == CFD else 2)
    nx = U.shape[1] - (1 if method == CFD else 2)
    sh = shapes(method, nx, ny)
    U = _f64(U, sh["U"], "U").copy()
    V = _f64(V, sh["V"], "V").copy()
    W = _f64(W, sh["W"], "W").copy()
    K = None if K is None else _f64(K, sh["K"], "K")
    Rv = None if Rv is None else _f64(Rv, sh["Rv"], "Rv")
    Rw = None if Rw is None else _f64(Rw, sh["Rw"], "Rw")
    p = make_params(method, nx, ny, h, dt, sweeps, order, src, t0, kappa0, rinv0, threads)
    rc = _load().oracle_run(ctypes.byref(p), _ptr(U), _ptr(V), _ptr(W),
                            _ptr(K), _ptr(Rv), _ptr(Rw), int(nsteps))
    if rc != 0:
        raise ValueError("oracle_run rejected its arguments")
    return U, V, W


def run_eps(method, U, V, W, *, h, dt, nsteps, eps, min_sweeps=2, sweeps=16, K=None, Rv=None,
            Rw=None, order=0, src=None, t0=0.0, kappa0=1.0, rinv0=1.0, threads=0):
    """As :func:`run`, with the tolerance test of Algorithms 3 and 4 instead
    of a fixed sweep count (``sweeps`` is then the cap).  Returns
    (U, V, W, used) with ``used[2 m + s]`` the sweeps of stage s of step m."""
    ny = U.shape[0] - (1 if method == CFD else 2)
    nx = U.shape[1] - (1 if method == CFD else 2)
    sh = shapes(method, nx, ny)
    U = _f64(U, sh["U"], "U").copy()
    V = _f64(V, sh["V"], "V").copy()
    W = _f64(W, sh["W"], "W").copy()
    K = None if K is None else _f64(K, sh["K"], "K")
    Rv = None if Rv is None else _f64(Rv, sh["Rv"], "Rv")
    Rw = None if Rw is None else _f64(Rw, sh["Rw"], "Rw")
    p = make_params(method, nx, ny, h, dt, sweeps, order, src, t0, kappa0, rinv0, threads)
    used = np.zeros(2 * int(nsteps), dtype=np.int32)
    rc = _load().oracle_run_eps(ctypes.byref(p), _ptr(U), _ptr(V), _ptr(W), _ptr(K), _ptr(Rv), _ptr(Rw),
                                int(nsteps), float(eps), int(min_sweeps),
                                used.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError("oracle_run_eps rejected its arguments")
    return U, V, W, used


def run_direct(method, U, V, W, *, h, dt, nsteps, K=None, Rv=None, Rw=None, order=0, src=None,
               t0=0.0, kappa0=1.0, rinv0=1.0, threads=0):
    """As :func:`run` with every stage's line systems solved exactly by
    dense Gaussian elimination with partial pivoting (the limit of infinitely
    many sweeps).  Cost grows as the cube of the line length: small grids."""
    ny = U.shape[0] - (1 if method == CFD else 2)
    nx = U.shape[1] - (1 if method == CFD else 2)
    sh = shapes(method, nx, ny)
    U = _f64(U, sh["U"], "U").copy()
    V = _f64(V, sh["V"], "V").copy()
    W = _f64(W, sh["W"], "W").copy()
    K = None if K is None else _f64(K, sh["K"], "K")
    Rv = None if Rv is None else _f64(Rv, sh["Rv"], "Rv")
    Rw = None if Rw is None else _f64(Rw, sh["Rw"], "Rw")
    p = make_params(method, nx, ny, h, dt, 0, order, src, t0, kappa0, rinv0, threads)
    rc = _load().oracle_run_direct(ctypes.byref(p), _ptr(U), _ptr(V), _ptr(W),
                                   _ptr(K), _ptr(Rv), _ptr(Rw), int(nsteps))
    if rc != 0:
        raise ValueError("oracle_run_direct rejected its arguments")
    return U, V, W


class _Signal(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32), ("f0", ctypes.c_double),
                ("t0", ctypes.c_double), ("amp", ctypes.c_double)]


SIGNAL_RICKER, SIGNAL_COS = 1, 2


def _signal(g):
    if g is None:
        return None
    s = _Signal()
    s.kind, s.f0, s.t0, s.amp = int(g["kind"]), float(g["f0"]), float(g.get("t0", 0.0)), float(g.get("amp", 1.0))
    return ctypes.byref(s)


def run_forced(method, U, V, W, *, h, dt, nsteps, sweeps=6, K=None, Rv=None, Rw=None, order=0, src=None,
               t0=0.0, kappa0=1.0, rinv0=1.0, threads=0, F=None, fsig=None, bsig=None):
    """As :func:`run` (or :func:`run_direct` with sweeps=0) with a
    distributed forcing f = F(x, y) s_F(t) (F pressure-shaped, fsig the
    signal dict: kind 1 Ricker / 2 cosine amp cos(2 pi f0 (t - t0)), f0, t0,
    amp) and, when bsig is given, Dirichlet wall values equal to U's entries
    on the walls times s_b(t)."""
    ny = U.shape[0] - (1 if method == CFD else 2)
    nx = U.shape[1] - (1 if method == CFD else 2)
    sh = shapes(method, nx, ny)
    U = _f64(U, sh["U"], "U").copy()
    V = _f64(V, sh["V"], "V").copy()
    W = _f64(W, sh["W"], "W").copy()
    K = None if K is None else _f64(K, sh["K"], "K")
    Rv = None if Rv is None else _f64(Rv, sh["Rv"], "Rv")
    Rw = None if Rw is None else _f64(Rw, sh["Rw"], "Rw")
    F = None if F is None else _f64(F, sh["U"], "F")
    p = make_params(method, nx, ny, h, dt, sweeps, order, src, t0, kappa0, rinv0, threads)
    rc = _load().oracle_run_forced(ctypes.byref(p), _ptr(U), _ptr(V), _ptr(W), _ptr(K), _ptr(Rv), _ptr(Rw),
                                   int(nsteps), _ptr(F), _signal(fsig), _signal(bsig))
    if rc != 0:
        raise ValueError("oracle_run_forced rejected its arguments")
    return U, V, W


def run_damped(method, U, V, W, *, h, dt, nsteps, d0, width, walls, sweeps=6, K=None, Rv=None, Rw=None,
               order=0, src=None, t0=0.0, kappa0=1.0, rinv0=1.0, threads=0):
    """As :func:`run` with damping layers: rate d0 (1 - dist/width)^2 within
    `width` cells of the walls in the mask (1: x = 0, 2: x = 1, 4: y = 0,
    8: y = 1; width 0 = uniform d0)."""
    ny = U.shape[0] - (1 if method == CFD else 2)
    nx = U.shape[1] - (1 if method == CFD else 2)
    sh = shapes(method, nx, ny)
    U = _f64(U, sh["U"], "U").copy()
    V = _f64(V, sh["V"], "V").copy()
    W = _f64(W, sh["W"], "W").copy()
    K = None if K is None else _f64(K, sh["K"], "K")
    Rv = None if Rv is None else _f64(Rv, sh["Rv"], "Rv")
    Rw = None if Rw is None else _f64(Rw, sh["Rw"], "Rw")
    p = make_params(method, nx, ny, h, dt, sweeps, order, src, t0, kappa0, rinv0, threads)
    damp = np.array([d0, width, walls], dtype=np.float64)
    rc = _load().oracle_run_damped(ctypes.byref(p), _ptr(U), _ptr(V), _ptr(W), _ptr(K), _ptr(Rv), _ptr(Rw),
                                   int(nsteps), _ptr(damp))
    if rc != 0:
        raise ValueError("oracle_run_damped rejected its arguments")
    return U, V, W


def source_value(src, h, t):
    """F(t) as the oracle applies it at the source point (Ricker / h^2)."""
    p = make_params(CFD, 8, 8, h, 1.0, src=src)
    return _load().oracle_source(ctypes.byref(p), float(t))


def _line(fn, n, h, x, nout):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(nout)
    if getattr(_load(), fn)(n, h, _ptr(x), _ptr(out)) != 0:
        raise ValueError(fn)
    return out


def cfd_d(f, h):
    """P^-1 Q f on nodes 0..n (Appendix A)."""
    n = len(f) - 1
    return _line("oracle_cfd_d", n, h, f, n + 1)


def cfd_dbar(v, h):
    """Pbar^-1 Qbar v on interior nodes 1..n-1 (Appendix A)."""
    n = len(v) - 1
    return _line("oracle_cfd_dbar", n, h, v, n - 1)


def mfd_g(u, h):
    """G4 u: u on X_cb (n+2 values) -> nodes (n+1 values) (Appendix B)."""
    n = len(u) - 2
    return _line("oracle_mfd_g", n, h, u, n + 1)


def mfd_d(v, h):
    """D4 v: v on nodes (n+1 values) -> cell centres (n values) (Appendix B)."""
    n = len(v) - 1
    return _line("oracle_mfd_d", n, h, v, n)


def cfd_matrices(n, h):
    """Dense P, Q, Pbar, Qbar as the oracle builds them."""
    P = np.zeros((n + 1, n + 1)); Q = np.zeros((n + 1, n + 1))
    Pb = np.zeros((n - 1, n - 1)); Qb = np.zeros((n - 1, n + 1))
    if _load().oracle_cfd_matrices(n, h, _ptr(P), _ptr(Q), _ptr(Pb), _ptr(Qb)) != 0:
        raise ValueError("n")
    return P, Q, Pb, Qb


def mfd_matrices(n, h):
    """Dense D4 (n x n+1) and G4 (n+1 x n+2) as the oracle builds them."""
    D = np.zeros((n, n + 1)); G = np.zeros((n + 1, n + 2))
    if _load().oracle_mfd_matrices(n, h, _ptr(D), _ptr(G)) != 0:
        raise ValueError("n")
    return D, G


def cfd_pivots(n):
    """No-pivot LU pivots of P (n+1) and Pbar (n-1)."""
    a = np.zeros(n + 1); b = np.zeros(n - 1)
    if _load().oracle_cfd_pivots(n, _ptr(a), _ptr(b)) != 0:
        raise ValueError("n")
    return a, b
