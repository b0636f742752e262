"""The exact line-solve core of the direct stages (csrc/direct_core.h),
built with g++ and run on the host: the whole-line solve satisfies the stage
equations written with the oracle's dense operators (Section 2.1, eqs.
ecua2:PR / ecua3:PR2; Appendices A, B), and windows with the computed margin
reproduce it to rounding."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2006_07583_amd", "csrc")


@pytest.fixture(scope="module")
def exe():
    d = tempfile.mkdtemp()
    path = os.path.join(d, "direct_core_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wno-unknown-pragmas", "-I", CSRC,
                    os.path.join(HERE, "direct_core_check.cpp"), "-o", path], check=True)
    return path


def _solve(exe, method, n, S, H, mode, h, A, B, K, R, src_s=-1, aF=0.0, Se=0):
    head = f"{method} {n} {S} {Se} {H} {mode} {1.0 / h!r} {src_s} {aF!r}\n"
    body = "\n".join(" ".join(repr(float(x)) for x in arr) for arr in (A, B, K, R))
    res = subprocess.run([exe, "solve"], input=head + body, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    return np.array(lines[0].split(), float), np.array(lines[1].split(), float)


def _margin(exe, method, c2, tol):
    return int(subprocess.run([exe, "margin", str(method), repr(float(c2)), repr(float(tol))], capture_output=True,
                              text=True, check=True).stdout)


def _line(method, n, h, cfl, seed):
    rng = np.random.default_rng(seed)
    a = 0.5 * cfl * h
    A = rng.standard_normal(n + 2)
    B = rng.standard_normal(n + 2)
    K = a * (0.5 + 0.5 * rng.random(n + 2))   # a kappa, kappa in [0.5, 1]
    R = a * (0.5 + 0.5 * rng.random(n + 2))   # a / rho
    A[0] = 0.0
    A[n if method == O.CFD else n + 1] = 0.0
    if method == O.CFD:
        A[n + 1] = B[n + 1] = 0.0
    else:
        B[n + 1] = 0.0
    return A, B, K, R


def _stage_residuals(method, n, h, A, B, K, R, U, V):
    if method == O.MFD:
        D, G = O.mfd_matrices(n, h)
        u = U[1:n + 1]
        r1 = u + K[1:n + 1] * (D @ V[:n + 1]) - A[1:n + 1]
        r2 = V[:n + 1] + R[:n + 1] * (G[:, 1:n + 1] @ u) - B[:n + 1]
    else:
        P, Q, Pb, Qb = O.cfd_matrices(n, h)
        Dbar, Gd = np.linalg.solve(Pb, Qb), np.linalg.solve(P, Q)
        u = U[1:n]
        r1 = u + K[1:n] * (Dbar @ V[:n + 1]) - A[1:n]
        r2 = V[:n + 1] + R[:n + 1] * (Gd[:, 1:n] @ u) - B[:n + 1]
    return r1, r2


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
@pytest.mark.parametrize("cfl", [0.8, 3.0])
def test_whole_line_solve_satisfies_stage_equations(exe, method, cfl):
    n = 120
    h = 1.0 / n
    A, B, K, R = _line(method, n, h, cfl, 3 + method)
    ns = n if method == O.MFD else n + 1
    U, V = _solve(exe, method, n, ns, 0, 1, h, A, B, K, R)
    r1, r2 = _stage_residuals(method, n, h, A, B, K, R, U, V)
    scale = max(np.abs(U).max(), np.abs(V).max())
    assert np.abs(r1).max() < 1e-12 * scale and np.abs(r2).max() < 1e-12 * scale


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
@pytest.mark.parametrize("cfl,S", [(0.8, 23), (3.0, 61)])
@pytest.mark.parametrize("short_ends", [False, True])
def test_windows_with_margin_equal_whole_line(exe, method, cfl, S, short_ends):
    """Windows of S output slots (ragged last window) with the margin sized
    for FP64 equal the single-window solve to 1e-13, in both output modes;
    the fused mode is 2 Ubar - A (+ aF at the source) and 2 vel - B."""
    n = 700
    h = 1.0 / n
    A, B, K, R = _line(method, n, h, cfl, 11 + method)
    c2 = (K.max() * R.max()) / h ** 2
    H = _margin(exe, method, c2, 1e-17)
    assert 0 < H < 400
    ns = n if method == O.MFD else n + 1
    U1, V1 = _solve(exe, method, n, ns, 0, 1, h, A, B, K, R)
    Se = H + 4 if short_ends else 0
    Uw, Vw = _solve(exe, method, n, S, H, 1, h, A, B, K, R, Se=Se)
    scale = max(np.abs(U1).max(), np.abs(V1).max())
    assert np.abs(Uw - U1).max() < 1e-13 * scale and np.abs(Vw - V1).max() < 1e-13 * scale
    src = n // 3
    Un, Vn = _solve(exe, method, n, S, H, 0, h, A, B, K, R, src_s=src, aF=0.25, Se=Se)
    lo, hi = (1, n) if method == O.MFD else (1, n - 1)
    want_u = 2 * U1[lo:hi + 1] - A[lo:hi + 1]
    want_u[src - lo] += 0.25
    assert np.abs(Un[lo:hi + 1] - want_u).max() < 1e-12 * scale
    assert np.abs(Vn[:n + 1] - (2 * V1[:n + 1] - B[:n + 1])).max() < 1e-12 * scale


def test_margin_grows_with_step(exe):
    for method in (O.CFD, O.MFD):
        hs = [_margin(exe, method, c2, 1e-17) for c2 in (0.04, 0.16, 1.0, 4.0)]
        assert all(b > a for a, b in zip(hs, hs[1:])), hs
        assert _margin(exe, method, 0.16, 1e-9) < hs[1]


def test_window_plan_invariants(exe):
    """The windows the kernels are launched over partition each line, the
    interior-band windows stay inside the interior rows, and every kept row
    fits the per-thread factor store (host check of the index ranges)."""
    res = subprocess.run([exe, "plan"], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "0", res.stdout + res.stderr


def test_gathered_pressure_stores(exe):
    """The pressure outputs of a window, put in descending slot order, land
    in their slots exactly once through the 32-byte piece stores and the
    single stores at the window edges (every window within 80 slots, FP32
    and FP64, gathering on and off); piece stores start on the piece grid."""
    res = subprocess.run([exe, "sink"], capture_output=True, text=True)
    assert res.returncode == 0 and res.stdout.strip() == "0", res.stdout + res.stderr
