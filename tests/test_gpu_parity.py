"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: FP64 max|gpu - oracle| / max|oracle| <= 1e-12 per field; FP32 relative
L2 <= 1e-4 per field after all steps.  Entries the method never writes must
come back unchanged.
"""
import math

import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import adi, inputs
from tests.gpu_util import log, max_rel, rel_l2, run_gpu, written_parts

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-4


def case(method, nx, ny, seed, medium=True, source=True):
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 1) if medium else {"K": None, "Rv": None, "Rw": None}
    cmax = 1.0
    if medium:
        cmax = math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    src = {"i": max(1, nx // 3), "j": max(1, ny // 2), "f0": 4.0, "t0": 0.1, "amp": 1.0} if source else None
    return h, f, med, cmax, src


def compare(method, dtype, nx, ny, seed, nsteps, cfl, sweeps=6, medium=True, source=True, chunks=None):
    h, f, med, cmax, src = case(method, nx, ny, seed, medium, source)
    dt = cfl * h / cmax
    log(f"case method={method} dtype={dtype} nx={nx} ny={ny} steps={nsteps} sweeps={sweeps} seed={seed}")
    ref = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=nsteps, sweeps=sweeps,
                K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src)
    got = run_gpu(method, dtype, f, h=h, dt=dt, c_max=cmax, nsteps=nsteps, sweeps=sweeps,
                  K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src, chunks=chunks)
    errs = []
    for g, r in zip(written_parts(method, *got), written_parts(method, *ref)):
        errs.append(max_rel(g, r) if dtype == adi.FP64 else rel_l2(g, r))
    # untouched entries
    U, V, W = got
    for a, b in ((U[0], f["U"][0]), (U[-1], f["U"][-1]), (U[:, 0], f["U"][:, 0]), (U[:, -1], f["U"][:, -1]),
                 (V[0], f["V"][0]), (V[-1], f["V"][-1]), (W[:, 0], f["W"][:, 0]), (W[:, -1], f["W"][:, -1])):
        tol = 0 if dtype == adi.FP64 else 1e-6 * np.abs(b).max()
        assert np.abs(a - b).max() <= tol
    log(f"  errors U,V,W = {errs}")
    return errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("nx,ny", [(8, 8), (9, 13), (33, 20), (64, 64)])
def test_small_grids_fp64(method, nx, ny):
    errs = compare(method, adi.FP64, nx, ny, 7 * nx + ny, 5, 0.6)
    assert max(errs) <= TOL64, errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("nx,ny", [(8, 8), (33, 20), (100, 77)])
def test_small_grids_fp32(method, nx, ny):
    errs = compare(method, adi.FP32, nx, ny, 3 * nx + ny, 5, 0.6)
    assert max(errs) <= TOL32, errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
def test_multi_window_lines(method, dtype):
    """Lines longer than one window (several overlapping windows, ragged tail)."""
    errs = compare(method, dtype, 1300, 600, 11, 3, 0.8 if method == adi.MFD else 1.0)
    assert max(errs) <= (TOL64 if dtype == adi.FP64 else TOL32), errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("sweeps", [2, 8, 16])
def test_sweep_counts(method, sweeps):
    errs = compare(method, adi.FP64, 530, 40, 5, 2, 0.5, sweeps=sweeps)
    assert max(errs) <= TOL64, errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
def test_constant_medium_no_source(method):
    errs = compare(method, adi.FP64, 70, 90, 2, 6, 0.7, medium=False, source=False)
    assert max(errs) <= TOL64, errs


@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
def test_split_runs_equal_one_run(dtype):
    """n + n steps in two calls give the same state as 2n steps in one call."""
    h, f, med, cmax, src = case(adi.MFD, 40, 50, 4)
    kw = dict(h=h, dt=0.5 * h / cmax, c_max=cmax, K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src)
    a = run_gpu(adi.MFD, dtype, f, nsteps=6, **kw)
    b = run_gpu(adi.MFD, dtype, f, nsteps=6, chunks=[3, 3], **kw)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= (1e-14 if dtype == adi.FP64 else 1e-6) * max(np.abs(x).max(), 1)


def test_config1_cfd_standing_wave_fp64():
    """CFD FP64, 101 x 101 nodes, c = 1, dt = h, 100 steps: parity with the
    oracle and the PR-CN time error 4.402e-4 against the exact solution."""
    N = 100
    h = 1.0 / N
    f = inputs.standing_mode(adi.CFD, N, N, h, 1, 1)
    log("case config1 CFD FP64 N=100 steps=100")
    ref = O.run(O.CFD, f["U"], f["V"], f["W"], h=h, dt=h, nsteps=N, sweeps=6)
    got = run_gpu(adi.CFD, adi.FP64, f, h=h, dt=h, c_max=1.0, nsteps=N)
    for g, r in zip(written_parts(adi.CFD, *got), written_parts(adi.CFD, *ref)):
        assert max_rel(g, r) <= TOL64
    err = np.abs(got[0] - f["U"] * math.cos(math.sqrt(2) * math.pi)).max()
    assert err == pytest.approx(4.402e-4, rel=1e-2)


def _order_run(method, dtype, f, med, src, h, dt, cmax, nsteps, order):
    from tests.gpu_util import run_gpu as rg
    return rg(method, dtype, f, h=h, dt=dt, c_max=cmax, nsteps=nsteps, K=med["K"], Rv=med["Rv"],
              Rw=med["Rw"], src=src, order=order)


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
@pytest.mark.parametrize("nx,ny", [(40, 29), (700, 530)])
def test_role_swap_transposed_problem_bitwise(method, dtype, nx, ny):
    """The row and column passes swap roles when the problem is transposed and
    the y-implicit stage goes first: the result is the exact transpose."""
    h, f, med, cmax, src = case(method, nx, ny, 17)
    dt = 0.7 * h / cmax
    log(f"case role-swap method={method} dtype={dtype} nx={nx} ny={ny}")
    a = _order_run(method, dtype, f, med, src, h, dt, cmax, 4, 0)
    fT = {"U": f["U"].T, "V": f["W"].T, "W": f["V"].T}
    medT = {"K": med["K"].T, "Rv": med["Rw"].T, "Rw": med["Rv"].T}
    srcT = dict(src, i=src["j"], j=src["i"])
    b = _order_run(method, dtype, fT, medT, srcT, h, dt, cmax, 4, 1)
    assert np.array_equal(b[0].T, a[0])
    assert np.array_equal(b[2].T, a[1])
    assert np.array_equal(b[1].T, a[2])


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
def test_order1_matches_oracle(method):
    h, f, med, cmax, src = case(method, 600, 90, 23)
    dt = 0.7 * h / cmax
    log(f"case order1 method={method}")
    ref = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=3, sweeps=6,
                K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src, order=1)
    got = _order_run(method, adi.FP64, f, med, src, h, dt, cmax, 3, 1)
    for g, r in zip(written_parts(method, *got), written_parts(method, *ref)):
        assert max_rel(g, r) <= TOL64


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("nx,ny", [(8, 8), (33, 20), (1300, 600)])
@pytest.mark.parametrize("order", [0, 1])
def test_compensated_fp32(method, nx, ny, order):
    h, f, med, cmax, src = case(method, nx, ny, 5 * nx + ny + order)
    dt = 0.6 * h / cmax
    log(f"case fp32c method={method} nx={nx} ny={ny} order={order}")
    ref = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=4, sweeps=6,
                K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src, order=order)
    got = run_gpu(method, adi.FP32C, f, h=h, dt=dt, c_max=cmax, nsteps=4, K=med["K"], Rv=med["Rv"],
                  Rw=med["Rw"], src=src, order=order)
    errs = [rel_l2(g, r) for g, r in zip(written_parts(method, *got), written_parts(method, *ref))]
    log(f"  errors {errs}")
    assert max(errs) <= TOL32, errs


@pytest.mark.parametrize("method,nsteps", [(adi.CFD, 100), (adi.MFD, 600)])
def test_compensated_error_not_above_plain_fp32(method, nsteps):
    """Smooth standing mode: the compensated FP32 state drifts from the FP64
    oracle no more than plain FP32 does.  The compact scheme runs a shorter
    horizon: its growing boundary modes amplify any rounding difference
    (the oracle's own included) within a few hundred steps."""
    N = 600
    h = 1.0 / N
    f = inputs.standing_mode(method, N, N, h, 3, 2)
    dt = 0.5 * h
    log(f"case fp32c-vs-fp32 method={method} steps={nsteps}")
    ref = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=nsteps, sweeps=6)
    e = {}
    for dt_ in (adi.FP32, adi.FP32C):
        got = run_gpu(method, dt_, f, h=h, dt=dt, c_max=1.0, nsteps=nsteps)
        e[dt_] = rel_l2(got[0][1:-1, 1:-1], ref[0][1:-1, 1:-1])
    log(f"  fp32 {e[adi.FP32]:.3e}  fp32c {e[adi.FP32C]:.3e}")
    assert e[adi.FP32C] <= e[adi.FP32] * 1.05
    assert e[adi.FP32C] <= TOL32


# Lines whose slot count sits at either side of each single-window tile shape
# (128, 256, 512 slots) and just past the multi-window threshold; slots per
# line are n + 1 (compact) and n + 2 (mimetic).
_EDGES = {adi.CFD: [127, 128, 255, 256, 511, 512], adi.MFD: [126, 127, 254, 255, 510, 511]}


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("shift", range(4))
@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
def test_last_window_off_grid(method, shift, dtype):
    """Lines just over one window: the last window starts `shift` slots past
    a multiple of 4 (its chunks are read from the grid slot below and shifted),
    for every shift, both layouts' roles and both methods."""
    ns0 = 512 + 4 + shift                      # line slots: n + 1 (CFD), n + 2 (MFD)
    n = ns0 - (1 if method == adi.CFD else 2)
    tol = TOL64 if dtype == adi.FP64 else TOL32
    for nx, ny in ((n, 12), (12, n)):
        errs = compare(method, dtype, nx, ny, seed=90 + shift, nsteps=3, cfl=0.6)
        assert max(errs) <= tol, (nx, ny, errs)


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("k", range(6))
@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
def test_window_shape_boundaries(method, k, dtype):
    n = _EDGES[method][k]
    tol = TOL64 if dtype == adi.FP64 else TOL32
    for nx, ny in ((n, 12), (12, n)):
        errs = compare(method, dtype, nx, ny, seed=70 + k, nsteps=3, cfl=0.6)
        assert max(errs) <= tol, (nx, ny, errs)
