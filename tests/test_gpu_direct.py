"""Direct (exact) line solves on the GPU (params.sweeps = 0) against the
oracle's direct mode: each stage's line systems solved exactly, the
Peaceman-Rachford step with no fixed-point error, run here also beyond the
step sizes where the sweeps diverge."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import adi, inputs
from tests.gpu_util import log, max_rel, rel_l2, run_gpu, written_parts

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-4


def _case(method, nx, ny, seed, cfl):
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 1)
    cmax = math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    src = {"i": nx // 3, "j": ny // 2, "f0": 4.0, "t0": 0.1, "amp": 1.0}
    return dict(h=h, dt=cfl * h / cmax, cmax=cmax, f=f, med=med, src=src)


def _compare(method, dtype, c, nsteps, order=0):
    m = c["med"]
    ref = O.run_direct(method, c["f"]["U"], c["f"]["V"], c["f"]["W"], h=c["h"], dt=c["dt"], nsteps=nsteps,
                       K=m["K"], Rv=m["Rv"], Rw=m["Rw"], src=c["src"], order=order)
    got = run_gpu(method, dtype, c["f"], h=c["h"], dt=c["dt"], c_max=c["cmax"], nsteps=nsteps, sweeps=0,
                  K=m["K"], Rv=m["Rv"], Rw=m["Rw"], src=c["src"], order=order)
    errs = []
    for g, r in zip(written_parts(method, *got), written_parts(method, *ref)):
        errs.append(max_rel(g, r) if dtype == adi.FP64 else rel_l2(g, r))
    return errs


# (nx, ny): lines of 150-210 slots, several windows each at cfl 0.6 with a
# ragged last one; cfl 2.0 is beyond the divergence limit of the sweeps of
# both methods (1.155 compact, 0.816 mimetic)
@pytest.mark.parametrize("method,nx,ny", [(adi.CFD, 200, 171), (adi.MFD, 210, 183)])
@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
@pytest.mark.parametrize("cfl", [0.6, 2.0])
def test_direct_matches_oracle(method, nx, ny, dtype, cfl):
    log(f"direct method={method} dtype={dtype} {nx}x{ny} cfl={cfl}")
    errs = _compare(method, dtype, _case(method, nx, ny, 5, cfl), 3)
    assert max(errs) <= (TOL64 if dtype == adi.FP64 else TOL32), errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
def test_direct_y_implicit_first(method):
    log(f"direct order 1 method={method}")
    errs = _compare(method, adi.FP64, _case(method, 150, 190, 9, 1.2), 2, order=1)
    assert max(errs) <= TOL64, errs


# lines longer than 512 slots take the multi-window explicit pass: 530 x 64
# mixes it (x) with the single-window one (y)
@pytest.mark.parametrize("method,nx,ny", [(adi.CFD, 530, 64), (adi.MFD, 530, 520)])
def test_direct_long_lines(method, nx, ny):
    log(f"direct layouts method={method} {nx}x{ny}")
    errs = _compare(method, adi.FP64, _case(method, nx, ny, 13, 0.8), 1)
    assert max(errs) <= TOL64, errs


@pytest.mark.parametrize("method,mode,dtype,tol",
                         [(adi.MFD, (2, 3), adi.FP64, 1e-9), (adi.CFD, (1, 1), adi.FP64, 1e-9),
                          (adi.MFD, (2, 3), adi.FP32, 2e-4), (adi.CFD, (1, 1), adi.FP32, 2e-4)])
def test_direct_full_size_standing_mode(method, mode, dtype, tol):
    """4096^2 at cfl 2: the standing mode follows the closed-form
    Peaceman-Rachford amplification (a property that holds at any size)."""
    from tests.test_oracle_pins import pr_mode_factor
    N = 4096
    h = 1.0 / N
    log(f"direct 4096 mode method={method} dtype={dtype}")
    f = inputs.standing_mode(method, N, N, h, *mode)
    dt, nsteps = 2.0 * h, 8
    U, V, W = run_gpu(method, dtype, f, h=h, dt=dt, c_max=1.0, nsteps=nsteps, sweeps=0)
    g = pr_mode_factor(mode[0] * math.pi, mode[1] * math.pi, dt / 2, nsteps)
    assert np.abs(U - g * f["U"]).max() < tol
    assert np.isfinite(V).all() and np.isfinite(W).all()


def test_direct_scope_errors():
    p = adi.make_params(adi.MFD, adi.FP32C, 64, 64, 1 / 64, 0.5 / 64, 1.0, sweeps=0)
    with pytest.raises(adi.AdiError):
        adi.Problem(p)
    p = adi.make_params(adi.MFD, adi.FP64, 64, 64, 1 / 64, 2.0 / 64, 1.0, sweeps=0)
    pb = adi.Problem(p)
    with pytest.raises(adi.AdiError):
        pb.set_tolerance(1e-3, 2)
    pb.close()
    # a fixed sweep count keeps the divergence limit of the sweeps
    p = adi.make_params(adi.MFD, adi.FP64, 64, 64, 1 / 64, 2.0 / 64, 1.0, sweeps=6)
    with pytest.raises(adi.AdiError):
        adi.Problem(p)


def test_direct_problems_refused_by_batches_and_servers():
    import torch
    n = 64
    f = inputs.random_fields(adi.MFD, n, n, 2)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", torch.float32)
    p = adi.make_params(adi.MFD, adi.FP32, n, n, 1 / n, 0.5 / n, 1.0, sweeps=0)
    pb = adi.Problem(p).bind(t(f["U"]), t(f["V"]), t(f["W"]))
    with pytest.raises(adi.AdiError):
        adi.Batch([pb])
    pb.close()
    srv = adi.Server(hbm_budget_bytes=64 << 20, max_active=4)
    arr = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    with pytest.raises(adi.AdiError):
        srv.submit(p, arr(f["U"]), arr(f["V"]), arr(f["W"]), nsteps=1)
    srv.close()


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("nx,ny", [(8, 8), (9, 12)])
def test_direct_tiny_grids(method, nx, ny):
    """The smallest grids: one window per line, every closure row of both
    ends in it (n = 8 leaves two interior mimetic rows)."""
    log(f"direct tiny method={method} {nx}x{ny}")
    errs = _compare(method, adi.FP64, _case(method, nx, ny, 17, 1.5), 4)
    assert max(errs) <= TOL64, errs


@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
def test_direct_rebind_with_new_materials(method):
    """The factor entries of a direction's matrix are stored by its first
    pass after a bind and reused by the later ones; binding again with other
    materials must store them anew: a problem run on one medium, then bound
    to a second medium and fresh fields, matches the oracle on the second."""
    import torch
    nx, ny = 170, 150
    c1, c2 = _case(method, nx, ny, 21, 0.9), _case(method, nx, ny, 31, 0.9)
    # one step size and c_max for both media: the larger bound of the two
    cmax = max(c1["cmax"], c2["cmax"])
    h = c1["h"]
    dt = 0.9 * h / cmax
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float64)
    log(f"direct rebind method={method} {nx}x{ny}")
    p = adi.make_params(method, adi.FP64, nx, ny, h, dt, cmax, sweeps=0, src=c1["src"])
    pb = adi.Problem(p)
    f1, m1 = c1["f"], c1["med"]
    pb.bind(t(f1["U"]), t(f1["V"]), t(f1["W"]), t(m1["K"]), t(m1["Rv"]), t(m1["Rw"]))
    pb.run(3)
    f2, m2 = c2["f"], c2["med"]
    U, V, W = t(f2["U"]), t(f2["V"]), t(f2["W"])
    pb.bind(U, V, W, t(m2["K"]), t(m2["Rv"]), t(m2["Rw"]))
    pb.run(3)
    pb.get_state()
    got = tuple(x.cpu().numpy() for x in (U, V, W))
    pb.close()
    ref = O.run_direct(method, f2["U"], f2["V"], f2["W"], h=h, dt=dt, nsteps=3, K=m2["K"], Rv=m2["Rv"],
                       Rw=m2["Rw"], src=c1["src"])
    errs = [max_rel(g, r) for g, r in zip(written_parts(method, *got), written_parts(method, *ref))]
    assert max(errs) <= TOL64, errs
