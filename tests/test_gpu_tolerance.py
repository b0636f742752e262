"""Tolerance-tested stages (adi_set_tolerance; the stopping rule of
Algorithms 3 and 4) against the oracle's tolerance mode: same sweep counts
per stage, same fields, and the limits equal to fixed-count runs."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import adi, inputs
from tests.gpu_util import log, max_rel, rel_l2, written_parts

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-4
# lines over one window both ways (wave-per-line kernel), within one window
# both ways (single-window kernel), and one of each
SIZES = {adi.CFD: [(530, 520), (120, 100), (600, 90)], adi.MFD: [(520, 515), (110, 130), (80, 600)]}


def _case(method, seed, size=0):
    nx, ny = SIZES[method][size]
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 1)
    cmax = math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    src = {"i": nx // 3, "j": ny // 2, "f0": 4.0, "t0": 0.1, "amp": 1.0}
    return dict(h=h, dt=0.6 * h / cmax, cmax=cmax, f=f, med=med, src=src)


def _oracle(method, c, nsteps, eps, kmin, cap):
    m = c["med"]
    return O.run_eps(method, c["f"]["U"], c["f"]["V"], c["f"]["W"], h=c["h"], dt=c["dt"], nsteps=nsteps,
                     eps=eps, min_sweeps=kmin, sweeps=cap, K=m["K"], Rv=m["Rv"], Rw=m["Rw"], src=c["src"])


def _gpu(method, dtype, c, nsteps, cap, eps=None, kmin=2):
    """Run on the GPU; eps None = fixed count `cap`.  Returns fields and stats."""
    import torch
    tdt = torch.float64 if dtype == adi.FP64 else torch.float32
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", tdt)
    f, m = c["f"], c["med"]
    U, V, W = t(f["U"]), t(f["V"]), t(f["W"])
    ny = U.shape[0] - (1 if method == adi.CFD else 2)
    nx = U.shape[1] - (1 if method == adi.CFD else 2)
    p = adi.make_params(method, dtype, nx, ny, c["h"], c["dt"], c["cmax"], sweeps=cap, src=c["src"])
    pb = adi.Problem(p).bind(U, V, W, t(m["K"]), t(m["Rv"]), t(m["Rw"]))
    if eps is not None:
        pb.set_tolerance(eps, kmin)
    pb.run(nsteps)
    pb.get_state()
    stats = pb.sweep_stats()
    out = tuple(x.double().cpu().numpy() for x in (U, V, W))
    pb.close()
    return out, stats


def _stable_eps(method, c, nsteps, kmin, cap, eps_list, deepest):
    """A tolerance whose oracle counts do not move when it changes by 10 %
    and that stops some stage strictly between kmin and cap, after at least
    `deepest` sweeps."""
    for eps in eps_list:
        used = _oracle(method, c, nsteps, eps, kmin, cap)[3]
        if not any(deepest <= u < cap for u in used):
            continue
        lo = _oracle(method, c, nsteps, eps / 1.1, kmin, cap)[3]
        hi = _oracle(method, c, nsteps, eps * 1.1, kmin, cap)[3]
        if np.array_equal(used, lo) and np.array_equal(used, hi):
            return eps, used
    raise AssertionError("no stable tolerance found")


@pytest.mark.parametrize("size", [0, 1, 2])
@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
@pytest.mark.parametrize("dtype", [adi.FP64, adi.FP32])
def test_tolerance_matches_oracle(method, dtype, size):
    nsteps, kmin, cap = 2, 2, 12
    c = _case(method, 11, size)
    # FP32 iterates carry rounding noise of ~1e-7 of the fields: test well above it
    eps_list = [x * s for x in (10.0, 1.0, 0.1, 0.01) for s in (3, 1)]
    if dtype == adi.FP64:
        eps_list += [x * s for x in (1e-3, 1e-4, 1e-5) for s in (3, 1)]
    eps, used = _stable_eps(method, c, nsteps, kmin, cap, eps_list, 6 if dtype == adi.FP64 else 4)
    log(f"case tolerance method={method} dtype={dtype} size={SIZES[method][size]} eps={eps:.3g} "
        f"counts={list(used)}")
    ref = _oracle(method, c, nsteps, eps, kmin, cap)
    got, (passes, sweeps) = _gpu(method, dtype, c, nsteps, cap, eps, kmin)
    assert passes == 2 * nsteps and sweeps == int(used.sum()), (passes, sweeps, list(used))
    for g, r in zip(written_parts(method, *got), written_parts(method, *ref[:3])):
        err = max_rel(g, r) if dtype == adi.FP64 else rel_l2(g, r)
        assert err <= (TOL64 if dtype == adi.FP64 else TOL32), err


@pytest.mark.parametrize("size", [0, 1])
@pytest.mark.parametrize("method", [adi.CFD, adi.MFD])
def test_tolerance_limits_equal_fixed_runs(method, size):
    """Every change passes: each stage stops at min_sweeps; none passes: each
    runs the cap.  Both equal the fixed-count runs: bit for bit at the cap;
    to rounding at min_sweeps, whose fixed run plans its windows with the
    margin of min_sweeps sweeps rather than of the cap."""
    nsteps, kmin, cap = 2, 4, 8
    c = _case(method, 12, size)
    for eps, k in ((1e30, kmin), (1e-300, cap)):
        log(f"case tolerance limit method={method} eps={eps:g}")
        got, (passes, sweeps) = _gpu(method, adi.FP64, c, nsteps, cap, eps, kmin)
        ref, _ = _gpu(method, adi.FP64, c, nsteps, k)
        assert (passes, sweeps) == (2 * nsteps, 2 * nsteps * k)
        for g, r in zip(got, ref):
            if k == cap:
                assert np.array_equal(g, r)
            else:
                assert max_rel(g, r) <= TOL64


def test_tolerance_scope_errors():
    import torch
    c = _case(adi.CFD, 13)
    log("case tolerance scope errors")
    # the compensated mode has no tolerance test
    f = inputs.random_fields(adi.CFD, 100, 90, 1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", torch.float64)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", torch.float32)
    p = adi.make_params(adi.CFD, adi.FP32C, 100, 90, 0.01, 0.005, 1.0)
    pb = adi.Problem(p).bind(t32(f["U"]), t32(f["V"]), t32(f["W"]))
    with pytest.raises(RuntimeError, match="FP32 or FP64"):
        pb.set_tolerance(1e-6, 2)
    assert pb.sweep_stats() == (0, 0)
    pb.close()
    # argument ranges, and batches refuse such a problem
    nx, ny = SIZES[adi.CFD][0]
    p = adi.make_params(adi.CFD, adi.FP64, nx, ny, c["h"], c["dt"], c["cmax"], sweeps=8)
    U, V, W = (t(c["f"][k]) for k in "UVW")
    pb = adi.Problem(p).bind(U, V, W)
    for eps, k in ((-1.0, 2), (float("nan"), 2), (1e-6, 3), (1e-6, 0), (1e-6, 10)):
        with pytest.raises(RuntimeError):
            pb.set_tolerance(eps, k)
    pb.set_tolerance(1e-6, 2)
    with pytest.raises(RuntimeError, match="tolerance"):
        adi.Batch([pb])
    pb.set_tolerance(0.0)
    b = adi.Batch([pb])
    b.close()
    pb.close()
