"""Served problems (adi_server_*): each request's result, returned in its own
host arrays, equals bit for bit the same problem run alone with adi_run and
matches the oracle; admission respects the memory budget and the
active-problem bound."""
import math

import torch  # noqa: F401  (first import on a fresh box is slow)

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import adi, inputs
from tests.gpu_util import log, max_rel, rel_l2, run_gpu, written_parts

pytestmark = pytest.mark.gpu

# (method, dtype, nx, ny, order, nsteps): single- and multi-window lines, all dtypes
MIX = [
    (adi.CFD, adi.FP32, 40, 60, 0, 7),
    (adi.MFD, adi.FP32, 130, 90, 0, 12),
    (adi.CFD, adi.FP64, 70, 33, 1, 5),
    (adi.MFD, adi.FP64, 520, 40, 0, 4),
    (adi.CFD, adi.FP32, 600, 80, 0, 9),
    (adi.MFD, adi.FP32C, 64, 64, 1, 6),
    (adi.CFD, adi.FP32C, 90, 48, 0, 3),
    (adi.MFD, adi.FP32, 8, 8, 0, 15),
    (adi.CFD, adi.FP64, 255, 20, 0, 11),
    (adi.MFD, adi.FP32, 300, 520, 1, 2),
]


def request(method, dtype, nx, ny, order, nsteps, seed):
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 1)
    cmax = math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    dt = 0.6 * h / cmax
    src = {"i": max(1, nx // 3), "j": max(1, ny // 2), "f0": 4.0, "t0": 0.1, "amp": 1.0}
    npdt = np.float64 if dtype == adi.FP64 else np.float32
    arrs = {k: np.array(f[k], dtype=npdt) for k in ("U", "V", "W")}   # copies: results overwrite them
    mats = {k: np.ascontiguousarray(med[k], dtype=npdt) for k in ("K", "Rv", "Rw")}
    p = adi.make_params(method, dtype, nx, ny, h, dt, cmax, src=src, order=order)
    return dict(p=p, arrs=arrs, mats=mats, h=h, dt=dt, cmax=cmax, src=src, nsteps=nsteps, order=order, f=f,
                med=med)


def solo(method, dtype, rq):
    return run_gpu(method, dtype, {k: v.astype(np.float64) for k, v in rq["arrs"].items()},
                   h=rq["h"], dt=rq["dt"], c_max=rq["cmax"], nsteps=rq["nsteps"],
                   K=rq["mats"]["K"].astype(np.float64), Rv=rq["mats"]["Rv"].astype(np.float64),
                   Rw=rq["mats"]["Rw"].astype(np.float64), src=rq["src"], order=rq["order"])


@pytest.mark.parametrize("budget,max_active", [(2 << 30, 6), (12 << 20, 64)])
def test_served_results_equal_solo_runs(budget, max_active):
    reqs = [request(*m, seed=300 + 5 * i) for i, m in enumerate(MIX)]
    ref = [solo(m[0], m[1], rq) for m, rq in zip(MIX, reqs)]
    log(f"server budget={budget} max_active={max_active}, {len(reqs)} requests")
    srv = adi.Server(hbm_budget_bytes=budget, max_active=max_active)
    tickets = [srv.submit(rq["p"], rq["arrs"]["U"], rq["arrs"]["V"], rq["arrs"]["W"],
                          rq["mats"]["K"], rq["mats"]["Rv"], rq["mats"]["Rw"], nsteps=rq["nsteps"])
               for rq in reqs]
    for t in tickets:
        srv.wait(t)
        assert srv.poll(t) == 2
    st = srv.stats()
    log(f"  stats {st}")
    assert st["done"] == len(reqs) and st["arena_used"] == 0 and st["queued"] == 0
    assert 1 <= st["peak_active"] <= max_active
    for i, (rq, r) in enumerate(zip(reqs, ref)):
        ts, t1, t2 = srv.times(tickets[i])
        assert 0 <= ts <= t1 <= t2
        for name, got, want in zip("UVW", (rq["arrs"][k] for k in "UVW"), r):
            assert np.array_equal(got.astype(np.float64), want), (i, MIX[i], name)
        f, med = rq["f"], rq["med"]
        oref = O.run(MIX[i][0], f["U"], f["V"], f["W"], h=rq["h"], dt=rq["dt"], nsteps=rq["nsteps"], sweeps=6,
                     K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=rq["src"], order=rq["order"])
        got = [rq["arrs"][k].astype(np.float64) for k in "UVW"]
        for g, o in zip(written_parts(MIX[i][0], *got), written_parts(MIX[i][0], *oref)):
            err = max_rel(g, o) if MIX[i][1] == adi.FP64 else rel_l2(g, o)
            assert err <= (1e-12 if MIX[i][1] == adi.FP64 else 1e-4), (i, MIX[i], err)
    srv.close()
