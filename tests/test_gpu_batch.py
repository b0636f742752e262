"""Batched runs (adi_batch_*): every problem of a mixed batch must come out
bit for bit equal to the same problem run alone with adi_run, with and
without graph replay, and across consecutive runs, and match the oracle
(FP64 max-relative 1e-12, FP32 relative L2 1e-4 per field)."""
import math

import torch

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import adi, inputs
from tests.gpu_util import log, max_rel, rel_l2, written_parts

pytestmark = pytest.mark.gpu

# (method, dtype, nx, ny, order): every single-window tile shape, the
# multi-window kernel, both orders, all dtypes
MIX = [
    (adi.CFD, adi.FP32, 60, 90, 0),
    (adi.MFD, adi.FP32, 70, 41, 0),
    (adi.CFD, adi.FP32, 200, 130, 0),
    (adi.MFD, adi.FP32, 300, 250, 1),
    (adi.CFD, adi.FP32, 600, 140, 0),
    (adi.MFD, adi.FP32, 530, 520, 0),
    (adi.CFD, adi.FP64, 90, 300, 0),
    (adi.MFD, adi.FP64, 520, 64, 1),
    (adi.CFD, adi.FP32C, 100, 120, 0),
    (adi.MFD, adi.FP32C, 140, 96, 1),
    (adi.CFD, adi.FP32, 8, 8, 1),
]


def make(method, dtype, nx, ny, order, seed, stream):
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 1)
    cmax = math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    dt = 0.6 * h / cmax
    src = {"i": max(1, nx // 3), "j": max(1, ny // 2), "f0": 4.0, "t0": 0.1, "amp": 1.0}
    tdt = torch.float64 if dtype == adi.FP64 else torch.float32
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", tdt)
    arrs = [t(f[k]) for k in ("U", "V", "W")]
    mats = [t(med[k]) for k in ("K", "Rv", "Rw")]
    p = adi.make_params(method, dtype, nx, ny, h, dt, cmax, src=src, order=order)
    pb = adi.Problem(p, stream).bind(*arrs, *mats)
    pb.inputs = dict(h=h, dt=dt, f=f, med=med, src=src, order=order)
    return pb, arrs


def build(seed0, stream):
    return [make(*m, seed=seed0 + 3 * i, stream=stream) for i, m in enumerate(MIX)]


@pytest.mark.parametrize("graph,one_stream", [(False, False), (True, False), (True, True)])
def test_batch_equals_individual_runs_bitwise(graph, one_stream):
    st = torch.cuda.Stream()
    alone = build(100, st)
    batch = build(100, st)
    chunks = [7, 2, 1, 4]
    log(f"batch of {len(MIX)} problems, graph={graph}, chunks={chunks}")
    for pb, _ in alone:
        for c in chunks:
            pb.run(c)
        pb.get_state()
    b = adi.Batch([pb for pb, _ in batch], st, graph=graph, one_stream=one_stream)
    for c in chunks:
        b.run(c)
    b.sync()
    for pb, _ in batch:
        pb.get_state()
    torch.cuda.synchronize()
    for i, ((pa, xa), (pbb, xb)) in enumerate(zip(alone, batch)):
        assert pa.step_index == pbb.step_index == sum(chunks)
        for name, u, v in zip("UVW", xa, xb):
            assert torch.equal(u, v), (i, MIX[i], name, float((u - v).abs().max()))
    b.close()


def test_batch_launch_count_is_per_variant_not_per_problem():
    st = torch.cuda.Stream()
    probs = build(200, st)
    b = adi.Batch([pb for pb, _ in probs], st)
    b.run(6)
    b.sync()
    n = b.launches
    log(f"grouped launches for 6 steps of {len(MIX)} problems: {n}")
    # at most one launch per variant per half-step; far fewer than one per pass
    assert 12 <= n < 6 * 2 * len(MIX)
    b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle(graph):
    """Every problem of the mixed batch (all tile shapes, both kernels of
    long lines, both orders, FP64, FP32 and compensated FP32) against the
    oracle after two batched runs."""
    st = torch.cuda.Stream()
    probs = build(400, st)
    b = adi.Batch([pb for pb, _ in probs], st, graph=graph)
    for c in (5, 4):
        b.run(c)
    b.sync()
    for i, (pb, arrs) in enumerate(probs):
        pb.get_state()
        x = pb.inputs
        ref = O.run(MIX[i][0], x["f"]["U"], x["f"]["V"], x["f"]["W"], h=x["h"], dt=x["dt"], nsteps=9, sweeps=6,
                    K=x["med"]["K"], Rv=x["med"]["Rv"], Rw=x["med"]["Rw"], src=x["src"], order=x["order"])
        got = [t.double().cpu().numpy() for t in arrs]
        for g, r in zip(written_parts(MIX[i][0], *got), written_parts(MIX[i][0], *ref)):
            err = max_rel(g, r) if MIX[i][1] == adi.FP64 else rel_l2(g, r)
            assert err <= (1e-12 if MIX[i][1] == adi.FP64 else 1e-4), (i, MIX[i], err)
    b.close()
