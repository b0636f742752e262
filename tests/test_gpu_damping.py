"""Absorbing damping layers on the GPU (adi_set_damping: the damped system,
each implicit line system divided by 1 + a d, each explicit part multiplied
by 1 - a d) against the oracle's damped mode, in single problems and in a
batch.

Bar: FP64 max|gpu - oracle| / max|oracle| <= 1e-12 per field; FP32 relative
L2 <= 1e-4 per field after all steps."""
import math

import torch

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import adi, inputs
from tests.gpu_util import log, max_rel, rel_l2, written_parts

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-4


def setup(method, nx, ny, seed):
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 1)
    cmax = math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    src = {"i": nx // 3, "j": ny // 2, "f0": 4.0, "t0": 0.1, "amp": 1.0}
    return h, f, med, cmax, src


def gpu_damped(method, dtype, f, med, *, h, dt, cmax, src, d0, width, walls, chunks, order=0, stream=None):
    tdt = torch.float64 if dtype == adi.FP64 else torch.float32
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", tdt)
    U, V, W = t(f["U"]), t(f["V"]), t(f["W"])
    ny = U.shape[0] - (1 if method == adi.CFD else 2)
    nx = U.shape[1] - (1 if method == adi.CFD else 2)
    p = adi.make_params(method, dtype, nx, ny, h, dt, cmax, src=src, order=order)
    pb = adi.Problem(p, stream).set_damping(d0, width, walls).bind(U, V, W, t(med["K"]), t(med["Rv"]), t(med["Rw"]))
    for c in chunks:
        pb.run(c)
    return pb, (U, V, W)


CASES = [(m, d, nx, ny, o, walls) for m in (adi.CFD, adi.MFD)
         for (nx, ny) in ((33, 20), (100, 77), (600, 90), (530, 520))
         for d, o, walls in ((adi.FP64, 0, 15), (adi.FP64, 1, 11), (adi.FP32, 0, 11))]


@pytest.mark.parametrize("method,dtype,nx,ny,order,walls", CASES)
def test_damping_matches_oracle(method, dtype, nx, ny, order, walls):
    """Layers 12 cells wide (rate 40 at the walls, a d up to 0.2), on all
    walls or all but the top (a free surface), run as 2 + 2 steps."""
    h, f, med, cmax, src = setup(method, nx, ny, 7 * nx + ny + walls)
    dt = 0.6 * h / cmax
    log(f"case damped method={method} dtype={dtype} {nx}x{ny} order={order} walls={walls}")
    ref = O.run_damped(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=4, d0=40.0 * max(nx, ny) / 100.0,
                       width=12, walls=walls, K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src, order=order)
    pb, x = gpu_damped(method, dtype, f, med, h=h, dt=dt, cmax=cmax, src=src, d0=40.0 * max(nx, ny) / 100.0,
                       width=12, walls=walls, chunks=[2, 2], order=order)
    pb.get_state()
    got = tuple(a.double().cpu().numpy() for a in x)
    pb.close()
    errs = [max_rel(g, r) if dtype == adi.FP64 else rel_l2(g, r)
            for g, r in zip(written_parts(method, *got), written_parts(method, *ref))]
    log(f"  errors U,V,W = {errs}")
    assert max(errs) <= (TOL64 if dtype == adi.FP64 else TOL32), errs


def test_damped_problems_in_a_batch_equal_solo_runs():
    st = torch.cuda.Stream()
    mix = [(adi.CFD, adi.FP32, 90, 60), (adi.MFD, adi.FP64, 600, 80), (adi.MFD, adi.FP32, 530, 520)]
    solo, batched = [], []
    for i, (m, d, nx, ny) in enumerate(mix):
        h, f, med, cmax, src = setup(m, nx, ny, 50 + i)
        kw = dict(h=h, dt=0.6 * h / cmax, cmax=cmax, src=src, d0=30.0, width=10, walls=11, stream=st)
        solo.append(gpu_damped(m, d, f, med, chunks=[5], **kw))
        batched.append(gpu_damped(m, d, f, med, chunks=[], **kw))
    b = adi.Batch([pb for pb, _ in batched], st, graph=True)
    b.run(5)
    b.sync()
    for (pa, xa), (pbb, xb) in zip(solo, batched):
        pa.get_state()
        pbb.get_state()
        for u, v in zip(xa, xb):
            assert torch.equal(u, v)
    b.close()


def test_damping_scope():
    n = 64
    for dtype, sweeps in ((adi.FP32C, 6), (adi.FP64, 0)):
        p = adi.make_params(adi.MFD, dtype, n, n, 1 / n, 0.5 / n, 1.0, sweeps=sweeps)
        pb = adi.Problem(p)
        with pytest.raises(adi.AdiError):
            pb.set_damping(10.0, 8, 15)
        pb.set_damping(0.0, 8, 15)      # off is always allowed
        pb.close()
