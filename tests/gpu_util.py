"""Helpers for the GPU tests: run the HIP library through the C ABI binding
on numpy inputs and compare with the oracle."""
import sys

import numpy as np

from paper_2006_07583_amd import adi


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(method, dtype, fields, *, h, dt, c_max, nsteps, sweeps=6, K=None, Rv=None, Rw=None,
            src=None, t0=0.0, kappa0=1.0, rinv0=1.0, chunks=None, order=0):
    """Copy (U, V, W, materials) to the GPU, run nsteps (optionally split into
    the given chunk sizes), return float64 numpy copies of U, V, W."""
    import torch
    tdt = torch.float64 if dtype == adi.FP64 else torch.float32
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev, tdt)
    U, V, W = t(fields["U"]), t(fields["V"]), t(fields["W"])
    ny = U.shape[0] - (1 if method == adi.CFD else 2)
    nx = U.shape[1] - (1 if method == adi.CFD else 2)
    p = adi.make_params(method, dtype, nx, ny, h, dt, c_max, sweeps=sweeps, src=src, t0=t0,
                        kappa0=kappa0, rinv0=rinv0, order=order)
    pb = adi.Problem(p).bind(U, V, W, t(K), t(Rv), t(Rw))
    for c in (chunks or [nsteps]):
        pb.run(c)
    pb.get_state()
    out = tuple(x.double().cpu().numpy() for x in (U, V, W))
    pb.close()
    return out


def written_parts(method, U, V, W):
    """The entries the method updates: interior U, interior rows of V,
    interior columns of W."""
    return U[1:-1, 1:-1], V[1:-1, :], W[:, 1:-1]


def max_rel(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def rel_l2(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
