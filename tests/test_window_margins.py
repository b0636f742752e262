"""Model of the window margins of the sweep kernels (host only).

The multi-window line passes cut every line into windows of 512 slots that
overlap by H slots on each side and write only their central slots.  A
window sees nothing beyond its edges: its derivative stencils drop the
outside neighbours and its compact solves start from the interior pivot
2 + sqrt 3 at the window's first row.  This model runs one line pass (the
sweeps of one stage and the explicit part of the next, as in the kernels)
once on a whole line, with the oracle's dense operators, and once on a
window cut out of it, and measures the error of the window's outputs against
the distance from its edges.

Compact operators couple the whole line, so the error decays geometrically
(like (2 - sqrt 3)^d times a polynomial from the 2K + 1 chained solves) and
the margin sets the truncation level: the kernels plan 18 + 2K slots in FP32
and, in FP64 and the compensated mode, 36 + 2K slots up to cfl 0.85 and
40 + 3K above.  Mimetic operators have finite stencils: K sweeps and the
final derivative reach 3K + 2 slots, and the kernels' 3K + 4 make the
windowed pass exact."""
import math

import numpy as np
import pytest
from scipy.linalg import solve_banded

import oracle as O

DELTA = 2.0 + math.sqrt(3.0)
WS = 512


def halo(dtype, method, sweeps, cfl):
    """The margins the line passes plan (dtype 0 = FP32, 1 = FP64, 2 =
    compensated FP32)."""
    if method == O.MFD:
        return 3 * sweeps + 4
    if dtype == 0:
        return 18 + 2 * sweeps
    return 36 + 2 * sweeps if cfl <= 0.85 else 40 + 3 * sweeps


def _tri(M):
    """Banded storage of a tridiagonal matrix."""
    n = M.shape[0]
    ab = np.zeros((3, n))
    ab[0, 1:] = np.diag(M, 1)
    ab[1] = np.diag(M)
    ab[2, :-1] = np.diag(M, -1)
    return ab


class LineOps:
    """G (pressure line -> velocity) and D (velocity -> interior pressure)
    of one method on the velocity slots [lo, hi) of a line of n cells;
    lo = 0, hi = n + 1 is the whole line, anything else a window whose
    coupling to the outside is dropped."""

    def __init__(self, method, n, h, lo=0, hi=None):
        hi = n + 1 if hi is None else hi
        self.method = method
        if method == O.CFD:
            P, Q, Pb, Qb = O.cfd_matrices(n, h)
            P, Q = P[lo:hi, lo:hi].copy(), Q[lo:hi, lo:hi]
            p0 = max(lo, 1)
            Pb, Qb = Pb[p0 - 1:hi - 1, p0 - 1:hi - 1].copy(), Qb[p0 - 1:hi - 1, lo:hi]
            if lo > 0:                      # a window edge inside the line
                P[0, 0] = DELTA
                Pb[0, 0] = DELTA
            self.P, self.Q, self.Pb, self.Qb = _tri(P), Q, _tri(Pb), Qb
            self.full = lo == 0             # G reads the boundary pressure slots
        else:
            D, G = O.mfd_matrices(n, h)
            self.D, self.G = D[max(lo, 1) - 1:hi - 1, lo:hi], G[lo:hi, lo:hi + 1 if hi == n + 1 else hi]
            self.full = lo == 0

    def grad(self, u):
        """u: interior pressure of the slots; the whole line adds the two
        (zero) Dirichlet values."""
        if self.full:
            u = np.concatenate([[0.0], u, [0.0]])
        if self.method == O.CFD:
            return solve_banded((1, 1), self.P, self.Q @ u)
        return self.G @ u

    def div(self, v):
        if self.method == O.CFD:
            return solve_banded((1, 1), self.Pb, self.Qb @ v)
        return self.D @ v


def line_pass(ops, A, B, aK, aR, sweeps):
    """Sweeps of one stage and the explicit part of the next, as one line
    pass of the kernels computes them: outputs 2 v_K - B and
    u_K - aK D(v_K)."""
    u = A - aK * ops.div(B)
    for _ in range(sweeps - 1):
        u = A - aK * ops.div(B - aR * ops.grad(u))
    v = B - aR * ops.grad(u)
    return 2 * v - B, u - aK * ops.div(v)


def window_error(method, cfl, sweeps, n=1000, lo=250, seed=0):
    """Largest relative error of a window's outputs at distance >= d from
    its edges, for every d (array indexed by d)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    a = 0.5 * cfl * h                      # c_max = 1: kappa and 1/rho up to 1
    nu = n - 1 if method == O.CFD else n
    A, B = rng.standard_normal(nu), rng.standard_normal(n + 1)
    aK, aR = a * rng.uniform(0.25, 1.0, nu), a * rng.uniform(0.25, 1.0, n + 1)
    aK[nu // 2] = aR[n // 2] = a           # the largest material value, inside the window
    vo, uo = line_pass(LineOps(method, n, h), A, B, aK, aR, sweeps)
    hi = lo + WS
    off = 1 if method == O.CFD else 1      # interior pressure slot s sits at index s - 1
    sl_u = slice(lo - off, hi - off)
    vw, uw = line_pass(LineOps(method, n, h, lo, hi), A[sl_u], B[lo:hi], aK[sl_u], aR[lo:hi], sweeps)
    e = np.maximum(np.abs(vw - vo[lo:hi]) / np.abs(vo).max(), np.abs(uw - uo[sl_u]) / np.abs(uo).max())
    dist = np.minimum(np.arange(WS), WS - 1 - np.arange(WS))
    return np.array([e[dist >= d].max() for d in range(WS // 2)])


@pytest.mark.parametrize("sweeps", [2, 4, 6, 8, 12, 16])
@pytest.mark.parametrize("cfl", [0.5, 0.8, 0.85, 1.0, 1.149])
def test_compact_margins(sweeps, cfl):
    """At the planned margin the truncation stays below the FP32 rounding
    unit 2^-24 (FP32) and at the FP64 rounding level (FP64, compensated)."""
    e = window_error(O.CFD, cfl, sweeps)
    assert e[halo(0, O.CFD, sweeps, cfl)] <= 2.0 ** -24, e[halo(0, O.CFD, sweeps, cfl)]
    assert e[halo(1, O.CFD, sweeps, cfl)] <= 1e-15, e[halo(1, O.CFD, sweeps, cfl)]
    # the model sees the truncation near the window edges
    assert e[8] > 1e-7


@pytest.mark.parametrize("sweeps", [2, 6, 16])
@pytest.mark.parametrize("cfl", [0.5, 0.809])
def test_mimetic_margins_cover_the_dependence_cone(sweeps, cfl):
    """The margin covers the cone: the windowed outputs there are bit for bit
    those of the whole line (the truncation error also decays geometrically
    inside the cone and reaches the rounding level some slots before it)."""
    e = window_error(O.MFD, cfl, sweeps)
    H = halo(0, O.MFD, sweeps, cfl)
    assert H >= 3 * sweeps + 2
    assert e[3 * sweeps + 2] == 0.0 and e[H] == 0.0, (e[3 * sweeps + 2], e[H])
    assert e[2] > 1e-6
