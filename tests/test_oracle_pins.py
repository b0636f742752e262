"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: the references are the printed
coefficients (Appendices A/B, via tests/golden), Taylor moments, LAPACK on the
dense matrices, a dense Kronecker assembly of the split (eqs. A1HA2H,
ecua2:PR, ecua3:PR2), the exact standing-wave solution and the closed-form
Peaceman-Rachford amplification of a single mode.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2006_07583_amd import inputs
from tests.dense_pr import DenseProblem

GOLD = os.path.join(os.path.dirname(__file__), "golden", "operators_appendix.json")


def frac(rows):
    return np.array([p / q for p, q in rows])


@pytest.fixture(scope="module")
def printed():
    with open(GOLD) as f:
        return {k: frac(v) for k, v in json.load(f).items() if not k.startswith("_")}


# ---------------------------------------------------------------- P1 operators

def test_cfd_operators_match_printed_rows(printed):
    n, h = 12, 1.0
    P, Q, Pb, Qb = O.cfd_matrices(n, h)
    assert np.array_equal(P[0, :2], printed["P4_row0"])
    assert np.array_equal(P[n, n - 1:], printed["P4_rowN"])
    assert np.array_equal(Q[0, :4], printed["Q4_row0"])
    assert np.array_equal(Q[n, n - 3:], printed["Q4_rowN"])
    for i in range(1, n):
        assert np.array_equal(P[i, i - 1:i + 2], printed["P4_interior"])
        assert np.array_equal(Q[i, i - 1:i + 2], printed["Q4_interior"])
    assert np.array_equal(Pb[0, :2], printed["Pbar4_row0"])
    assert np.array_equal(Pb[-1, -2:], printed["Pbar4_rowlast"])
    assert np.array_equal(Qb[0, :4], printed["Qbar4_row0"])
    assert np.array_equal(Qb[-1, -4:], printed["Qbar4_rowlast"])
    # the reduced first row removes f'_0 from row0 - 6 row1 of (P, Q) (Appendix A)
    assert np.array_equal(-(P[0, :3] - 6 * P[1, :3])[1:], Pb[0, :2])
    assert np.array_equal(-(Q[0, :4] - 6 * Q[1, :4]), Qb[0, :4])


def test_mfd_operators_match_printed_rows(printed):
    n, h = 12, 1.0
    D, G = O.mfd_matrices(n, h)
    assert np.allclose(D[0, :6], printed["D4_row0"], rtol=0, atol=1e-16)
    assert np.allclose(G[0, :6], printed["G4_row0"], rtol=0, atol=1e-15)
    assert np.allclose(G[1, :5], printed["G4_row1"], rtol=0, atol=1e-16)
    for r in range(1, n - 1):
        assert np.allclose(D[r, r - 1:r + 3], printed["D4_interior"], rtol=0, atol=1e-16)
    for r in range(2, n - 1):
        assert np.allclose(G[r, r - 1:r + 3], printed["G4_interior"], rtol=0, atol=1e-16)
    # bottom rows are the centro-skew mirror of the printed top rows
    assert np.array_equal(D[::-1, ::-1], -D)
    assert np.array_equal(G[::-1, ::-1], -G)


@pytest.mark.parametrize("n", [8, 13, 32])
def test_cfd_operators_are_fourth_order_exact(n):
    """P f' = Q f holds exactly for monomials of degree <= 4 on every row,
    boundary rows included, and fails at degree 5 (unit spacing)."""
    P, Q, Pb, Qb = O.cfd_matrices(n, 1.0)
    x = np.arange(n + 1, dtype=np.float64) / n     # scale to [0, 1] for conditioning
    P, Q, Pb, Qb = O.cfd_matrices(n, 1.0 / n)
    for p in range(6):
        f = x ** p
        fp = p * x ** (p - 1) if p else np.zeros_like(x)
        r = P @ fp - Q @ f
        rb = Pb @ fp[1:n] - Qb @ f
        if p <= 4:
            assert np.abs(r).max() < 1e-10 and np.abs(rb).max() < 1e-10, p
        else:
            assert np.abs(r).max() > 1e-6 and np.abs(rb).max() > 1e-6


@pytest.mark.parametrize("n", [8, 13, 32])
def test_mfd_operators_are_fourth_order_exact(n):
    h = 1.0 / n
    D, G = O.mfd_matrices(n, h)
    xn = inputs.node_coords(n, h)
    xc = inputs.cb_coords(n, h)
    for p in range(6):
        dv = D @ xn ** p - (p * xc[1:-1] ** (p - 1) if p else 0.0)
        gu = G @ xc ** p - (p * xn ** (p - 1) if p else 0.0)
        if p <= 4:
            assert np.abs(dv).max() < 1e-9 and np.abs(gu).max() < 1e-9, p
        else:
            assert np.abs(dv).max() > 1e-6 and np.abs(gu).max() > 1e-6


# ---------------------------------------------------------------- P2 line solves

def test_thomas_pivots_closed_form():
    """No-pivot LU of P and Pbar: pivots 6, 1, 3, 11/3, ... -> 2 + sqrt 3,
    last pivot 6 - 18/d; Pbar: 6, 3, 11/3, ... -> 6 sqrt 3 - 6 at the end."""
    n = 40
    pP, pB = O.cfd_pivots(n)
    assert pP[0] == 6.0 and pP[1] == 1.0 and pP[2] == 3.0
    assert abs(pP[3] - 11.0 / 3.0) < 1e-15
    assert abs(pP[n - 1] - (2 + math.sqrt(3))) < 1e-14
    assert abs(pP[n] - (6 - 18 / (2 + math.sqrt(3)))) < 1e-13
    assert pB[0] == 6.0 and pB[1] == 3.0
    assert abs(pB[-1] - (6 * math.sqrt(3) - 6)) < 1e-13
    assert (pP > 0).all() and (pB > 0).all()


@pytest.mark.parametrize("n", [8, 9, 31, 64])
def test_line_derivatives_match_lapack(n):
    rng = np.random.default_rng(n)
    h = 1.0 / n
    P, Q, Pb, Qb = O.cfd_matrices(n, h)
    f = rng.standard_normal(n + 1)
    ref = np.linalg.solve(P, Q @ f)
    got = O.cfd_d(f, h)
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
    refb = np.linalg.solve(Pb, Qb @ f)
    gotb = O.cfd_dbar(f, h)
    assert np.abs(gotb - refb).max() <= 1e-14 * np.abs(refb).max()
    D, G = O.mfd_matrices(n, h)
    u = rng.standard_normal(n + 2)
    assert np.abs(O.mfd_g(u, h) - G @ u).max() <= 1e-13 * np.abs(G @ u).max()
    assert np.abs(O.mfd_d(f, h) - D @ f).max() <= 1e-13 * np.abs(D @ f).max()


# ---------------------------------------------------------------- P3 accuracy

def _rate(errs, ns):
    return [math.log(errs[k] / errs[k + 1]) / math.log(ns[k + 1] / ns[k]) for k in range(len(ns) - 1)]


def _trimmed(rates):
    """Rate summary of Section 4: mean after dropping the highest and lowest."""
    r = sorted(rates)
    return sum(r[1:-1]) / len(r[1:-1])


def test_line_derivatives_fourth_order_under_refinement():
    ns = [16, 32, 64, 128]
    e = {"d": [], "dbar": [], "g": [], "D": []}
    for n in ns:
        h = 1.0 / n
        x = inputs.node_coords(n, h)
        xc = inputs.cb_coords(n, h)
        f = np.sin(2.3 * x + 0.4)
        e["d"].append(np.abs(O.cfd_d(f, h) - 2.3 * np.cos(2.3 * x + 0.4)).max())
        e["dbar"].append(np.abs(O.cfd_dbar(f, h) - 2.3 * np.cos(2.3 * x[1:n] + 0.4)).max())
        e["g"].append(np.abs(O.mfd_g(np.sin(2.3 * xc + 0.4), h) - 2.3 * np.cos(2.3 * x + 0.4)).max())
        e["D"].append(np.abs(O.mfd_d(f, h) - 2.3 * np.cos(2.3 * xc[1:-1] + 0.4)).max())
    for k, v in e.items():
        r = _rate(v, ns)
        assert min(r) > 3.7, (k, r)


# ---------------------------------------------------------------- P4 stage semantics

def _dense_for(method, nx, ny, h, a, K, Rv, Rw):
    if method == O.CFD:
        _, _, Pbx, Qbx = O.cfd_matrices(nx, h)
        Px, Qx, _, _ = O.cfd_matrices(nx, h)
        Py, Qy, Pby, Qby = O.cfd_matrices(ny, h)
        Dx, Gx = np.linalg.solve(Pbx, Qbx), np.linalg.solve(Px, Qx)
        Dy, Gy = np.linalg.solve(Pby, Qby), np.linalg.solve(Py, Qy)
    else:
        Dx, Gx = O.mfd_matrices(nx, h)
        Dy, Gy = O.mfd_matrices(ny, h)
    return DenseProblem(Dx, Gx, Dy, Gy, nx, ny, method,
                        K[1:-1, 1:-1], Rv[1:-1, :], Rw[:, 1:-1], a)


def _tiny_case(method, nx, ny, seed, with_src=True):
    h = 1.0 / max(nx, ny)
    f = inputs.random_fields(method, nx, ny, seed)
    med = inputs.random_medium(method, nx, ny, seed + 100)
    src = None
    if with_src:
        src = {"i": nx // 2, "j": ny // 3, "f0": 3.0, "t0": 0.2, "amp": 1.0}
    return h, f, med, src


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
@pytest.mark.parametrize("nx,ny", [(8, 8), (9, 12), (12, 10)])
def test_step_converged_sweeps_match_dense_lu(method, nx, ny):
    """64 sweeps (contraction <= 0.375 at cfl 0.5) reproduce the exactly
    solved stages of eqs. ecua2:PR / ecua3:PR2 assembled densely."""
    h, f, med, src = _tiny_case(method, nx, ny, 7 + nx + 3 * ny)
    kmax = med["K"].max() * max(med["Rv"].max(), med["Rw"].max())
    dt = 0.5 * h / math.sqrt(kmax)
    t0 = 0.05
    U, V, W = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=1, sweeps=64,
                    K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src, t0=t0)
    dp = _dense_for(method, nx, ny, h, dt / 2, med["K"], med["Rv"], med["Rw"])
    Fm = np.zeros((dp.niy, dp.nix)); Fm1 = np.zeros_like(Fm)
    Fm[src["j"] - 1, src["i"] - 1] = O.source_value(src, h, t0)
    Fm1[src["j"] - 1, src["i"] - 1] = O.source_value(src, h, t0 + dt)
    z = dp.pack(f["U"][1:-1, 1:-1], f["V"][1:-1, :], f["W"][:, 1:-1])
    Ue, Ve, We = dp.unpack(dp.step_exact(z, Fm, Fm1))
    for got, ref in ((U[1:-1, 1:-1], Ue), (V[1:-1, :], Ve), (W[:, 1:-1], We)):
        assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1.0)
    # entries the method never writes keep their values
    assert np.array_equal(U[0], f["U"][0]) and np.array_equal(U[:, -1], f["U"][:, -1])
    assert np.array_equal(V[0], f["V"][0]) and np.array_equal(V[-1], f["V"][-1])
    assert np.array_equal(W[:, 0], f["W"][:, 0]) and np.array_equal(W[:, -1], f["W"][:, -1])


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
@pytest.mark.parametrize("sweeps", [2, 6])
def test_finite_sweeps_match_dense_iteration(method, sweeps):
    """At a fixed sweep count the oracle equals the matrix form of eqs.
    adiSolve / adiSolve2 (V_0 = V^m, W_0 = W*), over three steps."""
    nx, ny = 11, 9
    h, f, med, src = _tiny_case(method, nx, ny, 3)
    dt = 0.8 * h / math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    U, V, W = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=3, sweeps=sweeps,
                    K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src)
    dp = _dense_for(method, nx, ny, h, dt / 2, med["K"], med["Rv"], med["Rw"])
    z = dp.pack(f["U"][1:-1, 1:-1], f["V"][1:-1, :], f["W"][:, 1:-1])
    for m in range(3):
        Fm = np.zeros((dp.niy, dp.nix)); Fm1 = np.zeros_like(Fm)
        Fm[src["j"] - 1, src["i"] - 1] = O.source_value(src, h, m * dt)
        Fm1[src["j"] - 1, src["i"] - 1] = O.source_value(src, h, (m + 1) * dt)
        z = dp.step_sweeps(z, Fm, Fm1, sweeps)
    Ue, Ve, We = dp.unpack(z)
    for got, ref in ((U[1:-1, 1:-1], Ue), (V[1:-1, :], Ve), (W[:, 1:-1], We)):
        assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)


@pytest.mark.parametrize("method,cfl,rate", [(O.CFD, 0.8, 0.48), (O.MFD, 0.5, 0.375)])
def test_sweeps_converge_geometrically_to_exact_stage(method, cfl, rate):
    """The error of K sweeps against the exact stages falls geometrically,
    no faster than the fixed-point contraction of the operators."""
    nx = ny = 10
    h, f, med, _ = _tiny_case(method, nx, ny, 11, with_src=False)
    one = np.ones_like
    med = {"K": one(med["K"]), "Rv": one(med["Rv"]), "Rw": one(med["Rw"])}
    dt = cfl * h
    dp = _dense_for(method, nx, ny, h, dt / 2, med["K"], med["Rv"], med["Rw"])
    z = dp.pack(f["U"][1:-1, 1:-1], f["V"][1:-1, :], f["W"][:, 1:-1])
    Z = np.zeros((dp.niy, dp.nix))
    Ue, _, _ = dp.unpack(dp.step_exact(z, Z, Z))
    errs = []
    for K in (4, 8, 12, 16):
        U, _, _ = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=1, sweeps=K, **med)
        errs.append(np.abs(U[1:-1, 1:-1] - Ue).max())
    per_sweep = [(errs[k + 1] / errs[k]) ** 0.25 for k in range(3)]
    assert all(0.2 * rate < r < 1.0 for r in per_sweep), per_sweep
    assert errs[-1] < 1e-2 * errs[0]


# ---------------------------------------------------------------- P5/P6 physics

def pr_mode_factor(alpha, beta, a, nsteps):
    """Closed-form PR-CN amplification of the mode (sin a x sin b y, cos sin,
    sin cos) with exact derivatives, c = rho = 1: pressure coefficient after
    nsteps steps (eqs. CN, ecua2:PR, ecua3:PR2 on a 3x3 symbol)."""
    A1 = np.array([[0, alpha, 0], [-alpha, 0, 0], [0, 0, 0.0]])
    A2 = np.array([[0, 0, beta], [0, 0, 0], [-beta, 0, 0.0]])
    I = np.eye(3)
    M = np.linalg.solve(I - a * A2, I + a * A1) @ np.linalg.solve(I - a * A1, I + a * A2)
    return np.linalg.matrix_power(M, nsteps)[0, 0]


@pytest.mark.parametrize("N,expect", [(24, 7.614e-3), (50, 1.760e-3), (100, 4.402e-4)])
def test_cfd_standing_wave_error_equals_pr_time_error(N, expect):
    """CFD, c = 1, dt = h, T = 1: the max error against the exact solution
    sin(pi x) sin(pi y) cos(sqrt 2 pi t) equals the closed-form PR-CN time
    error to within 1 %, and the remaining (spatial) error is tiny."""
    h = 1.0 / N
    f = inputs.standing_mode(O.CFD, N, N, h, 1, 1)
    U, V, W = O.run(O.CFD, f["U"], f["V"], f["W"], h=h, dt=h, nsteps=N, sweeps=6)
    exact = f["U"] * math.cos(math.sqrt(2) * math.pi)
    err = np.abs(U - exact).max()
    g = pr_mode_factor(math.pi, math.pi, h / 2, N)
    assert abs(g - math.cos(math.sqrt(2) * math.pi)) == pytest.approx(expect, rel=2e-3)
    assert err == pytest.approx(expect, rel=1e-2)
    assert np.abs(U - g * f["U"]).max() < 2e-3 * err


def test_rates_cfd():
    """Full error at dt = h converges at order 2 (time error dominates); the
    error against the time-discrete closed form converges at order ~4.  The
    spatial rate is taken on N <= 100: by 200 steps the roundoff-seeded
    growth of the CFD boundary modes (see the eigenvalue test below) reaches
    the 1e-9 level of the N = 200 spatial error."""
    ns = [24, 50, 100, 200]
    full, spatial = [], []
    for N in ns:
        h = 1.0 / N
        f = inputs.standing_mode(O.CFD, N, N, h, 1, 1)
        U, _, _ = O.run(O.CFD, f["U"], f["V"], f["W"], h=h, dt=h, nsteps=N, sweeps=6)
        full.append(np.abs(U - f["U"] * math.cos(math.sqrt(2) * math.pi)).max())
        spatial.append(np.abs(U - pr_mode_factor(math.pi, math.pi, h / 2, N) * f["U"]).max())
    rf, rs = _rate(full, ns), _rate(spatial[:3], ns[:3])
    assert all(abs(r - 2.0) < 0.05 for r in rf), rf
    assert min(rs) > 3.7, rs


def test_rates_mfd():
    """MFD standing mode sin(2 pi x) sin(3 pi y), dt = h/2, T = 0.25:
    spatial error (against the time-discrete closed form) at order ~4."""
    ns = [16, 32, 64, 128]
    spatial = []
    for N in ns:
        h = 1.0 / N
        f = inputs.standing_mode(O.MFD, N, N, h, 2, 3)
        nsteps = N // 2
        U, _, _ = O.run(O.MFD, f["U"], f["V"], f["W"], h=h, dt=h / 2, nsteps=nsteps, sweeps=6)
        g = pr_mode_factor(2 * math.pi, 3 * math.pi, h / 4, nsteps)
        spatial.append(np.abs(U - g * f["U"]).max())
    rs = _rate(spatial, ns)
    assert _trimmed(rs) > 3.9 and min(rs) > 3.5, rs


def pr_mode_state(alpha, beta, a, nsteps, kappa, rinv):
    """Closed-form PR-CN state of the mode (sin a x sin b y, cos sin, sin cos)
    with constant kappa and 1/rho and exact derivatives, from pressure 1 and
    zero velocities: the coefficients of pressure, x- and y-velocity after
    nsteps steps.  u_t = -kappa div v and v_t = -(1/rho) grad u act on the
    mode through the two direction blocks A1 (x) and A2 (y)."""
    A1 = np.array([[0, kappa * alpha, 0], [-rinv * alpha, 0, 0], [0, 0, 0.0]])
    A2 = np.array([[0, 0, kappa * beta], [0, 0, 0], [-rinv * beta, 0, 0.0]])
    I = np.eye(3)
    M = np.linalg.solve(I - a * A2, I + a * A1) @ np.linalg.solve(I - a * A1, I + a * A2)
    return np.linalg.matrix_power(M, nsteps)[:, 0]


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_constant_materials_follow_closed_form(method):
    """No material arrays: kappa0 = 2.25 and 1/rho0 = 0.64 (c = 1.2, kappa0
    and 1/rho0 distinct).  Pressure and both velocities of the standing mode
    (1, 2) follow the closed-form amplification with these constants, with
    fourth-order spatial error; exchanging the constants keeps c, hence the
    pressure, but scales the velocities by (1/rho0) / kappa0, which fails."""
    errs = {}
    for N in (64, 128):
        h = 1.0 / N
        f = inputs.standing_mode(method, N, N, h, 1, 2)
        dt, nsteps = 0.5 * h / 1.2, 40
        xp, xn = inputs.pressure_coords(method, N, h), inputs.node_coords(N, h)
        al, be = math.pi, 2 * math.pi
        u, v, w = pr_mode_state(al, be, dt / 2, nsteps, 2.25, 0.64)
        Ue = u * np.outer(np.sin(be * xp), np.sin(al * xp))
        Ve = v * np.outer(np.sin(be * xp), np.cos(al * xn))
        We = w * np.outer(np.cos(be * xn), np.sin(al * xp))
        for kap, rin in ((2.25, 0.64), (0.64, 2.25)):
            U, V, W = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=nsteps, kappa0=kap, rinv0=rin)
            errs[(N, kap)] = (np.abs(U - Ue)[1:-1, 1:-1].max(), np.abs(V - Ve)[1:-1, :].max(),
                              np.abs(W - We)[:, 1:-1].max())
    assert max(errs[(64, 2.25)]) < 5e-6, errs
    assert all(e64 / e128 > 12 for e64, e128 in zip(errs[(64, 2.25)], errs[(128, 2.25)])), errs
    assert min(errs[(64, 0.64)][1:]) > 0.1, errs


@pytest.mark.slow
def test_mfd_config2_mode_time_error_full_size():
    """The mimetic standing mode sin(2 pi x) sin(3 pi y) on 1024^2 cells,
    1000 steps of h/2 (T = 0.48828125): the max error against the exact mode
    equals the closed-form PR-CN time error 6.556e-6 within 1 %."""
    N = 1024
    h = 1.0 / N
    f = inputs.standing_mode(O.MFD, N, N, h, 2, 3)
    U, _, _ = O.run(O.MFD, f["U"], f["V"], f["W"], h=h, dt=h / 2, nsteps=1000, sweeps=6)
    T = 1000 * h / 2
    err = np.abs(U - f["U"] * math.cos(math.sqrt(13) * math.pi * T)).max()
    g = pr_mode_factor(2 * math.pi, 3 * math.pi, h / 4, 1000)
    assert abs(g - math.cos(math.sqrt(13) * math.pi * T)) == pytest.approx(6.556e-6, rel=1e-3)
    assert err == pytest.approx(6.556e-6, rel=1e-2)
    assert np.abs(U - g * f["U"]).max() < 1e-2 * err


def test_mfd_config2_mode_time_error_small_grid():
    """Same closed form for the MFD mode on a 128 grid, 100 steps of h/2."""
    N = 128
    h = 1.0 / N
    f = inputs.standing_mode(O.MFD, N, N, h, 2, 3)
    U, _, _ = O.run(O.MFD, f["U"], f["V"], f["W"], h=h, dt=h / 2, nsteps=100, sweeps=6)
    T = 100 * h / 2
    g = pr_mode_factor(2 * math.pi, 3 * math.pi, h / 4, 100)
    exact_err = abs(g - math.cos(math.sqrt(13) * math.pi * T)) * np.abs(f["U"]).max()
    err = np.abs(U - f["U"] * math.cos(math.sqrt(13) * math.pi * T)).max()
    assert err == pytest.approx(exact_err, rel=0.05)


# ---------------------------------------------------------------- P7 symmetry

@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_transposed_problem_with_swapped_order_is_bitwise_transpose(method):
    nx, ny = 13, 10
    h, f, med, src = _tiny_case(method, nx, ny, 21)
    dt = 0.6 * h / math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    kw = dict(h=h, dt=dt, nsteps=4, sweeps=6)
    U, V, W = O.run(method, f["U"], f["V"], f["W"], K=med["K"], Rv=med["Rv"], Rw=med["Rw"],
                    src=src, order=0, **kw)
    srcT = dict(src, i=src["j"], j=src["i"])
    Ut, Vt, Wt = O.run(method, f["U"].T, f["W"].T, f["V"].T, K=med["K"].T, Rv=med["Rw"].T,
                       Rw=med["Rv"].T, src=srcT, order=1, **kw)
    assert np.array_equal(Ut.T, U)
    assert np.array_equal(Wt.T, V)
    assert np.array_equal(Vt.T, W)


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_mirror_symmetric_problem_stays_symmetric(method):
    n = 16
    h = 1.0 / n
    sh = inputs.shapes(method, n, n)
    y = inputs.pressure_coords(method, n, h)
    K = np.repeat((1.0 + 0.5 * np.sin(3 * y))[:, None], sh["K"][1], axis=1)
    rng = np.random.default_rng(5)
    U = rng.standard_normal(sh["U"])
    U = 0.5 * (U + U[:, ::-1])
    U[0] = U[-1] = 0; U[:, 0] = U[:, -1] = 0
    V = np.zeros(sh["V"]); W = np.zeros(sh["W"])
    # a source on the mirror line (CFD node column n/2); the MFD centre line
    # carries no pressure point for even n, so that case runs unforced
    src = {"i": n // 2, "j": 5, "f0": 2.0, "t0": 0.3} if method == O.CFD else None
    U1, V1, W1 = O.run(method, U, V, W, h=h, dt=0.5 * h / 1.5, nsteps=10, sweeps=6, K=K, src=src)
    assert np.abs(U1 - U1[:, ::-1]).max() <= 1e-13 * np.abs(U1).max()
    assert np.abs(W1 - W1[:, ::-1]).max() <= 1e-13 * np.abs(W1).max()
    assert np.abs(V1 + V1[:, ::-1]).max() <= 1e-13 * np.abs(V1).max()


# ---------------------------------------------------------------- P8 stability

def _energy(f):
    return sum(float((a ** 2).sum()) for a in f)


def test_mfd_even_sweeps_bounded_odd_sweeps_grow():
    """At cfl 0.8 (fixed-point contraction ~0.96) an even sweep count keeps
    the MFD energy bounded; an odd count amplifies the unconverged modes."""
    n = 32
    h = 1.0 / n
    f = inputs.random_fields(O.MFD, n, n, 1)
    e0 = _energy((f["U"], f["V"], f["W"]))
    out = {}
    for K in (6, 7):
        g = O.run(O.MFD, f["U"], f["V"], f["W"], h=h, dt=0.8 * h, nsteps=100, sweeps=K)
        out[K] = _energy(g) / e0
    assert out[6] < 1.5
    assert out[7] > 1e6


def test_cfd_semidiscrete_operator_has_growing_boundary_modes():
    """The literal CFD pairing (Pbar^-1 Qbar on velocity, P^-1 Q with the
    4th-order closure on pressure, edge velocities evolved) has 1-D
    semi-discrete eigenvalues with Re(lambda) h ~ 0.1; the mimetic pair has
    none.  The growth is independent of the time step and of the sweeps."""
    n = 32
    h = 1.0 / n
    P, Q, Pb, Qb = O.cfd_matrices(n, h)
    Gc = np.linalg.solve(P, Q)[:, 1:n]
    Dc = np.linalg.solve(Pb, Qb)
    L = np.block([[np.zeros((n - 1, n - 1)), -Dc], [-Gc, np.zeros((n + 1, n + 1))]])
    re = np.linalg.eigvals(L).real * h
    assert 0.05 < re.max() < 0.2
    D, G = O.mfd_matrices(n, h)
    Lm = np.block([[np.zeros((n, n)), -D], [-G[:, 1:n + 1], np.zeros((n + 1, n + 1))]])
    assert np.linalg.eigvals(Lm).real.max() * h < 1e-12
    # the full 2-D scheme grows from roughness even with converged stages
    f = inputs.random_fields(O.CFD, n, n, 2)
    g = O.run(O.CFD, f["U"], f["V"], f["W"], h=h, dt=0.5 * h, nsteps=100, sweeps=40)
    assert _energy(g) / _energy((f["U"], f["V"], f["W"])) > 1e3


# ---------------------------------------------------------------- source

def test_ricker_source_closed_form():
    src = {"i": 3, "j": 4, "f0": 15.0, "t0": 1 / 15.0, "amp": 2.0}
    h = 5.0
    assert O.source_value(src, h, src["t0"]) == pytest.approx(2.0 / 25.0, rel=1e-15)
    tz = src["t0"] + 1.0 / (math.sqrt(2) * math.pi * 15.0)
    assert abs(O.source_value(src, h, tz)) < 1e-15
    # zero mean and even symmetry about the delay
    ts = np.linspace(src["t0"] - 0.5, src["t0"] + 0.5, 20001)
    vals = np.array([O.source_value(src, h, t) for t in ts])
    assert abs(np.trapezoid(vals, ts)) < 1e-9
    assert np.abs(vals - vals[::-1]).max() < 1e-12


# ---------------------------------------------------------------- tolerance test (stop rule)

@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_eps_mode_matches_dense_stop_rule(method):
    """The tolerance test of Algorithms 3 and 4 (whole-stage Frobenius norms,
    tested from min_sweeps on, count rounded up to even) against the same
    rule run on the dense matrix form: same sweep counts, same fields."""
    nx, ny = 11, 9
    h, f, med, src = _tiny_case(method, nx, ny, 5)
    dt = 0.8 * h / math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    dp = _dense_for(method, nx, ny, h, dt / 2, med["K"], med["Rv"], med["Rw"])
    z = dp.pack(f["U"][1:-1, 1:-1], f["V"][1:-1, :], f["W"][:, 1:-1])
    F = [np.zeros((dp.niy, dp.nix)) for _ in range(3)]
    for m in range(3):
        F[m][src["j"] - 1, src["i"] - 1] = O.source_value(src, h, m * dt)
    # a tolerance between the 5th and 6th changes of the first stage
    d = dp.stage1_changes(z, F[0], 8)
    assert all(d[k + 1] < d[k] for k in range(1, 7)), d
    eps = math.sqrt(d[4] * d[5])
    zz, used_ref = z, []
    for m in range(2):
        zz, u = dp.step_eps(zz, F[m], F[m + 1], eps, 2, 16)
        used_ref += u
    assert used_ref[0] == 6
    U, V, W, used = O.run_eps(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=2, eps=eps,
                              min_sweeps=2, sweeps=16, K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src)
    assert list(used) == used_ref
    Ue, Ve, We = dp.unpack(zz)
    for got, ref in ((U[1:-1, 1:-1], Ue), (V[1:-1, :], Ve), (W[:, 1:-1], We)):
        assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1.0)


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_eps_mode_limits(method):
    """A tolerance every change passes stops each stage at min_sweeps; one no
    change passes runs the cap: both equal the fixed-count runs bit for bit.
    Counts are even and grow as the tolerance shrinks."""
    nx, ny = 12, 10
    h, f, med, src = _tiny_case(method, nx, ny, 8)
    dt = 0.7 * h / math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    kw = dict(h=h, dt=dt, nsteps=3, K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src)
    for eps, k in ((1e30, 4), (1e-300, 10)):
        a = O.run_eps(method, f["U"], f["V"], f["W"], eps=eps, min_sweeps=4, sweeps=10, **kw)
        b = O.run(method, f["U"], f["V"], f["W"], sweeps=k, **kw)
        assert list(a[3]) == [k] * 6
        for x, y in zip(a[:3], b):
            assert np.array_equal(x, y)
    prev = None
    for eps in (1e-2, 1e-5, 1e-8, 1e-11):
        used = O.run_eps(method, f["U"], f["V"], f["W"], eps=eps, min_sweeps=2, sweeps=16, **kw)[3]
        assert all(u % 2 == 0 and 2 <= u <= 16 for u in used)
        if prev is not None:
            assert all(u >= p for u, p in zip(used, prev))
        prev = used


# ---------------------------------------------------------------- direct (exact) line solves

@pytest.mark.parametrize("method", [O.CFD, O.MFD])
@pytest.mark.parametrize("nx,ny", [(8, 8), (9, 12), (12, 10)])
def test_direct_matches_dense_exact_step(method, nx, ny):
    """Per-line exact solves equal the exactly solved stages of eqs.
    ecua2:PR / ecua3:PR2 assembled over the whole grid, at cfl 2.5, where
    the fixed-point sweeps diverge."""
    h, f, med, src = _tiny_case(method, nx, ny, 7 + nx)
    dt = 2.5 * h / math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    t0 = 0.05
    U, V, W = O.run_direct(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=1,
                           K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src, t0=t0)
    dp = _dense_for(method, nx, ny, h, dt / 2, med["K"], med["Rv"], med["Rw"])
    Fm = np.zeros((dp.niy, dp.nix)); Fm1 = np.zeros_like(Fm)
    Fm[src["j"] - 1, src["i"] - 1] = O.source_value(src, h, t0)
    Fm1[src["j"] - 1, src["i"] - 1] = O.source_value(src, h, t0 + dt)
    z = dp.pack(f["U"][1:-1, 1:-1], f["V"][1:-1, :], f["W"][:, 1:-1])
    Ue, Ve, We = dp.unpack(dp.step_exact(z, Fm, Fm1))
    for got, ref in ((U[1:-1, 1:-1], Ue), (V[1:-1, :], Ve), (W[:, 1:-1], We)):
        assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1.0)
    assert np.array_equal(U[0], f["U"][0]) and np.array_equal(U[:, -1], f["U"][:, -1])


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_direct_is_limit_of_sweeps_with_dirichlet_data(method):
    """With non-zero boundary pressure values (which the dense form above
    does not carry) the exact solves equal 60 sweeps at cfl 0.4, where the
    sweeps contract by at most 0.24 each, over two steps."""
    nx, ny = 13, 11
    h, f, med, src = _tiny_case(method, nx, ny, 21)
    rng = np.random.default_rng(5)
    U0 = f["U"].copy()
    for sl in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        U0[sl] = rng.standard_normal(U0[sl].shape)
    dt = 0.4 * h / math.sqrt(med["K"].max() * max(med["Rv"].max(), med["Rw"].max()))
    kw = dict(h=h, dt=dt, nsteps=2, K=med["K"], Rv=med["Rv"], Rw=med["Rw"], src=src)
    a = O.run_direct(method, U0, f["V"], f["W"], **kw)
    b = O.run(method, U0, f["V"], f["W"], sweeps=60, **kw)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()


@pytest.mark.parametrize("method,mode,tol", [(O.MFD, (2, 3), 1e-5), (O.CFD, (1, 1), 2e-7)])
@pytest.mark.parametrize("cfl", [2.0, 4.0])
def test_direct_beyond_fixed_point_limit_matches_closed_form(method, mode, tol, cfl):
    """At cfl 2 and 4, beyond the divergence limit of the sweeps, the exact
    solves follow the closed-form Peaceman-Rachford solution of the standing
    mode to within the spatial error, while 6 sweeps blow up."""
    N = 64
    h = 1.0 / N
    f = inputs.standing_mode(method, N, N, h, *mode)
    dt = cfl * h
    nsteps = int(round(0.5 / dt))
    U, _, _ = O.run_direct(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=nsteps)
    g = pr_mode_factor(mode[0] * math.pi, mode[1] * math.pi, dt / 2, nsteps)
    assert np.abs(U - g * f["U"]).max() < tol
    Us, _, _ = O.run(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=nsteps, sweeps=6)
    assert not np.abs(Us - g * f["U"]).max() < 1.0


# ------------------------------------------------- heterogeneous test (Section 4)

def _hetero_rates(method, gamma, k, ns, cfl, sweeps):
    errs = []
    for N in ns:
        pr = inputs.hetero_problem(method, N, gamma, k, cfl)
        U, V, W = O.run_forced(method, pr["U"], pr["V"], pr["W"], h=pr["h"], dt=pr["dt"], nsteps=pr["nsteps"],
                               sweeps=sweeps, F=pr["F"], fsig=pr["fsig"], bsig=pr["bsig"])
        ex = inputs.hetero_solution(method, N, N, pr["h"], gamma, k, pr["T"])
        errs.append(np.abs(U - ex["U"]).max())
    return errs, _rate(errs, ns)


@pytest.mark.parametrize("gamma", [2, 9])
def test_hetero_mimetic_converges_at_second_order(gamma):
    """Section 4's test with non-homogeneous walls (eq. harmonic_hetero, Gamma
    = k, lambda = 1/4, T = 1/sqrt 2, five periods): the max error converges at
    order 2 as in Table 5's Gamma = k columns (averages 1.99 and 1.88), the
    Crank-Nicolson time error dominating.  Run at cfl 0.4 with 16 sweeps, so
    that the stages are converged (contraction 0.24 per sweep) and the rate
    measures the scheme; the rate pins the intermediate level's wall values:
    the mid-step wall value alone converges at first order."""
    errs, rates = _hetero_rates(O.MFD, gamma, gamma, [48, 64, 96, 128], 0.4, 16)
    assert all(1.8 < r < 2.6 for r in rates[-2:]), (errs, rates)
    assert errs[-1] < 1.5e-3, errs


def test_hetero_homogeneous_limit():
    """Gamma = 0: the walls carry sin(8 pi x) sin(8 pi y) = 0, so the
    time-dependent wall data change nothing, and with the forcing alone the
    error converges at high order (Table 5's Gamma = 0 column averages 3.87)."""
    pr = inputs.hetero_problem(O.MFD, 48, 0, 2, 0.81)
    kw = dict(h=pr["h"], dt=pr["dt"], nsteps=pr["nsteps"], sweeps=6, F=pr["F"], fsig=pr["fsig"])
    a = O.run_forced(O.MFD, pr["U"], pr["V"], pr["W"], bsig=pr["bsig"], **kw)
    b = O.run_forced(O.MFD, pr["U"], pr["V"], pr["W"], **kw)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1.0)
    errs, rates = _hetero_rates(O.MFD, 0, 2, [64, 96, 128], 0.4, 16)
    assert min(rates) > 3.8, (errs, rates)


def test_hetero_forcing_enters_like_the_point_source():
    """A forcing field that is zero except at one interior point, h^-2 there,
    with a Ricker signal, is the point source: same fields."""
    n = 24
    h = 1.0 / n
    f = inputs.random_fields(O.MFD, n, n, 5)
    src = {"i": 7, "j": 11, "f0": 3.0, "t0": 0.2, "amp": 1.3}
    F = np.zeros(O.shapes(O.MFD, n, n)["U"])
    F[11, 7] = 1.0 / (h * h)
    a = O.run(O.MFD, f["U"], f["V"], f["W"], h=h, dt=0.5 * h, nsteps=5, src=src)
    b = O.run_forced(O.MFD, f["U"], f["V"], f["W"], h=h, dt=0.5 * h, nsteps=5, F=F,
                     fsig={"kind": O.SIGNAL_RICKER, "f0": 3.0, "t0": 0.2, "amp": 1.3})
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-14 * np.abs(x).max()


# ---------------------------------------------------------- damping layers (f4)

def pr_mode_state_damped(alpha, beta, a, nsteps, d):
    """pr_mode_state with kappa = rho = 1 and the uniform damping rate d in
    both directions: A1 gets -d on pressure and x-velocity, A2 -d on
    pressure and y-velocity."""
    A1 = np.array([[-d, alpha, 0], [-alpha, -d, 0], [0, 0, 0.0]])
    A2 = np.array([[-d, 0, beta], [0, 0, 0], [-beta, 0, -d]])
    I = np.eye(3)
    M = np.linalg.solve(I - a * A2, I + a * A1) @ np.linalg.solve(I - a * A1, I + a * A2)
    return np.linalg.matrix_power(M, nsteps)[:, 0]


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_damping_zero_rate_is_the_undamped_step(method):
    n = 30
    f = inputs.random_fields(method, n, n, 4)
    a = O.run(method, f["U"], f["V"], f["W"], h=1 / n, dt=0.5 / n, nsteps=4)
    b = O.run_damped(method, f["U"], f["V"], f["W"], h=1 / n, dt=0.5 / n, nsteps=4, d0=0.0, width=8, walls=15)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_uniform_damping_follows_closed_form(method):
    """A uniform rate d = 3 in both directions (width 0, all walls): the
    standing mode (1, 2) follows the closed-form amplification of the damped
    split, pressure and both velocities, at fourth order in h; damping the
    pressure once instead of with both directions' rates fails."""
    d = 3.0
    errs = {}
    for N in (64, 128):
        h = 1.0 / N
        f = inputs.standing_mode(method, N, N, h, 1, 2)
        dt, nsteps = 0.5 * h, 40
        xp, xn = inputs.pressure_coords(method, N, h), inputs.node_coords(N, h)
        al, be = math.pi, 2 * math.pi
        u, v, w = pr_mode_state_damped(al, be, dt / 2, nsteps, d)
        Ue = u * np.outer(np.sin(be * xp), np.sin(al * xp))
        Ve = v * np.outer(np.sin(be * xp), np.cos(al * xn))
        We = w * np.outer(np.cos(be * xn), np.sin(al * xp))
        U, V, W = O.run_damped(method, f["U"], f["V"], f["W"], h=h, dt=dt, nsteps=nsteps, d0=d, width=0, walls=15,
                               sweeps=16)
        errs[N] = (np.abs(U - Ue)[1:-1, 1:-1].max(), np.abs(V - Ve)[1:-1, :].max(), np.abs(W - We)[:, 1:-1].max())
    assert max(errs[64]) < 1e-6 and max(errs[128]) < 1e-7, errs
    assert all(a / b > 6 for a, b in zip(errs[64], errs[128])), errs
    u1, _, _ = pr_mode_state_damped(math.pi, 2 * math.pi, 0.25 / 64, 40, d / 2)
    u2, _, _ = pr_mode_state_damped(math.pi, 2 * math.pi, 0.25 / 64, 40, d)
    assert abs(u1 - u2) > 100 * max(errs[64])


def _pulse_energy(method, U, V, W, h):
    return float((U[1:-1, 1:-1] ** 2).sum() + (V[1:-1, :] ** 2).sum() + (W[:, 1:-1] ** 2).sum()) * h * h


@pytest.mark.parametrize("method", [O.CFD, O.MFD])
def test_damping_layers_absorb_an_outgoing_pulse(method):
    """A Gaussian pulse in a 128^2 box with 24-cell layers on all four walls:
    the energy never grows, and once the wave has reached the walls the
    energy left is a few per cent of what the reflecting box keeps."""
    N = 128
    h = 1.0 / N
    x = inputs.pressure_coords(method, N, h)
    U = np.exp(-((x[None, :] - 0.5) ** 2 + (x[:, None] - 0.5) ** 2) / (2 * 0.03 ** 2))
    U[0, :] = U[-1, :] = U[:, 0] = U[:, -1] = 0.0
    sh = O.shapes(method, N, N)
    V, W = np.zeros(sh["V"]), np.zeros(sh["W"])
    dt = 0.4 * h
    kw = dict(h=h, dt=dt, nsteps=100, sweeps=8)
    e0 = _pulse_energy(method, U, V, W, h)
    free = (U, V, W)
    damped = (U, V, W)
    ed = [e0]
    for _ in range(6):                       # 600 steps: t = 1.875, the front well past the walls
        free = O.run(method, *free, **kw)
        damped = O.run_damped(method, *damped, d0=60.0, width=24, walls=15, **kw)
        ed.append(_pulse_energy(method, *damped, h))
    ef = _pulse_energy(method, *free, h)
    assert all(b <= a * (1 + 1e-9) for a, b in zip(ed, ed[1:])), ed
    assert ed[-1] < 0.03 * ef, (ed[-1], ef)
