"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module only generates data (grid coordinates, initial fields, media,
source placement, problem mixes).  It holds none of the ADI arithmetic and
imports neither the GPU library nor the oracle.

Grid conventions follow Section 2 of the paper: row index j runs along y,
column index i along x, spacing h in both directions.
  * nodal CFD grid: pressure and both velocities at nodes (i h, j h);
  * staggered MFD grid: pressure at X_cb x Y_cb (faces 0 and n h plus the
    cell centres (k - 1/2) h), horizontal velocity at X_n x Y_cb, vertical
    velocity at X_cb x Y_n.
"""
from __future__ import annotations

import math

import numpy as np

CFD = 0
MFD = 1


def node_coords(n: int, h: float) -> np.ndarray:
    """X_n: nodes 0, h, ..., n h."""
    return np.arange(n + 1, dtype=np.float64) * h


def cb_coords(n: int, h: float) -> np.ndarray:
    """X_cb: the two faces plus the n cell centres (Section 2.2)."""
    x = np.empty(n + 2, dtype=np.float64)
    x[0] = 0.0
    x[1:n + 1] = (np.arange(n, dtype=np.float64) + 0.5) * h
    x[n + 1] = n * h
    return x


def pressure_coords(method: int, n: int, h: float) -> np.ndarray:
    return node_coords(n, h) if method == CFD else cb_coords(n, h)


def shapes(method: int, nx: int, ny: int) -> dict:
    """Array shapes (rows, cols) of U, V, W and the material arrays."""
    if method == CFD:
        s = (ny + 1, nx + 1)
        return {"U": s, "K": s, "V": s, "Rv": s, "W": s, "Rw": s}
    return {"U": (ny + 2, nx + 2), "K": (ny + 2, nx + 2),
            "V": (ny + 2, nx + 1), "Rv": (ny + 2, nx + 1),
            "W": (ny + 1, nx + 2), "Rw": (ny + 1, nx + 2)}


def standing_mode(method: int, nx: int, ny: int, h: float, kx: int, ky: int) -> dict:
    """U0 = sin(kx pi x) sin(ky pi y) at the pressure points, V0 = W0 = 0.

    On the unit square this vanishes on all four walls, so it satisfies the
    homogeneous Dirichlet condition; with c = 1 the exact solution is
    U0 cos(pi sqrt(kx^2 + ky^2) t).
    """
    x = pressure_coords(method, nx, h)
    y = pressure_coords(method, ny, h)
    U = np.outer(np.sin(ky * math.pi * y), np.sin(kx * math.pi * x))
    sh = shapes(method, nx, ny)
    U[0, :] = U[-1, :] = 0.0
    U[:, 0] = U[:, -1] = 0.0
    return {"U": U, "V": np.zeros(sh["V"]), "W": np.zeros(sh["W"])}


def random_fields(method: int, nx: int, ny: int, seed: int, scale: float = 1.0) -> dict:
    """Gaussian pressure and velocities (zero Dirichlet pressure on the walls)."""
    rng = np.random.default_rng(seed)
    sh = shapes(method, nx, ny)
    U = scale * rng.standard_normal(sh["U"])
    U[0, :] = U[-1, :] = 0.0
    U[:, 0] = U[:, -1] = 0.0
    return {"U": U, "V": scale * rng.standard_normal(sh["V"]),
            "W": scale * rng.standard_normal(sh["W"])}


def random_medium(method: int, nx: int, ny: int, seed: int, lo=0.5, hi=1.5) -> dict:
    """Smoothly varying positive kappa (pressure points) and 1/rho (velocity points)."""
    rng = np.random.default_rng(seed)
    sh = shapes(method, nx, ny)

    def smooth(shape):
        r, c = shape
        y = np.linspace(0.0, 1.0, r)[:, None]
        x = np.linspace(0.0, 1.0, c)[None, :]
        f = np.zeros(shape)
        for _ in range(3):
            a, b, p, q = rng.uniform(0.5, 3.0, 4)
            f += np.sin(a * math.pi * x + p) * np.cos(b * math.pi * y + q)
        f = (f - f.min()) / max(f.max() - f.min(), 1e-30)
        return lo + (hi - lo) * f

    return {"K": smooth(sh["K"]), "Rv": smooth(sh["Rv"]), "Rw": smooth(sh["Rw"])}


def layered_speed(method: int, nx: int, ny: int, h: float, seed: int) -> np.ndarray:
    """Layered wave speed c(x, y) [m/s] at the pressure points.

    Between 3 and 8 layers; interface depths drawn uniformly in
    (0.1, 0.95) * L_y and sorted; each interface undulates by at most
    0.03 * L_y through 1-3 sinusoids; layer speeds drawn uniformly in
    [1500, 4500] m/s and sorted to increase with depth; tanh transitions of
    width 2h.  Depth is measured from row j = 0 (the free surface).
    """
    rng = np.random.default_rng(seed)
    Lx, Ly = nx * h, ny * h
    nlayers = int(rng.integers(3, 9))
    depths = np.sort(rng.uniform(0.1, 0.95, nlayers - 1)) * Ly
    speeds = np.sort(rng.uniform(1500.0, 4500.0, nlayers))
    x = pressure_coords(method, nx, h)
    y = pressure_coords(method, ny, h)
    c = np.full((y.size, x.size), speeds[0])
    for k, z0 in enumerate(depths):
        nwaves = int(rng.integers(1, 4))
        amp = rng.uniform(0.0, 0.03 * Ly, nwaves) / nwaves
        wl = rng.uniform(0.2, 1.0, nwaves) * Lx
        ph = rng.uniform(0.0, 2.0 * math.pi, nwaves)
        z = z0 + sum(a * np.sin(2.0 * math.pi * x / w + p) for a, w, p in zip(amp, wl, ph))
        step = 0.5 * (1.0 + np.tanh((y[:, None] - z[None, :]) / (2.0 * h)))
        c = c + (speeds[k + 1] - speeds[k]) * step
    return c


def ricker_source(i: int, j: int, f0: float = 15.0, amp: float = 1.0) -> dict:
    """Point source placement and Ricker parameters (delay t0 = 1 / f0)."""
    return {"i": int(i), "j": int(j), "f0": float(f0), "t0": 1.0 / float(f0), "amp": float(amp)}


def seismic_problem(method: int, n: int, seed: int = 0, h: float = 5.0, cfl: float = 0.8) -> dict:
    """Layered-medium problem: n x n cells of h metres, rho = 1, kappa = c^2,
    15 Hz Ricker at (i = n/2, j = 16), zero initial fields, dt = cfl h / c_max."""
    c = layered_speed(method, n, n, h, seed)
    cmax = float(c.max())
    sh = shapes(method, n, n)
    return {
        "method": method, "nx": n, "ny": n, "h": h, "dt": cfl * h / cmax, "cmax": cmax,
        "K": c * c, "src": ricker_source(n // 2, 16),
        "U": np.zeros(sh["U"]), "V": np.zeros(sh["V"]), "W": np.zeros(sh["W"]),
    }


def batch_mix(seed: int = 0, count: int = 256, lo: int = 64, hi: int = 1024) -> list:
    """Problem mix of the batched workload: Nx, Ny independent and
    log-uniform on [lo, hi], method uniform on {CFD, MFD}, per-problem medium
    seed, Ricker source at a uniform interior point at least 8 cells from the
    walls."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        method = int(rng.integers(0, 2))
        si = int(rng.integers(8, nx - 8 + 1))
        sj = int(rng.integers(8, ny - 8 + 1))
        out.append({"method": method, "nx": nx, "ny": ny, "medium_seed": int(rng.integers(0, 2**31)),
                    "src_i": si, "src_j": sj})
    return out


def serve_mix(seed: int = 0, count: int = 2000, rate: float = 200.0, lo: int = 128, hi: int = 2048,
              steps_lo: int = 100, steps_hi: int = 2000) -> list:
    """Request stream of the served workload: Poisson arrivals at `rate` per
    second, Nx, Ny independent and log-uniform on [lo, hi], steps log-uniform
    on [steps_lo, steps_hi], method and dtype (FP32 / FP64) uniform, Ricker
    source at a uniform interior point at least 8 cells from the walls."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(1.0 / rate))
        nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        nsteps = int(round(math.exp(rng.uniform(math.log(steps_lo), math.log(steps_hi)))))
        out.append({"t": t, "nx": nx, "ny": ny, "nsteps": nsteps, "method": int(rng.integers(0, 2)),
                    "fp64": bool(rng.integers(0, 2)), "src_i": int(rng.integers(8, nx - 8 + 1)),
                    "src_j": int(rng.integers(8, ny - 8 + 1))})
    return out


def hetero_solution(method: int, nx: int, ny: int, h: float, gamma: float, k: int, t: float,
                    lam: float = 0.25, period: float = 1.0 / math.sqrt(2.0), rho: float = 1.0) -> dict:
    """The exact solution of the heterogeneous test of Section 4 (eq.
    harmonic_hetero) at time t, with c = 1 (kappa = rho):
        u = phi(x, y) cos(w t),
        phi = gamma (x^k - (1 - x)^k + y^k - (1 - y)^k) + sin(2 pi x / lam) sin(2 pi y / lam),
    w = 2 pi / period, and the velocities that make it a solution of
    rho v_t = -u_x, rho w_t = -u_y from zero at t = 0:
        v = -phi_x sin(w t) / (rho w),  w_vel = -phi_y sin(w t) / (rho w),
    at the method's pressure and velocity points.  gamma = 0 leaves the
    sinusoid, which vanishes on the walls (homogeneous Dirichlet data)."""
    om = 2.0 * math.pi / period
    al = 2.0 * math.pi / lam
    xp, yp = pressure_coords(method, nx, h), pressure_coords(method, ny, h)
    xn, yn = node_coords(nx, h), node_coords(ny, h)

    def poly(x):
        return x ** k - (1.0 - x) ** k

    def dpoly(x):
        return k * (x ** (k - 1) + (1.0 - x) ** (k - 1))

    phi = gamma * (poly(xp)[None, :] + poly(yp)[:, None]) + np.outer(np.sin(al * yp), np.sin(al * xp))
    # V at (x nodes, y pressure rows), W at (x pressure columns, y nodes)
    phix = gamma * dpoly(xn)[None, :] + al * np.outer(np.sin(al * yp), np.cos(al * xn))
    phiy = gamma * dpoly(yn)[:, None] + al * np.outer(np.cos(al * yn), np.sin(al * xp))
    phix = np.broadcast_to(phix, (yp.size, xn.size))
    phiy = np.broadcast_to(phiy, (yn.size, xp.size))
    s = math.sin(om * t) / (rho * om)
    return {"U": phi * math.cos(om * t), "V": -phix * s, "W": -phiy * s}


def hetero_problem(method: int, n: int, gamma: float, k: int, cfl: float, periods: float = 5.0,
                   lam: float = 0.25, period: float = 1.0 / math.sqrt(2.0)) -> dict:
    """The heterogeneous test of Section 4 on the unit square with n x n
    cells: initial fields (the exact solution at t = 0), the forcing that
    makes eq. harmonic_hetero a solution of eq. 1 with c = rho = kappa = 1,
        f = -sin(w t) (w phi + lap(phi) / w) = g(x, y) cos(w (t + period / 4)),
    as a field g with a cosine signal, the wall signal cos(w t) that scales
    the walls' initial values, and the step: the largest dt <= cfl h that
    divides the simulated time (periods x period) into whole steps."""
    h = 1.0 / n
    om = 2.0 * math.pi / period
    al = 2.0 * math.pi / lam
    x, y = pressure_coords(method, n, h), pressure_coords(method, n, h)

    def poly(z, kk):
        return z ** kk - (1.0 - z) ** kk

    phi = gamma * (poly(x, k)[None, :] + poly(y, k)[:, None]) + np.outer(np.sin(al * y), np.sin(al * x))
    lap = (gamma * k * (k - 1) * (poly(x, k - 2)[None, :] + poly(y, k - 2)[:, None]) if k >= 2 else 0.0) \
        - 2.0 * al * al * np.outer(np.sin(al * y), np.sin(al * x))
    g = om * phi + lap / om
    T = periods * period
    nsteps = int(math.ceil(T / (cfl * h) - 1e-9))
    f0 = hetero_solution(method, n, n, h, gamma, k, 0.0, lam, period)
    return {"method": method, "n": n, "h": h, "dt": T / nsteps, "nsteps": nsteps, "T": T,
            "U": f0["U"], "V": f0["V"], "W": f0["W"], "F": g,
            "fsig": {"kind": 2, "f0": 1.0 / period, "t0": -period / 4.0, "amp": 1.0},
            "bsig": {"kind": 2, "f0": 1.0 / period, "t0": 0.0, "amp": 1.0},
            "gamma": gamma, "k": k, "lam": lam, "period": period}
