"""Dense (Kronecker-product) form of the Peaceman-Rachford step on tiny grids.

Used only by tests to pin the oracle: it writes the operators A1h, A2h of
eqs. A1HA2H / A1HA2HMimetic as explicit matrices over the unknown vector
[Ubar, Vbar, Wbar] and solves the two stages of eqs. ecua2:PR / ecua3:PR2
either exactly (LU) or by the fixed-point sweeps of eqs. adiSolve /
adiSolve2 written in matrix form.  Only homogeneous Dirichlet pressure is
handled (boundary pressure = 0).
"""
from __future__ import annotations

import numpy as np


class DenseProblem:
    def __init__(self, Dx, Gx, Dy, Gy, nx, ny, method, K, Rv, Rw, a):
        """Dx: (nix, nx+1) velocity->pressure along x; Gx: (nx+1, nfx)
        pressure->velocity along x (full pressure line); same for y.
        K: interior kappa (niy, nix); Rv: (niy, nx+1) at the unknown V rows;
        Rw: (ny+1, nix) at the unknown W columns."""
        nix, niy = Dx.shape[0], Dy.shape[0]
        self.nix, self.niy, self.nx, self.ny = nix, niy, nx, ny
        nu, nv, nw = niy * nix, niy * (nx + 1), (ny + 1) * nix
        self.nu, self.nv, self.nw = nu, nv, nw
        Gxi = Gx[:, 1:-1]              # boundary pressure is zero
        Gyi = Gy[:, 1:-1]
        Iy, Ix = np.eye(niy), np.eye(nix)
        k = np.diag(K.ravel())
        # x-part:  dU = -K (Vbar Dx^T),  dV = -Rv (Ubar Gxi^T)
        DUx = k @ np.kron(Iy, Dx)                  # (nu, nv)
        DVx = np.diag(Rv.ravel()) @ np.kron(Iy, Gxi)   # (nv, nu)
        # y-part:  dU = -K (Dy Wbar),   dW = -Rw (Gyi Ubar)
        DUy = k @ np.kron(Dy, Ix)                  # (nu, nw)
        DWy = np.diag(Rw.ravel()) @ np.kron(Gyi, Ix)   # (nw, nu)
        n = nu + nv + nw
        A1 = np.zeros((n, n)); A2 = np.zeros((n, n))
        A1[:nu, nu:nu + nv] = -DUx
        A1[nu:nu + nv, :nu] = -DVx
        A2[:nu, nu + nv:] = -DUy
        A2[nu + nv:, :nu] = -DWy
        self.A1, self.A2, self.a = A1, A2, a
        self.DUx, self.DVx, self.DUy, self.DWy = DUx, DVx, DUy, DWy

    def pack(self, Ui, Vr, Wc):
        return np.concatenate([Ui.ravel(), Vr.ravel(), Wc.ravel()])

    def unpack(self, z):
        nu, nv = self.nu, self.nv
        return (z[:nu].reshape(self.niy, self.nix),
                z[nu:nu + nv].reshape(self.niy, self.nx + 1),
                z[nu + nv:].reshape(self.ny + 1, self.nix))

    def step_exact(self, z, Fm, Fm1):
        """Both stages solved exactly: the K -> infinity limit."""
        I = np.eye(z.size)
        a = self.a
        fm = np.zeros_like(z); fm[:self.nu] = Fm.ravel()
        fm1 = np.zeros_like(z); fm1[:self.nu] = Fm1.ravel()
        zs = np.linalg.solve(I - a * self.A1, (I + a * self.A2) @ z + a * fm)
        return np.linalg.solve(I - a * self.A2, (I + a * self.A1) @ zs + a * fm1)

    def step_sweeps(self, z, Fm, Fm1, sweeps):
        """Both stages by `sweeps` fixed-point sweeps: stage 1 starts from
        V^m, stage 2 from W* (the algorithm text)."""
        a = self.a
        U, V, W = (x.ravel() for x in self.unpack(z))
        # stage 1 (x implicit): A, W*, then the row sweeps
        A = U - a * (self.DUy @ W) + a * Fm.ravel()
        Ws = W - a * (self.DWy @ U)
        Vk = V.copy()
        for _ in range(sweeps):
            Uk = A - a * (self.DUx @ Vk)
            Vk = V - a * (self.DVx @ Uk)
        Us, Vs = Uk, Vk
        # stage 2 (y implicit): C, V^{m+1}, then the column sweeps
        C = Us - a * (self.DUx @ Vs) + a * Fm1.ravel()
        Vn = Vs - a * (self.DVx @ Us)
        Wk = Ws.copy()
        for _ in range(sweeps):
            Uk = C - a * (self.DUy @ Wk)
            Wk = Ws - a * (self.DWy @ Uk)
        return np.concatenate([Uk, Vn, Wk])
