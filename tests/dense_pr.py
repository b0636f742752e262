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

    def step_eps(self, z, Fm, Fm1, eps, min_sweeps, cap):
        """Both stages with the tolerance test of Algorithms 3 and 4: after
        sweep k >= max(2, min_sweeps), stop once ||U_k - U_{k-1}|| +
        ||vel_k - vel_{k-1}|| <= eps (Frobenius norms over the stage), the
        count rounded up to even, at most `cap`.  Returns (z, [k1, k2])."""
        a = self.a

        def sweeps(Arhs, vel0, DU, DV):
            Vk = vel0.copy()
            Uk = np.zeros(self.nu)
            k, last = 0, cap
            while k < last:
                Un = Arhs - a * (DU @ Vk)
                Vn = vel0 - a * (DV @ Un)
                d = np.linalg.norm(Un - Uk) + np.linalg.norm(Vn - Vk)
                Uk, Vk, k = Un, Vn, k + 1
                if last == cap and k >= max(2, min_sweeps) and d <= eps:
                    last = k + (k & 1)
            return Uk, Vk, last

        U, V, W = (x.ravel() for x in self.unpack(z))
        A = U - a * (self.DUy @ W) + a * Fm.ravel()
        Ws = W - a * (self.DWy @ U)
        Us, Vs, k1 = sweeps(A, V, self.DUx, self.DVx)
        C = Us - a * (self.DUx @ Vs) + a * Fm1.ravel()
        Vn = Vs - a * (self.DVx @ Us)
        Uk, Wk, k2 = sweeps(C, Ws, self.DUy, self.DWy)
        return np.concatenate([Uk, Vn, Wk]), [k1, k2]

    def stage1_changes(self, z, Fm, n):
        """||U_k - U_{k-1}|| + ||V_k - V_{k-1}|| of the first stage for
        k = 1..n (U_0 = 0)."""
        a = self.a
        U, V, W = (x.ravel() for x in self.unpack(z))
        A = U - a * (self.DUy @ W) + a * Fm.ravel()
        Vk, Uk, out = V.copy(), np.zeros(self.nu), []
        for _ in range(n):
            Un = A - a * (self.DUx @ Vk)
            Vn = V - a * (self.DVx @ Un)
            out.append(np.linalg.norm(Un - Uk) + np.linalg.norm(Vn - Vk))
            Uk, Vk = Un, Vn
        return out

