// Constants shared by the multi-window line-pass kernels: the interior
// factors of the compact matrices in scaled variables, the responses of a
// segment to its carries, the boundary-row correction of the compact
// solves, and the scaled mimetic interior stencils.
#pragma once
#include <hip/hip_runtime.h>

namespace adi {

constexpr double kAlpha = 0.26794919243112270647;   // 2 - sqrt 3

// The interior rows of the compact matrices are P = (1, 4, 1) and
// Q = (3/h)(-1, 0, 1).  With alpha = 2 - sqrt 3 the no-pivot LU of the
// interior has multiplier alpha and pivot 1/alpha, so with c = 3/h the scaled
// right-hand side y' = y/c and solution x'' = x/(c alpha) obey
//     y'_k  = (f_{k+1} - f_{k-1}) - alpha y'_{k-1}
//     x''_k = y'_k - alpha x''_{k+1}.
// A segment of R slots solved with zero carries is corrected by
//     x''_k += a_k Y + b_k X
// with Y the forward carry entering the segment and X the true first value
// of the next segment; a_k, b_k are the segment's responses and G = (-alpha)^R
// the forward carry's decay across one segment.
template <int R> struct Resp {
    double a[R], b[R], G;
    constexpr Resp() : a(), b(), G(0) {
        double g[R] = {};
        double gg = 1.0;
        for (int k = 0; k < R; ++k) { gg *= -kAlpha; g[k] = gg; }
        G = g[R - 1];
        double an = 0.0, bn = 1.0;
        for (int k = R - 1; k >= 0; --k) {
            a[k] = g[k] - kAlpha * an;
            an = a[k];
            bn = -kAlpha * bn;
            b[k] = bn;
        }
    }
};

// Near a physical boundary the compact rows differ from the constant-factor
// matrix Pc the kernel factorises (first row [2+sqrt3, 1], interior
// (1, 4, 1), last row (1, 4)): P4 row 0 is [6, 18] and row n is [18, 6]; the
// reduced Pbar4 has rows 1..n-1 with [6, 6] ends, handled as Pc-sized
// systems with the trivial rows x_0 = 0, x_n = 0 added.  The exact solution
// is the Pc solution minus a rank-1 (P) or rank-2 (Pbar) correction
// (Sherman-Morrison-Woodbury):  x = xc - Z C^-1 E xc, with E the row
// differences, Z = Pc^-1 [unit rows] (decaying like (2 - sqrt 3)^d from the
// boundary) and C = I + E Z.  All of these are constants of Pc.
struct BndResp {
    static constexpr int NZ = 48;
    double zl0[NZ], zl1[NZ];   // Pc^-1 e_0, Pc^-1 e_1, index = slot
    double zr0[NZ], zr1[NZ];   // Pc^-1 e_n, Pc^-1 e_{n-1}, index = n - slot
    double cl0, cr0;           // 1 / C for P at the left / right end
    double cl1[4], cr1[4];     // C^-1 (row-major 2 x 2) for Pbar at the left / right end
    constexpr BndResp() : zl0(), zl1(), zr0(), zr1(), cl0(0), cr0(0), cl1(), cr1() {
        constexpr int M = 160;
        constexpr double de = 3.7320508075688772935;
        // LU of Pc (multiplier alpha, pivots 2 + sqrt3) solving Pc x = e_j
        auto solve = [](int j, double* out) {
            double y[M] = {}, x[M] = {};
            for (int k = 0; k < M; ++k) y[k] = (k == j ? 1.0 : 0.0) - (k > 0 ? kAlpha * y[k - 1] : 0.0);
            x[M - 1] = y[M - 1] / de;
            for (int k = M - 2; k >= 0; --k) x[k] = (y[k] - x[k + 1]) / de;
            for (int k = 0; k < M; ++k) out[k] = x[k];
        };
        double a0[M] = {}, a1[M] = {}, b0[M] = {}, b1[M] = {};
        solve(0, a0);
        solve(1, a1);
        solve(M - 1, b0);
        solve(M - 2, b1);
        for (int k = 0; k < NZ; ++k) {
            zl0[k] = a0[k];
            zl1[k] = a1[k];
            zr0[k] = b0[M - 1 - k];
            zr1[k] = b1[M - 1 - k];
        }
        cl0 = 1.0 / (1.0 + (6.0 - de) * zl0[0] + 17.0 * zl0[1]);
        cr0 = 1.0 / (1.0 + 17.0 * zr0[1] + 2.0 * zr0[0]);
        // left Pbar: E rows [(1 - de), -1, 0] and [-1, 2, 5] on slots 0..2
        double L[4] = {1.0 + (1.0 - de) * zl0[0] - zl0[1], (1.0 - de) * zl1[0] - zl1[1],
                       -zl0[0] + 2.0 * zl0[1] + 5.0 * zl0[2], 1.0 - zl1[0] + 2.0 * zl1[1] + 5.0 * zl1[2]};
        double dl = L[0] * L[3] - L[1] * L[2];
        cl1[0] = L[3] / dl; cl1[1] = -L[1] / dl; cl1[2] = -L[2] / dl; cl1[3] = L[0] / dl;
        // right Pbar: E rows [5, 2, -1] on slots n-2, n-1, n and [-1, -3] on n-1, n;
        // Z columns Pc^-1 e_{n-1}, Pc^-1 e_n (index = n - slot)
        double Rm[4] = {1.0 + 5.0 * zr1[2] + 2.0 * zr1[1] - zr1[0], 5.0 * zr0[2] + 2.0 * zr0[1] - zr0[0],
                        -zr1[1] - 3.0 * zr1[0], 1.0 - zr0[1] - 3.0 * zr0[0]};
        double dr = Rm[0] * Rm[3] - Rm[1] * Rm[2];
        cr1[0] = Rm[3] / dr; cr1[1] = -Rm[1] / dr; cr1[2] = -Rm[2] / dr; cr1[3] = Rm[0] / dr;
    }
};

// Every column of Pc^-1 used above is geometric with ratio -alpha away from
// its first entry, so a correction is fully described by its value at the
// boundary row (W0) and at the next row (W1): w(d) = W1 (-alpha)^(d-1), d >= 1.

// Scaled mimetic stencils: G'u_k = (u_{k+1} - u_k) + r (u_{k+2} - u_{k-1}),
// D'v_k = (v_k - v_{k-1}) + r (v_{k+1} - v_{k-2}), r = -1/27; the factor
// 9/(8h) is folded into a kappa and a/rho.  Boundary rows (Appendix B) are
// divided by the same factor.
template <typename T>
__device__ __forceinline__ T mg(T um1, T u0, T u1, T u2) {
    return fma(T(-1.0 / 27.0), u2 - um1, u1 - u0);
}
template <typename T>
__device__ __forceinline__ T md(T vm2, T vm1, T v0, T v1) {
    return fma(T(-1.0 / 27.0), v1 - vm2, v0 - vm1);
}

}  // namespace adi
