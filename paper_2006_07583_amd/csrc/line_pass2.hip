// Line pass for lines longer than one window (the bulk of large grids).
//
// Same arithmetic as line_pass.hip (one launch = the fixed-point sweeps of a
// Peaceman-Rachford stage fused with the explicit part of the next stage,
// Algorithms 1-4), organised to need one workgroup barrier per derivative
// (compact scheme) or per sweep (mimetic scheme) and few VALU instructions:
//
//  * Scaled unknowns.  The compact interior rows are P = (1, 4, 1),
//    Q = (3/h)(-1, 0, 1).  With alpha = 2 - sqrt 3 the no-pivot LU of the
//    interior has multiplier alpha and pivot 1/alpha, so with c = 3/h the
//    scaled right-hand side y' = y/c and solution x'' = x/(c alpha) obey
//        y'_k  = (f_{k+1} - f_{k-1}) - alpha y'_{k-1}
//        x''_k = y'_k - alpha x''_{k+1}
//    one sub + two FMAs per slot; c alpha is folded into a kappa and a/rho.
//    Window edges inside a line get the pivot 1/alpha on their first row,
//    so every row away from the physical boundary has these factors.
//  * One exchange per solve.  A lane runs its segment with zero carries,
//    publishes (y'_last, x''_first, x''_last), and after one barrier
//    combines the carries of its TS neighbouring segments:
//        x''_k = x''^_k + a_k Y + b_k X
//    with Y the incoming forward carry, X the true first value of the next
//    segment and a_k, b_k the responses of the segment (compile-time
//    constants for interior segments, host tables near the physical
//    boundary).  The same data give the neighbours' edge values, so the
//    stencil halos of the next derivative are recomputed redundantly
//    instead of exchanged.
//  * Mimetic stencils: with the neighbours' last 3 / first 3 pressure values
//    a lane computes the velocity on its slots plus 2 left / 1 right, which
//    is all the next D4 needs: one exchange per sweep.
//
// Segments touching the physical boundary rows (and their neighbours) take
// the table path; the window placement keeps every boundary-row stencil
// inside one lane (first window starts at slot 0, last window ends at the
// last slot).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "line_pass.h"
#include "pass_common.h"
#include <type_traits>

namespace adi {

template <typename T> struct Cfg2;
template <> struct Cfg2<float> { static constexpr int LW = 16, R = 16, NW = 8, TS = 1, WPE = 4; };
template <> struct Cfg2<double> { static constexpr int LW = 8, R = 16, NW = 4, TS = 2, WPE = 2; };

constexpr double kAlpha = 0.26794919243112270647;   // 2 - sqrt 3

// Interior segment responses in scaled variables (see header comment).
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

template <typename T> struct K2 {
    static constexpr int LW = Cfg2<T>::LW, R = Cfg2<T>::R, NW = Cfg2<T>::NW, TS = Cfg2<T>::TS;
    static constexpr int SPW = 64 / LW, NSEG = NW * SPW, WS = NSEG * R, NT = NW * 64;
    static constexpr int PADS = TS > 2 ? TS : 2;           // zero segments on each side in LDS
    static constexpr int NSP = NSEG + 2 * PADS;
};
static_assert(K2<float>::WS == LINE_WS && K2<double>::WS == LINE_WS, "window size");

template <typename T, int METHOD> struct Pass2 {
    using C = K2<T>;
    static constexpr int LW = C::LW, R = C::R, NSEG = C::NSEG, WS = C::WS, TS = C::TS, NSP = C::NSP,
                         PADS = C::PADS;
    static constexpr int NF = METHOD == LINE_CFD ? 3 : 6;   // values published per exchange
    static constexpr int FIELD = NSP * LW;
    static constexpr int HALF = NF * FIELD;
    static constexpr int RING = 2 * HALF;
    static constexpr int TILEP = WS + 1;
    static constexpr int TILE = LW * TILEP;
    static constexpr int SMEM = RING > TILE ? RING : TILE;
    static constexpr int NTAB = 12;                          // table arrays per window (6 per kind)

    const LinePassArgs<T>& a;
    T* ring;
    int seg, lq, s0, n, xc;
    T yend;
    bool fast;               // segment and neighbours use the interior constants
    const T* tab;            // this window's tables (table path)

    __device__ Pass2(const LinePassArgs<T>& args, T* smem, int seg_, int lq_, int s0_, bool fast_,
                     const T* tab_)
        : a(args), ring(smem), seg(seg_), lq(lq_), s0(s0_), n(args.n), xc(0), fast(fast_), tab(tab_) {}

    __device__ __forceinline__ T* half() { return ring + (xc & 1) * HALF; }
    __device__ __forceinline__ int at(int f, int sg) const { return f * FIELD + (sg + PADS) * LW + lq; }

    // ================= compact scheme =================
    // Table layout per window, kind k (0: P, 1: Pbar), 6 arrays of WS:
    //   m (multiplier), dd (inverse pivot / alpha), e (sup * inverse pivot),
    //   a, b (segment responses), G (product of -m over the segment, at its
    //   first slot).  Rows outside the operator hold zeros.
    __device__ __forceinline__ const T* tk(int kind, int arr) const { return tab + (kind * 6 + arr) * WS; }

    // Right-hand side (scaled by 1/c) of the compact derivative of kind
    // `kind` (0: Q4 on pressure, 1: Qbar4 on velocity) into o.
    __device__ __forceinline__ void rhs(int kind, const T (&f)[R], T fl, T fr, T (&o)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T fp = k + 1 < R ? f[k + 1] : fr;
            const T fm = k > 0 ? f[k - 1] : fl;
            o[k] = fp - fm;
        }
        if (!fast) {
            const T third = T(1.0 / 3.0);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int s = s0 + k;
                if (kind == 0) {
                    if (s == 0 && k + 3 < R)
                        o[k] = third * (T(-17) * f[k] + T(9) * f[k + 1] + T(9) * f[k + 2] - f[k + 3]);
                    if (s == n && k >= 3)
                        o[k] = third * (f[k - 3] - T(9) * f[k - 2] - T(9) * f[k - 1] + T(17) * f[k]);
                } else {
                    if (s == 1 && k >= 1 && k + 2 < R)
                        o[k] = third * (-f[k - 1] - T(9) * f[k] + T(9) * f[k + 1] + f[k + 2]);
                    if (s == n - 1 && k >= 2 && k + 1 < R)
                        o[k] = third * (-f[k - 2] - T(9) * f[k - 1] + T(9) * f[k] + f[k + 1]);
                }
            }
        }
    }

    // Local forward + backward sweeps with zero carries, then publish.
    __device__ __forceinline__ void local_solve(int kind, T (&o)[R]) {
        if (fast) {
            const T al = T(kAlpha);
#pragma unroll
            for (int k = 1; k < R; ++k) o[k] = fma(-al, o[k - 1], o[k]);
            yend = o[R - 1];
#pragma unroll
            for (int k = R - 2; k >= 0; --k) o[k] = fma(-al, o[k + 1], o[k]);
        } else {
            const int sl = seg * R;
            const T* m = tk(kind, 0) + sl;
            const T* dd = tk(kind, 1) + sl;
            const T* e = tk(kind, 2) + sl;
#pragma unroll
            for (int k = 1; k < R; ++k) o[k] = fma(-m[k], o[k - 1], o[k]);
            yend = o[R - 1];
            o[R - 1] = o[R - 1] * dd[R - 1];
#pragma unroll
            for (int k = R - 2; k >= 0; --k) o[k] = fma(-e[k], o[k + 1], o[k] * dd[k]);
        }
        T* h = half();
        h[at(0, seg)] = yend;
        h[at(1, seg)] = o[0];
        h[at(2, seg)] = o[R - 1];
    }

    // After the barrier: combine carries, correct the segment, produce the
    // neighbours' edge values xl (slot -1) and xr (slot R) of the solution.
    __device__ __forceinline__ void finish_solve(int kind, T (&o)[R], T& xl, T& xr) {
        const T* h = half();
        ++xc;
        const bool has_next = seg + 1 < NSEG, has_prev = seg > 0;
        if (fast) {
            constexpr Resp<R> rs{};
            const T G = T(rs.G);
            T Y = h[at(0, seg - 1)];
            if (TS > 1) Y = fma(G, h[at(0, seg - 2)], Y);
            T Yv = fma(G, Y, yend);                 // forward carry into seg + 1
            T X = has_next ? fma(T(rs.a[0]), Yv, h[at(1, seg + 1)]) : T(0);
            if (TS > 1 && seg + 2 < NSEG) {
                const T Yv2 = fma(G, Yv, h[at(0, seg + 1)]);
                X = fma(T(rs.b[0]), fma(T(rs.a[0]), Yv2, h[at(1, seg + 2)]), X);
            }
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = fma(T(rs.a[k]), Y, fma(T(rs.b[k]), X, o[k]));
            const T Ym = TS > 1 ? h[at(0, seg - 2)] : T(0);   // forward carry into seg - 1
            xl = has_prev ? fma(T(rs.b[R - 1]), o[0], fma(T(rs.a[R - 1]), Ym, h[at(2, seg - 1)])) : T(0);
            xr = X;
        } else {
            const int sl = seg * R;
            const T* A = tk(kind, 3);
            const T* B = tk(kind, 4);
            const T* Gt = tk(kind, 5);
            const int sp = sl - R, sn = sl + R, sn2 = sl + 2 * R;
            const T Gp = seg > 0 ? Gt[sp] : T(0);
            const T Gs = Gt[sl];
            T Y = h[at(0, seg - 1)];
            if (TS > 1) Y = fma(Gp, h[at(0, seg - 2)], Y);
            T Yv = fma(Gs, Y, yend);
            const T an = has_next ? A[sn] : T(0);
            T X = has_next ? fma(an, Yv, h[at(1, seg + 1)]) : T(0);
            if (TS > 1 && seg + 2 < NSEG) {
                const T Gn = seg + 1 < NSEG ? Gt[sn] : T(0);
                const T bn = seg + 1 < NSEG ? B[sn] : T(0);
                const T an2 = seg + 2 < NSEG ? A[sn2] : T(0);
                const T Yv2 = fma(Gn, Yv, h[at(0, seg + 1)]);
                X = fma(bn, fma(an2, Yv2, h[at(1, seg + 2)]), X);
            }
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = fma(A[sl + k], Y, fma(B[sl + k], X, o[k]));
            const T Ym = TS > 1 ? h[at(0, seg - 2)] : T(0);
            const T ap = has_prev ? A[sl - 1] : T(0);
            const T bp = has_prev ? B[sl - 1] : T(0);
            xl = has_prev ? fma(bp, o[0], fma(ap, Ym, h[at(2, seg - 1)])) : T(0);
            xr = X;
        }
    }

    // ================= mimetic scheme =================
    // Publish the first 3 and last 3 pressure values of the lane.
    __device__ __forceinline__ void publish_u(const T (&u)[R]) {
        T* h = half();
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            h[at(i, seg)] = u[i];
            h[at(3 + i, seg)] = u[R - 3 + i];
        }
    }
    __device__ __forceinline__ void fetch_u(T (&ul)[3], T (&ur)[3]) {
        const T* h = half();
        ++xc;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ul[i] = h[at(3 + i, seg - 1)];
            ur[i] = h[at(i, seg + 1)];
        }
    }
};

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

// BND = false: windows away from the physical boundary (every segment uses
// the interior constants).  BND = true: the windows holding the boundary
// rows; segments near those rows use the host tables.
template <typename T, int METHOD, int MODE, bool BND, bool COMP>
__global__ void __launch_bounds__(K2<T>::NT)
__attribute__((amdgpu_waves_per_eu(BND ? 1 : Cfg2<T>::WPE, BND ? 8 : Cfg2<T>::WPE)))
line_pass2_kernel(const LinePassArgs<T> a) {
    using C = K2<T>;
    using P = Pass2<T, METHOD>;
    constexpr int LW = C::LW, R = C::R, SPW = C::SPW, WS = C::WS, NSEG = C::NSEG;
    __shared__ T smem[P::SMEM];

    // XCD-aware tile order: consecutive blocks of one XCD take neighbouring
    // line groups of the same window.
    const int nb = a.nlg * a.gcount;
    const int per = (nb + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= nb) return;
    const int lg = tile % a.nlg, g = a.gbase + (tile / a.nlg) * a.gstride;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lq = lane % LW;
    const int seg = wave * SPW + lane / LW;
    const int c0 = g * a.S;
    const int c1 = min(c0 + a.S, a.ns);
    const int w0 = max(0, min(c0 - a.H, a.ns - WS));
    const int s0 = w0 + seg * R;
    const int q = lg * LW + lq;
    const bool qok = q < a.nlines;
    const int n = a.n;
    const int uhi = METHOD == LINE_CFD ? n - 1 : n;

    // table path near the physical boundary rows
    bool fast;
    {
        const int zlo = 2 * R;
        auto cst = [&](int sg) {
            const int ss = w0 + sg * R;
            if (sg < 0 || sg >= NSEG) return true;
            const bool left_ok = (w0 > 0) || ss >= zlo;
            const bool right_ok = ss + R - 1 <= n - 2;
            return left_ok && right_ok;
        };
        fast = cst(seg - 1) && cst(seg) && cst(seg + 1);
        if (METHOD == LINE_MFD) fast = (s0 - 2 >= 2) && (s0 + R <= n - 2);
        if (!BND) fast = true;
    }
    const T* tab = METHOD == LINE_CFD ? a.coef + (size_t)g * P::NTAB * WS : nullptr;
    P p(a, smem, seg, lq, s0, fast, tab);

    // zero the padding segments of both ring halves
    for (int i = tid; i < 2 * P::NF * 2 * C::PADS * LW; i += C::NT) {
        const int l = i % LW;
        const int r = i / LW;
        const int pz = r % (2 * C::PADS);
        const int f = (r / (2 * C::PADS)) % P::NF;
        const int hh = r / (2 * C::PADS * P::NF);
        const int sp = pz < C::PADS ? pz : NSEG + pz;   // padded segment index
        smem[hh * P::HALF + f * P::FIELD + sp * LW + l] = T(0);
    }

    // ---- loads (own slots and the halo slots the scheme needs) ----
    T A[R], B[R], KK[R], RR[R], U[R], Tt[R];
    auto ldU = [&](const T* base, int64_t ld, int s) -> T {
        return (qok && s >= 1 && s <= uhi) ? base[(int64_t)(s - 1) * ld + q] : T(0);
    };
    auto ldV = [&](const T* base, int64_t ld, int s) -> T {
        return (qok && s >= 0 && s <= n) ? base[(int64_t)s * ld + q] : T(0);
    };
    // scale folded into the material arrays
    const T sc = METHOD == LINE_CFD ? T(3.0 * kAlpha) * a.inv_h : T(9.0 / 8.0) * a.inv_h;
    auto ldK = [&](int s) -> T {
        if (!(qok && s >= 1 && s <= uhi)) return T(0);
        return sc * (a.ak ? a.ak[(int64_t)(s - 1) * a.ak_ld + q] : a.ak0);
    };
    auto ldR = [&](int s) -> T {
        if (!(qok && s >= 0 && s <= n)) return T(0);
        return sc * (a.ar ? a.ar[(int64_t)s * a.ar_ld + q] : a.ar0);
    };
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int s = s0 + k;
        A[k] = ldU(a.uin, a.uin_ld, s);
        B[k] = ldV(a.vin, a.vin_ld, s);
        KK[k] = ldK(s);
        RR[k] = ldR(s);
    }

    if (METHOD == LINE_CFD) {
        // halo inputs at slots s0-1 and s0+R
        T Al = ldU(a.uin, a.uin_ld, s0 - 1), Ar = ldU(a.uin, a.uin_ld, s0 + R);
        const T Kl = ldK(s0 - 1), Kr = ldK(s0 + R);
        T Bl = ldV(a.vin, a.vin_ld, s0 - 1), Br = ldV(a.vin, a.vin_ld, s0 + R);
        const T Rl = ldR(s0 - 1), Rr = ldR(s0 + R);
        __syncthreads();   // padding zeros visible
        T xl, xr;
        if (MODE == LINE_EXPLICIT || COMP) {
            // derivatives of the state: G(A) into Tt, D(B) into U
            p.rhs(0, A, Al, Ar, Tt);
            p.local_solve(0, Tt);
            __syncthreads();
            p.finish_solve(0, Tt, xl, xr);
            const T gl = -Rl * xl, gr = -Rr * xr;
            p.rhs(1, B, Bl, Br, U);
            p.local_solve(1, U);
            __syncthreads();
            p.finish_solve(1, U, xl, xr);
            const T dl = -Kl * xl, dr = -Kr * xr;
            if (MODE == LINE_EXPLICIT) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    // W* = B - aR G(A),  A_out = A - aK D(B)   (increments when compensated)
                    Tt[k] = COMP ? -RR[k] * Tt[k] : fma(-RR[k], Tt[k], B[k]);
                    U[k] = COMP ? -KK[k] * U[k] : fma(-KK[k], U[k], A[k]);
                }
            } else {
                // compensated: iterate on the increments u - A and v - B, with
                // A' = -aK D(B) (= u_1 - A) and B' = -aR G(A)
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    A[k] = -KK[k] * U[k];
                    B[k] = -RR[k] * Tt[k];
                    U[k] = A[k];
                }
                Al = dl; Ar = dr; Bl = gl; Br = gr;
            }
        }
        if (MODE != LINE_EXPLICIT) {
            T Ul, Ur, Tl, Tr;
            if (!COMP) {
                // u_1 = A - aK D(B)
                p.rhs(1, B, Bl, Br, U);
                p.local_solve(1, U);
                __syncthreads();
                p.finish_solve(1, U, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
                Ul = fma(-Kl, xl, Al);
                Ur = fma(-Kr, xr, Ar);
            } else {
                Ul = Al;
                Ur = Ar;
            }
            for (int it = 1; it < a.sweeps; ++it) {
                p.rhs(0, U, Ul, Ur, Tt);
                p.local_solve(0, Tt);
                __syncthreads();
                p.finish_solve(0, Tt, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);
                Tl = fma(-Rl, xl, Bl);
                Tr = fma(-Rr, xr, Br);
                p.rhs(1, Tt, Tl, Tr, U);
                p.local_solve(1, U);
                __syncthreads();
                p.finish_solve(1, U, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
                Ul = fma(-Kl, xl, Al);
                Ur = fma(-Kr, xr, Ar);
            }
            p.rhs(0, U, Ul, Ur, Tt);
            p.local_solve(0, Tt);
            __syncthreads();
            p.finish_solve(0, Tt, xl, xr);
#pragma unroll
            for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);       // v_K
            if (MODE == LINE_SWEEP) {
                Tl = fma(-Rl, xl, Bl);
                Tr = fma(-Rr, xr, Br);
                if (COMP) {
#pragma unroll
                    for (int k = 0; k < R; ++k) U[k] += A[k];
                }
                p.rhs(1, Tt, Tl, Tr, A);
                p.local_solve(1, A);
                __syncthreads();
                p.finish_solve(1, A, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T vk = Tt[k];
                    Tt[k] = COMP ? vk + vk : vk + (vk - B[k]);
                    U[k] = fma(-KK[k], A[k], U[k]);
                }
            }
        }
    } else {
        // ---- mimetic ----
        T Bm2 = ldV(a.vin, a.vin_ld, s0 - 2), Bm1 = ldV(a.vin, a.vin_ld, s0 - 1),
          Bp = ldV(a.vin, a.vin_ld, s0 + R);
        const T Rm2 = ldR(s0 - 2), Rm1 = ldR(s0 - 1), Rp = ldR(s0 + R);
        const bool bnd = !fast;
        const T ih8 = T(8.0 / 9.0);   // boundary rows are divided by the folded 9/8
        const T d0c[6] = {T(-4751.0 / 5192.0), T(909.0 / 1298.0), T(6091.0 / 15576.0),
                          T(-1165.0 / 5192.0), T(129.0 / 2596.0), T(-25.0 / 15576.0)};
        const T g0c[6] = {T(-47888.0 / 14245.0), T(1790.0 / 407.0), T(-14545.0 / 9768.0),
                          T(8997.0 / 16280.0), T(-2335.0 / 22792.0), T(25.0 / 9768.0)};
        const T g1c[5] = {T(16.0 / 105.0), T(-31.0 / 24.0), T(29.0 / 24.0), T(-3.0 / 40.0),
                          T(1.0 / 168.0)};
        // D'(v) on own slots; v given on positions -2..R (vm2, vm1, v[0..R-1], vp)
        auto applyD = [&](const T (&v)[R], T vm2, T vm1, T vp, T (&o)[R]) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T a2 = k >= 2 ? v[k - 2] : (k == 1 ? vm1 : vm2);
                const T a1 = k >= 1 ? v[k - 1] : vm1;
                const T a3 = k + 1 < R ? v[k + 1] : vp;
                o[k] = md(a2, a1, v[k], a3);
            }
            if (bnd) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int s = s0 + k;
                    if (s == 1 && k >= 1 && k + 4 < R) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(d0c[c], v[k - 1 + c], acc);
                        o[k] = acc * ih8;
                    }
                    if (s == n && k >= 5) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(d0c[c], v[k - c], acc);
                        o[k] = -acc * ih8;
                    }
                }
            }
        };
        // G'(u) on own slots, u given on positions -3..R+2
        auto applyG = [&](const T (&u)[R], const T (&ul)[3], const T (&ur)[3], T (&o)[R]) {
            auto U_ = [&](int p) -> T { return p < 0 ? ul[3 + p] : (p < R ? u[p] : ur[p - R]); };
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = mg(U_(k - 1), U_(k), U_(k + 1), U_(k + 2));
            if (bnd) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int s = s0 + k;
                    if (s == 0 && k + 5 < R) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(g0c[c], u[k + c], acc);
                        o[k] = acc * ih8;
                    }
                    if (s == 1 && k >= 1 && k + 3 < R) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 5; ++c) acc = fma(g1c[c], u[k - 1 + c], acc);
                        o[k] = acc * ih8;
                    }
                    if (s == n - 1 && k >= 2 && k + 2 < R) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 5; ++c) acc = fma(g1c[c], u[k + 2 - c], acc);
                        o[k] = -acc * ih8;
                    }
                    if (s == n && k >= 4 && k + 1 < R) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(g0c[c], u[k + 1 - c], acc);
                        o[k] = -acc * ih8;
                    }
                }
            }
        };
        // velocity on own slots and on -2, -1, R from the exchanged pressure
        auto velocity = [&](const T (&u)[R], T (&o)[R], T& om2, T& om1, T& op) {
            T ul[3], ur[3];
            p.publish_u(u);
            __syncthreads();
            p.fetch_u(ul, ur);
            applyG(u, ul, ur, o);
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = fma(-RR[k], o[k], B[k]);
            om2 = fma(-Rm2, mg(ul[0], ul[1], ul[2], u[0]), Bm2);
            om1 = fma(-Rm1, mg(ul[1], ul[2], u[0], u[1]), Bm1);
            op = fma(-Rp, mg(u[R - 1], ur[0], ur[1], ur[2]), Bp);
        };
        if (MODE == LINE_EXPLICIT || COMP) {
            // derivatives of the state; A's halo comes from global memory
            T ul[3], ur[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ul[i] = ldU(a.uin, a.uin_ld, s0 - 3 + i);
                ur[i] = ldU(a.uin, a.uin_ld, s0 + R + i);
            }
            applyG(A, ul, ur, Tt);
            const T gm2 = mg(ul[0], ul[1], ul[2], A[0]), gm1 = mg(ul[1], ul[2], A[0], A[1]),
                    gp = mg(A[R - 1], ur[0], ur[1], ur[2]);
            applyD(B, Bm2, Bm1, Bp, U);
            if (MODE == LINE_EXPLICIT) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    Tt[k] = COMP ? -RR[k] * Tt[k] : fma(-RR[k], Tt[k], B[k]);
                    U[k] = COMP ? -KK[k] * U[k] : fma(-KK[k], U[k], A[k]);
                }
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    A[k] = -KK[k] * U[k];
                    B[k] = -RR[k] * Tt[k];
                    U[k] = A[k];
                }
                Bm2 = -Rm2 * gm2;
                Bm1 = -Rm1 * gm1;
                Bp = -Rp * gp;
            }
        }
        if (MODE != LINE_EXPLICIT) {
            __syncthreads();   // padding zeros visible
            T Tm2, Tm1, Tp;
            if (!COMP) {
                applyD(B, Bm2, Bm1, Bp, U);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
            }
            for (int it = 1; it < a.sweeps; ++it) {
                velocity(U, Tt, Tm2, Tm1, Tp);
                applyD(Tt, Tm2, Tm1, Tp, U);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
            }
            velocity(U, Tt, Tm2, Tm1, Tp);                                   // v_K
            if (MODE == LINE_SWEEP) {
                if (COMP) {
#pragma unroll
                    for (int k = 0; k < R; ++k) U[k] += A[k];
                }
                applyD(Tt, Tm2, Tm1, Tp, A);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T vk = Tt[k];
                    Tt[k] = COMP ? vk + vk : vk + (vk - B[k]);
                    U[k] = fma(-KK[k], A[k], U[k]);
                }
            }
        }
    }

    pass_outputs<T, R, LW, C::NT, P::TILEP, COMP>(a, smem, Tt, U, s0, q, qok, lq, lg, c0, c1, uhi, n, tid,
                                                 MODE != LINE_FINAL);
}

template <typename T, bool BND, bool COMP>
hipError_t launch_part(const LinePassArgs<T>& a, int method, int mode, hipStream_t st) {
    const int nb = a.nlg * a.gcount;
    if (nb <= 0) return hipSuccess;
    dim3 grid((unsigned)(((nb + 7) / 8) * 8)), block(K2<T>::NT);
#define LP2_CASE(M, MD)                                                                  \
    if (method == M && mode == MD) {                                                     \
        hipLaunchKernelGGL((line_pass2_kernel<T, M, MD, BND, COMP>), grid, block, 0, st, a);   \
        return hipGetLastError();                                                        \
    }
    LP2_CASE(LINE_CFD, LINE_SWEEP)
    LP2_CASE(LINE_CFD, LINE_FINAL)
    LP2_CASE(LINE_CFD, LINE_EXPLICIT)
    LP2_CASE(LINE_MFD, LINE_SWEEP)
    LP2_CASE(LINE_MFD, LINE_FINAL)
    LP2_CASE(LINE_MFD, LINE_EXPLICIT)
#undef LP2_CASE
    return hipErrorInvalidValue;
}

// The windows holding the physical boundary rows (first and last) run the
// table variant; the others run the constant-coefficient variant.
template <typename T, bool COMP>
hipError_t launch_split(const LinePassArgs<T>& a0, int method, int mode, hipStream_t st) {
    LinePassArgs<T> a = a0;
    a.gbase = 0;
    a.gstride = a0.nwin - 1;
    a.gcount = a0.nwin >= 2 ? 2 : 1;
    hipError_t e = launch_part<T, true, COMP>(a, method, mode, st);
    if (e != hipSuccess) return e;
    a.gbase = 1;
    a.gstride = 1;
    a.gcount = a0.nwin - 2;
    return launch_part<T, false, COMP>(a, method, mode, st);
}

template <typename T>
hipError_t launch_line_pass2(const LinePassArgs<T>& a, int method, int mode, hipStream_t st, bool comp) {
    if (!comp) return launch_split<T, false>(a, method, mode, st);
    if constexpr (std::is_same<T, float>::value) return launch_split<T, true>(a, method, mode, st);
    return hipErrorInvalidValue;
}

int line2_lanes(int dtype) { return dtype == 0 ? K2<float>::LW : K2<double>::LW; }
int line2_seg(int dtype) { return dtype == 0 ? K2<float>::R : K2<double>::R; }

template hipError_t launch_line_pass2<float>(const LinePassArgs<float>&, int, int, hipStream_t, bool);
template hipError_t launch_line_pass2<double>(const LinePassArgs<double>&, int, int, hipStream_t, bool);

}  // namespace adi
