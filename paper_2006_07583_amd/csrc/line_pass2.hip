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
//    segment and a_k, b_k the responses of a segment (compile-time
//    constants).  The same data give the neighbours' edge values, so the
//    stencil halos of the next derivative are recomputed redundantly
//    instead of exchanged.
//  * Mimetic stencils: with the neighbours' last 3 / first 3 pressure values
//    a lane computes the velocity on its slots plus 2 left / 1 right, which
//    is all the next D4 needs: one exchange per sweep.
//
//  * Physical boundary rows.  Every window solves with the same constant
//    factors; the windows holding the first or last slot of the line then
//    subtract a low-rank correction (Sherman-Morrison-Woodbury) that turns
//    the constant matrix into P4 / Pbar4 (one more exchange per solve).
//    The window placement keeps every boundary-row stencil inside one lane
//    (first window starts at slot 0, last window ends at the last slot).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "line_consts.h"
#include "line_pass.h"
#include "pass_common.h"
#include <type_traits>

namespace adi {

template <typename T> struct Cfg2;
template <> struct Cfg2<float> { static constexpr int LW = 16, R = 16, NW = 8, TS = 1, WPE = 4; };
template <> struct Cfg2<double> { static constexpr int LW = 8, R = 16, NW = 4, TS = 2, WPE = 2; };

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
    static constexpr int CB = 4 * LW;                        // boundary correction coefficients
    static constexpr int WORK = RING + CB;
    static constexpr int SMEM = WORK > TILE ? WORK : TILE;

    const LinePassArgs<T>& a;
    T* ring;
    T* cbuf;
    int seg, lq, s0, n, xc;
    T yend;
    bool bnd;                // lane holds physical boundary rows
    bool lwin, rwin;         // window holds the first / last slot of the line (block-uniform)

    __device__ Pass2(const LinePassArgs<T>& args, T* smem, int seg_, int lq_, int s0_, bool bnd_, bool lwin_,
                     bool rwin_)
        : a(args), ring(smem), cbuf(smem + RING), seg(seg_), lq(lq_), s0(s0_), n(args.n), xc(0), bnd(bnd_),
          lwin(lwin_), rwin(rwin_) {}

    __device__ __forceinline__ T* half() { return ring + (xc & 1) * HALF; }
    __device__ __forceinline__ int at(int f, int sg) const { return f * FIELD + (sg + PADS) * LW + lq; }

    // ================= compact scheme =================
    // Right-hand side (scaled by 1/c) of the compact derivative of kind
    // `kind` (0: Q4 on pressure, 1: Qbar4 on velocity) into o.  Boundary rows
    // use the closures of Appendix A; the trivial rows added to Pbar get 0.
    __device__ __forceinline__ void rhs(int kind, const T (&f)[R], T fl, T fr, T (&o)[R]) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T fp = k + 1 < R ? f[k + 1] : fr;
            const T fm = k > 0 ? f[k - 1] : fl;
            o[k] = fp - fm;
        }
        if (bnd) {
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
                    if (s == 0 || s == n) o[k] = T(0);
                    if (s == 1 && k >= 1 && k + 2 < R)
                        o[k] = third * (-f[k - 1] - T(9) * f[k] + T(9) * f[k + 1] + f[k + 2]);
                    if (s == n - 1 && k >= 2 && k + 1 < R)
                        o[k] = third * (-f[k - 2] - T(9) * f[k - 1] + T(9) * f[k] + f[k + 1]);
                }
            }
        }
    }

    // Local forward + backward sweeps with zero carries, then publish.
    __device__ __forceinline__ void local_solve(T (&o)[R]) {
        const T al = T(kAlpha);
#pragma unroll
        for (int k = 1; k < R; ++k) o[k] = fma(-al, o[k - 1], o[k]);
        yend = o[R - 1];
#pragma unroll
        for (int k = R - 2; k >= 0; --k) o[k] = fma(-al, o[k + 1], o[k]);
        T* h = half();
        h[at(0, seg)] = yend;
        h[at(1, seg)] = o[0];
        h[at(2, seg)] = o[R - 1];
    }

    // After the barrier: combine carries, correct the segment, produce the
    // neighbours' edge values xl (slot -1) and xr (slot R) of the solution;
    // then, in the windows holding a physical boundary, apply the boundary-row
    // correction (one more exchange).
    __device__ __forceinline__ void finish_solve(int kind, T (&o)[R], T& xl, T& xr) {
        const T* h = half();
        ++xc;
        const bool has_next = seg + 1 < NSEG, has_prev = seg > 0;
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
        if (lwin || rwin) correct(kind, o, xl, xr);
    }

    // Value of a boundary correction at distance d from the boundary row.
    __device__ static T corr_at(int d, T W0, T W1) {
        if (d < 0 || d >= BndResp::NZ) return T(0);
        if (d == 0) return W0;
        T w = W1;
        for (int i = 1; i < d; ++i) w *= T(-kAlpha);
        return w;
    }

    __device__ void correct(int kind, T (&o)[R], T& xl, T& xr) {
        constexpr BndResp kb{};
        constexpr double de = 3.7320508075688772935;
        constexpr int NZ = BndResp::NZ;
        // correction values at the boundary row and the next, from the lane
        // holding the boundary rows
        if (lwin && seg == 0) {
            T W0, W1;
            if (kind == 0) {
                const T c = T(kb.cl0) * fma(T(6.0 - de), o[0], T(17) * o[1]);
                W0 = T(kb.zl0[0]) * c;
                W1 = T(kb.zl0[1]) * c;
            } else {
                const T e0 = fma(T(1.0 - de), o[0], -o[1]);
                const T e1 = fma(T(2), o[1], fma(T(5), o[2], -o[0]));
                const T c0 = fma(T(kb.cl1[0]), e0, T(kb.cl1[1]) * e1);
                const T c1 = fma(T(kb.cl1[2]), e0, T(kb.cl1[3]) * e1);
                W0 = fma(T(kb.zl0[0]), c0, T(kb.zl1[0]) * c1);
                W1 = fma(T(kb.zl0[1]), c0, T(kb.zl1[1]) * c1);
            }
            cbuf[lq] = W0;
            cbuf[LW + lq] = W1;
        }
        if (rwin && seg == NSEG - 1) {
            // slot n is the last slot of the window (position R - 1)
            T V0, V1;
            if (kind == 0) {
                const T c = T(kb.cr0) * fma(T(17), o[R - 2], T(2) * o[R - 1]);
                V0 = T(kb.zr0[0]) * c;
                V1 = T(kb.zr0[1]) * c;
            } else {
                const T e0 = fma(T(5), o[R - 3], fma(T(2), o[R - 2], -o[R - 1]));
                const T e1 = fma(T(-3), o[R - 1], -o[R - 2]);
                const T c0 = fma(T(kb.cr1[0]), e0, T(kb.cr1[1]) * e1);
                const T c1 = fma(T(kb.cr1[2]), e0, T(kb.cr1[3]) * e1);
                V0 = fma(T(kb.zr1[0]), c0, T(kb.zr0[0]) * c1);
                V1 = fma(T(kb.zr1[1]), c0, T(kb.zr0[1]) * c1);
            }
            cbuf[2 * LW + lq] = V0;
            cbuf[3 * LW + lq] = V1;
        }
        __syncthreads();
        if (lwin && s0 - 1 < NZ) {
            const T W0 = cbuf[lq], W1 = cbuf[LW + lq];
            T w = s0 == 0 ? W0 : corr_at(s0, W0, W1);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                o[k] -= w;
                w = (s0 + k == 0) ? W1 : w * T(-kAlpha);
            }
            if (seg > 0) xl -= corr_at(s0 - 1, W0, W1);
            xr -= w;
        }
        if (rwin && n - (s0 + R) < NZ) {
            const T V0 = cbuf[2 * LW + lq], V1 = cbuf[3 * LW + lq];
            const int dlast = n - (s0 + R - 1);          // distance of the lane's last slot
            T w = corr_at(dlast, V0, V1);
#pragma unroll
            for (int k = R - 1; k >= 0; --k) {
                o[k] -= w;
                w = (n - (s0 + k) == 0) ? V1 : w * T(-kAlpha);
            }
            xl -= w;
            if (seg + 1 < NSEG) xr -= corr_at(dlast - 1, V0, V1);
        }
        __syncthreads();   // values read before the next correction writes them
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

// One workgroup's share of a pass: line group tile % nlg of window tile / nlg.
template <typename T, int METHOD, int MODE, bool COMP>
__device__ __forceinline__ void lp2_body(const LinePassArgs<T>& a, int tile, T* smem) {
    using C = K2<T>;
    using P = Pass2<T, METHOD>;
    constexpr int LW = C::LW, R = C::R, SPW = C::SPW, WS = C::WS, NSEG = C::NSEG;
    const int lg = tile % a.nlg, g = a.gbase + (tile / a.nlg) * a.gstride;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lq = lane % LW;
    const int seg = wave * SPW + lane / LW;
    // central slots written by window g: the end windows need no margin on
    // their physical side, so the first one owns WS - H slots
    const int c0 = g == 0 ? 0 : (WS - a.H) + (g - 1) * a.S;
    const int c1 = g == a.nwin - 1 ? a.ns : (WS - a.H) + g * a.S;
    const int w0 = max(0, min(c0 - a.H, a.ns - WS));
    const int s0 = w0 + seg * R;
    const int q = lg * LW + lq;
    const bool qok = q < a.nlines;
    const int n = a.n;
    const int uhi = METHOD == LINE_CFD ? n - 1 : n;

    // lanes holding physical boundary rows (closure stencils), and windows
    // holding the first / last slot of the line (boundary-row correction)
    const bool bnd = s0 <= 1 || s0 + R - 1 >= n - 1;
    const bool lwin = w0 == 0, rwin = w0 + WS >= a.ns;
    P p(a, smem, seg, lq, s0, bnd, lwin, rwin);

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
    // raw material values; the scale is applied after every load has been
    // issued (arithmetic on a loaded value inside its predicated branch would
    // make each load wait for all earlier ones)
    auto ldK = [&](int s) -> T {
        if (!(qok && s >= 1 && s <= uhi)) return T(0);
        return a.ak ? a.ak[(int64_t)(s - 1) * a.ak_ld + q] : a.ak0;
    };
    auto ldR = [&](int s) -> T {
        if (!(qok && s >= 0 && s <= n)) return T(0);
        return a.ar ? a.ar[(int64_t)s * a.ar_ld + q] : a.ar0;
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
        T Kl = ldK(s0 - 1), Kr = ldK(s0 + R);
        T Bl = ldV(a.vin, a.vin_ld, s0 - 1), Br = ldV(a.vin, a.vin_ld, s0 + R);
        T Rl = ldR(s0 - 1), Rr = ldR(s0 + R);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            KK[k] *= sc;
            RR[k] *= sc;
        }
        Kl *= sc; Kr *= sc; Rl *= sc; Rr *= sc;
        __syncthreads();   // padding zeros visible
        T xl, xr;
        if (MODE == LINE_EXPLICIT || COMP) {
            // derivatives of the state: G(A) into Tt, D(B) into U
            p.rhs(0, A, Al, Ar, Tt);
            p.local_solve(Tt);
            __syncthreads();
            p.finish_solve(0, Tt, xl, xr);
            const T gl = -Rl * xl, gr = -Rr * xr;
            p.rhs(1, B, Bl, Br, U);
            p.local_solve(U);
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
                p.local_solve(U);
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
                p.local_solve(Tt);
                __syncthreads();
                p.finish_solve(0, Tt, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);
                Tl = fma(-Rl, xl, Bl);
                Tr = fma(-Rr, xr, Br);
                p.rhs(1, Tt, Tl, Tr, U);
                p.local_solve(U);
                __syncthreads();
                p.finish_solve(1, U, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
                Ul = fma(-Kl, xl, Al);
                Ur = fma(-Kr, xr, Ar);
            }
            p.rhs(0, U, Ul, Ur, Tt);
            p.local_solve(Tt);
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
                p.local_solve(A);
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
        T Rm2 = ldR(s0 - 2), Rm1 = ldR(s0 - 1), Rp = ldR(s0 + R);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            KK[k] *= sc;
            RR[k] *= sc;
        }
        Rm2 *= sc; Rm1 *= sc; Rp *= sc;
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

template <typename T, int METHOD, int MODE, bool COMP>
__global__ void __launch_bounds__(K2<T>::NT)
__attribute__((amdgpu_waves_per_eu(Cfg2<T>::WPE, Cfg2<T>::WPE)))
line_pass2_kernel(const LinePassArgs<T> a) {
    __shared__ T smem[Pass2<T, METHOD>::SMEM];
    // XCD-aware tile order: consecutive blocks of one XCD take neighbouring
    // line groups of the same window.
    const int nb = a.nlg * a.gcount;
    const int per = (nb + 7) / 8;
    const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    if (tile >= nb) return;
    lp2_body<T, METHOD, MODE, COMP>(a, tile, smem);
}

template <typename T, int METHOD, int MODE, bool COMP>
__global__ void __launch_bounds__(K2<T>::NT)
__attribute__((amdgpu_waves_per_eu(Cfg2<T>::WPE, Cfg2<T>::WPE)))
line_pass2_group_kernel(const GroupArgs<T> ga) {
    __shared__ T smem[Pass2<T, METHOD>::SMEM];
    int tile;
    const int it = group_item(ga, tile);
    if (it < 0) return;
    LinePassArgs<T> a = ga.items[it];
    if (a.aFtab) a.aF = a.aFtab[*ga.tick];
    lp2_body<T, METHOD, MODE, COMP>(a, tile, smem);
}

template <typename T, bool COMP>
hipError_t launch_all(const LinePassArgs<T>* a, const GroupArgs<T>* ga, int method, int mode, hipStream_t st) {
    const int nb = a ? a->nlg * a->gcount : ga->total;
    if (nb <= 0) return hipSuccess;
    dim3 grid((unsigned)(((nb + 7) / 8) * 8)), block(K2<T>::NT);
#define LP2_CASE(M, MD)                                                                                  \
    if (method == M && mode == MD) {                                                                     \
        if (a)                                                                                           \
            hipLaunchKernelGGL((line_pass2_kernel<T, M, MD, COMP>), grid, block, 0, st, *a);            \
        else                                                                                             \
            hipLaunchKernelGGL((line_pass2_group_kernel<T, M, MD, COMP>), grid, block, 0, st, *ga);     \
        return hipGetLastError();                                                                        \
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

template <typename T>
hipError_t launch_line_pass2(const LinePassArgs<T>& a0, int method, int mode, hipStream_t st, bool comp) {
    LinePassArgs<T> a = a0;
    a.gbase = 0;
    a.gstride = 1;
    a.gcount = a0.nwin;
    if (!comp) return launch_all<T, false>(&a, nullptr, method, mode, st);
    if constexpr (std::is_same<T, float>::value) return launch_all<T, true>(&a, nullptr, method, mode, st);
    return hipErrorInvalidValue;
}

// Items must have gbase = 0, gstride = 1, gcount = nwin.
template <typename T>
hipError_t launch_line_group2(const GroupArgs<T>& ga, int method, int mode, hipStream_t st, bool comp) {
    if (!comp) return launch_all<T, false>(nullptr, &ga, method, mode, st);
    if constexpr (std::is_same<T, float>::value) return launch_all<T, true>(nullptr, &ga, method, mode, st);
    return hipErrorInvalidValue;
}

int line2_lanes(int dtype) { return dtype == 0 ? K2<float>::LW : K2<double>::LW; }
int line2_seg(int dtype) { return dtype == 0 ? K2<float>::R : K2<double>::R; }

template hipError_t launch_line_pass2<float>(const LinePassArgs<float>&, int, int, hipStream_t, bool);
template hipError_t launch_line_pass2<double>(const LinePassArgs<double>&, int, int, hipStream_t, bool);
template hipError_t launch_line_group2<float>(const GroupArgs<float>&, int, int, hipStream_t, bool);
template hipError_t launch_line_group2<double>(const GroupArgs<double>&, int, int, hipStream_t, bool);

}  // namespace adi
