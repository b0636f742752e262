// Windowed line pass of the Peaceman-Rachford ADI step on CDNA4 (gfx950).
//
// One launch performs, for every interior grid line of one direction, the
// implicit half of a Peaceman-Rachford stage (the fixed-point sweeps of
// eqs. adiSolve / adiSolve2, Algorithms 3 and 4) fused with the explicit half
// of the following stage along the same line (the C / V^{m+1} computations of
// Algorithm 1, or A / W* of the next step).  With a = dt/2 and, along the
// line, G = pressure->velocity derivative, D = velocity->pressure derivative:
//     u_1 = A - aK D(B)
//     u_k = A - aK D(B - aR G(u_{k-1}))           k = 2..K
//     v_K = B - aR G(u_K)
//     vel_out = 2 v_K - B   ( = v_K - aR G(u_K) )
//     U_out   = u_K - aK D(v_K) + aF
// (FINAL mode writes u_K and v_K instead; EXPLICIT mode writes
//  B - aR G(A) and A - aK D(B) + aF.)
//
// Data placement.  A workgroup owns LW adjacent lines (adjacent in memory,
// so every global access is a full 128-byte row segment) and a window of WS
// consecutive positions ("slots") along them.  Lane l of wave w handles line
// l % LW and the R consecutive slots of segment w*(64/LW) + l/LW; all line
// data of a window lives in VGPRs.  Stencil halos and the carries of the
// segmented tridiagonal recurrences cross segments through LDS.  Windows of
// one line overlap by H slots on each side; only the central slots are
// written.  The windowed problem drops the couplings to slots outside the
// window; for the compact scheme the inverse of P decays like
// (2 - sqrt 3)^d, so with H chosen per dtype the central values equal the
// full-line values to below the rounding unit (the mimetic stencils have a
// finite dependence cone and H covers it exactly).
//
// Compact operators (Appendix A): G = P^-1 Q, D = Pbar^-1 Qbar, each one
// tridiagonal solve with the no-pivot LU factors of the window-restricted
// matrix (precomputed on the host per window, staged in LDS).  A window edge
// inside the line gets the diagonal 2 + sqrt 3 so its factors equal the
// interior limit.  Within a workgroup the forward and backward recurrences
// are split over segments: each lane runs its segment with zero carry, the
// carries of the previous (next) TS segments are combined from LDS, and the
// segment is corrected with the products of the multipliers.  Carries from
// farther segments are below the rounding unit (factor (2 - sqrt 3)^(R TS)).
//
// Mimetic operators (Appendix B): explicit 4-tap stencils with the printed
// 6/5-tap boundary rows and their centro-skew mirrors.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "line_pass.h"
#include "pass_common.h"
#include <type_traits>

namespace adi {

// Tile shapes (lines per workgroup LW, slots per lane R, waves NW, carry
// reach TS in segments) for windows of 512, 256 and 128 slots.  Short lines
// take the smallest window that holds them, with more lines per workgroup.
// Shapes 3 .. 5 have the windows of 0 .. 2 with 4 waves and a quarter of the
// lines: four times the workgroups, for problems with few lines.
template <typename T, int CF> struct Tile;
template <> struct Tile<float, 0> { static constexpr int LW = 32, R = 16, NW = 16, TS = 2; };
template <> struct Tile<float, 1> { static constexpr int LW = 64, R = 16, NW = 16, TS = 2; };
template <> struct Tile<float, 2> { static constexpr int LW = 64, R = 8, NW = 16, TS = 4; };
template <> struct Tile<float, 3> { static constexpr int LW = 8, R = 16, NW = 4, TS = 2; };
template <> struct Tile<float, 4> { static constexpr int LW = 16, R = 16, NW = 4, TS = 2; };
template <> struct Tile<float, 5> { static constexpr int LW = 16, R = 8, NW = 4, TS = 4; };
template <> struct Tile<double, 0> { static constexpr int LW = 16, R = 8, NW = 16, TS = 4; };
template <> struct Tile<double, 1> { static constexpr int LW = 32, R = 8, NW = 16, TS = 4; };
template <> struct Tile<double, 2> { static constexpr int LW = 64, R = 8, NW = 16, TS = 4; };
template <> struct Tile<double, 3> { static constexpr int LW = 4, R = 8, NW = 4, TS = 4; };
template <> struct Tile<double, 4> { static constexpr int LW = 8, R = 8, NW = 4, TS = 4; };
template <> struct Tile<double, 5> { static constexpr int LW = 16, R = 8, NW = 4, TS = 4; };

template <typename T, int CF> struct K {
    static constexpr int LW = Tile<T, CF>::LW, R = Tile<T, CF>::R, NW = Tile<T, CF>::NW, TS = Tile<T, CF>::TS;
    static constexpr int SPW = 64 / LW;
    static constexpr int NSEG = NW * SPW;
    static constexpr int WS = NSEG * R;
    static constexpr int NT = NW * 64;
    static constexpr int SL = NSEG * LW;   // one LDS field: a value per lane
};

static_assert(K<float, 0>::WS == LINE_WS && K<double, 0>::WS == LINE_WS, "window size");
static_assert(K<float, 1>::WS == 256 && K<double, 1>::WS == 256, "window size");
static_assert(K<float, 2>::WS == 128 && K<double, 2>::WS == 128, "window size");
static_assert(K<float, 3>::WS == LINE_WS && K<double, 3>::WS == LINE_WS, "window size");
static_assert(K<float, 4>::WS == 256 && K<double, 4>::WS == 256, "window size");
static_assert(K<float, 5>::WS == 128 && K<double, 5>::WS == 128, "window size");

template <int METHOD> struct Halo;
template <> struct Halo<LINE_CFD> { static constexpr int N = 1, DEEP = 3; };
template <> struct Halo<LINE_MFD> { static constexpr int N = 2, DEEP = 5; };

// Value at compile-time position p of the lane's extended line: own slots,
// or halos from the neighbouring segments; zero beyond the halos.
template <typename T, int R, int D>
__device__ __forceinline__ T xv(const T (&x)[R], const T (&hl)[D], const T (&hr)[D], int p) {
    return p < -D ? T(0) : (p < 0 ? hl[D + p] : (p < R ? x[p] : (p < R + D ? hr[p - R] : T(0))));
}

template <typename T, int CF, int METHOD> struct Pass {
    using C = K<T, CF>;
    static constexpr int LW = C::LW, R = C::R, NSEG = C::NSEG, WS = C::WS, SL = C::SL, TS = C::TS;
    static constexpr int DN = Halo<METHOD>::N, DD = Halo<METHOD>::DEEP;
    static constexpr int HF = (4 * DN > 2 * DD ? 4 * DN : 2 * DD) / 2;   // fields per ring half
    static constexpr int RING = 2 * HF * SL;                              // elements
    static constexpr int TAB = METHOD == LINE_CFD ? 6 * WS : 0;
    static constexpr int TILEP = WS + 1;                                  // padded tile row
    static constexpr int TILE = LW * TILEP;
    static constexpr int WORK = RING + TAB;
    static constexpr int SMEM = WORK > TILE ? WORK : TILE;

    const LinePassArgs<T>& a;
    T* ring;
    const T* tab;
    int seg, lq, li, s0, q, n, xc;
    bool deep, bnd;

    __device__ Pass(const LinePassArgs<T>& args, T* smem, int seg_, int lq_, int s0_, int q_)
        : a(args), ring(smem), tab(smem + RING), seg(seg_), lq(lq_), li(seg_ * LW + lq_), s0(s0_),
          q(q_), n(args.n), xc(0), deep(args.deep != 0), bnd(s0_ <= 1 || s0_ + R - 1 >= args.n - 1) {}

    // ---- halo exchange of the first / last D values of x ----
    template <int D>
    __device__ __forceinline__ void publish(T* b, const T (&x)[R]) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            b[i * SL + li] = x[i];
            b[(D + i) * SL + li] = x[R - D + i];
        }
    }
    template <int D>
    __device__ __forceinline__ void fetch(const T* b, T (&hl)[D], T (&hr)[D]) {
#pragma unroll
        for (int i = 0; i < D; ++i) {
            hl[i] = seg > 0 ? b[(D + i) * SL + (seg - 1) * LW + lq] : T(0);
            hr[i] = seg < NSEG - 1 ? b[i * SL + (seg + 1) * LW + lq] : T(0);
        }
    }

    // ---- pressure -> velocity derivative right-hand side / stencil ----
    template <int D>
    __device__ __forceinline__ void stencil_g(const T (&x)[R], const T (&hl)[D], const T (&hr)[D], T (&o)[R]) {
        const T ih = a.inv_h;
        if (METHOD == LINE_CFD) {
            // Q4 u / h: interior 3 (u_{s+1} - u_{s-1}) / h
            const T c3 = T(3) * ih;
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = c3 * (xv(x, hl, hr, k + 1) - xv(x, hl, hr, k - 1));
            // (products and sums written as explicit fma chains here and
            // below: every instantiation of the kernel then rounds them alike)
            if (bnd) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int s = s0 + k;
                    if (s == 0)
                        o[k] = ih * fma(T(-17), xv(x, hl, hr, k),
                                        fma(T(9), xv(x, hl, hr, k + 1),
                                            fma(T(9), xv(x, hl, hr, k + 2), -xv(x, hl, hr, k + 3))));
                    if (s == n)
                        o[k] = ih * fma(T(17), xv(x, hl, hr, k),
                                        fma(T(-9), xv(x, hl, hr, k - 1),
                                            fma(T(-9), xv(x, hl, hr, k - 2), xv(x, hl, hr, k - 3))));
                }
            }
        } else {
            // G4 u: interior (u_{s-1} - 27 u_s + 27 u_{s+1} - u_{s+2}) / (24 h)
            const T c1 = T(9.0 / 8.0) * ih, c0 = T(-1.0 / 24.0) * ih;
#pragma unroll
            for (int k = 0; k < R; ++k)
                o[k] = fma(c1, xv(x, hl, hr, k + 1) - xv(x, hl, hr, k),
                           c0 * (xv(x, hl, hr, k + 2) - xv(x, hl, hr, k - 1)));
            if (bnd) {
                const T g0[6] = {T(-47888.0 / 14245.0), T(1790.0 / 407.0), T(-14545.0 / 9768.0),
                                 T(8997.0 / 16280.0), T(-2335.0 / 22792.0), T(25.0 / 9768.0)};
                const T g1[5] = {T(16.0 / 105.0), T(-31.0 / 24.0), T(29.0 / 24.0), T(-3.0 / 40.0),
                                 T(1.0 / 168.0)};
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int s = s0 + k;
                    if (s == 0) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(g0[c], xv(x, hl, hr, k + c), acc);
                        o[k] = acc * ih;
                    }
                    if (s == 1) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 5; ++c) acc = fma(g1[c], xv(x, hl, hr, k - 1 + c), acc);
                        o[k] = acc * ih;
                    }
                    if (s == n - 1) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 5; ++c) acc = fma(g1[c], xv(x, hl, hr, k + 2 - c), acc);
                        o[k] = -acc * ih;
                    }
                    if (s == n) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(g0[c], xv(x, hl, hr, k + 1 - c), acc);
                        o[k] = -acc * ih;
                    }
                }
            }
        }
    }

    // ---- velocity -> pressure derivative right-hand side / stencil ----
    template <int D>
    __device__ __forceinline__ void stencil_d(const T (&x)[R], const T (&hl)[D], const T (&hr)[D], T (&o)[R]) {
        const T ih = a.inv_h;
        if (METHOD == LINE_CFD) {
            const T c3 = T(3) * ih;
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = c3 * (xv(x, hl, hr, k + 1) - xv(x, hl, hr, k - 1));
            if (bnd) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int s = s0 + k;
                    if (s == 1)
                        o[k] = ih * fma(T(-9), xv(x, hl, hr, k),
                                        fma(T(9), xv(x, hl, hr, k + 1),
                                            xv(x, hl, hr, k + 2) - xv(x, hl, hr, k - 1)));
                    if (s == n - 1)
                        o[k] = ih * fma(T(-9), xv(x, hl, hr, k - 1),
                                        fma(T(9), xv(x, hl, hr, k), xv(x, hl, hr, k + 1) - xv(x, hl, hr, k - 2)));
                }
            }
        } else {
            const T c1 = T(9.0 / 8.0) * ih, c0 = T(-1.0 / 24.0) * ih;
#pragma unroll
            for (int k = 0; k < R; ++k)
                o[k] = fma(c1, xv(x, hl, hr, k) - xv(x, hl, hr, k - 1),
                           c0 * (xv(x, hl, hr, k + 1) - xv(x, hl, hr, k - 2)));
            if (bnd) {
                const T d0[6] = {T(-4751.0 / 5192.0), T(909.0 / 1298.0), T(6091.0 / 15576.0),
                                 T(-1165.0 / 5192.0), T(129.0 / 2596.0), T(-25.0 / 15576.0)};
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int s = s0 + k;
                    if (s == 1) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(d0[c], xv(x, hl, hr, k - 1 + c), acc);
                        o[k] = acc * ih;
                    }
                    if (s == n) {
                        T acc = T(0);
#pragma unroll
                        for (int c = 0; c < 6; ++c) acc = fma(d0[c], xv(x, hl, hr, k - c), acc);
                        o[k] = -acc * ih;
                    }
                }
            }
        }
    }

    // o = derivative (kind 0: pressure->velocity, 1: velocity->pressure) of x
    template <int KIND>
    __device__ __forceinline__ void deriv(const T (&x)[R], T (&o)[R]) {
        if (!deep) {
            T hl[DN], hr[DN];
            T* b = ring + (xc & 1) * HF * SL;
            ++xc;
            publish<DN>(b, x);
            __syncthreads();
            fetch<DN>(b, hl, hr);
            if (KIND == 0) stencil_g<DN>(x, hl, hr, o); else stencil_d<DN>(x, hl, hr, o);
        } else {
            T hl[DD], hr[DD];
            __syncthreads();
            publish<DD>(ring, x);
            __syncthreads();
            fetch<DD>(ring, hl, hr);
            __syncthreads();
            if (KIND == 0) stencil_g<DD>(x, hl, hr, o); else stencil_d<DD>(x, hl, hr, o);
        }
        if (METHOD == LINE_CFD) solve(o, tab + (KIND == 0 ? 0 : 3 * WS));
    }

    // In-place solve of the window's tridiagonal system (factor tables t:
    // multipliers, inverse pivots, superdiagonal times inverse pivot).
    __device__ __forceinline__ void solve(T (&x)[R], const T* t) {
        const int sl0 = seg * R;
        const T* m = t + sl0;
        const T* dv = t + WS + sl0;
        const T* e = t + 2 * WS + sl0;
        // forward elimination with zero carry-in
        T g = -m[0];
#pragma unroll
        for (int k = 1; k < R; ++k) {
            const T mk = m[k];
            x[k] = fma(-mk, x[k - 1], x[k]);
            g = -mk * g;
        }
        T* b = ring + (xc & 1) * HF * SL;
        ++xc;
        b[li] = x[R - 1];
        b[SL + li] = g;
        __syncthreads();
        T Y = T(0), pref = T(1);
#pragma unroll
        for (int tt = 1; tt <= TS; ++tt) {
            const int sg = seg - tt;
            if (sg >= 0) {
                Y = fma(pref, b[sg * LW + lq], Y);
                pref *= b[SL + sg * LW + lq];
            }
        }
        T gg = -m[0];
        x[0] = fma(gg, Y, x[0]);
#pragma unroll
        for (int k = 1; k < R; ++k) {
            gg = -m[k] * gg;
            x[k] = fma(gg, Y, x[k]);
        }
        // back substitution with zero carry-in
        x[R - 1] *= dv[R - 1];
        T qv = -e[R - 1];
#pragma unroll
        for (int k = R - 2; k >= 0; --k) {
            x[k] = fma(-e[k], x[k + 1], x[k] * dv[k]);
            qv = -e[k] * qv;
        }
        b = ring + (xc & 1) * HF * SL;
        ++xc;
        b[li] = x[0];
        b[SL + li] = qv;
        __syncthreads();
        T X = T(0);
        pref = T(1);
#pragma unroll
        for (int tt = 1; tt <= TS; ++tt) {
            const int sg = seg + tt;
            if (sg < NSEG) {
                X = fma(pref, b[sg * LW + lq], X);
                pref *= b[SL + sg * LW + lq];
            }
        }
        T qq = -e[R - 1];
        x[R - 1] = fma(qq, X, x[R - 1]);
#pragma unroll
        for (int k = R - 2; k >= 0; --k) {
            qq = -e[k] * qq;
            x[k] = fma(qq, X, x[k]);
        }
    }
};

// One workgroup's share of a pass: line group `tile` (one window per line).
// FULL: the variant with the optional features (damping layers, wall data,
// distributed forcing); the plain variant has none of their code.
// EPS: the tolerance-tested form (LinePassArgs::eps_part; Algorithms 3 and
// 4): the last two sweeps keep their previous iterate in a spare array and
// the squared changes of u_{K-1}, v_{K-1}, u_K and v_K over the slots the
// window writes become this tile's partials.
template <typename T, int CF, int METHOD, int MODE, bool COMP, bool FULL = false, bool EPS = false>
__device__ __forceinline__ void lp_body(const LinePassArgs<T>& a, int tile, T* smem) {
    static_assert(!(EPS && (COMP || FULL || MODE == LINE_EXPLICIT)), "tolerance-tested plain sweeps only");
    using P = Pass<T, CF, METHOD>;
    using C = K<T, CF>;
    constexpr int LW = C::LW, R = C::R, SPW = C::SPW, WS = C::WS;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lq = lane % LW;
    const int seg = wave * SPW + lane / LW;
    const int lg = tile % a.nlg;
    const int g = tile / a.nlg;
    const int c0 = g * a.S;
    const int c1 = min(c0 + a.S, a.ns);
    int w0 = 0;
    if (a.nwin > 1) w0 = max(0, min(c0 - a.H, a.ns - WS));
    const int s0 = w0 + seg * R;
    const int q = lg * LW + lq;
    const bool qok = q < a.nlines;
    const int n = a.n;
    const int ulo = 1, uhi = METHOD == LINE_CFD ? n - 1 : n;   // interior pressure slots
    const int vhi = n;                                          // velocity slots 0..n

    P p(a, smem, seg, lq, s0, q);
    T ev[4] = {T(0), T(0), T(0), T(0)};   // tolerance test: change sums (EPS only)

    if (METHOD == LINE_CFD) {
        const T* src = a.coef + (size_t)g * 6 * WS;
        for (int i = tid; i < 6 * WS; i += C::NT) smem[P::RING + i] = src[i];
    }

    T A[R], B[R], KK[R], RR[R], U[R], Tt[R];
    // Dirichlet wall values at the first and last pressure slots of the line
    T wl = T(0), wr = T(0);
    if ((FULL || COMP) && a.bnd && qok) {
        wl = a.bsc[0] * a.bnd[6 * q] + a.bsc[1] * a.bnd[6 * q + 1] + a.bsc[2] * a.bnd[6 * q + 2];
        wr = a.bsc[0] * a.bnd[6 * q + 3] + a.bsc[1] * a.bnd[6 * q + 4] + a.bsc[2] * a.bnd[6 * q + 5];
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int s = s0 + k;
        const bool uv = qok && s >= ulo && s <= uhi;
        const bool vv = qok && s <= vhi;
        A[k] = uv ? a.uin[(int64_t)(s - 1) * a.uin_ld + q] : (s == 0 ? wl : (s == uhi + 1 ? wr : T(0)));
        KK[k] = uv ? (a.ak ? a.ak[(int64_t)(s - 1) * a.ak_ld + q] : a.ak0) : T(0);
        B[k] = vv ? a.vin[(int64_t)s * a.vin_ld + q] : T(0);
        RR[k] = vv ? (a.ar ? a.ar[(int64_t)s * a.ar_ld + q] : a.ar0) : T(0);
    }
    if (METHOD == LINE_CFD) __syncthreads();   // tables visible

    // Damping layers (the damped system): implicit rows divided by 1 + a d,
    // explicit parts multiplied by 1 - a d; the pressure rows are divided
    // here, the velocity rows after the first half sweep
    const bool damp = FULL && !COMP && a.dmpm != 0;
    auto dpres = [&](int s) { return damp_at(a, pres_pos<METHOD, T>(s, n)); };
    auto dvel = [&](int s) { return damp_at(a, T(s)); };
    if (MODE != LINE_EXPLICIT && damp) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T e = T(1) / fma(a.ah, dpres(s0 + k), T(1));
            A[k] *= e;
            KK[k] *= e;
        }
    }

    if (MODE == LINE_EXPLICIT || COMP) {
        p.template deriv<0>(A, Tt);                 // G(A)
        p.template deriv<1>(B, U);                  // D(B)
        if (MODE == LINE_EXPLICIT) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                // W* = B - aR G(A), A_out = A - aK D(B)   (increments when compensated;
                // B, A times 1 - a d with damping)
                const T bb = damp ? B[k] * fma(-a.ah, dvel(s0 + k), T(1)) : B[k];
                const T aa = damp ? A[k] * fma(-a.ah, dpres(s0 + k), T(1)) : A[k];
                Tt[k] = COMP ? -RR[k] * Tt[k] : fma(-RR[k], Tt[k], bb);
                U[k] = COMP ? -KK[k] * U[k] : fma(-KK[k], U[k], aa);
            }
        } else {
            // compensated: iterate on the increments, A' = -aK D(B), B' = -aR G(A)
#pragma unroll
            for (int k = 0; k < R; ++k) {
                A[k] = -KK[k] * U[k];
                B[k] = -RR[k] * Tt[k];
                U[k] = A[k];
            }
        }
    }
    if (MODE != LINE_EXPLICIT) {
        if (!COMP) {
            p.template deriv<1>(B, U);
#pragma unroll
            for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
        }
        if (damp) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T e = T(1) / fma(a.ah, dvel(s0 + k), T(1));
                B[k] *= e;
                RR[k] *= e;
            }
        }
        if constexpr (EPS) {
            // the slots this window writes (pressure: interior slots;
            // velocity: slots 0..n); the masks pass through an empty asm at
            // each use so that the per-slot tests are not hoisted out of
            // the sweeps as lane masks, and the changes are masked by a
            // product rather than a select
            int umask = 0, vmask = 0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int s = s0 + k;
                const bool own = qok && s >= c0 && s < c1;
                if (own && s >= ulo && s <= uhi) umask |= 1 << k;
                if (own && s <= vhi) vmask |= 1 << k;
            }
            auto opaque = [](int m) {
                asm volatile("" : "+v"(m));
                return m;
            };
            auto chg = [](T x, T y, int on) {
                const T d = (x - y) * T(on);
                return d * d;
            };
            T X[R];
#pragma unroll
            for (int k = 0; k < R; ++k) Tt[k] = B[k];                     // v_0
            // one sweep (v_it, then u_{it+1}); tv: sum the change of v,
            // qi >= 0: sum the change of u into ev[qi]
            auto sweep = [&](bool tv, int qi) {
                const int vm = opaque(vmask), um = opaque(umask);
                p.template deriv<0>(U, X);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T vn = fma(-RR[k], X[k], B[k]);
                    if (tv) ev[1] += chg(vn, Tt[k], (vm >> k) & 1);
                    Tt[k] = vn;
                }
                p.template deriv<1>(Tt, X);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T un = fma(-KK[k], X[k], A[k]);
                    if (qi >= 0) ev[qi] += chg(un, U[k], (um >> k) & 1);
                    U[k] = un;
                }
            };
            // sweeps it = 1 .. K - 1: untracked, then u_{K-1}, then v_{K-1} and u_K
            for (int it = 1; it < a.sweeps - 2; ++it) sweep(false, -1);
            if (a.sweeps >= 3) sweep(false, 0);
            sweep(true, 2);
            const int vm = opaque(vmask);
            p.template deriv<0>(U, X);
#pragma unroll
            for (int k = 0; k < R; ++k) {                                  // v_K
                const T vn = fma(-RR[k], X[k], B[k]);
                ev[3] += chg(vn, Tt[k], (vm >> k) & 1);
                Tt[k] = vn;
            }
        } else {
            for (int it = 1; it < a.sweeps; ++it) {
                p.template deriv<0>(U, Tt);
#pragma unroll
                for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);
                p.template deriv<1>(Tt, U);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
            }
            p.template deriv<0>(U, Tt);
#pragma unroll
            for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);   // v_K
        }
        if (MODE == LINE_SWEEP) {
            if (COMP) {
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] += A[k];
            }
            p.template deriv<1>(Tt, A);                                   // D(v_K)
            if (damp) {
                // B and aK restored from their divided forms
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T dp = a.ah * dpres(s0 + k), vk = Tt[k];
                    Tt[k] = vk + (vk - B[k] * fma(a.ah, dvel(s0 + k), T(1)));
                    U[k] = fma(-KK[k] * (T(1) + dp), A[k], U[k] * (T(1) - dp));
                }
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const T vk = Tt[k];
                    Tt[k] = COMP ? vk + vk : vk + (vk - B[k]);             // 2 v_K - B
                    U[k] = fma(-KK[k], A[k], U[k]);                        // u_K - aK D(v_K)
                }
            }
        }
    }

    if constexpr (EPS) {
        // wave sums, then the workgroup's, stored as this tile's partials
        __shared__ double wsum[C::NW][4];
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            double v = (double)ev[qi];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) wsum[wave][qi] = v;
        }
        __syncthreads();
        if (tid < 4) {
            double v = 0.0;
            for (int w = 0; w < C::NW; ++w) v += wsum[w][tid];
            a.eps_part[(int64_t)tid * a.nlg * a.nwin + tile] = v;
        }
    }
    if ((FULL || COMP) && MODE != LINE_FINAL && a.ff) {
        // distributed forcing on the interior pressure slots
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int s = s0 + k;
            if (qok && s >= ulo && s <= uhi) U[k] = fma(a.aFf, a.ff[(int64_t)(s - 1) * a.ff_ld + q], U[k]);
        }
    }
    pass_outputs<T, R, LW, C::NT, P::TILEP, COMP>(a, smem, Tt, U, s0, q, qok, lq, lg, c0, c1, uhi, vhi,
                                                  tid, MODE != LINE_FINAL);
}

template <typename T, int CF, int METHOD, int MODE, bool COMP, bool FULL, bool EPS = false>
__global__ void __launch_bounds__((K<T, CF>::NT)) line_pass_kernel(const LinePassArgs<T> a) {
    __shared__ T smem[Pass<T, CF, METHOD>::SMEM];
    // uniform: an earlier attempt of a tolerance-tested pass converged
    if (EPS && *a.eps_go == 0) return;
    lp_body<T, CF, METHOD, MODE, COMP, FULL, EPS>(a, (int)blockIdx.x, smem);
}

// Several passes (of several problems) in one launch: each workgroup finds
// its pass in the prefix sums of the block counts.
template <typename T, int CF, int METHOD, int MODE, bool COMP, bool FULL>
__global__ void __launch_bounds__((K<T, CF>::NT)) line_pass_group_kernel(const GroupArgs<T> ga) {
    __shared__ T smem[Pass<T, CF, METHOD>::SMEM];
    int tile;
    const int it = group_item(ga, tile);
    if (it < 0) return;
    LinePassArgs<T> a = ga.items[it];
    if (a.aFtab) a.aF = a.aFtab[*ga.tick];
    lp_body<T, CF, METHOD, MODE, COMP, FULL>(a, tile, smem);
}

// ------------------------------------------------------------------------
// Setup kernels: scaled copy with optional transpose (32 x 32 LDS tiles).
//   dst[r * dld + c] = scale * src[r * srs + c * scs],  r < rows, c < cols
// With scs == 1 rows are read contiguously; with srs == 1 the tile is read
// along columns and written along rows (a transpose).
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) scaled_copy_kernel(T* __restrict__ dst, int64_t dld,
                                                          const T* __restrict__ src, int64_t srs,
                                                          int64_t scs, int rows, int cols, T scale,
                                                          const T* __restrict__ src2) {
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    if (srs == 1) {
        // source contiguous along r: read with tx along r
#pragma unroll
        for (int i = 0; i < 32; i += 8) {
            const int r = r0 + tx, c = c0 + ty + i;
            const int64_t o = (int64_t)r * srs + (int64_t)c * scs;
            tile[ty + i][tx] = (r < rows && c < cols) ? (src2 ? src[o] + src2[o] : src[o]) : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 32; i += 8) {
            const int r = r0 + ty + i, c = c0 + tx;
            if (r < rows && c < cols) dst[(int64_t)r * dld + c] = scale * tile[tx][ty + i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 32; i += 8) {
            const int r = r0 + ty + i, c = c0 + tx;
            if (r < rows && c < cols) {
                const int64_t o = (int64_t)r * srs + (int64_t)c * scs;
                dst[(int64_t)r * dld + c] = scale * (src2 ? src[o] + src2[o] : src[o]);
            }
        }
    }
}

template <typename T, int CF, bool COMP, bool FULL>
hipError_t launch_lp(const LinePassArgs<T>* a, const GroupArgs<T>* ga, int method, int mode, hipStream_t st) {
    const unsigned nb = a ? (unsigned)(a->nlg * a->nwin) : (unsigned)(((ga->total + 7) / 8) * 8);
    if (nb == 0) return hipSuccess;
    dim3 grid(nb), block(K<T, CF>::NT);
    const bool eps = a && a->eps_part;
    if (eps && (COMP || FULL || mode == LINE_EXPLICIT)) return hipErrorInvalidValue;
#define LP_CASE(M, MD)                                                                                  \
    if (method == M && mode == MD) {                                                                    \
        if constexpr (!COMP && !FULL && MD != LINE_EXPLICIT) {                                          \
            if (eps) {                                                                                  \
                hipLaunchKernelGGL((line_pass_kernel<T, CF, M, MD, false, false, true>), grid, block, 0, st, *a); \
                return hipGetLastError();                                                               \
            }                                                                                           \
        }                                                                                               \
        if (a)                                                                                          \
            hipLaunchKernelGGL((line_pass_kernel<T, CF, M, MD, COMP, FULL>), grid, block, 0, st, *a);        \
        else                                                                                                  \
            hipLaunchKernelGGL((line_pass_group_kernel<T, CF, M, MD, COMP, FULL>), grid, block, 0, st, *ga); \
        return hipGetLastError();                                                                       \
    }
    LP_CASE(LINE_CFD, LINE_SWEEP)
    LP_CASE(LINE_CFD, LINE_FINAL)
    LP_CASE(LINE_CFD, LINE_EXPLICIT)
    LP_CASE(LINE_MFD, LINE_SWEEP)
    LP_CASE(LINE_MFD, LINE_FINAL)
    LP_CASE(LINE_MFD, LINE_EXPLICIT)
#undef LP_CASE
    return hipErrorInvalidValue;
}

template <typename T, bool COMP, bool FULL>
hipError_t launch_lp_cfg(const LinePassArgs<T>* a, const GroupArgs<T>* ga, int cfg, int method, int mode,
                         hipStream_t st) {
    switch (cfg) {
        case 0: return launch_lp<T, 0, COMP, FULL>(a, ga, method, mode, st);
        case 1: return launch_lp<T, 1, COMP, FULL>(a, ga, method, mode, st);
        case 2: return launch_lp<T, 2, COMP, FULL>(a, ga, method, mode, st);
        case 3: return launch_lp<T, 3, COMP, FULL>(a, ga, method, mode, st);
        case 4: return launch_lp<T, 4, COMP, FULL>(a, ga, method, mode, st);
        case 5: return launch_lp<T, 5, COMP, FULL>(a, ga, method, mode, st);
        default: return hipErrorInvalidValue;
    }
}

// variants: plain, compensated (FP32; wall data and forcing included), with
// the optional features (damping layers, wall data, forcing; not compensated)
template <typename T>
hipError_t launch_lp_any(const LinePassArgs<T>* a, const GroupArgs<T>* ga, int cfg, int method, int mode,
                         hipStream_t st, bool comp, bool full) {
    if (comp && full) return hipErrorInvalidValue;
    if (full) return launch_lp_cfg<T, false, true>(a, ga, cfg, method, mode, st);
    if (!comp) return launch_lp_cfg<T, false, false>(a, ga, cfg, method, mode, st);
    if constexpr (std::is_same<T, float>::value) return launch_lp_cfg<T, true, false>(a, ga, cfg, method, mode, st);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_line_pass(const LinePassArgs<T>& a, int method, int mode, hipStream_t st, bool comp, int cfg,
                            bool full) {
    return launch_lp_any<T>(&a, nullptr, cfg, method, mode, st, comp, full);
}

template <typename T>
hipError_t launch_line_group(const GroupArgs<T>& ga, int cfg, int method, int mode, hipStream_t st, bool comp,
                             bool full) {
    if (ga.total <= 0) return hipSuccess;
    return launch_lp_any<T>(nullptr, &ga, cfg, method, mode, st, comp, full);
}

template <typename T>
hipError_t launch_scaled_copy(T* dst, int64_t dld, const T* src, int64_t srs, int64_t scs, int rows,
                              int cols, T scale, hipStream_t st, const T* src2) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32)), block(256);
    hipLaunchKernelGGL((scaled_copy_kernel<T>), grid, block, 0, st, dst, dld, src, srs, scs, rows, cols, scale,
                       src2);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) fill_zero_kernel(T* __restrict__ dst, int64_t dld, int rows, int cols) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (c < cols && r < rows) dst[(int64_t)r * dld + c] = T(0);
}

template <typename T>
hipError_t launch_fill_zero(T* dst, int64_t dld, int rows, int cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 255) / 256), (unsigned)rows), block(256);
    hipLaunchKernelGGL((fill_zero_kernel<T>), grid, block, 0, st, dst, dld, rows, cols);
    return hipGetLastError();
}

int line_lanes(int dtype, int cfg) {
    static const int lw[2][LINE_NCFG] = {
        {K<float, 0>::LW, K<float, 1>::LW, K<float, 2>::LW, K<float, 3>::LW, K<float, 4>::LW, K<float, 5>::LW},
        {K<double, 0>::LW, K<double, 1>::LW, K<double, 2>::LW, K<double, 3>::LW, K<double, 4>::LW,
         K<double, 5>::LW}};
    return lw[dtype == 1 ? 1 : 0][cfg];
}
int line_ws(int cfg) {
    static const int ws[LINE_NCFG] = {K<float, 0>::WS, K<float, 1>::WS, K<float, 2>::WS,
                                      K<float, 3>::WS, K<float, 4>::WS, K<float, 5>::WS};
    return ws[cfg];
}

// Overlap of neighbouring windows, in slots.  Mimetic: the dependence cone
// of K sweeps plus the final derivative is 3K + 2 slots; two slots spare.
// Compact: the window-edge error decays like (2 - sqrt 3)^d times a
// polynomial in d of the degree of the number of chained solves (2K + 1),
// and faster at smaller step sizes.  A model of one line pass on a whole
// line and on a window cut out of it (the outside dropped, the interior
// pivot at the window's first row) puts the truncation at these margins
// below 2^-24 (FP32) and at the FP64 rounding level (FP64 and the
// compensated mode) for K = 2..16 and every cfl up to 1.149; for K = 6 the
// FP32 margin leaves 3e-10 at cfl 0.8 and 2e-8 at 1.149.  All margins are
// even (K is even): the windows of the wave-per-line kernel then start on
// multiples of 4 slots.
int line_halo(int dtype, int method, int sweeps, double cfl) {
    if (method == LINE_MFD) return 3 * sweeps + 4;
    if (dtype == 0) return 18 + 2 * sweeps;
    return cfl <= 0.85 ? 36 + 2 * sweeps : 40 + 3 * sweeps;
}

template hipError_t launch_line_pass<float>(const LinePassArgs<float>&, int, int, hipStream_t, bool, int, bool);
template hipError_t launch_line_pass<double>(const LinePassArgs<double>&, int, int, hipStream_t, bool, int, bool);
template hipError_t launch_line_group<float>(const GroupArgs<float>&, int, int, int, hipStream_t, bool, bool);
template hipError_t launch_line_group<double>(const GroupArgs<double>&, int, int, int, hipStream_t, bool, bool);
template hipError_t launch_scaled_copy<float>(float*, int64_t, const float*, int64_t, int64_t, int, int, float,
                                             hipStream_t, const float*);
template hipError_t launch_scaled_copy<double>(double*, int64_t, const double*, int64_t, int64_t, int, int, double,
                                              hipStream_t, const double*);
template hipError_t launch_fill_zero<float>(float*, int64_t, int, int, hipStream_t);
template hipError_t launch_fill_zero<double>(double*, int64_t, int, int, hipStream_t);

}  // namespace adi
