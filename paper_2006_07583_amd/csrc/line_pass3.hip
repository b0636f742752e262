// Multi-window line pass with one grid line per half wave (lines longer than
// one window; FP32 and FP64).
//
// Same arithmetic as the other line-pass kernels: one launch performs the
// fixed-point sweeps of a Peaceman-Rachford stage along every line of one
// direction, fused with the explicit half of the following stage
// (Algorithms 1-4).  The difference is where a line lives:
//
//  * A line's window of 512 slots is held by 32 lanes of one wave, R = 16
//    consecutive slots per lane, two lines per wave.  Everything the
//    segmented solves and stencils exchange between neighbouring segments
//    moves between neighbouring lanes with DPP wave shifts: the sweep loop
//    has no workgroup barrier and no LDS traffic, and the waves of a
//    workgroup progress independently.
//  * The arrays of a direction are line-major (a line's slots contiguous,
//    rows padded); every global access moves whole 16-byte chunks along
//    the lines and passes through an LDS tile of the workgroup's LW lines,
//    whose per-lane chunks are rotated so that lanes never share a bank.  A
//    window that does not start on the 16-byte grid (the last one) is read
//    from the grid slot below it and shifted in LDS.  The pressure handed to
//    the other direction leaves the tile transposed, LW lines forming one
//    contiguous run of the other layout.
//  * Compact scheme: scaled unknowns, zero-carry segment solves, one
//    carry combination per solve (constants of the interior factors), and a
//    low-rank correction in the windows holding the first or last slot of
//    the line that turns the constant-factor matrix into P4 / Pbar4; the
//    correction values are broadcast from the lane holding the boundary
//    rows with readlane.
//  * Mimetic scheme: the 4-tap stencils need the last / first 3 values of
//    the neighbouring lanes: 6 lane shifts per velocity evaluation.
//  * Compensated FP32 (COMP): the carried state is a (value, low word) pair.
//    The pass takes the derivatives of the values once, iterates on the
//    increments u - A and v - B (small numbers, so FP32 loses little), and
//    adds the final increments to the pairs with TwoSum; the pairs are read
//    again through the tile for that last step.
//
// Lanes at the window edges see zeros beyond the window; the windows overlap
// by H slots on each side and only the central slots are written (the
// margins H are the ones the other kernels use).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "line_consts.h"
#include "line_pass.h"
#include "pass_common.h"
#include "tile_map.h"

namespace adi {

template <typename T> struct Cfg3;
// waves per workgroup, lines per wave, slots per lane, carry reach (segments), waves per SIMD
// (FP32: four workgroups of 4 waves per CU at 116 registers overlap the
// staging rounds of one with the sweeps of the others better than two of 8
// waves; the transposed pressure runs are then 8 lines, 32 bytes, long.)
template <> struct Cfg3<float> {
    static constexpr int NWV = 4, LPW = 2, R = 16, TS = 1, WPE = 4;
};
template <> struct Cfg3<double> {
    static constexpr int NWV = 4, LPW = 2, R = 16, TS = 2, WPE = 2;
};

template <typename T> struct K3 {
    static constexpr int NWV = Cfg3<T>::NWV, LPW = Cfg3<T>::LPW, R = Cfg3<T>::R, TS = Cfg3<T>::TS;
    static constexpr int LPL = 64 / LPW;          // lanes per line
    static constexpr int WS = LPL * R;             // slots per window
    static constexpr int LW = NWV * LPW;           // lines per workgroup
    static constexpr int NT = NWV * 64;
    // LDS tile row pitch: rows stay 16-byte aligned so that a lane moves its
    // segment with 128-bit LDS accesses
    static constexpr int TP = WS + 4;
    static constexpr int TILE = LW * TP;
    static constexpr int TPL = NT / LW;            // threads per line in the transposed store
};
static_assert(K3<float>::WS == LINE_WS && K3<double>::WS == LINE_WS, "window size");

// element (line, position) of the LDS tile
template <typename T>
__device__ __forceinline__ int tix(int line, int pos) {
    return line * K3<T>::TP + pos;
}

// Tile-row positions of the window slots (chunks rotated per lane, tile_map.h).
template <typename T> using TMap = TileMap<K3<T>::R, (int)sizeof(T)>;

// Lane shifts across the whole wave: lane l receives lane l - 1 (shr) or
// l + 1 (shl); lanes without a source receive 0 (bound control).
__device__ __forceinline__ int dpp_shr1(int x) { return __builtin_amdgcn_mov_dpp(x, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_shl1(int x) { return __builtin_amdgcn_mov_dpp(x, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float wshr(float x) { return __int_as_float(dpp_shr1(__float_as_int(x))); }
__device__ __forceinline__ float wshl(float x) { return __int_as_float(dpp_shl1(__float_as_int(x))); }
__device__ __forceinline__ double wshr(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_shr1((int)(b & 0xffffffffLL)), hi = dpp_shr1((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wshl(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_shl1((int)(b & 0xffffffffLL)), hi = dpp_shl1((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// value of lane `src` (uniform) of the wave
__device__ __forceinline__ float rlane(float x, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), src));
}
__device__ __forceinline__ double rlane(double x, int src) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Raw buffer accesses: 32-bit byte offsets within one array (a descriptor
// per array, range-checked by the hardware against the array's extent).
// They replace the 64-bit address arithmetic of each access; the kernel
// uses them only for accesses that are in range by construction.
constexpr int64_t kBufMax = (int64_t)1 << 31;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void bstore(float x, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
}
__device__ __forceinline__ void bstore(double x, __amdgpu_buffer_rsrc_t r, int off) {
    using v2u = __attribute__((ext_vector_type(2))) unsigned;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, x), r, off, 0, 0);
}
// scalar-offset forms: byte offset voff (per lane) + soff (uniform)
__device__ __forceinline__ void bstore(float x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, voff, soff, 0);
}
__device__ __forceinline__ void bstore(double x, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    using v2u = __attribute__((ext_vector_type(2))) unsigned;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, x), r, voff, soff, 0);
}
// 16-byte vectors
using u32x4 = __attribute__((ext_vector_type(4))) unsigned;
template <typename VT>
__device__ __forceinline__ VT bload16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <typename VT>
__device__ __forceinline__ void bstore16(VT v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
}

constexpr double pow_na(int e) {   // (-alpha)^e
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= -kAlpha;
    return r;
}

template <typename T, int METHOD> struct Line3 {
    using C = K3<T>;
    static constexpr int R = C::R, LPL = C::LPL, TS = C::TS;
    int i, h, s0, n;
    bool first, last, lwin, rwin;
    // Lanes holding boundary rows.  The first window starts at slot 0 and the
    // last one ends on the last slot of the line, so those rows sit at fixed
    // positions: slots 0, 1 at positions 0, 1 of lane 0; slots n, n - 1 at the
    // end of lane LPL - 1 (positions R - 1, R - 2 in the compact layout, where
    // the last slot is n; R - 2, R - 3 in the mimetic one, one slot longer).
    // Any other window reaches a boundary row only with its outermost slot,
    // H slots from what it writes, like the truncation at its other edges.
    bool bl, br;

    // neighbour values within the line (0 beyond the window)
    __device__ __forceinline__ T prev(T x) const {
        const T y = wshr(x);
        return first ? T(0) : y;
    }
    __device__ __forceinline__ T next(T x) const {
        const T y = wshl(x);
        return last ? T(0) : y;
    }
    // value of lane-in-line `src` of this line
    __device__ __forceinline__ T from_lane(T x, int src) const {
        const T v0 = rlane(x, src), v1 = rlane(x, LPL + src);
        return h ? v1 : v0;
    }

    // ================= compact scheme =================
    // Scaled right-hand side of the derivative of kind `kind` (0: Q4 on
    // pressure, 1: Qbar4 on velocity) into o; closures of Appendix A on the
    // boundary rows, zero on the trivial rows added to Pbar.
    __device__ __forceinline__ void rhs(int kind, const T (&f)[R], T fl, T fr, T (&o)[R]) const {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const T fp = k + 1 < R ? f[k + 1] : fr;
            const T fm = k > 0 ? f[k - 1] : fl;
            o[k] = fp - fm;
        }
        if (!(lwin || rwin)) return;   // uniform: only the end windows hold boundary rows
        const T third = T(1.0 / 3.0);
        constexpr int E = R - 1;   // slot n
        if (kind == 0) {
            if (bl) o[0] = third * (T(-17) * f[0] + T(9) * f[1] + T(9) * f[2] - f[3]);
            if (br) o[E] = third * (f[E - 3] - T(9) * f[E - 2] - T(9) * f[E - 1] + T(17) * f[E]);
        } else {
            if (bl) {
                o[0] = T(0);
                o[1] = third * (-f[0] - T(9) * f[1] + T(9) * f[2] + f[3]);
            }
            if (br) {
                o[E] = T(0);
                o[E - 1] = third * (-f[E - 3] - T(9) * f[E - 2] + T(9) * f[E - 1] + f[E]);
            }
        }
    }

    // Tridiagonal solve of the right-hand side in o (in place), and the
    // solution's values on the neighbouring lanes' edge slots: xl at slot
    // s0 - 1, xr at slot s0 + R.
    __device__ __forceinline__ void solve(int kind, T (&o)[R], T& xl, T& xr) const {
        const T al = T(kAlpha);
#pragma unroll
        for (int k = 1; k < R; ++k) o[k] = fma(-al, o[k - 1], o[k]);
        const T yend = o[R - 1];
#pragma unroll
        for (int k = R - 2; k >= 0; --k) o[k] = fma(-al, o[k + 1], o[k]);
        constexpr Resp<R> rs{};
        const T G = T(rs.G);
        const T rawf = o[0], rawl = o[R - 1];
        // The shifted values below are used as they come off the lane shift
        // (at a line's first / last lane they belong to the other line of the
        // wave); the line-edge masks are applied once, to the results.
        const T y1 = prev(yend);
        T Y = y1, Ym = T(0);
        if (TS > 1) {
            Ym = prev(y1);                       // forward carry into the previous lane
            Y = fma(G, Ym, Y);
        }
        const T Yv = fma(G, Y, yend);            // forward carry into the next lane
        const T nf = wshl(rawf);
        T X = last ? T(0) : fma(T(rs.a[0]), Yv, nf);
        if (TS > 1) {
            const T Yv2 = fma(G, Yv, wshl(yend));
            const T nf2 = wshl(nf);
            X = i < LPL - 2 ? fma(T(rs.b[0]), fma(T(rs.a[0]), Yv2, nf2), X) : X;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) o[k] = fma(T(rs.a[k]), Y, fma(T(rs.b[k]), X, o[k]));
        const T pl = wshr(rawl);
        const T xl0 = TS > 1 ? fma(T(rs.a[R - 1]), Ym, pl) : pl;
        xl = first ? T(0) : fma(T(rs.b[R - 1]), o[0], xl0);
        xr = X;
        if (lwin || rwin) correct(kind, o, xl, xr);
    }

    // Boundary-row correction (Sherman-Morrison-Woodbury) in the windows
    // holding the first or last slot of the line.  The correction is
    // geometric with ratio -alpha away from the boundary row:
    // w(0) = W0, w(d) = W1 (-alpha)^(d-1).
    __device__ void correct(int kind, T (&o)[R], T& xl, T& xr) const {
        constexpr BndResp kb{};
        constexpr double de = 3.7320508075688772935;
        constexpr int NZ = BndResp::NZ;
        const T na = T(-kAlpha);
        if (lwin) {
            // computed by every lane, meaningful in lane 0 (slots 0, 1, 2)
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
            W0 = from_lane(W0, 0);
            W1 = from_lane(W1, 0);
            if (s0 - 1 < NZ) {
                // lane i holds slots i R .. i R + R - 1
                T w;
                if (i == 0) w = W0;
                else if (i == 1) w = W1 * T(pow_na(R - 1));
                else if (i == 2) w = W1 * T(pow_na(2 * R - 1));
                else w = W1 * T(pow_na(3 * R - 1));
                // correction at slot s0 - 1 (last slot of the previous lane)
                const T wl = W1 * (i == 1 ? T(pow_na(R - 2)) : (i == 2 ? T(pow_na(2 * R - 2)) : T(pow_na(3 * R - 2))));
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    o[k] -= w;
                    w = (i == 0 && k == 0) ? W1 : w * na;
                }
                if (i > 0) xl -= wl;
                xr -= w;
            }
        }
        if (rwin) {
            // slot n is the last slot of the window: lane LPL - 1, position R - 1
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
            V0 = from_lane(V0, LPL - 1);
            V1 = from_lane(V1, LPL - 1);
            const int j = LPL - 1 - i;            // lanes from the right end
            if (n - (s0 + R) < NZ) {
                // distance of the lane's last slot from slot n: j R
                T w;
                if (j == 0) w = V0;
                else if (j == 1) w = V1 * T(pow_na(R - 1));
                else if (j == 2) w = V1 * T(pow_na(2 * R - 1));
                else w = V1 * T(pow_na(3 * R - 1));
                // correction at slot s0 + R (first slot of the next lane)
                const T wr = V1 * (j == 1 ? T(pow_na(R - 2)) : (j == 2 ? T(pow_na(2 * R - 2)) : T(pow_na(3 * R - 2))));
#pragma unroll
                for (int k = R - 1; k >= 0; --k) {
                    o[k] -= w;
                    w = (j == 0 && k == R - 1) ? V1 : w * na;
                }
                xl -= w;
                if (j > 0) xr -= wr;
            }
        }
    }
};

// One workgroup's share of a pass: LW lines (line group tile % nlg) over
// window tile / nlg.
// EPS: the tolerance-tested form (LinePassArgs::eps_part).  It keeps the
// previous iterates by solving into a spare array, and stores the squared
// changes of the last two sweeps over the slots the window writes.
// FULL: the variant with the optional features (damping layers, wall data,
// distributed forcing); the plain variant has none of their code.
template <typename T, int METHOD, int MODE, bool EPS = false, bool COMP = false, bool FULL = false>
__device__ __forceinline__ void lp3_body(const LinePassArgs<T>& a, int tile, T* smem) {
    static_assert(!(EPS && COMP), "the tolerance-tested form runs without compensation");
    using C = K3<T>;
    constexpr int R = C::R, LPL = C::LPL, WS = C::WS, LW = C::LW;
    const int lg = tile % a.nlg, g = tile / a.nlg;
    const int n = a.n, ns = a.ns;
    const int uhi = METHOD == LINE_CFD ? n - 1 : n;
    // central slots written by window g (the end windows need no margin on
    // their physical side)
    const int c0 = g == 0 ? 0 : (WS - a.H) + (g - 1) * a.S;
    const int c1 = g == a.nwin - 1 ? ns : (WS - a.H) + g * a.S;
    const int w0 = max(0, min(c0 - a.H, ns - WS));

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    Line3<T, METHOD> L;
    L.i = lane % LPL;
    L.h = lane / LPL;
    L.n = n;
    L.s0 = w0 + L.i * R;
    L.first = L.i == 0;
    L.last = L.i == LPL - 1;
    L.lwin = w0 == 0;
    L.rwin = w0 + WS >= ns;
    L.bl = L.lwin && L.first;
    L.br = L.rwin && L.last;
    const int s0 = L.s0;
    // Line-major rows are indexed r = q + 1 (row 0: a line of zeros), so that
    // the LW rows of a workgroup map onto LW-aligned runs of the other
    // direction's slots in the transposed pressure store.
    const int ln = wave * C::LPW + L.h;          // row of this lane's line within the workgroup
    const int r = lg * LW + ln, q = r - 1;
    const bool qok = q >= 0 && q < a.nlines;

    // ---- loads.  Line-major arrays: element (row r, slot s) at r * ld + s,
    // boundary slots stored as zeros, rows padded to whole line groups and
    // to at least 3 slots past the last one.  Staged: the LW lines of the
    // workgroup are read in 16-byte chunks starting at the slot wa = w0 - sh
    // on the 16-byte grid (sh = w0 mod VEC; only the last window has sh > 0,
    // the margin H being even), chunk c of line l into tile row l at position
    // c VEC (one extra chunk per line when sh > 0); lane i then takes its R
    // slots from positions sh + i R. ----
    constexpr int VEC = 16 / (int)sizeof(T);
    using VT = T __attribute__((ext_vector_type(16 / sizeof(T))));
    const int sh = w0 % VEC, wa = w0 - sh;
    constexpr int CPL = WS / VEC;                 // chunks per line
    constexpr int CPT = CPL * LW / C::NT;         // chunks per thread
    constexpr int RPJ = C::NT / CPL;              // lines covered by one staging step
    static_assert(CPT * C::NT == CPL * LW && RPJ * CPL == C::NT, "chunking");
    static_assert(C::TP >= WS + VEC, "tile row holds the extra chunk");
    // Thread tid moves chunk tid % CPL of the lines tid / CPL + j RPJ, and the
    // extra chunk (tile position WS) of line tid when sh > 0 and tid < LW.
    // The line-major arrays of this direction span nlg LW rows of ld
    // elements; when that fits 31 bits they are accessed through buffer
    // descriptors: a 32-bit lane offset plus a uniform row step.
    const int64_t lm_rows = (int64_t)a.nlg * LW;
    const int st_l = tid / CPL, st_c = tid % CPL;
    const bool xtra = sh != 0 && tid < LW;
    using TM = TMap<T>;
    constexpr int NC = TM::NC;
    // tile position of the chunk after this lane's segment
    const int nxt = L.i + 1 < LPL ? TM::chunk(L.i + 1, 0) : WS;
    auto stage_in = [&](const T* base, int64_t ld, VT (&ch)[CPT], VT& ce) {
        const int64_t bytes = lm_rows * ld * (int64_t)sizeof(T);
        if (bytes < kBufMax) {
            const auto rs = make_rsrc(base, bytes);
            const int vo = (int)(((int64_t)(lg * LW + st_l) * ld + wa + st_c * VEC) * (int64_t)sizeof(T));
            const int so = (int)((int64_t)RPJ * ld * (int64_t)sizeof(T));
#pragma unroll
            for (int j = 0; j < CPT; ++j) ch[j] = bload16<VT>(rs, vo, j * so);
            if (xtra) ce = bload16<VT>(rs, (int)(((int64_t)(lg * LW + tid) * ld + wa + WS) * (int64_t)sizeof(T)), 0);
        } else {
#pragma unroll
            for (int j = 0; j < CPT; ++j)
                ch[j] = *reinterpret_cast<const VT*>(base + (int64_t)(lg * LW + st_l + j * RPJ) * ld + wa + st_c * VEC);
            if (xtra) ce = *reinterpret_cast<const VT*>(base + (int64_t)(lg * LW + tid) * ld + wa + WS);
        }
    };
    // f(std::integral_constant<int, sh>) for the block's shift
    auto with_shift = [&](auto&& f) {
        if constexpr (VEC == 4) {
            switch (sh) {
                case 0: f(std::integral_constant<int, 0>{}); break;
                case 1: f(std::integral_constant<int, 1>{}); break;
                case 2: f(std::integral_constant<int, 2>{}); break;
                default: f(std::integral_constant<int, 3>{}); break;
            }
        } else {
            if (sh == 0) f(std::integral_constant<int, 0>{});
            else f(std::integral_constant<int, 1>{});
        }
    };
    // this lane's R slots from its tile row (positions SH + i R ...)
    auto read_seg = [&](auto shc, T (&dst)[R]) {
        constexpr int SH = decltype(shc)::value;
        constexpr int NR = SH ? NC + 1 : NC;
        T el[NR * VEC];
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const VT v = *reinterpret_cast<const VT*>(smem + tix<T>(ln, c < NC ? TM::chunk(L.i, c) : nxt));
#pragma unroll
            for (int e = 0; e < VEC; ++e) el[c * VEC + e] = v[e];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) dst[k] = el[SH + k];
    };
    // this lane's R slots into its tile row; with a shift, the first and the
    // last chunk are shared with the neighbouring lanes and written element-wise
    auto write_seg = [&](auto shc, const T (&src)[R]) {
        constexpr int SH = decltype(shc)::value;
        T* row = smem + tix<T>(ln, 0);
        if constexpr (SH == 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                VT v;
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[e] = src[c * VEC + e];
                *reinterpret_cast<VT*>(row + TM::chunk(L.i, c)) = v;
            }
        } else {
#pragma unroll
            for (int e = SH; e < VEC; ++e) row[TM::chunk(L.i, 0) + e] = src[e - SH];
#pragma unroll
            for (int c = 1; c < NC; ++c) {
                VT v;
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[e] = src[c * VEC + e - SH];
                *reinterpret_cast<VT*>(row + TM::chunk(L.i, c)) = v;
            }
#pragma unroll
            for (int e = 0; e < SH; ++e) row[nxt + e] = src[R - SH + e];
        }
    };
    auto stage_spread = [&](const VT (&ch)[CPT], const VT& ce, T (&dst)[R]) {
        __syncthreads();   // earlier readers of the tile are done
#pragma unroll
        for (int j = 0; j < CPT; ++j)
            *reinterpret_cast<VT*>(smem + tix<T>(st_l + j * RPJ, TM::chunk(st_c / NC, st_c % NC))) = ch[j];
        if (xtra) *reinterpret_cast<VT*>(smem + tix<T>(tid, WS)) = ce;
        __syncthreads();
        with_shift([&](auto shc) { read_seg(shc, dst); });
    };
    T A[R], B[R], KK[R], RR[R], U[R], Tt[R];
    {
        VT ca[CPT], cb[CPT], ck[CPT], cr[CPT], ea{}, eb{}, ek{}, er{};
        stage_in(a.uin, a.uin_ld, ca, ea);
        stage_in(a.vin, a.vin_ld, cb, eb);
        if (a.ak) stage_in(a.ak, a.ak_ld, ck, ek);
        if (a.ar) stage_in(a.ar, a.ar_ld, cr, er);
        stage_spread(ca, ea, A);
        stage_spread(cb, eb, B);
        if (a.ak) stage_spread(ck, ek, KK);
        if (a.ar) stage_spread(cr, er, RR);
    }
    // Dirichlet wall values: the first slot of the line (lane 0 of the first
    // window, position 0) and its last (last lane of the last window,
    // position R - 1); the material arrays are zero there, so the sweeps keep
    // them
    if ((FULL || COMP) && a.bnd && qok) {
        if (L.bl) A[0] = a.bsc[0] * a.bnd[6 * q] + a.bsc[1] * a.bnd[6 * q + 1] + a.bsc[2] * a.bnd[6 * q + 2];
        if (L.br)
            A[R - 1] = a.bsc[0] * a.bnd[6 * q + 3] + a.bsc[1] * a.bnd[6 * q + 4] + a.bsc[2] * a.bnd[6 * q + 5];
    }
    // scale folded into the material values (compact: 3 alpha / h; mimetic: 9 / (8 h))
    const T sc = METHOD == LINE_CFD ? T(3.0 * kAlpha) * a.inv_h : T(9.0 / 8.0) * a.inv_h;
    // The material arrays hold zeros outside the interior of the lines (slot
    // 0 and slots past the last unknown, row 0 and the padding rows), so
    // only the constant values need the masks.
    if (a.ak) {
#pragma unroll
        for (int k = 0; k < R; ++k) KK[k] *= sc;
    } else {
        const T v = sc * a.ak0;
#pragma unroll
        for (int k = 0; k < R; ++k) KK[k] = qok && s0 + k >= 1 && s0 + k <= uhi ? v : T(0);
    }
    if (a.ar) {
#pragma unroll
        for (int k = 0; k < R; ++k) RR[k] *= sc;
    } else {
        const T v = sc * a.ar0;
#pragma unroll
        for (int k = 0; k < R; ++k) RR[k] = qok && s0 + k <= n ? v : T(0);
    }
    // Damping layers (the damped system: each implicit line system divides
    // by 1 + a d, each explicit part multiplies by 1 - a d).  The implicit
    // pressure rows are divided here (A and a kappa); the velocity rows after
    // the first half sweep, which still reads the undivided B.
    const bool damp = FULL && !COMP && a.dmpm != 0;   // uniform
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
    auto damp_vel = [&](T& x, T& r, int s) {
        const T e = T(1) / fma(a.ah, dvel(s), T(1));
        x *= e;
        r *= e;
    };

    // Tolerance test: squared changes of the last two sweeps over the slots
    // this window writes (pressure: interior slots; velocity: slots 0..n).
    // (accumulated in the kernel's precision per lane, reduced in FP64)
    T ev[4] = {T(0), T(0), T(0), T(0)};
    int umask = 0, vmask = 0;
    if constexpr (EPS) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int s = s0 + k;
            const bool own = qok && s >= c0 && s < c1;
            if (own && s >= 1 && s <= uhi) umask |= 1 << k;
            if (own && s <= n) vmask |= 1 << k;
        }
    }
    // (on is 0 or 1: a product rather than a select, which would hold one
    // lane mask per slot in the scalar registers)
    auto chg = [](T x, T y, int on) {
        const T d = (x - y) * T(on);
        return d * d;
    };
    // The masks pass through an empty asm at each use: the per-slot tests
    // are then not hoisted out of the sweep loop as 2 R lane masks, which
    // would not fit the scalar registers.
    auto opaque = [](int m) {
        asm volatile("" : "+v"(m));
        return m;
    };

    if (METHOD == LINE_CFD) {
        // neighbours' edge values of the inputs
        T Al = L.prev(A[R - 1]), Ar = L.next(A[0]);
        const T Kl = L.prev(KK[R - 1]), Kr = L.next(KK[0]);
        T Bl = L.prev(B[R - 1]), Br = L.next(B[0]);
        T Rl = L.prev(RR[R - 1]), Rr = L.next(RR[0]);
        T xl, xr;
        if (MODE == LINE_EXPLICIT) {
            L.rhs(0, A, Al, Ar, Tt);
            L.solve(0, Tt, xl, xr);
            L.rhs(1, B, Bl, Br, U);
            L.solve(1, U, xl, xr);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                // W* = B - aR G(A), A - aK D(B) (the increments when compensated;
                // B, A times 1 - a d with damping)
                const T bb = damp ? B[k] * fma(-a.ah, dvel(s0 + k), T(1)) : B[k];
                const T aa = damp ? A[k] * fma(-a.ah, dpres(s0 + k), T(1)) : A[k];
                Tt[k] = COMP ? -RR[k] * Tt[k] : fma(-RR[k], Tt[k], bb);
                U[k] = COMP ? -KK[k] * U[k] : fma(-KK[k], U[k], aa);
            }
        } else {
            T Ul, Ur;
            if constexpr (COMP) {
                // derivatives of the state, then the sweeps on the increments:
                // A' = -aK D(B) (= u_1 - A) and B' = -aR G(A) replace A and B
                L.rhs(0, A, Al, Ar, Tt);
                L.solve(0, Tt, xl, xr);
                const T gl = -Rl * xl, gr = -Rr * xr;
                L.rhs(1, B, Bl, Br, U);
                L.solve(1, U, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    A[k] = -KK[k] * U[k];
                    B[k] = -RR[k] * Tt[k];
                    U[k] = A[k];
                }
                Al = -Kl * xl;
                Ar = -Kr * xr;
                Bl = gl;
                Br = gr;
                Ul = Al;
                Ur = Ar;
            } else {
                // u_1 = A - aK D(B)
                L.rhs(1, B, Bl, Br, U);
                L.solve(1, U, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
                Ul = fma(-Kl, xl, Al);
                Ur = fma(-Kr, xr, Ar);
            }
            if (damp) {
#pragma unroll
                for (int k = 0; k < R; ++k) damp_vel(B[k], RR[k], s0 + k);
                damp_vel(Bl, Rl, s0 - 1);
                damp_vel(Br, Rr, s0 + R);
            }
            T Tl, Tr;
            if constexpr (EPS) {
                T X[R];
#pragma unroll
                for (int k = 0; k < R; ++k) Tt[k] = B[k];                     // v_0
                // one sweep (v_it, then u_{it+1}); tv: sum the change of v,
                // q >= 0: sum the change of u into ev[q] (constants at each call)
                auto sweep = [&](bool tv, int q) {
                    const int vm = opaque(vmask), um = opaque(umask);
                    L.rhs(0, U, Ul, Ur, X);
                    L.solve(0, X, xl, xr);
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const T vn = fma(-RR[k], X[k], B[k]);
                        if (tv) ev[1] += chg(vn, Tt[k], (vm >> k) & 1);
                        Tt[k] = vn;
                    }
                    Tl = fma(-Rl, xl, Bl);
                    Tr = fma(-Rr, xr, Br);
                    L.rhs(1, Tt, Tl, Tr, X);
                    L.solve(1, X, xl, xr);
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const T un = fma(-KK[k], X[k], A[k]);
                        if (q >= 0) ev[q] += chg(un, U[k], (um >> k) & 1);
                        U[k] = un;
                    }
                    Ul = fma(-Kl, xl, Al);
                    Ur = fma(-Kr, xr, Ar);
                };
                // sweeps it = 1 .. K - 1: untracked, then u_{K-1}, then v_{K-1} and u_K
                for (int it = 1; it < a.sweeps - 2; ++it) sweep(false, -1);
                if (a.sweeps >= 3) sweep(false, 0);
                sweep(true, 2);
                const int vm = opaque(vmask);
                L.rhs(0, U, Ul, Ur, X);
                L.solve(0, X, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) {                                  // v_K
                    const T vn = fma(-RR[k], X[k], B[k]);
                    ev[3] += chg(vn, Tt[k], (vm >> k) & 1);
                    Tt[k] = vn;
                }
            } else {
                for (int it = 1; it < a.sweeps; ++it) {
                    L.rhs(0, U, Ul, Ur, Tt);
                    L.solve(0, Tt, xl, xr);
#pragma unroll
                    for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);
                    Tl = fma(-Rl, xl, Bl);
                    Tr = fma(-Rr, xr, Br);
                    L.rhs(1, Tt, Tl, Tr, U);
                    L.solve(1, U, xl, xr);
#pragma unroll
                    for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
                    Ul = fma(-Kl, xl, Al);
                    Ur = fma(-Kr, xr, Ar);
                }
                L.rhs(0, U, Ul, Ur, Tt);
                L.solve(0, Tt, xl, xr);
#pragma unroll
                for (int k = 0; k < R; ++k) Tt[k] = fma(-RR[k], Tt[k], B[k]);   // v_K
            }
            if (MODE == LINE_SWEEP) {
                Tl = fma(-Rl, xl, Bl);
                Tr = fma(-Rr, xr, Br);
                if constexpr (COMP) {
#pragma unroll
                    for (int k = 0; k < R; ++k) U[k] += A[k];                   // u_K - A + A'
                }
                L.rhs(1, Tt, Tl, Tr, A);
                L.solve(1, A, xl, xr);
                if (damp) {
                    // 2 v_K - B and u_K (1 - a d) - aK D(v_K), with B and aK
                    // restored from their divided forms
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
                        Tt[k] = COMP ? vk + vk : vk + (vk - B[k]);              // 2 v_K - B
                        U[k] = fma(-KK[k], A[k], U[k]);                         // u_K - aK D(v_K)
                    }
                }
            }
        }
    } else {
        // ---- mimetic ----
        T Bm2 = L.prev(B[R - 2]), Bm1 = L.prev(B[R - 1]), Bp = L.next(B[0]);
        T Rm2 = L.prev(RR[R - 2]), Rm1 = L.prev(RR[R - 1]), Rp = L.next(RR[0]);
        const T ih8 = T(8.0 / 9.0);   // boundary rows are divided by the folded 9/8
        const T d0c[6] = {T(-4751.0 / 5192.0), T(909.0 / 1298.0), T(6091.0 / 15576.0),
                          T(-1165.0 / 5192.0), T(129.0 / 2596.0), T(-25.0 / 15576.0)};
        const T g0c[6] = {T(-47888.0 / 14245.0), T(1790.0 / 407.0), T(-14545.0 / 9768.0),
                          T(8997.0 / 16280.0), T(-2335.0 / 22792.0), T(25.0 / 9768.0)};
        const T g1c[5] = {T(16.0 / 105.0), T(-31.0 / 24.0), T(29.0 / 24.0), T(-3.0 / 40.0),
                          T(1.0 / 168.0)};
        const bool bl = L.bl, br = L.br;
        constexpr int E = R - 2;   // slot n (the mimetic line has one more slot, n + 1)
        // D'(v) on own slots; v given on positions -2..R
        auto applyD = [&](const T (&v)[R], T vm2, T vm1, T vp, T (&o)[R]) {
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T a2 = k >= 2 ? v[k - 2] : (k == 1 ? vm1 : vm2);
                const T a1 = k >= 1 ? v[k - 1] : vm1;
                const T a3 = k + 1 < R ? v[k + 1] : vp;
                o[k] = md(a2, a1, v[k], a3);
            }
            if (!(L.lwin || L.rwin)) return;   // uniform: only the end windows hold boundary rows
            if (bl) {   // slot 1
                T acc = T(0);
#pragma unroll
                for (int c = 0; c < 6; ++c) acc = fma(d0c[c], v[c], acc);
                o[1] = acc * ih8;
            }
            if (br) {   // slot n
                T acc = T(0);
#pragma unroll
                for (int c = 0; c < 6; ++c) acc = fma(d0c[c], v[E - c], acc);
                o[E] = -acc * ih8;
            }
        };
        // G'(u) on own slots, u given on positions -3..R+2
        auto applyG = [&](const T (&u)[R], const T (&ul)[3], const T (&ur)[3], T (&o)[R]) {
            auto U_ = [&](int p) -> T { return p < 0 ? ul[3 + p] : (p < R ? u[p] : ur[p - R]); };
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = mg(U_(k - 1), U_(k), U_(k + 1), U_(k + 2));
            if (!(L.lwin || L.rwin)) return;   // uniform: only the end windows hold boundary rows
            if (bl) {   // slots 0, 1
                T acc0 = T(0), acc1 = T(0);
#pragma unroll
                for (int c = 0; c < 6; ++c) acc0 = fma(g0c[c], u[c], acc0);
#pragma unroll
                for (int c = 0; c < 5; ++c) acc1 = fma(g1c[c], u[c], acc1);
                o[0] = acc0 * ih8;
                o[1] = acc1 * ih8;
            }
            if (br) {   // slots n - 1, n
                T acc0 = T(0), acc1 = T(0);
#pragma unroll
                for (int c = 0; c < 6; ++c) acc0 = fma(g0c[c], u[E + 1 - c], acc0);
#pragma unroll
                for (int c = 0; c < 5; ++c) acc1 = fma(g1c[c], u[E + 1 - c], acc1);
                o[E] = -acc0 * ih8;
                o[E - 1] = -acc1 * ih8;
            }
        };
        auto halo_u = [&](const T (&u)[R], T (&ul)[3], T (&ur)[3]) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                ul[j] = L.prev(u[R - 3 + j]);
                ur[j] = L.next(u[j]);
            }
        };
        // velocity on own slots and on -2, -1, R
        auto velocity = [&](const T (&u)[R], T (&o)[R], T& om2, T& om1, T& op) {
            T ul[3], ur[3];
            halo_u(u, ul, ur);
            applyG(u, ul, ur, o);
#pragma unroll
            for (int k = 0; k < R; ++k) o[k] = fma(-RR[k], o[k], B[k]);
            om2 = fma(-Rm2, mg(ul[0], ul[1], ul[2], u[0]), Bm2);
            om1 = fma(-Rm1, mg(ul[1], ul[2], u[0], u[1]), Bm1);
            op = fma(-Rp, mg(u[R - 1], ur[0], ur[1], ur[2]), Bp);
        };
        if (MODE == LINE_EXPLICIT) {
            T ul[3], ur[3];
            halo_u(A, ul, ur);
            applyG(A, ul, ur, Tt);
            applyD(B, Bm2, Bm1, Bp, U);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const T bb = damp ? B[k] * fma(-a.ah, dvel(s0 + k), T(1)) : B[k];
                const T aa = damp ? A[k] * fma(-a.ah, dpres(s0 + k), T(1)) : A[k];
                Tt[k] = COMP ? -RR[k] * Tt[k] : fma(-RR[k], Tt[k], bb);
                U[k] = COMP ? -KK[k] * U[k] : fma(-KK[k], U[k], aa);
            }
        } else {
            T Tm2, Tm1, Tp;
            if constexpr (COMP) {
                // derivatives of the state, then the sweeps on the increments
                // (A' = -aK D(B), B' = -aR G(A), halos included)
                T ul[3], ur[3];
                halo_u(A, ul, ur);
                applyG(A, ul, ur, Tt);
                applyD(B, Bm2, Bm1, Bp, U);
                const T gm2 = -Rm2 * mg(ul[0], ul[1], ul[2], A[0]);
                const T gm1 = -Rm1 * mg(ul[1], ul[2], A[0], A[1]);
                const T gp = -Rp * mg(A[R - 1], ur[0], ur[1], ur[2]);
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    A[k] = -KK[k] * U[k];
                    B[k] = -RR[k] * Tt[k];
                    U[k] = A[k];
                }
                Bm2 = gm2;
                Bm1 = gm1;
                Bp = gp;
            } else {
                applyD(B, Bm2, Bm1, Bp, U);
#pragma unroll
                for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
            }
            if (damp) {
#pragma unroll
                for (int k = 0; k < R; ++k) damp_vel(B[k], RR[k], s0 + k);
                damp_vel(Bm2, Rm2, s0 - 2);
                damp_vel(Bm1, Rm1, s0 - 1);
                damp_vel(Bp, Rp, s0 + R);
            }
            if constexpr (EPS) {
                T X[R];
#pragma unroll
                for (int k = 0; k < R; ++k) Tt[k] = B[k];                     // v_0
                // one sweep (v_it, then u_{it+1}); tracking as in the compact form
                auto sweep = [&](bool tv, int q) {
                    const int vm = opaque(vmask), um = opaque(umask);
                    velocity(U, X, Tm2, Tm1, Tp);
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        if (tv) ev[1] += chg(X[k], Tt[k], (vm >> k) & 1);
                        Tt[k] = X[k];
                    }
                    applyD(Tt, Tm2, Tm1, Tp, X);
#pragma unroll
                    for (int k = 0; k < R; ++k) {
                        const T un = fma(-KK[k], X[k], A[k]);
                        if (q >= 0) ev[q] += chg(un, U[k], (um >> k) & 1);
                        U[k] = un;
                    }
                };
                for (int it = 1; it < a.sweeps - 2; ++it) sweep(false, -1);
                if (a.sweeps >= 3) sweep(false, 0);
                sweep(true, 2);
                const int vm = opaque(vmask);
                velocity(U, X, Tm2, Tm1, Tp);                                 // v_K
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    ev[3] += chg(X[k], Tt[k], (vm >> k) & 1);
                    Tt[k] = X[k];
                }
            } else {
                for (int it = 1; it < a.sweeps; ++it) {
                    velocity(U, Tt, Tm2, Tm1, Tp);
                    applyD(Tt, Tm2, Tm1, Tp, U);
#pragma unroll
                    for (int k = 0; k < R; ++k) U[k] = fma(-KK[k], U[k], A[k]);
                }
                velocity(U, Tt, Tm2, Tm1, Tp);                               // v_K
            }
            if (MODE == LINE_SWEEP) {
                if constexpr (COMP) {
#pragma unroll
                    for (int k = 0; k < R; ++k) U[k] += A[k];
                }
                applyD(Tt, Tm2, Tm1, Tp, A);
                if (damp) {
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
                        Tt[k] = COMP ? vk + vk : vk + (vk - B[k]);
                        U[k] = fma(-KK[k], A[k], U[k]);
                    }
                }
            }
        }
    }

    if constexpr (EPS) {
        // wave sums, then the workgroup's, stored as this tile's partials
        __shared__ double wsum[C::NWV][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double v = (double)ev[q];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) wsum[wave][q] = v;
        }
        __syncthreads();
        if (tid < 4) {
            double v = 0.0;
            for (int w = 0; w < C::NWV; ++w) v += wsum[w][tid];
            a.eps_part[(int64_t)tid * a.nlg * a.nwin + tile] = v;
        }
    }

    // ---- stores through the LDS tile: velocity, then pressure ----
    if (MODE != LINE_FINAL) {
        const int ks = a.src_s - s0;
        if (q == a.src_q && ks >= 0 && ks < R) {   // one lane of the grid
#pragma unroll
            for (int k = 0; k < R; ++k)
                if (k == ks) U[k] += a.aF;
        }
        if ((FULL || COMP) && a.ff) {
            // distributed forcing (zero outside the interior, like the
            // materials); KK is free after the last derivative
            VT cf[CPT], ef{};
            stage_in(a.ff, a.ff_ld, cf, ef);
            stage_spread(cf, ef, KK);
#pragma unroll
            for (int k = 0; k < R; ++k) U[k] = fma(a.aFf, KK[k], U[k]);
        }
    }
    // velocity into the line-major output (central slots only)
    auto store_vel = [&](const T (&vals)[R], T* out) {
        __syncthreads();   // readers of the tile are done
        with_shift([&](auto shc) { write_seg(shc, vals); });
        __syncthreads();
        const int64_t bytes = lm_rows * a.vout_ld * (int64_t)sizeof(T);
        const bool buf = bytes < kBufMax;
        const auto rs = make_rsrc(out, buf ? bytes : 0);
        // chunk at tile position pos (slots s .. s + VEC - 1) of tile row l
        auto put = [&](int l, int pos, int s) {
            const int rr = lg * LW + l;
            if (rr < 1 || rr > a.nlines || s + VEC <= c0 || s >= c1) return;
            const VT v = *reinterpret_cast<const VT*>(smem + tix<T>(l, pos));
            const int64_t off = (int64_t)rr * a.vout_ld + s;
            if (s >= c0 && s + VEC <= c1 && s + VEC - 1 <= n) {
                if (buf) bstore16(v, rs, (int)(off * (int64_t)sizeof(T)), 0);
                else *reinterpret_cast<VT*>(out + off) = v;
            } else {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    if (s + e >= c0 && s + e < c1 && s + e <= n) {
                        if (buf) bstore(v[e], rs, (int)((off + e) * (int64_t)sizeof(T)));
                        else out[off + e] = v[e];
                    }
            }
        };
#pragma unroll
        for (int j = 0; j < CPT; ++j) put(st_l + j * RPJ, TM::chunk(st_c / NC, st_c % NC), wa + st_c * VEC);
        if (xtra) put(tid, WS, wa + WS);
    };
    // pressure hand-off for the other direction, transposed through LDS
    auto store_pres = [&](const T (&vals)[R], T* uout) {
    __syncthreads();   // readers of the tile are done
    with_shift([&](auto shc) { write_seg(shc, vals); });
    __syncthreads();
    const int lo = max(c0, 1), hi = min(c1 - 1, uhi);
    // tile position of window position p (slot wa + p)
    auto tpos = [&](int p) { return p < WS ? TM::slot(p) : p; };
    if (a.utrans) {
        // uout[q * ld + (s - 1)]: TPL consecutive threads along the slots of a line
        constexpr int TPL = C::TPL;
        const int l2 = tid / TPL, t2 = tid % TPL;
        const int qq = lg * LW + l2 - 1;
        const int64_t bytes = (int64_t)a.nlines * a.uout_ld * (int64_t)sizeof(T);
        if (qq >= 0 && qq < a.nlines && bytes < kBufMax) {
            const auto rs = make_rsrc(uout, bytes);
            int o = (qq * (int)a.uout_ld + lo + t2 - 1) * (int)sizeof(T);
            for (int s = lo + t2; s <= hi; s += TPL, o += TPL * (int)sizeof(T)) bstore(smem[tix<T>(l2, tpos(s - wa))], rs, o);
        } else if (qq >= 0 && qq < a.nlines) {
            T* p = uout + (int64_t)qq * a.uout_ld - 1;
            for (int s = lo + t2; s <= hi; s += TPL) p[s] = smem[tix<T>(l2, tpos(s - wa))];
        }
    } else {
        // uout[(s - 1) * ld + q + 1] (the caller passes the base one element
        // lower).  Thread -> line pl, chunk columns pc + j PCJ: a chunk's VEC
        // slots go to VEC rows of the target, the LW lines of the workgroup
        // forming runs of LW consecutive elements that start on multiples of LW.
        constexpr int PCJ = C::NT / LW;            // chunk columns per step
        constexpr int PJ = CPL / PCJ;              // steps
        static_assert(PJ * PCJ == CPL, "pressure chunking");
        const int pl = tid % LW, pc = tid / LW;
        const int rr = lg * LW + pl;               // q + 1
        if (rr >= 1 && rr <= a.nlines) {
            // elements the pass writes from uout: up to (uhi - 1) ld + nlines
            const int64_t lim = ((int64_t)(uhi - 1) * a.uout_ld + a.nlines + 1) * (int64_t)sizeof(T);
            const bool buf = lim < kBufMax;
            const auto rs = make_rsrc(uout, buf ? lim : 0);
            const int ldb = buf ? (int)(a.uout_ld * (int64_t)sizeof(T)) : 0;
            const int rb = rr * (int)sizeof(T);
            // chunk at tile position pos of row pl: slots s .. s + VEC - 1
            auto put = [&](int pos, int s) {
                if (s + VEC - 1 < lo || s > hi) return;
                const VT v = *reinterpret_cast<const VT*>(smem + tix<T>(pl, pos));
                if (buf && s >= lo && s + VEC - 1 <= hi) {
                    const int o = (s - 1) * ldb + rb;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) bstore(v[e], rs, o, e * ldb);
                } else if (buf) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (s + e >= lo && s + e <= hi) bstore(v[e], rs, (s + e - 1) * ldb + rb, 0);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (s + e >= lo && s + e <= hi) uout[(int64_t)(s + e - 1) * a.uout_ld + rr] = v[e];
                }
            };
#pragma unroll
            for (int j = 0; j < PJ; ++j) {
                const int sc = pc + j * PCJ;
                put(TM::chunk(sc / NC, sc % NC), wa + sc * VEC);
            }
            if (sh != 0 && pc == 0) put(WS, wa + WS);
        }
    }
    };
    if constexpr (COMP) {
        // the pairs (value, low word) of the inputs plus the increments;
        // A, B, KK, RR are free now
        auto restage = [&](const T* hi, const T* lo, int64_t ld, T (&dh)[R], T (&dl)[R]) {
            VT ch[CPT], ce{};
            stage_in(hi, ld, ch, ce);
            stage_spread(ch, ce, dh);
            if (lo) {
                stage_in(lo, ld, ch, ce);
                stage_spread(ch, ce, dl);
            } else {
#pragma unroll
                for (int k = 0; k < R; ++k) dl[k] = T(0);
            }
        };
        restage(a.vin, a.vin_lo, a.vin_ld, A, B);
#pragma unroll
        for (int k = 0; k < R; ++k) acc_two_sum(A[k], B[k], Tt[k], Tt[k], A[k]);
        store_vel(Tt, a.vout);
        if (a.vout_lo) store_vel(A, a.vout_lo);
        restage(a.uin, a.uin_lo, a.uin_ld, B, KK);
#pragma unroll
        for (int k = 0; k < R; ++k) acc_two_sum(B[k], KK[k], U[k], U[k], B[k]);
        store_pres(U, a.uout);
        if (a.uout_lo) store_pres(B, a.uout_lo);
    } else {
        store_vel(Tt, a.vout);
        store_pres(U, a.uout);
    }
}

// Default tile order across the XCDs (LinePassArgs::torder), the fastest as
// measured: line group by line group, except for mimetic FP64 (window by
// window); FP32 passes over more than 6144 lines take windows in blocks of
// 32 line groups (8192^2: 385 against 461 us per pass).
int line3_torder(int dtype, int method, int nlines) {
    if (dtype != 1 && nlines > 6144) return 6;
    return method == LINE_CFD || dtype != 1 ? 0 : 1;
}

// The tolerance-tested form holds a spare array and the change sums: it
// runs at a lower occupancy (3 waves per SIMD in FP32, 1 in FP64) rather
// than spill.
template <typename T, bool EPS>
constexpr int kWpe = EPS ? (sizeof(T) == 4 ? 3 : 1) : Cfg3<T>::WPE;

template <typename T, int METHOD, int MODE, bool EPS = false, bool COMP = false, bool FULL = false>
__global__ void __launch_bounds__(K3<T>::NT)
__attribute__((amdgpu_waves_per_eu(kWpe<T, EPS>, kWpe<T, EPS>)))
line_pass3_kernel(const LinePassArgs<T> a) {
    __shared__ __align__(16) T smem[K3<T>::TILE];
    // Workgroups go round-robin to the eight XCDs; but with torder 2 each
    // XCD takes a contiguous range of the ordered tiles: line group by line
    // group (all windows of a group in turn, torder 0), window by window
    // (torder 1), or window by window within blocks of 2^(torder - 1) line
    // groups (torder 3 .. 6: the transposed pressure rows of a window then
    // fill in runs of that many groups); torder 2 keeps the launch order
    // (torder: a default per variant, or the autotuner's choice).
    const int nb = a.nlg * a.nwin;
    const int per = (nb + 7) / 8;
    auto order = [&](int b) { return a.torder == 2 ? b : (b % 8) * per + b / 8; };
    auto tile_of = [&](int t) {
        if (a.torder == 0) return (t % a.nwin) * a.nlg + t / a.nwin;
        if (a.torder <= 2) return t;
        const int gb = 1 << (a.torder - 1);
        const int sb = t / (gb * a.nwin), r = t - sb * gb * a.nwin;
        const int base = sb * gb, cnt = min(gb, a.nlg - base);
        return (r / cnt) * a.nlg + base + r % cnt;
    };
    // uniform: an earlier attempt of a tolerance-tested pass converged
    if (EPS && *a.eps_go == 0) return;
    const int t = order((int)blockIdx.x);
    if (t >= nb) return;
    lp3_body<T, METHOD, MODE, EPS, COMP, FULL>(a, tile_of(t), smem);
}

template <typename T, int METHOD, int MODE, bool COMP = false, bool FULL = false>
__global__ void __launch_bounds__(K3<T>::NT)
__attribute__((amdgpu_waves_per_eu(Cfg3<T>::WPE, Cfg3<T>::WPE)))
line_pass3_group_kernel(const GroupArgs<T> ga) {
    __shared__ __align__(16) T smem[K3<T>::TILE];
    int tile;
    const int it = group_item(ga, tile);
    if (it < 0) return;
    LinePassArgs<T> a = ga.items[it];
    if (a.aFtab) a.aF = a.aFtab[*ga.tick];
    lp3_body<T, METHOD, MODE, false, COMP, FULL>(a, tile, smem);
}

// compensated launches exist for FP32 only
template <typename T, int M, int MD>
hipError_t launch3_comp(const LinePassArgs<T>* a, const GroupArgs<T>* ga, dim3 grid, dim3 block, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
        if (a)
            hipLaunchKernelGGL((line_pass3_kernel<T, M, MD, false, true>), grid, block, 0, st, *a);
        else
            hipLaunchKernelGGL((line_pass3_group_kernel<T, M, MD, true>), grid, block, 0, st, *ga);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch3(const LinePassArgs<T>* a, const GroupArgs<T>* ga, int method, int mode, hipStream_t st,
                   bool comp, bool full) {
    const int nb = a ? a->nlg * a->nwin : ga->total;
    if (nb <= 0) return hipSuccess;
    const bool eps = a && a->eps_part;
    dim3 grid((unsigned)(((nb + 7) / 8) * 8)), block(K3<T>::NT);
    if (eps && (mode == LINE_EXPLICIT || comp || full)) return hipErrorInvalidValue;
    if (comp && full) return hipErrorInvalidValue;
#define LP3_CASE(M, MD)                                                                                  \
    if (method == M && mode == MD) {                                                                     \
        if (comp) return launch3_comp<T, M, MD>(a, ga, grid, block, st);                                  \
        if (full) {                                                                                      \
            if (a)                                                                                       \
                hipLaunchKernelGGL((line_pass3_kernel<T, M, MD, false, false, true>), grid, block, 0, st, *a); \
            else                                                                                         \
                hipLaunchKernelGGL((line_pass3_group_kernel<T, M, MD, false, true>), grid, block, 0, st, *ga); \
            return hipGetLastError();                                                                    \
        }                                                                                                \
        if (eps)                                                                                         \
            hipLaunchKernelGGL((line_pass3_kernel<T, M, MD, MD != LINE_EXPLICIT>), grid, block, 0, st, *a); \
        else if (a)                                                                                      \
            hipLaunchKernelGGL((line_pass3_kernel<T, M, MD>), grid, block, 0, st, *a);                  \
        else                                                                                             \
            hipLaunchKernelGGL((line_pass3_group_kernel<T, M, MD>), grid, block, 0, st, *ga);           \
        return hipGetLastError();                                                                        \
    }
    LP3_CASE(LINE_CFD, LINE_SWEEP)
    LP3_CASE(LINE_CFD, LINE_FINAL)
    LP3_CASE(LINE_CFD, LINE_EXPLICIT)
    LP3_CASE(LINE_MFD, LINE_SWEEP)
    LP3_CASE(LINE_MFD, LINE_FINAL)
    LP3_CASE(LINE_MFD, LINE_EXPLICIT)
#undef LP3_CASE
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_line_pass3(const LinePassArgs<T>& a, int method, int mode, hipStream_t st, bool comp, bool full) {
    return launch3<T>(&a, nullptr, method, mode, st, comp, full);
}

template <typename T>
hipError_t launch_line_group3(const GroupArgs<T>& ga, int method, int mode, hipStream_t st, bool comp, bool full) {
    return launch3<T>(nullptr, &ga, method, mode, st, comp, full);
}

int line3_lanes(int dtype) { return dtype == 1 ? K3<double>::LW : K3<float>::LW; }

// ---- tolerance-tested stages: control kernels ----

// after attempt j with K sweeps: the stage has converged if the change of
// sweep K - 1 (tested only from kmin on) or of sweep K is at most eps; the
// next attempt (K + 2 sweeps) runs only if this one ran and did not converge
// and K < kmax.  A deciding attempt adds one pass and its K sweeps to stats.
// The last attempt (K = kmax) always decides: its check is not launched
// when an earlier one exists, which counts it when it enables it.  go[0]
// stays 1; every other flag is written by the check before its attempt.
// One workgroup of 1024 threads; each thread sums its share of the four
// partial arrays with two loads per array in flight.
__global__ void __launch_bounds__(1024)
eps_check_kernel(const double* part, int nb, int* go, int j, int attempts, double eps, int K, int kmin, int kmax,
                 long long* stats) {
    constexpr int NT = 1024;
    __shared__ double red[4][NT];
    const int t = threadIdx.x;
    const bool ran = go[j] != 0;   // uniform
    if (ran) {
        double v[4][2] = {};
        int i = t;
        for (; i + NT < nb; i += 2 * NT)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q][0] += part[(int64_t)q * nb + i];
                v[q][1] += part[(int64_t)q * nb + i + NT];
            }
        if (i < nb)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q][0] += part[(int64_t)q * nb + i];
#pragma unroll
        for (int q = 0; q < 4; ++q) red[q][t] = v[q][0] + v[q][1];
        for (int w = NT / 2; w > 0; w >>= 1) {
            __syncthreads();
            if (t < w)
#pragma unroll
                for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + w];
        }
        __syncthreads();
    }
    if (t != 0) return;
    bool next = false;
    if (ran) {
        const bool t1 = K - 1 >= kmin && sqrt(red[0][0]) + sqrt(red[1][0]) <= eps;
        const bool t2 = sqrt(red[2][0]) + sqrt(red[3][0]) <= eps;
        const bool stop = t1 || t2 || K >= kmax;
        next = !stop;
        if (stop) {
            stats[0] += 1;
            stats[1] += K;
        } else if (j + 1 == attempts - 1) {
            stats[0] += 1;        // the last attempt runs and decides
            stats[1] += K + 2;
        }
    }
    go[j + 1] = next ? 1 : 0;
}

hipError_t launch_eps_check(const double* part, int nb, int* go, int j, int attempts, double eps, int K,
                            int kmin, int kmax, long long* stats, hipStream_t st) {
    hipLaunchKernelGGL(eps_check_kernel, dim3(1), dim3(1024), 0, st, part, nb, go, j, attempts, eps, K, kmin, kmax,
                       stats);
    return hipGetLastError();
}

template hipError_t launch_line_pass3<float>(const LinePassArgs<float>&, int, int, hipStream_t, bool, bool);
template hipError_t launch_line_pass3<double>(const LinePassArgs<double>&, int, int, hipStream_t, bool, bool);
template hipError_t launch_line_group3<float>(const GroupArgs<float>&, int, int, hipStream_t, bool, bool);
template hipError_t launch_line_group3<double>(const GroupArgs<double>&, int, int, hipStream_t, bool, bool);

}  // namespace adi
