// Exact line solves of one Peaceman-Rachford stage over a window of a line
// (the limit of infinitely many fixed-point sweeps).  Host- and
// device-callable: the GPU kernel runs it per (line, window) thread; the host
// runs it on a constant-coefficient line to size the window margins.
//
// Along a line with n cells, slot s holds the pressure value of index s and
// the velocity value of node s.  With ak = a kappa, ar = a / rho and the
// stage right-hand sides A (pressure, interior slots) and B (velocity, all
// nodes), a stage solves, per line,
//     Ubar + ak .* Dbar(vel) = A,      vel + ar .* G([0, Ubar, 0]) = B
// (Section 2.1, eqs. ecua2:PR / ecua3:PR2 with homogeneous Dirichlet
// pressure).  Both methods are rewritten as banded systems:
//   MFD (Appendix B): eliminating vel gives
//       (I - ak .* D4 (ar .* G4)) Ubar = A - ak .* D4 B,
//     one unknown per cell 1..n, bandwidths (6, 6) at the closure rows and
//     (3, 3) inside;
//   CFD (Appendix A): with z = Pbar^-1 Qbar vel and y = P^-1 Q U the pair
//       Pbar z + Qbar (ar .* y) = Qbar B,   P y + Q (ak .* z) = Q A
//     is banded; unknowns z_s, y_s interleaved per slot (z_0 = z_n = 0 as
//     trivial rows), bandwidths (7, 5).  Then Ubar = A - ak z, vel = B - ar y.
// A window solves the rows of its slot range [w0, w1] with the unknowns
// outside it dropped, by LU without pivoting in the Doolittle row order, and
// keeps only the slots at least H from a cut.  The inverse of these banded
// matrices decays geometrically away from the diagonal, so a margin H sized
// from that decay makes the kept values those of the whole-line solve to
// rounding.
#pragma once
#include <stdint.h>
#include <algorithm>
#include <cmath>
#include <vector>
#ifndef DIRECT_HD
#include <hip/hip_runtime.h>
#define DIRECT_HD __host__ __device__ __forceinline__
#else
#include <cmath>   // host-only build of this header (a host check)
#endif

namespace adi {
namespace direct {
#ifdef DIRECT_HOST_ONLY
using std::fma;
#endif

enum { MFD = 1, CFD = 0 };
enum { OUT_NEXT = 0, OUT_STAGE = 1 };   // fused next explicit part / the stage result

// Appendix B closure rows (first rows; the last rows are their centro-skew
// images) and the interior stencil, without the 1/h factor.
constexpr double D0[6] = {-4751.0 / 5192.0, 909.0 / 1298.0, 6091.0 / 15576.0,
                          -1165.0 / 5192.0, 129.0 / 2596.0, -25.0 / 15576.0};
constexpr double G0[6] = {-47888.0 / 14245.0, 1790.0 / 407.0, -14545.0 / 9768.0,
                          8997.0 / 16280.0, -2335.0 / 22792.0, 25.0 / 9768.0};
constexpr double G1[5] = {16.0 / 105.0, -31.0 / 24.0, 29.0 / 24.0, -3.0 / 40.0, 1.0 / 168.0};
constexpr double ST[4] = {1.0 / 24.0, -9.0 / 8.0, 9.0 / 8.0, -1.0 / 24.0};
// Appendix A closure rows without 1/h: h Q row 0 on nodes 0..3 (row n is
// its negated mirror) and h Qbar at node 1 on nodes 0..3 (node n-1 alike).
constexpr double Q0[4] = {-17.0, 9.0, 9.0, -1.0};
constexpr double QB1[4] = {-1.0, -9.0, 9.0, 1.0};

// Bandwidths of the window systems: with the closure rows of the line ends
// (WIDE) and of interior rows only, (3, 3) for both methods.
template <int METHOD> struct Band;
template <> struct Band<MFD> { static constexpr int ML = 6, MU = 6, RPS = 1; };
template <> struct Band<CFD> { static constexpr int ML = 7, MU = 5, RPS = 2; };
template <int METHOD, bool WIDE> struct BandOf {
    static constexpr int ML = WIDE ? Band<METHOD>::ML : 3, MU = WIDE ? Band<METHOD>::MU : 3;
};

// D4 entry (cell c = 1..n, face f = 0..n), without 1/h.
DIRECT_HD double dco(int n, int c, int f) {
    if (c == 1) return (f >= 0 && f <= 5) ? D0[f] : 0.0;
    if (c == n) { const int k = n - f; return (k >= 0 && k <= 5) ? -D0[k] : 0.0; }
    const int k = f - (c - 2);
    return (k >= 0 && k <= 3) ? ST[k] : 0.0;
}
// G4 entry (face f = 0..n, cell / boundary index c = 0..n+1), without 1/h.
DIRECT_HD double gco(int n, int f, int c) {
    if (f == 0) return (c >= 0 && c <= 5) ? G0[c] : 0.0;
    if (f == 1) return (c >= 0 && c <= 4) ? G1[c] : 0.0;
    if (f == n) { const int k = n + 1 - c; return (k >= 0 && k <= 5) ? -G0[k] : 0.0; }
    if (f == n - 1) { const int k = n + 1 - c; return (k >= 0 && k <= 4) ? -G1[k] : 0.0; }
    const int k = c - (f - 1);
    return (k >= 0 && k <= 3) ? ST[k] : 0.0;
}

// Window bounds in slots: output slots [o0, o1], solved slots [w0, w1].
// Windows of S output slots; with Se > 0 (and a line longer than 2 Se) the
// first and the last window keep only Se slots, so the windows that reach
// the closure rows are short.
struct Win {
    int o0, o1, w0, w1;
};
DIRECT_HD Win window(int smin, int smax, int S, int Se, int H, int w) {
    Win r;
    const int ns = smax - smin + 1;
    if (Se <= 0 || ns <= 2 * Se) {
        r.o0 = smin + w * S;
        r.o1 = r.o0 + S - 1 < smax ? r.o0 + S - 1 : smax;
    } else {
        const int m = (ns - 2 * Se + S - 1) / S;   // windows between the end windows
        if (w == 0) {
            r.o0 = smin;
            r.o1 = smin + Se - 1;
        } else if (w <= m) {
            r.o0 = smin + Se + (w - 1) * S;
            r.o1 = r.o0 + S - 1 < smax - Se ? r.o0 + S - 1 : smax - Se;
        } else {
            r.o0 = smax - Se + 1;
            r.o1 = smax;
        }
    }
    r.w0 = r.o0 - H > smin ? r.o0 - H : smin;
    r.w1 = r.o1 + H < smax ? r.o1 + H : smax;
    return r;
}
// First unknown row whose factor the back substitution reads: the MFD
// velocity of face f is formed at the step of its lowest cell, at most 4
// below the face (the last closure row).
DIRECT_HD int first_kept_row(int method, const Win& w) {
    if (method == CFD) return 2 * w.o0;
    return w.o0 - 4 > w.w0 ? w.o0 - 4 : w.w0;
}

// IO: A(s), B(s), K(s) (= ak), R(s) (= ar) reads; putU(s, x), putV(s, x)
// writes; st(i, k) / ld(i, k) the factor store of kept row i.
// Row i of the window system: e[k] is the entry in column i - ML + k.
template <typename T, int ML, int NB, bool WIDE, class IO>
DIRECT_HD void row_mfd(const IO& io, int n, T inv_h, int c, T* e, T& rhs) {
#pragma unroll
    for (int k = 0; k < NB; ++k) e[k] = T(0);
    const T akc = io.K(c);
    T dB = T(0);
    if (!WIDE || (c >= 4 && c <= n - 3)) {
        // interior: faces c-2..c+1, each coupling cells f-1..f+2
#pragma unroll
        for (int fo = -2; fo <= 1; ++fo) {
            const int f = c + fo;
            const T bf = io.B(f), rf = io.R(f);
            const T d = T(ST[fo + 2]);
            dB = fma(d, bf, dB);
            const T dr = d * rf;
#pragma unroll
            for (int go = -1; go <= 2; ++go) e[ML + fo + go] = fma(dr, T(ST[go + 1]), e[ML + fo + go]);
        }
    } else if constexpr (WIDE) {
        // closure rows: faces c-5..c+4 cover every D4 row, cells f-4..f+5
        // every G4 row
#pragma unroll
        for (int fo = -5; fo <= 4; ++fo) {
            const int f = c + fo;
            if (f < 0 || f > n) continue;
            const T d = T(dco(n, c, f));
            if (d == T(0)) continue;
            const T bf = io.B(f), rf = io.R(f);
            dB = fma(d, bf, dB);
            const T dr = d * rf;
#pragma unroll
            for (int go = -4; go <= 5; ++go) {
                const int cc = f + go;
                if (fo + go < -ML || fo + go > NB - 1 - ML) continue;
                if (cc < 1 || cc > n) continue;
                e[ML + fo + go] = fma(dr, T(gco(n, f, cc)), e[ML + fo + go]);
            }
        }
    }
    const T s = -akc * inv_h * inv_h;
#pragma unroll
    for (int k = 0; k < NB; ++k) e[k] *= s;
    e[ML] += T(1);
    rhs = io.A(c) - akc * inv_h * dB;
}

// CFD rows: i = 2 s is the z row of slot s, i = 2 s + 1 the y row.
template <typename T, int ML, int NB, bool WIDE, class IO>
DIRECT_HD void row_cfd(const IO& io, int n, T inv_h, int i, T* e, T& rhs) {
#pragma unroll
    for (int k = 0; k < NB; ++k) e[k] = T(0);
    const int s = i >> 1;
    rhs = T(0);
    if constexpr (!WIDE) {
        // interior slots 2..n-2 only: offsets within (3, 3)
        const T qh = T(3) * inv_h;
        e[ML - 2] = T(1); e[ML] = T(4); e[ML + 2] = T(1);
        if ((i & 1) == 0) {
            rhs = qh * (io.B(s + 1) - io.B(s - 1));
            e[ML - 1] = -qh * io.R(s - 1);
            e[ML + 3] = qh * io.R(s + 1);
        } else {
            rhs = qh * (io.A(s + 1) - io.A(s - 1));
            e[ML + 1] = qh * io.K(s + 1);
            e[ML - 3] = -qh * io.K(s - 1);
        }
        return;
    } else {
    if ((i & 1) == 0) {
        // z row: Pbar z + Qbar (ar y) = Qbar B on interior nodes; z_0 = z_n = 0
        if (s == 0 || s == n) { e[ML] = T(1); return; }
        // offsets: z_{s+k} at 2k, y_{s+k} at 2k + 1
        if (s == 1) {
            e[ML] = T(6); e[ML + 2] = T(6);
        } else if (s == n - 1) {
            e[ML - 2] = T(6); e[ML] = T(6);
        } else {
            e[ML - 2] = T(1); e[ML] = T(4); e[ML + 2] = T(1);
        }
        if (s == 1 || s == n - 1) {
            // nodes j0..j0+3 = 0..3 (offsets 2k - 1) or n-3..n (2k - 3); the
            // entries are placed by value selects so every index is fixed
            const bool first = s == 1;
            const int j0 = first ? 0 : n - 3;
            T ent[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T qh = T(QB1[k]) * inv_h;
                rhs = fma(qh, io.B(j0 + k), rhs);
                ent[k] = qh * io.R(j0 + k);
            }
            e[ML - 3] = first ? T(0) : ent[0];
            e[ML - 1] = first ? ent[0] : ent[1];
            e[ML + 1] = first ? ent[1] : ent[2];
            e[ML + 3] = first ? ent[2] : ent[3];
            e[ML + 5] = first ? ent[3] : T(0);
        } else {
            const T qh = T(3) * inv_h;
            rhs = qh * (io.B(s + 1) - io.B(s - 1));
            e[ML - 1] = -qh * io.R(s - 1);
            e[ML + 3] = qh * io.R(s + 1);
        }
        return;
    }
    // y row: P y + Q (ak z) = Q A, z and A on interior nodes only;
    // offsets: y_{s+k} at 2k, z_{s+k} at 2k - 1
    if (s == 0) {
        e[ML] = T(6); e[ML + 2] = T(18);
    } else if (s == n) {
        e[ML - 2] = T(18); e[ML] = T(6);
    } else {
        e[ML - 2] = T(1); e[ML] = T(4); e[ML + 2] = T(1);
    }
    if (s == 0 || s == n) {
        // nodes 1..3 (offsets 2k - 1) or n-3..n-1 (offsets 2k - 7); the
        // boundary node carries no unknown and is not read
        const bool first = s == 0;
        const int j0 = first ? 0 : n - 3;
        T ent[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool valid = first ? k >= 1 : k <= 2;
            const int j = valid ? j0 + k : (first ? 1 : n - 1);
            const T qh = valid ? (first ? T(Q0[k]) : T(-Q0[3 - k])) * inv_h : T(0);
            rhs = fma(qh, io.A(j), rhs);
            ent[k] = qh * io.K(j);
        }
        e[ML - 7] = first ? T(0) : ent[0];
        e[ML - 5] = first ? T(0) : ent[1];
        e[ML - 3] = first ? T(0) : ent[2];
        e[ML + 1] = first ? ent[1] : T(0);
        e[ML + 3] = first ? ent[2] : T(0);
        e[ML + 5] = first ? ent[3] : T(0);
    } else {
        const T qh = T(3) * inv_h;
        if (s + 1 <= n - 1) {
            rhs = fma(qh, io.A(s + 1), rhs);
            e[ML + 1] = qh * io.K(s + 1);
        }
        if (s - 1 >= 1) {
            rhs = fma(-qh, io.A(s - 1), rhs);
            e[ML - 3] = -qh * io.K(s - 1);
        }
    }
    }
}

// MFD: write the velocity of face f (owned faces fo0..fo1), whose G4 row
// reaches cells c..c+MU held in x.
template <typename T, int MU, class IO>
DIRECT_HD void put_face(const IO& io, int n, int f, int c, int fo0, int fo1, const T (&x)[MU + 1], T inv_h,
                        int mode) {
    if (f < fo0 || f > fo1) return;
    T g = T(0);
#pragma unroll
    for (int t = 0; t <= MU; ++t) {
        const int cc = c + t;
        if (cc >= 1 && cc <= n) g = fma(T(gco(n, f, cc)), x[t], g);
    }
    g *= inv_h;
    const T B = io.B(f), rr = io.R(f);
    io.putV(f, mode == OUT_NEXT ? fma(T(-2) * rr, g, B) : fma(-rr, g, B));
}

// One forward row: drop the unknowns outside the window, eliminate with the
// previous ML normalised U rows (ur[0] is row i - ML), push the new row and
// store it as kept row i - rb (rows before rb go to slot 0, which row rb
// overwrites: a store without a branch).  The U entries depend on the
// matrix only; when io.u_stored() says an earlier pass with the same matrix
// stored them, only the right-hand side value is written.
template <typename T, int ML, int MU, class IO>
DIRECT_HD void fwd_row(const IO& io, int i, int r0, int r1, int rb, T (&e)[ML + MU + 1], T r, T (&ur)[ML][MU],
                       T (&yr)[ML]) {
    constexpr int NB = ML + MU + 1;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int col = i - ML + k;
        if (col < r0 || col > r1) e[k] = T(0);
    }
#pragma unroll
    for (int c = 0; c < ML; ++c) {
        const T f = e[c];
#pragma unroll
        for (int t = 1; t <= MU; ++t)
            if (c + t < NB) e[c + t] = fma(-f, ur[c][t - 1], e[c + t]);
        r = fma(-f, yr[c], r);
    }
    const T inv = T(1) / e[ML];
#pragma unroll
    for (int j = 0; j < ML - 1; ++j) {
        yr[j] = yr[j + 1];
#pragma unroll
        for (int t = 0; t < MU; ++t) ur[j][t] = ur[j + 1][t];
    }
    yr[ML - 1] = r * inv;
#pragma unroll
    for (int t = 0; t < MU; ++t) ur[ML - 1][t] = e[ML + 1 + t] * inv;
    const int si = i >= rb ? i - rb : 0;
    io.st(si, 0, yr[ML - 1]);
    if (!io.u_stored()) {
#pragma unroll
        for (int t = 0; t < MU; ++t) io.st(si, t + 1, ur[ML - 1][t]);
    }
}

// One backward row: x_i = y_i - sum_t u_{i,t} x_{i+t}, pushed into x.
template <typename T, int MU, class IO>
DIRECT_HD T back_row(const IO& io, int i, int rb, T (&x)[MU + 1]) {
    T v = io.ld(i - rb, 0);
#pragma unroll
    for (int t = MU; t >= 1; --t) x[t] = x[t - 1];
#pragma unroll
    for (int t = 1; t <= MU; ++t) v = fma(-io.ld(i - rb, t), x[t], v);
    x[0] = v;
    return v;
}

// Pressure outputs written one at a time (the IO's putU).
struct PlainSink {
    template <typename T, class IO>
    DIRECT_HD void put(const IO& io, int s, T x) {
        io.putU(s, x);
    }
};

// Pressure outputs gathered into 32-byte pieces.  The outputs of a window
// arrive in descending slot order.  With a transposed target (consecutive
// slots of a line contiguous, the 64 lines of a wave in 64 rows), one store
// per lane and slot leaves each lane a partial 32-byte sector that the L2
// may evict before the rest arrives.  The slots [lo, hi] (the whole pieces
// within the output slots; a piece starts where s - 1 is a multiple of CH)
// are kept in a shift register instead and stored a piece at a time, with
// 16-byte stores at io.uptr(piece start); the others go through io.putU.
// The IO's target must hold slot s at uptr(s) = base + s - 1 with base
// 32-byte aligned whenever on is set.
template <typename T>
struct GatherSink {
    static constexpr int CH = 32 / sizeof(T);   // slots per piece
    struct alignas(16) P16 {
        T v[16 / sizeof(T)];
    };
    T b[CH];   // b[k]: slot s + k after slot s went in
    int lo, hi;
    bool on;
    // output slots o0..o1 (o0 >= 1)
    static DIRECT_HD GatherSink make(int o0, int o1, bool on) {
        GatherSink g;
        g.on = on;
        g.lo = 1 + ((o0 - 1 + CH - 1) / CH) * CH;   // first piece start >= o0
        g.hi = (o1 / CH) * CH;                       // last piece end <= o1
        return g;
    }
    template <class IO>
    DIRECT_HD void put(const IO& io, int s, T x) {
        if (!on || s < lo || s > hi) {
            io.putU(s, x);
            return;
        }
#pragma unroll
        for (int k = CH - 1; k > 0; --k) b[k] = b[k - 1];
        b[0] = x;
        if (((s - 1) & (CH - 1)) == 0 && io.live) {
            P16* p = (P16*)io.uptr(s);
            constexpr int E = 16 / sizeof(T);
#pragma unroll
            for (int j = 0; j < CH / E; ++j) {
                P16 w;
#pragma unroll
                for (int k = 0; k < E; ++k) w.v[k] = b[j * E + k];
                p[j] = w;
            }
        }
    }
};

// MFD pressure output of cell c from its solved value v, through sink sk.
template <typename T, class IO, class SK>
DIRECT_HD void put_cell(const IO& io, SK& sk, int c, T v, int mode, int src_s, T aF) {
    const T A = io.A(c);
    const T u = mode == OUT_NEXT ? fma(T(2), v, -A) : v;
    sk.put(io, c, u + (mode == OUT_NEXT && c == src_s ? aF : T(0)));
}

// Solve window w of one line and write its output slots.  mode OUT_NEXT
// writes 2 Ubar - A (+ aF at the source slot src_s when src_s > 0) and
// 2 vel - B, the explicit part of the next stage along the same lines;
// OUT_STAGE writes Ubar and vel.
// WIDE = false is for windows whose rows are all interior rows (see
// narrow_range).  The pressure outputs, produced in descending slot order,
// go through io.u_sink(first, last slot), which may gather them into wider
// stores.
template <typename T, int METHOD, bool WIDE, class IO>
DIRECT_HD void solve_window(const IO& io, int n, int S, int Se, int H, int w, T inv_h, int mode, int src_s,
                            T aF) {
    constexpr int ML = BandOf<METHOD, WIDE>::ML, MU = BandOf<METHOD, WIDE>::MU, NB = ML + MU + 1;
    const int smin = METHOD == MFD ? 1 : 0;
    const Win W = window(smin, n, S, Se, H, w);
    const int r0 = METHOD == MFD ? W.w0 : 2 * W.w0;
    const int r1 = METHOD == MFD ? W.w1 : 2 * W.w1 + 1;
    const int rb = first_kept_row(METHOD, W);

    // forward: Doolittle rows with the last ML normalised U rows in registers
    T ur[ML][MU], yr[ML];
#pragma unroll
    for (int j = 0; j < ML; ++j) {
        yr[j] = T(0);
#pragma unroll
        for (int t = 0; t < MU; ++t) ur[j][t] = T(0);
    }
    T x[MU + 1];   // backward ring: x[0] = x_i, x[t] = x_{i+t}
#pragma unroll
    for (int t = 0; t <= MU; ++t) x[t] = T(0);

    if constexpr (!WIDE) {
        // interior windows: branch-free loop bodies (unrolling them raised
        // the registers past the occupancy that hides the loads: kept rolled)
        auto sk = io.u_sink(W.o0, W.o1);
        if constexpr (METHOD == MFD) {
#pragma unroll 1
            for (int i = r0; i <= r1; ++i) {
                T e[NB], r;
                row_mfd<T, ML, NB, false>(io, n, inv_h, i, e, r);
                fwd_row<T, ML, MU>(io, i, r0, r1, rb, e, r, ur, yr);
            }
            int i = r1;
#pragma unroll 1
            for (; i > W.o1; --i) back_row<T, MU>(io, i, rb, x);
            // cell o1: its face o1 + 1 belongs to the next window
            {
                const T v = back_row<T, MU>(io, W.o1, rb, x);
                put_cell<T>(io, sk, W.o1, v, mode, src_s, aF);
            }
#pragma unroll 1
            for (i = W.o1 - 1; i >= W.o0; --i) {
                const T v = back_row<T, MU>(io, i, rb, x);
                put_cell<T>(io, sk, i, v, mode, src_s, aF);
                put_face<T, MU>(io, n, i + 1, i, W.o0, W.o1, x, inv_h, mode);
            }
            // face o0, whose lowest cell is o0 - 1
            back_row<T, MU>(io, W.o0 - 1, rb, x);
            put_face<T, MU>(io, n, W.o0, W.o0 - 1, W.o0, W.o1, x, inv_h, mode);
        } else {
#pragma unroll 1
            for (int sl = W.w0; sl <= W.w1; ++sl) {
                T e[NB], r;
                row_cfd<T, ML, NB, false>(io, n, inv_h, 2 * sl, e, r);
                fwd_row<T, ML, MU>(io, 2 * sl, r0, r1, rb, e, r, ur, yr);
                row_cfd<T, ML, NB, false>(io, n, inv_h, 2 * sl + 1, e, r);
                fwd_row<T, ML, MU>(io, 2 * sl + 1, r0, r1, rb, e, r, ur, yr);
            }
#pragma unroll 1
            for (int i = r1; i > 2 * W.o1 + 1; --i) back_row<T, MU>(io, i, rb, x);
#pragma unroll 1
            for (int sl = W.o1; sl >= W.o0; --sl) {
                const T y = back_row<T, MU>(io, 2 * sl + 1, rb, x);
                const T B = io.B(sl), rr = io.R(sl);
                io.putV(sl, mode == OUT_NEXT ? fma(T(-2) * rr, y, B) : fma(-rr, y, B));
                const T z = back_row<T, MU>(io, 2 * sl, rb, x);
                const T A = io.A(sl), kk = io.K(sl);
                const T u = mode == OUT_NEXT ? fma(T(-2) * kk, z, A) : fma(-kk, z, A);
                sk.put(io, sl, u + (mode == OUT_NEXT && sl == src_s ? aF : T(0)));
            }
        }
        return;
    }

    for (int i = r0; i <= r1; ++i) {
        T e[NB], r;
        if constexpr (METHOD == MFD) row_mfd<T, ML, NB, WIDE>(io, n, inv_h, i, e, r);
        else row_cfd<T, ML, NB, WIDE>(io, n, inv_h, i, e, r);
        fwd_row<T, ML, MU>(io, i, r0, r1, rb, e, r, ur, yr);
    }

    // backward: x_i = y_i - sum_t u_{i,t} x_{i+t}; the pressure outputs
    // (MFD cells o0..o1, CFD slots o0..o1 within 1..n-1) arrive in
    // descending order
    auto sk = METHOD == MFD ? io.u_sink(W.o0, W.o1) : io.u_sink(W.o0 > 1 ? W.o0 : 1, W.o1 < n - 1 ? W.o1 : n - 1);
    for (int i = r1; i >= rb; --i) {
        const T v = back_row<T, MU>(io, i, rb, x);
        if constexpr (METHOD == MFD) {
            const int c = i;
            if (c >= W.o0 && c <= W.o1) put_cell<T>(io, sk, c, v, mode, src_s, aF);
            // faces whose lowest cell is c
            const int fo0 = w == 0 ? 0 : W.o0;
            if (c == 1) {
                put_face<T, MU>(io, n, 0, c, fo0, W.o1, x, inv_h, mode);
                put_face<T, MU>(io, n, 1, c, fo0, W.o1, x, inv_h, mode);
            }
            if (c + 1 <= n - 2) put_face<T, MU>(io, n, c + 1, c, fo0, W.o1, x, inv_h, mode);
            if (c == n - 3) put_face<T, MU>(io, n, n - 1, c, fo0, W.o1, x, inv_h, mode);
            if (c == n - 4) put_face<T, MU>(io, n, n, c, fo0, W.o1, x, inv_h, mode);
        } else {
            const int s = i >> 1;
            if (s >= W.o0 && s <= W.o1) {
                if (i & 1) {
                    const T B = io.B(s), rr = io.R(s);
                    io.putV(s, mode == OUT_NEXT ? fma(T(-2) * rr, v, B) : fma(-rr, v, B));
                } else if (s >= 1 && s <= n - 1) {
                    const T A = io.A(s), kk = io.K(s);
                    T u = mode == OUT_NEXT ? fma(T(-2) * kk, v, A) : fma(-kk, v, A);
                    if (mode == OUT_NEXT && s == src_s) u += aF;
                    sk.put(io, s, u);
                }
            }
        }
    }
}

// Slots and kept unknown rows of the windows of a line.
DIRECT_HD int direct_smin(int method) { return method == MFD ? 1 : 0; }
inline int direct_nwin(int method, int n, int S, int Se) {
    const int ns = n - direct_smin(method) + 1;
    if (Se <= 0 || ns <= 2 * Se) return (ns + S - 1) / S;
    return (ns - 2 * Se + S - 1) / S + 2;
}
// Largest number of kept rows over the windows (factor store per thread).
inline int direct_rows(int method, int n, int S, int Se, int H) {
    int best = 0;
    const int nw = direct_nwin(method, n, S, Se), smin = direct_smin(method);
    for (int w = 0; w < nw; ++w) {
        const Win W = window(smin, n, S, Se, H, w);
        const int r1 = method == MFD ? W.w1 : 2 * W.w1 + 1;
        const int rows = r1 - first_kept_row(method, W) + 1;
        if (rows > best) best = rows;
    }
    return best;
}

// Windows wa..wb hold interior rows only (MFD cells 4..n-3, CFD slots
// 2..n-2) and are solved with the (3, 3) band; wa > wb when there are none.
// The window starts and ends grow with w, so the set is contiguous.
inline void narrow_range(int method, int n, int S, int Se, int H, int& wa, int& wb) {
    const int nw = direct_nwin(method, n, S, Se), smin = direct_smin(method);
    const int lo = method == MFD ? 4 : 2, hi = method == MFD ? n - 3 : n - 2;
    wa = nw;
    wb = -1;
    for (int w = 0; w < nw; ++w) {
        const Win W = window(smin, n, S, Se, H, w);
        if (W.w0 >= lo && W.w1 <= hi) {
            if (wa > w) wa = w;
            wb = w;
        }
    }
}

// A line held in host arrays (slots 0..n+1), for the margin computation
// and host checks.
template <typename T>
struct HostLine {
    const T *a, *b, *k, *r;
    T *u, *v, *fs;
    int nrow;   // kept rows per window (factor store stride)
    T A(int s) const { return a[s]; }
    T B(int s) const { return b[s]; }
    T K(int s) const { return k[s]; }
    T R(int s) const { return r[s]; }
    void putU(int s, T x) const { u[s] = x; }
    void putV(int s, T x) const { v[s] = x; }
    void st(int i, int kk, T x) const { fs[(size_t)i * 8 + kk] = x; }
    T ld(int i, int kk) const { return fs[(size_t)i * 8 + kk]; }
    PlainSink u_sink(int, int) const { return {}; }
    bool u_stored() const { return false; }
};

// Margin of the windows, in slots: the distance from a unit impulse in the
// pressure right-hand side beyond which the whole-line stage solution of a
// constant-coefficient line with (a kappa)(a / rho) / h^2 = c2 stays below
// tol of its peak, plus the reach of the operators.  -1 if the solution has
// not fallen that far within 4096 slots.
inline int direct_margin(int method, double c2, double tol) {
    const double ak = std::sqrt(c2);
    for (int L = 128; L <= 4096; L *= 2) {
        const int n = 2 * L;
        std::vector<double> A(n + 2, 0.0), B(n + 2, 0.0), K(n + 2, ak), R(n + 2, ak), U(n + 2, 0.0),
            V(n + 2, 0.0), F((size_t)2 * (n + 2) * 8, 0.0);
        A[L] = 1.0;
        HostLine<double> io{A.data(), B.data(), K.data(), R.data(), U.data(), V.data(), F.data(), 0};
        if (method == MFD) solve_window<double, MFD, true>(io, n, n, 0, 0, 0, 1.0, OUT_STAGE, -1, 0.0);
        else solve_window<double, CFD, true>(io, n, n + 1, 0, 0, 0, 1.0, OUT_STAGE, -1, 0.0);
        double peak = 0.0;
        for (int s = 0; s <= n; ++s) peak = std::fmax(peak, std::fmax(std::fabs(U[s]), std::fabs(V[s])));
        int far = -1;
        for (int s = 0; s <= n; ++s)
            if (std::fmax(std::fabs(U[s]), std::fabs(V[s])) >= tol * peak) far = std::max(far, std::abs(s - L));
        if (far < L - 16) return far + 6;
    }
    return -1;
}

}  // namespace direct
}  // namespace adi
