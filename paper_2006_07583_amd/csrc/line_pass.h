// Internal interface between the host layer and the line-pass kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adi {

enum { LINE_CFD = 0, LINE_MFD = 1 };
enum { LINE_SWEEP = 0, LINE_FINAL = 1, LINE_EXPLICIT = 2 };
enum { LINE_WS = 512 };   // slots per window of the multi-window kernel
// single-window tile shapes: windows of 512, 256, 128 slots (0 .. 2), and
// the same windows with a quarter of the lines per workgroup (3 .. 5)
enum { LINE_NCFG = 6 };

// Arguments of one line pass.  Along a line, slot s holds the pressure value
// of index s (interior slots 1..n-1 for CFD, 1..n for MFD) and the velocity
// value of node s (0..n).  For line q:
//   uin[(s-1)*uin_ld + q], ak[(s-1)*ak_ld + q]        pressure-type inputs
//   vin[s*vin_ld + q],     ar[s*ar_ld + q]            velocity-type inputs
//   vout[s*vout_ld + q]                                velocity output
//   uout[q*uout_ld + (s-1)]  (utrans = 1), or uout[(s-1)*uout_ld + q] (utrans = 0)
template <typename T>
struct LinePassArgs {
    const T* uin; int64_t uin_ld;
    const T* vin; int64_t vin_ld;
    const T* ak;  int64_t ak_ld;     // a*kappa, NULL -> ak0
    const T* ar;  int64_t ar_ld;     // a*(1/rho), NULL -> ar0
    T* vout; int64_t vout_ld;
    T* uout; int64_t uout_ld;
    const T* coef;                   // compact: [nwin][6][LINE_WS] factor tables
    T ak0, ar0, inv_h, aF;
    int nlines, n, ns, nlg, nwin, S, H, sweeps;
    int src_q, src_s;                // source (line, slot), -1 = none
    int deep;                        // single window: deep halo exchange
    int gbase, gstride, gcount;      // multi-window kernel: windows g = gbase + i*gstride, i < gcount
    int utrans;                      // 1: pressure output transposed (via LDS), 0: natural layout
    // compensated FP32 state: low words of the inputs (NULL = zero) and of
    // the outputs (NULL = store the rounded sum only)
    const T* uin_lo; const T* vin_lo; T* vout_lo; T* uout_lo;
    // grouped launches: when set, aF = aFtab[tick] (tick read from device memory)
    const T* aFtab;
    // tolerance-tested stages (wave-per-line kernel, single launches): when
    // eps_part is set the launch runs only if *eps_go != 0, and workgroup
    // `tile` stores the squared Frobenius norms of the changes of the last two
    // sweeps, {|u_{K-1} - u_{K-2}|^2, |v_{K-1} - v_{K-2}|^2, |u_K - u_{K-1}|^2,
    // |v_K - v_{K-1}|^2}, over the slots it writes at eps_part[q nlg nwin + tile]
    double* eps_part;
    const int* eps_go;
    // Dirichlet wall values (NULL: zero walls).  For line q the value at its
    // first pressure slot (0) is bnd[6q] bsc[0] + bnd[6q+1] bsc[1] +
    // bnd[6q+2] bsc[2], at its last (n for CFD, n + 1 for MFD) the same with
    // bnd[6q+3..6q+5].  Distributed forcing (NULL: none): aFf * ff at every
    // interior pressure slot, added to the pressure output (ff laid out like
    // ak).
    const T* bnd;
    T bsc[3];
    const T* ff; int64_t ff_ld;
    T aFf;
    // Damping layers along this direction (dmpm: bit 0 the line's first
    // wall, bit 1 its last; 0 = none): rate dmp0 (1 - dist * dmpiw)^2 at a
    // point dist cells from a wall with its bit set, dmp0 everywhere when
    // dmpiw = 0.  ah = dt / 2.
    T dmp0, dmpiw, ah;
    int dmpm;
    // wave-per-line kernel: order of the tiles across the XCDs (0: line
    // group by line group, 1: window by window, 2: launch order, 3 .. 6:
    // window by window within blocks of 2^(torder - 1) line groups)
    int torder;
};

// A grouped launch: the passes items[0..nitems) (any problems, any
// directions, one kernel variant) in one grid; starts[i] is the first tile
// of item i (prefix sums of nlg * nwin, starts[nitems] = total).
template <typename T>
struct GroupArgs {
    const LinePassArgs<T>* items;
    const int* starts;
    const int* tick;
    int nitems, total;
};

// Single-window kernel (line_pass.hip), tile shape cfg (window line_ws(cfg)).
template <typename T>
hipError_t launch_line_pass(const LinePassArgs<T>& a, int method, int mode, hipStream_t st, bool comp, int cfg,
                            bool full = false);
template <typename T>
hipError_t launch_line_group(const GroupArgs<T>& g, int cfg, int method, int mode, hipStream_t st, bool comp,
                             bool full = false);

// dst[r*dld + c] = scale * (src[r*srs + c*scs] + src2[same])   (src2 may be NULL)
template <typename T>
hipError_t launch_scaled_copy(T* dst, int64_t dld, const T* src, int64_t srs, int64_t scs, int rows,
                              int cols, T scale, hipStream_t st, const T* src2 = nullptr);

// dst[r*dld + c] = 0 for r < rows, c < cols
template <typename T>
hipError_t launch_fill_zero(T* dst, int64_t dld, int rows, int cols, hipStream_t st);

int line_lanes(int dtype, int cfg);
int line_ws(int cfg);
int line_halo(int dtype, int method, int sweeps, double cfl);

// Multi-window variant (line_pass2.hip): lines per workgroup and slots per
// lane segment.
template <typename T>
hipError_t launch_line_pass2(const LinePassArgs<T>& a, int method, int mode, hipStream_t st, bool comp = false);
template <typename T>
hipError_t launch_line_group2(const GroupArgs<T>& g, int method, int mode, hipStream_t st, bool comp);
int line2_lanes(int dtype);
int line2_seg(int dtype);

// Multi-window variant with one line per half wave (line_pass3.hip; FP32,
// FP64 and the compensated FP32 mode): lines per workgroup.
// full: the variant with the optional features (damping layers, wall data,
// distributed forcing)
template <typename T>
hipError_t launch_line_pass3(const LinePassArgs<T>& a, int method, int mode, hipStream_t st, bool comp = false,
                             bool full = false);
template <typename T>
hipError_t launch_line_group3(const GroupArgs<T>& g, int method, int mode, hipStream_t st, bool comp = false,
                              bool full = false);
int line3_lanes(int dtype);
int line3_torder(int dtype, int method, int nlines);

// Tolerance-tested stages (LinePassArgs::eps_part): a pass is `attempts`
// launches, attempt j with K = kmin + 2 j sweeps running while go[j] != 0
// (go[0] = 1 at the start of every pass).  After attempt j, eps_check reduces
// the nb per-workgroup partials, sets go[j + 1], and when the attempt decides
// the stage adds one pass and K sweeps to stats[0], stats[1]; the check of
// the last attempt also resets the flags for the next pass.
hipError_t launch_eps_check(const double* part, int nb, int* go, int j, int attempts, double eps, int K,
                            int kmin, int kmax, long long* stats, hipStream_t st);

// Direct (exact) line pass (line_direct.hip): thread t solves the
// (t / nlp)-th window of the launch on line t % nlp (lines padded to nlp, a
// multiple of 64).  Element
// (line q, slot s) of each array sits at base[q * x_l + s * x_s]; A and K are
// pressure-type (slots 1..n-1 for CFD, 1..n for MFD), B, R, V velocity-type
// (slots 0..n).  mode 0 writes 2 Ubar - A (+ aF at (src_q, src_s)) and
// 2 vel - B, mode 1 Ubar and vel.  fs holds nthr * drows * values-per-row
// elements.
template <typename T>
struct DirectArgs {
    const T* a; int64_t a_l, a_s;
    const T* b; int64_t b_l, b_s;
    const T* k; int64_t k_l, k_s;   // a kappa (a constant: one element, strides 0)
    const T* r; int64_t r_l, r_s;   // a / rho (likewise)
    T* u; int64_t u_l, u_s;
    T* v; int64_t v_l, v_s;
    T* fs;
    T inv_h, aF;
    int nlines, nlp, n, S, Se, H, nwin, mode;   // Se: output slots of the end windows
    int src_q, src_s;
    // this launch solves wcount windows: wbase + i for i < wsplit, then
    // wbase2 + (i - wsplit)
    int wbase, wcount, wsplit, wbase2;
    int drows;           // kept rows per thread in fs (the largest over the windows)
    int64_t nthr;        // nlp * wcount
};
// wide: the closure rows of the line ends are in reach (windows 0 and past
// narrow_last); otherwise the interior (3, 3) band.  ustored: the factor
// store already holds the U entries of this matrix, from an earlier launch
// over the same windows
template <typename T>
hipError_t launch_direct(const DirectArgs<T>& p, int method, bool wide, bool ustored, hipStream_t st);
int direct_values_per_row(int method);

}  // namespace adi
