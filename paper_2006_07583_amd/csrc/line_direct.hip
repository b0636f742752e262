// Direct (exact) line passes: each thread solves one window of one line with
// the banded LU of direct_core.h.  A wave holds 64 consecutive lines of the
// same window, so every branch on the slot index is uniform across the wave;
// the factor store is laid out [wave][kept row][value][lane]: each access is
// one contiguous 64-lane segment and a wave's rows follow each other.
#include "direct_core.h"
#include "line_pass.h"

namespace adi {

namespace {

template <typename T, int NV>   // NV: values per kept row
struct DevLine {
    DirectArgs<T> a;   // a copy: its fields stay in scalar registers
    int64_t q;
    int64_t tid;
    bool live;
    bool ugather;   // u_s == 1 and 32-byte pieces of a u row start where s - 1
                    // is a multiple of 32 / sizeof(T)
    bool ustored;   // the factor store already holds the U entries of this
                    // matrix (an earlier pass along the same lines)
    DIRECT_HD T A(int s) const { return a.a[q * a.a_l + s * a.a_s]; }
    DIRECT_HD T B(int s) const { return a.b[q * a.b_l + s * a.b_s]; }
    DIRECT_HD T K(int s) const { return a.k[q * a.k_l + s * a.k_s]; }
    DIRECT_HD T R(int s) const { return a.r[q * a.r_l + s * a.r_s]; }
    DIRECT_HD void putU(int s, T x) const {
        if (live) a.u[q * a.u_l + s * a.u_s] = x;
    }
    DIRECT_HD void putV(int s, T x) const {
        if (live) a.v[q * a.v_l + s * a.v_s] = x;
    }
    DIRECT_HD T* uptr(int s) const { return a.u + q * a.u_l + s * a.u_s; }
    DIRECT_HD bool u_stored() const { return ustored; }
    DIRECT_HD direct::GatherSink<T> u_sink(int o0, int o1) const {
        return direct::GatherSink<T>::make(o0, o1, ugather);
    }
    DIRECT_HD int64_t fi(int i, int k) const {
        return (((tid >> 6) * a.drows + i) * NV + k) * 64 + (tid & 63);
    }
    DIRECT_HD void st(int i, int k, T x) const { a.fs[fi(i, k)] = x; }
    DIRECT_HD T ld(int i, int k) const { return a.fs[fi(i, k)]; }
};

template <typename T, int METHOD, bool WIDE>
__global__ __launch_bounds__(64) void line_direct_kernel(DirectArgs<T> p, int ugather, int ustored) {
    const int64_t tid = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (tid >= p.nthr) return;
    const int q = (int)(tid % p.nlp), wi = (int)(tid / p.nlp);
    const int w = wi < p.wsplit ? p.wbase + wi : p.wbase2 + (wi - p.wsplit);
    const bool live = q < p.nlines;
    const DevLine<T, direct::BandOf<METHOD, WIDE>::MU + 1> io{p, live ? q : 0, tid, live, ugather != 0, ustored != 0};
    const int src = (live && q == p.src_q) ? p.src_s : -1;
    direct::solve_window<T, METHOD, WIDE>(io, p.n, p.S, p.Se, p.H, w, p.inv_h, p.mode, src, p.aF);
}

}  // namespace

template <typename T>
hipError_t launch_direct(const DirectArgs<T>& p, int method, bool wide, bool ustored, hipStream_t st) {
    // a transposed pressure target (u_s 1): slot s of line l at u + l u_l + s
    const int ug = p.u_s == 1 && ((uintptr_t)(p.u + 1) % 32) == 0 && (p.u_l * (int64_t)sizeof(T)) % 32 == 0;
    if (p.wcount <= 0 || p.wsplit < 0 || p.wsplit > p.wcount || p.wbase < 0 || p.wbase + p.wsplit > p.nwin ||
        p.wbase2 < 0 || p.wbase2 + (p.wcount - p.wsplit) > p.nwin || p.nlp % 64 || (int64_t)p.nlp * p.wcount != p.nthr)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)(p.nthr / 64)), block(64);
    if (method == LINE_MFD) {
        if (wide) hipLaunchKernelGGL((line_direct_kernel<T, direct::MFD, true>), grid, block, 0, st, p, ug, ustored ? 1 : 0);
        else hipLaunchKernelGGL((line_direct_kernel<T, direct::MFD, false>), grid, block, 0, st, p, ug, ustored ? 1 : 0);
    } else {
        if (wide) hipLaunchKernelGGL((line_direct_kernel<T, direct::CFD, true>), grid, block, 0, st, p, ug, ustored ? 1 : 0);
        else hipLaunchKernelGGL((line_direct_kernel<T, direct::CFD, false>), grid, block, 0, st, p, ug, ustored ? 1 : 0);
    }
    return hipGetLastError();
}

template hipError_t launch_direct<float>(const DirectArgs<float>&, int, bool, bool, hipStream_t);
template hipError_t launch_direct<double>(const DirectArgs<double>&, int, bool, bool, hipStream_t);

int direct_values_per_row(int method) {
    return method == LINE_MFD ? direct::Band<direct::MFD>::MU + 1 : direct::Band<direct::CFD>::MU + 1;
}

}  // namespace adi
