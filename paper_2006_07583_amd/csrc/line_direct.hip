// Direct (exact) line passes: each thread solves one window of one line with
// the banded LU of direct_core.h.  A wave holds 64 consecutive lines of the
// same window, so every branch on the slot index is uniform across the wave;
// the factor store is laid out [kept row][value][thread] so that each of its
// accesses is one contiguous 64-lane segment.
#include "direct_core.h"
#include "line_pass.h"

namespace adi {

namespace {

template <typename T, int METHOD>
struct DevLine {
    static constexpr int NV = direct::Band<METHOD>::MU + 1;   // values per kept row
    const DirectArgs<T>* p;
    int64_t q;
    int64_t tid;
    bool live;
    DIRECT_HD T A(int s) const { return p->a[q * p->a_l + s * p->a_s]; }
    DIRECT_HD T B(int s) const { return p->b[q * p->b_l + s * p->b_s]; }
    DIRECT_HD T K(int s) const { return p->k ? p->k[q * p->k_l + s * p->k_s] : p->k0; }
    DIRECT_HD T R(int s) const { return p->r ? p->r[q * p->r_l + s * p->r_s] : p->r0; }
    DIRECT_HD void putU(int s, T x) const {
        if (live) p->u[q * p->u_l + s * p->u_s] = x;
    }
    DIRECT_HD void putV(int s, T x) const {
        if (live) p->v[q * p->v_l + s * p->v_s] = x;
    }
    DIRECT_HD void st(int i, int k, T x) const { p->fs[((int64_t)i * NV + k) * p->nthr + tid] = x; }
    DIRECT_HD T ld(int i, int k) const { return p->fs[((int64_t)i * NV + k) * p->nthr + tid]; }
};

template <typename T, int METHOD>
__global__ __launch_bounds__(64) void line_direct_kernel(DirectArgs<T> p) {
    const int64_t tid = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (tid >= p.nthr) return;
    const int q = (int)(tid % p.nlp), w = (int)(tid / p.nlp);
    const bool live = q < p.nlines;
    const DevLine<T, METHOD> io{&p, live ? q : 0, tid, live};
    const int src = (live && q == p.src_q) ? p.src_s : -1;
    direct::solve_window<T, METHOD>(io, p.n, p.S, p.H, w, p.inv_h, p.mode, src, p.aF);
}

}  // namespace

template <typename T>
hipError_t launch_direct(const DirectArgs<T>& p, int method, hipStream_t st) {
    if (p.nthr <= 0 || p.nthr % 64 || p.nlp % 64 || (int64_t)p.nlp * p.nwin != p.nthr) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(p.nthr / 64)), block(64);
    if (method == LINE_MFD) hipLaunchKernelGGL((line_direct_kernel<T, direct::MFD>), grid, block, 0, st, p);
    else hipLaunchKernelGGL((line_direct_kernel<T, direct::CFD>), grid, block, 0, st, p);
    return hipGetLastError();
}

template hipError_t launch_direct<float>(const DirectArgs<float>&, int, hipStream_t);
template hipError_t launch_direct<double>(const DirectArgs<double>&, int, hipStream_t);

int direct_values_per_row(int method) {
    return method == LINE_MFD ? direct::Band<direct::MFD>::MU + 1 : direct::Band<direct::CFD>::MU + 1;
}

}  // namespace adi
