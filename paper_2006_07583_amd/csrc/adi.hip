// Host layer and C ABI of the Peaceman-Rachford ADI library (include/adi.h).
//
// Device state of a problem (all in one workspace allocation):
//   UAT  [x interior][y interior]   pressure-type hand-off read by the row pass
//                                    (A of eq. ecua1:ADI, stored transposed)
//   UC   [y interior][x interior]   hand-off read by the column pass (C)
//   VT   2 x [x node][y interior]   horizontal velocity, stored transposed
//   WSb  2 x [y node][x interior]   W* (vertical velocity after the explicit part)
//   aK, aKT, aRvT, aRw              a*kappa and a/rho in both line layouts
//   coefX, coefY                    compact-scheme factor tables per window
// A run of n steps is: transpose V in, one explicit column pass (A, W* of
// step m), then n x [row pass, column pass], the last column pass writing
// U^{m+n} and W^{m+n} into the caller's arrays, and V transposed back out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/adi.h"
#include "line_pass.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(ADI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr double kDelta = 3.7320508075688772935;   // 2 + sqrt 3, interior pivot of (1, 4, 1)

struct Plan {
    int n = 0, ns = 0, nlines = 0, nlg = 0, nwin = 0, S = 0, H = 0, deep = 0;
};

int64_t pad_to(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

Plan make_plan(int method, int dtype, int n, int nlines, int sweeps) {
    Plan p;
    p.n = n;
    p.ns = method == ADI_CFD ? n + 1 : n + 2;
    p.nlines = nlines;
    const int lw = adi::line_lanes(dtype);
    p.nlg = (nlines + lw - 1) / lw;
    p.H = adi::line_halo(dtype, method, sweeps);
    if (p.ns <= adi::LINE_WS) {
        p.nwin = 1;
        p.S = p.ns;
        p.deep = 1;
    } else {
        p.S = adi::LINE_WS - 2 * p.H;
        p.nwin = (p.ns + p.S - 1) / p.S;
        p.deep = 0;
    }
    return p;
}

int window_start(const Plan& p, int g) {
    if (p.nwin == 1) return 0;
    return std::max(0, std::min(g * p.S - p.H, p.ns - adi::LINE_WS));
}

// No-pivot LU of the tridiagonal matrix restricted to rows [r0, r1]; rows
// r0 > first / r1 < last are window edges inside the line: the coupling to
// the outside is dropped and the first edge row gets the interior pivot.
// Writes multipliers, inverse pivots and superdiagonal * inverse pivot at
// table index (row - w0).
void factor_rows(int r0, int r1, int first, int last, int w0,
                 double (*coef)(int row, int which, int n), int n,
                 double* tm, double* td, double* te) {
    if (r0 > r1) return;
    double dprev = 0.0, supprev = 0.0;
    for (int r = r0; r <= r1; ++r) {
        double sub = coef(r, 0, n), diag = coef(r, 1, n), sup = coef(r, 2, n);
        if (r == r0 && r0 > first) { sub = 0.0; diag = kDelta; }
        if (r == r0) sub = 0.0;
        if (r == r1 && r1 < last) sup = 0.0;
        double m = (r == r0) ? 0.0 : sub / dprev;
        double d = diag - m * supprev;
        tm[r - w0] = m;
        td[r - w0] = 1.0 / d;
        te[r - w0] = sup / d;
        dprev = d;
        supprev = sup;
    }
}

// P4 (Appendix A): rows 0..n, [6 18], [1 4 1], [18 6].
double coef_P(int r, int which, int n) {
    if (r == 0) return which == 0 ? 0.0 : (which == 1 ? 6.0 : 18.0);
    if (r == n) return which == 0 ? 18.0 : (which == 1 ? 6.0 : 0.0);
    return which == 1 ? 4.0 : 1.0;
}
// Reduced Pbar4: rows 1..n-1, [6 6], [1 4 1], [6 6].
double coef_Pbar(int r, int which, int n) {
    if (r == 1) return which == 0 ? 0.0 : 6.0;
    if (r == n - 1) return which == 2 ? 0.0 : 6.0;
    return which == 1 ? 4.0 : 1.0;
}

void build_tables(const Plan& p, std::vector<double>& out) {
    const int WS = adi::LINE_WS;
    out.assign((size_t)p.nwin * 6 * WS, 0.0);
    for (int g = 0; g < p.nwin; ++g) {
        double* t = out.data() + (size_t)g * 6 * WS;
        const int w0 = window_start(p, g);
        const int wl = std::min(w0 + WS, p.ns) - 1;
        factor_rows(std::max(w0, 0), std::min(wl, p.n), 0, p.n, w0, coef_P, p.n, t, t + WS, t + 2 * WS);
        factor_rows(std::max(w0, 1), std::min(wl, p.n - 1), 1, p.n - 1, w0, coef_Pbar, p.n,
                    t + 3 * WS, t + 4 * WS, t + 5 * WS);
    }
}

double ricker(const adi_params& p, double t) {
    const double x = kPi * p.src_f0 * (t - p.src_t0);
    const double x2 = x * x;
    return p.src_amp * (1.0 - 2.0 * x2) * std::exp(-x2);
}

}  // namespace

struct adi_problem {
    adi_params p{};
    hipStream_t st = nullptr;
    int dev = 0;
    int nix = 0, niy = 0;
    double a = 0.0;
    int64_t step = 0;
    bool bound = false;
    void *U = nullptr, *V = nullptr, *W = nullptr;
    int64_t ldU = 0, ldV = 0, ldW = 0;
    bool hasK = false, hasRv = false, hasRw = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    size_t esz = 4;
    int64_t ldx = 0, ldy = 0;
    void *UAT = nullptr, *UC = nullptr, *VT[2] = {nullptr, nullptr}, *WSb[2] = {nullptr, nullptr};
    void *aK = nullptr, *aKT = nullptr, *aRvT = nullptr, *aRw = nullptr, *coefX = nullptr, *coefY = nullptr;
    int vcur = 0, wcur = 0;
    Plan px, py;
};

namespace {

struct Layout {
    size_t off[12];
    size_t total;
};

// Offsets (bytes) of the workspace regions, each 256-byte aligned.
Layout layout(const adi_problem& pb) {
    const auto& p = pb.p;
    Layout L{};
    size_t cur = 0;
    auto put = [&](int idx, size_t elems) {
        L.off[idx] = cur;
        cur += (elems * pb.esz + 255) / 256 * 256;
    };
    const size_t nix = pb.nix, niy = pb.niy, ldx = pb.ldx, ldy = pb.ldy;
    put(0, nix * ldy);                                   // UAT
    put(1, niy * ldx);                                   // UC
    put(2, (size_t)(p.nx + 1) * ldy);                    // VT0
    put(3, (size_t)(p.nx + 1) * ldy);                    // VT1
    put(4, (size_t)(p.ny + 1) * ldx);                    // WS0
    put(5, (size_t)(p.ny + 1) * ldx);                    // WS1
    put(6, pb.hasK ? niy * ldx : 0);                     // aK
    put(7, pb.hasK ? nix * ldy : 0);                     // aKT
    put(8, pb.hasRv ? (size_t)(p.nx + 1) * ldy : 0);     // aRvT
    put(9, pb.hasRw ? (size_t)(p.ny + 1) * ldx : 0);     // aRw
    const bool cfd = p.method == ADI_CFD;
    put(10, cfd ? (size_t)pb.px.nwin * 6 * adi::LINE_WS : 0);   // coefX
    put(11, cfd ? (size_t)pb.py.nwin * 6 * adi::LINE_WS : 0);   // coefY
    L.total = cur;
    return L;
}

int validate(const adi_params* p) {
    if (!p) return fail(ADI_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(adi_params))
        return fail(ADI_EINVAL, "struct_size %u != %zu", p->struct_size, sizeof(adi_params));
    if (p->method != ADI_CFD && p->method != ADI_MFD) return fail(ADI_EINVAL, "unknown method %d", p->method);
    if (p->dtype != ADI_FP32 && p->dtype != ADI_FP64) return fail(ADI_EINVAL, "unknown dtype %d", p->dtype);
    if (p->order != 0) return fail(ADI_EINVAL, "order %d not supported (0 = x-implicit stage first)", p->order);
    if (p->nx < 8 || p->ny < 8) return fail(ADI_EINVAL, "nx, ny must be >= 8 (got %d, %d)", p->nx, p->ny);
    if (p->nx > (1 << 20) || p->ny > (1 << 20)) return fail(ADI_EINVAL, "grid too large");
    if (p->sweeps < 2 || p->sweeps > 16 || (p->sweeps & 1))
        return fail(ADI_EINVAL, "sweeps must be even and in [2, 16] (got %d)", p->sweeps);
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(ADI_EINVAL, "h must be positive");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(ADI_EINVAL, "dt must be positive");
    if (!(p->c_max > 0.0) || !std::isfinite(p->c_max)) return fail(ADI_EINVAL, "c_max must be positive");
    if (!std::isfinite(p->t0)) return fail(ADI_EINVAL, "t0 must be finite");
    if (!(p->kappa0 > 0.0) || !(p->rinv0 > 0.0)) return fail(ADI_EINVAL, "kappa0, rinv0 must be positive");
    const double cfl = p->dt * p->c_max / p->h;
    const double lim = p->method == ADI_CFD ? 1.15 : 0.81;
    if (!(cfl < lim))
        return fail(ADI_EINVAL, "cfl %.4f at or above the fixed-point limit %.2f of this method", cfl, lim);
    const int nix = p->method == ADI_CFD ? p->nx - 1 : p->nx;
    const int niy = p->method == ADI_CFD ? p->ny - 1 : p->ny;
    const bool has_src = p->src_i >= 0 || p->src_j >= 0;
    if (has_src) {
        if (p->src_i < 1 || p->src_i > nix || p->src_j < 1 || p->src_j > niy)
            return fail(ADI_EINVAL, "source (%d, %d) is not an interior pressure point", p->src_i, p->src_j);
        if (!std::isfinite(p->src_f0) || !std::isfinite(p->src_t0) || !std::isfinite(p->src_amp))
            return fail(ADI_EINVAL, "source parameters must be finite");
    }
    return ADI_OK;
}

void derive(adi_problem* pb) {
    const auto& p = pb->p;
    pb->esz = p.dtype == ADI_FP32 ? 4 : 8;
    pb->nix = p.method == ADI_CFD ? p.nx - 1 : p.nx;
    pb->niy = p.method == ADI_CFD ? p.ny - 1 : p.ny;
    pb->a = 0.5 * p.dt;
    const int64_t padm = 256 / (int64_t)pb->esz;   // 256-byte rows
    pb->ldx = pad_to(pb->nix, padm);
    pb->ldy = pad_to(pb->niy, padm);
    pb->px = make_plan(p.method, p.dtype, p.nx, pb->niy, p.sweeps);
    pb->py = make_plan(p.method, p.dtype, p.ny, pb->nix, p.sweeps);
}

template <typename T>
adi::LinePassArgs<T> base_args(const adi_problem& pb, const Plan& pl, const void* coef) {
    adi::LinePassArgs<T> a{};
    a.ak0 = (T)(pb.a * pb.p.kappa0);
    a.ar0 = (T)(pb.a * pb.p.rinv0);
    a.inv_h = (T)(1.0 / pb.p.h);
    a.nlines = pl.nlines;
    a.n = pl.n;
    a.ns = pl.ns;
    a.nlg = pl.nlg;
    a.nwin = pl.nwin;
    a.S = pl.S;
    a.H = pl.H;
    a.sweeps = pb.p.sweeps;
    a.deep = pl.deep;
    a.coef = (const T*)coef;
    a.src_q = a.src_s = -1;
    return a;
}

template <typename T>
int run_impl(adi_problem* pb, int64_t nsteps) {
    const auto& p = pb->p;
    const int method = p.method;
    hipStream_t st = pb->st;
    T* U = (T*)pb->U;
    T* V = (T*)pb->V;
    T* W = (T*)pb->W;
    const bool has_src = p.src_i >= 0;
    const double h2 = p.h * p.h;
    auto aF = [&](int64_t m) -> T {
        if (!has_src) return T(0);
        return (T)(pb->a * ricker(p, p.t0 + (double)m * p.dt) / h2);
    };

    // V (interior rows) -> VT
    HIP_TRY(adi::launch_scaled_copy<T>((T*)pb->VT[pb->vcur], pb->ldy, V + pb->ldV, 1, pb->ldV, p.nx + 1,
                                       pb->niy, T(1), st), "transpose V");
    // explicit part of stage 1 along columns: A and W* of step m
    {
        auto a = base_args<T>(*pb, pb->py, pb->coefY);
        a.uin = U + pb->ldU + 1;  a.uin_ld = pb->ldU;
        a.vin = W + 1;            a.vin_ld = pb->ldW;
        a.ak = pb->hasK ? (const T*)pb->aK : nullptr;   a.ak_ld = pb->ldx;
        a.ar = pb->hasRw ? (const T*)pb->aRw : nullptr; a.ar_ld = pb->ldx;
        a.vout = (T*)pb->WSb[pb->wcur]; a.vout_ld = pb->ldx;
        a.uout = (T*)pb->UAT;           a.uout_ld = pb->ldy;
        if (has_src) { a.src_q = p.src_i - 1; a.src_s = p.src_j; a.aF = aF(pb->step); }
        HIP_TRY(adi::launch_line_pass<T>(a, method, adi::LINE_EXPLICIT, st), "explicit pass");
    }
    for (int64_t s = 0; s < nsteps; ++s) {
        const int64_t m = pb->step + s;
        const T f1 = aF(m + 1);
        // row pass: stage-1 sweeps along x, then C and V^{m+1}
        {
            auto a = base_args<T>(*pb, pb->px, pb->coefX);
            a.uin = (const T*)pb->UAT;          a.uin_ld = pb->ldy;
            a.vin = (const T*)pb->VT[pb->vcur]; a.vin_ld = pb->ldy;
            a.ak = pb->hasK ? (const T*)pb->aKT : nullptr;   a.ak_ld = pb->ldy;
            a.ar = pb->hasRv ? (const T*)pb->aRvT : nullptr; a.ar_ld = pb->ldy;
            a.vout = (T*)pb->VT[1 - pb->vcur]; a.vout_ld = pb->ldy;
            a.uout = (T*)pb->UC;               a.uout_ld = pb->ldx;
            if (has_src) { a.src_q = p.src_j - 1; a.src_s = p.src_i; a.aF = f1; }
            HIP_TRY(adi::launch_line_pass<T>(a, method, adi::LINE_SWEEP, st), "row pass");
            pb->vcur ^= 1;
        }
        // column pass: stage-2 sweeps along y, then the next step's A and W*
        {
            const bool last = s == nsteps - 1;
            auto a = base_args<T>(*pb, pb->py, pb->coefY);
            a.uin = (const T*)pb->UC;            a.uin_ld = pb->ldx;
            a.vin = (const T*)pb->WSb[pb->wcur]; a.vin_ld = pb->ldx;
            a.ak = pb->hasK ? (const T*)pb->aK : nullptr;   a.ak_ld = pb->ldx;
            a.ar = pb->hasRw ? (const T*)pb->aRw : nullptr; a.ar_ld = pb->ldx;
            if (last) {
                a.vout = W + 1;             a.vout_ld = pb->ldW;
                a.uout = U + pb->ldU + 1;   a.uout_ld = pb->ldU;
                HIP_TRY(adi::launch_line_pass<T>(a, method, adi::LINE_FINAL, st), "column pass");
            } else {
                a.vout = (T*)pb->WSb[1 - pb->wcur]; a.vout_ld = pb->ldx;
                a.uout = (T*)pb->UAT;               a.uout_ld = pb->ldy;
                if (has_src) { a.src_q = p.src_i - 1; a.src_s = p.src_j; a.aF = f1; }
                HIP_TRY(adi::launch_line_pass<T>(a, method, adi::LINE_SWEEP, st), "column pass");
                pb->wcur ^= 1;
            }
        }
    }
    // VT -> V (interior rows)
    HIP_TRY(adi::launch_scaled_copy<T>(V + pb->ldV, pb->ldV, (const T*)pb->VT[pb->vcur], 1, pb->ldy, pb->niy,
                                       p.nx + 1, T(1), st), "transpose V back");
    pb->step += nsteps;
    return ADI_OK;
}

template <typename T>
int bind_materials(adi_problem* pb, const T* K, const T* Rv, const T* Rw, int64_t ldK, int64_t ldRv, int64_t ldRw) {
    const auto& p = pb->p;
    hipStream_t st = pb->st;
    const T a = (T)pb->a;
    if (K) {
        HIP_TRY(adi::launch_scaled_copy<T>((T*)pb->aK, pb->ldx, K + ldK + 1, ldK, 1, pb->niy, pb->nix, a, st), "aK");
        HIP_TRY(adi::launch_scaled_copy<T>((T*)pb->aKT, pb->ldy, K + ldK + 1, 1, ldK, pb->nix, pb->niy, a, st), "aKT");
    }
    if (Rv)
        HIP_TRY(adi::launch_scaled_copy<T>((T*)pb->aRvT, pb->ldy, Rv + ldRv, 1, ldRv, p.nx + 1, pb->niy, a, st), "aRvT");
    if (Rw)
        HIP_TRY(adi::launch_scaled_copy<T>((T*)pb->aRw, pb->ldx, Rw + 1, ldRw, 1, p.ny + 1, pb->nix, a, st), "aRw");
    if (p.method == ADI_CFD) {
        std::vector<double> tx, ty;
        build_tables(pb->px, tx);
        build_tables(pb->py, ty);
        std::vector<T> cx(tx.begin(), tx.end()), cy(ty.begin(), ty.end());
        HIP_TRY(hipMemcpyAsync(pb->coefX, cx.data(), cx.size() * sizeof(T), hipMemcpyHostToDevice, st), "coefX");
        HIP_TRY(hipMemcpyAsync(pb->coefY, cy.data(), cy.size() * sizeof(T), hipMemcpyHostToDevice, st), "coefY");
        HIP_TRY(hipStreamSynchronize(st), "bind sync");
        return ADI_OK;
    }
    HIP_TRY(hipStreamSynchronize(st), "bind sync");
    return ADI_OK;
}

}  // namespace

extern "C" {

const char* adi_status_string(int status) {
    switch (status) {
        case ADI_OK: return "ADI_OK";
        case ADI_EINVAL: return "ADI_EINVAL";
        case ADI_ENOMEM: return "ADI_ENOMEM";
        case ADI_EDEVICE: return "ADI_EDEVICE";
        case ADI_EBUSY: return "ADI_EBUSY";
        case ADI_ENOTREADY: return "ADI_ENOTREADY";
        case ADI_ENUMERIC: return "ADI_ENUMERIC";
        default: return "ADI_UNKNOWN";
    }
}

const char* adi_last_error(void) { return g_err.c_str(); }

int adi_params_init(adi_params* p) {
    if (!p) return fail(ADI_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(adi_params);
    p->method = ADI_CFD;
    p->dtype = ADI_FP32;
    p->order = 0;
    p->sweeps = 6;
    p->src_i = p->src_j = -1;
    p->kappa0 = 1.0;
    p->rinv0 = 1.0;
    p->src_amp = 1.0;
    return ADI_OK;
}

int adi_create(const adi_params* p, void* hip_stream, adi_problem** out) {
    g_err.clear();
    if (!out) return fail(ADI_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc != ADI_OK) return rc;
    adi_problem* pb = new (std::nothrow) adi_problem();
    if (!pb) return fail(ADI_ENOMEM, "host allocation failed");
    pb->p = *p;
    pb->st = (hipStream_t)hip_stream;
    derive(pb);
    hipError_t e = hipGetDevice(&pb->dev);
    if (e != hipSuccess) {
        delete pb;
        return hip_fail(e, "hipGetDevice");
    }
    *out = pb;
    return ADI_OK;
}

int adi_workspace_size(const adi_params* p, int has_K, int has_Rv, int has_Rw, size_t* bytes) {
    g_err.clear();
    if (!bytes) return fail(ADI_EINVAL, "bytes is NULL");
    int rc = validate(p);
    if (rc != ADI_OK) return rc;
    adi_problem tmp;
    tmp.p = *p;
    derive(&tmp);
    tmp.hasK = has_K != 0;
    tmp.hasRv = has_Rv != 0;
    tmp.hasRw = has_Rw != 0;
    *bytes = layout(tmp).total;
    return ADI_OK;
}

int adi_bind(adi_problem* pb, void* U, void* V, void* W, const void* K, const void* Rv, const void* Rw,
             const int64_t* ld, void* workspace, size_t workspace_bytes) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!U || !V || !W) return fail(ADI_EINVAL, "U, V and W are required");
    const auto& p = pb->p;
    const bool cfd = p.method == ADI_CFD;
    const int64_t colsU = cfd ? p.nx + 1 : p.nx + 2, colsV = p.nx + 1, colsW = cfd ? p.nx + 1 : p.nx + 2;
    int64_t l[6] = {colsU, colsV, colsW, colsU, colsV, colsW};
    if (ld)
        for (int i = 0; i < 6; ++i)
            if (ld[i] != 0) {
                if (ld[i] < l[i]) return fail(ADI_EINVAL, "ld[%d] = %lld below the row length %lld", i,
                                              (long long)ld[i], (long long)l[i]);
                l[i] = ld[i];
            }
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    if (pb->own_ws && pb->ws) {
        (void)hipFree(pb->ws);
        pb->ws = nullptr;
        pb->own_ws = false;
    }
    pb->bound = false;
    pb->hasK = K != nullptr;
    pb->hasRv = Rv != nullptr;
    pb->hasRw = Rw != nullptr;
    Layout L = layout(*pb);
    if (workspace) {
        if ((uintptr_t)workspace % 256) return fail(ADI_EINVAL, "workspace must be 256-byte aligned");
        if (workspace_bytes < L.total)
            return fail(ADI_EINVAL, "workspace of %zu bytes, %zu needed", workspace_bytes, L.total);
        pb->ws = (char*)workspace;
        pb->own_ws = false;
    } else {
        void* mem = nullptr;
        hipError_t e = hipMalloc(&mem, L.total);
        if (e != hipSuccess) return fail(ADI_ENOMEM, "hipMalloc(%zu): %s", L.total, hipGetErrorString(e));
        pb->ws = (char*)mem;
        pb->own_ws = true;
    }
    pb->ws_bytes = L.total;
    void** slots[12] = {&pb->UAT, &pb->UC, &pb->VT[0], &pb->VT[1], &pb->WSb[0], &pb->WSb[1],
                        &pb->aK, &pb->aKT, &pb->aRvT, &pb->aRw, &pb->coefX, &pb->coefY};
    for (int i = 0; i < 12; ++i) *slots[i] = pb->ws + L.off[i];
    pb->U = U; pb->V = V; pb->W = W;
    pb->ldU = l[0]; pb->ldV = l[1]; pb->ldW = l[2];
    pb->vcur = pb->wcur = 0;
    pb->step = 0;
    int rc = p.dtype == ADI_FP32
                 ? bind_materials<float>(pb, (const float*)K, (const float*)Rv, (const float*)Rw, l[3], l[4], l[5])
                 : bind_materials<double>(pb, (const double*)K, (const double*)Rv, (const double*)Rw, l[3], l[4], l[5]);
    if (rc != ADI_OK) return rc;
    pb->bound = true;
    return ADI_OK;
}

int adi_run(adi_problem* pb, int64_t nsteps) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!pb->bound) return fail(ADI_ENOTREADY, "problem has no bound arrays");
    if (nsteps < 0) return fail(ADI_EINVAL, "nsteps < 0");
    if (nsteps == 0) return ADI_OK;
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    return pb->p.dtype == ADI_FP32 ? run_impl<float>(pb, nsteps) : run_impl<double>(pb, nsteps);
}

int adi_step(adi_problem* pb) { return adi_run(pb, 1); }

int adi_sync(adi_problem* pb) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    return ADI_OK;
}

int adi_get_step(const adi_problem* pb, int64_t* m) {
    if (!pb || !m) return fail(ADI_EINVAL, "NULL argument");
    *m = pb->step;
    return ADI_OK;
}

int adi_set_step(adi_problem* pb, int64_t m) {
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (m < 0) return fail(ADI_EINVAL, "step < 0");
    pb->step = m;
    return ADI_OK;
}

int adi_destroy(adi_problem* pb) {
    if (!pb) return ADI_OK;
    if (pb->own_ws && pb->ws) {
        (void)hipSetDevice(pb->dev);
        (void)hipStreamSynchronize(pb->st);
        (void)hipFree(pb->ws);
    }
    delete pb;
    return ADI_OK;
}

}  // extern "C"
