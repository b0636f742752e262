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
//   Vs                              spare velocity of the direction that ends a step
// The first run after adi_bind transposes U, V, W in and runs one explicit
// column pass (A, W* of step m); every step is then [row pass, column pass],
// the column pass leaving the next step's A and W*, so the state stays in
// the workspace between runs.  adi_get_state re-runs the last column pass in
// its final form (U^{m}, W^{m} instead of the hand-off) into the target
// arrays and transposes V out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "../../include/adi.h"
#include "direct_core.h"
#include "line_pass.h"
#include "problem.h"

namespace {
thread_local std::string g_err;
}

namespace adi {

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

}  // namespace adi

namespace {

using adi::fail;
using adi::hip_fail;
using adi::Plan;


constexpr double kPi = 3.14159265358979323846;
constexpr double kDelta = 3.7320508075688772935;   // 2 + sqrt 3, interior pivot of (1, 4, 1)

int64_t pad_to(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

Plan make_plan(int method, int dtype, int n, int nlines, int sweeps, double cfl) {
    Plan p;
    p.n = n;
    p.ns = method == ADI_CFD ? n + 1 : n + 2;
    p.nlines = nlines;
    p.H = adi::line_halo(dtype, method, sweeps, cfl);
    if (p.ns <= adi::LINE_WS) {
        // single window: the smallest of the shapes 0 .. 2 whose window
        // holds the line, or its quarter-width twin (3 .. 5) when the wide
        // shape would launch fewer than 1024 workgroups (a workgroup's
        // passes are latency-bound: 120^2 to 500^2 FP32 passes took 24-35
        // us wide and 21-27 us narrow, FP64 25-44 against 14-27)
        p.ver = 1;
        p.cfg = 0;
        for (int c = 2; c >= 0; --c)
            if (p.ns <= adi::line_ws(c)) { p.cfg = c; break; }
        if ((nlines + adi::line_lanes(dtype, p.cfg) - 1) / adi::line_lanes(dtype, p.cfg) < 1024) p.cfg += 3;
        p.nwin = 1;
        p.S = p.ns;
        p.deep = 1;
    } else {
        // multi-window: the wave-per-line kernel (barrier-free sweeps, all
        // three number modes); the direct solves keep the slot-major layout
        // of the segment kernel, which their thread-per-line passes read (64
        // lines at one slot are contiguous)
        p.ver = sweeps == 0 ? 2 : 3;
        p.seg = adi::line2_seg(dtype);
        // windows of LINE_WS slots overlapping by 2H; the first and last own
        // LINE_WS - H central slots, the others S = LINE_WS - 2H
        p.S = adi::LINE_WS - 2 * p.H;
        const int F = adi::LINE_WS - p.H;
        p.nwin = p.ns <= 2 * F ? 2 : 2 + (p.ns - 2 * F + p.S - 1) / p.S;
        p.deep = 0;
    }
    const int lw = p.ver == 1 ? adi::line_lanes(dtype, p.cfg)
                              : (p.ver == 2 ? adi::line2_lanes(dtype) : adi::line3_lanes(dtype));
    // the wave-per-line kernel indexes its rows r = q + 1 (row 0 all zeros)
    p.nlg = (nlines + (p.ver == 3 ? 1 : 0) + lw - 1) / lw;
    p.torder = adi::line3_torder(dtype, method, nlines);
    return p;
}

// Single-window tile shape cfg for a plan (lines per workgroup follow it).
void set_cfg(Plan& p, int dtype, int cfg) {
    p.cfg = cfg;
    const int lw = adi::line_lanes(dtype, cfg);
    p.nlg = (p.nlines + lw - 1) / lw;
}

// ---- tuned plans ----
//
// The launch choices the autotuner times: the tile shape of the
// single-window kernel (every shape whose window holds the line) and the
// tile order of the wave-per-line kernel.  The other kernels have none.
int plan_choices(const Plan& p, int* c) {
    int k = 0;
    if (p.ver == 1) {
        for (int cfg = 0; cfg < adi::LINE_NCFG; ++cfg)
            if (p.ns <= adi::line_ws(cfg)) c[k++] = cfg;
    } else if (p.ver == 3) {
        for (int o = 0; o < 7; ++o) c[k++] = o;
    }
    return k;
}

int plan_choice(const Plan& p) { return p.ver == 1 ? p.cfg : p.torder; }

void apply_choice(Plan& p, int dtype, int ch) {
    if (p.ver == 1)
        set_cfg(p, dtype, ch);
    else
        p.torder = ch;
}

// Process-wide cache of tuned choices: (device architecture, method, dtype,
// slots per line, lines, margin, kernel) -> choice.  With the environment
// variable ADI_TUNE_CACHE naming a file, the cache reads it when a plan is
// first made with that name set (entries of the file replace those held)
// and writes itself back to it after each tuning.
using TuneKey = std::tuple<std::string, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;
std::string g_tune_path;   // the file last read
std::string g_arch[64];

std::string device_arch() {   // caller holds g_tune_mu
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return "unknown";
    if (g_arch[dev].empty()) {
        hipDeviceProp_t pr;
        g_arch[dev] = hipGetDeviceProperties(&pr, dev) == hipSuccess ? std::string(pr.gcnArchName) : "unknown";
        for (char& ch : g_arch[dev])
            if (ch == ' ') ch = '_';
    }
    return g_arch[dev];
}

TuneKey tune_key(const std::string& arch, int method, int dtype, const Plan& p) {
    return TuneKey(arch, method, dtype, p.ns, p.nlines, p.H, p.ver);
}

// Cache file lines: "adi-tune arch method dtype ns nlines H ver choice".
void tune_load() {   // caller holds g_tune_mu
    const char* path = std::getenv("ADI_TUNE_CACHE");
    if (!path || !*path || g_tune_path == path) return;
    g_tune_path = path;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string tag, arch;
        int v[7];
        if (!(in >> tag >> arch) || tag != "adi-tune") continue;
        bool ok = true;
        for (int& x : v) ok = ok && (bool)(in >> x);
        if (ok) g_tune[TuneKey(arch, v[0], v[1], v[2], v[3], v[4], v[5])] = v[6];
    }
}

int tune_save() {   // caller holds g_tune_mu
    const char* path = std::getenv("ADI_TUNE_CACHE");
    if (!path || !*path) return ADI_OK;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        for (const auto& kv : g_tune) {
            const auto& k = kv.first;
            f << "adi-tune " << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' '
              << std::get<3>(k) << ' ' << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << std::get<6>(k) << ' '
              << kv.second << '\n';
        }
        if (!f) return fail(ADI_EINVAL, "cannot write the tuning cache %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(ADI_EINVAL, "cannot replace the tuning cache %s", path);
    return ADI_OK;
}

// A cached choice for the plan, if any (valid for the plan's kernel).
void apply_tuned(Plan& p, int method, int dtype) {
    int c[8];
    const int nc = plan_choices(p, c);
    if (nc == 0) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();
    const auto it = g_tune.find(tune_key(device_arch(), method, dtype, p));
    if (it == g_tune.end()) return;
    for (int i = 0; i < nc; ++i)
        if (c[i] == it->second) {
            apply_choice(p, dtype, it->second);
            p.tuned = true;
        }
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

// Factor tables of the single-window kernel (one window per line): [6][WS],
// WS = window of the plan's tile shape, into t[0 .. 6 WS).
void build_tables(const Plan& p, double* t) {
    const int WS = adi::line_ws(p.cfg);
    for (int i = 0; i < 6 * WS; ++i) t[i] = 0.0;
    factor_rows(0, p.n, 0, p.n, 0, coef_P, p.n, t, t + WS, t + 2 * WS);
    factor_rows(1, p.n - 1, 1, p.n - 1, 0, coef_Pbar, p.n, t + 3 * WS, t + 4 * WS, t + 5 * WS);
}

double ricker(const adi_params& p, double t) {
    const double x = kPi * p.src_f0 * (t - p.src_t0);
    const double x2 = x * x;
    return p.src_amp * (1.0 - 2.0 * x2) * std::exp(-x2);
}

double signal_at(const adi_signal& g, double t) {
    if (g.kind == ADI_SIGNAL_RICKER) {
        const double x = kPi * g.f0 * (t - g.t0);
        return g.amp * (1.0 - 2.0 * x * x) * std::exp(-x * x);
    }
    if (g.kind == ADI_SIGNAL_COS) return g.amp * std::cos(2.0 * kPi * g.f0 * (t - g.t0));
    return 0.0;
}

}  // namespace

namespace {

// Workspace regions of one direction: P, V0, V1, K, R, Plo, V0lo, V1lo, coef,
// Vs, Vslo, FF (forcing field), BND (wall coefficients).
struct Layout {
    size_t off[2][13];
    size_t fs_off[2];   // factor stores of the direct solves, one per direction
    size_t dc_off;    // their constant materials
    size_t red_off;   // per-block partial maxima of the material check at bind
    size_t chk_off;   // health check: per-block partials and the running state
    size_t total;
};
constexpr int kRedBlocks = 256;
// health check state after the partials: {non-finite seen, largest
// magnitude, first step found non-finite + 1, step of the last check}
constexpr int kChkState = 2 * kRedBlocks;

// Direction of the pass that ends a step.
int last_dir(const adi_params& p) { return p.order == 0 ? 1 : 0; }

// Offsets (bytes) of the workspace regions, each 256-byte aligned.
Layout layout(const adi_problem& pb) {
    const auto& p = pb.p;
    Layout L{};
    size_t cur = 0;
    const bool cfd = p.method == ADI_CFD, comp = p.dtype == ADI_FP32C;
    for (int d = 0; d < 2; ++d) {
        const auto& D = pb.d[d];
        const Plan& pl = d == 0 ? pb.px : pb.py;
        const size_t pe = (size_t)D.rows_p * D.ld, ve = (size_t)D.rows_v * D.ld;
        const bool hasR = d == 0 ? pb.hasRv : pb.hasRw;
        // the final re-run of adi_get_state writes its velocity here unless it
        // can go straight into the target (slot-major column passes)
        const bool spare = d == last_dir(p) && (d == 0 || D.lm);
        const size_t sizes[13] = {pe, ve, ve, pb.hasK ? pe : 0, hasR ? ve : 0, comp ? pe : 0, comp ? ve : 0,
                                  comp ? ve : 0, cfd && pl.ver == 1 ? (size_t)6 * adi::LINE_WS : 0,
                                  spare ? ve : 0, spare && comp ? ve : 0, pb.fsig.kind ? pe : 0,
                                  pb.bsig.kind ? (size_t)6 * (pl.nlines + 64) : 0};
        for (int i = 0; i < 13; ++i) {
            L.off[d][i] = cur;
            cur += (sizes[i] * pb.esz + 255) / 256 * 256;
        }
    }
    L.fs_off[0] = L.fs_off[1] = cur;
    if (p.sweeps == 0) {
        const int nv = adi::direct_values_per_row(p.method == ADI_MFD ? adi::LINE_MFD : adi::LINE_CFD);
        // one factor store per direction: the U entries of a direction's
        // matrix stay from one pass to the next
        for (int d = 0; d < 2; ++d) {
            const Plan* pl = d == 0 ? &pb.px : &pb.py;
            L.fs_off[d] = cur;
            cur += ((size_t)pl->dnlp * pl->dnwin * pl->drows * nv * pb.esz + 255) / 256 * 256;
        }
    }
    L.dc_off = cur;
    if (p.sweeps == 0) cur += 256;
    L.red_off = cur;
    cur += 3 * kRedBlocks * sizeof(double);
    L.chk_off = cur;
    cur += (2 * kRedBlocks + 4) * sizeof(double) + 224;
    L.total = cur;
    return L;
}

// Window margin of the direct solves (slots): the decay of the line
// inverse at the largest (a c / h)^2, to 1e-17 (FP64) or 1e-9 (FP32) of its
// peak.
int direct_margin_of(const adi_params& p) {
    const double ac = 0.5 * p.dt * p.c_max / p.h;
    const int m = p.method == ADI_MFD ? adi::direct::MFD : adi::direct::CFD;
    return adi::direct::direct_margin(m, ac * ac, p.dtype == ADI_FP64 ? 1e-17 : 1e-9);
}

// Windows of the direct solves along one direction: enough windows for
// about 2^18 threads, 2^17 for mimetic FP64 (measured best of 2^17..2^20 on
// 4096^2 lines), each keeping at least twice its margin.
void direct_plan(Plan& pl, const adi_params& p) {
    const int m = p.method == ADI_MFD ? adi::direct::MFD : adi::direct::CFD;
    const int ns = pl.n - adi::direct::direct_smin(m) + 1;
    pl.dH = direct_margin_of(p);
    pl.dnlp = (pl.nlines + 63) / 64 * 64;
    const int target = m == adi::direct::MFD && p.dtype == ADI_FP64 ? 1 << 17 : 1 << 18;
    const int want = std::max(1, target / pl.dnlp);
    int S = std::max({2 * pl.dH, 16, (ns + want - 1) / want});
    pl.dS = std::min(S, ns);
    // the end windows keep H + 4 slots: short chains for the wide band,
    // and the next window starts inside the interior rows
    pl.dSe = pl.dH + 4;
    pl.dnwin = adi::direct::direct_nwin(m, pl.n, pl.dS, pl.dSe);
    pl.drows = adi::direct::direct_rows(m, pl.n, pl.dS, pl.dSe, pl.dH);
    adi::direct::narrow_range(m, pl.n, pl.dS, pl.dSe, pl.dH, pl.dwa, pl.dwb);
}

int validate(const adi_params* p) {
    if (!p) return fail(ADI_EINVAL, "params is NULL");
    if (p->struct_size != sizeof(adi_params))
        return fail(ADI_EINVAL, "struct_size %u != %zu", p->struct_size, sizeof(adi_params));
    if (p->method != ADI_CFD && p->method != ADI_MFD) return fail(ADI_EINVAL, "unknown method %d", p->method);
    if (p->dtype != ADI_FP32 && p->dtype != ADI_FP64 && p->dtype != ADI_FP32C)
        return fail(ADI_EINVAL, "unknown dtype %d", p->dtype);
    if (p->order != 0 && p->order != 1)
        return fail(ADI_EINVAL, "order must be 0 (x-implicit stage first) or 1 (y-implicit first)");
    if (p->nx < 8 || p->ny < 8) return fail(ADI_EINVAL, "nx, ny must be >= 8 (got %d, %d)", p->nx, p->ny);
    if (p->nx > (1 << 20) || p->ny > (1 << 20)) return fail(ADI_EINVAL, "grid too large");
    if (p->sweeps != 0 && (p->sweeps < 2 || p->sweeps > 16 || (p->sweeps & 1)))
        return fail(ADI_EINVAL, "sweeps must be 0 (direct solves) or even and in [2, 16] (got %d)", p->sweeps);
    if (p->sweeps == 0 && p->dtype == ADI_FP32C)
        return fail(ADI_EINVAL, "direct solves (sweeps 0) run in FP32 or FP64, not the compensated mode");
    if (!(p->h > 0.0) || !std::isfinite(p->h)) return fail(ADI_EINVAL, "h must be positive");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(ADI_EINVAL, "dt must be positive");
    if (!(p->c_max > 0.0) || !std::isfinite(p->c_max)) return fail(ADI_EINVAL, "c_max must be positive");
    if (!std::isfinite(p->t0)) return fail(ADI_EINVAL, "t0 must be finite");
    if (!(p->kappa0 > 0.0) || !(p->rinv0 > 0.0)) return fail(ADI_EINVAL, "kappa0, rinv0 must be positive");
    const double cfl = p->dt * p->c_max / p->h;
    const double lim = p->method == ADI_CFD ? 1.15 : 0.81;
    if (p->sweeps != 0 && !(cfl < lim))
        return fail(ADI_EINVAL, "cfl %.4f at or above the fixed-point limit %.2f of this method", cfl, lim);
    if (p->sweeps == 0 && direct_margin_of(*p) < 0)
        return fail(ADI_EINVAL, "cfl %.4f too large for the windows of the direct solves", cfl);
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
    pb->esz = p.dtype == ADI_FP64 ? 8 : 4;
    pb->nix = p.method == ADI_CFD ? p.nx - 1 : p.nx;
    pb->niy = p.method == ADI_CFD ? p.ny - 1 : p.ny;
    pb->a = 0.5 * p.dt;
    const int64_t padm = 256 / (int64_t)pb->esz;   // 256-byte rows
    const double cfl = p.dt * p.c_max / p.h;
    pb->px = make_plan(p.method, p.dtype, p.nx, pb->niy, p.sweeps, cfl);
    pb->py = make_plan(p.method, p.dtype, p.ny, pb->nix, p.sweeps, cfl);
    if (p.sweeps == 0) {
        direct_plan(pb->px, p);
        direct_plan(pb->py, p);
    } else {
        apply_tuned(pb->px, p.method, p.dtype);
        apply_tuned(pb->py, p.method, p.dtype);
    }
    for (int d = 0; d < 2; ++d) {
        const Plan& pl = d == 0 ? pb->px : pb->py;
        auto& D = pb->d[d];
        D.lm = pl.ver == 3;
        if (D.lm) {
            // rows hold 3 slots past the last one: the wave-per-line kernel reads
            // whole 16-byte chunks from a window start rounded down to the grid
            D.ld = pad_to(pl.ns + 3, padm);
            D.rows_p = D.rows_v = pad_to(pl.nlines + 1, adi::line3_lanes(p.dtype));   // row = line + 1
        } else {
            D.ld = pad_to(pl.nlines, padm);
            D.rows_p = p.method == ADI_CFD ? pl.n - 1 : pl.n;   // interior slots
            D.rows_v = pl.n + 1;
        }
    }
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
    a.gbase = 0;
    a.gstride = 1;
    a.gcount = pl.nwin;
    a.torder = pl.torder;
    return a;
}

// One buffer of the device state: value array plus, for the compensated
// FP32 mode, its low-word array.
template <typename T> struct Buf {
    T* hi;
    T* lo;
    int64_t ld;
};

template <typename T> Buf<T> nolo(const Buf<T>& b) { return Buf<T>{b.hi, nullptr, b.ld}; }

template <typename T> Buf<T> pres(const adi_problem* pb, int d) {
    const auto& D = pb->d[d];
    return {(T*)D.P, (T*)D.Plo, D.ld};
}
template <typename T> Buf<T> vel(const adi_problem* pb, int d, int i) {
    const auto& D = pb->d[d];
    return {(T*)D.V[i], (T*)D.Vlo[i], D.ld};
}
// Pressure hand-off written by the passes along `from` for the passes along
// the other direction, in that direction's layout: line-major target (rows
// indexed by line + 1): element s * ld + (q + 1), i.e. (s - 1) * ld + q from
// base + ld + 1 (utrans 0); slot-major target: element q * ld + (s - 1)
// (utrans 1).
template <typename T> Buf<T> pres_out(const adi_problem* pb, int from, int& utrans) {
    const auto& O = pb->d[1 - from];
    utrans = O.lm ? 0 : 1;
    return O.lm ? Buf<T>{(T*)O.P + O.ld + 1, O.Plo ? (T*)O.Plo + O.ld + 1 : nullptr, O.ld}
                : Buf<T>{(T*)O.P, (T*)O.Plo, O.ld};
}

// Copies between the caller's natural arrays (row = y) and the arrays of
// direction d: pressure-type (interior points) and velocity-type (V for
// d = 0: interior rows, all x nodes; W for d = 1: interior columns, all y
// nodes), scaled by `scale`.
template <typename T>
hipError_t pres_to_dir(const adi_problem* pb, int d, T* dst, const T* U, int64_t ldU, T scale, hipStream_t st) {
    const auto& D = pb->d[d];
    const T* src = U + ldU + 1;
    T* lmd = dst + D.ld + 1;   // line-major: row q + 1, slot 1 first
    if (d == 0)
        return D.lm ? adi::launch_scaled_copy<T>(lmd, D.ld, src, ldU, 1, pb->niy, pb->nix, scale, st)
                    : adi::launch_scaled_copy<T>(dst, D.ld, src, 1, ldU, pb->nix, pb->niy, scale, st);
    return D.lm ? adi::launch_scaled_copy<T>(lmd, D.ld, src, 1, ldU, pb->nix, pb->niy, scale, st)
                : adi::launch_scaled_copy<T>(dst, D.ld, src, ldU, 1, pb->niy, pb->nix, scale, st);
}
template <typename T>
hipError_t vel_to_dir(const adi_problem* pb, int d, T* dst, const T* X, int64_t ldX, T scale, hipStream_t st) {
    const auto& D = pb->d[d];
    const auto& p = pb->p;
    T* lmd = dst + D.ld;       // line-major: row q + 1
    if (d == 0)
        return D.lm ? adi::launch_scaled_copy<T>(lmd, D.ld, X + ldX, ldX, 1, pb->niy, p.nx + 1, scale, st)
                    : adi::launch_scaled_copy<T>(dst, D.ld, X + ldX, 1, ldX, p.nx + 1, pb->niy, scale, st);
    return D.lm ? adi::launch_scaled_copy<T>(lmd, D.ld, X + 1, 1, ldX, pb->nix, p.ny + 1, scale, st)
                : adi::launch_scaled_copy<T>(dst, D.ld, X + 1, ldX, 1, p.ny + 1, pb->nix, scale, st);
}
template <typename T>
hipError_t vel_from_dir(const adi_problem* pb, int d, T* X, int64_t ldX, const Buf<T>& b, hipStream_t st) {
    const auto& D = pb->d[d];
    const auto& p = pb->p;
    const T* lms = b.hi + D.ld;   // line-major: row q + 1
    if (d == 0)
        return D.lm ? adi::launch_scaled_copy<T>(X + ldX, ldX, lms, D.ld, 1, pb->niy, p.nx + 1, T(1), st, b.lo)
                    : adi::launch_scaled_copy<T>(X + ldX, ldX, b.hi, 1, D.ld, pb->niy, p.nx + 1, T(1), st, b.lo);
    return D.lm ? adi::launch_scaled_copy<T>(X + 1, ldX, lms, 1, D.ld, p.ny + 1, pb->nix, T(1), st, b.lo)
                : adi::launch_scaled_copy<T>(X + 1, ldX, b.hi, D.ld, 1, p.ny + 1, pb->nix, T(1), st, b.lo);
}
template <typename T>
hipError_t zero_lo(const adi_problem* pb, int d, T* lo, bool ptype, hipStream_t st) {
    const auto& D = pb->d[d];
    return adi::launch_fill_zero<T>(lo, D.ld, (int)(ptype ? D.rows_p : D.rows_v), (int)D.ld, st);
}

// Pass along x (dir 0: lines = interior rows) or along y (dir 1: lines =
// interior columns); the materials come from the direction's arrays.
// Per-pass scalars of the wall values and the distributed forcing for step
// m: level 0 (walls at t^m, forcing F^m: the explicit pass of step m and the
// final form of the pass that ended step m - 1), 1 (the intermediate walls
// of step m -> m + 1, forcing F^{m+1}: the first pass of step m), 2 (walls
// at t^{m+1}, forcing F^{m+1}: the second pass).
struct PassScalars {
    double bsc[3] = {0.0, 0.0, 0.0};
    double aFf = 0.0;
};
PassScalars pass_scalars(const adi_problem& pb, int64_t m, int level) {
    PassScalars r;
    const auto& p = pb.p;
    const double tm = p.t0 + (double)m * p.dt, tm1 = tm + p.dt;
    if (pb.fsig.kind) r.aFf = pb.a * signal_at(pb.fsig, level == 0 ? tm : tm1);
    if (pb.bsig.kind) {
        if (level == 1) {
            r.bsc[0] = 0.5 * (signal_at(pb.bsig, tm) + signal_at(pb.bsig, tm1));
            r.bsc[1] = -pb.a * pb.a * signal_at(pb.bsig, tm + 0.5 * p.dt);
            r.bsc[2] = pb.fsig.kind ? 0.5 * pb.a * (signal_at(pb.fsig, tm) - signal_at(pb.fsig, tm1)) : 0.0;
        } else {
            r.bsc[0] = signal_at(pb.bsig, level == 0 ? tm : tm1);
        }
    }
    return r;
}

template <typename T>
adi::PassDesc<T> make_pass(const adi_problem* pb, int dir, const Buf<T>& uin, const Buf<T>& vin,
                           const Buf<T>& vout, const Buf<T>& uout, int utrans, T f, const T* aFtab, int mode,
                           const PassScalars& ps = PassScalars()) {
    const auto& p = pb->p;
    const Plan& pl = dir == 0 ? pb->px : pb->py;
    const auto& D = pb->d[dir];
    adi::PassDesc<T> d{};
    auto& a = d.a;
    a = base_args<T>(*pb, pl, D.coef);
    a.uin = uin.hi; a.uin_lo = uin.lo; a.uin_ld = uin.ld;
    a.vin = vin.hi; a.vin_lo = vin.lo; a.vin_ld = vin.ld;
    a.ak = (const T*)D.K; a.ak_ld = D.ld;
    a.ar = (const T*)D.R; a.ar_ld = D.ld;
    a.vout = vout.hi; a.vout_lo = vout.lo; a.vout_ld = vout.ld;
    a.uout = uout.hi; a.uout_lo = uout.lo; a.uout_ld = uout.ld;
    a.utrans = utrans;
    a.bnd = (const T*)D.BND;
    for (int i = 0; i < 3; ++i) a.bsc[i] = (T)ps.bsc[i];
    a.ff = (const T*)D.FF;
    a.ff_ld = D.ld;
    a.aFf = (T)ps.aFf;
    a.ah = (T)pb->a;
    a.dmpm = pb->dmp0 != 0.0 ? (pb->dmpwalls >> (2 * dir)) & 3 : 0;
    a.dmp0 = (T)pb->dmp0;
    a.dmpiw = pb->dmpw > 0.0 ? (T)(1.0 / pb->dmpw) : T(0);
    // the wave-per-line kernel writes the natural-layout pressure at
    // (s - 1) * ld + (q + 1): its base is one element lower
    if (pl.ver == 3 && utrans == 0) {
        a.uout = uout.hi - 1;
        if (uout.lo) a.uout_lo = uout.lo - 1;
    }
    if (p.src_i >= 0) {
        a.src_q = dir == 0 ? p.src_j - 1 : p.src_i - 1;
        a.src_s = dir == 0 ? p.src_i : p.src_j;
        a.aF = f;
        a.aFtab = mode == adi::LINE_SWEEP ? aFtab : nullptr;
    }
    d.ver = pl.ver;
    d.dir = dir;
    d.cfg = pl.ver == 1 ? pl.cfg : 0;
    d.method = p.method;
    d.mode = mode;
    d.comp = p.dtype == ADI_FP32C;
    return d;
}

}  // namespace

namespace adi {

double source_term(const adi_problem& pb, int64_t m) {
    const auto& p = pb.p;
    if (p.src_i < 0) return 0.0;
    return pb.a * ricker(p, p.t0 + (double)m * p.dt) / (p.h * p.h);
}

template <typename T>
hipError_t launch_pass(const PassDesc<T>& d, hipStream_t st) {
    if (d.ver == 1) return launch_line_pass<T>(d.a, d.method, d.mode, st, d.comp, d.cfg, (d.full() && !d.comp));
    if (d.ver == 2) return launch_line_pass2<T>(d.a, d.method, d.mode, st, d.comp);
    return launch_line_pass3<T>(d.a, d.method, d.mode, st, d.comp, (d.full() && !d.comp));
}

template <typename T>
int run_begin(adi_problem* pb, hipStream_t st) {
    const auto& p = pb->p;
    const bool comp = p.dtype == ADI_FP32C;
    T* U = (T*)pb->U;
    T* V = (T*)pb->V;
    T* W = (T*)pb->W;
    const T f0 = (T)source_term(*pb, pb->step);
    const PassScalars ps = pass_scalars(*pb, pb->step, 0);
    int ut;
    // V -> velocity arrays of the x passes; low words start at zero
    HIP_TRY(vel_to_dir<T>(pb, 0, (T*)pb->d[0].V[pb->vcur], V, pb->ldV, T(1), st), "V in");
    if (comp) HIP_TRY(zero_lo<T>(pb, 0, (T*)pb->d[0].Vlo[pb->vcur], false, st), "zero V low words");
    if (p.order == 0) {
        // explicit y part of stage 1: A and W* of step m
        if (pb->d[1].lm) {
            HIP_TRY(pres_to_dir<T>(pb, 1, (T*)pb->d[1].P, U, pb->ldU, T(1), st), "U in");
            HIP_TRY(vel_to_dir<T>(pb, 1, (T*)pb->d[1].V[pb->wcur], W, pb->ldW, T(1), st), "W in");
            const Buf<T> out = pres_out<T>(pb, 1, ut);
            auto d = make_pass<T>(pb, 1, nolo(pres<T>(pb, 1)), nolo(vel<T>(pb, 1, pb->wcur)), vel<T>(pb, 1, 1 - pb->wcur),
                                  out, ut, f0, nullptr, LINE_EXPLICIT, ps);
            HIP_TRY(launch_pass<T>(d, st), "explicit column pass");
            pb->wcur ^= 1;
        } else {
            const Buf<T> Uu{U + pb->ldU + 1, nullptr, pb->ldU}, Wu{W + 1, nullptr, pb->ldW};
            const Buf<T> out = pres_out<T>(pb, 1, ut);
            auto d = make_pass<T>(pb, 1, Uu, Wu, vel<T>(pb, 1, pb->wcur), out, ut, f0, nullptr, LINE_EXPLICIT, ps);
            HIP_TRY(launch_pass<T>(d, st), "explicit column pass");
        }
    } else {
        // y-implicit stage first: U -> pressure of the x passes, W -> velocity
        // of the y passes, explicit x part of stage 1
        HIP_TRY(pres_to_dir<T>(pb, 0, (T*)pb->d[0].P, U, pb->ldU, T(1), st), "U in");
        HIP_TRY(vel_to_dir<T>(pb, 1, (T*)pb->d[1].V[pb->wcur], W, pb->ldW, T(1), st), "W in");
        if (comp) HIP_TRY(zero_lo<T>(pb, 1, (T*)pb->d[1].Vlo[pb->wcur], false, st), "zero W low words");
        const Buf<T> out = pres_out<T>(pb, 0, ut);
        auto d = make_pass<T>(pb, 0, nolo(pres<T>(pb, 0)), nolo(vel<T>(pb, 0, pb->vcur)), vel<T>(pb, 0, 1 - pb->vcur),
                              out, ut, f0, nullptr, LINE_EXPLICIT, ps);
        HIP_TRY(launch_pass<T>(d, st), "explicit row pass");
        pb->vcur ^= 1;
    }
    pb->ready = true;
    return ADI_OK;
}

template <typename T>
PassDesc<T> run_pass(adi_problem* pb, int64_t s, int half, bool final_pass, const T* aFtab) {
    const bool last = final_pass;
    const T f1 = (T)source_term(*pb, pb->step + s + 1);
    const PassScalars ps = pass_scalars(*pb, pb->step + s, half == 0 ? 1 : 2);
    T* U = (T*)pb->U;
    T* W = (T*)pb->W;
    int ut;
    PassDesc<T> d;
    // dir: the direction of this half step
    const int dir = pb->p.order == 0 ? half : 1 - half;
    int& cur = dir == 0 ? pb->vcur : pb->wcur;
    const Buf<T> uin = pres<T>(pb, dir), vin = vel<T>(pb, dir, cur), vout = vel<T>(pb, dir, 1 - cur);
    if (half == 1 && last) {
        // last pass of the run: U^{m+n} into the caller's array; the
        // velocity into the caller's W directly when the y arrays are
        // slot-major, else through the workspace (copied out by run_end)
        if (dir == 1) {
            const Buf<T> Uu{U + pb->ldU + 1, nullptr, pb->ldU}, Wu{W + 1, nullptr, pb->ldW};
            if (pb->d[1].lm) {
                d = make_pass<T>(pb, 1, uin, vin, vout, Uu, 0, T(0), nullptr, LINE_FINAL, ps);
                cur ^= 1;
            } else {
                d = make_pass<T>(pb, 1, uin, vin, Wu, Uu, 0, T(0), nullptr, LINE_FINAL, ps);
            }
        } else {
            const Buf<T> Ux{U + pb->ldU + 1, nullptr, pb->ldU};
            d = make_pass<T>(pb, 0, uin, vin, vout, Ux, 1, T(0), nullptr, LINE_FINAL, ps);
            cur ^= 1;
        }
        return d;
    }
    // sweeps of this stage, then the explicit part of the next stage
    const Buf<T> out = pres_out<T>(pb, dir, ut);
    d = make_pass<T>(pb, dir, uin, vin, vout, out, ut, f1, aFtab, LINE_SWEEP, ps);
    cur ^= 1;
    return d;
}

template <typename T>
int run_end(adi_problem* pb, hipStream_t st, int64_t nsteps) {
    const auto& p = pb->p;
    T* V = (T*)pb->V;
    T* W = (T*)pb->W;
    // W^{m+n} back to the caller unless the last pass wrote it
    if (p.order == 1 || pb->d[1].lm)
        HIP_TRY(vel_from_dir<T>(pb, 1, W, pb->ldW, vel<T>(pb, 1, pb->wcur), st), "W out");
    HIP_TRY(vel_from_dir<T>(pb, 0, V, pb->ldV, vel<T>(pb, 0, pb->vcur), st), "V out");
    pb->step += nsteps;
    pb->ready = false;
    return ADI_OK;
}

template <typename T>
hipError_t launch_grouped(const PassDesc<T>& d, const GroupArgs<T>& ga, hipStream_t st) {
    if (d.ver == 1) return launch_line_group<T>(ga, d.cfg, d.method, d.mode, st, d.comp, (d.full() && !d.comp));
    if (d.ver == 2) return launch_line_group2<T>(ga, d.method, d.mode, st, d.comp);
    return launch_line_group3<T>(ga, d.method, d.mode, st, d.comp, (d.full() && !d.comp));
}

template hipError_t launch_grouped<float>(const PassDesc<float>&, const GroupArgs<float>&, hipStream_t);
template hipError_t launch_grouped<double>(const PassDesc<double>&, const GroupArgs<double>&, hipStream_t);
template int run_begin<float>(adi_problem*, hipStream_t);
template int run_begin<double>(adi_problem*, hipStream_t);
template PassDesc<float> run_pass<float>(adi_problem*, int64_t, int, bool, const float*);
template PassDesc<double> run_pass<double>(adi_problem*, int64_t, int, bool, const double*);
template int run_end<float>(adi_problem*, hipStream_t, int64_t);
template int run_end<double>(adi_problem*, hipStream_t, int64_t);
template hipError_t launch_pass<float>(const PassDesc<float>&, hipStream_t);
template hipError_t launch_pass<double>(const PassDesc<double>&, hipStream_t);

}  // namespace adi

namespace {

// Device state of the tolerance-tested stages: the per-workgroup change
// partials of one attempt (4 x the largest tile count of the two
// directions), the attempt flags, and the counters of passes decided and
// sweeps used.
constexpr int kMaxAttempts = 8;   // (16 - 2) / 2 + 1: sweeps <= 16, min_sweeps >= 2
struct EpsLayout {
    double* part;
    int* go;
    long long* stats;
};
// (the most tiles any tile shape of the plan's kernel launches: the
// autotuner may change the shape after the buffer exists)
int max_tiles(const Plan& p, int dtype) {
    if (p.ver != 1) return p.nlg * p.nwin;
    int lw = adi::line_lanes(dtype, 0);
    for (int c = 1; c < adi::LINE_NCFG; ++c) lw = std::min(lw, adi::line_lanes(dtype, c));
    return (p.nlines + lw - 1) / lw;
}
size_t eps_tiles(const adi_problem* pb) {
    return (size_t)std::max(max_tiles(pb->px, pb->p.dtype), max_tiles(pb->py, pb->p.dtype));
}
size_t eps_bytes(const adi_problem* pb) { return 4 * eps_tiles(pb) * sizeof(double) + 64 + 2 * sizeof(long long); }
EpsLayout eps_layout(const adi_problem* pb) {
    char* b = (char*)pb->eps_buf;
    const size_t po = 4 * eps_tiles(pb) * sizeof(double);
    return {(double*)b, (int*)(b + po), (long long*)(b + po + 64)};
}
static_assert((kMaxAttempts + 1) * sizeof(int) <= 64, "flags");

// One tolerance-tested pass (Algorithms 3 and 4): attempts with K = kmin,
// kmin + 2, .. sweeps sweeps, each recomputing the pass from its unchanged
// inputs and running only while the earlier ones have not converged; the
// decisions stay on the device.  Each attempt of a multi-window plan has
// the windows of its own K (the margin grows with K).
template <typename T>
hipError_t launch_tested(adi_problem* pb, adi::PassDesc<T> d) {
    const auto& p = pb->p;
    const int kmin = pb->eps_kmin, kmax = p.sweeps;
    const int J = (kmax - kmin) / 2 + 1;
    const EpsLayout L = eps_layout(pb);
    const Plan& pl = d.dir == 0 ? pb->px : pb->py;
    const double cfl = p.dt * p.c_max / p.h;
    hipError_t e = hipSuccess;
    for (int j = 0; j < J && e == hipSuccess; ++j) {
        const int K = kmin + 2 * j;
        d.a.sweeps = K;
        if (pl.ver == 3) {
            const Plan pk = make_plan(p.method, p.dtype, pl.n, pl.nlines, K, cfl);
            d.a.H = pk.H;
            d.a.S = pk.S;
            d.a.nwin = pk.nwin;
        }
        d.a.eps_part = L.part;
        d.a.eps_go = L.go + j;
        const int nb = d.a.nlg * d.a.nwin;
        e = adi::launch_pass<T>(d, pb->st);
        // the last attempt decides by itself (the check before it counted it)
        if (e == hipSuccess && (j < J - 1 || J == 1))
            e = adi::launch_eps_check(L.part, nb, L.go, j, J, pb->eps, K, kmin, kmax, L.stats, pb->st);
    }
    return e;
}

// A line pass of the direct solves (sweeps 0): the same hand-off buffers as
// the sweep pass it replaces, read through (line, slot) strides.  Along a
// line-major direction element (q, s) is at (q + 1) ld + s; along a
// slot-major one pressure-type arrays hold (s - 1) ld + q and velocity-type
// arrays s ld + q; the pressure output is written transposed (utrans 1:
// q ld + s - 1) or slot-major ((s - 1) ld + q).
template <typename T>
hipError_t launch_direct_pass(adi_problem* pb, const adi::PassDesc<T>& d) {
    const auto& a = d.a;
    const Plan& pl = d.dir == 0 ? pb->px : pb->py;
    const bool lm = pb->d[d.dir].lm;
    adi::DirectArgs<T> g{};
    auto pres_in = [&](const T* base, int64_t ld, const T*& o, int64_t& l, int64_t& s) {
        if (!base) { o = nullptr; l = s = 0; return; }
        if (lm) { o = base + ld; l = ld; s = 1; }
        else { o = base - ld; l = 1; s = ld; }
    };
    auto vel_at = [&](const T* base, int64_t ld, const T*& o, int64_t& l, int64_t& s) {
        if (!base) { o = nullptr; l = s = 0; return; }
        if (lm) { o = base + ld; l = ld; s = 1; }
        else { o = base; l = 1; s = ld; }
    };
    pres_in(a.uin, a.uin_ld, g.a, g.a_l, g.a_s);
    pres_in(a.ak, a.ak_ld, g.k, g.k_l, g.k_s);
    vel_at(a.vin, a.vin_ld, g.b, g.b_l, g.b_s);
    vel_at(a.ar, a.ar_ld, g.r, g.r_l, g.r_s);
    // constant materials: the two values bind_materials stored, strides 0
    if (!g.k) g.k = (const T*)pb->dconst;
    if (!g.r) g.r = (const T*)pb->dconst + 1;
    const T* vo;
    vel_at(a.vout, a.vout_ld, vo, g.v_l, g.v_s);
    g.v = const_cast<T*>(vo);
    // the wave-per-line pass addresses a line-major pressure target one
    // element lower; undo that shift
    T* uo = a.uout + (pl.ver == 3 && a.utrans == 0 ? 1 : 0);
    if (a.utrans) { g.u = uo - 1; g.u_l = a.uout_ld; g.u_s = 1; }
    else { g.u = uo - a.uout_ld; g.u_l = 1; g.u_s = a.uout_ld; }
    g.fs = (T*)pb->dfs[d.dir];
    g.inv_h = a.inv_h;
    g.aF = a.aF;
    g.nlines = a.nlines;
    g.nlp = pl.dnlp;
    g.n = a.n;
    g.S = pl.dS;
    g.Se = pl.dSe;
    g.H = pl.dH;
    g.nwin = pl.dnwin;
    g.drows = pl.drows;
    g.mode = d.mode == adi::LINE_FINAL ? 1 : 0;
    g.src_q = d.mode == adi::LINE_FINAL ? -1 : a.src_q;
    g.src_s = a.src_s;
    // windows before dwa and after dwb reach the closure rows: they run on
    // the second stream beside the interior windows, each launch with its
    // own part of the factor store
    const int nv_wide = adi::direct_values_per_row(d.method), nv_narrow = 4;
    T* fs = (T*)pb->dfs[d.dir];
    const bool ustored = pb->dfs_u[d.dir];
    // windows [wbase, wbase + n1) and [wbase2, wbase2 + n2) in one launch
    auto go = [&](int wbase, int n1, int wbase2, int n2, bool wide, hipStream_t s) {
        g.wbase = wbase;
        g.wsplit = n1;
        g.wbase2 = wbase2;
        g.wcount = n1 + n2;
        g.nthr = (int64_t)pl.dnlp * g.wcount;
        g.fs = fs;
        fs += g.nthr * pl.drows * (wide ? nv_wide : nv_narrow);
        return adi::launch_direct<T>(g, d.method, wide, ustored, s);
    };
    hipError_t e;
    if (pl.dwa > pl.dwb) {
        e = go(0, pl.dnwin, 0, 0, true, pb->st);
    } else {
        e = hipEventRecord(pb->dev_in, pb->st);
        if (e == hipSuccess) e = hipStreamWaitEvent(pb->dst2, pb->dev_in, 0);
        if (e == hipSuccess) e = go(0, pl.dwa, pl.dwb + 1, pl.dnwin - pl.dwb - 1, true, pb->dst2);
        if (e == hipSuccess) e = hipEventRecord(pb->dev_out, pb->dst2);
        if (e == hipSuccess) e = go(pl.dwa, pl.dwb - pl.dwa + 1, 0, 0, false, pb->st);
        if (e == hipSuccess) e = hipStreamWaitEvent(pb->st, pb->dev_out, 0);
    }
    // later passes along these lines (stream-ordered after this one) find
    // the U entries stored
    if (e == hipSuccess) pb->dfs_u[d.dir] = true;
    return e;
}

// rows x cols of U, V, W
void state_shapes(const adi_params& p, int64_t rows[3], int64_t cols[3]) {
    const bool cfd = p.method == ADI_CFD;
    rows[0] = cfd ? p.ny + 1 : p.ny + 2; cols[0] = cfd ? p.nx + 1 : p.nx + 2;
    rows[1] = cfd ? p.ny + 1 : p.ny + 2; cols[1] = p.nx + 1;
    rows[2] = p.ny + 1;                  cols[2] = cfd ? p.nx + 1 : p.nx + 2;
}

// Health check, first level: per block, whether x[0..n) holds a non-finite
// value and its largest finite magnitude, into part[2 b], part[2 b + 1].
template <typename T>
__global__ void __launch_bounds__(256) health_kernel(const T* __restrict__ x, int64_t n, double* part) {
    __shared__ double red[256];
    __shared__ int bad[256];
    double m = 0.0;
    int nf = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = (double)x[i];
        if (isfinite(v)) m = fmax(m, fabs(v));
        else nf = 1;
    }
    red[threadIdx.x] = m;
    bad[threadIdx.x] = nf;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            bad[threadIdx.x] |= bad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = bad[0] ? 1.0 : 0.0;
        part[2 * blockIdx.x + 1] = red[0];
    }
}

// Second level: the partials into the running state (sticky flag, largest
// magnitude, first step found non-finite, step of this check).
__global__ void __launch_bounds__(256) health_merge_kernel(const double* part, int nb, double* state, double step) {
    __shared__ double red[256];
    __shared__ double bad[256];
    double m = 0.0, f = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        f = fmax(f, part[2 * i]);
        m = fmax(m, part[2 * i + 1]);
    }
    red[threadIdx.x] = m;
    bad[threadIdx.x] = f;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            bad[threadIdx.x] = fmax(bad[threadIdx.x], bad[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (bad[0] > 0.0 && state[0] == 0.0) state[2] = step + 1.0;
        state[0] = fmax(state[0], bad[0]);
        state[1] = fmax(state[1], red[0]);
        state[3] = step;
    }
}

template <typename T>
hipError_t launch_health(adi_problem* pb, const T* x, int64_t n, int64_t step) {
    double* part = (double*)(pb->ws + layout(*pb).chk_off);
    hipLaunchKernelGGL(health_kernel<T>, dim3(kRedBlocks), dim3(256), 0, pb->st, x, n, part);
    hipLaunchKernelGGL(health_merge_kernel, dim3(1), dim3(256), 0, pb->st, (const double*)part, kRedBlocks,
                       part + kChkState, (double)step);
    return hipGetLastError();
}

// The state of a ready problem into U, V, W (the bound leading dimensions):
// the pass that ended the last step is run again in its final form.  Its
// inputs are still in the workspace (that pass wrote the other ping-pong
// buffer and the other direction's hand-off); it writes U^m and its
// direction's velocity instead of the next step's hand-off, the velocity
// into the spare buffer (or straight into the target for slot-major column
// passes).  The other velocity is current in its ping-pong buffer.
template <typename T>
int materialize_ready(adi_problem* pb, T* U, T* V, T* W) {
    const int dl = last_dir(pb->p), o = 1 - dl;
    const int cur = dl == 0 ? pb->vcur : pb->wcur;
    const auto& D = pb->d[dl];
    const Buf<T> uin = pres<T>(pb, dl), vin = vel<T>(pb, dl, 1 - cur);
    const Buf<T> Uu{U + pb->ldU + 1, nullptr, pb->ldU};
    const Buf<T> spare{(T*)D.Vs, (T*)D.Vslo, D.ld};
    const bool straight = dl == 1 && !D.lm;
    const Buf<T> vout = straight ? Buf<T>{W + 1, nullptr, pb->ldW} : spare;
    const auto d = make_pass<T>(pb, dl, uin, vin, vout, Uu, dl == 0 ? 1 : 0, T(0), nullptr, adi::LINE_FINAL,
                                pass_scalars(*pb, pb->step, 0));
    if (pb->p.sweeps == 0)
        HIP_TRY(launch_direct_pass<T>(pb, d), "final direct pass");
    else
        HIP_TRY(adi::launch_pass<T>(d, pb->st), "final line pass");
    if (!straight)
        HIP_TRY(vel_from_dir<T>(pb, dl, dl == 0 ? V : W, dl == 0 ? pb->ldV : pb->ldW, spare, pb->st), "velocity out");
    const int co = o == 0 ? pb->vcur : pb->wcur;
    HIP_TRY(vel_from_dir<T>(pb, o, o == 0 ? V : W, o == 0 ? pb->ldV : pb->ldW, vel<T>(pb, o, co), pb->st),
            "velocity out");
    return ADI_OK;
}

template <typename T>
int run_impl(adi_problem* pb, int64_t nsteps) {
    const bool tested = pb->eps > 0.0;
    int rc = ADI_OK;
    if (tested && pb->ready) {
        // tolerance-tested runs start from and end in the bound arrays
        rc = materialize_ready<T>(pb, (T*)pb->U, (T*)pb->V, (T*)pb->W);
        if (rc != ADI_OK) return rc;
        pb->ready = false;
    }
    if (!pb->ready) rc = adi::run_begin<T>(pb, pb->st);
    if (rc != ADI_OK) return rc;
    for (int64_t s = 0; s < nsteps; ++s) {
        const bool fin = tested && s == nsteps - 1;
        for (int half = 0; half < 2; ++half) {
            const auto d = adi::run_pass<T>(pb, s, half, fin && half == 1, nullptr);
            if (pb->p.sweeps == 0)
                HIP_TRY(launch_direct_pass<T>(pb, d), half == 0 ? "first direct pass" : "second direct pass");
            else if (tested)
                HIP_TRY(launch_tested<T>(pb, d), half == 0 ? "first line pass" : "second line pass");
            else
                HIP_TRY(adi::launch_pass<T>(d, pb->st), half == 0 ? "first line pass" : "second line pass");
        }
        const int64_t m = pb->step + s + 1;
        if (pb->chk_every > 0 && m % pb->chk_every == 0) {
            // the pressure of the new level: the hand-off the step left for
            // the next one, or U itself after a final pass
            if (fin) {
                int64_t rows[3], cols[3];
                state_shapes(pb->p, rows, cols);
                HIP_TRY(launch_health<T>(pb, (const T*)pb->U, (rows[0] - 1) * pb->ldU + cols[0], m), "health check");
            } else {
                const auto& D = pb->d[1 - last_dir(pb->p)];
                HIP_TRY(launch_health<T>(pb, (const T*)D.P, D.rows_p * D.ld, m), "health check");
            }
        }
    }
    if (tested) return adi::run_end<T>(pb, pb->st, nsteps);
    adi::run_advance(pb, nsteps);
    return ADI_OK;
}

// Factor tables of a direction's single-window compact plan into its coef
// region (nothing for other plans); host (6 LINE_WS values) must live until
// the copy has run.
template <typename T>
int upload_tables(adi_problem* pb, int d, T* host, hipStream_t st) {
    const Plan& pl = d == 0 ? pb->px : pb->py;
    if (pb->p.method != ADI_CFD || pl.ver != 1) return ADI_OK;
    double t64[6 * adi::LINE_WS];
    build_tables(pl, t64);
    const int cnt = 6 * adi::line_ws(pl.cfg);
    for (int i = 0; i < cnt; ++i) host[i] = (T)t64[i];
    HIP_TRY(hipMemcpyAsync(pb->d[d].coef, host, cnt * sizeof(T), hipMemcpyHostToDevice, st), "factor tables");
    return ADI_OK;
}

struct EventPair {
    hipEvent_t e[2] = {nullptr, nullptr};
    ~EventPair() {
        for (auto x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// Times every launch choice of each direction's sweep pass on the problem's
// own data and keeps the fastest (adi_autotune).  The state goes to the
// bound arrays first; the timed passes advance a copy of it in the
// workspace, and the next run starts again from the bound arrays.
template <typename T>
int autotune_impl(adi_problem* pb, int reps, double* pass_us) {
    const auto& p = pb->p;
    hipStream_t st = pb->st;
    if (pb->ready) {
        const int rc = materialize_ready<T>(pb, (T*)pb->U, (T*)pb->V, (T*)pb->W);
        if (rc != ADI_OK) return rc;
        pb->ready = false;
    }
    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.e[0]), "tuning events");
    HIP_TRY(hipEventCreate(&ev.e[1]), "tuning events");
    int rc = adi::run_begin<T>(pb, st);
    if (rc != ADI_OK) return rc;
    static thread_local T host[6 * adi::LINE_WS];
    std::string arch;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        arch = device_arch();
    }
    for (int d = 0; d < 2; ++d) {
        Plan& pl = d == 0 ? pb->px : pb->py;
        pass_us[d] = 0.0;
        int c[8];
        const int nc = plan_choices(pl, c);
        if (nc == 0) continue;
        const int half = p.order == 0 ? d : 1 - d;
        auto pass = [&]() -> int {
            const auto desc = adi::run_pass<T>(pb, 0, half, false, nullptr);
            HIP_TRY(adi::launch_pass<T>(desc, st), "tuning pass");
            return ADI_OK;
        };
        const Plan dflt = make_plan(p.method, p.dtype, pl.n, pl.nlines, p.sweeps, p.dt * p.c_max / p.h);
        double t[8];
        for (int i = 0; i < nc; ++i) t[i] = 1e300;
        // three rounds over the choices, the best time of each kept
        for (int round = 0; round < 3; ++round)
            for (int i = 0; i < nc; ++i) {
                apply_choice(pl, p.dtype, c[i]);
                if ((rc = upload_tables<T>(pb, d, host, st)) != ADI_OK) return rc;
                HIP_TRY(hipStreamSynchronize(st), "factor tables");   // host is reused
                for (int w = 0; w < 2; ++w)
                    if ((rc = pass()) != ADI_OK) return rc;
                HIP_TRY(hipEventRecord(ev.e[0], st), "tuning events");
                for (int r = 0; r < reps; ++r)
                    if ((rc = pass()) != ADI_OK) return rc;
                HIP_TRY(hipEventRecord(ev.e[1], st), "tuning events");
                HIP_TRY(hipEventSynchronize(ev.e[1]), "tuning events");
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]), "tuning events");
                t[i] = std::min(t[i], 1e3 * ms / reps);
            }
        // the default choice stays unless another is more than 1% faster
        int best = 0;
        for (int i = 0; i < nc; ++i)
            if (c[i] == plan_choice(dflt)) best = i;
        for (int i = 0; i < nc; ++i)
            if (t[i] < 0.99 * t[best]) best = i;
        apply_choice(pl, p.dtype, c[best]);
        pl.tuned = true;
        if ((rc = upload_tables<T>(pb, d, host, st)) != ADI_OK) return rc;
        HIP_TRY(hipStreamSynchronize(st), "tuning");
        pass_us[d] = t[best];
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();
        g_tune[tune_key(arch, p.method, p.dtype, pl)] = c[best];
    }
    HIP_TRY(hipStreamSynchronize(st), "tuning");
    pb->ready = false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return tune_save();
}

// ADI_ENUMERIC when the health check has seen a non-finite value or a
// magnitude above its bound (after the problem's stream has drained).
int health_status(adi_problem* pb) {
    if (pb->chk_every <= 0) return ADI_OK;
    double st[4];
    HIP_TRY(hipMemcpy(st, (double*)(pb->ws + layout(*pb).chk_off) + kChkState, sizeof(st), hipMemcpyDeviceToHost),
            "health check state");
    if (st[0] > 0.0)
        return fail(ADI_ENUMERIC, "non-finite values in the state at step %lld", (long long)st[2] - 1);
    if (pb->chk_max > 0.0 && st[1] > pb->chk_max)
        return fail(ADI_ENUMERIC, "largest pressure magnitude %.6g above the bound %.6g (checked at step %lld)", st[1],
                    pb->chk_max, (long long)st[3]);
    return ADI_OK;
}


}  // namespace

namespace adi {

int materialize(adi_problem* pb, void* U, void* V, void* W) {
    if (pb->ready)
        return pb->p.dtype == ADI_FP64 ? materialize_ready<double>(pb, (double*)U, (double*)V, (double*)W)
                                       : materialize_ready<float>(pb, (float*)U, (float*)V, (float*)W);
    int64_t rows[3], cols[3];
    state_shapes(pb->p, rows, cols);
    void* dst[3] = {U, V, W};
    const void* src[3] = {pb->U, pb->V, pb->W};
    const int64_t ld[3] = {pb->ldU, pb->ldV, pb->ldW};
    for (int i = 0; i < 3; ++i)
        if (dst[i] != src[i])
            HIP_TRY(hipMemcpy2DAsync(dst[i], ld[i] * pb->esz, src[i], ld[i] * pb->esz, cols[i] * pb->esz, rows[i],
                                     hipMemcpyDeviceToDevice, pb->st),
                    "state copy");
    return ADI_OK;
}

}  // namespace adi

namespace {

__global__ void __launch_bounds__(256) clear_kernel(uint4* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Per-block maxima of x[0..n) (non-negative values) into out[blockIdx.x].
template <typename T>
__global__ void __launch_bounds__(256) block_max_kernel(const T* __restrict__ x, int64_t n, double* out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        m = fmax(m, (double)x[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Pressure coordinate of index k along a direction of n cells.
double pcoord(int method, int n, double h, int k) {
    if (method == ADI_CFD) return k * h;
    return k == 0 ? 0.0 : (k == n + 1 ? n * h : (k - 0.5) * h);
}

// Wall coefficients of the time-dependent Dirichlet data (adi_set_boundary),
// per direction d and line q (interior index l = q + 1 across the lines),
// at both ends: the wall value Ub, c^2 times its three-point second
// difference along the wall (across the lines), and the forcing field's
// value there.  Read from the bound U, the materials and the forcing field
// (wall rows and columns only), computed in FP64, stored in the direction's
// BND region.
template <typename T>
int wall_coefficients(adi_problem* pb, const T* K, const T* Rv, const T* Rw, int64_t ldK, int64_t ldRv,
                      int64_t ldRw) {
    const auto& p = pb->p;
    hipStream_t st = pb->st;
    HIP_TRY(hipStreamSynchronize(st), "wall data");
    const int m = p.method;
    const int ru = m == ADI_CFD ? p.ny + 1 : p.ny + 2, cu = m == ADI_CFD ? p.nx + 1 : p.nx + 2;
    // column c (all rows) / row r (all columns) of a device array
    auto col = [&](const T* a, int64_t ld, int rows, int c, std::vector<double>& out) -> hipError_t {
        std::vector<T> tmp(rows);
        out.assign(rows, 0.0);
        const hipError_t e = hipMemcpy2D(tmp.data(), sizeof(T), a + c, ld * sizeof(T), sizeof(T), rows,
                                         hipMemcpyDeviceToHost);
        for (int i = 0; i < rows; ++i) out[i] = (double)tmp[i];
        return e;
    };
    auto row = [&](const T* a, int64_t ld, int cols, int r, std::vector<double>& out) -> hipError_t {
        std::vector<T> tmp(cols);
        out.assign(cols, 0.0);
        const hipError_t e = hipMemcpy(tmp.data(), a + (int64_t)r * ld, cols * sizeof(T), hipMemcpyDeviceToHost);
        for (int i = 0; i < cols; ++i) out[i] = (double)tmp[i];
        return e;
    };
    const T* U = (const T*)pb->U;
    const T* F = (const T*)pb->fF;
    for (int d = 0; d < 2; ++d) {
        const int nl = d == 0 ? pb->niy : pb->nix;           // lines
        const int na = d == 0 ? p.ny : p.nx;                 // cells across the lines (along the walls)
        const int ends[2] = {0, d == 0 ? cu - 1 : ru - 1};   // wall index along the lines
        std::vector<double> coef((size_t)6 * nl, 0.0);
        for (int e = 0; e < 2; ++e) {
            std::vector<double> ub, kb, rb, fb;
            const int w = ends[e];
            const int wv = (e && m == ADI_MFD) ? w - 1 : w;  // the velocity point at the wall
            if (d == 0) {
                HIP_TRY(col(U, pb->ldU, ru, w, ub), "wall data");
                if (K) HIP_TRY(col(K, ldK, ru, w, kb), "wall data");
                if (Rv) HIP_TRY(col(Rv, ldRv, ru, wv, rb), "wall data");
                if (F) HIP_TRY(col(F, pb->fF_ld, ru, w, fb), "wall data");
            } else {
                HIP_TRY(row(U, pb->ldU, cu, w, ub), "wall data");
                if (K) HIP_TRY(row(K, ldK, cu, w, kb), "wall data");
                if (Rw) HIP_TRY(row(Rw, ldRw, cu, wv, rb), "wall data");
                if (F) HIP_TRY(row(F, pb->fF_ld, cu, w, fb), "wall data");
            }
            for (int q = 0; q < nl; ++q) {
                const int l = q + 1;
                const double ym = pcoord(m, na, p.h, l - 1), y0 = pcoord(m, na, p.h, l), yp = pcoord(m, na, p.h, l + 1);
                const double dll = 2.0 * ((ub[l + 1] - ub[l]) / (yp - y0) - (ub[l] - ub[l - 1]) / (y0 - ym)) / (yp - ym);
                const double c2 = (K ? kb[l] : p.kappa0) * (rb.empty() ? p.rinv0 : rb[l]);
                coef[(size_t)6 * q + 3 * e] = ub[l];
                coef[(size_t)6 * q + 3 * e + 1] = c2 * dll;
                coef[(size_t)6 * q + 3 * e + 2] = F ? fb[l] : 0.0;
            }
        }
        std::vector<T> ct(coef.begin(), coef.end());
        HIP_TRY(hipMemcpy(pb->d[d].BND, ct.data(), ct.size() * sizeof(T), hipMemcpyHostToDevice), "wall coefficients");
    }
    return ADI_OK;
}

template <typename T>
int bind_materials(adi_problem* pb, const T* K, const T* Rv, const T* Rw, int64_t ldK, int64_t ldRv, int64_t ldRw) {
    const auto& p = pb->p;
    hipStream_t st = pb->st;
    const T a = (T)pb->a;
    // the workspace starts zeroed: line-major arrays keep zeros on the
    // boundary slots and on the padding lines
    hipLaunchKernelGGL(clear_kernel, dim3((unsigned)std::min<size_t>(4096, (pb->ws_bytes / 16 + 255) / 256)),
                       dim3(256), 0, st, (uint4*)pb->ws, pb->ws_bytes / 16);
    HIP_TRY(hipGetLastError(), "workspace clear");
    // factor tables of the compact single-window kernel (the multi-window
    // kernel uses compile-time constants); the host copies live until the
    // synchronisation below
    T tab[2][6 * adi::LINE_WS];
    for (int d = 0; d < 2; ++d) {
        const int rc = upload_tables<T>(pb, d, tab[d], st);
        if (rc != ADI_OK) return rc;
    }
    // distributed forcing in both directions' layouts
    if (pb->fsig.kind)
        for (int d = 0; d < 2; ++d)
            HIP_TRY(pres_to_dir<T>(pb, d, (T*)pb->d[d].FF, (const T*)pb->fF, pb->fF_ld, T(1), st), "forcing field");
    if (pb->bsig.kind) {
        const int rc = wall_coefficients<T>(pb, K, Rv, Rw, ldK, ldRv, ldRw);
        if (rc != ADI_OK) return rc;
    }
    const T dconst[2] = {(T)(pb->a * p.kappa0), (T)(pb->a * p.rinv0)};
    if (pb->dconst)
        HIP_TRY(hipMemcpyAsync(pb->dconst, dconst, sizeof(dconst), hipMemcpyHostToDevice, st), "constant materials");
    for (int d = 0; d < 2; ++d) {
        if (K) HIP_TRY(pres_to_dir<T>(pb, d, (T*)pb->d[d].K, K, ldK, a, st), "a kappa");
        const T* R = d == 0 ? Rv : Rw;
        if (R) HIP_TRY(vel_to_dir<T>(pb, d, (T*)pb->d[d].R, R, d == 0 ? ldRv : ldRw, a, st), "a / rho");
    }
    // The step size was validated, and the margins of the direct solves
    // planned, for c_max: the bound materials must not exceed it.  Largest
    // a kappa and a / rho over the interior points the passes read.
    {
        double* part = (double*)(pb->ws + layout(*pb).red_off);
        const void* arr[3] = {pb->d[0].K, pb->d[0].R, pb->d[1].R};
        const int64_t n[3] = {pb->d[0].rows_p * pb->d[0].ld, pb->d[0].rows_v * pb->d[0].ld,
                              pb->d[1].rows_v * pb->d[1].ld};
        for (int i = 0; i < 3; ++i)
            if (arr[i]) {
                hipLaunchKernelGGL(block_max_kernel<T>, dim3(kRedBlocks), dim3(256), 0, st, (const T*)arr[i], n[i],
                                   part + i * kRedBlocks);
                HIP_TRY(hipGetLastError(), "material check");
            }
        double host[3 * kRedBlocks];
        HIP_TRY(hipMemcpyAsync(host, part, sizeof(host), hipMemcpyDeviceToHost, st), "material check");
        HIP_TRY(hipStreamSynchronize(st), "material check");
        double mx[3] = {pb->a * p.kappa0, pb->a * p.rinv0, pb->a * p.rinv0};
        for (int i = 0; i < 3; ++i)
            if (arr[i]) {
                mx[i] = 0.0;
                for (int b = 0; b < kRedBlocks; ++b) mx[i] = std::max(mx[i], host[i * kRedBlocks + b]);
            }
        const double c2 = mx[0] * std::max(mx[1], mx[2]) / (pb->a * pb->a);
        if (!(c2 <= p.c_max * p.c_max * (1.0 + 1e-5)))
            return fail(ADI_EINVAL, "max kappa * max 1/rho = %.6g exceeds c_max^2 = %.6g", c2, p.c_max * p.c_max);
    }
    HIP_TRY(hipStreamSynchronize(st), "bind sync");
    return ADI_OK;
}

// Leading dimensions of U, V, W, K, Rv, Rw: ld[i] when given and non-zero
// (at least the row length), else the row length.
int leading_dims(const adi_params& p, const int64_t* ld, int64_t l[6]) {
    const bool cfd = p.method == ADI_CFD;
    const int64_t colsU = cfd ? p.nx + 1 : p.nx + 2, colsV = p.nx + 1, colsW = cfd ? p.nx + 1 : p.nx + 2;
    const int64_t c[6] = {colsU, colsV, colsW, colsU, colsV, colsW};
    for (int i = 0; i < 6; ++i) {
        l[i] = c[i];
        if (ld && ld[i] != 0) {
            if (ld[i] < c[i])
                return fail(ADI_EINVAL, "ld[%d] = %lld below the row length %lld", i, (long long)ld[i], (long long)c[i]);
            l[i] = ld[i];
        }
    }
    return ADI_OK;
}

// Point the problem's device arrays into the workspace w laid out by L.
void place(adi_problem* pb, const Layout& L, char* w) {
    const auto& p = pb->p;
    const bool comp = p.dtype == ADI_FP32C;
    pb->ws = w;
    pb->ws_bytes = L.total;
    for (int d = 0; d < 2; ++d) {
        auto& D = pb->d[d];
        const bool hasR = d == 0 ? pb->hasRv : pb->hasRw;
        D.P = w + L.off[d][0];
        D.V[0] = w + L.off[d][1];
        D.V[1] = w + L.off[d][2];
        D.K = pb->hasK ? w + L.off[d][3] : nullptr;
        D.R = hasR ? w + L.off[d][4] : nullptr;
        D.Plo = comp ? w + L.off[d][5] : nullptr;
        D.Vlo[0] = comp ? w + L.off[d][6] : nullptr;
        D.Vlo[1] = comp ? w + L.off[d][7] : nullptr;
        D.coef = w + L.off[d][8];
        D.Vs = L.off[d][9] != L.off[d][10] ? w + L.off[d][9] : nullptr;
        D.Vslo = comp && D.Vs ? w + L.off[d][10] : nullptr;
        D.FF = pb->fsig.kind ? w + L.off[d][11] : nullptr;
        D.BND = pb->bsig.kind ? w + L.off[d][12] : nullptr;
    }
    for (int d = 0; d < 2; ++d) {
        pb->dfs[d] = p.sweeps == 0 ? w + L.fs_off[d] : nullptr;
        pb->dfs_u[d] = false;
    }
    pb->dconst = p.sweeps == 0 ? w + L.dc_off : nullptr;
}

// Workspace of adi_run_noalloc: one static device array per GPU, held until
// the process ends.  Host code never names it in device work: the address
// comes from hipGetSymbolAddress, once per device, with the device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

int scratch_of_device(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(ADI_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = (char*)ptr;
    }
    *out = g_scratch[dev];
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

int adi_set_forcing(adi_problem* pb, const void* F, int64_t ldF, const adi_signal* s) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!F) {
        pb->set_fF = nullptr;
        pb->set_fsig = adi_signal{};
        return ADI_OK;
    }
    if (pb->p.sweeps == 0) return fail(ADI_EINVAL, "direct solves (sweeps 0) take no distributed forcing");
    if (!s || (s->kind != ADI_SIGNAL_RICKER && s->kind != ADI_SIGNAL_COS))
        return fail(ADI_EINVAL, "forcing needs a Ricker or cosine signal");
    if (!std::isfinite(s->f0) || !std::isfinite(s->t0) || !std::isfinite(s->amp))
        return fail(ADI_EINVAL, "signal parameters must be finite");
    const int64_t cu = pb->p.method == ADI_CFD ? pb->p.nx + 1 : pb->p.nx + 2;
    if (ldF != 0 && ldF < cu) return fail(ADI_EINVAL, "ldF below the row length %lld", (long long)cu);
    pb->set_fF = F;
    pb->set_fF_ld = ldF ? ldF : cu;
    pb->set_fsig = *s;
    return ADI_OK;
}

int adi_set_damping(adi_problem* pb, double d0, double width, int walls) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!(d0 >= 0.0) || !std::isfinite(d0)) return fail(ADI_EINVAL, "the damping rate must be finite and >= 0");
    if (!(width >= 0.0) || !std::isfinite(width)) return fail(ADI_EINVAL, "the layer width must be finite and >= 0");
    if (walls & ~15) return fail(ADI_EINVAL, "unknown wall bits 0x%x", walls);
    if (d0 > 0.0 && walls) {
        if (pb->p.sweeps == 0) return fail(ADI_EINVAL, "direct solves (sweeps 0) run without damping layers");
        if (pb->eps > 0.0) return fail(ADI_EINVAL, "tolerance-tested stages run without damping layers");
        if (pb->p.dtype == ADI_FP32C) return fail(ADI_EINVAL, "damping layers run in FP32 or FP64, not the compensated mode");
    }
    pb->dmp0 = walls ? d0 : 0.0;
    pb->dmpw = width;
    pb->dmpwalls = walls;
    return ADI_OK;
}

int adi_set_boundary(adi_problem* pb, const adi_signal* s) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!s) {
        pb->set_bsig = adi_signal{};
        return ADI_OK;
    }
    if (pb->p.sweeps == 0) return fail(ADI_EINVAL, "direct solves (sweeps 0) take homogeneous walls only");
    if (s->kind != ADI_SIGNAL_RICKER && s->kind != ADI_SIGNAL_COS)
        return fail(ADI_EINVAL, "wall data need a Ricker or cosine signal");
    if (!std::isfinite(s->f0) || !std::isfinite(s->t0) || !std::isfinite(s->amp))
        return fail(ADI_EINVAL, "signal parameters must be finite");
    pb->set_bsig = *s;
    return ADI_OK;
}

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
    int64_t l[6];
    int rc = leading_dims(p, ld, l);
    if (rc != ADI_OK) return rc;
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    if (pb->own_ws && pb->ws) {
        (void)hipFree(pb->ws);
        pb->ws = nullptr;
        pb->own_ws = false;
    }
    if (pb->eps > 0.0 && (pb->set_fsig.kind || pb->set_bsig.kind))
        return fail(ADI_EINVAL, "tolerance-tested stages run without wall data or a forcing field");
    pb->bound = false;
    pb->fF = pb->set_fF;
    pb->fF_ld = pb->set_fF_ld;
    pb->fsig = pb->set_fsig;
    pb->bsig = pb->set_bsig;
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
    place(pb, L, pb->ws);
    if (p.sweeps == 0 && !pb->dst2) {
        HIP_TRY(hipStreamCreateWithFlags(&pb->dst2, hipStreamNonBlocking), "direct solves: second stream");
        HIP_TRY(hipEventCreateWithFlags(&pb->dev_in, hipEventDisableTiming), "direct solves: event");
        HIP_TRY(hipEventCreateWithFlags(&pb->dev_out, hipEventDisableTiming), "direct solves: event");
    }
    pb->U = U; pb->V = V; pb->W = W;
    pb->ldU = l[0]; pb->ldV = l[1]; pb->ldW = l[2];
    pb->vcur = pb->wcur = 0;
    pb->step = 0;
    pb->ready = false;
    rc = p.dtype != ADI_FP64
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
    // graph replay: the problem as a batch of one (the steady steps from a
    // captured graph); runs with a health check or the tolerance test take
    // the launch path
    if (pb->graph && nsteps >= 3 && pb->chk_every <= 0 && pb->eps <= 0.0 && !pb->fsig.kind && !pb->bsig.kind) {
        if (!pb->gbatch) {
            adi_problem* one[1] = {pb};
            const int rc = adi_batch_create(one, 1, pb->st, ADI_BATCH_GRAPH | ADI_BATCH_ONE_STREAM, &pb->gbatch);
            if (rc != ADI_OK) return rc;
        }
        return adi_batch_run(pb->gbatch, nsteps);
    }
    return pb->p.dtype != ADI_FP64 ? run_impl<float>(pb, nsteps) : run_impl<double>(pb, nsteps);
}

int adi_set_graph(adi_problem* pb, int on) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (on) {
        if (!pb->st) return fail(ADI_EINVAL, "graph replay needs a created stream, not the null stream");
        if (pb->p.sweeps == 0) return fail(ADI_EINVAL, "direct solves (sweeps 0) run without graph replay");
        if (pb->fsig.kind || pb->bsig.kind || pb->set_fsig.kind || pb->set_bsig.kind)
            return fail(ADI_EINVAL, "problems with a forcing field or wall data run without graph replay");
    } else if (pb->gbatch) {
        HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
        adi_batch_destroy(pb->gbatch);
        pb->gbatch = nullptr;
    }
    pb->graph = on != 0;
    return ADI_OK;
}

int adi_step(adi_problem* pb) { return adi_run(pb, 1); }

int adi_get_state(adi_problem* pb, void* U, void* V, void* W) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!pb->bound) return fail(ADI_ENOTREADY, "problem has no bound arrays");
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    const int rc = adi::materialize(pb, U ? U : pb->U, V ? V : pb->V, W ? W : pb->W);
    if (rc != ADI_OK) return rc;
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    return health_status(pb);
}

int adi_sync(adi_problem* pb) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    return pb->bound ? health_status(pb) : ADI_OK;
}

int adi_set_check(adi_problem* pb, int64_t every, double max_abs) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!pb->bound) return fail(ADI_ENOTREADY, "problem has no bound arrays");
    if (every < 0) return fail(ADI_EINVAL, "every must be >= 0");
    if (!(max_abs >= 0.0)) return fail(ADI_EINVAL, "max_abs must be >= 0");
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    // clear the running state (queued after earlier work on the stream)
    const Layout L = layout(*pb);
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(256), 0, pb->st, (uint4*)(pb->ws + L.chk_off), (L.total - L.chk_off) / 16);
    HIP_TRY(hipGetLastError(), "health check reset");
    pb->chk_every = every;
    pb->chk_max = max_abs;
    return ADI_OK;
}

int adi_autotune(adi_problem* pb, int reps, double* pass_us) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!pb->bound) return fail(ADI_ENOTREADY, "problem has no bound arrays");
    if (reps < 0 || reps > 1000) return fail(ADI_EINVAL, "reps must be in [0, 1000]");
    double us[2] = {0.0, 0.0};
    if (pb->p.sweeps == 0) {
        if (pass_us) pass_us[0] = pass_us[1] = 0.0;
        return ADI_OK;   // the direct solves have no launch choices
    }
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    const int r = reps ? reps : 10;
    const int rc = pb->p.dtype == ADI_FP64 ? autotune_impl<double>(pb, r, us) : autotune_impl<float>(pb, r, us);
    if (pass_us) {
        pass_us[0] = us[0];
        pass_us[1] = us[1];
    }
    return rc;
}

int adi_set_plan(adi_problem* pb, int dir, int choice) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (dir != 0 && dir != 1) return fail(ADI_EINVAL, "dir must be 0 (x lines) or 1 (y lines)");
    Plan& pl = dir == 0 ? pb->px : pb->py;
    int c[8];
    const int nc = pb->p.sweeps == 0 ? 0 : plan_choices(pl, c);
    bool ok = false;
    for (int i = 0; i < nc; ++i) ok = ok || c[i] == choice;
    if (!ok) return fail(ADI_EINVAL, "choice %d is not a launch choice of this plan (%d choices)", choice, nc);
    apply_choice(pl, pb->p.dtype, choice);
    pl.tuned = false;
    if (!pb->bound) return ADI_OK;
    // the tables of the new tile shape, after the queued passes that read
    // the old ones
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    double host64[6 * adi::LINE_WS];
    float host32[6 * adi::LINE_WS];
    const int rc = pb->p.dtype == ADI_FP64 ? upload_tables<double>(pb, dir, host64, pb->st)
                                           : upload_tables<float>(pb, dir, host32, pb->st);
    if (rc != ADI_OK) return rc;
    HIP_TRY(hipStreamSynchronize(pb->st), "factor tables");
    return ADI_OK;
}

int adi_get_plan(const adi_problem* pb, int dir, adi_plan_info* info) {
    g_err.clear();
    if (!pb || !info) return fail(ADI_EINVAL, "NULL argument");
    if (dir != 0 && dir != 1) return fail(ADI_EINVAL, "dir must be 0 (x lines) or 1 (y lines)");
    const Plan& pl = dir == 0 ? pb->px : pb->py;
    std::memset(info, 0, sizeof(*info));
    info->kernel = pb->p.sweeps == 0 ? ADI_KERNEL_DIRECT
                                     : (pl.ver == 1 ? ADI_KERNEL_SINGLE : (pl.ver == 3 ? ADI_KERNEL_WAVE : 0));
    info->lines = pl.nlines;
    info->slots = pl.ns;
    if (pb->p.sweeps == 0) {
        info->windows = pl.dnwin;
        info->window = pl.dS;
        info->margin = pl.dH;
        return ADI_OK;
    }
    info->windows = pl.nwin;
    info->window = pl.ver == 1 ? adi::line_ws(pl.cfg) : adi::LINE_WS;
    info->margin = pl.ver == 1 ? 0 : pl.H;
    info->lines_per_group = pl.ver == 1 ? adi::line_lanes(pb->p.dtype, pl.cfg) : adi::line3_lanes(pb->p.dtype);
    info->workgroups = pl.nlg * pl.nwin;
    info->tile_shape = pl.ver == 1 ? pl.cfg : -1;
    info->tile_order = pl.ver == 3 ? pl.torder : -1;
    info->tuned = pl.tuned ? 1 : 0;
    return ADI_OK;
}

int adi_check_stats(adi_problem* pb, double* max_abs, int* nonfinite) {
    g_err.clear();
    if (!pb || !max_abs || !nonfinite) return fail(ADI_EINVAL, "NULL argument");
    *max_abs = 0.0;
    *nonfinite = 0;
    if (!pb->bound) return fail(ADI_ENOTREADY, "problem has no bound arrays");
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    double st[4];
    HIP_TRY(hipMemcpy(st, (double*)(pb->ws + layout(*pb).chk_off) + kChkState, sizeof(st), hipMemcpyDeviceToHost),
            "health check state");
    *max_abs = st[1];
    *nonfinite = st[0] > 0.0 ? 1 : 0;
    return ADI_OK;
}

int adi_run_noalloc(const adi_params* p, void* hip_stream, void* U, void* V, void* W, const void* K,
                    const void* Rv, const void* Rw, const int64_t* ld, int64_t nsteps) {
    g_err.clear();
    int rc = validate(p);
    if (rc != ADI_OK) return rc;
    if (p->sweeps == 0) return fail(ADI_EINVAL, "adi_run_noalloc runs fixed sweep counts, not direct solves");
    if (!U || !V || !W) return fail(ADI_EINVAL, "U, V and W are required");
    if (nsteps < 0) return fail(ADI_EINVAL, "nsteps < 0");
    adi_problem pb;
    pb.p = *p;
    pb.st = (hipStream_t)hip_stream;
    derive(&pb);
    pb.hasK = K != nullptr;
    pb.hasRv = Rv != nullptr;
    pb.hasRw = Rw != nullptr;
    const Layout L = layout(pb);
    if (L.total > kScratchBytes)
        return fail(ADI_EINVAL, "workspace of %zu bytes exceeds the %zu bytes of adi_run_noalloc", L.total,
                    kScratchBytes);
    int64_t l[6];
    rc = leading_dims(pb.p, ld, l);
    if (rc != ADI_OK) return rc;
    HIP_TRY(hipGetDevice(&pb.dev), "hipGetDevice");
    char* w = nullptr;
    rc = scratch_of_device(pb.dev, &w);
    if (rc != ADI_OK) return rc;
    place(&pb, L, w);
    pb.U = U; pb.V = V; pb.W = W;
    pb.ldU = l[0]; pb.ldV = l[1]; pb.ldW = l[2];
    rc = p->dtype != ADI_FP64
             ? bind_materials<float>(&pb, (const float*)K, (const float*)Rv, (const float*)Rw, l[3], l[4], l[5])
             : bind_materials<double>(&pb, (const double*)K, (const double*)Rv, (const double*)Rw, l[3], l[4], l[5]);
    if (rc != ADI_OK) return rc;
    pb.bound = true;
    if (nsteps == 0) return ADI_OK;
    rc = p->dtype != ADI_FP64 ? run_impl<float>(&pb, nsteps) : run_impl<double>(&pb, nsteps);
    if (rc != ADI_OK) return rc;
    return adi::materialize(&pb, U, V, W);
}

int adi_get_step(const adi_problem* pb, int64_t* m) {
    if (!pb || !m) return fail(ADI_EINVAL, "NULL argument");
    *m = pb->step;
    return ADI_OK;
}

int adi_set_step(adi_problem* pb, int64_t m) {
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (m < 0) return fail(ADI_EINVAL, "step < 0");
    if (pb->ready && m != pb->step) {
        // the hand-off in the workspace holds the forcing of the old time
        // level: the state goes back to the bound arrays and the next run
        // starts from them
        HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
        const int rc = adi::materialize(pb, pb->U, pb->V, pb->W);
        if (rc != ADI_OK) return rc;
        pb->ready = false;
    }
    pb->step = m;
    return ADI_OK;
}

int adi_set_tolerance(adi_problem* pb, double eps, int min_sweeps) {
    g_err.clear();
    if (!pb) return fail(ADI_EINVAL, "problem is NULL");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ADI_EINVAL, "eps must be finite and >= 0");
    if (eps == 0.0) {
        pb->eps = 0.0;
        pb->eps_kmin = 0;
        return ADI_OK;
    }
    if (pb->p.sweeps == 0) return fail(ADI_EINVAL, "direct solves (sweeps 0) take no tolerance");
    if (min_sweeps < 2 || (min_sweeps & 1) || min_sweeps > pb->p.sweeps)
        return fail(ADI_EINVAL, "min_sweeps must be even and in [2, sweeps] (got %d, sweeps %d)", min_sweeps,
                    pb->p.sweeps);
    if (pb->p.dtype == ADI_FP32C) return fail(ADI_EINVAL, "tolerance-tested stages: FP32 or FP64 only");
    if (pb->dmp0 != 0.0) return fail(ADI_EINVAL, "tolerance-tested stages run without damping layers");
    if (pb->fsig.kind || pb->bsig.kind)
        return fail(ADI_EINVAL, "tolerance-tested stages run without wall data or a forcing field");
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    if (pb->ready) {
        // tolerance-tested runs start from the bound arrays
        const int rc = adi::materialize(pb, pb->U, pb->V, pb->W);
        if (rc != ADI_OK) return rc;
        pb->ready = false;
    }
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    // single-window plans take the quarter-width tile shapes: the tested
    // form's spare array does not fit the registers of the 16-wave shapes
    for (int d = 0; d < 2; ++d) {
        Plan& pl = d == 0 ? pb->px : pb->py;
        if (pl.ver != 1 || pl.cfg >= 3) continue;
        set_cfg(pl, pb->p.dtype, pl.cfg + 3);
        pl.tuned = false;
        double h64[6 * adi::LINE_WS];
        float h32[6 * adi::LINE_WS];
        const int rc = pb->p.dtype == ADI_FP64 ? upload_tables<double>(pb, d, h64, pb->st)
                                               : upload_tables<float>(pb, d, h32, pb->st);
        if (rc != ADI_OK) return rc;
        HIP_TRY(hipStreamSynchronize(pb->st), "factor tables");
    }
    if (!pb->eps_buf) HIP_TRY(hipMalloc(&pb->eps_buf, eps_bytes(pb)), "tolerance state");
    // flags: attempt 0 of the next pass runs; counters cleared
    const EpsLayout L = eps_layout(pb);
    int go[kMaxAttempts + 1] = {1};
    const long long zero[2] = {0, 0};
    HIP_TRY(hipMemcpy(L.go, go, sizeof(go), hipMemcpyHostToDevice), "tolerance flags");
    HIP_TRY(hipMemcpy(L.stats, zero, sizeof(zero), hipMemcpyHostToDevice), "tolerance counters");
    pb->eps = eps;
    pb->eps_kmin = min_sweeps;
    return ADI_OK;
}

int adi_sweep_stats(adi_problem* pb, int64_t* passes, int64_t* sweeps) {
    g_err.clear();
    if (!pb || !passes || !sweeps) return fail(ADI_EINVAL, "NULL argument");
    *passes = *sweeps = 0;
    if (!pb->eps_buf) return ADI_OK;
    HIP_TRY(hipSetDevice(pb->dev), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(pb->st), "hipStreamSynchronize");
    long long st[2];
    HIP_TRY(hipMemcpy(st, eps_layout(pb).stats, sizeof(st), hipMemcpyDeviceToHost), "tolerance counters");
    *passes = st[0];
    *sweeps = st[1];
    return ADI_OK;
}

int adi_destroy(adi_problem* pb) {
    if (!pb) return ADI_OK;
    if (pb->gbatch) {
        (void)hipSetDevice(pb->dev);
        adi_batch_destroy(pb->gbatch);
    }
    if ((pb->own_ws && pb->ws) || pb->eps_buf || pb->dst2) {
        (void)hipSetDevice(pb->dev);
        (void)hipStreamSynchronize(pb->st);
        if (pb->dst2) (void)hipStreamSynchronize(pb->dst2);
        if (pb->own_ws && pb->ws) (void)hipFree(pb->ws);
        if (pb->eps_buf) (void)hipFree(pb->eps_buf);
        if (pb->dev_in) (void)hipEventDestroy(pb->dev_in);
        if (pb->dev_out) (void)hipEventDestroy(pb->dev_out);
        if (pb->dst2) (void)hipStreamDestroy(pb->dst2);
    }
    delete pb;
    return ADI_OK;
}

}  // extern "C"
