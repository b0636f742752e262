// Internal state of a problem and the pieces of a run, shared by the
// single-problem entry points (adi.hip) and the batched ones (batch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/adi.h"
#include "line_pass.h"

namespace adi {

// Launch plan of the passes along one direction.
struct Plan {
    int n = 0, ns = 0, nlines = 0, nlg = 0, nwin = 0, S = 0, H = 0, deep = 0;
    int ver = 1;   // 1: single-window kernel (line_pass.hip); multi-window: 2 (line_pass2.hip,
                   // compensated mode) or 3 (line_pass3.hip)
    int cfg = 0;   // tile shape of the single-window kernel
    int torder = 0;   // tile order of the wave-per-line kernel (LinePassArgs::torder)
    bool tuned = false;   // cfg / torder from the autotuner (adi_autotune)
    int seg = 0;   // slots per lane segment of the multi-window kernel
    // direct (exact) line solves: output slots per window (and of the two
    // end windows), margin, windows,
    // kept rows per window, lines padded to a multiple of 64
    // interior-band windows dwa..dwb
    int dS = 0, dSe = 0, dH = 0, dnwin = 0, drows = 0, dnlp = 0, dwa = 0, dwb = -1;
};

// One pass, ready to launch.
template <typename T>
struct PassDesc {
    LinePassArgs<T> a;
    int ver, cfg, method, mode;
    bool comp;
    int dir;
    // the kernel variant with damping layers, wall data or a forcing field
    bool full() const { return a.dmpm != 0 || a.bnd != nullptr || a.ff != nullptr; }
    int tiles() const { return a.nlg * a.nwin; }
    // kernel variant: passes with equal keys can share a grouped launch
    int key() const { return (((ver * 8 + cfg) * 2 + method) * 8 + mode * 2 + (comp ? 1 : 0)) * 2 + (full() ? 1 : 0); }
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

#define HIP_TRY(expr, what)                                  \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return adi::hip_fail(e_, what); \
    } while (0)

}  // namespace adi

struct adi_problem {
    adi_params p{};
    hipStream_t st = nullptr;
    int dev = 0;
    int nix = 0, niy = 0;
    double a = 0.0;
    int64_t step = 0;
    bool bound = false;
    // graph replay of adi_run (adi_set_graph): a batch of this problem alone
    bool graph = false;
    adi_batch* gbatch = nullptr;
    // ready: the state of time level `step` lives in the workspace (the
    // pressure hand-off and velocities of the next pass); otherwise it is in
    // the bound arrays U, V, W
    bool ready = false;
    void *U = nullptr, *V = nullptr, *W = nullptr;
    int64_t ldU = 0, ldV = 0, ldW = 0;
    bool hasK = false, hasRv = false, hasRw = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    size_t esz = 4;
    // Device arrays of the passes of one direction (d[0]: along x, lines =
    // interior rows; d[1]: along y, lines = interior columns).  Line index q,
    // slot s along the line.  Slot-major (the segment and single-window
    // kernels): pressure-type element (s - 1) * ld + q, velocity-type s * ld + q.
    // Line-major (the wave-per-line kernel): element q * ld + s for both, the
    // boundary slots stored as zeros, rows padded to whole line groups.
    struct Dir {
        bool lm = false;
        int64_t ld = 0;                       // leading dimension (elements)
        int64_t rows_p = 0, rows_v = 0;       // rows of the pressure- / velocity-type arrays
        void *P = nullptr;                    // pressure hand-off read by these passes
        void *V[2] = {nullptr, nullptr};      // velocity along the lines (ping-pong)
        void *K = nullptr, *R = nullptr;      // a*kappa, a/rho (NULL when constant)
        void *Plo = nullptr, *Vlo[2] = {nullptr, nullptr};   // compensated low words
        void *coef = nullptr;                 // single-window compact tables
        // spare velocity buffer (and its low words) of the direction whose
        // pass ends a step: adi_get_state re-runs that pass into it
        void *Vs = nullptr, *Vslo = nullptr;
        // forcing field in this direction's pressure layout; wall
        // coefficients per line, {value, c^2 d_ll value, forcing} at each end
        void *FF = nullptr, *BND = nullptr;
    } d[2];
    int vcur = 0, wcur = 0;
    adi::Plan px, py;
    // tolerance-tested stages (adi_set_tolerance): eps > 0 switches them on;
    // eps_buf holds the per-attempt change sums, the attempt flags and the
    // pass / sweep counters (layout in adi.hip, eps_layout)
    double eps = 0.0;
    int eps_kmin = 0;
    void* eps_buf = nullptr;
    // health check (adi_set_check): every chk_every steps, largest pressure
    // magnitude allowed (0: non-finite values only); state in the workspace
    int64_t chk_every = 0;
    double chk_max = 0.0;
    // distributed forcing F(x, y) s_F(t) and wall data Ub(x, y) s_b(t)
    // (adi_set_forcing / adi_set_boundary); kind 0 = none.  The set_ values
    // take effect at the next adi_bind.
    const void* fF = nullptr;
    int64_t fF_ld = 0;
    adi_signal fsig{};
    adi_signal bsig{};
    const void* set_fF = nullptr;
    int64_t set_fF_ld = 0;
    adi_signal set_fsig{};
    adi_signal set_bsig{};
    // damping layers (adi_set_damping): rate, width in cells (0: uniform),
    // walls (bit 0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1)
    double dmp0 = 0.0, dmpw = 0.0;
    int dmpwalls = 0;
    // factor stores of the direct solves (sweeps 0), one per direction, and
    // the constant materials {a kappa0, a rinv0} they read when K or R is
    // absent, all part of the workspace; dfs_u[d]: the store of direction d
    // holds the U entries of its matrix (set by its first pass after a bind)
    void* dfs[2] = {nullptr, nullptr};
    bool dfs_u[2] = {false, false};
    void* dconst = nullptr;
    // second stream and its two events: the windows at the line ends run
    // beside the interior windows
    hipStream_t dst2 = nullptr;
    hipEvent_t dev_in = nullptr, dev_out = nullptr;
};

namespace adi {

// Steps of one problem are
//   run_begin (when the state is not ready), then for s = 0..nsteps-1 the
//   passes run_pass(s, 0) and run_pass(s, 1), then either
//   run_end (the last pass final: the state goes back to the bound arrays)
//   or nothing (every pass a sweep pass: the state stays in the workspace,
//   step advanced by the caller through run_advance).
// run_begin queues the set-up copies and the explicit pass of step m on st
// and marks the state ready; run_pass returns the pass (and advances the
// ping-pong buffers); its source term is aF(m + s + 1), taken from
// aFtab[tick] when aFtab is given (grouped launches) and computed on the host
// otherwise.  `final_pass` (half 1 only) writes U^{m+s+1} into the bound U
// instead of the next step's hand-off.
template <typename T> int run_begin(adi_problem* pb, hipStream_t st);
template <typename T>
PassDesc<T> run_pass(adi_problem* pb, int64_t s, int half, bool final_pass, const T* aFtab);
template <typename T> int run_end(adi_problem* pb, hipStream_t st, int64_t nsteps);
inline void run_advance(adi_problem* pb, int64_t nsteps) { pb->step += nsteps; }
// Write the state of time level `step` into U, V, W (device arrays with the
// bound leading dimensions) on the problem's stream; a ready problem's
// workspace state is left as it was, a problem that is not ready is copied
// from its bound arrays where the targets differ.
int materialize(adi_problem* pb, void* U, void* V, void* W);
template <typename T> hipError_t launch_pass(const PassDesc<T>& d, hipStream_t st);
// One grouped launch of passes sharing the kernel variant of `proto`.
template <typename T> hipError_t launch_grouped(const PassDesc<T>& proto, const GroupArgs<T>& ga, hipStream_t st);

// a * s(t) / h^2 at time level m (0 without a source)
double source_term(const adi_problem& pb, int64_t m);

}  // namespace adi
