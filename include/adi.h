/*
 * adi.h - C ABI of the MI355X Peaceman-Rachford ADI library (libadi.so).
 *
 * The library advances the 2-D velocity-pressure acoustic system
 *     u_t = -kappa div(v) + f,   rho v_t = -grad u            (Section 2, eq. 1)
 * on a rectangular grid of nx x ny cells of spacing h, with homogeneous
 * Dirichlet pressure on the four walls, by the Crank-Nicolson time
 * discretisation factored with the Peaceman-Rachford split (eqs. CN, PR two
 * stages).  Each stage couples pressure and one velocity component along the
 * grid lines of one direction and is solved by a fixed, even number of
 * fixed-point sweeps (eqs. adiSolve, adiSolve2; Algorithms 3 and 4), or
 * exactly (params.sweeps = 0, the limit of infinitely many sweeps; see
 * below).  Two spatial discretisations are offered:
 *   ADI_CFD  nodal fourth-order compact differences, P4/Q4 and the reduced
 *            Pbar4/Qbar4 (Section 2.1, Appendix A): every derivative along a
 *            line is one tridiagonal solve;
 *   ADI_MFD  staggered fourth-order mimetic operators D4/G4 (Section 2.2,
 *            Appendix B): every derivative is a banded stencil.
 * One step applies, in order: the explicit y-part of stage 1 (A, W*), the
 * row iterations (Ubar*, V*), the explicit x-part of stage 2 (C, V^{m+1}) and
 * the column iterations (U^{m+1}, W^{m+1}) (Algorithms 1 and 2).
 *
 * Arrays are row-major, row index j along y, column index i along x, all of
 * the problem's dtype (float for ADI_FP32, double for ADI_FP64), in device
 * memory (ADI_FP32C uses float arrays).  Shapes (rows x cols):
 *                 CFD                MFD
 *   U, K          (ny+1) x (nx+1)    (ny+2) x (nx+2)   pressure points
 *   V, Rv         (ny+1) x (nx+1)    (ny+2) x (nx+1)   horizontal velocity
 *   W, Rw         (ny+1) x (nx+1)    (ny+1) x (nx+2)   vertical velocity
 * K holds kappa at the pressure points, Rv and Rw hold 1/rho at the velocity
 * points.  Boundary pressure entries are Dirichlet data and stay zero; the
 * first and last rows of V and the first and last columns of W are never
 * read or written.
 *
 * Status codes: every entry point returns an adi_status; arguments are
 * validated on the host before any device work is queued.  No entry point
 * aborts, throws or prints.
 *
 * Threads: one adi_problem must not be used by two host threads at once.
 * Device work is queued asynchronously on the stream given at creation.
 */
#ifndef ADI_H
#define ADI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum adi_status {
    ADI_OK = 0,
    ADI_EINVAL = -1,     /* invalid argument (message: adi_last_error) */
    ADI_ENOMEM = -2,     /* device allocation failed */
    ADI_EDEVICE = -3,    /* a HIP runtime call failed */
    ADI_EBUSY = -4,      /* object in use */
    ADI_ENOTREADY = -5,  /* problem not bound yet */
    ADI_ENUMERIC = -6    /* non-finite values detected */
} adi_status;

typedef enum adi_method { ADI_CFD = 0, ADI_MFD = 1 } adi_method;
/* ADI_FP32C: FP32 arithmetic and FP32 caller arrays; the state carried
 * between passes is kept as (value, low word) pairs and every pass
 * accumulates its FP32 increment with TwoSum, so rounding does not build up
 * over many steps.  The low words live in the workspace with the rest of the
 * state (adi_get_state writes the rounded sums). */
typedef enum adi_dtype { ADI_FP32 = 0, ADI_FP64 = 1, ADI_FP32C = 2 } adi_dtype;

/* Problem description.  Set struct_size = sizeof(adi_params); fill the rest
 * or start from adi_params_init. */
typedef struct adi_params {
    uint32_t struct_size;
    int32_t method;      /* adi_method */
    int32_t dtype;       /* adi_dtype */
    int32_t order;       /* 0: x-implicit stage first (the paper's order); 1: y-implicit first */
    int32_t nx, ny;      /* cells per direction, each >= 8 */
    int32_t sweeps;      /* fixed-point sweeps per stage: even, in [2, 16] (paper: 6-8);
                            0 = direct (exact) line solves, see below */
    int32_t src_i, src_j;/* pressure index (column i, row j) of the Ricker point
                            source, both interior; -1 = no source */
    int32_t reserved0;
    double h;            /* grid spacing (both directions) */
    double dt;           /* time step; cfl = dt c_max / h must stay below the
                            fixed-point limit: 1.15 (CFD), 0.81 (MFD) */
    double t0;           /* time of step 0 */
    double c_max;        /* maximum wave speed sqrt(kappa / rho) */
    double kappa0;       /* kappa when no K array is bound */
    double rinv0;        /* 1/rho when no Rv / Rw array is bound */
    double src_f0;       /* Ricker peak frequency */
    double src_t0;       /* Ricker delay */
    double src_amp;      /* Ricker amplitude; forcing = s(t) / h^2 at the point */
} adi_params;

typedef struct adi_problem adi_problem;

/* A time signal s(t): ADI_SIGNAL_RICKER amp (1 - 2 x^2) exp(-x^2) with
 * x = pi f0 (t - t0); ADI_SIGNAL_COS amp cos(2 pi f0 (t - t0)) (f0 = 0: the
 * constant amp). */
enum { ADI_SIGNAL_RICKER = 1, ADI_SIGNAL_COS = 2 };
typedef struct adi_signal {
    int32_t kind;
    int32_t reserved0;
    double f0, t0, amp;
} adi_signal;

/* Human-readable name of a status code (static storage). */
const char* adi_status_string(int status);

/* Message of the last error raised on this host thread ("" if none). */
const char* adi_last_error(void);

/* Direct line solves (params.sweeps = 0).  Each stage's coupled line
 * systems (Section 2.1, eqs. ecua2:PR and ecua3:PR2 along every grid line)
 * are solved exactly instead of by fixed-point sweeps: the step is the
 * Peaceman-Rachford step itself, with no iteration error and no step-size
 * limit from the iteration (the sweeps diverge at cfl 1.155 compact and
 * 0.816 mimetic; adi_create rejects those step sizes when sweeps > 0).
 * Each line system is rewritten as a banded system (mimetic: the pressure
 * system after eliminating the velocity; compact: the two derivative
 * unknowns interleaved) and solved by LU without pivoting over overlapping
 * windows of the line, whose margins come from the decay of the inverse of
 * the line matrix at the largest a c / h (to 1e-17 of its peak in FP64,
 * 1e-9 in FP32).  The workspace (adi_workspace_size) then also holds the
 * factors of every window, about (window + margin) x 4..7 values per line
 * slot.  Scope: ADI_FP32 and ADI_FP64, single problems; adi_create rejects
 * ADI_FP32C and step sizes whose margin exceeds 4096 slots, and batches,
 * servers and adi_set_tolerance refuse such problems (ADI_EINVAL). */

/* Distributed forcing and Dirichlet data that vary in time (the
 * heterogeneous tests of Section 4, eq. harmonic_hetero, which need both).
 * Call after adi_create and before adi_bind; both are read at adi_bind.
 *
 * adi_set_forcing: f(x, y, t) = F(x, y) s(t) at every interior pressure
 * point, in addition to the point source: F^m enters the first stage of a
 * step and F^{m+1} the second, as in eqs. ecua2:PR and ecua3:PR2.  F is a
 * device array shaped like U (leading dimension ldF, 0 = dense), read by
 * adi_bind; NULL removes the forcing.  Costs one more array read per pass.
 *
 * adi_set_boundary: the pressure on the walls is u = Ub(x, y) s(t), Ub the
 * wall entries of the U bound by adi_bind (so at t = 0, s(0) = 1 gives back
 * the initial data); s = NULL restores homogeneous walls.  The paper does
 * not say which wall values the intermediate level of the split carries;
 * this library uses the pressure component of the split's own identity
 * U* = (I + a A2) U^m / 2 + (I - a A2) U^{m+1} / 2 + a (F^m - F^{m+1}) / 2
 * on the wall data, i.e. (u_b^m + u_b^{m+1}) / 2 - a^2 c^2 d_ll u_b(t^m +
 * dt/2) + a (f^m - f^{m+1}) / 2 with d_ll the second difference along the
 * wall and c^2 = kappa / rho at the wall point; the other stages see the
 * walls at t^m and t^{m+1}.  This keeps the time error second order (the
 * mid-step wall value alone converges at first order).
 *
 * Scope: fixed sweep counts (ADI_EINVAL with sweeps 0), single problems
 * (batches refuse them).  Settings take effect at the next adi_bind; the
 * workspace then holds the forcing field in both line layouts and six
 * values per line, beyond what adi_workspace_size reports (pass no
 * workspace to adi_bind, or a larger one: adi_bind names the size it needs). */
int adi_set_forcing(adi_problem* pb, const void* F, int64_t ldF, const adi_signal* s);
int adi_set_boundary(adi_problem* pb, const adi_signal* s);

/* Absorbing layers: the damped system, a reformulation the paper points to
 * for absorbing boundaries (Section 2.1, closing remarks),
 *   u_t = -kappa div v - (d_x + d_y) u + f,
 *   rho v_t = -u_x - rho d_x v,   rho w_t = -u_y - rho d_y w,
 * with d_x (d_y) the rate of the layers along the x (y) walls.  The split
 * keeps each rate with its direction (A1 gets -d_x on u and v, A2 -d_y on u
 * and w), so every implicit line system divides by 1 + a d and every
 * explicit part multiplies by 1 - a d: the line passes compute the factors
 * per slot, with no extra memory traffic.  Profile: d = d0 (1 - dist /
 * width)^2 within `width` cells of each wall whose bit is set (ADI_WALL_*),
 * 0 beyond; width 0 = the uniform rate d0 in each direction with a wall bit
 * set.  A free surface (the top of the layered workloads) keeps its bit
 * clear.  d0 = 0 or walls = 0 switches the layers off (the default).
 * Takes effect at the next pass.  Scope: FP32 and FP64 with fixed sweep
 * counts, single problems and batches; ADI_EINVAL for the compensated mode,
 * direct solves and tolerance-tested stages. */
enum { ADI_WALL_X0 = 1, ADI_WALL_X1 = 2, ADI_WALL_Y0 = 4, ADI_WALL_Y1 = 8 };
int adi_set_damping(adi_problem* pb, double d0, double width, int walls);

/* Fill *p with defaults: CFD, FP32, order 0, 6 sweeps, no source,
 * kappa0 = rinv0 = 1, struct_size set.  Sizes, h, dt, c_max left zero. */
int adi_params_init(adi_params* p);

/* Validate *p and create a problem bound to the current HIP device and to
 * hip_stream (a hipStream_t, or NULL for the null stream).  No device memory
 * is allocated until adi_bind.  *out receives the handle; release it with
 * adi_destroy. */
int adi_create(const adi_params* p, void* hip_stream, adi_problem** out);

/* Bytes of device workspace adi_bind needs for these parameters, given which
 * material arrays will be bound (non-zero flag = array present). */
int adi_workspace_size(const adi_params* p, int has_K, int has_Rv, int has_Rw,
                       size_t* bytes);

/* Attach the caller's device arrays (shapes above).  U, V, W hold the
 * initial state (time level 0, see adi_set_step): the first adi_run reads
 * them into the workspace, where the state then stays between runs;
 * adi_get_state writes it out.  K, Rv, Rw may be NULL (constant kappa0 /
 * rinv0) and are read during this call only.  ld[0..5]
 * are the leading dimensions (elements) of U, V, W, K, Rv, Rw; NULL or 0
 * entries mean densely packed rows.  workspace may be NULL (the library then
 * allocates and owns it) or caller memory of at least adi_workspace_size
 * bytes, 256-byte aligned, which the caller keeps alive until adi_destroy.
 * The call returns after the device has consumed K, Rv, Rw.  Resets the step
 * counter to 0.
 * The step size was validated for c_max: ADI_EINVAL if the bound materials
 * exceed it, i.e. if (max kappa) (max 1/rho) over the interior points the
 * passes read (kappa0, rinv0 for absent arrays) is above c_max^2 by more than
 * rounding. */
int adi_bind(adi_problem* pb, void* U, void* V, void* W,
             const void* K, const void* Rv, const void* Rw,
             const int64_t* ld, void* workspace, size_t workspace_bytes);

/* Queue nsteps Peaceman-Rachford steps (Algorithm 1 / 2 loop body) on the
 * problem's stream, advancing the state from time level m to m + nsteps.
 * The state stays in the workspace in the layouts of the line passes (the
 * pressure hand-off and velocities of the next pass), so consecutive runs
 * continue without copies; the bound U, V, W are not written (adi_get_state
 * does that).  Runs with tolerance-tested stages (adi_set_tolerance) instead
 * start from and end in the bound arrays, as if adi_get_state followed. */
int adi_run(adi_problem* pb, int64_t nsteps);

/* adi_run(pb, 1). */
int adi_step(adi_problem* pb);

/* Wait for all queued work of the problem; ADI_ENUMERIC if the health check
 * (adi_set_check) has flagged the state. */
int adi_sync(adi_problem* pb);

/* Numerical health check, without host synchronisation during runs: every
 * `every` steps of adi_run (0 = off, the default) a device-side reduction
 * scans the pressure-type array of the new time level (the hand-off the step
 * leaves for the next one; U itself after a run's final pass) for non-finite
 * values and its largest magnitude, and folds them into a running state in
 * the workspace.  adi_sync and adi_get_state then return ADI_ENUMERIC (after
 * the work has drained) once a non-finite value has been seen, or, with
 * max_abs > 0, once the largest magnitude exceeded max_abs: the compact
 * scheme's boundary modes grow from rounding and make runs of a few thousand
 * steps on some inputs diverge, and a bound shows that before the values
 * overflow.  Cost: one read of a pressure-type array per check (about 13 us
 * at 4096^2 FP32).  The call resets the running state; batches and servers
 * do not run the check.  ADI_ENOTREADY before adi_bind. */
int adi_set_check(adi_problem* pb, int64_t every, double max_abs);

/* The running state of the health check: the largest magnitude seen and
 * whether a non-finite value was seen (waits for the problem's work). */
int adi_check_stats(adi_problem* pb, double* max_abs, int* nonfinite);

/* Launch autotuner.  The line passes (Section 3: one implicit sweep stage
 * and the next stage's explicit part per launch) have launch choices that
 * change their speed but not what they compute: the single-window kernel's
 * tile shape (0 .. 2: windows of 512, 256 or 128 slots with 32/64/64 lines
 * per workgroup in FP32, 16/32/64 in FP64; 3 .. 5: the same windows with a
 * quarter of the lines and of the waves per workgroup; every shape whose
 * window holds the line is a candidate) and the wave-per-line kernel's order of tiles across
 * the eight XCDs (0: each XCD takes whole line groups, 1: whole windows, 2:
 * no XCD mapping, 3 .. 6: whole windows within blocks of 4, 8, 16, 32 line
 * groups).  adi_autotune times each candidate of each direction's
 * sweep pass on the bound problem's own data (reps passes per timing, 0 =
 * 10; three rounds, best kept), keeps the fastest (the default stays unless
 * another is more than 1% faster), and stores the choice in a process-wide
 * cache keyed by (device architecture, method, dtype, slots per line,
 * lines, window margin, kernel).  Problems created later with the same key
 * (adi_create, batches, servers, adi_run_noalloc) start with the cached
 * choice.  With the environment variable ADI_TUNE_CACHE naming a file, the
 * cache is read from it at first use and rewritten after each tuning
 * (ADI_EINVAL if it cannot be written; the choice is kept in memory).
 * pass_us (optional, 2 values) receives the chosen pass time per direction
 * in microseconds (0 where a direction has no choice).  The current state
 * goes to the bound arrays first; the next run starts from them.  Tile
 * order changes nothing in the results; a tile shape may change FP rounding
 * of the single-window compact solves.  Direct solves (sweeps 0) have no
 * choices: the call returns at once.  Waits for the problem's stream; call
 * it before creating batches that hold the problem.  ADI_ENOTREADY before
 * adi_bind. */
int adi_autotune(adi_problem* pb, int reps, double* pass_us);

/* Graph replay for adi_run (on = 1; 0 turns it off).  The paper found
 * launch costs above the work of small problems (Section 5); with this set,
 * a run of at least 3 steps goes through a batch of this problem alone
 * (adi_batch_*, ADI_BATCH_GRAPH): two steps are captured once per run and
 * replayed, the source term read from a device table.  Results equal the
 * launched run bit for bit.  Needs the problem's own created stream (not the
 * null stream); refused for direct solves and for problems with a forcing
 * field or wall data.  Runs with the health check or the tolerance test on
 * take the launch path. */
int adi_set_graph(adi_problem* pb, int on);

enum { ADI_KERNEL_SINGLE = 1, ADI_KERNEL_WAVE = 3, ADI_KERNEL_DIRECT = 4 };

/* The launch plan of one direction (dir 0: the x lines, along which i
 * runs; 1: the y lines). */
typedef struct adi_plan_info {
    int kernel;          /* ADI_KERNEL_SINGLE (one window per line), ADI_KERNEL_WAVE
                            (wave per line, windows of 512 slots) or ADI_KERNEL_DIRECT */
    int lines;           /* lines of the direction */
    int slots;           /* velocity slots per line */
    int windows;         /* windows per line */
    int window;          /* slots per window (direct solves: output slots per inner window) */
    int margin;          /* overlap margin of the multi-window plans (slots per side) */
    int lines_per_group; /* lines per workgroup */
    int workgroups;      /* workgroups of one pass */
    int tile_shape;      /* single-window tile shape 0 .. 5 (windows 512, 256, 128, 512, 256, 128); -1 otherwise */
    int tile_order;      /* wave-per-line tile order 0 .. 6; -1 otherwise */
    int tuned;           /* 1 when the choice came from adi_autotune or its cache */
    int reserved[5];
} adi_plan_info;

int adi_get_plan(const adi_problem* pb, int dir, adi_plan_info* info);

/* Pin one direction's launch choice by hand: the tile shape (0 .. 5) of a
 * single-window plan, whose window must hold the line, or the tile order
 * (0 .. 6) of a wave-per-line plan; ADI_EINVAL for any other value and for
 * direct solves.  Allowed before or after adi_bind and between runs (the
 * resident state is kept; the call waits for the problem's stream).  The
 * cache is not changed; adi_get_plan then reports tuned = 0. */
int adi_set_plan(adi_problem* pb, int dir, int choice);

/* Write the state of the current time level m into the device arrays U, V,
 * W (shapes and leading dimensions of the bound arrays; NULL = the bound
 * array itself) and wait for it.  Only the entries the method updates are
 * written: interior pressure points, interior rows of V, interior columns
 * of W (Dirichlet boundary values and the unused velocity rows/columns are
 * left as they are).  The workspace state is not changed: runs continue from
 * m either way.  Cost: the pass that ended the last step run once more in its
 * final form (pressure U^m and its velocity instead of the next step's
 * hand-off), plus transposed copies of the velocities. */
int adi_get_state(adi_problem* pb, void* U, void* V, void* W);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): create,
 * bind, run nsteps steps (as adi_run) and write the state into U, V, W (as
 * adi_get_state) in one call, with no problem object and no allocation.  The
 * arguments are those of adi_create, adi_bind and adi_run; the workspace is
 * a static device array of 64 MiB per GPU (held from the library's first
 * use of that GPU until the process ends), so problems whose
 * adi_workspace_size exceeds 64 MiB are refused (ADI_EINVAL), as are direct
 * solves (sweeps 0).  The call waits for the stream once (the material check
 * of adi_bind) and returns with the steps and the write-out queued on
 * hip_stream.  Every call on a GPU shares that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (other host threads,
 * other streams) race and must be serialised by the caller; calls queued on
 * one stream are ordered. */
int adi_run_noalloc(const adi_params* p, void* hip_stream, void* U, void* V, void* W,
                    const void* K, const void* Rv, const void* Rw, const int64_t* ld,
                    int64_t nsteps);

/* Current time level m (time t0 + m dt) / set it (checkpoint resume).
 * Setting another level while the state is in the workspace first writes the
 * state into the bound arrays; the next run starts from them. */
int adi_get_step(const adi_problem* pb, int64_t* m);
int adi_set_step(adi_problem* pb, int64_t m);

/* Tolerance-tested stages: the stopping rule of the ADI iterations in
 * Algorithms 3 and 4 (Appendix C) instead of a fixed sweep count.  After
 * sweep k of a stage, k >= min_sweeps, the Frobenius norms of the changes of
 * the whole stage, ||Ubar_k - Ubar_{k-1}|| + ||vel_k - vel_{k-1}||, are summed
 * and compared with eps; the first count that passes is rounded up to an
 * even count (odd counts amplify the unconverged modes), and params.sweeps
 * is the cap.  Like the paper's GPU codes (Section 3), the test starts after
 * a minimum number of sweeps; unlike them, the decision never leaves the
 * device: each pass is queued as attempts with min_sweeps, min_sweeps + 2,
 * .. sweeps sweeps, each recomputing the pass from its unchanged inputs and
 * running only while the earlier ones have not converged.
 *   eps         > 0 switches the test on, 0 restores the fixed count.
 *   min_sweeps  even, in [2, params.sweeps].
 * Applies to FP32 and FP64 problems of any size (fixed sweeps, no damping
 * layers, wall data or forcing field), run with adi_run / adi_step; such a
 * problem cannot join a batch.  If runs have left the state in the workspace
 * it is first written into the bound arrays, where tolerance-tested runs
 * start and end.  Clears the counters of adi_sweep_stats.  Allocates 32
 * bytes of device memory per workgroup of a pass (about 150 KiB at 4096^2)
 * the first time.
 * Errors: ADI_EINVAL for a NULL problem, eps < 0 or not finite, min_sweeps
 * out of range, or a problem outside the scope above. */
int adi_set_tolerance(adi_problem* pb, double eps, int min_sweeps);

/* Tolerance-tested passes run and the sweeps they used since the last
 * adi_set_tolerance (both 0 if it was never called).  Waits for the
 * problem's queued work. */
int adi_sweep_stats(adi_problem* pb, int64_t* passes, int64_t* sweeps);

/* Free the problem and any workspace the library allocated. */
int adi_destroy(adi_problem* pb);

/* ---- Batched runs ----------------------------------------------------
 * Many independent problems advanced together.  The paper observes
 * (Sections 3.2 and 5) that overlapping many small kernels with streams did
 * not pay because launch costs exceeded the work per launch; here each
 * half-step of all problems is one launch per kernel variant (tile shape x
 * method x mode, at most a few), each workgroup picking its problem and
 * line group from a table.  Results are identical, bit for bit, to running
 * every problem alone with adi_run; as after adi_run, each problem's state
 * stays in its workspace (read it with adi_get_state). */
typedef struct adi_batch adi_batch;

/* Replay the launches of the steady-state steps from a captured hipGraph. */
#define ADI_BATCH_GRAPH 1
/* Issue the grouped launches of a half-step one after the other on the
 * batch stream.  By default they are spread over the batch stream and three
 * more streams of the batch (fork and join per half-step, captured as
 * parallel branches with ADI_BATCH_GRAPH): one variant's grid is often too
 * small to fill the 256 compute units alone. */
#define ADI_BATCH_ONE_STREAM 2

/* Group count bound problems (any methods, dtypes, sizes, orders) of the
 * current device.  The batch keeps the pointers, not the problems: they must
 * stay alive and bound while the batch is used.  Work is queued on
 * hip_stream (NULL = null stream; ADI_BATCH_GRAPH needs a created stream),
 * ordered after each problem's own stream and before later work on it.
 * flags: 0 or a combination of ADI_BATCH_GRAPH and ADI_BATCH_ONE_STREAM. */
int adi_batch_create(adi_problem* const* problems, int count, void* hip_stream, int flags,
                     adi_batch** out);

/* Queue nsteps steps of every problem of the batch (each problem ends at
 * its own time level m + nsteps, as after adi_run(problem, nsteps); a
 * problem may have been run alone or in other batches before).  The call
 * allocates a descriptor buffer on first use and blocks until the previous
 * run of the batch has finished.  adi_get_state on a problem waits for the
 * batch's work through the problem's stream. */
int adi_batch_run(adi_batch* b, int64_t nsteps);

/* Wait for the batch's queued work. */
int adi_batch_sync(adi_batch* b);

/* Number of grouped line-pass launches of the last adi_batch_run (graph
 * replays included; the per-problem set-up and explicit passes excluded). */
int adi_batch_launches(const adi_batch* b, int64_t* n);

/* Free the batch (not its problems). */
int adi_batch_destroy(adi_batch* b);

/* ---- Served problems ---------------------------------------------------
 * A server takes requests (a problem description, host arrays and a step
 * count) at any time and returns each result in the request's own host
 * arrays, or, for requests flagged ADI_REQUEST_HOLD, keeps it on the device
 * until adi_fetch copies it out.  Every tick advances all admitted problems by one step with the
 * grouped launches of the batched form (bit-for-bit the result of running
 * the problem alone).  Device memory is one arena of hbm_budget_bytes
 * allocated by adi_server_create; a request is admitted, first come first
 * served, once its arrays and workspace fit and fewer than max_active are
 * running.  The server owns three HIP streams and three host threads (a
 * scheduler, an uploader and a downloader); every adi_server_* call and
 * adi_submit / adi_poll / adi_wait may come from any host thread.  Pinned
 * host arrays (hipHostMalloc, torch pin_memory) make the copies true DMA;
 * pageable arrays work but keep the transfer threads busy longer. */
typedef struct adi_server adi_server;

typedef struct adi_server_params {
    uint32_t struct_size;
    int32_t max_active;          /* problems advanced together, at most */
    uint64_t hbm_budget_bytes;   /* device arena (arrays + workspaces) */
} adi_server_params;

/* adi_request.flags: keep the result in the server's device memory after
 * completion (the request's host arrays are then inputs only) until
 * adi_fetch; held results count against hbm_budget_bytes. */
#define ADI_REQUEST_HOLD 1

typedef struct adi_request {
    uint32_t struct_size;        /* sizeof(adi_request) */
    int32_t flags;               /* 0 or ADI_REQUEST_HOLD */
    adi_params params;           /* as for adi_create; order, sweeps, source included */
    int64_t nsteps;              /* >= 1 */
    void *U, *V, *W;             /* host arrays (shapes of adi_bind) with time level 0,
                                    overwritten with time level nsteps when the request
                                    completes (unless ADI_REQUEST_HOLD) */
    const void *K, *Rv, *Rw;     /* host arrays or NULL (kappa0 / rinv0) */
    int64_t ld[6];               /* leading dimensions (elements) of U, V, W, K, Rv, Rw;
                                    0 = densely packed */
} adi_request;

typedef struct adi_server_stats {
    int64_t queued, active, done, peak_active, ticks, launches;
    uint64_t arena_used;         /* bytes */
} adi_server_stats;

/* Defaults: 16 GiB budget, 256 active problems. */
int adi_server_params_init(adi_server_params* p);

/* Create a server on the current device (allocates the arena). */
int adi_server_create(const adi_server_params* p, adi_server** out);

/* Queue a request; *ticket identifies it.  The host arrays must stay valid
 * and untouched until the request is done.  Validation is that of
 * adi_create plus: the arrays and workspace must fit in the budget. */
int adi_submit(adi_server* s, const adi_request* r, uint64_t* ticket);

/* *state: 0 queued, 1 running, 2 done.  Returns the request's status once
 * done (ADI_OK or the error that failed it). */
int adi_poll(adi_server* s, uint64_t ticket, int* state);

/* Block until the request is done; returns its status. */
int adi_wait(adi_server* s, uint64_t ticket);

/* Block until the request is done and copy its result (time level nsteps)
 * into the host arrays U, V, W, laid out like the request's arrays (same
 * shapes and leading dimensions; NULL skips an array).  A held request
 * (ADI_REQUEST_HOLD) is copied from device memory, which is then released:
 * it can be fetched once (ADI_EINVAL afterwards).  Otherwise the result is
 * copied from the request's own host arrays.  Returns the request's status. */
int adi_fetch(adi_server* s, uint64_t ticket, void* U, void* V, void* W);

/* Seconds since the server's creation (steady clock) at submission, at the
 * first step and at completion (results in the host arrays). */
int adi_request_times(adi_server* s, uint64_t ticket, double* t_submit, double* t_start, double* t_done);

int adi_server_get_stats(adi_server* s, adi_server_stats* st);

/* Wait for every submitted request, then stop the threads and free the
 * arena, streams and staging buffers. */
int adi_server_destroy(adi_server* s);

/* ---- Measurement ------------------------------------------------------
 * The achievable HBM ceiling of a line pass (Section 5 compares kernel
 * times; the roofline needs the device's reachable rate, not only its
 * nominal peak).  A pass streams three arrays in and two out, each element
 * once; this call queues one kernel that does the same with trivial
 * arithmetic: x = a - c b, y = b - a over n elements of dtype (ADI_FP32 or
 * ADI_FP64) in 16-byte vectors.  The five device arrays are 16-byte aligned
 * and n times the element size is a multiple of 16 (else ADI_EINVAL); x and
 * y must not overlap the inputs.  Queued on hip_stream, no synchronisation:
 * time it with events on that stream. */
int adi_stream_ceiling(int dtype, const void* a, const void* b, const void* c, void* x, void* y, int64_t n,
                       void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ADI_H */
