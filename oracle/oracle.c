/*
 * FP64 CPU oracle for the Peaceman-Rachford ADI step of the 2-D
 * velocity-pressure acoustic system (Otero, Rojas, Moya, Castillo,
 * arXiv 2006.07583), in both spatial variants of the paper:
 *   - nodal compact finite differences (CFD, Section 2.1, Appendix A),
 *   - staggered mimetic finite differences (MFD, Section 2.2, Appendix B).
 *
 * TEST INFRASTRUCTURE.  This file is the plain, slow reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Conventions (all arrays row-major, row = y index j, column = x index i):
 *   CFD: U, V, W, K, Rv, Rw are (ny+1) x (nx+1) nodal arrays.
 *   MFD: U, K are (ny+2) x (nx+2)   (X_cb x Y_cb: faces + cell centres),
 *        V, Rv are (ny+2) x (nx+1)   (X_n x Y_cb),
 *        W, Rw are (ny+1) x (nx+2)   (X_cb x Y_n).
 *   K holds kappa at pressure points, Rv / Rw hold 1/rho at the velocity
 *   points.  A NULL material pointer means the constant kappa0 / rinv0.
 *   Interior pressure points: CFD 1..n-1, MFD 1..n in each direction.
 *   Boundary pressure values are Dirichlet data: read, never written.
 *
 * Method (Section 2.1, eqs. CN, PR two-stage split, adiSolve, adiSolve2;
 * Algorithms 1-4).  With a = dt/2, one step is two stages.  Each stage first
 * applies the explicit part of the split in one direction e and then solves
 * the coupled (pressure, velocity) line systems of the other direction d by
 * a fixed number of fixed-point sweeps:
 *   explicit (direction e):  R_U = U - a (K .* Dbar_e(vel_e) - F)
 *                            vel_e <- vel_e - a R_e .* G_e(U)
 *   implicit (direction d):  vel_0 = vel_d
 *                            repeat K times:
 *                              Ubar_k  = R_U - a K .* Dbar_d(vel_{k-1})
 *                              vel_k   = vel_d - a R_d .* G_d([U_bnd, Ubar_k, U_bnd])
 *                            U <- Ubar_K, vel_d <- vel_K
 * where G is the pressure-to-velocity derivative (CFD: P^-1 Q, MFD: G4) and
 * Dbar the velocity-to-pressure derivative (CFD: Pbar^-1 Qbar, MFD: D4).
 * Order 0 (the paper's): stage (d=x, e=y, F^m) then (d=y, e=x, F^{m+1}),
 * i.e. A and W* first, then ADI-rows, then C and V^{m+1}, then ADI-columns.
 * Order 1 swaps the roles of x and y.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *   - the reduced CFD operators are (n-1)x(n-1) and (n-1)x(n+1) (Appendix A
 *     prints (N-2)); A and C live on the interior pressure points;
 *   - A and C are taken in pressure scale (the form of Algorithm 3), which
 *     equals the eq. adiSolve form for constant kappa;
 *   - D4 and G4 carry a 1/h factor; their last rows are the centro-skew
 *     mirror images of the printed first rows;
 *   - W* and V^{m+1} apply G to the full pressure line (boundary values
 *     included);
 *   - the second-stage iteration starts from W* (the algorithm text), not W^m;
 *   - exactly `sweeps` fixed-point sweeps per stage (oracle_run), or the
 *     tolerance test of Algorithms 3 and 4 (oracle_run_eps): after sweep k,
 *     k >= min_sweeps, the change of the whole stage
 *       ||Ubar_k - Ubar_{k-1}||_F + ||vel_k - vel_{k-1}||_F
 *     is compared with eps; the first count that passes is rounded up to an
 *     even count (odd counts amplify the unconverged modes) and `sweeps` is
 *     the cap.  The first test comes after the second sweep at the earliest,
 *     as the paper's GPU codes also run a minimum number of sweeps first;
 *   - direct mode (oracle_run_direct): each stage's line systems solved
 *     exactly, the limit of infinitely many sweeps, which is the
 *     Peaceman-Rachford step itself (eqs. ecua2:PR, ecua3:PR2) with no
 *     fixed-point error and no step-size limit from the iteration;
 *   - time-dependent Dirichlet data and a distributed forcing
 *     (oracle_run_forced; the heterogeneous tests of Section 4, eq.
 *     harmonic_hetero): u = Ub(x, y) s_b(t) on the walls, f = F(x, y) s_F(t)
 *     in the interior.  The paper does not say which wall values the
 *     intermediate level U* carries.  Reading taken: the explicit part of the
 *     first stage reads the walls along its lines at t^m, the implicit part
 *     of the second stage at t^{m+1}; the walls across the first stage's
 *     lines (x = 0, 1 in order 0) carry the pressure component of the
 *     split's own identity for the intermediate level,
 *       U* = (1/2)(I + a A2) U^m + (1/2)(I - a A2) U^{m+1} + (a/2)(F^m - F^{m+1}),
 *     evaluated on the wall data: with rho w_t = -u_y the A2 terms become
 *     -a^2 c^2 d_yy u_b at t^m + dt/2 (d_yy the second difference along the
 *     wall, c^2 = kappa / rho at the wall point), so
 *       U*_wall = (u_b^m + u_b^{m+1}) / 2 - a^2 c^2 d_yy u_b(t^m + dt/2)
 *                 + (a/2)(f^m - f^{m+1}).
 *     Without the last two terms the wall values are off by O(dt^2) each
 *     step and the error converges at first order only.  F^m enters the
 *     first stage and F^{m+1} the second, as the point source does.
 *
 * Built with -O2 -ffp-contract=off and no fast-math so every operation is
 * rounded as written.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_CFD 0
#define ORC_MFD 1

/* A time signal: kind 1 Ricker amp (1 - 2 x^2) exp(-x^2), x = pi f0 (t - t0);
 * kind 2 cosine amp cos(2 pi f0 (t - t0)); kind 0 zero. */
typedef struct {
    int32_t kind, pad;
    double f0, t0, amp;
} oracle_signal;

typedef struct {
    int32_t method;   /* 0 = CFD, 1 = MFD */
    int32_t order;    /* 0 = x-implicit stage first, 1 = y-implicit first */
    int32_t nx, ny;   /* cells per direction */
    int32_t sweeps;   /* fixed-point sweeps per stage */
    int32_t src_i, src_j; /* pressure index of the point source, -1 = none */
    int32_t threads;  /* OpenMP threads, <= 0 = runtime default */
    double h, dt, t0; /* spacing, time step, time of step 0 */
    double src_f0, src_t0, src_amp; /* Ricker peak frequency, delay, amplitude */
    double kappa0, rinv0;           /* constants used when K / R are NULL */
} oracle_params;

/* ------------------------------------------------------------------ */
/* Appendix A: compact operators P4, Q4 and their reduced forms.       */
/* ------------------------------------------------------------------ */

/* Tridiagonal matrix of order m given by its three diagonals
 * (sub[0] and sup[m-1] unused). */
typedef struct {
    int m;
    double *sub, *diag, *sup;
    /* LU without pivoting (Section 2.1, complexity analysis: no pivoting):
     * L unit lower bidiagonal with multipliers mul[i], U upper bidiagonal
     * with pivots piv[i] and superdiagonal sup[i]. */
    double *mul, *piv;
} tridiag;

static void tridiag_alloc(tridiag* t, int m) {
    t->m = m;
    t->sub = calloc((size_t)m, sizeof(double));
    t->diag = calloc((size_t)m, sizeof(double));
    t->sup = calloc((size_t)m, sizeof(double));
    t->mul = calloc((size_t)m, sizeof(double));
    t->piv = calloc((size_t)m, sizeof(double));
}

static void tridiag_free(tridiag* t) {
    free(t->sub); free(t->diag); free(t->sup); free(t->mul); free(t->piv);
    memset(t, 0, sizeof(*t));
}

/* Doolittle LU of a tridiagonal matrix, no pivoting. */
static void tridiag_factor(tridiag* t) {
    t->piv[0] = t->diag[0];
    t->mul[0] = 0.0;
    for (int i = 1; i < t->m; ++i) {
        t->mul[i] = t->sub[i] / t->piv[i - 1];
        t->piv[i] = t->diag[i] - t->mul[i] * t->sup[i - 1];
    }
}

/* Forward then backward substitution, in place (rhs -> solution). */
static void tridiag_solve(const tridiag* t, double* x) {
    for (int i = 1; i < t->m; ++i) x[i] = x[i] - t->mul[i] * x[i - 1];
    x[t->m - 1] = x[t->m - 1] / t->piv[t->m - 1];
    for (int i = t->m - 2; i >= 0; --i) x[i] = (x[i] - t->sup[i] * x[i + 1]) / t->piv[i];
}

/* P4, (n+1)x(n+1): rows [6 18], [1 4 1], ..., [18 6]. */
static void build_P(tridiag* t, int n) {
    tridiag_alloc(t, n + 1);
    for (int i = 0; i <= n; ++i) { t->sub[i] = 1.0; t->diag[i] = 4.0; t->sup[i] = 1.0; }
    t->diag[0] = 6.0; t->sup[0] = 18.0;
    t->sub[n] = 18.0; t->diag[n] = 6.0;
    t->sub[0] = 0.0; t->sup[n] = 0.0;
    tridiag_factor(t);
}

/* Reduced Pbar4 on interior nodes 1..n-1, order n-1: rows [6 6], [1 4 1],
 * ..., [6 6].  The first row is (row 0) - 6 (row 1) of P4 with the sign
 * flipped, which removes the boundary derivative (Appendix A). */
static void build_Pbar(tridiag* t, int n) {
    int m = n - 1;
    tridiag_alloc(t, m);
    for (int i = 0; i < m; ++i) { t->sub[i] = 1.0; t->diag[i] = 4.0; t->sup[i] = 1.0; }
    t->diag[0] = 6.0; t->sup[0] = 6.0;
    t->sub[m - 1] = 6.0; t->diag[m - 1] = 6.0;
    t->sub[0] = 0.0; t->sup[m - 1] = 0.0;
    tridiag_factor(t);
}

/* Q4 f, f and out of length n+1 (nodes 0..n). */
static void apply_Q(int n, double h, const double* f, double* out) {
    out[0] = (-17.0 * f[0] + 9.0 * f[1] + 9.0 * f[2] - f[3]) / h;
    for (int i = 1; i < n; ++i) out[i] = 3.0 * (f[i + 1] - f[i - 1]) / h;
    out[n] = (f[n - 3] - 9.0 * f[n - 2] - 9.0 * f[n - 1] + 17.0 * f[n]) / h;
}

/* Qbar4 f, f of length n+1, out of length n-1 (out[k] is node k+1). */
static void apply_Qbar(int n, double h, const double* f, double* out) {
    out[0] = (-f[0] - 9.0 * f[1] + 9.0 * f[2] + f[3]) / h;
    for (int i = 2; i <= n - 2; ++i) out[i - 1] = 3.0 * (f[i + 1] - f[i - 1]) / h;
    out[n - 2] = (-f[n - 3] - 9.0 * f[n - 2] + 9.0 * f[n - 1] + f[n]) / h;
}

/* ------------------------------------------------------------------ */
/* Appendix B: mimetic operators D4 (n x (n+1)) and G4 ((n+1)x(n+2)).  */
/* ------------------------------------------------------------------ */

static const double D4_ROW0[6] = {
    -4751.0 / 5192.0, 909.0 / 1298.0, 6091.0 / 15576.0,
    -1165.0 / 5192.0, 129.0 / 2596.0, -25.0 / 15576.0};
static const double G4_ROW0[6] = {
    -47888.0 / 14245.0, 1790.0 / 407.0, -14545.0 / 9768.0,
    8997.0 / 16280.0, -2335.0 / 22792.0, 25.0 / 9768.0};
static const double G4_ROW1[5] = {
    16.0 / 105.0, -31.0 / 24.0, 29.0 / 24.0, -3.0 / 40.0, 1.0 / 168.0};
static const double SG4[4] = {1.0 / 24.0, -9.0 / 8.0, 9.0 / 8.0, -1.0 / 24.0};

/* Dense D4 entry (row r, column c), 1/h applied. */
static double D4_entry(int n, double h, int r, int c) {
    if (r == 0) return (c <= 5) ? D4_ROW0[c] / h : 0.0;
    if (r == n - 1) { int cc = n - c; return (cc >= 0 && cc <= 5) ? -D4_ROW0[cc] / h : 0.0; }
    int k = c - (r - 1);
    return (k >= 0 && k <= 3) ? SG4[k] / h : 0.0;
}

/* Dense G4 entry (row r, column c), 1/h applied. */
static double G4_entry(int n, double h, int r, int c) {
    if (r == 0) return (c <= 5) ? G4_ROW0[c] / h : 0.0;
    if (r == 1) return (c <= 4) ? G4_ROW1[c] / h : 0.0;
    if (r == n) { int cc = n + 1 - c; return (cc >= 0 && cc <= 5) ? -G4_ROW0[cc] / h : 0.0; }
    if (r == n - 1) { int cc = n + 1 - c; return (cc >= 0 && cc <= 4) ? -G4_ROW1[cc] / h : 0.0; }
    int k = c - (r - 1);
    return (k >= 0 && k <= 3) ? SG4[k] / h : 0.0;
}

/* D4 v: v on nodes 0..n, out[r] at cell centre r+1/2, r = 0..n-1. */
static void apply_D4(int n, double h, const double* v, double* out) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) s += D4_ROW0[c] * v[c];
    out[0] = s / h;
    for (int r = 1; r <= n - 2; ++r)
        out[r] = (SG4[0] * v[r - 1] + SG4[1] * v[r] + SG4[2] * v[r + 1] + SG4[3] * v[r + 2]) / h;
    s = 0.0;
    for (int c = 0; c < 6; ++c) s += D4_ROW0[c] * v[n - c];
    out[n - 1] = -s / h;
}

/* G4 u: u on X_cb indices 0..n+1, out[r] at node r, r = 0..n. */
static void apply_G4(int n, double h, const double* u, double* out) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) s += G4_ROW0[c] * u[c];
    out[0] = s / h;
    s = 0.0;
    for (int c = 0; c < 5; ++c) s += G4_ROW1[c] * u[c];
    out[1] = s / h;
    for (int r = 2; r <= n - 2; ++r)
        out[r] = (SG4[0] * u[r - 1] + SG4[1] * u[r] + SG4[2] * u[r + 1] + SG4[3] * u[r + 2]) / h;
    s = 0.0;
    for (int c = 0; c < 5; ++c) s += G4_ROW1[c] * u[n + 1 - c];
    out[n - 1] = -s / h;
    s = 0.0;
    for (int c = 0; c < 6; ++c) s += G4_ROW0[c] * u[n + 1 - c];
    out[n] = -s / h;
}

/* ------------------------------------------------------------------ */
/* The two line derivatives of each method along one grid direction.   */
/* ------------------------------------------------------------------ */

typedef struct {
    int method, n;
    double h;
    tridiag P, Pbar;      /* CFD only */
    double* work;         /* scratch of length n+2 per call site (not shared) */
} line_ops;

static void line_ops_init(line_ops* o, int method, int n, double h) {
    memset(o, 0, sizeof(*o));
    o->method = method; o->n = n; o->h = h;
    if (method == ORC_CFD) { build_P(&o->P, n); build_Pbar(&o->Pbar, n); }
}

static void line_ops_free(line_ops* o) {
    if (o->method == ORC_CFD) { tridiag_free(&o->P); tridiag_free(&o->Pbar); }
}

/* Number of pressure values on a full line (boundary included). */
static int n_ufull(int method, int n) { return method == ORC_CFD ? n + 1 : n + 2; }
/* Number of interior pressure values on a line. */
static int n_uint(int method, int n) { return method == ORC_CFD ? n - 1 : n; }

/* Pressure -> velocity derivative: u has u_full values, out n+1 values. */
static void deriv_G(const line_ops* o, const double* u, double* out) {
    if (o->method == ORC_CFD) {
        apply_Q(o->n, o->h, u, out);          /* P out = Q u */
        tridiag_solve(&o->P, out);
    } else {
        apply_G4(o->n, o->h, u, out);
    }
}

/* Velocity -> pressure derivative: v has n+1 values, out u_int values. */
static void deriv_D(const line_ops* o, const double* v, double* out) {
    if (o->method == ORC_CFD) {
        apply_Qbar(o->n, o->h, v, out);       /* Pbar out = Qbar v */
        tridiag_solve(&o->Pbar, out);
    } else {
        apply_D4(o->n, o->h, v, out);
    }
}

/* ------------------------------------------------------------------ */
/* Strided 2-D views.                                                   */
/* ------------------------------------------------------------------ */

typedef struct { double* p; int rows, cols; } field;   /* dense row-major */

/* Element (line l, position k) of a field seen along direction dir
 * (0 = x: lines are rows; 1 = y: lines are columns). */
static inline double* at(const field* f, int dir, int line, int k) {
    return dir == 0 ? f->p + (size_t)line * f->cols + k : f->p + (size_t)k * f->cols + line;
}

static void gather(const field* f, int dir, int line, int k0, int len, double* dst) {
    for (int k = 0; k < len; ++k) dst[k] = *at(f, dir, line, k0 + k);
}

static void scatter(field* f, int dir, int line, int k0, int len, const double* src) {
    for (int k = 0; k < len; ++k) *at(f, dir, line, k0 + k) = src[k];
}

/* Material value at a point, constant when the array is absent. */
static inline double mat(const field* f, int dir, int line, int k, double c) {
    return f->p ? *at(f, dir, line, k) : c;
}

/* Ricker wavelet of the point source (peak frequency f0, delay t0). */
static double ricker(double t, double f0, double t0, double amp) {
    const double pi = 3.14159265358979323846;
    double x = pi * f0 * (t - t0);
    x = x * x;
    return amp * (1.0 - 2.0 * x) * exp(-x);
}

typedef struct {
    int method, nx, ny;
    double a;                  /* dt / 2 */
    double kappa0, rinv0;
    field U, V, W, K, Rv, Rw;  /* Rv/Rw/K .p may be NULL */
    line_ops ox, oy;
    double* RU;                /* interior pressure right-hand side */
    int src_i, src_j;
    double h;
    /* damping layers (oracle_run_damped): rate d0 (1 - dist / width)^2 within
     * `width` cells of each wall whose bit is set in dmask (1: x = 0, 2: x = 1,
     * 4: y = 0, 8: y = 1); width 0: the uniform rate d0 in every direction
     * with a bit set */
    double d0, dwidth;
    int dmask;
} problem;

/* Damping rate at index k along direction dir: pressure points (vel = 0)
 * or velocity points (vel = 1), from the distances to the two walls. */
static double damp_rate(const problem* pb, int dir, int vel, int k) {
    const int bits = (pb->dmask >> (2 * dir)) & 3;
    if (!bits || pb->d0 == 0.0) return 0.0;
    if (pb->dwidth <= 0.0) return pb->d0;
    const int n = dir == 0 ? pb->nx : pb->ny;
    double lo;
    if (vel || pb->method == ORC_CFD) lo = k;
    else lo = k == 0 ? 0.0 : (k == n + 1 ? (double)n : k - 0.5);
    const double hi = n - lo;
    double r = 0.0;
    if (bits & 1) { const double x = 1.0 - lo / pb->dwidth; if (x > 0.0) r += pb->d0 * x * x; }
    if (bits & 2) { const double x = 1.0 - hi / pb->dwidth; if (x > 0.0) r += pb->d0 * x * x; }
    return r;
}

/* One stage of the Peaceman-Rachford split with the implicit direction d
 * and explicit direction e = 1-d, forcing value F at the source point.
 * Stage (d = x) is eq. ecua2:PR solved through eqs. ecua1:ADI / adiSolve;
 * stage (d = y) is eq. ecua3:PR solved through eq. adiSolve2. */
static void implicit_eps(problem* pb, int d, int sweeps, int nthreads, double eps, int min_sweeps, int32_t* used);
static void implicit_direct(problem* pb, int d, int nthreads);

static void stage(problem* pb, int d, double Fsrc, const double* Ffield, double Fscale, int sweeps,
                  int nthreads, double eps, int min_sweeps, int32_t* used) {
    const int e = 1 - d;
    const int method = pb->method;
    const double a = pb->a;
    const int nd = d == 0 ? pb->nx : pb->ny;   /* cells along the implicit lines */
    const int ne = e == 0 ? pb->nx : pb->ny;   /* cells along the explicit lines */
    const line_ops* od = d == 0 ? &pb->ox : &pb->oy;
    const line_ops* oe = e == 0 ? &pb->ox : &pb->oy;
    field* vel_d = d == 0 ? &pb->V : &pb->W;
    field* vel_e = e == 0 ? &pb->V : &pb->W;
    const field* R_d = d == 0 ? &pb->Rv : &pb->Rw;
    const field* R_e = e == 0 ? &pb->Rv : &pb->Rw;
    const int niu_d = n_uint(method, nd), niu_e = n_uint(method, ne);
    const int nfu_d = n_ufull(method, nd), nfu_e = n_ufull(method, ne);
    /* interior pressure array RU is stored row-major over interior (j, i) */
    const int ni_x = n_uint(method, pb->nx);
    double* RU = pb->RU;
#define RU_AT(jj, ii) RU[(size_t)(jj) * ni_x + (ii)]

    /* ---- explicit part along direction e: for every interior line of e,
     *      i.e. every interior index l along direction d ---- */
#pragma omp parallel num_threads(nthreads)
    {
        double* ubuf = malloc(sizeof(double) * (size_t)(nfu_e + 2));
        double* vbuf = malloc(sizeof(double) * (size_t)(ne + 2));
        double* tmp = malloc(sizeof(double) * (size_t)(ne + 2));
#pragma omp for schedule(static)
        for (int l = 1; l <= niu_d; ++l) {
            /* R_U = U - a (K .* Dbar_e(vel_e) - F) on interior points of this line */
            gather(vel_e, e, l, 0, ne + 1, vbuf);
            deriv_D(oe, vbuf, tmp);
            for (int k = 1; k <= niu_e; ++k) {
                double kap = mat(&pb->K, e, l, k, pb->kappa0);
                int j = e == 0 ? l : k, i = e == 0 ? k : l;
                double f = (i == pb->src_i && j == pb->src_j) ? Fsrc : 0.0;
                if (Ffield) f += Fscale * Ffield[(size_t)j * pb->U.cols + i];
                const double g = 1.0 - a * damp_rate(pb, e, 0, k);   /* damping along e */
                RU_AT(j - 1, i - 1) = g * *at(&pb->U, e, l, k) - a * (kap * tmp[k - 1] - f);
            }
            /* vel_e <- vel_e - a R_e .* G_e(U) (full pressure line) */
            gather(&pb->U, e, l, 0, nfu_e, ubuf);
            deriv_G(oe, ubuf, tmp);
            for (int k = 0; k <= ne; ++k) {
                double r = mat(R_e, e, l, k, pb->rinv0);
                *at(vel_e, e, l, k) = (1.0 - a * damp_rate(pb, e, 1, k)) * vbuf[k] - a * r * tmp[k];
            }
        }
        free(ubuf); free(vbuf); free(tmp);
    }

    if (sweeps == 0) {
        implicit_direct(pb, d, nthreads);
        if (used) *used = 0;
        return;
    }
    if (eps > 0.0) {
        implicit_eps(pb, d, sweeps, nthreads, eps, min_sweeps, used);
        return;
    }
    if (used) *used = sweeps;

    /* ---- implicit part along direction d: fixed-point sweeps per line ---- */
#pragma omp parallel num_threads(nthreads)
    {
        double* ubuf = malloc(sizeof(double) * (size_t)(nfu_d + 2));
        double* vold = malloc(sizeof(double) * (size_t)(nd + 2));
        double* vk = malloc(sizeof(double) * (size_t)(nd + 2));
        double* tmp = malloc(sizeof(double) * (size_t)(nd + 2));
        double* rhs = malloc(sizeof(double) * (size_t)(nfu_d + 2));
#pragma omp for schedule(static)
        for (int l = 1; l <= niu_e; ++l) {
            gather(vel_d, d, l, 0, nd + 1, vold);
            memcpy(vk, vold, sizeof(double) * (size_t)(nd + 1));   /* vel_0 = vel_d */
            gather(&pb->U, d, l, 0, nfu_d, ubuf);                   /* boundary values */
            for (int k = 1; k <= niu_d; ++k) {
                int j = d == 0 ? l : k, i = d == 0 ? k : l;
                rhs[k] = RU_AT(j - 1, i - 1);
            }
            for (int s = 0; s < sweeps; ++s) {
                /* Ubar_k = R_U - a K .* Dbar_d(vel_{k-1}) */
                deriv_D(od, vk, tmp);
                for (int k = 1; k <= niu_d; ++k) {
                    double kap = mat(&pb->K, d, l, k, pb->kappa0);
                    ubuf[k] = (rhs[k] - a * kap * tmp[k - 1]) / (1.0 + a * damp_rate(pb, d, 0, k));
                }
                /* vel_k = vel_d - a R_d .* G_d(U_k) */
                deriv_G(od, ubuf, tmp);
                for (int k = 0; k <= nd; ++k) {
                    double r = mat(R_d, d, l, k, pb->rinv0);
                    vk[k] = (vold[k] - a * r * tmp[k]) / (1.0 + a * damp_rate(pb, d, 1, k));
                }
            }
            scatter(&pb->U, d, l, 1, niu_d, ubuf + 1);
            scatter(vel_d, d, l, 0, nd + 1, vk);
        }
        free(ubuf); free(vold); free(vk); free(tmp); free(rhs);
    }
#undef RU_AT
}

/* Implicit part along direction d with the tolerance test (Algorithms 3
 * and 4): every line advances one sweep at a time, and after each sweep the
 * Frobenius norms of the changes of the whole stage are summed and tested. */
static void implicit_eps(problem* pb, int d, int sweeps, int nthreads, double eps, int min_sweeps, int32_t* used) {
    const int e = 1 - d;
    const int method = pb->method;
    const double a = pb->a;
    const int nd = d == 0 ? pb->nx : pb->ny;
    const line_ops* od = d == 0 ? &pb->ox : &pb->oy;
    field* vel_d = d == 0 ? &pb->V : &pb->W;
    const field* R_d = d == 0 ? &pb->Rv : &pb->Rw;
    const int ne = e == 0 ? pb->nx : pb->ny;
    const int niu_d = n_uint(method, nd), niu_e = n_uint(method, ne);
    const int nfu_d = n_ufull(method, nd);
    const int ni_x = n_uint(method, pb->nx);
    const double* RU = pb->RU;
    /* state of every line: interior pressure iterate, velocity iterate, and
     * the velocity the stage started from */
    double* Ub = calloc((size_t)niu_e * (size_t)niu_d, sizeof(double));
    double* Vk = malloc(sizeof(double) * (size_t)niu_e * (size_t)(nd + 1));
    double* V0 = malloc(sizeof(double) * (size_t)niu_e * (size_t)(nd + 1));
    for (int l = 1; l <= niu_e; ++l) {
        gather(vel_d, d, l, 0, nd + 1, V0 + (size_t)(l - 1) * (nd + 1));
        gather(vel_d, d, l, 0, nd + 1, Vk + (size_t)(l - 1) * (nd + 1));
    }
    int k = 0, last = sweeps;
    while (k < last) {
        double su = 0.0, sv = 0.0;
#pragma omp parallel num_threads(nthreads) reduction(+ : su, sv)
        {
            double* ubuf = malloc(sizeof(double) * (size_t)(nfu_d + 2));
            double* tmp = malloc(sizeof(double) * (size_t)(nd + 2));
#pragma omp for schedule(static)
            for (int l = 1; l <= niu_e; ++l) {
                double* ub = Ub + (size_t)(l - 1) * niu_d;
                double* vk = Vk + (size_t)(l - 1) * (nd + 1);
                const double* v0 = V0 + (size_t)(l - 1) * (nd + 1);
                /* Ubar_k = R_U - a K .* Dbar_d(vel_{k-1}) */
                deriv_D(od, vk, tmp);
                gather(&pb->U, d, l, 0, nfu_d, ubuf);   /* boundary values */
                for (int q = 1; q <= niu_d; ++q) {
                    int j = d == 0 ? l : q, i = d == 0 ? q : l;
                    double kap = mat(&pb->K, d, l, q, pb->kappa0);
                    double un = RU[(size_t)(j - 1) * ni_x + (i - 1)] - a * kap * tmp[q - 1];
                    su += (un - ub[q - 1]) * (un - ub[q - 1]);
                    ub[q - 1] = un;
                    ubuf[q] = un;
                }
                /* vel_k = vel_d - a R_d .* G_d(U_k) */
                deriv_G(od, ubuf, tmp);
                for (int q = 0; q <= nd; ++q) {
                    double r = mat(R_d, d, l, q, pb->rinv0);
                    double vn = v0[q] - a * r * tmp[q];
                    sv += (vn - vk[q]) * (vn - vk[q]);
                    vk[q] = vn;
                }
            }
            free(ubuf); free(tmp);
        }
        ++k;
        /* the change of the first sweep has no earlier iterate of Ubar */
        if (last == sweeps && k >= min_sweeps && k >= 2 && sqrt(su) + sqrt(sv) <= eps)
            last = k + (k & 1);   /* round up to even */
    }
    for (int l = 1; l <= niu_e; ++l) {
        scatter(&pb->U, d, l, 1, niu_d, Ub + (size_t)(l - 1) * niu_d);
        scatter(vel_d, d, l, 0, nd + 1, Vk + (size_t)(l - 1) * (nd + 1));
    }
    if (used) *used = last;
    free(Ub); free(Vk); free(V0);
}

/* Solve the dense m x m system M x = b in place by Gaussian elimination
 * with partial pivoting (row interchanges); M is row-major and destroyed,
 * b becomes x.  Returns -1 for an exactly singular matrix. */
static int dense_solve(int m, double* M, double* b) {
    for (int k = 0; k < m; ++k) {
        int p = k;
        for (int i = k + 1; i < m; ++i)
            if (fabs(M[(size_t)i * m + k]) > fabs(M[(size_t)p * m + k])) p = i;
        if (M[(size_t)p * m + k] == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < m; ++j) {
                double t = M[(size_t)k * m + j];
                M[(size_t)k * m + j] = M[(size_t)p * m + j];
                M[(size_t)p * m + j] = t;
            }
            double t = b[k]; b[k] = b[p]; b[p] = t;
        }
        for (int i = k + 1; i < m; ++i) {
            double l = M[(size_t)i * m + k] / M[(size_t)k * m + k];
            if (l == 0.0) continue;
            for (int j = k; j < m; ++j) M[(size_t)i * m + j] -= l * M[(size_t)k * m + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j < m; ++j) s -= M[(size_t)i * m + j] * b[j];
        b[i] = s / M[(size_t)i * m + i];
    }
    return 0;
}

/* Implicit part along direction d solved exactly (the limit of infinitely
 * many sweeps).  For each line the stage equations
 *     Ubar + a K .* Dbar_d(vel)                 = R_U
 *     vel  + a R_d .* G_d([U_bnd, Ubar, U_bnd]) = vel_d
 * are one linear system in the unknowns [Ubar (interior points), vel (all
 * nodes)].  Its matrix is assembled from the columns of Dbar_d and G_d,
 * obtained by applying the line derivatives to unit vectors, and the system
 * is solved by Gaussian elimination with partial pivoting.  The Dirichlet
 * values U_bnd move to the right-hand side. */
static void implicit_direct(problem* pb, int d, int nthreads) {
    const int e = 1 - d;
    const int method = pb->method;
    const double a = pb->a;
    const int nd = d == 0 ? pb->nx : pb->ny;
    const int ne = e == 0 ? pb->nx : pb->ny;
    const line_ops* od = d == 0 ? &pb->ox : &pb->oy;
    field* vel_d = d == 0 ? &pb->V : &pb->W;
    const field* R_d = d == 0 ? &pb->Rv : &pb->Rw;
    const int niu = n_uint(method, nd), niu_e = n_uint(method, ne);
    const int nfu = n_ufull(method, nd), nv = nd + 1;
    const int m = niu + nv;
    const int ni_x = n_uint(method, pb->nx);
    /* the line derivatives as dense matrices: Dm (niu x nv), Gm (nv x nfu) */
    double* Dm = calloc((size_t)niu * nv, sizeof(double));
    double* Gm = calloc((size_t)nv * nfu, sizeof(double));
    {
        double* unit = calloc((size_t)(nfu + nv), sizeof(double));
        double* col = calloc((size_t)(nfu + nv), sizeof(double));
        for (int c = 0; c < nv; ++c) {
            memset(unit, 0, sizeof(double) * (size_t)(nfu + nv));
            unit[c] = 1.0;
            deriv_D(od, unit, col);
            for (int r = 0; r < niu; ++r) Dm[(size_t)r * nv + c] = col[r];
        }
        for (int c = 0; c < nfu; ++c) {
            memset(unit, 0, sizeof(double) * (size_t)(nfu + nv));
            unit[c] = 1.0;
            deriv_G(od, unit, col);
            for (int r = 0; r < nv; ++r) Gm[(size_t)r * nfu + c] = col[r];
        }
        free(unit); free(col);
    }
#pragma omp parallel num_threads(nthreads)
    {
        double* M = malloc(sizeof(double) * (size_t)m * m);
        double* b = malloc(sizeof(double) * (size_t)m);
        double* ubuf = malloc(sizeof(double) * (size_t)nfu);
#pragma omp for schedule(dynamic)
        for (int l = 1; l <= niu_e; ++l) {
            memset(M, 0, sizeof(double) * (size_t)m * m);
            gather(&pb->U, d, l, 0, nfu, ubuf);
            /* pressure rows: Ubar_q + a K_q sum_c Dm[q][c] vel_c = R_U */
            for (int q = 0; q < niu; ++q) {
                int k = q + 1;
                int j = d == 0 ? l : k, i = d == 0 ? k : l;
                double kap = mat(&pb->K, d, l, k, pb->kappa0);
                M[(size_t)q * m + q] = 1.0;
                for (int c = 0; c < nv; ++c) M[(size_t)q * m + niu + c] = a * kap * Dm[(size_t)q * nv + c];
                b[q] = pb->RU[(size_t)(j - 1) * ni_x + (i - 1)];
            }
            /* velocity rows: vel_f + a R_f sum_q G[f][q+1] Ubar_q
             *                = vel_d_f - a R_f (G[f][0] U_0 + G[f][nfu-1] U_last) */
            for (int f = 0; f < nv; ++f) {
                double r = mat(R_d, d, l, f, pb->rinv0);
                size_t row = (size_t)(niu + f) * m;
                M[row + niu + f] = 1.0;
                for (int q = 0; q < niu; ++q) M[row + q] = a * r * Gm[(size_t)f * nfu + q + 1];
                double gb = Gm[(size_t)f * nfu] * ubuf[0] + Gm[(size_t)f * nfu + nfu - 1] * ubuf[nfu - 1];
                b[niu + f] = *at(vel_d, d, l, f) - a * r * gb;
            }
            dense_solve(m, M, b);
            scatter(&pb->U, d, l, 1, niu, b);
            scatter(vel_d, d, l, 0, nv, b + niu);
        }
        free(M); free(b); free(ubuf);
    }
    free(Dm); free(Gm);
}

static int check_params(const oracle_params* p) {
    if (!p) return -1;
    if (p->method != ORC_CFD && p->method != ORC_MFD) return -1;
    if (p->nx < 8 || p->ny < 8) return -1;
    if (p->sweeps < 0) return -1;   /* 0: direct (exact) line solves */
    if (!(p->h > 0.0) || !(p->dt > 0.0)) return -1;
    if (p->order != 0 && p->order != 1) return -1;
    return 0;
}

static double signal(const oracle_signal* g, double t) {
    const double pi = 3.14159265358979323846;
    if (!g || g->kind == 0) return 0.0;
    if (g->kind == 1) return ricker(t, g->f0, g->t0, g->amp);
    return g->amp * cos(2.0 * pi * g->f0 * (t - g->t0));
}

/* Wall values of U: the walls across the lines of direction d (the two
 * ends of every interior line along d) set to Ub times the boundary signal
 * at time t. */
static void set_walls(problem* pb, int d, const double* Ub, const oracle_signal* bs, double t) {
    const double sc = signal(bs, t);
    const int nd = d == 0 ? pb->nx : pb->ny, ne = d == 0 ? pb->ny : pb->nx;
    const int last = n_ufull(pb->method, nd) - 1;
    for (int l = 1; l <= n_uint(pb->method, ne); ++l) {
        double* a = at(&pb->U, d, l, 0);
        double* b = at(&pb->U, d, l, last);
        *a = sc * Ub[a - pb->U.p];
        *b = sc * Ub[b - pb->U.p];
    }
}

/* Coordinate of pressure index k along a direction of n cells. */
static double pcoord(int method, int n, double h, int k) {
    if (method == ORC_CFD) return k * h;
    return k == 0 ? 0.0 : (k == n + 1 ? n * h : (k - 0.5) * h);
}

/* The intermediate level's wall values across the lines of direction d (the
 * reading in the header): for each interior line l along d and each of its
 * two wall points, (u_b^m + u_b^{m+1})/2 - a^2 c^2 d_ll u_b(t_half) +
 * (a/2)(f^m - f^{m+1}), d_ll the three-point second difference along the
 * wall (across the lines), c^2 = kappa * (1/rho of the velocity along d at
 * that point). */
static void set_walls_half(problem* pb, int d, const double* Ub, const double* F, const oracle_signal* bs,
                           const oracle_signal* fs, double tm, double dt) {
    const int m = pb->method;
    const int nd = d == 0 ? pb->nx : pb->ny, ne = d == 0 ? pb->ny : pb->nx;
    const int last = n_ufull(m, nd) - 1;
    const double a = pb->a;
    const double sav = 0.5 * (signal(bs, tm) + signal(bs, tm + dt)), shalf = signal(bs, tm + 0.5 * dt);
    const double fdif = F ? 0.5 * a * (signal(fs, tm) - signal(fs, tm + dt)) : 0.0;
    const field* R = d == 0 ? &pb->Rv : &pb->Rw;
    for (int l = 1; l <= n_uint(m, ne); ++l) {
        const double ym = pcoord(m, ne, pb->h, l - 1), y0 = pcoord(m, ne, pb->h, l), yp = pcoord(m, ne, pb->h, l + 1);
        for (int e = 0; e < 2; ++e) {
            const int k = e ? last : 0;
            double* u = at(&pb->U, d, l, k);
            const size_t o = (size_t)(u - pb->U.p);
            const double um = Ub[at(&pb->U, d, l - 1, k) - pb->U.p], u0 = Ub[o], up = Ub[at(&pb->U, d, l + 1, k) - pb->U.p];
            const double dll = 2.0 * ((up - u0) / (yp - y0) - (u0 - um) / (y0 - ym)) / (yp - ym);
            const double c2 = mat(&pb->K, d, l, k, pb->kappa0) * mat(R, d, l, (e && m == ORC_MFD) ? k - 1 : k, pb->rinv0);
            *u = sav * u0 - a * a * c2 * dll * shalf + (F ? fdif * F[o] : 0.0);
        }
    }
}

static int run_impl(const oracle_params* p, double* U, double* V, double* W, const double* K,
                    const double* Rv, const double* Rw, int64_t nsteps, double eps, int min_sweeps,
                    int32_t* used, const double* F, const oracle_signal* fs, const oracle_signal* bs,
                    const double* damp) {
    if (check_params(p) || !U || !V || !W || nsteps < 0) return -1;
    problem pb;
    memset(&pb, 0, sizeof(pb));
    const int m = p->method, nx = p->nx, ny = p->ny;
    pb.method = m; pb.nx = nx; pb.ny = ny; pb.h = p->h;
    pb.a = 0.5 * p->dt;
    pb.kappa0 = p->kappa0; pb.rinv0 = p->rinv0;
    int fu_x = n_ufull(m, nx), fu_y = n_ufull(m, ny);
    pb.U = (field){U, fu_y, fu_x};
    pb.K = (field){(double*)K, fu_y, fu_x};
    pb.V = (field){V, fu_y, nx + 1};
    pb.Rv = (field){(double*)Rv, fu_y, nx + 1};
    pb.W = (field){W, ny + 1, fu_x};
    pb.Rw = (field){(double*)Rw, ny + 1, fu_x};
    if (m == ORC_CFD) {   /* CFD: all nodal (ny+1) x (nx+1) */
        pb.V.rows = pb.Rv.rows = ny + 1;
        pb.W.cols = pb.Rw.cols = nx + 1;
    }
    pb.src_i = p->src_i; pb.src_j = p->src_j;
    if (damp) {
        pb.d0 = damp[0];
        pb.dwidth = damp[1];
        pb.dmask = (int)damp[2];
    }
    line_ops_init(&pb.ox, m, nx, p->h);
    line_ops_init(&pb.oy, m, ny, p->h);
    pb.RU = calloc((size_t)n_uint(m, nx) * (size_t)n_uint(m, ny), sizeof(double));
    int nthreads = p->threads;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    const double h2 = p->h * p->h;
    const int has_src = p->src_i >= 0 && p->src_j >= 0;
    /* wall values at t = 0 scale the boundary signal */
    double* Ub = NULL;
    if (bs) {
        const size_t nu = (size_t)pb.U.rows * pb.U.cols;
        Ub = malloc(nu * sizeof(double));
        memcpy(Ub, U, nu * sizeof(double));
    }
    const int d1 = p->order == 0 ? 0 : 1, d2 = 1 - d1;   /* implicit directions of the two stages */
    for (int64_t s = 0; s < nsteps; ++s) {
        double tm = p->t0 + (double)s * p->dt, tm1 = p->t0 + (double)(s + 1) * p->dt;
        double Fm = has_src ? ricker(tm, p->src_f0, p->src_t0, p->src_amp) / h2 : 0.0;
        double Fm1 = has_src ? ricker(tm1, p->src_f0, p->src_t0, p->src_amp) / h2 : 0.0;
        int32_t* u0 = used ? used + 2 * s : NULL;
        int32_t* u1 = used ? used + 2 * s + 1 : NULL;
        if (Ub) {
            set_walls(&pb, d2, Ub, bs, tm);                    /* read by the first explicit part */
            set_walls_half(&pb, d1, Ub, F, bs, fs, tm, p->dt); /* the intermediate level */
        }
        stage(&pb, d1, Fm, F, signal(fs, tm), p->sweeps, nthreads, eps, min_sweeps, u0);
        if (Ub) set_walls(&pb, d2, Ub, bs, tm1);
        stage(&pb, d2, Fm1, F, signal(fs, tm1), p->sweeps, nthreads, eps, min_sweeps, u1);
        if (Ub) set_walls(&pb, d1, Ub, bs, tm1);               /* U^{m+1} whole */
    }
    free(Ub);
    free(pb.RU);
    line_ops_free(&pb.ox);
    line_ops_free(&pb.oy);
    return 0;
}

/* Advance (U, V, W) by nsteps Peaceman-Rachford steps in place, exactly
 * `sweeps` sweeps per stage.  Step m runs from t0 + m dt to t0 + (m+1) dt.
 * Returns 0 or -1. */
int oracle_run(const oracle_params* p, double* U, double* V, double* W,
               const double* K, const double* Rv, const double* Rw, int64_t nsteps) {
    if (!p || p->sweeps < 1) return -1;
    return run_impl(p, U, V, W, K, Rv, Rw, nsteps, 0.0, 0, NULL, NULL, NULL, NULL, NULL);
}

/* As oracle_run (sweeps >= 1) or oracle_run_direct (sweeps 0), with a
 * distributed forcing F (pressure-shaped; NULL = none) times the signal fs,
 * and, when bs is given, Dirichlet wall values equal to the entries of U on
 * the walls at the call times the signal bs (see the reading in the
 * header).  Returns 0 or -1. */
int oracle_run_forced(const oracle_params* p, double* U, double* V, double* W, const double* K,
                      const double* Rv, const double* Rw, int64_t nsteps, const double* F,
                      const oracle_signal* fs, const oracle_signal* bs) {
    if (!p || p->sweeps < 0) return -1;
    if (F && !fs) return -1;
    return run_impl(p, U, V, W, K, Rv, Rw, nsteps, 0.0, 0, NULL, F, fs, bs, NULL);
}

/* As oracle_run, with the tolerance test: eps > 0, min_sweeps even in
 * [2, sweeps].  used (NULL or 2 nsteps entries) receives the sweep count of
 * each stage in order. */
int oracle_run_eps(const oracle_params* p, double* U, double* V, double* W, const double* K,
                   const double* Rv, const double* Rw, int64_t nsteps, double eps, int min_sweeps,
                   int32_t* used) {
    if (!(eps > 0.0) || min_sweeps < 2 || (min_sweeps & 1) || !p || min_sweeps > p->sweeps) return -1;
    return run_impl(p, U, V, W, K, Rv, Rw, nsteps, eps, min_sweeps, used, NULL, NULL, NULL, NULL);
}

/* As oracle_run with damping layers (the damped system, a reformulation the
 * paper points to for absorbing boundaries, Section 2.1): u_t = -kappa div v
 * - (d_x + d_y) u + f, v_t = -(1/rho) u_x - d_x v, w_t = -(1/rho) u_y - d_y w,
 * with d_x (d_y) the rate of the x (y) walls' layers.  The split keeps
 * each rate with its direction: A1 gets -d_x on u and v, A2 gets -d_y on u
 * and w, so a stage's implicit line systems divide by 1 + a d and its
 * explicit part multiplies by 1 - a d.  damp = {d0, width in cells, wall
 * mask}, the profile of damp_rate.  Fixed sweep counts only. */
int oracle_run_damped(const oracle_params* p, double* U, double* V, double* W, const double* K,
                      const double* Rv, const double* Rw, int64_t nsteps, const double* damp) {
    if (!p || p->sweeps < 1 || !damp) return -1;
    return run_impl(p, U, V, W, K, Rv, Rw, nsteps, 0.0, 0, NULL, NULL, NULL, NULL, damp);
}

/* As oracle_run with every stage's line systems solved exactly (the limit
 * of infinitely many sweeps); p->sweeps is ignored. */
int oracle_run_direct(const oracle_params* p, double* U, double* V, double* W, const double* K,
                      const double* Rv, const double* Rw, int64_t nsteps) {
    if (!p) return -1;
    oracle_params q = *p;
    q.sweeps = 0;
    return run_impl(&q, U, V, W, K, Rv, Rw, nsteps, 0.0, 0, NULL, NULL, NULL, NULL, NULL);
}

/* Ricker source value F(t) = s(t) / h^2 as the oracle applies it. */
double oracle_source(const oracle_params* p, double t) {
    if (p->src_i < 0 || p->src_j < 0) return 0.0;
    return ricker(t, p->src_f0, p->src_t0, p->src_amp) / (p->h * p->h);
}

/* ---- single-line operators, for the operator pins ---- */

/* CFD P^-1 Q f: f and out of length n+1. */
int oracle_cfd_d(int n, double h, const double* f, double* out) {
    if (n < 8) return -1;
    line_ops o; line_ops_init(&o, ORC_CFD, n, h);
    deriv_G(&o, f, out);
    line_ops_free(&o);
    return 0;
}

/* CFD Pbar^-1 Qbar v: v of length n+1, out of length n-1 (nodes 1..n-1). */
int oracle_cfd_dbar(int n, double h, const double* v, double* out) {
    if (n < 8) return -1;
    line_ops o; line_ops_init(&o, ORC_CFD, n, h);
    deriv_D(&o, v, out);
    line_ops_free(&o);
    return 0;
}

/* MFD G4 u: u of length n+2, out of length n+1. */
int oracle_mfd_g(int n, double h, const double* u, double* out) {
    if (n < 8) return -1;
    apply_G4(n, h, u, out);
    return 0;
}

/* MFD D4 v: v of length n+1, out of length n. */
int oracle_mfd_d(int n, double h, const double* v, double* out) {
    if (n < 8) return -1;
    apply_D4(n, h, v, out);
    return 0;
}

/* Dense CFD operators: P, Q (n+1)^2; Pbar (n-1)^2; Qbar (n-1)x(n+1). */
int oracle_cfd_matrices(int n, double h, double* P, double* Q, double* Pbar, double* Qbar) {
    if (n < 8) return -1;
    tridiag tp, tb;
    build_P(&tp, n); build_Pbar(&tb, n);
    const int N1 = n + 1, M = n - 1;
    memset(P, 0, sizeof(double) * (size_t)N1 * N1);
    memset(Pbar, 0, sizeof(double) * (size_t)M * M);
    for (int i = 0; i < N1; ++i) {
        P[(size_t)i * N1 + i] = tp.diag[i];
        if (i > 0) P[(size_t)i * N1 + i - 1] = tp.sub[i];
        if (i < n) P[(size_t)i * N1 + i + 1] = tp.sup[i];
    }
    for (int i = 0; i < M; ++i) {
        Pbar[(size_t)i * M + i] = tb.diag[i];
        if (i > 0) Pbar[(size_t)i * M + i - 1] = tb.sub[i];
        if (i < M - 1) Pbar[(size_t)i * M + i + 1] = tb.sup[i];
    }
    /* Q and Qbar column by column through the apply routines on unit vectors */
    double* e = calloc((size_t)N1, sizeof(double));
    double* col = calloc((size_t)N1, sizeof(double));
    for (int c = 0; c < N1; ++c) {
        memset(e, 0, sizeof(double) * (size_t)N1);
        e[c] = 1.0;
        apply_Q(n, h, e, col);
        for (int r = 0; r < N1; ++r) Q[(size_t)r * N1 + c] = col[r];
        apply_Qbar(n, h, e, col);
        for (int r = 0; r < M; ++r) Qbar[(size_t)r * N1 + c] = col[r];
    }
    free(e); free(col);
    tridiag_free(&tp); tridiag_free(&tb);
    return 0;
}

/* Dense MFD operators: D n x (n+1), G (n+1) x (n+2), from the printed rows. */
int oracle_mfd_matrices(int n, double h, double* D, double* G) {
    if (n < 8) return -1;
    for (int r = 0; r < n; ++r)
        for (int c = 0; c <= n; ++c) D[(size_t)r * (n + 1) + c] = D4_entry(n, h, r, c);
    for (int r = 0; r <= n; ++r)
        for (int c = 0; c <= n + 1; ++c) G[(size_t)r * (n + 2) + c] = G4_entry(n, h, r, c);
    return 0;
}

/* LU pivots of P and Pbar as the oracle factors them (no pivoting). */
int oracle_cfd_pivots(int n, double* pivP, double* pivPbar) {
    if (n < 8) return -1;
    tridiag tp, tb;
    build_P(&tp, n); build_Pbar(&tb, n);
    memcpy(pivP, tp.piv, sizeof(double) * (size_t)(n + 1));
    memcpy(pivPbar, tb.piv, sizeof(double) * (size_t)(n - 1));
    tridiag_free(&tp); tridiag_free(&tb);
    return 0;
}
