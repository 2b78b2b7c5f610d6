/*
 * FT-GCR reference oracle (plain C, FP64; serial, or threaded with bitwise
 * identical results).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library; it is
 * not part of the product path.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no source with the
 * HIP library: the two are written independently from the paper (Gillard &
 * Benacchio, "FT-GCR: a fault-tolerant generalized conjugate residual elliptic
 * solver", arXiv 2103.07210) and from the frozen operator readings.
 *
 * What it computes
 *   - the synthetic elliptic operator A (7-point flux-form div(c grad) on a
 *     lat-lon-height shell, periodic in longitude, zero flux through the poles,
 *     bottom and top, plus a relative Helmholtz shift), standing in for the
 *     paper's operator L of Eq. (1);
 *   - the column preconditioner P (the vertical tridiagonal part of A), solved
 *     by the Thomas algorithm; the paper only says the solver is
 *     left-preconditioned for the anisotropy of the domain (Section 2);
 *   - FT-GCR(k) of Algorithm 1, red (fault tolerance) part included or not,
 *     with the sign, restart, backup and tie readings listed in the design
 *     notes, plus a harness-driven bit-flip fault plan.
 *
 * Layout: every field is C-order [nz][ny][nx], longitude fastest.  Flat index
 * of cell (i, j, k) is i + nx*(j + ny*k).
 *
 * What pins each function (closed forms, dense solves, library GMRES, predicted
 * fault outcomes) is listed in the docstring of the Python wrapper,
 * oracle/oracle.py; the pins themselves are tests/test_oracle_*.py.
 */
#ifndef FTGCR_ORACLE_H
#define FTGCR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;       /* longitudes, latitudes, levels                  */
    double shell_depth;       /* vertical extent H_s of the shell (unit sphere) */
    double hill_lon, hill_lat;/* hill centre (radians)                          */
    double hill_amp;          /* a_h in c = 1 + a_h h g                         */
    double hill_width;        /* w in h = exp(-(gc/w)^2)                        */
    double decay_z;           /* g = exp(-zeta/decay_z)                         */
    double helmholtz;         /* sigma: A = A0 + sigma diag(A0)                 */
} orc_problem;

/* Face weights of the flux-form operator, all FP64.
 *   wx[(k*ny + j)*nx + i]       face between cells i and i+1 (periodic)
 *   wy[(k*(ny+1) + j)*nx + i]   face between latitude rows j-1 and j, j=0..ny
 *                               (exactly zero for j=0 and j=ny: the poles)
 *   wz[(k*ny + j)*nx + i]       face between levels k-1 and k, k=0..nz
 *                               (exactly zero for k=0 and k=nz)
 * Sizes: nx*ny*nz, nx*(ny+1)*nz, nx*ny*(nz+1).  Caller-owned. */
void orc_face_weights(const orc_problem* pb, double* wx, double* wy, double* wz);

/* Hill height h(lon, lat) in [0, 1]. */
double orc_hill(const orc_problem* pb, double lon, double lat);

/* y = A x. */
void orc_apply_A(const orc_problem* pb, const double* wx, const double* wy,
                 const double* wz, const double* x, double* y);

/* e = P^{-1} r, P = vertical tridiagonal part of A (one Thomas solve per column). */
void orc_apply_pinv(const orc_problem* pb, const double* wx, const double* wy,
                    const double* wz, const double* r, double* e);

/* Threads for the operator and preconditioner applications (OpenMP builds;
 * results are bitwise independent of the count).  orc_set_threads returns 0,
 * or -1 for n < 1 (or n > 1 in a build without OpenMP); orc_threads gives
 * the count in use. */
int orc_set_threads(int32_t n);
int32_t orc_threads(void);

/* Plain left-to-right FP64 inner product over n entries. */
double orc_dot(int64_t n, const double* a, const double* b);

/* One fault event: XOR bit(s) into the IEEE-754 binary64 pattern of entries of
 * one working vector during executed step `step` (1-based).  X, R, P, AP: the
 * iterate, the residual, the current direction or its image, at the start of
 * the step before it reads anything.  E: the preconditioner output
 * e = P^{-1}(r) of the step, right after it is computed and before L(e) and
 * the new direction read it (the paper's injection site, Section 3); a step
 * that exits or rolls back never computes e, so its E events do not apply.
 * idx == NULL means the contiguous range [start, start+count).  bits == NULL
 * means every entry gets bit `bit`. */
enum { ORC_V_X = 0, ORC_V_R = 1, ORC_V_P = 2, ORC_V_AP = 3, ORC_V_E = 4 };
typedef struct {
    int64_t step;
    int32_t vec;
    int32_t bit;
    int64_t count;
    int64_t start;
    const int64_t* idx;
    const uint8_t* bits;
} orc_event;

enum { ORC_CONVERGED = 0, ORC_MAX_STEPS = 1, ORC_STAGNATED = 2, ORC_BREAKDOWN = 3 };

typedef struct {
    int64_t step;       /* executed step at which the detector fired            */
    int32_t nu;         /* inner index nu of that step                          */
    int32_t action;     /* 0 = rolled back, 1 = accepted as stagnation          */
    double rr_old, rr_new;
} orc_detect;

typedef struct {
    int32_t status;
    int32_t detections;
    int32_t stagnation_accepts;
    int32_t events_applied;
    int64_t steps_executed;
    int64_t steps_accepted;
    int64_t steps_wasted;
    int64_t cycles;              /* number of nu = 0 steps executed              */
    double rhs_norm2;            /* <R,R>                                        */
    double rr_final;             /* recursive <r,r> at return                    */
    double rel_res_recursive;    /* sqrt(rr_final / rhs_norm2)                   */
    int32_t log_len;
    int32_t pad_;
    int64_t hist_len;
} orc_stats;

/* FT-GCR(k) solve of A x = rhs, x in/out (initial guess in).  Returns 0, or -1
 * on invalid arguments / allocation failure.  tol is relative on the recursive
 * residual: stop when <r,r> <= tol^2 <rhs,rhs>.  ft = 0 runs plain GCR(k).
 * log (log_cap entries) and hist (<r,r> after each executed step, hist_cap
 * entries) are optional. */
int orc_solve(const orc_problem* pb, const double* rhs, double* x, double tol,
              int32_t k, int64_t max_steps, int32_t ft,
              const orc_event* events, int32_t n_events, orc_stats* st,
              orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap);

/* Same, plus optional per-step orthogonality diagnostics (cap entries each,
 * NULL to skip): cos_r_ap[s-1] = max over l <= nu of |<r^{nu+1}, Lp^l>| /
 * (|r^{nu+1}| |Lp^l|) after the update of step s, and cos_ap[s-1] = max over
 * l <= nu of |<Lp^{nu+1}, Lp^l>| / (|Lp^{nu+1}| |Lp^l|) after its new
 * direction (0 for steps that exit or roll back). */
int orc_solve_traced(const orc_problem* pb, const double* rhs, double* x, double tol,
                     int32_t k, int64_t max_steps, int32_t ft,
                     const orc_event* events, int32_t n_events, orc_stats* st,
                     orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap,
                     double* cos_r_ap, double* cos_ap, int64_t trace_cap);

/* FT-GMRES(k): right-preconditioned restarted GMRES(k) with the same fault
 * layer (the residual-norm test after every step and at the end of every
 * cycle, the backup [x, |R - A x|^2] after each cycle that passes, the
 * rollback and the stagnation rule); see the comment above its definition.
 * Arguments, outcomes and the log as for orc_solve (a cycle-end detection
 * has nu = -1); tol is relative: stop when |R - A x|^2 <= tol^2 |R|^2 on
 * the explicit residual at a cycle end.  hist gets the step's squared
 * residual norm |g_{j+1}|^2 of the Arnoldi least-squares problem. */
int orc_gmres_solve(const orc_problem* pb, const double* rhs, double* x, double tol,
                    int32_t k, int64_t max_steps, int32_t ft,
                    const orc_event* events, int32_t n_events, orc_stats* st,
                    orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap);

/* FT-GCR(k) (method 0) or FT-GMRES(k) (method 1) on a lat-lon problem with
 * the column preconditioner (precond 1) or none (precond 0: P = I);
 * arguments and outcomes as for orc_solve. */
int orc_solve_pc(const orc_problem* pb, int32_t precond, int32_t method, const double* rhs, double* x,
                 double tol, int32_t k, int64_t max_steps, int32_t ft,
                 const orc_event* events, int32_t n_events, orc_stats* st,
                 orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap);

/* Octahedral reduced Gaussian grid O_N (Section 3, Table 1): 2N rings of
 * 4i + 16 points (i = 1..N from either pole), 4N(N+9) points per level, at
 * the Gaussian latitudes, with the node-centred finite-volume operator on the
 * triangulated mesh described above its definition.  Coefficients and shift
 * as for the lat-lon problem. */
typedef struct {
    int32_t N, nz;
    double shell_depth, hill_lon, hill_lat, hill_amp, hill_width, decay_z, helmholtz;
} orc_oct_problem;

int64_t orc_oct_cells(int32_t N);                 /* 4N(N+9), cells per level */
int32_t orc_oct_ring_points(int32_t N, int32_t j);/* points of ring j (0 = southernmost) */
/* The 2N Gauss-Legendre nodes (sines of the ring latitudes, ascending) and weights. */
void orc_oct_gauss(int32_t N, double* mu, double* w);
/* Longitude, latitude and control area of every point (4N(N+9) each), and
 * the number of edges of the triangulation. */
int orc_oct_mesh(const orc_oct_problem* pb, double* lon, double* lat, double* area, int64_t* nedge);
int orc_oct_apply_A(const orc_oct_problem* pb, const double* x, double* y);
int orc_oct_apply_pinv(const orc_oct_problem* pb, const double* r, double* e);
/* FT-GCR(k) (method 0) or FT-GMRES(k) (method 1) on an O_N problem;
 * arguments and outcomes as for orc_solve / orc_gmres_solve. */
int orc_oct_solve(const orc_oct_problem* pb, const double* rhs, double* x, double tol,
                  int32_t k, int64_t max_steps, int32_t ft, int32_t method,
                  const orc_event* events, int32_t n_events, orc_stats* st,
                  orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap);
/* Same with the column preconditioner (precond 1) or none (precond 0: P = I). */
int orc_oct_solve_pc(const orc_oct_problem* pb, int32_t precond, int32_t method, const double* rhs, double* x,
                     double tol, int32_t k, int64_t max_steps, int32_t ft,
                     const orc_event* events, int32_t n_events, orc_stats* st,
                     orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap);

#ifdef __cplusplus
}
#endif
#endif
