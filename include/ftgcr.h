/*
 * ftgcr.h -- C ABI of the MI355X (gfx950) FT-GCR library, libftgcr.so.
 *
 * FT-GCR (Gillard & Benacchio, "FT-GCR: a fault-tolerant generalized
 * conjugate residual elliptic solver", arXiv 2103.07210) is preconditioned
 * GCR(k) (Algorithm 1, black part) plus a soft-fault layer (Algorithm 1, red
 * part): after every update the residual norm must strictly decrease (the
 * Krylov nesting argument of Section 2); if it does not, the solver restores
 * the last known-good state [phi, r, p, L(p)]* taken at the start of the
 * previous complete pass (Section 2, text after Algorithm 1) and redoes it.
 *
 * The operator is a synthetic stand-in for the paper's elliptic operator L
 * of Eq. (1): a 7-point flux-form -div(c grad) on a lat-lon-height shell of
 * the unit sphere (longitude periodic, zero flux through the poles, bottom
 * and top) with c = 1 + hill_amp * h(lon, lat) * exp(-zeta / decay_z),
 * h = exp(-(gc / hill_width)^2) (gc: great-circle distance to the hill
 * centre), plus a shift: A = A0 + helmholtz * diag(A0).  The preconditioner
 * P is the vertical (column) tridiagonal part of A, or P = I; the paper only
 * states that GCR is left-preconditioned for the anisotropy of the domain
 * (Section 2).  The same operator is built on the octahedral reduced
 * Gaussian grid O_N of the paper's experiments (Section 3, Table 1), and the
 * fault layer is also offered on restarted GMRES(k), the other Krylov
 * solver the method is meant to carry over to (abstract, Section 1).
 *
 * Conventions
 *  - Every field is a contiguous C-order array [nz][nlat][nlon] (longitude
 *    fastest); flat index of cell (i, j, k) is i + nlon*(j + nlat*k).  On the
 *    octahedral mesh, [nz][points]: point p of level k is p + points*k.
 *  - Device pointers are HIP device memory of the handle's device; the
 *    caller owns them.  Host pointers (plans, stats, logs) are read or written
 *    only during the call.
 *  - Every call returns ftgcr_status: 0 on success, < 0 on misuse or runtime
 *    failure, with a message from ftgcr_last_error().  No C++ exception
 *    crosses the ABI.  Not converging is an outcome, not an error: the solve
 *    returns FTGCR_OK with stats.status = FTGCR_MAX_STEPS or FTGCR_BREAKDOWN.
 *  - Work is enqueued on the handle's stream; solves return when done
 *    (the step count is data dependent).  A handle is not thread-safe.
 */
#ifndef FTGCR_H
#define FTGCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FTGCR_OK = 0,
    FTGCR_E_INVALID = -1,      /* bad argument                                   */
    FTGCR_E_HIP = -2,          /* HIP runtime error                              */
    FTGCR_E_NOMEM = -3,        /* device or host allocation failed               */
    FTGCR_E_WORKSPACE = -4,    /* no workspace, or smaller than required         */
    FTGCR_E_UNSUPPORTED = -5   /* valid but outside what the library supports    */
} ftgcr_status;

typedef enum { FTGCR_FP64 = 0, FTGCR_MIXED = 1 } ftgcr_precision;
/* Preconditioner P of the left-preconditioned iteration (Section 2: the
 * paper preconditions for the anisotropy of the domain without giving P):
 * COLUMN is the vertical tridiagonal part of A (A's diagonal and vertical
 * couplings), solved per column; NONE is P = I. */
typedef enum { FTGCR_PRECOND_NONE = 0, FTGCR_PRECOND_COLUMN = 1 } ftgcr_precond;

/* Solve outcomes (ftgcr_stats.status). */
enum { FTGCR_CONVERGED = 0, FTGCR_MAX_STEPS = 1, FTGCR_STAGNATED = 2, FTGCR_BREAKDOWN = 3 };

/* Largest Krylov space size k (kmax) a handle may be created with. */
#define FTGCR_KMAX 16
/* Capacity of the device-side detection log per solve. */
#define FTGCR_LOG_CAP 256

/* Meshes (ftgcr_grid.mesh).
 * LATLON: nlon x nlat cell centres of a regular longitude-latitude grid,
 *   the 7-point flux form described at the top of this file.
 * OCTAHEDRAL: the octahedral reduced Gaussian grid O_N of the paper's
 *   experiments (Section 3, Table 1), N = nlat (nlon is ignored): 2N rings at
 *   the Gaussian latitudes (the sines are the roots of the Legendre
 *   polynomial P_2N), the i-th ring from either pole (i = 1..N) with 4i + 16
 *   equally spaced points starting at longitude 0, 4N(N+9) points per level,
 *   numbered ring by ring from the south pole, eastward, then level by
 *   level.  Node-centred finite volumes on the triangulation that joins
 *   neighbouring rings (walking both eastward from longitude 0, the ring whose
 *   next point comes first -- the southern one on a tie -- adds a triangle;
 *   the polar caps stay open: no flux through the poles): the control area
 *   of a point is its circumcentric region of the inscribed polyhedron, the
 *   horizontal face weight of an edge is c dz (cot a + cot b) / 2 (the angles
 *   opposite it), the vertical ones c area / dz, c at the face centre.
 *   Single solves: FT-GCR in FP64 or MIXED (binary32 copies of the tables),
 *   FT-GMRES in FP64. */
enum { FTGCR_MESH_LATLON = 0, FTGCR_MESH_OCTAHEDRAL = 1 };

typedef struct {
    int32_t nlon;          /* LATLON: >= 3; OCTAHEDRAL: ignored                 */
    int32_t nlat;          /* LATLON: >= 1; OCTAHEDRAL: N >= 1                  */
    int32_t nz;            /* 1 .. 96 with the column preconditioner            */
    double shell_depth;    /* vertical extent of the shell, unit sphere; > 0    */
    int32_t mesh;          /* FTGCR_MESH_LATLON (0) or FTGCR_MESH_OCTAHEDRAL    */
} ftgcr_grid;

typedef struct {
    double hill_lon, hill_lat;  /* hill centre, radians                         */
    double hill_amp;            /* >= 0                                         */
    double hill_width;          /* > 0                                          */
    double decay_z;             /* > 0                                          */
    double helmholtz;           /* > 0 (SPD); the shift relative to diag(A0)    */
} ftgcr_coeffs;

typedef struct {
    int32_t ft;              /* 1: FT-GCR (Algorithm 1 with the red part); 0: GCR */
    int32_t poll_steps;      /* steps enqueued between status reads (>= 1)      */
    int64_t max_steps;       /* cap on executed inner steps (all refinements)   */
    double inner_tol;        /* MIXED: inner stop, relative to the refinement's
                                true residual                                    */
    int32_t max_refinements; /* MIXED: cap on outer refinement rounds           */
    int32_t inner_max_steps; /* MIXED: cap on inner steps per round            */
    int64_t hist_cap;        /* entries of the per-step residual history kept   */
    int32_t use_graphs;      /* 1: replay captured step sequences (hipGraph)     */
    int32_t levels_per_block;/* stencil kernels: levels per block (0 = auto)    */
    int32_t profile_kernels; /* time step kernels with a HIP event pair each,
                                stamped by the kernel's own dispatch on the
                                solve stream (ftgcr_kernel_times).  Bits 0-7:
                                0 off, 1 all three, else a mask of bit 1
                                update_thomas, bit 2 stencil_dots, bit 3
                                dir_update; bits 8-15: a stride s > 1 times
                                only steps whose number is a multiple of s   */
    int32_t batch_levels_per_block; /* ftgcr_solve_batch with this handle as
                                the first member: stencil levels per block of
                                the combined launches (1, 2, 4, 8 or 16; 0 =
                                the largest member's own tiling); set by
                                ftgcr_autotune_batch                            */
    int32_t method;          /* Krylov method of ftgcr_solve: FTGCR_METHOD_GCR
                                (FT-GCR(k), Algorithm 1) or FTGCR_METHOD_GMRES
                                (the same fault layer on restarted GMRES(k);
                                FP64 handles, single solves)                    */
    int32_t order_stencil;   /* block order of the stencil-grid passes (the
                                dots pass of L(e), the residual and the final
                                x): FTGCR_ORDER_*; 0 = auto (ftgcr_autotune's
                                choice, else the mesh's default)              */
    int32_t order_dir;       /* block order of the direction pass, likewise  */
} ftgcr_options;

/* options.order_stencil / order_dir: the order in which a pass's blocks (a
 * column tile times a chunk of levels) are assigned to the launch's
 * workgroups.  The result does not depend on it beyond the order of the
 * block partial sums.
 *   X    the tiles of one level chunk in a row, then the next chunk (the
 *        lat-lon default);
 *   Z    a tile's level chunks in a row, so its vertical halo levels and
 *        per-column tables are re-read while still cached;
 *   XCD  as Z, with each of the GPU's 8 accelerator dies (XCDs, each with its
 *        own L2; consecutive workgroups go to consecutive dies) given one
 *        contiguous range of tiles, so neighbouring tiles share an L2 (the
 *        octahedral default: its slot tables and neighbour gathers). */
enum { FTGCR_ORDER_AUTO = 0, FTGCR_ORDER_X = 1, FTGCR_ORDER_Z = 2, FTGCR_ORDER_XCD = 3 };

/* options.method.  FTGCR_METHOD_GMRES: right-preconditioned restarted
 * GMRES(k) with classical Gram-Schmidt and Givens rotations, wrapped in the
 * fault layer of Algorithm 1 as the paper proposes for other Krylov solvers
 * (abstract; Section 1): the residual norm must strictly decrease after every
 * step (the least-squares residual |g_{j+1}| of the cycle) and at the end of
 * every cycle (the explicit |R - A x|); otherwise x is restored from the
 * backup taken after the last cycle that passed, and the cycle is redone.
 * Stats as for GCR; a cycle-end detection is logged with nu = -1, and the
 * residual history holds |g_{j+1}|^2 per step.  Fault events: X flips x at
 * the start of the step, R the Arnoldi vector v_j (before P^{-1} reads it),
 * P and E the preconditioned z_j = P^{-1} v_j, AP w = A z_j before the inner
 * products. */
enum { FTGCR_METHOD_GCR = 0, FTGCR_METHOD_GMRES = 1 };

/* Fault injection (test harness).  XOR bit `bit` (or bits[t] per entry) into
 * the IEEE-754 pattern of entries of one working vector (binary64 in FP64
 * handles, binary32 in MIXED handles: bits 0..31; the iterate x is always
 * binary64) during executed inner step `step` (1-based, counted over the
 * whole solve):
 *   X, R, P, AP  the iterate x, the residual r, the current direction p^nu or
 *                its image L(p^nu), at the start of the step, before the step
 *                reads anything;
 *   E            the preconditioner output e = P^{-1}(r+) of the step, right
 *                after the column solve and before L(e) and the new direction
 *                read it: the paper's injection site (Section 3).  Applied
 *                only when the step passes its exit and fault tests (otherwise
 *                e is never used).
 * idx == NULL means the range [start, start+count).  An event whose step is
 * never reached is not applied. */
typedef enum { FTGCR_V_X = 0, FTGCR_V_R = 1, FTGCR_V_P = 2, FTGCR_V_AP = 3, FTGCR_V_E = 4 } ftgcr_vec;
typedef struct {
    int64_t step;
    int32_t vec;           /* ftgcr_vec                                         */
    int32_t bit;
    int64_t count;
    int64_t start;
    const int64_t* idx;    /* host, count entries, each in [0, N)               */
    const uint8_t* bits;   /* host, count entries, or NULL                      */
} ftgcr_fault_event;

typedef struct {
    int32_t n_events;
    const ftgcr_fault_event* events;   /* host array                            */
} ftgcr_fault_plan;

typedef struct {
    int64_t step;          /* executed step whose residual failed to decrease   */
    int32_t nu;            /* pass index nu of that step                        */
    int32_t action;        /* 0: rolled back to the backup; 1: accepted as
                              stagnation (same place again, no fault since)     */
    double rr_old, rr_new; /* <r,r> before and after the update                 */
} ftgcr_detect_rec;

typedef struct {
    int32_t status;              /* FTGCR_CONVERGED, _MAX_STEPS, _BREAKDOWN      */
    int32_t detections;
    int32_t stagnation_accepts;
    int32_t events_applied;
    int64_t steps_executed;      /* inner steps run, including wasted ones       */
    int64_t steps_accepted;
    int64_t steps_wasted;        /* steps undone by rollbacks                    */
    int64_t cycles;              /* passes with nu = 0 executed                  */
    int32_t refinements;         /* MIXED: outer rounds run                      */
    int32_t log_len;             /* records written to log (<= log_cap)          */
    double rhs_norm2;            /* <R, R>                                       */
    double rr_final;             /* recursive <r, r> at return (last round)      */
    double rel_res_recursive;
    double rel_res_true;         /* ||A x - R|| / ||R|| in FP64 on the returned x */
    double time_ms;              /* device time of the solve                     */
    int32_t log_cap;             /* in: capacity of log (0: no log)              */
    int32_t pad_;
    ftgcr_detect_rec* log;       /* in: caller-owned host array or NULL          */
    int64_t hist_cap;            /* in: capacity of hist (0: none)               */
    int64_t hist_len;            /* out                                          */
    double* hist;                /* in: caller-owned host array: <r,r> after each
                                    executed step (detector value)              */
} ftgcr_stats;

typedef struct ftgcr_handle ftgcr_handle;

/* Fill *opt with defaults: ft=1 (the fault layer of Algorithm 1 on),
 * method=GCR, poll_steps=16, max_steps=100000, inner_tol=3e-5,
 * max_refinements=20, inner_max_steps=5000, hist_cap=65536, use_graphs=1,
 * levels_per_block=0, order_stencil=order_dir=0 (auto).  opt must not be
 * NULL. */
void ftgcr_default_options(ftgcr_options* opt);

/* Create a solver for one grid and coefficient set on the current HIP device
 * (the operator L of Eq. (1) discretised as described at the top; the
 * preconditioner of Section 2).  Builds the FP64 coefficient tables (hill at
 * cell and face centres, vertical decay, metric factors; on O_N the mesh's
 * neighbour lists, face weights and control areas), binary32 copies of the
 * per-column and per-point ones, and the device state.
 *  grid, coeffs : host, read during the call.  nz <= 96.
 *  precond      : FTGCR_PRECOND_COLUMN or FTGCR_PRECOND_NONE (P = I).
 *  precision    : FTGCR_FP64 or FTGCR_MIXED (either mesh).
 *  kmax         : bounds k in later solves (1 <= kmax <= FTGCR_KMAX).
 *  hip_stream   : a hipStream_t (NULL: the default stream).
 *  out          : receives the handle (NULL on failure); free with
 *                 ftgcr_destroy.
 * Returns E_INVALID for bad arguments, E_UNSUPPORTED for valid combinations
 * that are not built, E_NOMEM / E_HIP on allocation or runtime failure;
 * ftgcr_last_error(NULL) then holds the message. */
ftgcr_status ftgcr_create(const ftgcr_grid* grid, const ftgcr_coeffs* coeffs,
                          ftgcr_precond precond, ftgcr_precision precision,
                          int32_t kmax, void* hip_stream, ftgcr_handle** out);

/* Replace the handle's options (read from host *opt during the call);
 * E_INVALID, options unchanged, when a field is out of range (k-independent
 * fields only: k is checked by each solve) or a method is asked for that the
 * handle's precision does not build (FT-GMRES: FP64 handles, either mesh). */
ftgcr_status ftgcr_set_options(ftgcr_handle* h, const ftgcr_options* opt);
/* Copy the handle's options to host *opt. */
ftgcr_status ftgcr_get_options(const ftgcr_handle* h, ftgcr_options* opt);
/* Enqueue later work on hip_stream (a hipStream_t of the handle's device,
 * NULL: the default stream). */
ftgcr_status ftgcr_set_stream(ftgcr_handle* h, void* hip_stream);

/* Device workspace the caller must provide (bytes), for the handle's kmax:
 * the working vectors of Algorithm 1 in the storage precision -- the
 * directions p^l and their images L(p^l) with their backup copies (the
 * saved state of Section 2), three residual buffers and e = P^{-1} r, on
 * the octahedral mesh also L(e) -- one
 * FP64 iterate buffer, block partial sums and the residual history (for
 * FT-GMRES the k+1 basis vectors, k preconditioned vectors and the
 * backup).  0 when h is NULL. */
size_t ftgcr_workspace_bytes(const ftgcr_handle* h);
/* dev_ptr: device memory of at least ftgcr_workspace_bytes(h) bytes, 256-byte
 * aligned, owned by the caller and kept alive while the handle solves. */
ftgcr_status ftgcr_set_workspace(ftgcr_handle* h, void* dev_ptr, size_t bytes);

/* Solve A x = rhs (Eq. (1)) with FT-GCR(k), Algorithm 1 (with
 * options.method = GMRES: FT-GMRES(k), the fault layer on restarted GMRES).
 *  rhs_dev : device, FP64, N entries (read only).
 *  x_dev   : device, FP64, N entries; in: initial guess phi^0, out: solution.
 *  tol     : FP64 handles stop when <r,r> <= tol^2 <R,R> on the recursive
 *            residual; MIXED handles stop when the FP64 true residual
 *            ||A x - R|| <= tol ||R|| (iterative refinement, inner FT-GCR with
 *            binary32 vectors and FP64 arithmetic, inner products and detector).
 *  k       : Krylov space size, 1 <= k <= kmax.
 *  plan    : fault plan or NULL.
 *  stats   : NULL or caller-owned; log/hist fields are inputs.
 * The residual-norm test, the backup at each pass nu = 0 and the rollback are
 * those of Algorithm 1 (red part) when options.ft = 1. */
ftgcr_status ftgcr_solve(ftgcr_handle* h, const double* rhs_dev, double* x_dev,
                         double tol, int32_t k, const ftgcr_fault_plan* plan,
                         ftgcr_stats* stats);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  As ftgcr_solve, but the working vectors and the fault plan's
 * entry lists live in a device scratch array of FTGCR_NOALLOC_SCRATCH_BYTES
 * that the library holds on every device it runs on until the process ends,
 * not in the workspace of ftgcr_set_workspace (none need be set).  Limit:
 * ftgcr_workspace_bytes(h) rounded up to 256, plus 9 bytes per fault-plan
 * entry given as an index list, must fit the scratch; otherwise the call
 * returns FTGCR_E_WORKSPACE with a message and runs nothing.  The call
 * allocates nothing (no hipMalloc, hipFree, graph or event creation):
 * options.use_graphs and options.profile_kernels are ignored.  Every call on
 * one device shares that device's scratch, which keeps the last call's
 * contents (nothing in it must start at zero); calls that overlap on one GPU
 * (from other threads or streams) race, and the caller must serialise them. */
#define FTGCR_NOALLOC_SCRATCH_BYTES (64u << 20)
ftgcr_status ftgcr_solve_noalloc(ftgcr_handle* h, const double* rhs_dev, double* x_dev, double tol, int32_t k,
                                 const ftgcr_fault_plan* plan, ftgcr_stats* stats);

/* Solve n independent problems at once (an ensemble of the elliptic solves
 * of Eq. (1), each with FT-GCR(k) of Algorithm 1): every handle must be FP64,
 * GCR, on the first handle's mesh (either mesh), with the same
 * preconditioner, have its own workspace and share the first handle's
 * stream; their
 * step kernels run as combined launches over all unfinished members, each
 * member keeping its own convergence and fault state on the device.
 * rhs[m], x[m], tol[m] as in ftgcr_solve; plans may be NULL (no faults) or an
 * array of n plans; stats may be NULL or an array of n. */
ftgcr_status ftgcr_solve_batch(ftgcr_handle* const* hs, int32_t n,
                               const double* const* rhs, double* const* x,
                               const double* tol, int32_t k,
                               const ftgcr_fault_plan* plans, ftgcr_stats* stats);

/* Tiling autotune of a batch (the ensemble's launch shape; measurement of
 * the solve of ftgcr_solve_batch, no change to its arithmetic): times `steps`
 * batched steps of these members (fault-free, from x = 0) at 2, 4 and 8
 * stencil levels per block (those not above the deepest member's nz), keeps
 * the fastest in hs[0]'s options.batch_levels_per_block and writes it to
 * *chosen (optional).  Arguments as in ftgcr_solve_batch; x_scratch[m] is an
 * FP64 device buffer of member m's N entries, overwritten.  Every member's
 * other options are as before on return, also on error. */
ftgcr_status ftgcr_autotune_batch(ftgcr_handle* const* hs, int32_t n,
                                  const double* const* rhs, double* const* x_scratch,
                                  int32_t k, int32_t steps, int32_t* chosen);

/* Autotuner of the stencil tiling of the operator application L(p) of
 * Algorithm 1 (the results do not depend on the choice beyond the order of
 * the block partial sums): times `steps` steps of this problem for each
 * candidate number of levels of a column per block, then, at the fastest,
 * each pair of block orders (FTGCR_ORDER_X, _Z, _XCD) of the dots pass and
 * the direction pass by those kernels' own times (the mesh's default pair
 * unless another is at least 1% faster), and keeps the fastest for
 * this handle (options.levels_per_block = 0, order_stencil = order_dir = 0)
 * and for every later handle with the same mesh, grid and precision in this
 * process.  x_scratch_dev: FP64 device buffer of N entries, overwritten.
 * *chosen (optional) gets the levels per block. */
ftgcr_status ftgcr_autotune(ftgcr_handle* h, const double* rhs_dev, double* x_scratch_dev, int32_t k,
                            int32_t steps, int32_t* chosen);

/* The stencil tiling in effect for this handle's next single solve (from
 * its options, else ftgcr_autotune's choice, else the defaults): levels of
 * a column per block of the dots pass and of the direction pass, and the
 * two passes' block orders (FTGCR_ORDER_X, _Z or _XCD, never AUTO).  Any
 * output pointer may be NULL. */
ftgcr_status ftgcr_get_tiling(const ftgcr_handle* h, int32_t* levels_per_block, int32_t* levels_per_block_dir,
                              int32_t* order_stencil, int32_t* order_dir);

/* Per-kernel device time (measurement of the step of Algorithm 1)
 * accumulated while options.profile_kernels != 0:
 * one record per kernel of the step sequence (update_thomas, stencil_dots,
 * dir_update), each the sum of its launches' execution times (start and
 * stop events stamped by each dispatch)
 * (launches enqueued after the solve ended are not counted).  Writes min(cap, count) records
 * and the count to *n_out. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} ftgcr_kernel_time;
ftgcr_status ftgcr_kernel_times(const ftgcr_handle* h, ftgcr_kernel_time* out, int32_t cap, int32_t* n_out);
/* Zero the accumulated kernel times. */
ftgcr_status ftgcr_reset_kernel_times(ftgcr_handle* h);

/* Free the handle and its device state (not the caller's workspace, which
 * the caller frees after this call).  NULL is a no-op. */
void ftgcr_destroy(ftgcr_handle* h);

/* HBM bandwidth probe (measurement, no solver state): copies `bytes` from
 * src_dev to dst_dev once to warm up, then `reps` times with a plain
 * streaming copy kernel on hip_stream (NULL: default stream), and writes the
 * achieved rate 2 * bytes * reps / elapsed (read plus write, GB/s = 1e9 B/s)
 * to *gbs.  The two buffers are device memory of the current device, 16-byte
 * aligned, not overlapping; bytes is a positive multiple of 16.  Synchronous.
 * Errors are reported by ftgcr_last_error(NULL). */
ftgcr_status ftgcr_bw_probe(const void* src_dev, void* dst_dev, size_t bytes, int32_t reps, void* hip_stream,
                            double* gbs);

/* Message of the last failed call on h (or of the last failed create when h
 * is NULL).  Valid until the next call on the same handle. */
const char* ftgcr_last_error(const ftgcr_handle* h);

/* Parity entry points (FP64, device pointers of N entries in the field
 * layout above, caller-owned, not overlapping, on the handle's stream,
 * synchronous): out = A in (the operator L of Eq. (1)), and
 * out = P^{-1} in (the preconditioner of Section 2; a copy for P = I).
 * Both run in FP64 whatever the handle's precision. */
ftgcr_status ftgcr_debug_apply_A(ftgcr_handle* h, const double* in_dev, double* out_dev);
ftgcr_status ftgcr_debug_apply_Pinv(ftgcr_handle* h, const double* in_dev, double* out_dev);

#ifdef __cplusplus
}
#endif
#endif
