// Internal types shared by the FT-GCR kernels and the host engine.
//
// One solve ("instance") keeps all of its control state on the device in a
// SolveState; the step kernels read it to find the pass index nu, the buffer
// roles and the scalars of Algorithm 1, so a step is the same fixed kernel
// sequence whatever happened before (rollbacks included) and can be enqueued
// or replayed without reading anything back.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ftgcr.h"

namespace ftgcr {

constexpr int KMAX = FTGCR_KMAX;
constexpr int LOG_CAP = FTGCR_LOG_CAP;
constexpr int NV_MAX = KMAX + 2;     // reduction values per block
constexpr int DOT_ROW0 = 2;          // first partials row of the dots pass (rows 0, 1:
                                     // the column pass's, still unread when a
                                     // speculative dots pass runs)
constexpr int RUNNING = -1;

// Block shapes.  Column kernels: 256 threads = 4 waves, each wave owns 32
// columns (lanes 0..31 the lower half of each column, 32..63 the upper half).
constexpr int COL_THREADS = 256;
constexpr int COLS_PER_BLOCK = 128;

// Columns per block of the column pass: the binary32 form with half columns
// of at most 32 levels uses one lane per column (k_update_thomas1), the
// others two lanes per column.
inline int col_block_cols(int elem_bytes, int H)
{
    return (elem_bytes == 4 && H <= 32) ? COL_THREADS : COLS_PER_BLOCK;
}
// Stencil kernels: 64 longitudes x 4 latitudes per block, KC levels each.
constexpr int ST_TX = 64;
constexpr int ST_TY = 4;
constexpr int ST_THREADS = ST_TX * ST_TY;
constexpr int RED_THREADS = 1024;
// Octahedral mesh: neighbour slots per point (the triangulation's valence
// is at most 6); a block of the stencil kernels covers ST_THREADS
// consecutive points.
constexpr int NB_OCT = 6;
// Block orders of the stencil-grid launches (a block is a column tile times
// a chunk of levels; FTGCR_ORDER_* minus 1): tiles of a level chunk in a row
// (X); a tile's level chunks in a row (Z); as Z, with each accelerator die
// given one contiguous range of blocks (XCD).  Consecutive workgroups are
// placed on the XCDS dies round robin, each die with its own L2.
enum { ORD_X = 0, ORD_Z = 1, ORD_XCD = 2 };
constexpr int XCDS = 8;

struct DetectRec {
    long long step;
    int nu;
    int action;
    double rr_old, rr_new;
};

// Per-solve control state (device memory, written by single-thread kernel
// sections only).
struct SolveState {
    int status;          // RUNNING or an FTGCR_* outcome
    int active;          // 1: this step goes on to P^{-1}, L and the new direction
    int nu;              // pass index of the current step
    int k;
    int ft;
    int mixed;
    int detections, stagnation_accepts, events_applied, events_since_rb;
    long long s;         // executed steps
    long long max_steps; // stop when s reaches this (global or round cap)
    long long accepted;
    long long cycles;
    long long last_rb_pos;
    double tol2;         // tol^2 (FP64) or inner tol^2 (mixed round)
    double T;            // exit threshold on <r,r>
    double RR;           // <R,R>
    double rt2;          // <r_t, r_t> of the last true-residual pass
    double rr_old, rr_new;
    double beta_num;     // <r, L p^nu>
    double d_cur;        // <L p^nu, L p^nu>
    double d[KMAX + 1];
    double beta[KMAX + 1];
    double alpha[KMAX + 1];
    int slot[KMAX + 1];  // buffer index of p^l / L(p^l)
    int r_cur, r_dst, r_bak;
    int x_base, x_base_nu, x_bak, x_dst;
    int x_final_hi;      // materialise x with beta_l p^l for l <= this at the end
    int b_slot0;
    long long b_accepted;
    double b_rr, b_beta_num, b_d0;
    // fault-event staging (set by the event preparation kernel)
    int ev_ok;           // the event applies (solve still running)
    int ev_vec;
    int ev_copy;         // 1: copy src -> dst buffer before flipping
    int ev_src, ev_dst;  // buffer indices for the copy
    int ev_lo, ev_hi;    // x materialisation: beta terms l in [lo, hi)
    int log_len;
    int e_ok;            // 1: this step passed its tests, its e feeds a new direction
    DetectRec log[LOG_CAP];
};

// Geometry / coefficient tables of one grid (device, FP64).
struct Geo {
    int nx, ny, nz;
    int ncols;               // nx * ny
    long long n;             // nx * ny * nz
    double opsig;            // 1 + helmholtz
    const double* hx;        // [ny][nx]    hill_amp * h at east face (i+1/2, j)
    const double* hy;        // [ny+1][nx]  hill_amp * h at face (i, j-1/2)
    const double* hc;        // [ny][nx]    hill_amp * h at centre (i, j)
    const double* gc;        // [nz]        exp(-zeta_k / decay)
    const double* gf;        // [nz+1]      exp(-zeta_{k-1/2} / decay)
    const double* Gx;        // [ny]        dlat dz / (cos(lat_j) dlon)
    const double* Gy;        // [ny+1]      cos(lat_{j-1/2}) dlon dz / dlat, 0 at poles
    const double* Gz;        // [ny]        cos(lat_j) dlon dlat / dz
    // binary32 copies of the per-column hill tables, read by the binary32
    // stencil and column solve (half the bytes of the FP64 ones)
    const float* hx32;
    const float* hy32;
    const float* hc32;
    // octahedral mesh (mesh == FTGCR_MESH_OCTAHEDRAL; then nx = points per
    // level, ny = 1): per point and neighbour slot q (slot-major, [q][point])
    // the neighbour (-1: empty slot), the metric part of the face weight and
    // that times hill_amp * h at the face centre; per point the sums of both
    // over its slots, the vertical face metric (control area / dz) and
    // hill_amp * h at the point
    int mesh;
    const int* onb;
    const double* ogw;
    const double* ohw;
    const double* oh0;
    const double* oh1;
    const double* ogz;
    const double* ohc;
    // binary32 copies of the octahedral tables (rounded to nearest), read by
    // the binary32 stencil and column solve of the mixed form
    const float* ogw32;
    const float* ohw32;
    const float* oh0_32;
    const float* oh1_32;
    const float* ogz32;
    const float* ohc32;
};

// Everything one instance's kernels need (device copy per solve).
template <typename T>
struct Inst {
    Geo g;
    T* P[KMAX + 1];
    T* AP[KMAX + 1];
    T* R[3];
    T* E;
    // octahedral mesh: L(e) of the step, stored by the dots pass and read by
    // the direction pass instead of a second indirect stencil (null on the
    // lat-lon mesh)
    T* LE;
    double* X[2];            // X[0]: caller's x, X[1]: workspace
    const double* rhs;
    SolveState* st;
    double* part;            // block partials [NV_MAX][pstride] (value-major)
    long long pstride;       // >= blocks of either grid
    double* hist;
    long long hist_cap;
    int nblk_col;            // blocks of the column grid
    int nblk_st;             // blocks of the stencil grid
    int kc;                  // stencil levels per block
    int tx, ty, tz;          // stencil tiles per dimension
    // the direction pass (the most registers per level) has its own level
    // tiling over the same columns
    int nblk_dir, kc_dir, tz_dir;
    // block orders (ORD_*) of the stencil grid and of the direction grid
    int ord_st, ord_dir;
};

// FT-GMRES(k) control state of one solve (device memory; written by single
// threads of the one-block kernels, and by the event preparation kernel).
struct GmState {
    int status;          // RUNNING or an FTGCR_* outcome
    int active;          // 1: the cycle's steps run
    int j;               // step index inside the cycle
    int k, ft;
    int phase;           // next restart pass: GM_INIT, GM_CHECK (a cycle ended), GM_REDO (after a rollback)
    int jdone;           // steps of this cycle that count
    int cycle_end;       // 1: the cycle is complete, its correction is pending
    int capped;          // 1: the step cap cut the cycle
    int x_cur, x_bak, x_dst;
    int detections, stagnation_accepts, events_applied, events_since_rb;
    int log_len;
    int ev_ok, ev_vec, ev_copy, ev_src, ev_dst;
    long long s, max_steps, accepted, cycles, last_rb_pos, b_accepted;
    double tol2, T, RR;
    double rho2;         // explicit |R - A x|^2 of the cycle's start (or of the last check)
    double b_rho2;       // the backup's
    double rr_old;       // |g_j|^2 of the previous step (the detector's reference)
    double den[KMAX + 1];            // stored U[i] = den[i] * v_i (1 once stored normalised)
    double H[(KMAX + 1) * KMAX];     // Hessenberg, row-major with row stride KMAX, rotated in place
    double cs[KMAX], sn[KMAX];       // Givens rotations
    double g[KMAX + 1];              // rotated right-hand side, g_0 = |s|
    DetectRec log[LOG_CAP];
};

// Everything the FT-GMRES kernels of one solve need (device copy per solve).
struct GmInst {
    Geo g;
    double* U[KMAX + 1];     // Arnoldi vectors v_i (v_0 = s / |s|), stored scaled by den[i] until normalised
    double* Z[KMAX];         // z_i = P^{-1} v_i
    double* W;               // A z_j, then the orthogonalised vector
    double* X[2];            // X[0]: caller's x, X[1]: workspace
    const double* rhs;
    GmState* st;
    double* part;
    long long pstride;
    double* hist;
    long long hist_cap;
    int nblk_st, kc, tx, ty, tz;
    int ord;                 // block order (ORD_*) of the stencil kernels
};

// Launch table for combined (batched) launches: block b of a launch belongs
// to instance inst_of(b); blk0[m] is the first block of instance m.
template <typename T>
struct Table {
    const Inst<T>* inst;
    const int* blk0_col;     // n + 1 prefix sums (column grid)
    const int* blk0_st;      // n + 1 prefix sums (stencil grid)
    const int* blk0_dir;     // n + 1 prefix sums (direction-pass grid)
    int n;
    int mesh = 0;            // every instance's mesh (FTGCR_MESH_*)
    int precond = FTGCR_PRECOND_COLUMN;   // every instance's preconditioner
    // 1: every instance's columns fill the two-lane column grid exactly
    // (nz = 2H levels, a whole number of 128-column blocks), so every lane
    // of the column pass owns every row it touches
    int full = 0;
};

// Whether a problem of ncols columns and nz levels fills the two-lane column
// grid exactly (Table::full).
inline bool full_columns(long long ncols, int nz, int H)
{
    return nz == 2 * H && ncols % COLS_PER_BLOCK == 0;
}

// Kernel launchers (kernels.hip).
template <typename T> struct Launch {
    static void init_state(const Table<T>& tb, int k, int ft, int mixed, long long max_steps, double tol2,
                           int reset_counters, int grid, hipStream_t s);
    static void set_round(const Table<T>& tb, double tol2, long long max_steps, hipStream_t s);
    static void residual(const Table<T>& tb, int total_st_blocks, int kc, int store, int set_T, hipStream_t s);
    // update_thomas, stencil_dots and dir_update take optional events that
    // the dispatch itself stamps with its start and stop times
    static void update_thomas(const Table<T>& tb, int total_col_blocks, int H, int mode, hipStream_t s,
                              hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
    static void finish_col(const Table<T>& tb, int mode, hipStream_t s);
    // spec = 1: before the step's decision, followed by finish_step
    static void stencil_dots(const Table<T>& tb, int total_st_blocks, int kc, int spec, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
    static void finish_step(const Table<T>& tb, hipStream_t s);   // finish_col + finish_alpha
    static void finish_alpha(const Table<T>& tb, hipStream_t s);
    static void finish_beta(const Table<T>& tb, int init, hipStream_t s);
    // nt_ap: load the L(p^l) with the non-temporal hint (nt_ap_hint)
    static void dir_update(const Table<T>& tb, int total_st_blocks, int kc, int init, bool nt_ap, hipStream_t s,
                           hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
    static void finalize_x(const Table<T>& tb, int total_st_blocks, int kc, hipStream_t s);
    // fault events (single instance)
    static void event_prep(const Table<T>& tb, int vec, hipStream_t s);
    static void event_copy(const Table<T>& tb, int grid, hipStream_t s);
    static void event_inject(const Table<T>& tb, int grid, const long long* idx, const unsigned char* bits,
                             long long count, long long start, int bit, hipStream_t s);
    static void beta_dots(const Table<T>& tb, int total_st_blocks, hipStream_t s);
    static void gather_status(const Table<T>& tb, long long* out, hipStream_t s);
    // parity entry points (FP64 only)
    static void debug_apply_A(const Table<T>& tb, int total_st_blocks, int kc, const double* in, double* out, hipStream_t s);
    static void debug_pinv(const Table<T>& tb, int total_col_blocks, int H, const double* in, double* out, hipStream_t s);
};

// FT-GMRES(k) launchers (kernels.hip); gi is the device copy of the solve's
// GmInst, `tb` the handle's single-instance table (geometry and column grid)
// for the column pass.
struct GmLaunch {
    static void init(const GmInst* gi, int k, int ft, long long max_steps, double tol2, hipStream_t s);
    static void residual(const GmInst* gi, int nblk_st, int kc, int mesh, hipStream_t s);
    static void restart(const GmInst* gi, hipStream_t s);
    static void precond(const Table<double>& tb, const GmInst* gi, int nblk_col, int H, hipStream_t s);
    // dots = 0: store A z_j only (the dots follow a fault event on it)
    static void stencil(const GmInst* gi, int nblk_st, int kc, int dots, int mesh, hipStream_t s);
    static void dots(const GmInst* gi, int nblk_st, int kc, hipStream_t s);
    static void finish_h(const GmInst* gi, hipStream_t s);
    static void orth(const GmInst* gi, int nblk_st, int kc, hipStream_t s);
    static void finish_step(const GmInst* gi, hipStream_t s);
    static void xupd(const GmInst* gi, int nblk_st, int kc, hipStream_t s);
    static void finish_x(const GmInst* gi, hipStream_t s);
    static void finalize(const GmInst* gi, int nblk_st, int kc, hipStream_t s);
    static void event_prep(const GmInst* gi, int vec, long long step, hipStream_t s);
    static void event_copy(const GmInst* gi, int nblk_st, int kc, hipStream_t s);
    static void event_inject(const GmInst* gi, int grid, const long long* idx, const unsigned char* bits,
                             long long count, long long start, int bit, hipStream_t s);
};

// Plain streaming copy of `bytes` (a multiple of 16, 16-byte aligned
// pointers): the bandwidth probe.
void launch_bw_copy(const void* src, void* dst, long long bytes, hipStream_t s);

// Smallest supported register-array depth H >= levels per column half.
int thomas_depth(int nz);

// Whether the direction pass should load the L(p^l) with the non-temporal
// hint: when the k + 1 images of A p of all solves in flight (n_total
// entries of elem bytes each) exceed most of the 256 MB Infinity Cache, so
// the next dots pass would not find them there anyway.
inline bool nt_ap_hint(int k, long long n_total, int elem)
{
    return (double)(k + 1) * (double)n_total * elem > 192.0 * 1024 * 1024;
}

}  // namespace ftgcr
