// FT-GCR device kernels for gfx950 (MI355X).
//
// One inner step of Algorithm 1 (FT-GCR(k), arXiv 2103.07210) runs as six
// launches, each a streaming pass over HBM or a one-block decision:
//
//   update_thomas   r+ = r + beta L(p^nu), <r+, r+> partials, e = P^{-1} r+
//   reduce_decide   exit test, monotone-norm fault test, backup or rollback
//   stencil_dots    L(e) and the partials of <L(e), L(p^l)>, l = 0..nu
//   reduce_alpha    alpha_l = -<L(e), L(p^l)> / <L(p^l), L(p^l)>
//   dir_update      p^{nu+1}, L(p^{nu+1}) (L(e) recomputed), the next beta's
//                   inner products, and at the end of a cycle the deferred
//                   iterate update phi += sum_l beta_l p^l
//   reduce_beta     beta numerator / denominator, pass and cycle bookkeeping
//
// Every reduction is deterministic: fixed per-block partition and order,
// butterfly wave sums (bitwise equal on every lane), fixed cross-wave order,
// then a fixed-order sum over block partials.  The detector's <r, r> is
// therefore a function of r alone, as the equality case of the test needs.
//
// Storage type T is double (FP64 solve) or float (mixed precision: binary32
// vectors, FP64 arithmetic in registers, FP64 inner products and iterate).
#include "ftgcr_internal.h"

namespace ftgcr {

enum { MODE_STEP = 0, MODE_INIT = 1, MODE_DEBUG = 2 };

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int find_inst(const int* blk0, int n, int b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (blk0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum over a 256-thread block; every thread gets the result.
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Fixed-order sum of one value over an instance's block partials.
__device__ __forceinline__ double sum_partials(const double* part, int nblk, int q, double* sh)
{
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RED_THREADS) acc += part[(long long)b * NV_MAX + q];
    return block_sum(acc, sh);
}

// Per-column constants: hill_amp * h at the five horizontal positions and
// the metric factors of the faces.
struct ColW {
    double hw, he, hs, hn, hc;
    double gx, gys, gyn, gz;
};

__device__ __forceinline__ ColW col_weights(const Geo& g, int i, int j)
{
    ColW c;
    const int iw = (i == 0) ? g.nx - 1 : i - 1;
    c.hw = g.hx[(long long)j * g.nx + iw];
    c.he = g.hx[(long long)j * g.nx + i];
    c.hs = g.hy[(long long)j * g.nx + i];
    c.hn = g.hy[(long long)(j + 1) * g.nx + i];
    c.hc = g.hc[(long long)j * g.nx + i];
    c.gx = g.Gx[j];
    c.gys = g.Gy[j];
    c.gyn = g.Gy[j + 1];
    c.gz = g.Gz[j];
    return c;
}

// Face weights W = c_face * metric of cell (i, j, k) and the diagonal
// (1 + sigma) * sum(W).  Zero-flux faces (poles, bottom, top) are exactly 0.
struct LevW {
    double w, e, s, n, b, a, diag;
};

__device__ __forceinline__ LevW level_weights(const ColW& c, const Geo& g, int k)
{
    LevW L;
    const double gk = g.gc[k];
    L.w = c.gx * (1.0 + c.hw * gk);
    L.e = c.gx * (1.0 + c.he * gk);
    L.s = c.gys * (1.0 + c.hs * gk);
    L.n = c.gyn * (1.0 + c.hn * gk);
    L.b = (k > 0) ? c.gz * (1.0 + c.hc * g.gf[k]) : 0.0;
    L.a = (k < g.nz - 1) ? c.gz * (1.0 + c.hc * g.gf[k + 1]) : 0.0;
    const double d0 = ((((L.w + L.e) + L.s) + L.n) + L.b) + L.a;
    L.diag = g.opsig * d0;
    return L;
}

__device__ __forceinline__ double apply_row(const LevW& L, double xc, double xw, double xe,
                                            double xs, double xn, double xb, double xa)
{
    double off = L.w * xw;
    off = fma(L.e, xe, off);
    off = fma(L.s, xs, off);
    off = fma(L.n, xn, off);
    off = fma(L.b, xb, off);
    off = fma(L.a, xa, off);
    return fma(L.diag, xc, -off);
}

// (A x) at levels k0 .. k0+KC-1 of column (i, j); missing neighbours
// (beyond the poles, bottom, top) enter as 0 with weight 0.
template <typename TI, int KC>
__device__ __forceinline__ void stencil_chunk(const Geo& g, const TI* __restrict__ x, int i, int j,
                                              int k0, double (&out)[KC])
{
    const ColW c = col_weights(g, i, j);
    const long long plane = (long long)g.ncols;
    const int iw = (i == 0) ? g.nx - 1 : i - 1;
    const int ie = (i == g.nx - 1) ? 0 : i + 1;
    const long long row = (long long)j * g.nx;
    double xprev = (k0 > 0) ? (double)x[row + i + plane * (k0 - 1)] : 0.0;
    double xcur = (double)x[row + i + plane * k0];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        if (k < g.nz) {
            const long long o = row + plane * k;
            const double xnext = (k + 1 < g.nz) ? (double)x[o + plane + i] : 0.0;
            const double xw = (double)x[o + iw];
            const double xe = (double)x[o + ie];
            const double xs = (j > 0) ? (double)x[o - g.nx + i] : 0.0;
            const double xn = (j < g.ny - 1) ? (double)x[o + g.nx + i] : 0.0;
            const LevW L = level_weights(c, g, k);
            out[kk] = apply_row(L, xcur, xw, xe, xs, xn, xprev, xnext);
            xprev = xcur;
            xcur = xnext;
        } else {
            out[kk] = 0.0;
        }
    }
}

// Stencil-grid coordinates of this thread.
struct StPos {
    int i, j, k0;
    bool valid;
};

template <typename T>
__device__ __forceinline__ StPos st_pos(const Inst<T>& in, int lb)
{
    StPos p;
    const int bx = lb % in.tx;
    const int t = lb / in.tx;
    const int by = t % in.ty;
    const int bz = t / in.ty;
    p.i = bx * ST_TX + (threadIdx.x & (ST_TX - 1));
    p.j = by * ST_TY + (threadIdx.x / ST_TX);
    p.k0 = bz * in.kc;
    p.valid = p.i < in.g.nx && p.j < in.g.ny && p.k0 < in.g.nz;
    return p;
}

template <typename T>
__device__ __forceinline__ void write_xor(T* p, int bit);

template <>
__device__ __forceinline__ void write_xor<double>(double* p, int bit)
{
    atomicXor(reinterpret_cast<unsigned long long*>(p), 1ull << bit);
}

template <>
__device__ __forceinline__ void write_xor<float>(float* p, int bit)
{
    atomicXor(reinterpret_cast<unsigned int*>(p), 1u << bit);
}

__device__ __forceinline__ int other_r(int a, int b)
{
    for (int q = 0; q < 3; ++q)
        if (q != a && q != b) return q;
    return 0;
}

__device__ __forceinline__ void assign_slots(SolveState* st, int k)
{
    const int s0 = st->slot[0];
    int q = 1;
    for (int l = 0; l <= k; ++l)
        if (l != s0) st->slot[q++] = l;
}

// ---------------------------------------------------------------------------
// state setup
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_init_state(Table<T> tb, int k, int ft, int mixed, long long max_steps, double tol2,
                             int reset_counters)
{
    const int m = blockIdx.x;
    if (m >= tb.n || threadIdx.x != 0) return;
    SolveState* st = tb.inst[m].st;
    if (reset_counters) {
        st->s = 0;
        st->accepted = 0;
        st->cycles = 0;
        st->detections = 0;
        st->stagnation_accepts = 0;
        st->events_applied = 0;
        st->log_len = 0;
    }
    st->last_rb_pos = -1;
    st->events_since_rb = 1;
    st->status = RUNNING;
    st->active = 0;
    st->nu = 0;
    st->k = k;
    st->ft = ft;
    st->mixed = mixed;
    st->max_steps = max_steps;
    st->tol2 = tol2;
    for (int l = 0; l <= KMAX; ++l) {
        st->slot[l] = l;
        st->d[l] = 0.0;
        st->beta[l] = 0.0;
        st->alpha[l] = 0.0;
    }
    st->r_cur = 0;
    st->r_dst = 0;
    st->r_bak = 0;
    st->x_base = 0;
    st->x_base_nu = 0;
    st->x_bak = 0;
    st->x_dst = 0;
    st->x_final_hi = -1;
    st->ev_ok = 0;
}

// r = A x - R (x = caller's FP64 iterate), stored in R[r_dst] when `store`;
// partials: <R, R> and <r, r> of the unrounded FP64 residual.
template <typename T, int KC>
__global__ __launch_bounds__(ST_THREADS) void k_residual(Table<T> tb, int store)
{
    __shared__ double sh[4];
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    const StPos ps = st_pos(in, lb);
    double rr = 0.0, bb = 0.0;
    if (ps.valid) {
        double ax[KC];
        stencil_chunk<double, KC>(in.g, in.X[0], ps.i, ps.j, ps.k0, ax);
        T* rout = in.R[in.st->r_dst];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int k = ps.k0 + kk;
            if (k < in.g.nz) {
                const long long c = (long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * k;
                const double b = in.rhs[c];
                const double r = ax[kk] - b;
                if (store) rout[c] = (T)r;
                rr = fma(r, r, rr);
                bb = fma(b, b, bb);
            }
        }
    }
    const double sb = block_sum(bb, sh);
    const double sr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        in.part[(long long)lb * NV_MAX + 0] = sb;
        in.part[(long long)lb * NV_MAX + 1] = sr;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_residual(Table<T> tb, int set_T)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[blockIdx.x];
    const double RR = sum_partials(in.part, in.nblk_st, 0, sh);
    const double rt2 = sum_partials(in.part, in.nblk_st, 1, sh);
    if (threadIdx.x == 0) {
        SolveState* st = in.st;
        st->RR = RR;
        st->rt2 = rt2;
        if (set_T) st->T = st->tol2 * (st->mixed ? rt2 : RR);
    }
}

// ---------------------------------------------------------------------------
// update + column preconditioner
// ---------------------------------------------------------------------------
//
// Each column (i, j) is split between two lanes of a wave (lane l and l+32):
// the lower lane eliminates levels 0 .. h-1 upward (Thomas forward sweep),
// the upper lane levels nz-1 .. h downward; they meet at row h-1, exchange
// one pivot pair by a lane shuffle, and each back-substitutes its half.  The
// elimination state of a half column (at most H levels) stays in registers.
// P's rows: a_k e_{k-1} + b_k e_k + u_k e_{k+1} = r_k with b the diagonal of
// A and a, u minus the vertical face weights.

template <typename T, int H>
__global__ __launch_bounds__(COL_THREADS) void k_update_thomas(Table<T> tb, int mode, const T* dbg_in,
                                                               T* dbg_out)
{
    __shared__ double sh[4];
    const int m = find_inst(tb.blk0_col, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_col[m];
    SolveState* st = in.st;
    if (mode != MODE_DEBUG) {
        if (st->status != RUNNING) return;
        if (mode == MODE_STEP && st->d_cur == 0.0) return;
    }
    const Geo& g = in.g;
    const int lane = threadIdx.x & 63;
    const bool upper = lane >= 32;
    const int col = lb * COLS_PER_BLOCK + (threadIdx.x >> 6) * 32 + (lane & 31);
    const bool valid = col < g.ncols;
    const int j = valid ? col / g.nx : 0;
    const int i = valid ? col - j * g.nx : 0;
    const long long plane = (long long)g.ncols;
    const int nz = g.nz;
    const int h = (nz + 1) >> 1;   // lower half: levels [0, h)
    const int nup = nz - h;        // upper half: levels [h, nz)
    const ColW c = col_weights(g, i, j);

    const T* rin;
    const T* ap = nullptr;
    T* rout = nullptr;
    T* eout;
    double beta = 0.0;
    if (mode == MODE_DEBUG) {
        rin = dbg_in;
        eout = dbg_out;
    } else {
        rin = in.R[st->r_cur];
        eout = in.E;
        if (mode == MODE_STEP) {
            ap = in.AP[st->slot[st->nu]];
            rout = in.R[st->r_dst];
            beta = -st->beta_num / st->d_cur;
        }
    }

    double acc_new = 0.0, acc_st = 0.0;
    double ga[H], de[H];
    double carry_g = 0.0, carry_d = 0.0;   // pivot pair carried along the sweep
    double mm = 1.0, ff = 0.0, uu = 0.0;   // meeting row (lower lane)
    const int nmine = upper ? nup : h;

#pragma unroll
    for (int q = 0; q < H; ++q) {
        if (q < nmine) {
            const int k = upper ? nz - 1 - q : q;
            const long long o = (long long)col + plane * k;
            double rp = 0.0;
            if (valid) {
                if (mode == MODE_STEP) {
                    const double v = fma(beta, (double)ap[o], (double)rin[o]);
                    const T sv = (T)v;
                    rout[o] = sv;
                    rp = (double)sv;
                    acc_new = fma(v, v, acc_new);
                    acc_st = fma(rp, rp, acc_st);
                } else {
                    rp = (double)rin[o];
                    acc_new = fma(rp, rp, acc_new);
                    acc_st = fma(rp, rp, acc_st);
                }
            }
            const LevW L = level_weights(c, g, k);
            const double a = -L.b, u = -L.a, b = L.diag;
            if (!upper) {
                const double mk = (q == 0) ? b : b - a * carry_g;
                const double fk = (q == 0) ? rp : rp - a * carry_d;
                if (q < h - 1) {
                    const double inv = 1.0 / mk;
                    carry_g = u * inv;
                    carry_d = fk * inv;
                    ga[q] = carry_g;
                    de[q] = carry_d;
                } else {
                    mm = mk;
                    ff = fk;
                    uu = u;
                }
            } else {
                const double den = (q == 0) ? b : b - u * carry_g;
                const double fk = (q == 0) ? rp : rp - u * carry_d;
                const double inv = 1.0 / den;
                carry_g = a * inv;
                carry_d = fk * inv;
                ga[q] = carry_g;
                de[q] = carry_d;
            }
        }
    }
    // meeting row: lower lane gets (zeta_h, eps_h) from its upper partner
    const double zx = __shfl_xor(carry_g, 32);
    const double ex = __shfl_xor(carry_d, 32);
    double xm = 0.0;
    if (!upper) xm = (ff - uu * ex) / (mm - uu * zx);
    const double xl = __shfl_xor(xm, 32);
    if (valid) {
        if (!upper) {
            eout[(long long)col + plane * (h - 1)] = (T)xm;
            double xv = xm;
#pragma unroll
            for (int q = H - 1; q >= 0; --q) {
                if (q <= h - 2) {
                    xv = de[q] - ga[q] * xv;
                    eout[(long long)col + plane * q] = (T)xv;
                }
            }
        } else {
            double xv = xl;
#pragma unroll
            for (int q = H - 1; q >= 0; --q) {
                if (q < nup) {
                    xv = de[q] - ga[q] * xv;
                    eout[(long long)col + plane * (nz - 1 - q)] = (T)xv;
                }
            }
        }
    }
    if (mode != MODE_DEBUG) {
        const double sn = block_sum(acc_new, sh);
        const double ss = block_sum(acc_st, sh);
        if (threadIdx.x == 0) {
            in.part[(long long)lb * NV_MAX + 0] = sn;
            in.part[(long long)lb * NV_MAX + 1] = ss;
        }
    }
}

// After the initial residual and P^{-1} r^0: <r^0, r^0>, the exit test, and
// the initial known-good state.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_init(Table<T> tb)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    if (st->status != RUNNING) return;
    const double rn = sum_partials(in.part, in.nblk_col, 0, sh);
    const double rs = sum_partials(in.part, in.nblk_col, 1, sh);
    if (threadIdx.x == 0) {
        st->rr_new = rn;
        st->rr_old = rs;
        if (rs <= st->T) {
            st->status = FTGCR_CONVERGED;
            st->x_final_hi = -1;
        }
        st->b_rr = rs;
        st->b_accepted = st->accepted;
        st->b_slot0 = st->slot[0];
        st->r_bak = st->r_cur;
        st->x_bak = st->x_base;
    }
}

// ---------------------------------------------------------------------------
// decision of one step (Algorithm 1, exit test and red part)
// ---------------------------------------------------------------------------

__device__ void rollback(SolveState* st)
{
    st->slot[0] = st->b_slot0;
    assign_slots(st, st->k);
    st->r_cur = st->r_bak;
    st->r_dst = other_r(st->r_cur, st->r_cur);
    st->x_base = st->x_bak;
    st->x_base_nu = 0;
    st->rr_old = st->b_rr;
    st->beta_num = st->b_beta_num;
    st->d_cur = st->b_d0;
    st->d[0] = st->b_d0;
    st->accepted = st->b_accepted;
    st->nu = 0;
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_decide(Table<T> tb)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    if (st->status != RUNNING) return;
    const double rn = sum_partials(in.part, in.nblk_col, 0, sh);
    const double rs = sum_partials(in.part, in.nblk_col, 1, sh);
    if (threadIdx.x != 0) return;
    const int nu = st->nu;
    st->s += 1;
    const long long s = st->s;
    if (st->d_cur == 0.0) {   // <L p, L p> = 0: beta undefined
        st->status = FTGCR_BREAKDOWN;
        st->x_final_hi = nu - 1;
        st->active = 0;
        return;
    }
    if (nu == 0) st->cycles += 1;
    if (s <= in.hist_cap) in.hist[s - 1] = rn;
    st->beta[nu] = -st->beta_num / st->d_cur;
    st->rr_new = rn;
    if (rs <= st->T) {   // exit test first
        st->accepted += 1;
        st->rr_old = rs;
        st->r_cur = st->r_dst;
        st->status = FTGCR_CONVERGED;
        st->x_final_hi = nu;
        st->active = 0;
        return;
    }
    if (st->ft && !(rn < st->rr_old)) {   // norm did not decrease (NaN included)
        const long long pos = st->accepted + 1;
        const int stag = (pos == st->last_rb_pos) && !st->events_since_rb;
        st->detections += 1;
        if (st->log_len < LOG_CAP) {
            DetectRec& rec = st->log[st->log_len++];
            rec.step = s;
            rec.nu = nu;
            rec.action = stag;
            rec.rr_old = st->rr_old;
            rec.rr_new = rn;
        }
        if (!stag) {
            rollback(st);
            st->last_rb_pos = pos;
            st->events_since_rb = 0;
            st->active = 0;
            if (s >= st->max_steps) {
                st->status = FTGCR_MAX_STEPS;
                st->x_final_hi = -1;
            }
            return;
        }
        st->stagnation_accepts += 1;
    }
    if (st->ft && nu == 0) {   // this pass opens a cycle: it becomes the backup
        st->b_rr = st->rr_old;
        st->b_beta_num = st->beta_num;
        st->b_d0 = st->d_cur;
        st->b_accepted = st->accepted;
        st->b_slot0 = st->slot[0];
        st->r_bak = st->r_cur;
        st->x_bak = st->x_base;
    }
    st->accepted += 1;
    st->rr_old = rs;
    st->r_cur = st->r_dst;
    st->active = 1;
    if (s >= st->max_steps) {
        st->status = FTGCR_MAX_STEPS;
        st->x_final_hi = nu;
        st->active = 0;
    }
}

// ---------------------------------------------------------------------------
// L(e) and orthogonalisation inner products
// ---------------------------------------------------------------------------

template <typename T, int KC>
__global__ __launch_bounds__(ST_THREADS) void k_stencil_dots(Table<T> tb)
{
    __shared__ double sh[4];
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    const SolveState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    const int nu = st->nu;
    const StPos ps = st_pos(in, lb);
    double le[KC];
    if (ps.valid) stencil_chunk<T, KC>(in.g, in.E, ps.i, ps.j, ps.k0, le);
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * ps.k0;
    for (int l = 0; l <= nu; ++l) {
        const T* apl = in.AP[st->slot[l]];
        double acc = 0.0;
        if (ps.valid) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk)
                if (ps.k0 + kk < in.g.nz) acc = fma(le[kk], (double)apl[c0 + (long long)in.g.ncols * kk], acc);
        }
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0) in.part[(long long)lb * NV_MAX + l] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_alpha(Table<T> tb)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    const int nu = st->nu;
    for (int l = 0; l <= nu; ++l) {
        const double s = sum_partials(in.part, in.nblk_st, l, sh);
        if (threadIdx.x == 0) st->alpha[l] = -s / st->d[l];
    }
    if (threadIdx.x == 0) st->x_dst = (st->x_base == st->x_bak) ? 1 - st->x_base : st->x_base;
}

// ---------------------------------------------------------------------------
// new direction, its image, next beta's inner products, deferred iterate
// ---------------------------------------------------------------------------

template <typename T, int KC>
__global__ __launch_bounds__(ST_THREADS) void k_dir_update(Table<T> tb, int init)
{
    __shared__ double sh[4];
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    const SolveState* st = in.st;
    if (st->status != RUNNING) return;
    if (!init && !st->active) return;
    const int nu = init ? -1 : st->nu;
    const int target = st->slot[nu + 1];
    const bool xupd = !init && (nu == st->k - 1);
    const int xlo = st->x_base_nu;
    const StPos ps = st_pos(in, lb);
    double le[KC];
    if (ps.valid) stencil_chunk<T, KC>(in.g, in.E, ps.i, ps.j, ps.k0, le);
    double acc_num = 0.0, acc_d = 0.0;
    if (ps.valid) {
        T* pout = in.P[target];
        T* apout = in.AP[target];
        const T* r = in.R[st->r_cur];
        const double* xb = in.X[st->x_base];
        double* xo = in.X[st->x_dst];
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            if (ps.k0 + kk < in.g.nz) {
                const long long c = (long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * (ps.k0 + kk);
                double p = (double)in.E[c];
                double a = le[kk];
                double xa = xupd ? xb[c] : 0.0;
                for (int l = 0; l <= nu; ++l) {
                    const int sl = st->slot[l];
                    const double pl = (double)in.P[sl][c];
                    const double al = st->alpha[l];
                    p = fma(al, pl, p);
                    a = fma(al, (double)in.AP[sl][c], a);
                    if (xupd && l >= xlo) xa = fma(st->beta[l], pl, xa);
                }
                const T ps_ = (T)p;
                const T as_ = (T)a;
                pout[c] = ps_;
                apout[c] = as_;
                if (xupd) xo[c] = xa;
                const double ad = (double)as_;
                acc_num = fma((double)r[c], ad, acc_num);
                acc_d = fma(ad, ad, acc_d);
            }
        }
    }
    const double sn = block_sum(acc_num, sh);
    const double sd = block_sum(acc_d, sh);
    if (threadIdx.x == 0) {
        in.part[(long long)lb * NV_MAX + 0] = sn;
        in.part[(long long)lb * NV_MAX + 1] = sd;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_beta(Table<T> tb, int init)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    if (st->status != RUNNING) return;
    if (!init && !st->active) return;
    const double num = sum_partials(in.part, in.nblk_st, 0, sh);
    const double dn = sum_partials(in.part, in.nblk_st, 1, sh);
    if (threadIdx.x != 0) return;
    st->beta_num = num;
    st->d_cur = dn;
    if (init) {
        st->d[0] = dn;
        st->b_beta_num = num;
        st->b_d0 = dn;
        st->r_dst = other_r(st->r_cur, st->r_bak);
        return;
    }
    const int nu = st->nu;
    if (nu + 1 == st->k) {   // end of the k passes: p^k opens the next cycle
        st->x_base = st->x_dst;
        st->x_base_nu = 0;
        st->slot[0] = st->slot[st->k];
        assign_slots(st, st->k);
        st->nu = 0;
        st->d[0] = dn;
        st->r_dst = other_r(st->r_cur, st->r_bak);
    } else {
        st->nu = nu + 1;
        st->d[nu + 1] = dn;
        st->r_dst = st->r_cur;
    }
}

// x = x_base + sum_{l = x_base_nu .. x_final_hi} beta_l p^l, into X[0].
template <typename T, int KC>
__global__ __launch_bounds__(ST_THREADS) void k_finalize_x(Table<T> tb)
{
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    const SolveState* st = in.st;
    const int lo = st->x_base_nu, hi = st->x_final_hi;
    if (st->x_base == 0 && hi < lo) return;
    const StPos ps = st_pos(in, lb);
    if (!ps.valid) return;
    const double* xb = in.X[st->x_base];
    double* xo = in.X[0];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        if (ps.k0 + kk < in.g.nz) {
            const long long c = (long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * (ps.k0 + kk);
            double xa = xb[c];
            for (int l = lo; l <= hi; ++l) xa = fma(st->beta[l], (double)in.P[st->slot[l]][c], xa);
            xo[c] = xa;
        }
    }
}

// ---------------------------------------------------------------------------
// fault events (harness): prepare target buffers, copy-on-write, flip bits
// ---------------------------------------------------------------------------
//
// The working vectors share buffers with the backup where that is free
// (the backup of p^0 / L(p^0) is the slot itself; x and r keep their
// cycle-start buffer).  A flip must never reach the backup, so when the
// current vector still is the backup's buffer it is first copied.

template <typename T>
__global__ void k_event_prep(Table<T> tb, int vec)
{
    if (threadIdx.x != 0) return;
    SolveState* st = tb.inst[0].st;
    st->ev_ok = (st->status == RUNNING);
    if (!st->ev_ok) return;
    st->ev_vec = vec;
    st->ev_copy = 0;
    const int nu = st->nu;
    if (vec == FTGCR_V_X) {
        // materialise the iterate of this step: x_base + sum_{l < nu} beta_l p^l
        const int src = st->x_base;
        const int dst = (st->x_base == st->x_bak) ? 1 - st->x_base : st->x_base;
        st->ev_src = src;
        st->ev_dst = dst;
        st->ev_lo = st->x_base_nu;
        st->ev_hi = nu;
        st->ev_copy = (src != dst) || (nu > st->x_base_nu);
        st->x_base = dst;
        st->x_base_nu = nu;
    } else if (vec == FTGCR_V_R) {
        if (st->r_cur == st->r_bak) {
            const int dst = other_r(st->r_cur, st->r_dst);
            st->ev_src = st->r_cur;
            st->ev_dst = dst;
            st->ev_copy = 1;
            st->r_cur = dst;
            if (nu > 0) st->r_dst = dst;
        }
    } else {
        if (nu == 0 && st->slot[0] == st->b_slot0) {
            const int src = st->slot[0];
            const int dst = st->slot[1];
            st->ev_src = src;
            st->ev_dst = dst;
            st->ev_copy = 1;
            st->slot[0] = dst;
            st->slot[1] = src;
        }
    }
}

template <typename T>
__global__ void k_event_copy(Table<T> tb)
{
    const Inst<T>& in = tb.inst[0];
    const SolveState* st = in.st;
    if (!st->ev_ok || !st->ev_copy) return;
    const long long n = in.g.n;
    const int vec = st->ev_vec;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += stride) {
        if (vec == FTGCR_V_X) {
            double xa = in.X[st->ev_src][c];
            for (int l = st->ev_lo; l < st->ev_hi; ++l)
                xa = fma(st->beta[l], (double)in.P[st->slot[l]][c], xa);
            in.X[st->ev_dst][c] = xa;
        } else if (vec == FTGCR_V_R) {
            in.R[st->ev_dst][c] = in.R[st->ev_src][c];
        } else {
            in.P[st->ev_dst][c] = in.P[st->ev_src][c];
            in.AP[st->ev_dst][c] = in.AP[st->ev_src][c];
        }
    }
}

template <typename T>
__global__ void k_event_inject(Table<T> tb, const long long* idx, const unsigned char* bits, long long count,
                               long long start, int bit0)
{
    const Inst<T>& in = tb.inst[0];
    SolveState* st = in.st;
    if (!st->ev_ok) return;
    const int vec = st->ev_vec;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        const long long at = idx ? idx[t] : start + t;
        const int bit = bits ? (int)bits[t] : bit0;
        if (vec == FTGCR_V_X) write_xor<double>(in.X[st->x_base] + at, bit);
        else if (vec == FTGCR_V_R) write_xor<T>(in.R[st->r_cur] + at, bit);
        else if (vec == FTGCR_V_P) write_xor<T>(in.P[st->slot[st->nu]] + at, bit);
        else write_xor<T>(in.AP[st->slot[st->nu]] + at, bit);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->events_applied += 1;
        st->events_since_rb = 1;
    }
}

// <r, L p^nu> and <L p^nu, L p^nu> recomputed after a flip in r or L(p^nu).
template <typename T>
__global__ __launch_bounds__(ST_THREADS) void k_beta_dots(Table<T> tb)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[0];
    const SolveState* st = in.st;
    if (!st->ev_ok) return;
    const int lb = blockIdx.x;
    const StPos ps = st_pos(in, lb);
    double an = 0.0, ad = 0.0;
    if (ps.valid) {
        const T* r = in.R[st->r_cur];
        const T* ap = in.AP[st->slot[st->nu]];
        for (int kk = 0; kk < in.kc; ++kk) {
            if (ps.k0 + kk < in.g.nz) {
                const long long c = (long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * (ps.k0 + kk);
                const double a = (double)ap[c];
                an = fma((double)r[c], a, an);
                ad = fma(a, a, ad);
            }
        }
    }
    const double sn = block_sum(an, sh);
    const double sd = block_sum(ad, sh);
    if (threadIdx.x == 0) {
        in.part[(long long)lb * NV_MAX + 0] = sn;
        in.part[(long long)lb * NV_MAX + 1] = sd;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_reduce_beta_dots(Table<T> tb)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[0];
    SolveState* st = in.st;
    if (!st->ev_ok) return;
    const double num = sum_partials(in.part, in.nblk_st, 0, sh);
    const double dn = sum_partials(in.part, in.nblk_st, 1, sh);
    if (threadIdx.x == 0) {
        st->beta_num = num;
        st->d_cur = dn;
        st->d[st->nu] = dn;
    }
}

// ---------------------------------------------------------------------------
// parity entry points
// ---------------------------------------------------------------------------

template <int KC>
__global__ __launch_bounds__(ST_THREADS) void k_debug_apply_A(Table<double> tb, const double* x, double* y)
{
    const Inst<double>& in = tb.inst[0];
    const StPos ps = st_pos(in, blockIdx.x);
    if (!ps.valid) return;
    double ax[KC];
    stencil_chunk<double, KC>(in.g, x, ps.i, ps.j, ps.k0, ax);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
        if (ps.k0 + kk < in.g.nz)
            y[(long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * (ps.k0 + kk)] = ax[kk];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define FTGCR_KC_SWITCH(kc, CALL)            \
    switch (kc) {                            \
    case 1: { constexpr int KCV = 1; CALL; } break;   \
    case 2: { constexpr int KCV = 2; CALL; } break;   \
    case 4: { constexpr int KCV = 4; CALL; } break;   \
    case 8: { constexpr int KCV = 8; CALL; } break;   \
    default: { constexpr int KCV = 16; CALL; } break; \
    }

#define FTGCR_H_SWITCH(H, CALL)                       \
    switch (H) {                                      \
    case 4: { constexpr int HV = 4; CALL; } break;    \
    case 8: { constexpr int HV = 8; CALL; } break;    \
    case 16: { constexpr int HV = 16; CALL; } break;  \
    case 24: { constexpr int HV = 24; CALL; } break;  \
    case 32: { constexpr int HV = 32; CALL; } break;  \
    default: { constexpr int HV = 48; CALL; } break;  \
    }

int thomas_depth(int nz)
{
    const int h = (nz + 1) / 2;
    const int depths[] = {4, 8, 16, 24, 32, 48};
    for (int d : depths)
        if (h <= d) return d;
    return -1;
}

template <typename T>
void Launch<T>::init_state(const Table<T>& tb, int k, int ft, int mixed, long long max_steps, double tol2,
                           int reset_counters, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state<T>, dim3(grid), dim3(64), 0, s, tb, k, ft, mixed, max_steps, tol2,
                       reset_counters);
}

template <typename T>
void Launch<T>::residual(const Table<T>& tb, int total, int kc, int store, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_residual<T, KCV>), dim3(total), dim3(ST_THREADS), 0, s, tb, store));
}

template <typename T>
void Launch<T>::reduce_residual(const Table<T>& tb, int n, int set_T, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_residual<T>, dim3(n), dim3(RED_THREADS), 0, s, tb, set_T);
}

template <typename T>
void Launch<T>::update_thomas(const Table<T>& tb, int total, int H, int mode, hipStream_t s)
{
    FTGCR_H_SWITCH(H, hipLaunchKernelGGL((k_update_thomas<T, HV>), dim3(total), dim3(COL_THREADS), 0, s, tb,
                                         mode, (const T*)nullptr, (T*)nullptr));
}

template <typename T>
void Launch<T>::reduce_init(const Table<T>& tb, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_init<T>, dim3(n), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::reduce_decide(const Table<T>& tb, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_decide<T>, dim3(n), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::stencil_dots(const Table<T>& tb, int total, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_stencil_dots<T, KCV>), dim3(total), dim3(ST_THREADS), 0, s, tb));
}

template <typename T>
void Launch<T>::reduce_alpha(const Table<T>& tb, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_alpha<T>, dim3(n), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::dir_update(const Table<T>& tb, int total, int kc, int init, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_dir_update<T, KCV>), dim3(total), dim3(ST_THREADS), 0, s, tb, init));
}

template <typename T>
void Launch<T>::reduce_beta(const Table<T>& tb, int n, int init, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_beta<T>, dim3(n), dim3(RED_THREADS), 0, s, tb, init);
}

template <typename T>
void Launch<T>::finalize_x(const Table<T>& tb, int total, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_finalize_x<T, KCV>), dim3(total), dim3(ST_THREADS), 0, s, tb));
}

template <typename T>
void Launch<T>::event_prep(const Table<T>& tb, int vec, hipStream_t s)
{
    hipLaunchKernelGGL(k_event_prep<T>, dim3(1), dim3(64), 0, s, tb, vec);
}

template <typename T>
void Launch<T>::event_copy(const Table<T>& tb, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_event_copy<T>, dim3(grid), dim3(256), 0, s, tb);
}

template <typename T>
void Launch<T>::event_inject(const Table<T>& tb, int grid, const long long* idx, const unsigned char* bits,
                             long long count, long long start, int bit, hipStream_t s)
{
    hipLaunchKernelGGL(k_event_inject<T>, dim3(grid), dim3(256), 0, s, tb, idx, bits, count, start, bit);
}

template <typename T>
void Launch<T>::beta_dots(const Table<T>& tb, int total, hipStream_t s)
{
    hipLaunchKernelGGL(k_beta_dots<T>, dim3(total), dim3(ST_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::reduce_beta_dots(const Table<T>& tb, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_beta_dots<T>, dim3(n), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::debug_apply_A(const Table<T>&, int, int, const double*, double*, hipStream_t)
{
}

template <>
void Launch<double>::debug_apply_A(const Table<double>& tb, int total, int kc, const double* in, double* out,
                                   hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_debug_apply_A<KCV>), dim3(total), dim3(ST_THREADS), 0, s, tb, in, out));
}

template <typename T>
void Launch<T>::debug_pinv(const Table<T>&, int, int, const double*, double*, hipStream_t)
{
}

template <>
void Launch<double>::debug_pinv(const Table<double>& tb, int total, int H, const double* in, double* out,
                                hipStream_t s)
{
    FTGCR_H_SWITCH(H, hipLaunchKernelGGL((k_update_thomas<double, HV>), dim3(total), dim3(COL_THREADS), 0, s,
                                         tb, (int)MODE_DEBUG, in, out));
}

template struct Launch<double>;
template struct Launch<float>;

}  // namespace ftgcr
