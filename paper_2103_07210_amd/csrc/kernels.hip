// FT-GCR device kernels for gfx950 (MI355X).
//
// One inner step of Algorithm 1 (FT-GCR(k), arXiv 2103.07210) runs as three
// streaming passes over HBM and two one-block reductions:
//
//   update_thomas   r+ = r + beta L(p^nu), <r+, r+> partials, e = P^{-1} r+
//   stencil_dots    L(e) and the partials of <L(e), L(p^l)>, l = 0..nu
//                   (launched before the step's decision: it writes only
//                   its partials and reads nothing the decision changes)
//     finish_step   exit test, monotone-norm fault test, backup or rollback
//                   (Algorithm 1, red part), then
//                   alpha_l = -<L(e), L(p^l)> / <L(p^l), L(p^l)>
//   dir_update      p^{nu+1}, L(p^{nu+1}) (L(e) recomputed), the next beta's
//                   inner products, and at the end of a cycle the deferred
//                   iterate update phi += sum_l beta_l p^l
//     finish_beta   beta, pass and cycle bookkeeping
//
// A step with faults to inject into e takes the decision in a launch of its
// own (finish_col) so the injection can follow it, then finish_alpha after
// the dots pass: the same arithmetic in the same order.
//
// The reductions are separate launches on purpose: a grid-wide "last block
// finishes" scheme needs a device-scope fence and a same-address atomic per
// block, which across the eight XCDs (eight L2s) of MI355X costs far more
// than a launch.  Every reduction is deterministic: fixed per-block partition
// and order, butterfly wave sums (bitwise equal on every lane), fixed
// cross-wave order, then a fixed-order sum over the block partials.  The
// detector's <r, r> is therefore a function of r alone, as the equality case
// of the test needs.
//
// Storage type T is double (FP64 solve) or float (mixed precision: binary32
// vectors, FP64 arithmetic in registers, FP64 inner products and iterate).
#include <hip/hip_ext.h>

#include <cstddef>

#include "ftgcr_internal.h"

namespace ftgcr {

enum { MODE_STEP = 0, MODE_INIT = 1, MODE_DEBUG = 2, MODE_GM = 3 };
enum { GM_INIT = 0, GM_CHECK = 1, GM_REDO = 2 };

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

// Pointers that pass through LDS (per-block tables of the direction
// vectors) or through an empty asm statement come back as generic pointers,
// and accesses through them compile to flat instructions, which count
// against both the memory and the LDS counters: every LDS access and wave
// shuffle after them would wait for all outstanding HBM traffic.  The
// vectors are in global memory; these views say so.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
using gptr_mut = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p)
{
    return (gptr<T>)p;
}

template <typename T>
__device__ __forceinline__ gptr_mut<T> as_global_mut(T* p)
{
    return (gptr_mut<T>)p;
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_read(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes as a pairwise tree in lane order,
// ((v0 + v1) + (v2 + v3)) + ..., bitwise equal in every lane: DPP moves
// pair lanes l ^ 1 and l ^ 2 (quad permutes), then quads and half rows
// (half-row and row mirrors: every lane of a quad, then of a half row,
// holds the same value, so a mirror pairs the right partial sums; a + b and
// b + a round alike); the four row sums are read by readlane.  No LDS
// traffic.  Every lane must be active.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_mov_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov_f64<0x141>(v);   // row_half_mirror
    v += dpp_mov_f64<0x140>(v);   // row_mirror
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
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

// Fixed-order sums of values 0..nv-1 over an instance's block partials
// (value-major: a value's partials are contiguous, value q in row row0 + q),
// by one RED_THREADS block:
// thread t adds blocks t, t + RED_THREADS, ... in order, then the waves are
// summed in a fixed order.  Values are taken G at a time, and each thread
// issues the loads of U of its blocks for all G values before the first add,
// so up to G * U * RED_THREADS partials cost one round trip to memory; the
// order of the additions is the same for every (G, U).  The returned LDS
// array holds the nv sums; out, if not null, gets the first two of them in
// registers.  Both are valid in every thread.
template <int G, int U, typename I>
__device__ __forceinline__ const double* sum_partials(const I& in, int nblk, int row0, int nv, double* out)
{
    constexpr int NW = RED_THREADS / 64;
    __shared__ double sh[NV_MAX][NW];
    __shared__ double res[NV_MAX];
    const gptr<double> part = as_global(in.part);
    const long long stride = in.pstride;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q0 = 0; q0 < nv; q0 += G) {
        double acc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] = 0.0;
        for (int b0 = threadIdx.x; b0 < nblk; b0 += U * RED_THREADS) {
            double v[U][G];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int b = b0 + u * RED_THREADS;
#pragma unroll
                for (int g = 0; g < G; ++g)
                    v[u][g] = (b < nblk && q0 + g < nv) ? part[(long long)(row0 + q0 + g) * stride + b] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (b0 + u * RED_THREADS < nblk) {
#pragma unroll
                    for (int g = 0; g < G; ++g) acc[g] += v[u][g];
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (q0 + g < nv) {
                const double t = wave_sum(acc[g]);
                if (lane == 0) sh[q0 + g][w] = t;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double t = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) t += sh[threadIdx.x][ww];
        res[threadIdx.x] = t;
    }
    __syncthreads();
    if (out != nullptr)
        for (int q = 0; q < 2 && q < nv; ++q) out[q] = res[q];
    return res;
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

// Per-column constants of a row of A.  A horizontal face weight is
// G * (1 + h * g_k) (metric G, hill term h, vertical decay g_k at the cell's
// level), so the horizontal part of a row splits into a level-independent
// sum and a second one scaled by g_k:
//   sum_f W_f x_f = (Gx (x_w + x_e) + Gy_s x_s + Gy_n x_n)
//                 + g_k (Gx h_w x_w + Gx h_e x_e + Gy_s h_s x_s + Gy_n h_n x_n)
// and the horizontal part of the diagonal is h0 + g_k h1.  The column solve
// forms the same diagonal from the same constants, so P's diagonal is A's
// bit for bit.
struct RowC {
    double gx, gys, gyn;     // face metrics
    double cw, ce, cs, cn;   // metric * hill term of the four side faces
    double h0, h1;           // horizontal diagonal = h0 + g_k h1
    double gz, hc;           // vertical face weight = gz (1 + hc g_face)
};

__device__ __forceinline__ RowC row_consts(const ColW& c)
{
    RowC r;
    r.gx = c.gx;
    r.gys = c.gys;
    r.gyn = c.gyn;
    r.cw = c.gx * c.hw;
    r.ce = c.gx * c.he;
    r.cs = c.gys * c.hs;
    r.cn = c.gyn * c.hn;
    r.h0 = ((c.gx + c.gx) + c.gys) + c.gyn;
    r.h1 = ((c.gx * (c.hw + c.he) + c.gys * c.hs) + c.gyn * c.hn);
    r.gz = c.gz;
    r.hc = c.hc;
    return r;
}

// Vertical face weight of face f (between levels f-1 and f); 0 at the
// bottom (f = 0) and top (f = nz) faces.
__device__ __forceinline__ double vface(const RowC& r, double gf, int f, int nz)
{
    return (f > 0 && f < nz) ? r.gz * fma(r.hc, gf, 1.0) : 0.0;
}

// The same constants in binary32, for the stencil and column solve of the
// mixed form (binary32 vectors): there L(e) is stored in binary32, so
// forming it in binary32 arithmetic changes it by the order of that
// rounding, at half the vector-ALU cost of FP64 (row_consts32 below).
struct RowCf {
    float gx, gys, gyn, cw, ce, cs, cn, h0, h1, gz, hc;
};

template <typename AT>
struct RowOf;
template <>
struct RowOf<double> {
    using type = RowC;
};
template <>
struct RowOf<float> {
    using type = RowCf;
};

// The binary32 row constants straight from the binary32 hill tables (the
// per-row metric factors rounded from FP64), in the same operation order as
// row_consts: the binary32 stencil and column solve read half the table
// bytes, and their diagonals agree with each other as the FP64 ones do.
__device__ __forceinline__ RowCf row_consts32(const Geo& g, int i, int j)
{
    const int iw = (i == 0) ? g.nx - 1 : i - 1;
    const float hw = g.hx32[(long long)j * g.nx + iw];
    const float he = g.hx32[(long long)j * g.nx + i];
    const float hs = g.hy32[(long long)j * g.nx + i];
    const float hn = g.hy32[(long long)(j + 1) * g.nx + i];
    RowCf r;
    r.gx = (float)g.Gx[j];
    r.gys = (float)g.Gy[j];
    r.gyn = (float)g.Gy[j + 1];
    r.cw = r.gx * hw;
    r.ce = r.gx * he;
    r.cs = r.gys * hs;
    r.cn = r.gyn * hn;
    r.h0 = ((r.gx + r.gx) + r.gys) + r.gyn;
    r.h1 = ((r.gx * (hw + he) + r.gys * hs) + r.gyn * hn);
    r.gz = (float)g.Gz[j];
    r.hc = g.hc32[(long long)j * g.nx + i];
    return r;
}

template <typename AT>
__device__ __forceinline__ typename RowOf<AT>::type row_consts_for(const Geo& g, int i, int j)
{
    if constexpr (sizeof(AT) == 4) return row_consts32(g, i, j);
    else return row_consts(col_weights(g, i, j));
}

// Row constants of the column solve on either mesh: the octahedral mesh
// reads its per-point sums (only h0, h1, gz and hc are used by the solve).
template <typename AT>
__device__ __forceinline__ typename RowOf<AT>::type col_consts_for(const Geo& g, int i, int j)
{
    if (g.mesh == FTGCR_MESH_OCTAHEDRAL) {
        typename RowOf<AT>::type r = {};
        if constexpr (sizeof(AT) == 8) {
            r.h0 = g.oh0[i];
            r.h1 = g.oh1[i];
            r.gz = g.ogz[i];
            r.hc = g.ohc[i];
        } else {
            r.h0 = g.oh0_32[i];
            r.h1 = g.oh1_32[i];
            r.gz = g.ogz32[i];
            r.hc = g.ohc32[i];
        }
        return r;
    }
    return row_consts_for<AT>(g, i, j);
}

__device__ __forceinline__ float vface(const RowCf& r, float gf, int f, int nz)
{
    return (f > 0 && f < nz) ? r.gz * fmaf(r.hc, gf, 1.0f) : 0.0f;
}

// Wavefront shifts by one lane (DPP): lane l receives lane l-1's value
// (shift_up) or lane l+1's (shift_down); lanes with no source get 0.  Every
// lane of the wavefront must be active.
__device__ __forceinline__ double lane_shift(double v, int ctrl_up)
{
    const long long b = __double_as_longlong(v);
    int lo, hi;
    if (ctrl_up) {
        lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xF, 0xF, false);        // wave_shr:1
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xF, 0xF, false);
    } else {
        lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xF, 0xF, false);        // wave_shl:1
        hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xF, 0xF, false);
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float lane_shift(float v, int ctrl_up)
{
    const int b = __float_as_int(v);
    const int r = ctrl_up ? __builtin_amdgcn_update_dpp(0, b, 0x138, 0xF, 0xF, false)
                          : __builtin_amdgcn_update_dpp(0, b, 0x130, 0xF, 0xF, false);
    return __int_as_float(r);
}

__device__ __forceinline__ float lane_read(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// (A x) at levels k0 .. k0+KC-1 of column (i, j) (i, j clamped in range,
// k0 < nz), for a whole block: a block is a 64 x 4 tile of columns, one
// wavefront per row (lane = i - tile start), so most neighbours are values
// other lanes already loaded:
//   west / east  the adjacent lanes' centre values, moved by DPP; the row
//                segment's two edge values (one of them the periodic wrap)
//                come from one load instruction, lanes 0..KC-1 west and
//                32..32+KC-1 east, broadcast by readlane;
//   south/north  FP64: the adjacent rows' centre values through LDS, only
//                the tile's first and last rows load a halo row; binary32:
//                each row loads its own south and north rows;
//   below/above  registers (each thread holds its KC levels and one more on
//                either side).
// All loads use clamped in-range addresses and are issued before the first
// is used; missing neighbours (beyond the poles, bottom, top) are selected
// to 0 (a select, not a product, so a NaN at a clamped address cannot leak)
// and carry weight 0.  Entries at levels >= nz or in clamped columns are
// garbage and must be masked by the caller.  `centre`, if given, receives
// x at the KC levels (as loaded).  Every thread of the block must call this
// (the FP64 form holds a barrier).
template <typename TI, int KC>
__device__ __forceinline__ void stencil_chunk(const Geo& g, const TI* __restrict__ x, int i, int j,
                                              int k0, double (&out)[KC], double* centre = nullptr)
{
    static_assert(ST_TX == 64 && ST_TY * ST_TX == ST_THREADS, "one wavefront per tile row");
    static_assert(KC <= 32, "edge lanes");
    using AT = TI;   // arithmetic type: FP64 for FP64 vectors, binary32 for binary32
    __shared__ AT s_row[ST_TY][KC][ST_TX];
    const typename RowOf<AT>::type rc = row_consts_for<AT>(g, i, j);
    const int nz = g.nz, nx = g.nx;
    const long long plane = (long long)g.ncols;
    const int lane = threadIdx.x & (ST_TX - 1);
    const int w = threadIdx.x / ST_TX;
    // tile start (lane 0 is never a clamped column) and the last real lane
    const int i0 = __builtin_amdgcn_readlane(i, 0);
    const int last = (nx - 1 - i0 < ST_TX - 1) ? nx - 1 - i0 : ST_TX - 1;
    const int iw0 = (i0 == 0) ? nx - 1 : i0 - 1;
    const int ie0 = (i0 + last + 1 == nx) ? 0 : i0 + last + 1;
    const bool has_s = j > 0, has_n = j < g.ny - 1;
    const long long row = (long long)j * nx;
    AT xv[KC + 2], xs[KC], xn[KC];
#pragma unroll
    for (int t = 0; t < KC + 2; ++t) {
        int k = k0 - 1 + t;
        k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
        xv[t] = (AT)x[row + i + plane * k];
    }
    AT edge;
    {
        const int t = lane < 32 ? lane : lane - 32;
        int k = k0 + (t < KC ? t : KC - 1);
        k = k > nz - 1 ? nz - 1 : k;
        edge = (AT)x[row + plane * k + (lane < 32 ? iw0 : ie0)];
    }
    if constexpr (sizeof(AT) == 8) {
        // halo rows of the tile (first row: south, last row: north); the
        // inner rows come from the adjacent waves through LDS
        if (w == 0) {
            const long long so = has_s ? -(long long)nx : 0;
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int k = (k0 + kk > nz - 1) ? nz - 1 : k0 + kk;
                xs[kk] = (AT)x[row + so + plane * k + i];
            }
        }
        if (w == ST_TY - 1) {
            const long long no = has_n ? (long long)nx : 0;
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int k = (k0 + kk > nz - 1) ? nz - 1 : k0 + kk;
                xn[kk] = (AT)x[row + no + plane * k + i];
            }
        }
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) s_row[w][kk][lane] = xv[kk + 1];
        __syncthreads();
        if (w > 0) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) xs[kk] = s_row[w - 1][kk][lane];
        }
        if (w < ST_TY - 1) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) xn[kk] = s_row[w + 1][kk][lane];
        }
    } else {
        // binary32: every wave loads its south and north rows itself (the
        // adjacent waves' rows, cache hits); no LDS exchange and no barrier,
        // so no wave waits for the tile's slowest (measured faster in
        // binary32; in FP64 the extra values in flight cost occupancy)
        const long long so = has_s ? -(long long)nx : 0;
        const long long no = has_n ? (long long)nx : 0;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int k = (k0 + kk > nz - 1) ? nz - 1 : k0 + kk;
            xs[kk] = (AT)x[row + so + plane * k + i];
            xn[kk] = (AT)x[row + no + plane * k + i];
        }
    }
    AT xw[KC], xe[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const AT up = lane_shift(xv[kk + 1], 1);
        const AT dn = lane_shift(xv[kk + 1], 0);
        const AT we = lane_read(edge, kk);
        const AT ee = lane_read(edge, 32 + kk);
        xw[kk] = (lane == 0) ? we : up;
        xe[kk] = (lane == last) ? ee : dn;
    }
    // vertical face weights of faces k0 .. k0+KC (level k has faces k, k+1)
    AT wf[KC + 1];
#pragma unroll
    for (int t = 0; t <= KC; ++t) {
        const int f = k0 + t;
        const int fq = f > nz ? nz : f;
        wf[t] = vface(rc, (AT)g.gf[fq], f, nz);
    }
    const AT opsig = (AT)g.opsig;
    const AT zero = AT(0);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        const int kq = (k > nz - 1) ? nz - 1 : k;
        const AT gk = (AT)g.gc[kq];
        const AT wb = wf[kk], wa = wf[kk + 1];
        const AT xsv = has_s ? xs[kk] : zero;
        const AT xnv = has_n ? xn[kk] : zero;
        const AT xb = (k > 0) ? xv[kk] : zero;
        const AT xa = (k + 1 < nz) ? xv[kk + 2] : zero;
        AT t1 = rc.gx * (xw[kk] + xe[kk]);
        t1 = fma(rc.gys, xsv, t1);
        t1 = fma(rc.gyn, xnv, t1);
        AT t2 = rc.cw * xw[kk];
        t2 = fma(rc.ce, xe[kk], t2);
        t2 = fma(rc.cs, xsv, t2);
        t2 = fma(rc.cn, xnv, t2);
        AT off = fma(gk, t2, t1);
        off = fma(wb, xb, off);
        off = fma(wa, xa, off);
        const AT diag = opsig * ((fma(gk, rc.h1, rc.h0) + wb) + wa);
        out[kk] = (double)fma(diag, xv[kk + 1], -off);
        if (centre) centre[kk] = (double)xv[kk + 1];
    }
}

// Depth of the direction-term load pipeline of the direction pass: the
// loads of term l + TERM_PIPE - 1 are issued before term l is used.
// binary32 loads carry half the bytes and the binary32 kernel has registers
// to spare, so it keeps one more term in flight (64.1 vs 65.2 us on
// 512 x 256 x 64; three stages in FP64 would cost occupancy).
template <typename T>
constexpr int TERM_PIPE = sizeof(T) == 4 ? 3 : 2;

// Stencil-grid coordinates of this thread: (i, j) clamped into the grid for
// addressing, `col_ok` whether the thread owns a real column.
struct StPos {
    int i, j, k0;
    bool col_ok;
};

// Block lb of a stencil-grid launch of nct column tiles times tz level
// chunks -> its column tile ct and level chunk bz, in block order `ord`
// (ORD_X: ct fastest; ORD_Z: bz fastest; ORD_XCD: bz fastest after
// renumbering, so that the blocks the hardware places on one die (those
// congruent modulo XCDS) take one contiguous range of the order).  A
// bijection on [0, nct * tz) for every order.
__device__ __forceinline__ void block_tile(int lb, int nct, int tz, int ord, int& ct, int& bz)
{
    if (ord == ORD_X) {
        ct = lb % nct;
        bz = lb / nct;
        return;
    }
    if (ord == ORD_XCD) {
        const int n = nct * tz;
        const int q = n / XCDS, r = n % XCDS, d = lb % XCDS;
        lb = d * q + (d < r ? d : r) + lb / XCDS;
    }
    bz = lb % tz;
    ct = lb / tz;
}

// Lat-lon: a block is a 64 x 4 tile of columns times kc levels.
template <typename T>
__device__ __forceinline__ StPos st_pos(const Inst<T>& in, int lb, int kc, int ord)
{
    StPos p;
    int ct, bz;
    block_tile(lb, in.tx * in.ty, (in.g.nz + kc - 1) / kc, ord, ct, bz);
    const int bx = ct % in.tx;
    const int by = ct / in.tx;
    const int i = bx * ST_TX + (threadIdx.x & (ST_TX - 1));
    const int j = by * ST_TY + (threadIdx.x / ST_TX);
    p.col_ok = i < in.g.nx && j < in.g.ny;
    p.i = i < in.g.nx ? i : in.g.nx - 1;
    p.j = j < in.g.ny ? j : in.g.ny - 1;
    p.k0 = bz * kc;
    return p;
}

// Position on either mesh: lat-lon as above; octahedral (nx = points per
// level, ny = 1): ST_THREADS consecutive points per block, i = the point.
template <int MESH, typename T>
__device__ __forceinline__ StPos st_pos_m(const Inst<T>& in, int lb, int kc, int ord)
{
    if constexpr (MESH == FTGCR_MESH_OCTAHEDRAL) {
        StPos p;
        int bx, bz;
        block_tile(lb, in.tx, (in.g.nz + kc - 1) / kc, ord, bx, bz);
        const int i = bx * ST_THREADS + threadIdx.x;
        p.col_ok = i < in.g.nx;
        p.i = p.col_ok ? i : in.g.nx - 1;
        p.j = 0;
        p.k0 = bz * kc;
        return p;
    } else {
        return st_pos(in, lb, kc, ord);
    }
}

// A table entry of the octahedral mesh in the arithmetic type: the FP64
// table, or its binary32 copy (rounded to nearest) for binary32 arithmetic.
template <typename AT>
__device__ __forceinline__ AT oct_tab(const double* d, const float* f, long long q)
{
    if constexpr (sizeof(AT) == 8) return d[q];
    else return f[q];
}

// (A x) at levels k0 .. k0+KC-1 of point c of the octahedral mesh, in the
// same operation order as a lat-lon row (off-diagonal sums of metric and
// metric-times-hill terms, combined with g_k; diagonal h0 + g_k h1 plus the
// vertical faces, as the column solve forms it), neighbours gathered through
// the slot tables; an empty slot contributes a selected 0, not a product.
// The arithmetic runs in the vector type (binary32 vectors: binary32 tables
// and arithmetic, as on the lat-lon mesh).
template <typename TI, int KC>
__device__ __forceinline__ void stencil_oct(const Geo& g, const TI* __restrict__ x, int c, int k0,
                                            double (&out)[KC], double* centre = nullptr)
{
    using AT = TI;
    const int nz = g.nz;
    const long long plane = (long long)g.ncols;
    const AT h0 = oct_tab<AT>(g.oh0, g.oh0_32, c), h1 = oct_tab<AT>(g.oh1, g.oh1_32, c);
    const AT gz = oct_tab<AT>(g.ogz, g.ogz32, c), hc = oct_tab<AT>(g.ohc, g.ohc32, c);
    AT xv[KC + 2], t1[KC], t2[KC];
#pragma unroll
    for (int t = 0; t < KC + 2; ++t) {
        int k = k0 - 1 + t;
        k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
        xv[t] = x[c + plane * k];
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        t1[kk] = AT(0);
        t2[kk] = AT(0);
    }
#pragma unroll
    for (int q = 0; q < NB_OCT; ++q) {
        const long long slot = (long long)q * g.ncols + c;
        const int nb = g.onb[slot];
        const AT gw = oct_tab<AT>(g.ogw, g.ogw32, slot), hw = oct_tab<AT>(g.ohw, g.ohw32, slot);
        const long long base = nb >= 0 ? nb : c;
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int k = (k0 + kk > nz - 1) ? nz - 1 : k0 + kk;
            const AT v = x[base + plane * k];
            const AT vs = nb >= 0 ? v : AT(0);
            t1[kk] = fma(gw, vs, t1[kk]);
            t2[kk] = fma(hw, vs, t2[kk]);
        }
    }
    AT wf[KC + 1];
#pragma unroll
    for (int t = 0; t <= KC; ++t) {
        const int f = k0 + t;
        const int fq = f > nz ? nz : f;
        wf[t] = (f > 0 && f < nz) ? gz * fma(hc, (AT)g.gf[fq], AT(1)) : AT(0);
    }
    const AT opsig = (AT)g.opsig;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int k = k0 + kk;
        const int kq = (k > nz - 1) ? nz - 1 : k;
        const AT gk = (AT)g.gc[kq];
        const AT wb = wf[kk], wa = wf[kk + 1];
        const AT xb = (k > 0) ? xv[kk] : AT(0);
        const AT xa = (k + 1 < nz) ? xv[kk + 2] : AT(0);
        AT off = fma(gk, t2[kk], t1[kk]);
        off = fma(wb, xb, off);
        off = fma(wa, xa, off);
        const AT diag = opsig * ((fma(gk, h1, h0) + wb) + wa);
        out[kk] = (double)fma(diag, xv[kk + 1], -off);
        if (centre) centre[kk] = (double)xv[kk + 1];
    }
}

// The stencil on either mesh.
template <typename TI, int KC, int MESH>
__device__ __forceinline__ void stencil_m(const Geo& g, const TI* __restrict__ x, const StPos& ps, double (&out)[KC],
                                          double* centre = nullptr)
{
    if constexpr (MESH == FTGCR_MESH_OCTAHEDRAL) {
        stencil_oct<TI, KC>(g, x, ps.i, ps.k0, out, centre);
    } else {
        stencil_chunk<TI, KC>(g, x, ps.i, ps.j, ps.k0, out, centre);
    }
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

// Tolerance and step cap of an inner round of the mixed-precision
// refinement: exit when <r,r> <= tau^2 <r_t, r_t>.
template <typename T>
__global__ void k_set_round(Table<T> tb, double tol2, long long max_steps)
{
    const int m = blockIdx.x;
    if (m >= tb.n || threadIdx.x != 0) return;
    SolveState* st = tb.inst[m].st;
    st->tol2 = tol2;
    st->max_steps = max_steps;
    st->T = tol2 * (st->mixed ? st->rt2 : st->RR);
}

// r = A x - R (x = caller's FP64 iterate), stored in R[r_dst] when `store`;
// partials of <R, R> and of the unrounded FP64 <r, r>.
template <typename T, int KC, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_residual(Table<T> tb, int store)
{
    __shared__ double sh[4];
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    const StPos ps = st_pos_m<MESH>(in, lb, in.kc, in.ord_st);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    T* rout = in.R[in.st->r_dst];
    const double* rhs = in.rhs;
    double ax[KC], b[KC];
    stencil_m<double, KC, MESH>(in.g, in.X[0], ps, ax);
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        b[kk] = rhs[c0 + plane * kq];
    }
    double rr = 0.0, bb = 0.0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        const double r = ok ? ax[kk] - b[kk] : 0.0;
        const double bv = ok ? b[kk] : 0.0;
        if (ok && store) rout[c0 + plane * (ps.k0 + kk)] = (T)r;
        rr = fma(r, r, rr);
        bb = fma(bv, bv, bb);
    }
    const double sb = block_sum(bb, sh);
    const double sr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        in.part[(long long)(0) * in.pstride + lb] = sb;
        in.part[(long long)(1) * in.pstride + lb] = sr;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_finish_residual(Table<T> tb, int set_T)
{
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    double v[2];
    sum_partials<2, 8>(in, in.nblk_st, 0, 2, v);
    const double RR = v[0], rt2 = v[1];
    if (threadIdx.x == 0) {
        st->RR = RR;
        st->rt2 = rt2;
        if (set_T) st->T = st->tol2 * (st->mixed ? rt2 : RR);
    }
}

// ---------------------------------------------------------------------------
// decisions (single thread of the last block)
// ---------------------------------------------------------------------------

// The control state staged in LDS for a reduction block.  Every field read
// by the decision logic would otherwise be a dependent round trip to memory
// (and a read after a store to another field of the same type must go
// back to memory); instead each of the first ST_WORDS threads loads one
// 8-byte word of the state (all fields before the detection log) together
// with the block's other loads, the decision runs on the LDS copy, and the
// words are stored back once.  Barriers separate the word-wise copies from
// the field accesses.
constexpr int ST_WORDS = (int)(offsetof(SolveState, log) / 8);
static_assert(offsetof(SolveState, log) % 8 == 0, "state words");
static_assert(ST_WORDS <= RED_THREADS, "one word per thread");

__device__ __forceinline__ long long state_word_load(const SolveState* g)
{
    const gptr<long long> w = as_global(reinterpret_cast<const long long*>(g));
    return ((int)threadIdx.x < ST_WORDS) ? w[threadIdx.x] : 0;
}

__device__ __forceinline__ void state_word_stage(SolveState* s, long long w)
{
    if ((int)threadIdx.x < ST_WORDS) reinterpret_cast<long long*>(s)[threadIdx.x] = w;
}

__device__ __forceinline__ void state_word_store(SolveState* g, const SolveState* s)
{
    if ((int)threadIdx.x < ST_WORDS)
        as_global_mut(reinterpret_cast<long long*>(g))[threadIdx.x] = reinterpret_cast<const long long*>(s)[threadIdx.x];
}

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

// After the initial residual and P^{-1} r^0: <r^0, r^0>, the exit test, and
// the initial known-good state.
__device__ void decide_init(SolveState* st, double rn, double rs)
{
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

// One step's decision: exit test first, then the monotone residual-norm
// fault test with rollback to the backup, else (first pass of a cycle) the
// new backup.  rn: <r+, r+> of the unrounded update (detector), rs: of the
// stored r+ (exit test and next reference); equal in FP64.
// `log` is the state's detection log (st itself may be a staged copy
// without one).
__device__ void decide_step(SolveState* st, DetectRec* log, double rn, double rs, double* hist,
                            long long hist_cap)
{
    const int nu = st->nu;
    st->s += 1;
    st->e_ok = 0;
    const long long s = st->s;
    if (st->d_cur == 0.0) {   // <L p, L p> = 0: beta undefined
        st->status = FTGCR_BREAKDOWN;
        st->x_final_hi = nu - 1;
        st->active = 0;
        return;
    }
    if (nu == 0) st->cycles += 1;
    if (s <= hist_cap) hist[s - 1] = rn;
    st->beta[nu] = -st->beta_num / st->d_cur;
    st->rr_new = rn;
    if (rs <= st->T) {
        st->accepted += 1;
        st->rr_old = rs;
        st->r_cur = st->r_dst;
        st->status = FTGCR_CONVERGED;
        st->x_final_hi = nu;
        st->active = 0;
        return;
    }
    if (st->ft && !(rn < st->rr_old)) {   // the norm did not decrease (NaN included)
        const long long pos = st->accepted + 1;
        const int stag = (pos == st->last_rb_pos) && !st->events_since_rb;
        st->detections += 1;
        if (st->log_len < LOG_CAP) {
            DetectRec& rec = log[st->log_len++];
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
    st->e_ok = 1;
    if (s >= st->max_steps) {
        st->status = FTGCR_MAX_STEPS;
        st->x_final_hi = nu;
        st->active = 0;
    }
}

// After the new direction: the next beta's inner products, then pass and
// cycle bookkeeping (p^k opens the next cycle).
__device__ void decide_beta(SolveState* st, double num, double dn, int init)
{
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
    if (nu + 1 == st->k) {
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

// ---------------------------------------------------------------------------
// update + column preconditioner (+ the step's decision)
// ---------------------------------------------------------------------------
//
// Each column (i, j) is split between two lanes of a wave (lane l and l+32):
// the lower lane eliminates levels 0 .. h-1 upward (Thomas forward sweep),
// the upper lane levels nz-1 .. h downward; they meet at row h-1, exchange
// one pivot pair by a lane shuffle, and each back-substitutes its half.  The
// elimination state of a half column (at most H levels) stays in registers.
// P's rows: a_k e_{k-1} + b_k e_k + u_k e_{k+1} = r_k with b the diagonal of
// A and a, u minus the vertical face weights.  All loads of a half column are
// issued before its first store (r is updated in place after the first pass
// of a cycle, so program order must not interleave them).

// MODE_GM (FT-GMRES, FP64): the current Arnoldi vector U[j] is divided by
// den[j] (normalised, written back in place) and z_j = P^{-1} v_j goes to
// Z[j]; no norms.
template <typename T, int H, int mode, bool FULL>
__device__ __forceinline__ void update_thomas_body(Table<T> tb, const T* dbg_in, T* dbg_out, const GmInst* gm)
{
    // The column solve runs in the storage precision: FP64 for FP64 solves;
    // binary32 for the mixed form, where e = P^{-1} r only has to be a fixed
    // preconditioner application (L(e) is formed from the stored e).  The
    // update r+ = r + beta L(p) and both norms stay FP64.
    using CT = T;
    __shared__ double sh[4];
    __shared__ CT s_gc[2 * H];
    __shared__ CT s_gf[2 * H + 1];
    // Half columns longer than 32 levels: the multipliers of the first LH
    // rows (the last ones the back-substitution reads) wait in LDS, the rest
    // in registers, so that the kernel fits two waves per SIMD (all 48
    // levels in registers take about 370 registers in FP64: one wave)
    constexpr int LH = H > 32 ? (sizeof(CT) == 8 ? 19 : 16) : 0;
    constexpr int RH = H - LH;
    __shared__ CT s_stk[LH > 0 ? LH : 1][2][COL_THREADS];
    const int m = find_inst(tb.blk0_col, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_col[m];
    SolveState* st = in.st;
    if (mode == MODE_STEP || mode == MODE_INIT) {
        if (st->status != RUNNING) return;
        if (mode == MODE_STEP && st->d_cur == 0.0) return;   // the decision records the breakdown
    }
    if (mode == MODE_GM) {
        if (gm->st->status != RUNNING || !gm->st->active) return;
    }
    // everything read from the instance and the state is copied to registers
    // before the first store, so no later access can wait behind a store
    const Geo& g = in.g;
    const int nx = g.nx, nz = g.nz, ncols = g.ncols;
    const double opsig = g.opsig;
    // vertical decay tables in LDS (LDS reads do not queue behind stores)
    for (int t = threadIdx.x; t < nz; t += blockDim.x) s_gc[t] = (CT)g.gc[t];
    for (int t = threadIdx.x; t <= nz; t += blockDim.x) s_gf[t] = (CT)g.gf[t];
    const CT opsig_c = (CT)opsig;
    const T* rin;
    const T* ap;
    T* rout;
    T* eout;
    double beta = 0.0;
    double den = 1.0;
    if (mode == MODE_DEBUG) {
        rin = dbg_in;
        ap = dbg_in;
        rout = nullptr;
        eout = dbg_out;
    } else if (mode == MODE_GM) {
        const int jj = gm->st->j;
        rin = (const T*)gm->U[jj];
        ap = rin;
        rout = (T*)gm->U[jj];
        eout = (T*)gm->Z[jj];
        den = gm->st->den[jj];
    } else {
        rin = in.R[st->r_cur];
        eout = in.E;
        ap = rin;
        rout = nullptr;
        if (mode == MODE_STEP) {
            ap = in.AP[st->slot[st->nu]];
            rout = in.R[st->r_dst];
            beta = -st->beta_num / st->d_cur;
        }
    }
    double* part = in.part;
    const long long pstride = in.pstride;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const bool upper = lane >= 32;
    const int col = lb * COLS_PER_BLOCK + (threadIdx.x >> 6) * 32 + (lane & 31);
    const bool valid = col < ncols;
    const int colc = valid ? col : 0;
    const int j = colc / nx;
    const int i = colc - j * nx;
    const long long plane = (long long)ncols;
    const int h = (nz + 1) >> 1;   // lower half: levels [0, h)
    const int nup = nz - h;        // upper half: levels [h, nz)
    const int nmine = upper ? nup : h;
    // diagonal h0 + g_k h1 + vertical faces, from the same per-column
    // constants and in the same order as the stencil rows (identical)
    const typename RowOf<CT>::type rcst = col_consts_for<CT>(g, i, j);
    const CT h0 = rcst.h0;
    const CT h1 = rcst.h1;
    const CT gz = rcst.gz, hc = rcst.hc;

    // The half column streams in chunks of CH levels, each chunk's loads
    // issued one chunk ahead of its elimination (a two-stage software
    // pipeline): loads are branch-free (clamped addresses, results
    // selected), so a chunk's loads are all in flight together, and they are
    // issued before the previous chunk's stores, so waiting for them never
    // waits for a store.  The elimination is the same instruction stream
    // for both halves: the lower lane eliminates towards level 0 (near
    // coupling a_k, far coupling u_k), the upper lane towards nz-1 (near
    // u_k, far a_k).
    // r is loaded with the non-temporal hint: this is its last use in the
    // step (the direction pass reads r+), and the hint leaves the Infinity
    // Cache to what the next passes re-read (e, r+, the L(p^l)).
    // FP64 streams in 4-level chunks: with 8 the half column's registers
    // exceed 256 and the kernel drops to one wave per SIMD.  binary32 values
    // are half the bytes per load, so it streams 16 levels ahead where the
    // half column allows (more bytes in flight per wave)
    constexpr int CHW = sizeof(T) == 8 ? 4 : (H % 16 == 0 ? 16 : (H % 8 == 0 ? 8 : 4));
    constexpr int CH = H < CHW ? H : CHW;
    constexpr int NCH = H / CH;
    static_assert(H % CH == 0, "chunks must tile the half column");
    T bufr[2][CH], bufa[2][CH];
    CT de[RH], ga[RH];
    double acc_new = 0.0, acc_st = 0.0;
    CT carry_g = 0, carry_d = 0;
    CT mm = 1, ff = 0, uu = 0;   // meeting row of the lower lane
    CT w_near = 0;                // face below level 0 / above level nz-1
    // r+ is stored through a pointer that walks one level per row (a fresh
    // induction value, so the loads' 64-bit addresses need not stay live)
    const long long wstep = upper ? -plane : plane;
    gptr_mut<T> rw = as_global_mut((mode == MODE_STEP || mode == MODE_GM) ? rout : eout) + (long long)colc +
                     plane * (upper ? nz - 1 : 0);
    asm volatile("" : "+v"(rw));
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        int k = upper ? nz - 1 - t : t;
        k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
        const long long o = (long long)colc + plane * k;
        bufr[0][t] = __builtin_nontemporal_load(&rin[o]);
        bufa[0][t] = (mode == MODE_STEP) ? ap[o] : T(0);
    }
#pragma unroll
    for (int cb = 0; cb < NCH; ++cb) {
        const int b = cb & 1;
        // keep the pipeline depth at one chunk: without this fence the
        // scheduler hoists every chunk's loads and the half column's raw
        // values all sit in registers at once (occupancy 1)
        __builtin_amdgcn_sched_barrier(0);
        if (cb + 1 < NCH) {
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                const int q = (cb + 1) * CH + t;
                int k = upper ? nz - 1 - q : q;
                k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
                const long long o = (long long)colc + plane * k;
                bufr[b ^ 1][t] = __builtin_nontemporal_load(&rin[o]);
                bufa[b ^ 1][t] = (mode == MODE_STEP) ? ap[o] : T(0);
            }
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const int q = cb * CH + t;
            const bool mine = q < nmine;
            int k = upper ? nz - 1 - q : q;
            k = k < 0 ? 0 : (k > nz - 1 ? nz - 1 : k);
            const double v = (mode == MODE_STEP) ? fma(beta, (double)bufa[b][t], (double)bufr[b][t])
                             : (mode == MODE_GM) ? (double)bufr[b][t] / den
                                                 : (double)bufr[b][t];
            const T sv = (T)v;
            const double rp = (double)sv;
            const CT rc = (CT)sv;
            // When the columns fill the grid exactly (FULL), every lane owns
            // every row it touches and stores r+ unguarded: behind a guard
            // the compiler moves all rows' eliminations after all the
            // stores, holding every row's values at once
            if constexpr (FULL) {
                if (mode == MODE_STEP || mode == MODE_GM) *rw = sv;
                acc_new = fma(v, v, acc_new);
                acc_st = fma(rp, rp, acc_st);
            } else if (mine && valid) {
                if (mode == MODE_STEP || mode == MODE_GM) *rw = sv;
                acc_new = fma(v, v, acc_new);
                acc_st = fma(rp, rp, acc_st);
            }
            rw += wstep;
            // vertical face weights of row k: the face shared with the
            // previous row of this lane was computed there (w_near); the far
            // face (k + 1 for the lower lane, k for the upper one) is new
            const int f = upper ? k : k + 1;
            const CT gff = s_gf[f];
            const CT w_far = (f > 0 && f < nz) ? gz * fma(hc, gff, CT(1)) : CT(0);
            const CT wb = upper ? w_far : w_near;
            const CT wa = upper ? w_near : w_far;
            w_near = w_far;
            const CT diag = opsig_c * ((fma(s_gc[k], h1, h0) + wb) + wa);
            const CT near = upper ? -wa : -wb;
            const CT far = upper ? -wb : -wa;
            const CT mk = (q == 0) ? diag : diag - near * carry_g;
            const CT fk = (q == 0) ? rc : rc - near * carry_d;
            const bool meet = !upper && q == h - 1;
            if (meet) {
                mm = mk;
                ff = fk;
                uu = far;
            }
            // binary32 column solve: the hardware reciprocal (about 1 ulp;
            // the preconditioner only has to be a fixed operator); FP64:
            // the correctly rounded quotient
            CT inv;
            if constexpr (sizeof(CT) == 4) inv = __builtin_amdgcn_rcpf(mk);
            else inv = CT(1) / mk;
            const CT g_new = far * inv;
            const CT d_new = fk * inv;
            if (mine) {
                carry_g = meet ? carry_g : g_new;
                carry_d = meet ? carry_d : d_new;
            }
            if (q < LH) {
                s_stk[q < LH ? q : 0][0][threadIdx.x] = g_new;
                s_stk[q < LH ? q : 0][1][threadIdx.x] = d_new;
            } else {
                ga[q - LH] = g_new;
                de[q - LH] = d_new;
            }
        }
    }
    // meeting row: the lower lane gets (zeta_h, eps_h) from its upper partner
    const CT zx = __shfl_xor(carry_g, 32);
    const CT ex = __shfl_xor(carry_d, 32);
    const CT xm = (ff - uu * ex) / (mm - uu * zx);
    const CT xl = __shfl_xor(xm, 32);
    // back-substitution: lower lane from level h-2 down to 0 (after storing
    // the meeting value at h-1), upper lane from level h up to nz-1
    CT xv = upper ? xl : xm;
    if (valid && !upper) eout[(long long)colc + plane * (h - 1)] = (T)xm;
    const int nback = upper ? nup : h - 1;
    // the store address walks one level per row from a fresh base: were it
    // recomputed from the forward sweep's expressions, the compiler would
    // keep all of the half column's 64-bit addresses live across the sweep
    const long long estep = upper ? plane : -plane;
    gptr_mut<T> ep = as_global_mut(eout) + (long long)colc + plane * (upper ? h : h - 2);
    asm volatile("" : "+v"(ep));
#pragma unroll
    for (int q = H - 1; q >= 0; --q) {
        if (q < nback) {
            CT gq, dq;
            if (q < LH) {
                gq = s_stk[q < LH ? q : 0][0][threadIdx.x];
                dq = s_stk[q < LH ? q : 0][1][threadIdx.x];
            } else {
                gq = ga[q - LH];
                dq = de[q - LH];
            }
            xv = dq - gq * xv;
            if (valid) *ep = (T)xv;
            ep += estep;
        }
    }
    if (mode == MODE_DEBUG || mode == MODE_GM) return;
    const double sn = block_sum(acc_new, sh);
    const double ss = block_sum(acc_st, sh);
    if (threadIdx.x == 0) {
        part[(long long)(0) * pstride + lb] = sn;
        part[(long long)(1) * pstride + lb] = ss;
    }
}

template <typename T, int H, int mode>
__global__ __launch_bounds__(COL_THREADS) void k_update_thomas(Table<T> tb, const T* dbg_in, T* dbg_out)
{
    update_thomas_body<T, H, mode, false>(tb, dbg_in, dbg_out, nullptr);
}

// The step pass on columns that fill the grid exactly, held to two waves
// per SIMD (its unguarded stores keep the long columns within 256 registers)
template <typename T, int H>
__global__ __launch_bounds__(COL_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_update_thomas_full(
    Table<T> tb)
{
    update_thomas_body<T, H, MODE_STEP, true>(tb, nullptr, nullptr, nullptr);
}

template <int H>
__global__ __launch_bounds__(COL_THREADS) void k_update_thomas_gm(Table<double> tb, const GmInst* gm)
{
    update_thomas_body<double, H, MODE_GM, false>(tb, nullptr, nullptr, gm);
}

template <int H>
__global__ __launch_bounds__(COL_THREADS) __attribute__((amdgpu_waves_per_eu(2))) void k_update_thomas_gm_full(
    Table<double> tb, const GmInst* gm)
{
    update_thomas_body<double, H, MODE_GM, true>(tb, nullptr, nullptr, gm);
}

// The binary32 column pass with one lane per column (256 columns per
// block), for columns of at most NZ = 64 levels.  The two-lane kernel above
// needs more registers per lane in binary32 than fit four waves per SIMD, so
// its 4096 waves on 512 x 256 columns take 1.33 rounds of the chip at three
// per SIMD; with one lane per column there are half as many waves, which fit
// in one round at two per SIMD, and every load is a full 256-byte wave
// segment.  Same update, norms, faces, diagonal and elimination as above
// (the lower lane's order, extended to the whole column), so P is the same
// fixed operator up to rounding.
template <typename T, int NZ, int mode>
__global__ __launch_bounds__(COL_THREADS) void k_update_thomas1(Table<T> tb)
{
    static_assert(sizeof(T) == 4 && NZ % 8 == 0, "binary32, whole chunks");
    using CT = T;
    __shared__ double sh[4];
    __shared__ CT s_gc[NZ];
    __shared__ CT s_gf[NZ + 1];
    const int m = find_inst(tb.blk0_col, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_col[m];
    SolveState* st = in.st;
    if (st->status != RUNNING) return;
    if (mode == MODE_STEP && st->d_cur == 0.0) return;   // the decision records the breakdown
    const Geo& g = in.g;
    const int nx = g.nx, nz = g.nz, ncols = g.ncols;
    for (int t = threadIdx.x; t < nz; t += blockDim.x) s_gc[t] = (CT)g.gc[t];
    for (int t = threadIdx.x; t <= nz; t += blockDim.x) s_gf[t] = (CT)g.gf[t];
    const CT opsig_c = (CT)g.opsig;
    const T* rin = in.R[st->r_cur];
    const T* ap = rin;
    T* rout = nullptr;
    double beta = 0.0;
    if (mode == MODE_STEP) {
        ap = in.AP[st->slot[st->nu]];
        rout = in.R[st->r_dst];
        beta = -st->beta_num / st->d_cur;
    }
    T* eout = in.E;
    double* part = in.part;
    const long long pstride = in.pstride;
    __syncthreads();

    const int col = lb * COL_THREADS + threadIdx.x;
    const bool valid = col < ncols;
    const int colc = valid ? col : 0;
    const int j = colc / nx;
    const int i = colc - j * nx;
    const long long plane = (long long)ncols;
    const RowCf rcst = col_consts_for<float>(g, i, j);
    const CT h0 = rcst.h0;
    const CT h1 = rcst.h1;
    const CT gz = rcst.gz, hc = rcst.hc;

    // levels stream in 8-level chunks, each chunk's loads issued one chunk
    // ahead (as in the two-lane kernel); r is read with the non-temporal
    // hint (its last use in the step)
    constexpr int CH = 8;
    constexpr int NCH = NZ / CH;
    T bufr[2][CH], bufa[2][CH];
    CT de[NZ], ga[NZ];
    double acc_new = 0.0, acc_st = 0.0;
    CT carry_g = 0, carry_d = 0;
    CT w_near = 0;   // face below level 0
    gptr_mut<T> rw = as_global_mut(mode == MODE_STEP ? rout : eout) + (long long)colc;
    asm volatile("" : "+v"(rw));
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const int k = t > nz - 1 ? nz - 1 : t;
        const long long o = (long long)colc + plane * k;
        bufr[0][t] = __builtin_nontemporal_load(&rin[o]);
        bufa[0][t] = (mode == MODE_STEP) ? ap[o] : T(0);
    }
#pragma unroll
    for (int cb = 0; cb < NCH; ++cb) {
        const int b = cb & 1;
        __builtin_amdgcn_sched_barrier(0);
        if (cb + 1 < NCH) {
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                int k = (cb + 1) * CH + t;
                k = k > nz - 1 ? nz - 1 : k;
                const long long o = (long long)colc + plane * k;
                bufr[b ^ 1][t] = __builtin_nontemporal_load(&rin[o]);
                bufa[b ^ 1][t] = (mode == MODE_STEP) ? ap[o] : T(0);
            }
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            const int q = cb * CH + t;   // level
            const bool mine = q < nz;
            const int k = q > nz - 1 ? nz - 1 : q;
            const double v = (mode == MODE_STEP) ? fma(beta, (double)bufa[b][t], (double)bufr[b][t])
                                                 : (double)bufr[b][t];
            const T sv = (T)v;
            const double rp = (double)sv;
            const CT rc = (CT)sv;
            if (mine && valid) {
                if (mode == MODE_STEP) *rw = sv;
                acc_new = fma(v, v, acc_new);
                acc_st = fma(rp, rp, acc_st);
            }
            rw += plane;
            const int f = k + 1;
            const CT gff = s_gf[f];
            const CT w_far = (f > 0 && f < nz) ? gz * fma(hc, gff, CT(1)) : CT(0);
            const CT wb = w_near, wa = w_far;
            w_near = w_far;
            const CT diag = opsig_c * ((fma(s_gc[k], h1, h0) + wb) + wa);
            const CT near = -wb;
            const CT far = -wa;
            const CT mk = (q == 0) ? diag : diag - near * carry_g;
            const CT fk = (q == 0) ? rc : rc - near * carry_d;
            const CT inv = __builtin_amdgcn_rcpf(mk);
            const CT g_new = far * inv;
            const CT d_new = fk * inv;
            if (mine) {
                carry_g = g_new;
                carry_d = d_new;
            }
            ga[q] = g_new;
            de[q] = d_new;
        }
    }
    // back-substitution from the top level down
    CT xv = carry_d;
    gptr_mut<T> ep = as_global_mut(eout) + (long long)colc + plane * (nz - 1);
    asm volatile("" : "+v"(ep));
    if (valid) *ep = (T)xv;
    ep -= plane;
#pragma unroll
    for (int q = NZ - 2; q >= 0; --q) {
        if (q < nz - 1) {
            xv = de[q] - ga[q] * xv;
            if (valid) *ep = (T)xv;
            ep -= plane;
        }
    }
    const double sn = block_sum(acc_new, sh);
    const double ss = block_sum(acc_st, sh);
    if (threadIdx.x == 0) {
        part[(long long)(0) * pstride + lb] = sn;
        part[(long long)(1) * pstride + lb] = ss;
    }
}

// No preconditioner (P = I): the column pass's update, stored r+ and norms,
// with e = r+ (MODE_GM: v_j normalised and z_j = v_j; MODE_DEBUG: out = in).
// It runs on the column grid (cpb columns per block, all their levels), so
// the decision kernels read the same partial rows.
template <typename T, int mode>
__global__ __launch_bounds__(COL_THREADS) void k_update_copy(Table<T> tb, const T* dbg_in, T* dbg_out,
                                                             const GmInst* gm, int cpb)
{
    __shared__ double sh[4];
    const int m = find_inst(tb.blk0_col, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_col[m];
    SolveState* st = in.st;
    if (mode == MODE_STEP || mode == MODE_INIT) {
        if (st->status != RUNNING) return;
        if (mode == MODE_STEP && st->d_cur == 0.0) return;   // the decision records the breakdown
    }
    if (mode == MODE_GM) {
        if (gm->st->status != RUNNING || !gm->st->active) return;
    }
    const T* rin;
    const T* ap = nullptr;
    T* rout = nullptr;
    T* eout;
    double beta = 0.0, den = 1.0;
    if (mode == MODE_DEBUG) {
        rin = dbg_in;
        eout = dbg_out;
    } else if (mode == MODE_GM) {
        const int jj = gm->st->j;
        rin = (const T*)gm->U[jj];
        rout = (T*)gm->U[jj];
        eout = (T*)gm->Z[jj];
        den = gm->st->den[jj];
    } else {
        rin = in.R[st->r_cur];
        eout = in.E;
        if (mode == MODE_STEP) {
            ap = in.AP[st->slot[st->nu]];
            rout = in.R[st->r_dst];
            beta = -st->beta_num / st->d_cur;
        }
    }
    const int ncols = in.g.ncols, nz = in.g.nz;
    const long long plane = (long long)ncols;
    const int c0 = lb * cpb;
    const int cols = ncols - c0 < cpb ? ncols - c0 : cpb;
    double acc_new = 0.0, acc_st = 0.0;
    for (int t = threadIdx.x; t < cpb * nz; t += COL_THREADS) {
        const int q = t % cpb, k = t / cpb;
        if (q >= cols) continue;
        const long long o = (long long)(c0 + q) + plane * k;
        const double v = (mode == MODE_STEP) ? fma(beta, (double)ap[o], (double)rin[o])
                         : (mode == MODE_GM) ? (double)rin[o] / den
                                             : (double)rin[o];
        const T sv = (T)v;
        const double rp = (double)sv;
        if (mode == MODE_STEP || mode == MODE_GM) rout[o] = sv;
        eout[o] = sv;
        acc_new = fma(v, v, acc_new);
        acc_st = fma(rp, rp, acc_st);
    }
    if (mode == MODE_DEBUG || mode == MODE_GM) return;
    const double sn = block_sum(acc_new, sh);
    const double ss = block_sum(acc_st, sh);
    if (threadIdx.x == 0) {
        in.part[(long long)(0) * in.pstride + lb] = sn;
        in.part[(long long)(1) * in.pstride + lb] = ss;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_finish_col(Table<T> tb, int mode)
{
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    if (st->status != RUNNING) return;
    double v[2];
    sum_partials<2, 8>(in, in.nblk_col, 0, 2, v);
    const double rn = v[0], rs = v[1];
    if (threadIdx.x == 0) {
        if (mode == MODE_STEP) decide_step(st, st->log, rn, rs, in.hist, in.hist_cap);
        else decide_init(st, rn, rs);
    }
}

// ---------------------------------------------------------------------------
// L(e) and orthogonalisation inner products (+ alpha)
// ---------------------------------------------------------------------------

// spec = 1: launched before the step's decision (k_finish_step takes it
// afterwards); it runs whenever the column pass ran, and its partials are
// discarded if the step is rejected or ends the solve.  Nothing it reads
// (nu, the slots, e, the L(p^l)) is changed by the decision.
template <typename T, int KC, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_stencil_dots(Table<T> tb, int spec)
{
    __shared__ double sh[KMAX + 1][4];
    __shared__ const T* s_ap[KMAX + 1];
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    SolveState* st = in.st;
    if (st->status != RUNNING || (spec ? st->d_cur == 0.0 : !st->active)) return;
    const int nu = st->nu;
    if ((int)threadIdx.x <= nu) s_ap[threadIdx.x] = in.AP[st->slot[threadIdx.x]];
    __syncthreads();
    const StPos ps = st_pos_m<MESH>(in, lb, in.kc, in.ord_st);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    double le[KC];
    stencil_m<T, KC, MESH>(in.g, in.E, ps, le);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        // octahedral mesh: L(e) kept for the direction pass (exact in T: the
        // stencil rounds to T's precision, so the direction pass starts from
        // the same value as if it had formed L(e) itself)
        if constexpr (MESH == FTGCR_MESH_OCTAHEDRAL)
            if (ok) in.LE[c0 + plane * (ps.k0 + kk)] = (T)le[kk];
        if (!ok) le[kk] = 0.0;
    }
    // every <L(e), L(p^l)>, one uniform branch per l; the loads of term
    // l + 1 are issued before term l's values are used (a two-stage
    // pipeline), so the terms cost one memory round trip together, not one
    // each
    // (two buffers alternating with the parity of l, which is a compile-time
    // constant after unrolling: no register copies, so the wait for term l
    // comes after term l + 1's loads are issued)
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // PD - 1 terms in flight ahead of the one in use (a deeper pipeline
    // costs this pass occupancy without a gain, measured in both forms)
    constexpr int PD = 2;
    T buf[PD][KC];
#pragma unroll
    for (int l0 = 0; l0 < PD - 1; ++l0) {
        if (l0 == 0 || l0 <= nu) {   // nu >= 0 here
            const gptr<T> apn = as_global(s_ap[l0]);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                buf[l0][kk] = apn[c0 + plane * kq];
            }
        }
    }
#pragma unroll
    for (int l = 0; l <= KMAX; ++l) {
        if (l <= nu) {
            double acc = 0.0;
            const int ln = l + PD - 1;
            if (ln <= KMAX && ln <= nu) {
                const gptr<T> apn = as_global(s_ap[ln]);
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                    buf[ln % PD][kk] = apn[c0 + plane * kq];
                }
            }
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const bool ok = ps.col_ok && ps.k0 + kk < nz;
                acc = fma(le[kk], ok ? (double)buf[l % PD][kk] : 0.0, acc);
            }
            // this term's wave sum now, while the next term's loads are in
            // flight (binary32 dots 27.4 -> 26.6 us on 512 x 256 x 64)
            const double v = wave_sum(acc);
            if (lane == 0) sh[l][w] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= nu) {
        const int l = threadIdx.x;
        in.part[(long long)(DOT_ROW0 + l) * in.pstride + lb] = ((sh[l][0] + sh[l][1]) + sh[l][2]) + sh[l][3];
    }
}

// alpha_l = -<L(e), L(p^l)> / <L(p^l), L(p^l)> and the iterate buffer the
// direction pass writes; every thread of the block calls it.
template <typename T>
__device__ __forceinline__ void finish_alpha_body(const Inst<T>& in, SolveState* st)
{
    const int nu = st->nu;
    const double* v = sum_partials<4, 4>(in, in.nblk_st, DOT_ROW0, nu + 1, nullptr);
    if ((int)threadIdx.x <= nu) st->alpha[threadIdx.x] = -v[threadIdx.x] / st->d[threadIdx.x];
    if (threadIdx.x == 0) st->x_dst = (st->x_base == st->x_bak) ? 1 - st->x_base : st->x_base;
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_finish_alpha(Table<T> tb)
{
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    finish_alpha_body(in, st);
}

// The step's decision (k_finish_col) and, if the step goes on, its alpha
// (k_finish_alpha) in one launch, after a speculative dots pass.
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_finish_step(Table<T> tb)
{
    __shared__ SolveState s_st;
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* gst = in.st;
    // the state's words and the column pass's partials in one round trip
    // (the partials of a solve that is no longer running are read and
    // ignored)
    const long long word = state_word_load(gst);
    double v[2];
    sum_partials<2, 8>(in, in.nblk_col, 0, 2, v);
    state_word_stage(&s_st, word);
    __syncthreads();
    SolveState* st = &s_st;
    if (st->status != RUNNING) return;
    if (threadIdx.x == 0) decide_step(st, gst->log, v[0], v[1], in.hist, in.hist_cap);
    __syncthreads();
    if (st->status == RUNNING && st->active) finish_alpha_body(in, st);
    __syncthreads();
    state_word_store(gst, st);
}

// ---------------------------------------------------------------------------
// new direction, its image, next beta's inner products, deferred iterate
// ---------------------------------------------------------------------------

// Cache hints: the p^l, the iterate and the new p^{nu+1} are next touched
// a whole step later (more than the Infinity Cache holds in between), so
// they are loaded and stored with the non-temporal hint, leaving the cache
// to e, r+ and L(p^{nu+1}), which the next passes read within the step.
// NTAP extends the hint to the L(p^l) loads: set when the solve's k + 1
// images of A p do not fit the cache anyway (otherwise the next dots pass
// finds them there).
template <typename T, int KC, bool NTAP, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_dir_update(Table<T> tb, int init)
{
    __shared__ double sh[4];
    __shared__ const T* s_p[KMAX + 1];
    __shared__ const T* s_ap[KMAX + 1];
    __shared__ double s_al[KMAX + 1];
    __shared__ double s_be[KMAX + 1];
    const int m = find_inst(tb.blk0_dir, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_dir[m];
    SolveState* st = in.st;
    if (st->status != RUNNING) return;
    if (!init && !st->active) return;
    const int nu = init ? -1 : st->nu;
    const int target = st->slot[nu + 1];
    const bool xupd = !init && (nu == st->k - 1);
    const int xlo = st->x_base_nu;
    T* pout = in.P[target];
    T* apout = in.AP[target];
    const T* rv = in.R[st->r_cur];
    const double* xb = in.X[st->x_base];
    double* xo = in.X[st->x_dst];
    if ((int)threadIdx.x <= nu) {
        const int sl = st->slot[threadIdx.x];
        s_p[threadIdx.x] = in.P[sl];
        s_ap[threadIdx.x] = in.AP[sl];
        s_al[threadIdx.x] = st->alpha[threadIdx.x];
        s_be[threadIdx.x] = (xupd && (int)threadIdx.x >= xlo) ? st->beta[threadIdx.x] : 0.0;
    }
    __syncthreads();
    const StPos ps = st_pos_m<MESH>(in, lb, in.kc_dir, in.ord_dir);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    double a[KC], p[KC], xa[KC], r[KC];
    // p starts from e: the stencil's own centre values (no second load).
    // On the octahedral mesh the step's dots pass has stored L(e): e and
    // L(e) are loaded instead of gathering six neighbours again (the first
    // direction of a solve or round, with no dots pass before it, forms it)
    bool formed = false;
    if constexpr (MESH == FTGCR_MESH_OCTAHEDRAL) {
        if (!init) {
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                const long long c = c0 + plane * kq;
                p[kk] = (double)in.E[c];
                a[kk] = (double)in.LE[c];
            }
            formed = true;
        }
    }
    if (!formed) stencil_m<T, KC, MESH>(in.g, in.E, ps, a, p);
    // r is needed only for the next beta's products at the end: binary32
    // loads it there (the registers it frees give that kernel a sixth wave
    // per SIMD); FP64 loads it with the iterate (there a late load is
    // slower, the occupancy being the same)
    constexpr bool R_LATE = sizeof(T) == 4;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        const long long c = c0 + plane * kq;
        if constexpr (!R_LATE) r[kk] = (double)rv[c];
        xa[kk] = xupd ? __builtin_nontemporal_load(&xb[c]) : 0.0;
    }
    // sums over l in ascending order; term l + 1's loads are issued before
    // term l's values are used (two-stage pipeline, as in the dots pass)
    constexpr int PD = TERM_PIPE<T>;
    T pb[PD][KC], ab[PD][KC];
#pragma unroll
    for (int l0 = 0; l0 < PD - 1; ++l0) {
        if (l0 <= nu) {
            const gptr<T> pn = as_global(s_p[l0]);
            const gptr<T> apn = as_global(s_ap[l0]);
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                pb[l0][kk] = __builtin_nontemporal_load(&pn[c0 + plane * kq]);
                ab[l0][kk] = NTAP ? __builtin_nontemporal_load(&apn[c0 + plane * kq]) : apn[c0 + plane * kq];
            }
        }
    }
#pragma unroll
    for (int l = 0; l < KMAX; ++l) {
        if (l <= nu) {
            const double al = s_al[l];
            const double bl = s_be[l];
            const int ln = l + PD - 1;
            if (ln < KMAX && ln <= nu) {
                const gptr<T> pn = as_global(s_p[ln]);
                const gptr<T> apn = as_global(s_ap[ln]);
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                    pb[ln % PD][kk] = __builtin_nontemporal_load(&pn[c0 + plane * kq]);
                    ab[ln % PD][kk] = NTAP ? __builtin_nontemporal_load(&apn[c0 + plane * kq])
                                           : apn[c0 + plane * kq];
                }
            }
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                p[kk] = fma(al, (double)pb[l % PD][kk], p[kk]);
                a[kk] = fma(al, (double)ab[l % PD][kk], a[kk]);
                if (xupd) xa[kk] = fma(bl, (double)pb[l % PD][kk], xa[kk]);
            }
        }
    }
    if constexpr (R_LATE) {
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) {
            const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
            r[kk] = (double)rv[c0 + plane * kq];
        }
    }
    double acc_num = 0.0, acc_d = 0.0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        const T ps_ = (T)p[kk];
        const T as_ = (T)a[kk];
        if (ok) {
            const long long c = c0 + plane * (ps.k0 + kk);
            __builtin_nontemporal_store(ps_, &pout[c]);
            apout[c] = as_;
            if (xupd) __builtin_nontemporal_store(xa[kk], &xo[c]);
        }
        const double ad = ok ? (double)as_ : 0.0;
        const double rd = ok ? r[kk] : 0.0;
        acc_num = fma(rd, ad, acc_num);
        acc_d = fma(ad, ad, acc_d);
    }
    const double sn = block_sum(acc_num, sh);
    const double sd = block_sum(acc_d, sh);
    if (threadIdx.x == 0) {
        in.part[(long long)(0) * in.pstride + lb] = sn;
        in.part[(long long)(1) * in.pstride + lb] = sd;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_finish_beta(Table<T> tb, int init)
{
    __shared__ SolveState s_st;
    const Inst<T>& in = tb.inst[blockIdx.x];
    SolveState* gst = in.st;
    const long long word = state_word_load(gst);
    double v[2];
    sum_partials<2, 8>(in, in.nblk_dir, 0, 2, v);
    state_word_stage(&s_st, word);
    __syncthreads();
    SolveState* st = &s_st;
    if (st->status != RUNNING) return;
    if (!init && !st->active) return;
    if (threadIdx.x == 0) decide_beta(st, v[0], v[1], init);
    __syncthreads();
    state_word_store(gst, st);
}

// x = x_base + sum_{l = x_base_nu .. x_final_hi} beta_l p^l, into X[0].
template <typename T, int KC, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_finalize_x(Table<T> tb)
{
    const int m = find_inst(tb.blk0_st, tb.n, blockIdx.x);
    const Inst<T>& in = tb.inst[m];
    const int lb = blockIdx.x - tb.blk0_st[m];
    const SolveState* st = in.st;
    const int lo = st->x_base_nu, hi = st->x_final_hi;
    if (st->x_base == 0 && hi < lo) return;
    const StPos ps = st_pos_m<MESH>(in, lb, in.kc, in.ord_st);
    if (!ps.col_ok) return;
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
    // e events run between the step's decision and its stencil pass: they
    // apply when the step passed its tests (its e feeds the new direction);
    // e belongs to no backup, so nothing is copied first
    st->ev_ok = (vec == FTGCR_V_E) ? st->e_ok : (st->status == RUNNING);
    if (!st->ev_ok) return;
    st->ev_vec = vec;
    st->ev_copy = 0;
    if (vec == FTGCR_V_E) return;
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
        else if (vec == FTGCR_V_AP) write_xor<T>(in.AP[st->slot[st->nu]] + at, bit);
        else write_xor<T>(in.E + at, bit);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->events_applied += 1;
        st->events_since_rb = 1;
    }
}

// <r, L p^nu> and <L p^nu, L p^nu> recomputed after a flip in r or L(p^nu).
template <typename T, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_beta_dots(Table<T> tb)
{
    __shared__ double sh[4];
    const Inst<T>& in = tb.inst[0];
    SolveState* st = in.st;
    if (!st->ev_ok) return;
    const int lb = blockIdx.x;
    const StPos ps = st_pos_m<MESH>(in, lb, in.kc, in.ord_st);
    double an = 0.0, ad = 0.0;
    if (ps.col_ok) {
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
        in.part[(long long)(0) * in.pstride + lb] = sn;
        in.part[(long long)(1) * in.pstride + lb] = sd;
    }
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void k_finish_beta_dots(Table<T> tb)
{
    const Inst<T>& in = tb.inst[0];
    SolveState* st = in.st;
    if (!st->ev_ok) return;
    double v[2];
    sum_partials<2, 8>(in, in.nblk_st, 0, 2, v);
    const double num = v[0], dn = v[1];
    if (threadIdx.x == 0) {
        st->beta_num = num;
        st->d_cur = dn;
        st->d[st->nu] = dn;
    }
}

// ---------------------------------------------------------------------------
// parity entry points
// ---------------------------------------------------------------------------

template <int KC, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_debug_apply_A(Table<double> tb, const double* x, double* y)
{
    const Inst<double>& in = tb.inst[0];
    const StPos ps = st_pos_m<MESH>(in, blockIdx.x, in.kc, in.ord_st);
    double ax[KC];
    stencil_m<double, KC, MESH>(in.g, x, ps, ax);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
        if (ps.col_ok && ps.k0 + kk < in.g.nz)
            y[(long long)ps.i + (long long)in.g.nx * ps.j + (long long)in.g.ncols * (ps.k0 + kk)] = ax[kk];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

#define FTGCR_KC_SWITCH(kc, CALL)                         \
    switch (kc) {                                         \
    case 1: { constexpr int KCV = 1; CALL; } break;       \
    case 2: { constexpr int KCV = 2; CALL; } break;       \
    case 4: { constexpr int KCV = 4; CALL; } break;       \
    case 8: { constexpr int KCV = 8; CALL; } break;       \
    default: { constexpr int KCV = 16; CALL; } break;     \
    }

// A launch whose start and stop times, if events are given, are taken by
// the dispatch itself (no separate event packets on the stream).
#define FTGCR_TIMED_LAUNCH(E0, E1, KERNEL, GRID, BLOCK, S, ...)                       \
    do {                                                                              \
        if (E0)                                                                       \
            hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, S, E0, E1, 0, __VA_ARGS__); \
        else                                                                          \
            hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, S, __VA_ARGS__);               \
    } while (0)

#define FTGCR_H_SWITCH(H, CALL)                           \
    switch (H) {                                          \
    case 4: { constexpr int HV = 4; CALL; } break;        \
    case 8: { constexpr int HV = 8; CALL; } break;        \
    case 16: { constexpr int HV = 16; CALL; } break;      \
    case 24: { constexpr int HV = 24; CALL; } break;      \
    case 28: { constexpr int HV = 28; CALL; } break;      \
    case 32: { constexpr int HV = 32; CALL; } break;      \
    default: { constexpr int HV = 48; CALL; } break;      \
    }

// Half-column depth of the column pass: the smallest template depth that
// holds (nz + 1) / 2 levels (28 serves the paper's 51-level O_N columns,
// half columns of 26, with 8 phantom rows instead of 12 at 32: 44.5 ->
// 41.4 us per launch on O160 x 51).
int thomas_depth(int nz)
{
    const int h = (nz + 1) / 2;
    const int depths[] = {4, 8, 16, 24, 28, 32, 48};
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
void Launch<T>::set_round(const Table<T>& tb, double tol2, long long max_steps, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_round<T>, dim3(tb.n), dim3(64), 0, s, tb, tol2, max_steps);
}

// A stencil-pass launch on the table's mesh.
#define FTGCR_MESH_LAUNCH(tb, LAUNCH0, LAUNCH1)                                   \
    do {                                                                          \
        if ((tb).mesh == FTGCR_MESH_OCTAHEDRAL) {                                 \
            constexpr int MESHV = FTGCR_MESH_OCTAHEDRAL;                          \
            LAUNCH1;                                                              \
        } else {                                                                  \
            constexpr int MESHV = FTGCR_MESH_LATLON;                              \
            LAUNCH0;                                                              \
        }                                                                         \
    } while (0)

template <typename T>
void Launch<T>::residual(const Table<T>& tb, int total, int kc, int store, int set_T, hipStream_t s)
{
    FTGCR_MESH_LAUNCH(tb,
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_residual<T, KCV, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb,
                                               store)),
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_residual<T, KCV, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb,
                                               store)));
    hipLaunchKernelGGL(k_finish_residual<T>, dim3(tb.n), dim3(RED_THREADS), 0, s, tb, set_T);
}

template <typename T>
void Launch<T>::update_thomas(const Table<T>& tb, int total, int H, int mode, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1)
{
    if (tb.precond == FTGCR_PRECOND_NONE) {
        const int cpb = col_block_cols((int)sizeof(T), H);
        if (mode == MODE_STEP)
            FTGCR_TIMED_LAUNCH(e0, e1, (k_update_copy<T, MODE_STEP>), dim3(total), dim3(COL_THREADS), s, tb,
                               (const T*)nullptr, (T*)nullptr, (const GmInst*)nullptr, cpb);
        else
            hipLaunchKernelGGL((k_update_copy<T, MODE_INIT>), dim3(total), dim3(COL_THREADS), 0, s, tb,
                               (const T*)nullptr, (T*)nullptr, (const GmInst*)nullptr, cpb);
        return;
    }
    if constexpr (sizeof(T) == 4) {
        if (col_block_cols((int)sizeof(T), H) == COL_THREADS) {
            // one lane per column: NZ = 2H levels at most (H <= 32)
#define FTGCR_T1(HH)                                                                                        \
    if (mode == MODE_STEP)                                                                                  \
        FTGCR_TIMED_LAUNCH(e0, e1, (k_update_thomas1<T, 2 * HH, MODE_STEP>), dim3(total), dim3(COL_THREADS), \
                           s, tb);                                                                          \
    else                                                                                                    \
        hipLaunchKernelGGL((k_update_thomas1<T, 2 * HH, MODE_INIT>), dim3(total), dim3(COL_THREADS), 0, s, tb);
            switch (H) {
            case 4: FTGCR_T1(4) break;
            case 8: FTGCR_T1(8) break;
            case 16: FTGCR_T1(16) break;
            case 24: FTGCR_T1(24) break;
            case 28: FTGCR_T1(28) break;
            default: FTGCR_T1(32) break;
            }
#undef FTGCR_T1
            return;
        }
    }
    if (mode == MODE_STEP && tb.full)
        FTGCR_H_SWITCH(H, FTGCR_TIMED_LAUNCH(e0, e1, (k_update_thomas_full<T, HV>), dim3(total), dim3(COL_THREADS),
                                             s, tb))
    else if (mode == MODE_STEP)
        FTGCR_H_SWITCH(H, FTGCR_TIMED_LAUNCH(e0, e1, (k_update_thomas<T, HV, MODE_STEP>), dim3(total),
                                             dim3(COL_THREADS), s, tb, (const T*)nullptr, (T*)nullptr))
    else
        FTGCR_H_SWITCH(H, hipLaunchKernelGGL((k_update_thomas<T, HV, MODE_INIT>), dim3(total), dim3(COL_THREADS), 0,
                                             s, tb, (const T*)nullptr, (T*)nullptr))
}

template <typename T>
void Launch<T>::finish_col(const Table<T>& tb, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_col<T>, dim3(tb.n), dim3(RED_THREADS), 0, s, tb, mode);
}

template <typename T>
void Launch<T>::finish_alpha(const Table<T>& tb, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_alpha<T>, dim3(tb.n), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::finish_beta(const Table<T>& tb, int init, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_beta<T>, dim3(tb.n), dim3(RED_THREADS), 0, s, tb, init);
}

template <typename T>
void Launch<T>::stencil_dots(const Table<T>& tb, int total, int kc, int spec, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1)
{
    FTGCR_MESH_LAUNCH(tb,
        FTGCR_KC_SWITCH(kc, FTGCR_TIMED_LAUNCH(e0, e1, (k_stencil_dots<T, KCV, MESHV>), dim3(total),
                                               dim3(ST_THREADS), s, tb, spec)),
        FTGCR_KC_SWITCH(kc, FTGCR_TIMED_LAUNCH(e0, e1, (k_stencil_dots<T, KCV, MESHV>), dim3(total),
                                               dim3(ST_THREADS), s, tb, spec)));
}

template <typename T>
void Launch<T>::finish_step(const Table<T>& tb, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_step<T>, dim3(tb.n), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::dir_update(const Table<T>& tb, int total, int kc, int init, bool nt_ap, hipStream_t s,
                           hipEvent_t e0, hipEvent_t e1)
{
    if (nt_ap)
        FTGCR_MESH_LAUNCH(tb,
            FTGCR_KC_SWITCH(kc, FTGCR_TIMED_LAUNCH(e0, e1, (k_dir_update<T, KCV, true, MESHV>), dim3(total),
                                                   dim3(ST_THREADS), s, tb, init)),
            FTGCR_KC_SWITCH(kc, FTGCR_TIMED_LAUNCH(e0, e1, (k_dir_update<T, KCV, true, MESHV>), dim3(total),
                                                   dim3(ST_THREADS), s, tb, init)));
    else
        FTGCR_MESH_LAUNCH(tb,
            FTGCR_KC_SWITCH(kc, FTGCR_TIMED_LAUNCH(e0, e1, (k_dir_update<T, KCV, false, MESHV>), dim3(total),
                                                   dim3(ST_THREADS), s, tb, init)),
            FTGCR_KC_SWITCH(kc, FTGCR_TIMED_LAUNCH(e0, e1, (k_dir_update<T, KCV, false, MESHV>), dim3(total),
                                                   dim3(ST_THREADS), s, tb, init)));
}

template <typename T>
void Launch<T>::finalize_x(const Table<T>& tb, int total, int kc, hipStream_t s)
{
    FTGCR_MESH_LAUNCH(tb,
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_finalize_x<T, KCV, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb)),
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_finalize_x<T, KCV, MESHV>), dim3(total), dim3(ST_THREADS), 0, s,
                                               tb)));
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
    FTGCR_MESH_LAUNCH(tb, hipLaunchKernelGGL((k_beta_dots<T, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb),
                      hipLaunchKernelGGL((k_beta_dots<T, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb));
    hipLaunchKernelGGL(k_finish_beta_dots<T>, dim3(1), dim3(RED_THREADS), 0, s, tb);
}

template <typename T>
void Launch<T>::debug_apply_A(const Table<T>&, int, int, const double*, double*, hipStream_t)
{
}

template <>
void Launch<double>::debug_apply_A(const Table<double>& tb, int total, int kc, const double* in, double* out,
                                   hipStream_t s)
{
    FTGCR_MESH_LAUNCH(tb,
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_debug_apply_A<KCV, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb,
                                               in, out)),
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_debug_apply_A<KCV, MESHV>), dim3(total), dim3(ST_THREADS), 0, s, tb,
                                               in, out)));
}

template <typename T>
void Launch<T>::debug_pinv(const Table<T>&, int, int, const double*, double*, hipStream_t)
{
}

template <>
void Launch<double>::debug_pinv(const Table<double>& tb, int total, int H, const double* in, double* out,
                                hipStream_t s)
{
    if (tb.precond == FTGCR_PRECOND_NONE) {
        hipLaunchKernelGGL((k_update_copy<double, MODE_DEBUG>), dim3(total), dim3(COL_THREADS), 0, s, tb, in, out,
                           (const GmInst*)nullptr, COLS_PER_BLOCK);
        return;
    }
    FTGCR_H_SWITCH(H, hipLaunchKernelGGL((k_update_thomas<double, HV, MODE_DEBUG>), dim3(total), dim3(COL_THREADS),
                                         0, s, tb, in, out));
}

// Status and step count of every instance into a small device array (one
// read-back per poll of a batched solve).
template <typename T>
__global__ void k_gather_status(Table<T> tb, long long* out)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= tb.n) return;
    const SolveState* st = tb.inst[m].st;
    out[2 * m] = st->status;
    out[2 * m + 1] = st->s;
}

template <typename T>
void Launch<T>::gather_status(const Table<T>& tb, long long* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_gather_status<T>, dim3((tb.n + 63) / 64), dim3(64), 0, s, tb, out);
}

template struct Launch<double>;
template struct Launch<float>;

// ---------------------------------------------------------------------------
// FT-GMRES(k): the fault layer of Algorithm 1 on restarted GMRES(k)
// ---------------------------------------------------------------------------
//
// Right-preconditioned restarted GMRES with classical Gram-Schmidt and Givens
// rotations; the residual-norm test after every step (on the rotated
// right-hand side |g_{j+1}|, the minimised residual norm of the cycle) and on
// the explicit residual at the end of every cycle, the backup [x, |s|^2] of
// each cycle that passes, the rollback and the stagnation rule of FT-GCR.
// Per cycle the host enqueues: residual s = R - A x (into U[0]), restart (the
// cycle-end decisions, then g_0 = |s|); k steps of
//   precond      v_j = U[j] / den[j] (written back), z_j = P^{-1} v_j
//   stencil      w = A z_j (stored) and the partials of <w, v_i>, i <= j
//   finish_h     h_ij
//   orth         w - sum_i h_ij v_i into U[j+1], partials of its norm
//   finish_step  h_{j+1,j}, rotations, |g_{j+1}|^2, exit and fault tests
// then xupd (x + sum_i y_i z_i, y from the triangular system) and finish_x.
// Every step kernel returns at once once the cycle is inactive (ended,
// rolled back or the solve finished), so a cycle is a fixed launch sequence.

__device__ __forceinline__ StPos gm_pos(const GmInst& in, int lb)
{
    StPos p;
    int ct, bz;
    block_tile(lb, in.tx * in.ty, in.tz, in.ord, ct, bz);
    if (in.g.mesh == FTGCR_MESH_OCTAHEDRAL) {   // ST_THREADS consecutive points per block
        const int i = ct * ST_THREADS + threadIdx.x;
        p.col_ok = i < in.g.nx;
        p.i = p.col_ok ? i : in.g.nx - 1;
        p.j = 0;
        p.k0 = bz * in.kc;
        return p;
    }
    const int bx = ct % in.tx;
    const int by = ct / in.tx;
    const int i = bx * ST_TX + (threadIdx.x & (ST_TX - 1));
    const int j = by * ST_TY + (threadIdx.x / ST_TX);
    p.col_ok = i < in.g.nx && j < in.g.ny;
    p.i = i < in.g.nx ? i : in.g.nx - 1;
    p.j = j < in.g.ny ? j : in.g.ny - 1;
    p.k0 = bz * in.kc;
    return p;
}

__global__ void k_gm_init(const GmInst* gi, int k, int ft, long long max_steps, double tol2)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    GmState* st = gi->st;
    st->status = RUNNING;
    st->active = 0;
    st->j = 0;
    st->k = k;
    st->ft = ft;
    st->phase = GM_INIT;
    st->jdone = 0;
    st->cycle_end = 0;
    st->capped = 0;
    st->x_cur = 0;
    st->x_bak = 0;
    st->x_dst = 0;
    st->detections = 0;
    st->stagnation_accepts = 0;
    st->events_applied = 0;
    st->events_since_rb = 1;
    st->log_len = 0;
    st->ev_ok = 0;
    st->s = 0;
    st->max_steps = max_steps;
    st->accepted = 0;
    st->cycles = 0;
    st->last_rb_pos = -1;
    st->b_accepted = 0;
    st->tol2 = tol2;
}

// s = R - A x into U[0]; partials of <R, R> (row 0) and <s, s> (row 1).
template <int KC, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_gm_residual(const GmInst* gi)
{
    __shared__ double sh[4];
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (st->status != RUNNING) return;
    const StPos ps = gm_pos(in, blockIdx.x);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    double ax[KC], b[KC];
    stencil_m<double, KC, MESH>(in.g, in.X[st->x_cur], ps, ax);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        b[kk] = in.rhs[c0 + plane * kq];
    }
    double ss = 0.0, bb = 0.0;
    double* u0 = in.U[0];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        const double r = ok ? b[kk] - ax[kk] : 0.0;
        const double bv = ok ? b[kk] : 0.0;
        if (ok) u0[c0 + plane * (ps.k0 + kk)] = r;
        ss = fma(r, r, ss);
        bb = fma(bv, bv, bb);
    }
    const double sb = block_sum(bb, sh);
    const double sr = block_sum(ss, sh);
    if (threadIdx.x == 0) {
        in.part[blockIdx.x] = sb;
        in.part[in.pstride + blockIdx.x] = sr;
    }
}

__device__ void gm_log(GmState* st, long long step, int nu, int action, double rr_old, double rr_new)
{
    st->detections += 1;
    if (st->log_len < LOG_CAP) {
        DetectRec& rec = st->log[st->log_len++];
        rec.step = step;
        rec.nu = nu;
        rec.action = action;
        rec.rr_old = rr_old;
        rec.rr_new = rr_new;
    }
}

// The explicit residual's decisions (first pass: the initial state; after
// a cycle: exit test, then the fault test against the backup, then the new
// backup; after a rollback: none), then a new cycle from |s|.
__global__ __launch_bounds__(RED_THREADS) void k_gm_restart(const GmInst* gi)
{
    const GmInst& in = *gi;
    GmState* st = in.st;
    if (st->status != RUNNING) return;
    double v[2];
    sum_partials<2, 8>(in, in.nblk_st, 0, 2, v);
    if (threadIdx.x != 0) return;
    const double rho2 = v[1];
    st->rho2 = rho2;
    if (st->phase == GM_INIT) {
        st->RR = v[0];
        st->T = st->tol2 * v[0];
        if (rho2 <= st->T) {
            st->status = FTGCR_CONVERGED;
            return;
        }
        st->x_bak = st->x_cur;
        st->b_rho2 = rho2;
        st->b_accepted = 0;
    } else if (st->phase == GM_CHECK) {
        if (st->capped || (st->s >= st->max_steps && rho2 > st->T)) {
            st->status = FTGCR_MAX_STEPS;
            return;
        }
        if (rho2 <= st->T) {
            st->status = FTGCR_CONVERGED;
            return;
        }
        if (st->ft && !(rho2 < st->b_rho2)) {   // NaN included
            const long long pos = 2 * st->accepted + 1;
            const int stag = (pos == st->last_rb_pos) && !st->events_since_rb;
            gm_log(st, st->s, -1, stag, st->b_rho2, rho2);
            if (!stag) {
                st->x_cur = st->x_bak;
                st->accepted = st->b_accepted;
                st->last_rb_pos = pos;
                st->events_since_rb = 0;
                st->phase = GM_REDO;
                st->active = 0;
                st->cycle_end = 0;
                return;   // the next residual pass is that of the restored x
            }
            st->stagnation_accepts += 1;
        }
        if (st->ft) {
            st->x_bak = st->x_cur;
            st->b_rho2 = rho2;
            st->b_accepted = st->accepted;
        }
    }
    if (st->s >= st->max_steps) {
        st->status = FTGCR_MAX_STEPS;
        return;
    }
    const double rho = sqrt(rho2);
    st->den[0] = rho;
    st->g[0] = rho;
    for (int i = 1; i <= st->k; ++i) st->g[i] = 0.0;
    st->rr_old = rho2;
    st->j = 0;
    st->jdone = 0;
    st->cycle_end = 0;
    st->capped = 0;
    st->active = 1;
    st->phase = GM_CHECK;
}

// The partials of <w, v_i>, i <= j, of a block's cells (rows DOT_ROW0 + i).
// The loop over i is unrolled to KMAX with a uniform guard, and the loads of
// v_{i+1} are issued before v_i's values are used (two buffers alternating
// with the parity of i), so the terms cost one memory round trip together
// rather than one each.
template <int KC>
__device__ __forceinline__ void gm_dots(const GmInst& in, const StPos& ps, const double (&w)[KC], int j)
{
    __shared__ double sh[KMAX + 1][4];
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double buf[2][KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        buf[0][kk] = in.U[0][c0 + plane * kq];
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (i <= j) {
            if (i + 1 < KMAX && i + 1 <= j) {
                const double* vn = in.U[i + 1];
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                    buf[(i + 1) & 1][kk] = vn[c0 + plane * kq];
                }
            }
            double acc = 0.0;
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) {
                const bool ok = ps.col_ok && ps.k0 + kk < nz;
                acc = fma(w[kk], ok ? buf[i & 1][kk] : 0.0, acc);
            }
            const double t = wave_sum(acc);
            if (lane == 0) sh[i][wv] = t;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= j) {
        const int i = threadIdx.x;
        in.part[(long long)(DOT_ROW0 + i) * in.pstride + blockIdx.x] = ((sh[i][0] + sh[i][1]) + sh[i][2]) + sh[i][3];
    }
}

// w = A z_j into W; with DOTS also the partials of <w, v_i>.
template <int KC, int DOTS, int MESH>
__global__ __launch_bounds__(ST_THREADS) void k_gm_stencil(const GmInst* gi)
{
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    const int j = st->j;
    const StPos ps = gm_pos(in, blockIdx.x);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    double w[KC];
    stencil_m<double, KC, MESH>(in.g, in.Z[j], ps, w);
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        if (ok) in.W[c0 + plane * (ps.k0 + kk)] = w[kk];
        else w[kk] = 0.0;
    }
    if (DOTS) gm_dots<KC>(in, ps, w, j);
}

// The partials of <w, v_i> from the stored w (after a fault event on it).
template <int KC>
__global__ __launch_bounds__(ST_THREADS) void k_gm_dots(const GmInst* gi)
{
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    const StPos ps = gm_pos(in, blockIdx.x);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    double w[KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        const double v = in.W[c0 + plane * kq];
        w[kk] = ok ? v : 0.0;
    }
    gm_dots<KC>(in, ps, w, st->j);
}

__global__ __launch_bounds__(RED_THREADS) void k_gm_finish_h(const GmInst* gi)
{
    const GmInst& in = *gi;
    GmState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    const int j = st->j;
    const double* v = sum_partials<4, 4>(in, in.nblk_st, DOT_ROW0, j + 1, nullptr);
    if ((int)threadIdx.x <= j) st->H[threadIdx.x * KMAX + j] = v[threadIdx.x];
}

// U[j+1] = w - sum_i h_ij v_i (ascending i); partials of its squared norm.
// Each cell takes the same operations in the same order as a loop over i
// per cell; the loop over i runs outside (unrolled to KMAX, uniform guard)
// with v_{i+1}'s loads issued before v_i is used.
template <int KC>
__global__ __launch_bounds__(ST_THREADS) void k_gm_orth(const GmInst* gi)
{
    __shared__ double sh[4];
    __shared__ double s_h[KMAX + 1];
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    const int j = st->j;
    if ((int)threadIdx.x <= j) s_h[threadIdx.x] = st->H[threadIdx.x * KMAX + j];
    __syncthreads();
    const StPos ps = gm_pos(in, blockIdx.x);
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    double* un = in.U[j + 1];
    double w[KC], buf[2][KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        const long long c = c0 + plane * kq;
        w[kk] = in.W[c];
        buf[0][kk] = in.U[0][c];
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (i <= j) {
            if (i + 1 < KMAX && i + 1 <= j) {
                const double* vn = in.U[i + 1];
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                    buf[(i + 1) & 1][kk] = vn[c0 + plane * kq];
                }
            }
            const double h = s_h[i];
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) w[kk] = w[kk] - h * buf[i & 1][kk];
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const bool ok = ps.col_ok && ps.k0 + kk < nz;
        if (ok) un[c0 + plane * (ps.k0 + kk)] = w[kk];
        const double wd = ok ? w[kk] : 0.0;
        acc = fma(wd, wd, acc);
    }
    const double sw = block_sum(acc, sh);
    if (threadIdx.x == 0) in.part[blockIdx.x] = sw;
}

// h_{j+1,j}, the rotations, the step's residual norm |g_{j+1}|^2, then the
// exit test and the fault test of the step.
__global__ __launch_bounds__(RED_THREADS) void k_gm_finish_step(const GmInst* gi)
{
    const GmInst& in = *gi;
    GmState* st = in.st;
    if (st->status != RUNNING || !st->active) return;
    double v[2];
    sum_partials<2, 8>(in, in.nblk_st, 0, 1, v);
    if (threadIdx.x != 0) return;
    const int j = st->j;
    double* H = st->H;
    const double hn = sqrt(v[0]);
    H[(j + 1) * KMAX + j] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = H[i * KMAX + j], b = H[(i + 1) * KMAX + j];
        H[i * KMAX + j] = st->cs[i] * a + st->sn[i] * b;
        H[(i + 1) * KMAX + j] = -st->sn[i] * a + st->cs[i] * b;
    }
    {
        const double a = H[j * KMAX + j], b = H[(j + 1) * KMAX + j];
        const double den = sqrt(a * a + b * b);
        st->cs[j] = a / den;
        st->sn[j] = b / den;
        H[j * KMAX + j] = den;
        H[(j + 1) * KMAX + j] = 0.0;
        st->g[j + 1] = -st->sn[j] * st->g[j];
        st->g[j] = st->cs[j] * st->g[j];
    }
    const double rr_new = st->g[j + 1] * st->g[j + 1];
    st->s += 1;
    const long long s = st->s;
    if (j == 0) st->cycles += 1;
    if (s <= in.hist_cap) in.hist[s - 1] = rr_new;
    st->jdone = j + 1;
    if (rr_new <= st->T) {   // exit test first: the cycle ends, the check follows
        st->accepted += 1;
        st->rr_old = rr_new;
        st->cycle_end = 1;
        st->active = 0;
        return;
    }
    if (st->ft && !(rr_new < st->rr_old)) {   // NaN included
        const long long pos = 2 * (st->accepted + 1);
        const int stag = (pos == st->last_rb_pos) && !st->events_since_rb;
        gm_log(st, s, j, stag, st->rr_old, rr_new);
        if (!stag) {
            st->x_cur = st->x_bak;
            st->accepted = st->b_accepted;
            st->last_rb_pos = pos;
            st->events_since_rb = 0;
            st->phase = GM_REDO;
            st->active = 0;
            st->cycle_end = 0;
            return;
        }
        st->stagnation_accepts += 1;
    }
    st->accepted += 1;
    st->rr_old = rr_new;
    if (hn == 0.0 || j + 1 == st->k) {   // the cycle is complete (or its space holds the solution)
        st->cycle_end = 1;
        st->active = 0;
        return;
    }
    st->den[j + 1] = hn;
    st->j = j + 1;
    if (s >= st->max_steps) {   // the next step would pass the cap
        st->capped = 1;
        st->cycle_end = 1;
        st->active = 0;
    }
}

// The cycle's correction: y from the rotated triangular system over the
// steps done, then x + sum_i y_i z_i (ascending i) into a buffer that is not
// the backup.
template <int KC>
__global__ __launch_bounds__(ST_THREADS) void k_gm_xupd(const GmInst* gi)
{
    __shared__ double y[KMAX];
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (st->status != RUNNING || !st->cycle_end) return;
    const int jd = st->jdone;
    if (threadIdx.x == 0) {
        const double* H = st->H;
        for (int i = jd - 1; i >= 0; --i) {
            double acc = st->g[i];
            for (int l = i + 1; l < jd; ++l) acc = acc - H[i * KMAX + l] * y[l];
            y[i] = acc / H[i * KMAX + i];
        }
    }
    __syncthreads();
    const StPos ps = gm_pos(in, blockIdx.x);
    if (!ps.col_ok) return;
    const int nz = in.g.nz;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    const int xs = st->x_cur;
    const int xd = (st->x_cur == st->x_bak) ? 1 - st->x_cur : st->x_cur;
    const double* xsrc = in.X[xs];
    double* xdst = in.X[xd];
    // per cell x + y_0 z_0 + y_1 z_1 + ... in ascending i, the loop over i
    // outside (unrolled to KMAX, uniform guard) with z_{i+1}'s loads issued
    // before z_i is used
    double xv[KC], buf[2][KC];
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
        const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
        const long long c = c0 + plane * kq;
        xv[kk] = xsrc[c];
        buf[0][kk] = jd > 0 ? in.Z[0][c] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (i < jd) {
            if (i + 1 < KMAX && i + 1 < jd) {
                const double* zn = in.Z[i + 1];
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    const int kq = (ps.k0 + kk > nz - 1) ? nz - 1 : ps.k0 + kk;
                    buf[(i + 1) & 1][kk] = zn[c0 + plane * kq];
                }
            }
            const double yi = y[i];
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) xv[kk] = xv[kk] + yi * buf[i & 1][kk];
        }
    }
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
        if (ps.k0 + kk < nz) xdst[c0 + plane * (ps.k0 + kk)] = xv[kk];
}

__global__ void k_gm_finish_x(const GmInst* gi)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    GmState* st = gi->st;
    if (st->status != RUNNING || !st->cycle_end) return;
    st->x_cur = (st->x_cur == st->x_bak) ? 1 - st->x_cur : st->x_cur;
}

// The returned iterate into the caller's buffer X[0].
template <int KC>
__global__ __launch_bounds__(ST_THREADS) void k_gm_finalize(const GmInst* gi)
{
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (st->x_cur == 0) return;
    const StPos ps = gm_pos(in, blockIdx.x);
    if (!ps.col_ok) return;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    for (int kk = 0; kk < KC; ++kk) {
        if (ps.k0 + kk >= in.g.nz) break;
        in.X[0][c0 + plane * (ps.k0 + kk)] = in.X[st->x_cur][c0 + plane * (ps.k0 + kk)];
    }
}

// Fault events of executed step `step` (they apply only if that step is the
// one about to run, in an active cycle).  X: x at the start of the step,
// copied first if it still is the backup's buffer; R: v_j at the start of
// the step, stored normalised first (the flip acts on v_j itself); P and E:
// z_j after the preconditioner; AP: w = A z_j before the inner products.
__global__ void k_gm_event_prep(const GmInst* gi, int vec, long long step)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    GmState* st = gi->st;
    st->ev_ok = (st->status == RUNNING && st->active && st->s + 1 == step);
    st->ev_vec = vec;
    st->ev_copy = 0;
    if (!st->ev_ok) return;
    if (vec == FTGCR_V_X && st->x_cur == st->x_bak) {
        st->ev_copy = 1;
        st->ev_src = st->x_cur;
        st->ev_dst = 1 - st->x_cur;
        st->x_cur = st->ev_dst;
    } else if (vec == FTGCR_V_R && st->den[st->j] != 1.0) {
        st->ev_copy = 1;
    }
}

template <int KC>
__global__ __launch_bounds__(ST_THREADS) void k_gm_event_copy(const GmInst* gi)
{
    const GmInst& in = *gi;
    const GmState* st = in.st;
    if (!st->ev_ok || !st->ev_copy) return;
    const StPos ps = gm_pos(in, blockIdx.x);
    if (!ps.col_ok) return;
    const long long plane = (long long)in.g.ncols;
    const long long c0 = (long long)ps.i + (long long)in.g.nx * ps.j;
    const int j = st->j;
    const double den = st->den[j];
    for (int kk = 0; kk < KC; ++kk) {
        if (ps.k0 + kk >= in.g.nz) break;
        const long long c = c0 + plane * (ps.k0 + kk);
        if (st->ev_vec == FTGCR_V_X) in.X[st->ev_dst][c] = in.X[st->ev_src][c];
        else in.U[j][c] = in.U[j][c] / den;
    }
}

__global__ void k_gm_event_inject(const GmInst* gi, const long long* idx, const unsigned char* bits, long long count,
                                  long long start, int bit0)
{
    const GmInst& in = *gi;
    GmState* st = in.st;
    if (!st->ev_ok) return;
    const int vec = st->ev_vec;
    const int j = st->j;
    double* target = vec == FTGCR_V_X ? in.X[st->x_cur]
                   : vec == FTGCR_V_R ? in.U[j]
                   : vec == FTGCR_V_AP ? in.W : in.Z[j];
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride) {
        const long long at = idx ? idx[t] : start + t;
        const int bit = bits ? (int)bits[t] : bit0;
        write_xor<double>(target + at, bit);
    }
    // the grid's last use of the prepared state is above; the one-thread
    // bookkeeping below touches fields no thread reads here
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->events_applied += 1;
        st->events_since_rb = 1;
        if (vec == FTGCR_V_R) st->den[j] = 1.0;   // v_j is stored normalised now
    }
}

void GmLaunch::init(const GmInst* gi, int k, int ft, long long max_steps, double tol2, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(64), 0, s, gi, k, ft, max_steps, tol2);
}

void GmLaunch::residual(const GmInst* gi, int nblk, int kc, int mesh, hipStream_t s)
{
    if (mesh == FTGCR_MESH_OCTAHEDRAL)
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_residual<KCV, FTGCR_MESH_OCTAHEDRAL>), dim3(nblk),
                                               dim3(ST_THREADS), 0, s, gi))
    else
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_residual<KCV, FTGCR_MESH_LATLON>), dim3(nblk),
                                               dim3(ST_THREADS), 0, s, gi))
}

void GmLaunch::restart(const GmInst* gi, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_restart, dim3(1), dim3(RED_THREADS), 0, s, gi);
}

void GmLaunch::precond(const Table<double>& tb, const GmInst* gi, int nblk_col, int H, hipStream_t s)
{
    if (tb.precond == FTGCR_PRECOND_NONE) {
        hipLaunchKernelGGL((k_update_copy<double, MODE_GM>), dim3(nblk_col), dim3(COL_THREADS), 0, s, tb,
                           (const double*)nullptr, (double*)nullptr, gi, COLS_PER_BLOCK);
        return;
    }
    if (tb.full)
        FTGCR_H_SWITCH(H, hipLaunchKernelGGL((k_update_thomas_gm_full<HV>), dim3(nblk_col), dim3(COL_THREADS), 0, s,
                                             tb, gi))
    else
        FTGCR_H_SWITCH(H, hipLaunchKernelGGL((k_update_thomas_gm<HV>), dim3(nblk_col), dim3(COL_THREADS), 0, s, tb,
                                             gi))
}

void GmLaunch::stencil(const GmInst* gi, int nblk, int kc, int dots, int mesh, hipStream_t s)
{
#define FTGCR_GM_STENCIL(MV)                                                                                  \
    if (dots)                                                                                                 \
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_stencil<KCV, 1, MV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi)) \
    else                                                                                                      \
        FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_stencil<KCV, 0, MV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi))
    if (mesh == FTGCR_MESH_OCTAHEDRAL) {
        FTGCR_GM_STENCIL(FTGCR_MESH_OCTAHEDRAL)
    } else {
        FTGCR_GM_STENCIL(FTGCR_MESH_LATLON)
    }
#undef FTGCR_GM_STENCIL
}

void GmLaunch::dots(const GmInst* gi, int nblk, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_dots<KCV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi));
}

void GmLaunch::finish_h(const GmInst* gi, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_finish_h, dim3(1), dim3(RED_THREADS), 0, s, gi);
}

void GmLaunch::orth(const GmInst* gi, int nblk, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_orth<KCV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi));
}

void GmLaunch::finish_step(const GmInst* gi, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_finish_step, dim3(1), dim3(RED_THREADS), 0, s, gi);
}

void GmLaunch::xupd(const GmInst* gi, int nblk, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_xupd<KCV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi));
}

void GmLaunch::finish_x(const GmInst* gi, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_finish_x, dim3(1), dim3(64), 0, s, gi);
}

void GmLaunch::finalize(const GmInst* gi, int nblk, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_finalize<KCV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi));
}

void GmLaunch::event_prep(const GmInst* gi, int vec, long long step, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_event_prep, dim3(1), dim3(64), 0, s, gi, vec, step);
}

void GmLaunch::event_copy(const GmInst* gi, int nblk, int kc, hipStream_t s)
{
    FTGCR_KC_SWITCH(kc, hipLaunchKernelGGL((k_gm_event_copy<KCV>), dim3(nblk), dim3(ST_THREADS), 0, s, gi));
}

void GmLaunch::event_inject(const GmInst* gi, int grid, const long long* idx, const unsigned char* bits,
                            long long count, long long start, int bit, hipStream_t s)
{
    hipLaunchKernelGGL(k_gm_event_inject, dim3(grid), dim3(256), 0, s, gi, idx, bits, count, start, bit);
}

// ---------------------------------------------------------------------------
// bandwidth probe: a plain streaming copy, the reference for what a kernel
// that reads and writes each byte once can reach on this device
// ---------------------------------------------------------------------------

// Each thread moves COPY_UNROLL 16-byte vectors, a block's vectors
// contiguous per unrolled step (full 1 KiB wave segments); all loads of a
// thread are issued before its first store.
constexpr int COPY_UNROLL = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_bw_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                 long long nvec)
{
    const long long base = (long long)blockIdx.x * (256 * COPY_UNROLL) + threadIdx.x;
    u32x4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const long long q = base + (long long)u * 256;
        const long long qc = q < nvec ? q : nvec - 1;   // clamped: branch-free loads
        v[u] = __builtin_nontemporal_load(&src[qc]);
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const long long q = base + (long long)u * 256;
        if (q < nvec) __builtin_nontemporal_store(v[u], &dst[q]);
    }
}

void launch_bw_copy(const void* src, void* dst, long long bytes, hipStream_t s)
{
    const long long nvec = bytes / 16;
    const long long blocks = (nvec + 256 * COPY_UNROLL - 1) / (256 * COPY_UNROLL);
    hipLaunchKernelGGL(k_bw_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const u32x4*)src, (u32x4*)dst, nvec);
}

}  // namespace ftgcr
