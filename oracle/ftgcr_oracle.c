/*
 * FT-GCR reference oracle -- TEST INFRASTRUCTURE ONLY (see ftgcr_oracle.h).
 *
 * Plain FP64 C, written to be checked by eye against the paper (Gillard &
 * Benacchio, arXiv 2103.07210) and the frozen operator readings.  No
 * blocking, fusion or reordering: every step of Algorithm 1 is a separate
 * whole-vector pass, every inner product is a left-to-right sum.
 *
 * Threads (OpenMP builds, orc_set_threads): only the face weights and the
 * operator and preconditioner applications are split, by whole planes or
 * columns whose
 * outputs are disjoint and computed with the same operations in the same
 * order as in the serial loop, so every result is bitwise the serial one;
 * inner products and vector updates stay single serial loops.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -fPIC -shared -lm
 */
#include "ftgcr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#define ORC_OMP(x) _Pragma(#x)
#else
#define ORC_OMP(x)
#endif

/* fields smaller than this are never split across threads */
#define ORC_PAR_MIN 65536

int orc_set_threads(int32_t n)
{
    if (n < 1) return -1;
#ifdef _OPENMP
    omp_set_num_threads(n);
    return 0;
#else
    return n == 1 ? 0 : -1;
#endif
}

int32_t orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------- */
/* Geometry of the lat-lon-height shell (unit sphere, normalised height).     */
/* Cell centres lon (i+1/2) dlon, lat -pi/2 + (j+1/2) dlat, zeta (k+1/2)/nz;  */
/* face i+1/2 at lon (i+1) dlon, face j-1/2 at lat -pi/2 + j dlat, face k-1/2 */
/* at zeta k/nz.                                                             */
/* ------------------------------------------------------------------------- */

static double lon_centre(const orc_problem* pb, int i) { return (i + 0.5) * (2.0 * M_PI / pb->nx); }
static double lon_face_east(const orc_problem* pb, int i) { return (i + 1.0) * (2.0 * M_PI / pb->nx); }
static double lat_centre(const orc_problem* pb, int j) { return -0.5 * M_PI + (j + 0.5) * (M_PI / pb->ny); }
static double lat_face_south(const orc_problem* pb, int j) { return -0.5 * M_PI + j * (M_PI / pb->ny); }
static double zeta_centre(const orc_problem* pb, int k) { return (k + 0.5) / pb->nz; }
static double zeta_face_below(const orc_problem* pb, int k) { return (double)k / pb->nz; }

/* Great-circle distance to the hill centre, haversine form (accurate near
 * the centre, where the arccos form loses about half the digits). */
double orc_hill(const orc_problem* pb, double lon, double lat)
{
    double s_lat = sin(0.5 * (lat - pb->hill_lat));
    double s_lon = sin(0.5 * (lon - pb->hill_lon));
    double hav = s_lat * s_lat + cos(lat) * cos(pb->hill_lat) * s_lon * s_lon;
    double root = sqrt(hav);
    if (root > 1.0) root = 1.0;
    double gc = 2.0 * asin(root);
    double q = gc / pb->hill_width;
    return exp(-(q * q));
}

/* Coefficient c(lon, lat, zeta) = 1 + a_h h(lon, lat) exp(-zeta / decay). */
static double coeff_c(const orc_problem* pb, double lon, double lat, double zeta)
{
    return 1.0 + pb->hill_amp * orc_hill(pb, lon, lat) * exp(-zeta / pb->decay_z);
}

void orc_face_weights(const orc_problem* pb, double* wx, double* wy, double* wz)
{
    const int nx = pb->nx, ny = pb->ny, nz = pb->nz;
    const double dlon = 2.0 * M_PI / nx;
    const double dlat = M_PI / ny;
    const double dz = pb->shell_depth / nz;
    const int par = (int64_t)nx * ny * nz >= ORC_PAR_MIN;
    (void)par;

    /* Longitude faces: flux c * (1/cos(lat)) d/dlon over a face of area
     * dlat*dz, difference over dlon. */
    ORC_OMP(omp parallel for schedule(static) if(par))
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = coeff_c(pb, lon_face_east(pb, i), lat_centre(pb, j), zeta_centre(pb, k));
                wx[((int64_t)k * ny + j) * nx + i] = c * dlat * dz / (cos(lat_centre(pb, j)) * dlon);
            }

    /* Latitude faces: flux c d/dlat over a face of area cos(lat_face)*dlon*dz;
     * zero flux through the two polar faces. */
    ORC_OMP(omp parallel for schedule(static) if(par))
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double w = 0.0;
                if (j > 0 && j < ny) {
                    double lat = lat_face_south(pb, j);
                    double c = coeff_c(pb, lon_centre(pb, i), lat, zeta_centre(pb, k));
                    w = c * cos(lat) * dlon * dz / dlat;
                }
                wy[((int64_t)k * (ny + 1) + j) * nx + i] = w;
            }

    /* Vertical faces: flux c d/dz over a face of area cos(lat)*dlon*dlat;
     * zero flux through bottom and top. */
    ORC_OMP(omp parallel for schedule(static) if(par))
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double w = 0.0;
                if (k > 0 && k < nz) {
                    double lat = lat_centre(pb, j);
                    double c = coeff_c(pb, lon_centre(pb, i), lat, zeta_face_below(pb, k));
                    w = c * cos(lat) * dlon * dlat / dz;
                }
                wz[((int64_t)k * ny + j) * nx + i] = w;
            }
}

/* Weights of the six faces of cell (i, j, k), in the order
 * west, east, south, north, below, above. */
static void cell_faces(const orc_problem* pb, const double* wx, const double* wy,
                       const double* wz, int i, int j, int k, double w[6])
{
    const int nx = pb->nx, ny = pb->ny;
    int iw = (i == 0) ? nx - 1 : i - 1;
    w[0] = wx[((int64_t)k * ny + j) * nx + iw];
    w[1] = wx[((int64_t)k * ny + j) * nx + i];
    w[2] = wy[((int64_t)k * (ny + 1) + j) * nx + i];
    w[3] = wy[((int64_t)k * (ny + 1) + j + 1) * nx + i];
    w[4] = wz[((int64_t)k * ny + j) * nx + i];
    w[5] = wz[((int64_t)(k + 1) * ny + j) * nx + i];
}

/* Diagonal of A at a cell: (1 + sigma) * (sum of the six face weights). */
static double diag_A(const orc_problem* pb, const double w[6])
{
    double d0 = w[0] + w[1] + w[2] + w[3] + w[4] + w[5];
    return (1.0 + pb->helmholtz) * d0;
}

void orc_apply_A(const orc_problem* pb, const double* wx, const double* wy,
                 const double* wz, const double* x, double* y)
{
    const int nx = pb->nx, ny = pb->ny, nz = pb->nz;
    const int64_t plane = (int64_t)nx * ny;
    const int par = plane * nz >= ORC_PAR_MIN;
    (void)par;
    ORC_OMP(omp parallel for schedule(static) if(par))
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double w[6];
                cell_faces(pb, wx, wy, wz, i, j, k, w);
                int64_t c = i + (int64_t)nx * (j + (int64_t)ny * k);
                int iw = (i == 0) ? nx - 1 : i - 1;
                int ie = (i == nx - 1) ? 0 : i + 1;
                double off = 0.0;
                off += w[0] * x[c - i + iw];
                off += w[1] * x[c - i + ie];
                if (j > 0) off += w[2] * x[c - nx];
                if (j < ny - 1) off += w[3] * x[c + nx];
                if (k > 0) off += w[4] * x[c - plane];
                if (k < nz - 1) off += w[5] * x[c + plane];
                y[c] = diag_A(pb, w) * x[c] - off;
            }
}

void orc_apply_pinv(const orc_problem* pb, const double* wx, const double* wy,
                    const double* wz, const double* r, double* e)
{
    const int nx = pb->nx, ny = pb->ny, nz = pb->nz;
    const int64_t plane = (int64_t)nx * ny;
    const int par = plane * nz >= ORC_PAR_MIN;
    (void)par;
    ORC_OMP(omp parallel if(par))
    {
    double* gam = (double*)malloc(sizeof(double) * nz);
    double* del = (double*)malloc(sizeof(double) * nz);
    ORC_OMP(omp for schedule(static))
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            /* Rows of the column system: a_k e_{k-1} + b_k e_k + u_k e_{k+1} = r_k,
             * with b = diagonal of A, a and u = minus the vertical face weights. */
            for (int k = 0; k < nz; ++k) {
                double w[6];
                cell_faces(pb, wx, wy, wz, i, j, k, w);
                double b = diag_A(pb, w);
                double a = -w[4];
                double u = -w[5];
                double rk = r[i + (int64_t)nx * j + plane * k];
                if (k == 0) {
                    gam[0] = u / b;
                    del[0] = rk / b;
                } else {
                    double m = b - a * gam[k - 1];
                    gam[k] = u / m;
                    del[k] = (rk - a * del[k - 1]) / m;
                }
            }
            e[i + (int64_t)nx * j + plane * (nz - 1)] = del[nz - 1];
            for (int k = nz - 2; k >= 0; --k)
                e[i + (int64_t)nx * j + plane * k] =
                    del[k] - gam[k] * e[i + (int64_t)nx * j + plane * (k + 1)];
        }
    free(gam);
    free(del);
    }
}

double orc_dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t t = 0; t < n; ++t) s += a[t] * b[t];
    return s;
}

/* ------------------------------------------------------------------------- */
/* FT-GCR(k), Algorithm 1.                                                    */
/* ------------------------------------------------------------------------- */

static void flip_bit(double* v, int bit)
{
    uint64_t u;
    memcpy(&u, v, sizeof u);
    u ^= (uint64_t)1 << bit;
    memcpy(v, &u, sizeof u);
}

static void apply_event(const orc_event* ev, double* target)
{
    for (int64_t t = 0; t < ev->count; ++t) {
        int64_t at = ev->idx ? ev->idx[t] : ev->start + t;
        int bit = ev->bits ? (int)ev->bits[t] : (int)ev->bit;
        flip_bit(&target[at], bit);
    }
}

static void copy_vec(int64_t n, const double* src, double* dst) { memcpy(dst, src, sizeof(double) * (size_t)n); }

/* |<a, b>| / (|a| |b|), 0 when either vector is zero. */
static double abs_cos(int64_t n, const double* a, const double* b)
{
    double den = sqrt(orc_dot(n, a, a)) * sqrt(orc_dot(n, b, b));
    return den > 0.0 ? fabs(orc_dot(n, a, b)) / den : 0.0;
}

int orc_solve(const orc_problem* pb, const double* rhs, double* x, double tol,
              int32_t k, int64_t max_steps, int32_t ft,
              const orc_event* events, int32_t n_events, orc_stats* st,
              orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    return orc_solve_traced(pb, rhs, x, tol, k, max_steps, ft, events, n_events, st,
                            log, log_cap, hist, hist_cap, NULL, NULL, 0);
}

/* The operator pair a solver applies, y = A x and e = P^{-1} r over n
 * entries, so one rendering of each solver serves every mesh. */
typedef struct {
    int64_t n;
    void (*apply_A)(const void* ctx, const double* x, double* y);
    void (*apply_pinv)(const void* ctx, const double* r, double* e);
    const void* ctx;
} op_pair;

typedef struct {
    const orc_problem* pb;
    double* w;   /* face weights wx, wy, wz, one allocation */
    const double *wx, *wy, *wz;
} latlon_ctx;

static void latlon_A(const void* c, const double* x, double* y)
{
    const latlon_ctx* q = (const latlon_ctx*)c;
    orc_apply_A(q->pb, q->wx, q->wy, q->wz, x, y);
}

static void latlon_pinv(const void* c, const double* r, double* e)
{
    const latlon_ctx* q = (const latlon_ctx*)c;
    orc_apply_pinv(q->pb, q->wx, q->wy, q->wz, r, e);
}

/* Face weights of a lat-lon problem and the operator pair over them. */
static int latlon_open(const orc_problem* pb, latlon_ctx* q, op_pair* op)
{
    const int64_t n = (int64_t)pb->nx * pb->ny * pb->nz;
    const int64_t nwy = (int64_t)pb->nx * (pb->ny + 1) * pb->nz, nwz = (int64_t)pb->nx * pb->ny * (pb->nz + 1);
    q->pb = pb;
    q->w = (double*)malloc(sizeof(double) * (size_t)(n + nwy + nwz));
    if (!q->w) return -1;
    q->wx = q->w;
    q->wy = q->w + n;
    q->wz = q->w + n + nwy;
    orc_face_weights(pb, q->w, q->w + n, q->w + n + nwy);
    op->n = n;
    op->apply_A = latlon_A;
    op->apply_pinv = latlon_pinv;
    op->ctx = q;
    return 0;
}

static void latlon_close(latlon_ctx* q) { free(q->w); }

static int gcr_core(const op_pair* op, const double* rhs, double* x, double tol,
                    int32_t k, int64_t max_steps, int32_t ft,
                    const orc_event* events, int32_t n_events, orc_stats* st,
                    orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap,
                    double* cos_r_ap, double* cos_ap, int64_t trace_cap)
{
    if (!rhs || !x || !st || k < 1 || !(tol > 0.0) || max_steps < 0) return -1;
    const int64_t n = op->n;
    for (int32_t q = 0; q < n_events; ++q) {
        const orc_event* ev = &events[q];
        if (ev->vec < ORC_V_X || ev->vec > ORC_V_E || ev->count < 0) return -1;
        for (int64_t t = 0; t < ev->count; ++t) {
            int64_t at = ev->idx ? ev->idx[t] : ev->start + t;
            int bit = ev->bits ? (int)ev->bits[t] : (int)ev->bit;
            if (at < 0 || at >= n || bit < 0 || bit > 63) return -1;
        }
    }

    memset(st, 0, sizeof *st);
    /* Working set: x, r, e, L(e), p^0..p^k, L(p^0)..L(p^k), plus the backup
     * [x, r, p^0, L(p^0)]* and the cycle-start copies of x and r. */
    const int nvec = 2 * (k + 1) + 9;
    double* pool = (double*)malloc(sizeof(double) * (size_t)(nvec * n));
    if (!pool) return -1;
    double* r = pool;
    double* e = r + n;
    double* le = e + n;
    double* bx = le + n;   /* backup x   */
    double* br = bx + n;   /* backup r   */
    double* bp = br + n;   /* backup p0  */
    double* bap = bp + n;  /* backup Lp0 */
    double* x0 = bap + n;  /* x at the start of the current pass nu = 0 */
    double* r0 = x0 + n;
    double* pv = r0 + n;               /* p^l  = pv  + l*n */
    double* apv = pv + (int64_t)(k + 1) * n;  /* Lp^l = apv + l*n */
    double* d = (double*)malloc(sizeof(double) * (size_t)(k + 1));
    double* alpha = (double*)malloc(sizeof(double) * (size_t)(k + 1));
    if (!d || !alpha) { free(pool); free(d); free(alpha); return -1; }

    /* Initialisation (first line of Algorithm 1): r = L(x) - R, p^0 = P^{-1} r,
     * and L(p^0), which the first beta needs. */
    const double RR = orc_dot(n, rhs, rhs);
    const double T = tol * tol * RR;
    st->rhs_norm2 = RR;
    op->apply_A(op->ctx, x, r);
    for (int64_t t = 0; t < n; ++t) r[t] = r[t] - rhs[t];
    op->apply_pinv(op->ctx, r, pv);
    op->apply_A(op->ctx, pv, apv);
    double rr_old = orc_dot(n, r, r);

    int status = -1;
    if (rr_old <= T) status = ORC_CONVERGED;

    /* The initial state is the first known-good state. */
    copy_vec(n, x, bx); copy_vec(n, r, br); copy_vec(n, pv, bp); copy_vec(n, apv, bap);
    double b_rr = rr_old;
    int64_t b_accepted = 0;

    int64_t s = 0, accepted = 0;
    int64_t last_rb_pos = -1;   /* logical position of the last rollback      */
    int events_since_rb = 1;    /* an event fired since that rollback          */

    while (status < 0) {
        int restart = 0;
        for (int nu = 0; nu < k && status < 0 && !restart; ++nu) {
            double* p_nu = pv + (int64_t)nu * n;
            double* ap_nu = apv + (int64_t)nu * n;
            if (s >= max_steps) { status = ORC_MAX_STEPS; break; }
            s += 1;
            if (nu == 0) st->cycles += 1;

            /* S1: harness-planned bit flips, before anything reads this step. */
            for (int32_t q = 0; q < n_events; ++q) {
                if (events[q].step != s || events[q].vec == ORC_V_E) continue;
                double* target = events[q].vec == ORC_V_X ? x
                               : events[q].vec == ORC_V_R ? r
                               : events[q].vec == ORC_V_P ? p_nu : ap_nu;
                apply_event(&events[q], target);
                st->events_applied += 1;
                events_since_rb = 1;
            }

            /* S2: beta = -<r, Lp> / <Lp, Lp> (minus sign restored). */
            d[nu] = orc_dot(n, ap_nu, ap_nu);
            if (d[nu] == 0.0) { status = ORC_BREAKDOWN; break; }
            double beta = -orc_dot(n, r, ap_nu) / d[nu];
            if (nu == 0) { copy_vec(n, x, x0); copy_vec(n, r, r0); }

            /* S3: phi += beta p, r += beta L(p), and the new residual norm. */
            for (int64_t t = 0; t < n; ++t) x[t] = x[t] + beta * p_nu[t];
            for (int64_t t = 0; t < n; ++t) r[t] = r[t] + beta * ap_nu[t];
            double rr_new = orc_dot(n, r, r);
            if (hist && s <= hist_cap) hist[s - 1] = rr_new;
            if (s <= trace_cap) {
                if (cos_r_ap) {
                    double worst = 0.0;
                    for (int l = 0; l <= nu; ++l) {
                        double c = abs_cos(n, r, apv + (int64_t)l * n);
                        if (c > worst) worst = c;
                    }
                    cos_r_ap[s - 1] = worst;
                }
                if (cos_ap) cos_ap[s - 1] = 0.0;
            }

            /* S4: exit test first, then the fault test, then the backup. */
            if (rr_new <= T) { accepted += 1; rr_old = rr_new; status = ORC_CONVERGED; break; }
            if (ft && !(rr_new < rr_old)) {
                int64_t pos = accepted + 1;
                int stagnation = (pos == last_rb_pos) && !events_since_rb;
                st->detections += 1;
                if (log && st->log_len < log_cap) {
                    orc_detect* rec = &log[st->log_len++];
                    rec->step = s; rec->nu = nu; rec->action = stagnation ? 1 : 0;
                    rec->rr_old = rr_old; rec->rr_new = rr_new;
                }
                if (!stagnation) {
                    /* Roll back to the last known-good state and redo the pass. */
                    copy_vec(n, bx, x); copy_vec(n, br, r);
                    copy_vec(n, bp, pv); copy_vec(n, bap, apv);
                    rr_old = b_rr;
                    accepted = b_accepted;
                    last_rb_pos = pos;
                    events_since_rb = 0;
                    restart = 1;
                    break;
                }
                st->stagnation_accepts += 1;
            }
            if (ft && nu == 0) {
                copy_vec(n, x0, bx); copy_vec(n, r0, br);
                copy_vec(n, pv, bp); copy_vec(n, apv, bap);
                b_rr = rr_old;
                b_accepted = accepted;
            }
            accepted += 1;
            rr_old = rr_new;

            /* S5: e = P^{-1} r, L(e), alpha_l = -<L(e), Lp^l> / <Lp^l, Lp^l>.
             * Planned flips of the preconditioner output (the paper's injection
             * site, Section 3) land on e before anything reads it. */
            op->apply_pinv(op->ctx, r, e);
            for (int32_t q = 0; q < n_events; ++q) {
                if (events[q].step != s || events[q].vec != ORC_V_E) continue;
                apply_event(&events[q], e);
                st->events_applied += 1;
                events_since_rb = 1;
            }
            op->apply_A(op->ctx, e, le);
            for (int l = 0; l <= nu; ++l)
                alpha[l] = -orc_dot(n, le, apv + (int64_t)l * n) / d[l];

            /* S6: new direction and its image, sums in ascending l. */
            double* p_next = pv + (int64_t)(nu + 1) * n;
            double* ap_next = apv + (int64_t)(nu + 1) * n;
            copy_vec(n, e, p_next);
            copy_vec(n, le, ap_next);
            for (int l = 0; l <= nu; ++l) {
                const double* pl = pv + (int64_t)l * n;
                const double* apl = apv + (int64_t)l * n;
                for (int64_t t = 0; t < n; ++t) p_next[t] = p_next[t] + alpha[l] * pl[t];
                for (int64_t t = 0; t < n; ++t) ap_next[t] = ap_next[t] + alpha[l] * apl[t];
            }
            if (cos_ap && s <= trace_cap) {
                double worst = 0.0;
                for (int l = 0; l <= nu; ++l) {
                    double c = abs_cos(n, ap_next, apv + (int64_t)l * n);
                    if (c > worst) worst = c;
                }
                cos_ap[s - 1] = worst;
            }
        }
        if (status < 0 && !restart) {
            /* End of the k passes: the last direction opens the next cycle. */
            copy_vec(n, pv + (int64_t)k * n, pv);
            copy_vec(n, apv + (int64_t)k * n, apv);
        }
    }

    st->status = status;
    st->steps_executed = s;
    st->steps_accepted = accepted;
    st->steps_wasted = s - accepted;
    st->rr_final = rr_old;
    st->rel_res_recursive = RR > 0.0 ? sqrt(rr_old / RR) : 0.0;
    st->hist_len = s < hist_cap ? s : hist_cap;
    free(pool); free(d); free(alpha);
    return 0;
}

int orc_solve_traced(const orc_problem* pb, const double* rhs, double* x, double tol,
                     int32_t k, int64_t max_steps, int32_t ft,
                     const orc_event* events, int32_t n_events, orc_stats* st,
                     orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap,
                     double* cos_r_ap, double* cos_ap, int64_t trace_cap)
{
    if (!pb || pb->nx < 3 || pb->ny < 1 || pb->nz < 1) return -1;
    latlon_ctx q;
    op_pair op;
    if (latlon_open(pb, &q, &op) != 0) return -1;
    const int rc = gcr_core(&op, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap, hist,
                            hist_cap, cos_r_ap, cos_ap, trace_cap);
    latlon_close(&q);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* FT-GMRES(k): the same fault-tolerance layer on restarted GMRES.            */
/* ------------------------------------------------------------------------- */
/*
 * The paper presents its detector as compatible with other Krylov solvers
 * (abstract; Section 1 contrasts it with FT-GMRES, which bounds Hessenberg
 * entries instead).  Here the residual-norm test, the backup of a known-good
 * state after each complete Krylov cycle and the rollback of Algorithm 1
 * (red part) wrap right-preconditioned restarted GMRES(k):
 *
 *   cycle:  s = R - A x, rho = |s|, v_0 = s / rho, g = (rho, 0, ...)
 *     step j = 0..k-1:  z_j = P^{-1} v_j;  w = A z_j;
 *                       h_ij = <w, v_i> (i <= j, classical Gram-Schmidt);
 *                       w -= sum_i h_ij v_i (ascending i);  h_{j+1,j} = |w|;
 *                       rotate column j by the earlier Givens rotations, form
 *                       the rotation that zeroes h_{j+1,j}, apply it to g;
 *                       the step's residual norm is |g_{j+1}| (the norm of
 *                       R - A (x + sum y_i z_i) minimised over the cycle);
 *                       exit test, then fault test !(g_{j+1}^2 < g_j^2);
 *                       v_{j+1} = w / h_{j+1,j}
 *     end:   y = H^{-1} g (upper triangular, the steps done), x += sum y_i z_i
 *            (ascending i), then the explicit residual s = R - A x: exit if
 *            |s|^2 <= tol^2 |R|^2, fault if !(|s|^2 < the cycle start's),
 *            else the new backup [x, |s|^2].
 *
 * A fault test that fires inside a cycle or at its end restores x and |s|^2
 * from the backup and restarts the cycle from the residual of the restored x
 * (inside a cycle x is not yet changed, so only the Krylov basis is lost).
 * The stagnation rule is that of FT-GCR: a detection at the same place after
 * a rollback with no fault event since is accepted.  Places are numbered
 * 2 (accepted + 1) for a step and 2 accepted + 1 for a cycle-end check.
 * Fault events: X flips x at the start of the step, R flips v_j at the start
 * of the step (before P^{-1} reads it), P and E flip z_j = P^{-1} v_j right
 * after the preconditioner, AP flips w = A z_j before the inner products.
 * The residual history holds g_{j+1}^2 per executed step; a cycle-end
 * detection is logged with nu = -1 and the explicit squared norms.
 */

static void residual_RAx(const op_pair* op, const double* rhs, const double* x, double* s, int64_t n)
{
    op->apply_A(op->ctx, x, s);
    for (int64_t t = 0; t < n; ++t) s[t] = rhs[t] - s[t];
}

static void log_detection(orc_stats* st, orc_detect* log, int32_t log_cap, int64_t step, int nu, int action,
                          double rr_old, double rr_new)
{
    st->detections += 1;
    if (log && st->log_len < log_cap) {
        orc_detect* rec = &log[st->log_len++];
        rec->step = step; rec->nu = nu; rec->action = action;
        rec->rr_old = rr_old; rec->rr_new = rr_new;
    }
}

static void apply_events_at(const orc_event* events, int32_t n_events, int64_t step, int vec_a, int vec_b,
                            double* target, orc_stats* st, int* events_since_rb)
{
    for (int32_t q = 0; q < n_events; ++q) {
        if (events[q].step != step || (events[q].vec != vec_a && events[q].vec != vec_b)) continue;
        apply_event(&events[q], target);
        st->events_applied += 1;
        *events_since_rb = 1;
    }
}

static int gmres_core(const op_pair* op, const double* rhs, double* x, double tol,
                      int32_t k, int64_t max_steps, int32_t ft,
                      const orc_event* events, int32_t n_events, orc_stats* st,
                      orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    if (!rhs || !x || !st || k < 1 || !(tol > 0.0) || max_steps < 0) return -1;
    const int64_t n = op->n;
    for (int32_t q = 0; q < n_events; ++q) {
        const orc_event* ev = &events[q];
        if (ev->vec < ORC_V_X || ev->vec > ORC_V_E || ev->count < 0) return -1;
        for (int64_t t = 0; t < ev->count; ++t) {
            int64_t at = ev->idx ? ev->idx[t] : ev->start + t;
            int bit = ev->bits ? (int)ev->bits[t] : (int)ev->bit;
            if (at < 0 || at >= n || bit < 0 || bit > 63) return -1;
        }
    }
    memset(st, 0, sizeof *st);
    /* s, w, the backup of x, v_0..v_k, z_0..z_{k-1} */
    const int64_t nvec = 3 + (k + 1) + k;
    double* pool = (double*)malloc(sizeof(double) * (size_t)(nvec * n));
    double* hh = (double*)calloc((size_t)(k + 1) * k, sizeof(double));   /* H[i][j] = hh[i*k + j] */
    double* cs = (double*)calloc((size_t)k, sizeof(double));
    double* sn = (double*)calloc((size_t)k, sizeof(double));
    double* g = (double*)calloc((size_t)k + 1, sizeof(double));
    double* y = (double*)calloc((size_t)k, sizeof(double));
    if (!pool || !hh || !cs || !sn || !g || !y) {
        free(pool); free(hh); free(cs); free(sn); free(g); free(y);
        return -1;
    }
    double* s = pool;
    double* w = s + n;
    double* xb = w + n;
    double* V = xb + n;                  /* v_i = V + i*n, i = 0..k  */
    double* Z = V + (int64_t)(k + 1) * n; /* z_i = Z + i*n, i < k    */

    const double RR = orc_dot(n, rhs, rhs);
    const double T = tol * tol * RR;
    st->rhs_norm2 = RR;
    residual_RAx(op, rhs, x, s, n);
    double rho2 = orc_dot(n, s, s);
    int status = -1;
    if (rho2 <= T) status = ORC_CONVERGED;
    /* the initial state is the first known-good state */
    copy_vec(n, x, xb);
    double b_rho2 = rho2;
    int64_t b_accepted = 0;
    int64_t sx = 0, accepted = 0;
    int64_t last_rb_pos = -1;
    int events_since_rb = 1;

    while (status < 0) {
        /* a new cycle from the residual s of x */
        const double rho = sqrt(rho2);
        for (int64_t t = 0; t < n; ++t) V[t] = s[t] / rho;
        for (int i = 0; i <= k; ++i) g[i] = 0.0;
        g[0] = rho;
        double rr_old = rho2;
        int jdone = 0, rolled = 0, capped = 0;
        for (int j = 0; j < k; ++j) {
            double* vj = V + (int64_t)j * n;
            double* zj = Z + (int64_t)j * n;
            if (sx >= max_steps) { capped = 1; break; }
            sx += 1;
            if (j == 0) st->cycles += 1;
            apply_events_at(events, n_events, sx, ORC_V_X, ORC_V_X, x, st, &events_since_rb);
            apply_events_at(events, n_events, sx, ORC_V_R, ORC_V_R, vj, st, &events_since_rb);
            op->apply_pinv(op->ctx, vj, zj);
            apply_events_at(events, n_events, sx, ORC_V_P, ORC_V_E, zj, st, &events_since_rb);
            op->apply_A(op->ctx, zj, w);
            apply_events_at(events, n_events, sx, ORC_V_AP, ORC_V_AP, w, st, &events_since_rb);
            for (int i = 0; i <= j; ++i) hh[i * k + j] = orc_dot(n, w, V + (int64_t)i * n);
            for (int i = 0; i <= j; ++i) {
                const double* vi = V + (int64_t)i * n;
                const double hij = hh[i * k + j];
                for (int64_t t = 0; t < n; ++t) w[t] = w[t] - hij * vi[t];
            }
            const double hn = sqrt(orc_dot(n, w, w));
            hh[(j + 1) * k + j] = hn;
            /* earlier rotations on column j, then the new one */
            for (int i = 0; i < j; ++i) {
                const double a = hh[i * k + j], b = hh[(i + 1) * k + j];
                hh[i * k + j] = cs[i] * a + sn[i] * b;
                hh[(i + 1) * k + j] = -sn[i] * a + cs[i] * b;
            }
            {
                const double a = hh[j * k + j], b = hh[(j + 1) * k + j];
                const double den = sqrt(a * a + b * b);
                cs[j] = a / den;
                sn[j] = b / den;
                hh[j * k + j] = den;
                hh[(j + 1) * k + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
            }
            const double rr_new = g[j + 1] * g[j + 1];
            if (hist && sx <= hist_cap) hist[sx - 1] = rr_new;
            jdone = j + 1;
            /* exit test first, then the fault test */
            if (rr_new <= T) { accepted += 1; rr_old = rr_new; break; }
            if (ft && !(rr_new < rr_old)) {
                const int64_t pos = 2 * (accepted + 1);
                const int stag = (pos == last_rb_pos) && !events_since_rb;
                log_detection(st, log, log_cap, sx, j, stag, rr_old, rr_new);
                if (!stag) {
                    copy_vec(n, xb, x);
                    accepted = b_accepted;
                    last_rb_pos = pos;
                    events_since_rb = 0;
                    rolled = 1;
                    break;
                }
                st->stagnation_accepts += 1;
            }
            accepted += 1;
            rr_old = rr_new;
            if (hn == 0.0) break;   /* the cycle's space holds the solution */
            double* vn = V + (int64_t)(j + 1) * n;
            for (int64_t t = 0; t < n; ++t) vn[t] = w[t] / hn;
        }
        if (rolled) {
            residual_RAx(op, rhs, x, s, n);
            rho2 = orc_dot(n, s, s);
            continue;
        }
        /* the cycle's correction: H y = g over the steps done, x += sum y_i z_i */
        for (int i = jdone - 1; i >= 0; --i) {
            double acc = g[i];
            for (int l = i + 1; l < jdone; ++l) acc = acc - hh[i * k + l] * y[l];
            y[i] = acc / hh[i * k + i];
        }
        for (int i = 0; i < jdone; ++i) {
            const double* zi = Z + (int64_t)i * n;
            for (int64_t t = 0; t < n; ++t) x[t] = x[t] + y[i] * zi[t];
        }
        residual_RAx(op, rhs, x, s, n);
        const double rho2_new = orc_dot(n, s, s);
        if (capped || (sx >= max_steps && rho2_new > T)) {
            rho2 = rho2_new;
            status = ORC_MAX_STEPS;
            break;
        }
        if (rho2_new <= T) { rho2 = rho2_new; status = ORC_CONVERGED; break; }
        if (ft && !(rho2_new < b_rho2)) {
            const int64_t pos = 2 * accepted + 1;
            const int stag = (pos == last_rb_pos) && !events_since_rb;
            log_detection(st, log, log_cap, sx, -1, stag, b_rho2, rho2_new);
            if (!stag) {
                copy_vec(n, xb, x);
                accepted = b_accepted;
                last_rb_pos = pos;
                events_since_rb = 0;
                residual_RAx(op, rhs, x, s, n);
                rho2 = orc_dot(n, s, s);
                continue;
            }
            st->stagnation_accepts += 1;
        }
        /* the cycle passed: its output is the new known-good state */
        if (ft) {
            copy_vec(n, x, xb);
            b_rho2 = rho2_new;
            b_accepted = accepted;
        }
        rho2 = rho2_new;
    }
    st->status = status;
    st->steps_executed = sx;
    st->steps_accepted = accepted;
    st->steps_wasted = sx - accepted;
    st->rr_final = rho2;
    st->rel_res_recursive = RR > 0.0 ? sqrt(rho2 / RR) : 0.0;
    st->hist_len = sx < hist_cap ? sx : hist_cap;
    free(pool); free(hh); free(cs); free(sn); free(g); free(y);
    return 0;
}

int orc_gmres_solve(const orc_problem* pb, const double* rhs, double* x, double tol,
                    int32_t k, int64_t max_steps, int32_t ft,
                    const orc_event* events, int32_t n_events, orc_stats* st,
                    orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    if (!pb || pb->nx < 3 || pb->ny < 1 || pb->nz < 1) return -1;
    latlon_ctx q;
    op_pair op;
    if (latlon_open(pb, &q, &op) != 0) return -1;
    const int rc = gmres_core(&op, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap, hist, hist_cap);
    latlon_close(&q);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Octahedral reduced Gaussian grid O_N (Section 3, Table 1)                  */
/* ------------------------------------------------------------------------- */
/*
 * 2N latitude rings; the i-th ring from either pole (i = 1..N) holds 4i + 16
 * points, 4N(N+9) per level (Table 1).  Ring latitudes are the Gaussian
 * latitudes: their sines are the roots of the Legendre polynomial P_{2N}.
 * Point m of a ring of n points sits at longitude 2 pi m / n.  Rings are
 * numbered from the south pole; flat index = (first point of the ring + m)
 * + points * k.
 *
 * Node-centred finite volumes on the triangulated mesh: the points are the
 * vertices of the polyhedron inscribed in the unit sphere whose triangles
 * join neighbouring rings ("zipper": walking both rings eastward from
 * longitude 0, the ring whose next point comes first -- the lower ring on a
 * tie -- adds a triangle); the polar caps stay open (no flux through the
 * poles).  A point's control area is its circumcentric (Voronoi) region,
 * A_a = (1/4) sum_b W_ab |x_a - x_b|^2, and the face between the control
 * volumes of the ends of an edge (a, b) is orthogonal to it, with length
 * over edge length W_ab = (cot alpha + cot beta) / 2 (the angles opposite
 * the edge in its one or two triangles).  Weights, c at the face centre as
 * on the lat-lon grid (an edge's centre: its chord's midpoint projected
 * back onto the sphere):
 *   horizontal   c dz W_ab
 *   vertical     c A_a / dz between levels, none at bottom and top.
 * A = A0 + sigma diag(A0) as on the lat-lon grid; P is again the vertical
 * tridiagonal part of A.
 */

int64_t orc_oct_cells(int32_t N) { return 4LL * N * (N + 9); }

int32_t orc_oct_ring_points(int32_t N, int32_t j)
{
    const int32_t i = j < N ? j + 1 : 2 * N - j;   /* ring index from the nearer pole */
    return 4 * i + 16;
}

/* Legendre polynomial P_n(x) and its derivative, by the three-term recurrence. */
static void legendre(int n, double x, double* p, double* dp)
{
    double p0 = 1.0, p1 = x;
    for (int l = 2; l <= n; ++l) {
        const double p2 = ((2.0 * l - 1.0) * x * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void orc_oct_gauss(int32_t N, double* mu, double* w)
{
    const int n = 2 * N;
    for (int l = 0; l < n; ++l) {
        /* Newton from the usual first guess for the l-th root (descending) */
        double x = cos(M_PI * (l + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, x, &p, &dp);
            const double dx = p / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p, dp;
        legendre(n, x, &p, &dp);
        mu[n - 1 - l] = x;                          /* ascending: south to north */
        w[n - 1 - l] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

typedef struct {
    const orc_oct_problem* pb;
    int32_t nring;
    int64_t ncell;
    int32_t* npts;        /* points per ring                              */
    int64_t* first;       /* first point of each ring                     */
    double *lon, *lat;    /* per point                                    */
    double *px, *py, *pz; /* per point, on the unit sphere                */
    double* area;         /* Voronoi control area per point               */
    double* hcell;        /* hill height at each point                    */
    int64_t nedge, cap;
    int64_t *ea, *eb;     /* edge ends                                    */
    int64_t* inc;         /* incident edges of every point, OCT_INC each  */
    int32_t* ninc;
    double* ew;           /* (cot alpha + cot beta) / 2                   */
    double* eh;           /* hill height at the edge's centre             */
} oct_mesh;

static double oct_hill(const orc_oct_problem* pb, double lon, double lat)
{
    orc_problem q;
    memset(&q, 0, sizeof q);
    q.hill_lon = pb->hill_lon;
    q.hill_lat = pb->hill_lat;
    q.hill_width = pb->hill_width;
    return orc_hill(&q, lon, lat);
}

enum { OCT_INC = 16 };   /* room for incident edges per point (the mesh has at most 6) */

static void oct_mesh_free(oct_mesh* m)
{
    free(m->npts); free(m->first); free(m->lon); free(m->lat); free(m->px); free(m->py); free(m->pz);
    free(m->area); free(m->hcell); free(m->ea); free(m->eb); free(m->ew); free(m->eh);
    free(m->inc); free(m->ninc);
}

/* Index of edge (a, b), added if new (a search of a's incident edges). */
static int64_t oct_edge(oct_mesh* m, int64_t a, int64_t b)
{
    for (int32_t q = 0; q < m->ninc[a]; ++q) {
        const int64_t e = m->inc[a * OCT_INC + q];
        if ((m->ea[e] == a && m->eb[e] == b) || (m->ea[e] == b && m->eb[e] == a)) return e;
    }
    if (m->ninc[a] == OCT_INC || m->ninc[b] == OCT_INC) return -1;
    if (m->nedge == m->cap) {
        m->cap = m->cap ? 2 * m->cap : 1024;
        int64_t* ea = (int64_t*)realloc(m->ea, sizeof(int64_t) * (size_t)m->cap);
        if (ea) m->ea = ea;
        int64_t* eb = (int64_t*)realloc(m->eb, sizeof(int64_t) * (size_t)m->cap);
        if (eb) m->eb = eb;
        double* ew = (double*)realloc(m->ew, sizeof(double) * (size_t)m->cap);
        if (ew) m->ew = ew;
        if (!ea || !eb || !ew) return -1;
    }
    m->ea[m->nedge] = a;
    m->eb[m->nedge] = b;
    m->ew[m->nedge] = 0.0;
    m->inc[a * OCT_INC + m->ninc[a]++] = m->nedge;
    m->inc[b * OCT_INC + m->ninc[b]++] = m->nedge;
    return m->nedge++;
}

/* cot of the angle at p0 between the chords to p1 and p2 */
static double oct_cot(const oct_mesh* m, int64_t p0, int64_t p1, int64_t p2)
{
    const double ux = m->px[p1] - m->px[p0], uy = m->py[p1] - m->py[p0], uz = m->pz[p1] - m->pz[p0];
    const double vx = m->px[p2] - m->px[p0], vy = m->py[p2] - m->py[p0], vz = m->pz[p2] - m->pz[p0];
    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    return (ux * vx + uy * vy + uz * vz) / sqrt(cx * cx + cy * cy + cz * cz);
}

/* A triangle's contribution: half the cotangent of each angle to the
 * weight of the opposite edge. */
static int oct_triangle(oct_mesh* m, int64_t a, int64_t b, int64_t c)
{
    const int64_t t[3] = {a, b, c};
    for (int r = 0; r < 3; ++r) {
        const int64_t p0 = t[r], p1 = t[(r + 1) % 3], p2 = t[(r + 2) % 3];
        const int64_t e = oct_edge(m, p1, p2);
        if (e < 0) return -1;
        m->ew[e] += 0.5 * oct_cot(m, p0, p1, p2);
    }
    return 0;
}

static int oct_mesh_build(const orc_oct_problem* pb, oct_mesh* m)
{
    memset(m, 0, sizeof *m);
    m->pb = pb;
    const int32_t N = pb->N, nr = 2 * N;
    const int64_t nc = orc_oct_cells(N);
    m->nring = nr;
    m->ncell = nc;
    m->npts = (int32_t*)malloc(sizeof(int32_t) * nr);
    m->first = (int64_t*)malloc(sizeof(int64_t) * nr);
    m->lon = (double*)malloc(sizeof(double) * (size_t)nc);
    m->lat = (double*)malloc(sizeof(double) * (size_t)nc);
    m->px = (double*)malloc(sizeof(double) * (size_t)nc);
    m->py = (double*)malloc(sizeof(double) * (size_t)nc);
    m->pz = (double*)malloc(sizeof(double) * (size_t)nc);
    m->area = (double*)calloc((size_t)nc, sizeof(double));
    m->hcell = (double*)malloc(sizeof(double) * (size_t)nc);
    m->inc = (int64_t*)malloc(sizeof(int64_t) * (size_t)nc * OCT_INC);
    m->ninc = (int32_t*)calloc((size_t)nc, sizeof(int32_t));
    double* mu = (double*)malloc(sizeof(double) * nr);
    double* wg = (double*)malloc(sizeof(double) * nr);
    if (!m->npts || !m->first || !m->lon || !m->lat || !m->px || !m->py || !m->pz || !m->area || !m->hcell ||
        !m->inc || !m->ninc || !mu || !wg) {
        free(mu); free(wg); oct_mesh_free(m);
        return -1;
    }
    orc_oct_gauss(N, mu, wg);
    int64_t off = 0;
    for (int j = 0; j < nr; ++j) {
        m->npts[j] = orc_oct_ring_points(N, j);
        m->first[j] = off;
        const double lat = asin(mu[j]);
        for (int q = 0; q < m->npts[j]; ++q) {
            const int64_t c = off + q;
            m->lat[c] = lat;
            m->lon[c] = 2.0 * M_PI * q / m->npts[j];
            m->px[c] = cos(lat) * cos(m->lon[c]);
            m->py[c] = cos(lat) * sin(m->lon[c]);
            m->pz[c] = sin(lat);
            m->hcell[c] = oct_hill(pb, m->lon[c], lat);
        }
        off += m->npts[j];
    }
    free(mu); free(wg);
    /* the triangles between each pair of neighbouring rings */
    for (int j = 0; j + 1 < nr; ++j) {
        const int64_t n = m->npts[j], n2 = m->npts[j + 1];
        const int64_t f1 = m->first[j], f2 = m->first[j + 1];
        int64_t a = 0, b = 0;
        while (a < n || b < n2) {
            int rc;
            /* point a+1 of ring j comes no later than point b+1 of ring j+1:
             * (a+1)/n <= (b+1)/n2, compared exactly in integers */
            if (a < n && (b >= n2 || (a + 1) * n2 <= (b + 1) * n)) {
                rc = oct_triangle(m, f1 + a % n, f1 + (a + 1) % n, f2 + b % n2);
                a += 1;
            } else {
                rc = oct_triangle(m, f1 + a % n, f2 + b % n2, f2 + (b + 1) % n2);
                b += 1;
            }
            if (rc != 0) { oct_mesh_free(m); return -1; }
        }
    }
    /* Voronoi areas and the hill at every edge's centre */
    m->eh = (double*)malloc(sizeof(double) * (size_t)(m->nedge ? m->nedge : 1));
    if (!m->eh) { oct_mesh_free(m); return -1; }
    for (int64_t e = 0; e < m->nedge; ++e) {
        const int64_t a = m->ea[e], b = m->eb[e];
        const double dx = m->px[a] - m->px[b], dy = m->py[a] - m->py[b], dz = m->pz[a] - m->pz[b];
        const double q = 0.25 * m->ew[e] * (dx * dx + dy * dy + dz * dz);
        m->area[a] += q;
        m->area[b] += q;
        const double mx = m->px[a] + m->px[b], my = m->py[a] + m->py[b], mz = m->pz[a] + m->pz[b];
        const double r = sqrt(mx * mx + my * my + mz * mz);
        m->eh[e] = oct_hill(pb, atan2(my, mx), asin(mz / r));
    }
    return 0;
}

/* The diagonal (1 + sigma) * (sum of the point's face weights) at every point
 * and level, into d (points * nz), and the vertical weights below each level
 * into wzb (points * (nz + 1)). */
static void oct_weights(const oct_mesh* m, double* d, double* wzb)
{
    const orc_oct_problem* pb = m->pb;
    const int64_t nc = m->ncell;
    const double dz = pb->shell_depth / pb->nz;
    for (int k = 0; k <= pb->nz; ++k)
        for (int64_t c = 0; c < nc; ++c) {
            double w = 0.0;
            if (k > 0 && k < pb->nz) {
                const double cc = 1.0 + pb->hill_amp * m->hcell[c] * exp(-((double)k / pb->nz) / pb->decay_z);
                w = cc * m->area[c] / dz;
            }
            wzb[c + nc * k] = w;
        }
    for (int k = 0; k < pb->nz; ++k) {
        const double gk = exp(-((k + 0.5) / pb->nz) / pb->decay_z);
        double* dk = d + nc * k;
        for (int64_t c = 0; c < nc; ++c) dk[c] = 0.0;
        for (int64_t e = 0; e < m->nedge; ++e) {
            const double w = (1.0 + pb->hill_amp * m->eh[e] * gk) * dz * m->ew[e];
            dk[m->ea[e]] += w;
            dk[m->eb[e]] += w;
        }
        for (int64_t c = 0; c < nc; ++c) dk[c] = (1.0 + pb->helmholtz) * (dk[c] + wzb[c + nc * k] + wzb[c + nc * (k + 1)]);
    }
}

typedef struct {
    oct_mesh m;
    double* d;
    double* wzb;
} oct_ctx;

static void oct_A(const void* cx, const double* x, double* y)
{
    const oct_ctx* q = (const oct_ctx*)cx;
    const oct_mesh* m = &q->m;
    const orc_oct_problem* pb = m->pb;
    const int64_t nc = m->ncell;
    const double dz = pb->shell_depth / pb->nz;
    const int par = nc * pb->nz >= ORC_PAR_MIN;
    (void)par;
    ORC_OMP(omp parallel if(par))
    {
    double* off = (double*)malloc(sizeof(double) * (size_t)nc);
    ORC_OMP(omp for schedule(static))
    for (int k = 0; k < pb->nz; ++k) {
        const double gk = exp(-((k + 0.5) / pb->nz) / pb->decay_z);
        const double* xk = x + nc * k;
        for (int64_t c = 0; c < nc; ++c) off[c] = 0.0;
        for (int64_t e = 0; e < m->nedge; ++e) {
            const double w = (1.0 + pb->hill_amp * m->eh[e] * gk) * dz * m->ew[e];
            off[m->ea[e]] += w * xk[m->eb[e]];
            off[m->eb[e]] += w * xk[m->ea[e]];
        }
        for (int64_t c = 0; c < nc; ++c) {
            double o = off[c];
            if (k > 0) o += q->wzb[c + nc * k] * x[c + nc * (k - 1)];
            if (k < pb->nz - 1) o += q->wzb[c + nc * (k + 1)] * x[c + nc * (k + 1)];
            y[c + nc * k] = q->d[c + nc * k] * xk[c] - o;
        }
    }
    free(off);
    }
}

static void oct_pinv(const void* cx, const double* r, double* e)
{
    const oct_ctx* q = (const oct_ctx*)cx;
    const int64_t nc = q->m.ncell;
    const int nz = q->m.pb->nz;
    const int par = nc * nz >= ORC_PAR_MIN;
    (void)par;
    ORC_OMP(omp parallel if(par))
    {
    double* gam = (double*)malloc(sizeof(double) * nz);
    double* del = (double*)malloc(sizeof(double) * nz);
    ORC_OMP(omp for schedule(static))
    for (int64_t c = 0; c < nc; ++c) {
        /* a_k e_{k-1} + b_k e_k + u_k e_{k+1} = r_k: b the diagonal of A, a and u
         * minus the vertical face weights */
        for (int k = 0; k < nz; ++k) {
            const double b = q->d[c + nc * k];
            const double a = -q->wzb[c + nc * k];
            const double u = -q->wzb[c + nc * (k + 1)];
            const double rk = r[c + nc * k];
            if (k == 0) {
                gam[0] = u / b;
                del[0] = rk / b;
            } else {
                const double mk = b - a * gam[k - 1];
                gam[k] = u / mk;
                del[k] = (rk - a * del[k - 1]) / mk;
            }
        }
        e[c + nc * (nz - 1)] = del[nz - 1];
        for (int k = nz - 2; k >= 0; --k) e[c + nc * k] = del[k] - gam[k] * e[c + nc * (k + 1)];
    }
    free(gam);
    free(del);
    }
}

static void oct_close(oct_ctx* q)
{
    oct_mesh_free(&q->m);
    free(q->d);
    free(q->wzb);
}

static int oct_open(const orc_oct_problem* pb, oct_ctx* q, op_pair* op)
{
    memset(q, 0, sizeof *q);
    if (!pb || pb->N < 1 || pb->nz < 1) return -1;
    if (oct_mesh_build(pb, &q->m) != 0) return -1;
    const int64_t nc = q->m.ncell;
    q->d = (double*)malloc(sizeof(double) * (size_t)(nc * pb->nz));
    q->wzb = (double*)malloc(sizeof(double) * (size_t)(nc * (pb->nz + 1)));
    if (!q->d || !q->wzb) {
        oct_close(q);
        return -1;
    }
    oct_weights(&q->m, q->d, q->wzb);
    op->n = nc * pb->nz;
    op->apply_A = oct_A;
    op->apply_pinv = oct_pinv;
    op->ctx = q;
    return 0;
}

int orc_oct_apply_A(const orc_oct_problem* pb, const double* x, double* y)
{
    oct_ctx q;
    op_pair op;
    if (oct_open(pb, &q, &op) != 0) return -1;
    op.apply_A(op.ctx, x, y);
    oct_close(&q);
    return 0;
}

int orc_oct_apply_pinv(const orc_oct_problem* pb, const double* r, double* e)
{
    oct_ctx q;
    op_pair op;
    if (oct_open(pb, &q, &op) != 0) return -1;
    op.apply_pinv(op.ctx, r, e);
    oct_close(&q);
    return 0;
}

int orc_oct_mesh(const orc_oct_problem* pb, double* lon, double* lat, double* area, int64_t* nedge)
{
    oct_mesh m;
    if (!pb || pb->N < 1 || oct_mesh_build(pb, &m) != 0) return -1;
    for (int64_t c = 0; c < m.ncell; ++c) {
        lon[c] = m.lon[c];
        lat[c] = m.lat[c];
        area[c] = m.area[c];
    }
    *nedge = m.nedge;
    oct_mesh_free(&m);
    return 0;
}

/* e = r on the O_N mesh: no preconditioner */
static void oct_identity(const void* cx, const double* r, double* e)
{
    const oct_ctx* q = (const oct_ctx*)cx;
    copy_vec(q->m.ncell * q->m.pb->nz, r, e);
}

int orc_oct_solve(const orc_oct_problem* pb, const double* rhs, double* x, double tol,
                  int32_t k, int64_t max_steps, int32_t ft, int32_t method,
                  const orc_event* events, int32_t n_events, orc_stats* st,
                  orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    return orc_oct_solve_pc(pb, 1, method, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap,
                            hist, hist_cap);
}

int orc_oct_solve_pc(const orc_oct_problem* pb, int32_t precond, int32_t method, const double* rhs, double* x,
                     double tol, int32_t k, int64_t max_steps, int32_t ft,
                     const orc_event* events, int32_t n_events, orc_stats* st,
                     orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    if (precond != 0 && precond != 1) return -1;
    oct_ctx q;
    op_pair op;
    if (oct_open(pb, &q, &op) != 0) return -1;
    if (precond == 0) op.apply_pinv = oct_identity;
    const int rc = method == 1
        ? gmres_core(&op, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap, hist, hist_cap)
        : gcr_core(&op, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap, hist, hist_cap,
                   NULL, NULL, 0);
    oct_close(&q);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Solves with a chosen preconditioner: the column one, or none (P = I).      */
/* ------------------------------------------------------------------------- */

typedef struct {
    latlon_ctx q;
    int64_t n;
} latlon_id_ctx;

static void latlon_A_id(const void* c, const double* x, double* y)
{
    const latlon_id_ctx* q = (const latlon_id_ctx*)c;
    orc_apply_A(q->q.pb, q->q.wx, q->q.wy, q->q.wz, x, y);
}

/* e = r: no preconditioner */
static void identity_pinv(const void* c, const double* r, double* e)
{
    const latlon_id_ctx* q = (const latlon_id_ctx*)c;
    copy_vec(q->n, r, e);
}

int orc_solve_pc(const orc_problem* pb, int32_t precond, int32_t method, const double* rhs, double* x,
                 double tol, int32_t k, int64_t max_steps, int32_t ft,
                 const orc_event* events, int32_t n_events, orc_stats* st,
                 orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    if (!pb || pb->nx < 3 || pb->ny < 1 || pb->nz < 1 || (precond != 0 && precond != 1)) return -1;
    latlon_id_ctx c;
    op_pair op;
    if (latlon_open(pb, &c.q, &op) != 0) return -1;
    c.n = op.n;
    if (precond == 0) {
        op.apply_A = latlon_A_id;
        op.apply_pinv = identity_pinv;
        op.ctx = &c;
    }
    const int rc = method == 1
        ? gmres_core(&op, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap, hist, hist_cap)
        : gcr_core(&op, rhs, x, tol, k, max_steps, ft, events, n_events, st, log, log_cap, hist, hist_cap,
                   NULL, NULL, 0);
    latlon_close(&c.q);
    return rc;
}
