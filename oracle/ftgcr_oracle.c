/*
 * FT-GCR reference oracle -- TEST INFRASTRUCTURE ONLY (see ftgcr_oracle.h).
 *
 * Plain, serial FP64 C, written to be checked by eye against the paper
 * (Gillard & Benacchio, arXiv 2103.07210) and the frozen operator readings.
 * No blocking, fusion or reordering: every step of Algorithm 1 is a separate
 * whole-vector pass, every inner product is a left-to-right sum.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fPIC -shared -lm
 */
#include "ftgcr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

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

    /* Longitude faces: flux c * (1/cos(lat)) d/dlon over a face of area
     * dlat*dz, difference over dlon. */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double c = coeff_c(pb, lon_face_east(pb, i), lat_centre(pb, j), zeta_centre(pb, k));
                wx[((int64_t)k * ny + j) * nx + i] = c * dlat * dz / (cos(lat_centre(pb, j)) * dlon);
            }

    /* Latitude faces: flux c d/dlat over a face of area cos(lat_face)*dlon*dz;
     * zero flux through the two polar faces. */
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
    double* gam = (double*)malloc(sizeof(double) * nz);
    double* del = (double*)malloc(sizeof(double) * nz);
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

int orc_solve_traced(const orc_problem* pb, const double* rhs, double* x, double tol,
                     int32_t k, int64_t max_steps, int32_t ft,
                     const orc_event* events, int32_t n_events, orc_stats* st,
                     orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap,
                     double* cos_r_ap, double* cos_ap, int64_t trace_cap)
{
    if (!pb || !rhs || !x || !st || k < 1 || !(tol > 0.0) || max_steps < 0) return -1;
    if (pb->nx < 3 || pb->ny < 1 || pb->nz < 1) return -1;
    const int64_t n = (int64_t)pb->nx * pb->ny * pb->nz;
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
    const int64_t nwx = n, nwy = (int64_t)pb->nx * (pb->ny + 1) * pb->nz,
                  nwz = (int64_t)pb->nx * pb->ny * (pb->nz + 1);
    /* Working set: x, r, e, L(e), p^0..p^k, L(p^0)..L(p^k), plus the backup
     * [x, r, p^0, L(p^0)]* and the cycle-start copies of x and r. */
    const int nvec = 2 * (k + 1) + 9;
    double* pool = (double*)malloc(sizeof(double) * (size_t)(nwx + nwy + nwz + nvec * n));
    if (!pool) return -1;
    double* wx = pool;
    double* wy = wx + nwx;
    double* wz = wy + nwy;
    double* r = wz + nwz;
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

    orc_face_weights(pb, wx, wy, wz);

    /* Initialisation (first line of Algorithm 1): r = L(x) - R, p^0 = P^{-1} r,
     * and L(p^0), which the first beta needs. */
    const double RR = orc_dot(n, rhs, rhs);
    const double T = tol * tol * RR;
    st->rhs_norm2 = RR;
    orc_apply_A(pb, wx, wy, wz, x, r);
    for (int64_t t = 0; t < n; ++t) r[t] = r[t] - rhs[t];
    orc_apply_pinv(pb, wx, wy, wz, r, pv);
    orc_apply_A(pb, wx, wy, wz, pv, apv);
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
            orc_apply_pinv(pb, wx, wy, wz, r, e);
            for (int32_t q = 0; q < n_events; ++q) {
                if (events[q].step != s || events[q].vec != ORC_V_E) continue;
                apply_event(&events[q], e);
                st->events_applied += 1;
                events_since_rb = 1;
            }
            orc_apply_A(pb, wx, wy, wz, e, le);
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

static void residual_RAx(const orc_problem* pb, const double* wx, const double* wy, const double* wz,
                         const double* rhs, const double* x, double* s, int64_t n)
{
    orc_apply_A(pb, wx, wy, wz, x, s);
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

int orc_gmres_solve(const orc_problem* pb, const double* rhs, double* x, double tol,
                    int32_t k, int64_t max_steps, int32_t ft,
                    const orc_event* events, int32_t n_events, orc_stats* st,
                    orc_detect* log, int32_t log_cap, double* hist, int64_t hist_cap)
{
    if (!pb || !rhs || !x || !st || k < 1 || !(tol > 0.0) || max_steps < 0) return -1;
    if (pb->nx < 3 || pb->ny < 1 || pb->nz < 1) return -1;
    const int64_t n = (int64_t)pb->nx * pb->ny * pb->nz;
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
    const int64_t nwx = n, nwy = (int64_t)pb->nx * (pb->ny + 1) * pb->nz,
                  nwz = (int64_t)pb->nx * pb->ny * (pb->nz + 1);
    /* s, w, the backup of x, v_0..v_k, z_0..z_{k-1} */
    const int64_t nvec = 3 + (k + 1) + k;
    double* pool = (double*)malloc(sizeof(double) * (size_t)(nwx + nwy + nwz + nvec * n));
    double* hh = (double*)calloc((size_t)(k + 1) * k, sizeof(double));   /* H[i][j] = hh[i*k + j] */
    double* cs = (double*)calloc((size_t)k, sizeof(double));
    double* sn = (double*)calloc((size_t)k, sizeof(double));
    double* g = (double*)calloc((size_t)k + 1, sizeof(double));
    double* y = (double*)calloc((size_t)k, sizeof(double));
    if (!pool || !hh || !cs || !sn || !g || !y) {
        free(pool); free(hh); free(cs); free(sn); free(g); free(y);
        return -1;
    }
    double* wx = pool;
    double* wy = wx + nwx;
    double* wz = wy + nwy;
    double* s = wz + nwz;
    double* w = s + n;
    double* xb = w + n;
    double* V = xb + n;                  /* v_i = V + i*n, i = 0..k  */
    double* Z = V + (int64_t)(k + 1) * n; /* z_i = Z + i*n, i < k    */
    orc_face_weights(pb, wx, wy, wz);

    const double RR = orc_dot(n, rhs, rhs);
    const double T = tol * tol * RR;
    st->rhs_norm2 = RR;
    residual_RAx(pb, wx, wy, wz, rhs, x, s, n);
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
            orc_apply_pinv(pb, wx, wy, wz, vj, zj);
            apply_events_at(events, n_events, sx, ORC_V_P, ORC_V_E, zj, st, &events_since_rb);
            orc_apply_A(pb, wx, wy, wz, zj, w);
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
            residual_RAx(pb, wx, wy, wz, rhs, x, s, n);
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
        residual_RAx(pb, wx, wy, wz, rhs, x, s, n);
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
                residual_RAx(pb, wx, wy, wz, rhs, x, s, n);
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
