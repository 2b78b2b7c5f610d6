/*
 * Memory and undefined-behaviour check of the oracle (test infrastructure).
 *
 * A small driver, built together with ftgcr_oracle.c under gcc's address and
 * undefined-behaviour sanitizers by the CPU test suite, that calls every
 * entry point of the oracle on tiny problems: the lat-lon operator and
 * preconditioner, FT-GCR(k) and FT-GMRES(k) with and without a
 * preconditioner, fault plans given as index lists, ranges and per-entry bit
 * lists, truncated logs and histories, the traced solve, invalid arguments,
 * and the octahedral mesh, operator and solves.  Any out-of-bounds access,
 * use after free, leak or undefined operation aborts the run with the
 * sanitizer's report; a wrong return code exits non-zero.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ftgcr_oracle.h"

static int failures = 0;

#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__,    \
                    __LINE__, #cond);                                       \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

/* deterministic uniform(-1, 1) values (a 64-bit linear congruential step) */
static void fill(double* v, int64_t n, uint64_t seed)
{
    uint64_t s = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    for (int64_t t = 0; t < n; ++t) {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        v[t] = (double)(s >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

static void latlon_cases(void)
{
    orc_problem pb = {12, 6, 5, 0.2, 1.57, 0.52, 0.7, 0.35, 0.3, 1e-3};
    const int64_t n = (int64_t)pb.nx * pb.ny * pb.nz;
    double* wx = malloc(sizeof(double) * (size_t)(pb.nx * pb.ny * pb.nz));
    double* wy = malloc(sizeof(double) * (size_t)(pb.nx * (pb.ny + 1) * pb.nz));
    double* wz = malloc(sizeof(double) * (size_t)(pb.nx * pb.ny * (pb.nz + 1)));
    double* x = malloc(sizeof(double) * (size_t)n);
    double* y = malloc(sizeof(double) * (size_t)n);
    double* rhs = malloc(sizeof(double) * (size_t)n);
    double hist[7];
    orc_detect log[1];
    orc_stats st;
    orc_face_weights(&pb, wx, wy, wz);
    fill(x, n, 1);
    orc_apply_A(&pb, wx, wy, wz, x, y);
    orc_apply_pinv(&pb, wx, wy, wz, x, y);
    EXPECT(isfinite(orc_dot(n, x, y)));
    EXPECT(orc_hill(&pb, pb.hill_lon, pb.hill_lat) == 1.0);
    fill(rhs, n, 2);

    /* fault plans of every shape, with a one-entry log and a short history */
    int64_t idx[3] = {0, n / 2, n - 1};
    uint8_t bits[3] = {62, 0, 63};
    orc_event ev[5] = {
        {2, ORC_V_R, 62, 3, 0, idx, NULL},
        {3, ORC_V_AP, 0, 3, 0, idx, bits},
        {4, ORC_V_E, 52, n / 10, n - n / 10, NULL, NULL},
        {5, ORC_V_X, 61, 1, 7, NULL, NULL},
        {6, ORC_V_P, 62, 2, 0, idx + 1, NULL},
    };
    for (int method = 0; method < 2; ++method) {
        for (int precond = 0; precond < 2; ++precond) {
            for (int32_t k = 1; k <= 4; k += 3) {
                memset(x, 0, sizeof(double) * (size_t)n);
                EXPECT(orc_solve_pc(&pb, precond, method, rhs, x, 1e-8, k, 400, 1, ev, 5, &st, log, 1, hist, 7)
                       == 0);
                EXPECT(st.log_len <= 1 && st.hist_len <= 7);
                memset(x, 0, sizeof(double) * (size_t)n);
                EXPECT(orc_solve_pc(&pb, precond, method, rhs, x, 1e-8, k, 400, 0, NULL, 0, &st, NULL, 0, NULL, 0)
                       == 0);
            }
        }
    }
    /* the traced solve, its short trace and a zero step cap */
    double cra[5], ca[5];
    memset(x, 0, sizeof(double) * (size_t)n);
    EXPECT(orc_solve_traced(&pb, rhs, x, 1e-10, 3, 300, 1, ev, 2, &st, log, 1, hist, 7, cra, ca, 5) == 0);
    memset(x, 0, sizeof(double) * (size_t)n);
    EXPECT(orc_solve(&pb, rhs, x, 1e-10, 3, 0, 1, NULL, 0, &st, NULL, 0, NULL, 0) == 0);
    EXPECT(st.steps_executed == 0 && st.status == ORC_MAX_STEPS);
    EXPECT(orc_gmres_solve(&pb, rhs, x, 1e-10, 3, 50, 1, NULL, 0, &st, NULL, 0, hist, 7) == 0);
    /* invalid arguments are refused */
    EXPECT(orc_solve(&pb, rhs, x, 1e-10, 0, 10, 1, NULL, 0, &st, NULL, 0, NULL, 0) == -1);
    EXPECT(orc_solve_pc(&pb, 2, 0, rhs, x, 1e-10, 3, 10, 1, NULL, 0, &st, NULL, 0, NULL, 0) == -1);
    orc_event bad = {1, ORC_V_R, 64, 1, 0, idx, NULL};
    EXPECT(orc_solve(&pb, rhs, x, 1e-10, 3, 10, 1, &bad, 1, &st, NULL, 0, NULL, 0) == -1);
    bad.bit = 3;
    bad.idx = NULL;
    bad.start = n;
    EXPECT(orc_solve(&pb, rhs, x, 1e-10, 3, 10, 1, &bad, 1, &st, NULL, 0, NULL, 0) == -1);
    free(wx);
    free(wy);
    free(wz);
    free(x);
    free(y);
    free(rhs);
}

static void octahedral_cases(void)
{
    for (int32_t N = 1; N <= 4; N += 3) {
        orc_oct_problem pb = {N, 3, 0.2, 1.57, 0.52, 0.7, 0.35, 0.3, 1e-3};
        const int64_t pts = orc_oct_cells(N), n = pts * pb.nz;
        int64_t sum = 0;
        for (int32_t j = 0; j < 2 * N; ++j) sum += orc_oct_ring_points(N, j);
        EXPECT(sum == pts);
        double* mu = malloc(sizeof(double) * (size_t)(2 * N));
        double* w = malloc(sizeof(double) * (size_t)(2 * N));
        orc_oct_gauss(N, mu, w);
        double* lon = malloc(sizeof(double) * (size_t)pts);
        double* lat = malloc(sizeof(double) * (size_t)pts);
        double* area = malloc(sizeof(double) * (size_t)pts);
        int64_t nedge = 0;
        EXPECT(orc_oct_mesh(&pb, lon, lat, area, &nedge) == 0);
        /* Euler on a sphere whose two polar rings of 20 points bound open
         * caps: 2E = 3(F - 2) + 40 and V - E + F = 2 give E = 3V - 40 */
        EXPECT(nedge == 3 * pts - 40);
        double* x = malloc(sizeof(double) * (size_t)n);
        double* y = malloc(sizeof(double) * (size_t)n);
        double* rhs = malloc(sizeof(double) * (size_t)n);
        fill(x, n, 3);
        EXPECT(orc_oct_apply_A(&pb, x, y) == 0);
        EXPECT(orc_oct_apply_pinv(&pb, x, y) == 0);
        fill(rhs, n, 4);
        int64_t idx[2] = {0, n - 1};
        orc_event ev[2] = {{2, ORC_V_R, 62, 2, 0, idx, NULL}, {3, ORC_V_E, 40, n / 3, 0, NULL, NULL}};
        orc_detect log[2];
        double hist[5];
        orc_stats st;
        for (int method = 0; method < 2; ++method) {
            memset(x, 0, sizeof(double) * (size_t)n);
            EXPECT(orc_oct_solve(&pb, rhs, x, 1e-8, 3, 500, 1, method, ev, 2, &st, log, 2, hist, 5) == 0);
            memset(x, 0, sizeof(double) * (size_t)n);
            EXPECT(orc_oct_solve_pc(&pb, 0, method, rhs, x, 1e-8, 3, 500, 1, ev, 2, &st, log, 2, hist, 5) == 0);
        }
        EXPECT(orc_oct_solve_pc(&pb, 3, 0, rhs, x, 1e-8, 3, 500, 1, NULL, 0, &st, NULL, 0, NULL, 0) == -1);
        free(mu);
        free(w);
        free(lon);
        free(lat);
        free(area);
        free(x);
        free(y);
        free(rhs);
    }
}

int main(void)
{
    latlon_cases();
    octahedral_cases();
    if (failures) {
        fprintf(stderr, "%d expectations failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: all entry points ran clean\n");
    return 0;
}
