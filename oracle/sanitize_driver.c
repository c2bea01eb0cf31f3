/*
 * sanitize_driver.c -- runs the oracle's routines on small problems so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer can check
 * them for memory and undefined-behaviour errors (test infrastructure; the
 * CPU test suite compiles and runs it).  Exits 0 when every call returns.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "slmo.h"

static void run_problem(int dim, int nx, int nt, int p, int relax, int coarse_op, int kmax, double rtol)
{
    slmo_term alpha[2] = {{1.0, 0, 0, 0, 0, 0, 0}, {0.5, 1.0, -1.5707963267948966, 0, 0, 2.0, 0}};
    slmo_term beta[1] = {{0.7, 1.0, -1.5707963267948966, 0, 0, 1.0, 0}};
    int m[2] = {4, 2};
    slmo_problem pr = {dim, nx, nt, 1.3 * 2.0 / nx, p, p, alpha, 2, beta, dim == 2 ? 1 : 0};
    slmo_solver sv = {m, 2, 8, 2, relax, coarse_op, kmax, rtol, 1e-10, SLMO_TOL_REL, 40};
    long long S = dim == 1 ? nx : (long long)nx * nx;
    double *u0 = malloc(sizeof(double) * S), *u = calloc((size_t)(nt + 1) * S, sizeof(double));
    double *lam = calloc((size_t)(nt + 1) * S, sizeof(double)), hist[64], grad[4];
    for (long long i = 0; i < S; i++) u0[i] = sin(0.37 * (double)i) + 0.1 * (double)(i % 7);
    slmo_seeded_iterate(11, nt, S, m[0], u);
    slmo_ctx *c = slmo_setup(&pr, &sv);
    slmo_stats st;
    slmo_mgrit(c, u0, u, hist, 64, &st);
    if (coarse_op == SLMO_COARSE_MODIFIED && p % 2 == 1) {
        double *mu = calloc((size_t)(nt + 1) * S, sizeof(double));
        slmo_mgrit_adjoint(c, u0, mu, hist, 64, &st);
        free(mu);
    }
    slmo_seq_fine(&pr, u0, u);
    slmo_adjoint_seq(&pr, u0, lam);
    slmo_grad_theta(&pr, u, lam, grad);
    slmo_free(c);
    free(u0); free(u); free(lam);
}

int main(void)
{
    /* operators on their own */
    double w[8], taps[8], tab_c[6], tab_a[36], tab_b[6];
    for (int p = 1; p <= 5; p++) {
        slmo_weights(p, 0.3, w);
        slmo_weights_deps(p, 0.6, w);
        slmo_dop_taps(p, taps);
    }
    for (int r = 1; r <= 5; r++) slmo_erk_tableau(r, tab_c, tab_a, tab_b);
    double fine[4 * 16], coarse[16];
    for (int i = 0; i < 64; i++) fine[i] = -1.0 + (i % 16) * (2.0 / 16) - 0.05 * (i / 16);
    slmo_backtrack_1d(16, 4, fine, coarse);
    double *fx = malloc(sizeof(double) * 3 * 64), *fy = malloc(sizeof(double) * 3 * 64), cx[64], cy[64];
    for (int i = 0; i < 3 * 64; i++) { fx[i] = -1.0 + (i % 8) * 0.25 - 0.03; fy[i] = -1.0 + ((i / 8) % 8) * 0.25 + 0.02; }
    slmo_backtrack_2d(8, 3, fx, fy, cx, cy);
    free(fx); free(fy);
    /* GMRES with more iterations than the usual ten */
    double sx[32], b[32], y[32];
    for (int i = 0; i < 32; i++) { sx[i] = -0.2 - 0.01 * i; b[i] = cos(0.3 * i); }
    slmo_bsolve(1, 32, 3, sx, NULL, b, y, 32, 0.0);
    slmo_bsolve_T(1, 32, 3, sx, NULL, b, y, 20, 1e-12);
    /* whole solves: 1D and 2D, F and FCF, every coarse operator */
    run_problem(1, 32, 64, 3, SLMO_RELAX_FCF, SLMO_COARSE_MODIFIED, 10, 1e-2);
    run_problem(1, 20, 48, 5, SLMO_RELAX_F, SLMO_COARSE_MODIFIED, 10, 0.0);
    run_problem(1, 32, 64, 2, SLMO_RELAX_FCF, SLMO_COARSE_REDISC, 10, 1e-2);
    run_problem(1, 32, 64, 1, SLMO_RELAX_FCF, SLMO_COARSE_FWD, 10, 1e-2);
    run_problem(1, 32, 64, 3, SLMO_RELAX_FCF, SLMO_COARSE_IDEAL, 10, 1e-2);
    run_problem(2, 12, 24, 3, SLMO_RELAX_FCF, SLMO_COARSE_MODIFIED, 10, 1e-2);
    run_problem(2, 10, 16, 1, SLMO_RELAX_F, SLMO_COARSE_REDISC, 10, 1e-2);
    puts("sanitized oracle run ok");
    return 0;
}
