/*
 * slmo.c -- FP64 CPU oracle for semi-Lagrangian MGRIT (arXiv 2203.13382).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the GPU library.  Plain loops,
 * no blocking, no fusion, summations in index order.  See slmo.h for the
 * conventions.  Readings of passages where the paper is silent are marked
 * "Reading:".
 *
 * Threads (OpenMP, when compiled with it): the coarse intervals of a
 * relaxation sweep, the time steps of the setup and the nodes of one
 * interpolation are independent and may run on several threads.  Every sum
 * is still taken in index order on one thread, so results do not depend on
 * the thread count.
 */
#include "slmo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SLMO_PI 3.14159265358979323846
#define SLMO_MAXL 64

static long long pmod(long long a, long long n) { long long r = a % n; return r < 0 ? r + n : r; }

void slmo_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int slmo_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Problem data                                                              */
/* ------------------------------------------------------------------------ */

/* Wave speed evaluated from its term list (Sec. 2.1 asks only that alpha be
 * computable at any (x,t)).  Reading: each term is
 * coef*cos(kx*pi*x+px)*cos(ky*pi*y+py)*cos(kt*pi*t+pt). */
double slmo_wave(const slmo_term *t, int n, double x, double y, double time)
{
    double s = 0.0;
    for (int k = 0; k < n; k++)
        s += t[k].coef * cos(t[k].kx * SLMO_PI * x + t[k].px)
                       * cos(t[k].ky * SLMO_PI * y + t[k].py)
                       * cos(t[k].kt * SLMO_PI * time + t[k].pt);
    return s;
}

/* Explicit Runge-Kutta tableaux (Sec. 2.1: one ERK step of global order r
 * traces each departure point).  The paper takes its tableaux from a thesis
 * that is not reproduced; Reading: r=1 forward Euler, r=2 Heun, r=3 Kutta's
 * third-order method, r=4 the classical fourth-order method, r=5 Butcher's
 * six-stage fifth-order method (Butcher 1964).  Returns the stage count. */
int slmo_erk_tableau(int r, double *c, double *a, double *b)
{
    for (int i = 0; i < 36; i++) a[i] = 0.0;
    for (int i = 0; i < 6; i++) { c[i] = 0.0; b[i] = 0.0; }
#define A(i, j) a[(i) * 6 + (j)]
    switch (r) {
    case 1:
        b[0] = 1.0;
        return 1;
    case 2:
        c[1] = 1.0; A(1, 0) = 1.0;
        b[0] = 0.5; b[1] = 0.5;
        return 2;
    case 3:
        c[1] = 0.5; c[2] = 1.0;
        A(1, 0) = 0.5;
        A(2, 0) = -1.0; A(2, 1) = 2.0;
        b[0] = 1.0 / 6.0; b[1] = 2.0 / 3.0; b[2] = 1.0 / 6.0;
        return 3;
    case 4:
        c[1] = 0.5; c[2] = 0.5; c[3] = 1.0;
        A(1, 0) = 0.5; A(2, 1) = 0.5; A(3, 2) = 1.0;
        b[0] = 1.0 / 6.0; b[1] = 1.0 / 3.0; b[2] = 1.0 / 3.0; b[3] = 1.0 / 6.0;
        return 4;
    case 5:
        c[1] = 0.25; c[2] = 0.25; c[3] = 0.5; c[4] = 0.75; c[5] = 1.0;
        A(1, 0) = 0.25;
        A(2, 0) = 0.125; A(2, 1) = 0.125;
        A(3, 0) = 0.0; A(3, 1) = -0.5; A(3, 2) = 1.0;
        A(4, 0) = 3.0 / 16.0; A(4, 3) = 9.0 / 16.0;
        A(5, 0) = -3.0 / 7.0; A(5, 1) = 2.0 / 7.0; A(5, 2) = 12.0 / 7.0;
        A(5, 3) = -12.0 / 7.0; A(5, 4) = 8.0 / 7.0;
        b[0] = 7.0 / 90.0; b[2] = 32.0 / 90.0; b[3] = 12.0 / 90.0;
        b[4] = 32.0 / 90.0; b[5] = 7.0 / 90.0;
        return 6;
    default:
        return 0;
    }
#undef A
}

/* One ERK step of size dt backwards in time along a characteristic that
 * arrives at (x,y) at time t_arr: the final-value problem of eq. (depart_ODE)
 * in 1D and eqs. (SL2D_char1-2) in 2D.  The step size of the integration is
 * -dt. */
void slmo_erk_back(const slmo_problem *pr, double x, double y, double t_arr,
                   double dt, double *xd, double *yd)
{
    double c[6], a[36], b[6], kx[6], ky[6];
    int s = slmo_erk_tableau(pr->r, c, a, b);
    double hs = -dt;
    for (int i = 0; i < s; i++) {
        double X = x, Y = y;
        for (int j = 0; j < i; j++) {
            X += hs * a[i * 6 + j] * kx[j];
            Y += hs * a[i * 6 + j] * ky[j];
        }
        double ti = t_arr + c[i] * hs;
        kx[i] = slmo_wave(pr->alpha, pr->n_alpha, X, Y, ti);
        ky[i] = pr->dim == 2 ? slmo_wave(pr->beta, pr->n_beta, X, Y, ti) : 0.0;
    }
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < s; i++) { sx += b[i] * kx[i]; sy += b[i] * ky[i]; }
    *xd = x + hs * sx;
    *yd = pr->dim == 2 ? y + hs * sy : y;
}

/* ------------------------------------------------------------------------ */
/* Interpolation stencil (Sec. 2.1, eq. depart_decompose)                    */
/* ------------------------------------------------------------------------ */

/* A departure point xi is written as x_E - h*eps with x_E the mesh node
 * immediately east of it and eps in [0,1).  Reading: a departure point on a
 * node has that node as x_E and eps = 0 (ceil rule).  E is unwrapped. */
void slmo_decompose(int nx, double xi, long long *E, double *eps)
{
    double h = 2.0 / nx;
    double s = (xi + 1.0) / h;
    double e = ceil(s);
    *E = (long long)e;
    *eps = e - s;
}

/* West and east extents l(p), r(p) of the p+1 nearest nodes (Sec. 2.1).
 * Odd p: l = (p+1)/2, r = (p-1)/2.  Even p: a one-point bias that depends on
 * whether eps exceeds one half; Reading: eps > 1/2 takes the extra node on
 * the west (the departure point is then nearer x_E - h). */
void slmo_stencil(int p, double eps, int *ell, int *rr)
{
    if (p % 2 == 1) { *ell = (p + 1) / 2; *rr = (p - 1) / 2; }
    else if (eps > 0.5) { *ell = p / 2 + 1; *rr = p / 2 - 1; }
    else { *ell = p / 2; *rr = p / 2; }
}

/* Lagrange weights of the degree-p polynomial through nodes x_E + j h,
 * j = -l..r, evaluated at x_E - h eps (Sec. 2.1).  w[j+l]. */
void slmo_weights(int p, double eps, double *w)
{
    int ell, rr;
    slmo_stencil(p, eps, &ell, &rr);
    double z = -eps;
    for (int j = -ell; j <= rr; j++) {
        double num = 1.0, den = 1.0;
        for (int k = -ell; k <= rr; k++) {
            if (k == j) continue;
            num *= z - k;
            den *= (double)(j - k);
        }
        w[j + ell] = num / den;
    }
}

/* f_{p+1}(z) of eq. (fpoly_def): (1/(p+1)!) prod_{q=-l(p)}^{r(p)} (q + z). */
double slmo_fpoly(int p, double z)
{
    int ell, rr;
    slmo_stencil(p, z, &ell, &rr);
    double prod = 1.0, fact = 1.0;
    for (int q = -ell; q <= rr; q++) prod *= (q + z);
    for (int k = 2; k <= p + 1; k++) fact *= k;
    return prod / fact;
}

/* D_{p+1} of eq. (Dp+1_def): periodic, second-order finite-difference rule
 * with h^{-(p+1)} D_{p+1} ~ d^{p+1}/dx^{p+1} (odd p only: p+1 even).
 * Reading: the central difference (delta^2)^{(p+1)/2}, whose taps are
 * (-1)^{k+q} binom(2q, k+q), k = -q..q, q = (p+1)/2.  taps[k+q]. */
void slmo_dop_taps(int p, double *taps)
{
    int q = (p + 1) / 2;
    for (int k = -q; k <= q; k++) {
        double bin = 1.0;           /* binom(2q, k+q) */
        for (int t = 1; t <= k + q; t++) bin = bin * (2 * q - t + 1) / t;
        taps[k + q] = ((k + q) % 2 == 0 ? 1.0 : -1.0) * bin;
    }
}

/* ------------------------------------------------------------------------ */
/* Vector operators                                                          */
/* ------------------------------------------------------------------------ */

/* Fine-grid departure points of step n (t_n -> t_{n+1}) for every node. */
void slmo_depart_fine(const slmo_problem *pr, int n, double *xi, double *eta)
{
    int nx = pr->nx;
    double h = 2.0 / nx;
    double t_arr = (n + 1) * pr->dt;
    if (pr->dim == 1) {
        for (int i = 0; i < nx; i++) {
            double yd;
            slmo_erk_back(pr, -1.0 + i * h, 0.0, t_arr, pr->dt, &xi[i], &yd);
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int j = 0; j < nx; j++)
            for (int i = 0; i < nx; i++)
                slmo_erk_back(pr, -1.0 + i * h, -1.0 + j * h, t_arr, pr->dt,
                              &xi[j * nx + i], &eta[j * nx + i]);
    }
}

/* Semi-Lagrangian interpolation S (Sec. 2.1; 2D tensor product Sec. 4.1):
 * out[k] = interpolant of u at the departure point of node k. */
void slmo_interp(int dim, int nx, int p, const double *xi, const double *eta,
                 const double *u, double *out)
{
    double wx[8], wy[8];
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            long long E; double eps; int ell, rr;
            slmo_decompose(nx, xi[i], &E, &eps);
            slmo_stencil(p, eps, &ell, &rr);
            slmo_weights(p, eps, wx);
            double s = 0.0;
            for (int j = -ell; j <= rr; j++) s += wx[j + ell] * u[pmod(E + j, nx)];
            out[i] = s;
        }
        return;
    }
    long long S = (long long)nx * nx;
#pragma omp parallel for schedule(static) private(wx, wy)
    for (long long k = 0; k < S; k++) {
        long long E, N; double eps, nu; int lx, rx, ly, ry;
        slmo_decompose(nx, xi[k], &E, &eps);
        slmo_decompose(nx, eta[k], &N, &nu);
        slmo_stencil(p, eps, &lx, &rx);
        slmo_stencil(p, nu, &ly, &ry);
        slmo_weights(p, eps, wx);
        slmo_weights(p, nu, wy);
        double s = 0.0;
        for (int b = -ly; b <= ry; b++) {
            long long row = pmod(N + b, nx);
            double sr = 0.0;
            for (int a = -lx; a <= rx; a++) sr += wx[a + lx] * u[row * nx + pmod(E + a, nx)];
            s += wy[b + ly] * sr;
        }
        out[k] = s;
    }
}

/* out = D_{p+1} v on a periodic 1D mesh. */
void slmo_apply_D(int nx, int p, const double *v, double *out)
{
    double taps[8];
    int q = (p + 1) / 2;
    slmo_dop_taps(p, taps);
    for (int i = 0; i < nx; i++) {
        double s = 0.0;
        for (int k = -q; k <= q; k++) s += taps[k + q] * v[pmod(i + k, nx)];
        out[i] = s;
    }
}

/* out = [I + diag(sx) D_x + diag(sy) D_y] v: the explicit forward-Euler
 * correction F_{p+1} of eq. (Fp_def), applied after the coarse SL step; the
 * coefficients are the same phi / sigma as for the backward-Euler operator. */
void slmo_apply_F(int dim, int nx, int p, const double *sx, const double *sy,
                  const double *v, double *out)
{
    double taps[8];
    int q = (p + 1) / 2;
    slmo_dop_taps(p, taps);
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            double d = 0.0;
            for (int k = -q; k <= q; k++) d += taps[k + q] * v[pmod(i + k, nx)];
            out[i] = v[i] + sx[i] * d;
        }
        return;
    }
    for (int j = 0; j < nx; j++)
        for (int i = 0; i < nx; i++) {
            double dx = 0.0, dy = 0.0;
            for (int k = -q; k <= q; k++) {
                dx += taps[k + q] * v[(long long)j * nx + pmod(i + k, nx)];
                dy += taps[k + q] * v[pmod(j + k, nx) * nx + i];
            }
            long long id = (long long)j * nx + i;
            out[id] = v[id] + sx[id] * dx + sy[id] * dy;
        }
}

/* Transpose of slmo_apply_F: out = v + D_x (sx .* v) + D_y (sy .* v). */
void slmo_apply_FT(int dim, int nx, int p, const double *sx, const double *sy,
                   const double *v, double *out)
{
    double taps[8];
    int q = (p + 1) / 2;
    slmo_dop_taps(p, taps);
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            double d = 0.0;
            for (int k = -q; k <= q; k++) {
                long long t = pmod(i + k, nx);
                d += taps[k + q] * sx[t] * v[t];
            }
            out[i] = v[i] + d;
        }
        return;
    }
    for (int j = 0; j < nx; j++)
        for (int i = 0; i < nx; i++) {
            double dx = 0.0, dy = 0.0;
            for (int k = -q; k <= q; k++) {
                long long tx = (long long)j * nx + pmod(i + k, nx), ty = pmod(j + k, nx) * nx + i;
                dx += taps[k + q] * sx[tx] * v[tx];
                dy += taps[k + q] * sy[ty] * v[ty];
            }
            long long id = (long long)j * nx + i;
            out[id] = v[id] + dx + dy;
        }
}

/* out = [I - diag(sx) D_x - diag(sy) D_y] v: the matrix inverted by the
 * backward-Euler correction, eq. (Phi_multilevel) in 1D and eq. (BEOper_2D)
 * in 2D, with D_x = I (x) D_{p+1} and D_y = D_{p+1} (x) I (Sec. 4.2). */
void slmo_apply_B(int dim, int nx, int p, const double *sx, const double *sy,
                  const double *v, double *out)
{
    double taps[8];
    int q = (p + 1) / 2;
    slmo_dop_taps(p, taps);
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            double d = 0.0;
            for (int k = -q; k <= q; k++) d += taps[k + q] * v[pmod(i + k, nx)];
            out[i] = v[i] - sx[i] * d;
        }
        return;
    }
    for (int j = 0; j < nx; j++)
        for (int i = 0; i < nx; i++) {
            double dx = 0.0, dy = 0.0;
            for (int k = -q; k <= q; k++) {
                dx += taps[k + q] * v[(long long)j * nx + pmod(i + k, nx)];
                dy += taps[k + q] * v[pmod(j + k, nx) * nx + i];
            }
            long long id = (long long)j * nx + i;
            out[id] = v[id] - sx[id] * dx - sy[id] * dy;
        }
}

/* out = B^T v = [I - D_x diag(sx) - D_y diag(sy)] v: the transpose of
 * slmo_apply_B (D_{p+1} is symmetric), used by the adjoint coarse operator. */
void slmo_apply_BT(int dim, int nx, int p, const double *sx, const double *sy,
                   const double *v, double *out)
{
    double taps[8];
    int q = (p + 1) / 2;
    slmo_dop_taps(p, taps);
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            double d = 0.0;
            for (int k = -q; k <= q; k++) {
                long long t = pmod(i + k, nx);
                d += taps[k + q] * sx[t] * v[t];
            }
            out[i] = v[i] - d;
        }
        return;
    }
    for (int j = 0; j < nx; j++)
        for (int i = 0; i < nx; i++) {
            double dx = 0.0, dy = 0.0;
            for (int k = -q; k <= q; k++) {
                long long tx = (long long)j * nx + pmod(i + k, nx);
                long long ty = pmod(j + k, nx) * nx + i;
                dx += taps[k + q] * sx[tx] * v[tx];
                dy += taps[k + q] * sy[ty] * v[ty];
            }
            long long id = (long long)j * nx + i;
            out[id] = v[id] - dx - dy;
        }
}

static double dot(long long n, const double *a, const double *b)
{
    double s = 0.0;
    for (long long i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* GMRES for [I - diag(sx)D_x - diag(sy)D_y] y = b with a zero initial guess
 * (Sec. 3.3: ten iterations; Sec. 3.4 and 4.3: stop once the relative
 * residual is at most 1e-2 or after ten iterations).  Reading: no
 * preconditioner; Arnoldi with classical Gram-Schmidt (one pass: every
 * projection coefficient is taken of the same vector w = A v_j).  The new
 * vector's norm follows from the same pass by Pythagoras,
 * ||w - V h||^2 = ||w||^2 - sum h_i^2 (V orthonormal), unless that
 * difference is below 1e-3 ||w||^2, where cancellation would cost more than
 * three digits: then it is computed from the updated vector.  Givens rotations for the
 * least-squares problem; the relative residual is the Givens estimate
 * |g_{j+1}|/||b||, tested after each iteration; rtol = 0 runs all kmax
 * iterations; b = 0 returns y = 0.  Returns the iterations done. */
static int bsolve_gen(int dim, int nx, int p, const double *sx, const double *sy,
                     const double *b, double *y, int kmax, double rtol, int transpose);

int slmo_bsolve(int dim, int nx, int p, const double *sx, const double *sy,
                const double *b, double *y, int kmax, double rtol)
{
    return bsolve_gen(dim, nx, p, sx, sy, b, y, kmax, rtol, 0);
}

/* The same GMRES for the transposed system B^T y = b (adjoint coarse
 * operator). */
int slmo_bsolve_T(int dim, int nx, int p, const double *sx, const double *sy,
                  const double *b, double *y, int kmax, double rtol)
{
    return bsolve_gen(dim, nx, p, sx, sy, b, y, kmax, rtol, 1);
}

static int bsolve_gen(int dim, int nx, int p, const double *sx, const double *sy,
                      const double *b, double *y, int kmax, double rtol, int transpose)
{
    long long S = dim == 1 ? nx : (long long)nx * nx;
    double beta = sqrt(dot(S, b, b));
    for (long long i = 0; i < S; i++) y[i] = 0.0;
    if (beta == 0.0 || kmax <= 0) return 0;
    double *V = (double *)malloc(sizeof(double) * S * (kmax + 1));
    double *w = (double *)malloc(sizeof(double) * S);
    double *H = (double *)calloc((size_t)(kmax + 1) * kmax, sizeof(double)); /* R, column-major */
    double *cs = (double *)calloc(kmax, sizeof(double));
    double *sn = (double *)calloc(kmax, sizeof(double));
    double *g = (double *)calloc(kmax + 1, sizeof(double));
    double *hcol = (double *)calloc(kmax + 1, sizeof(double));
    double *z = (double *)calloc(kmax + 1, sizeof(double));
    for (long long i = 0; i < S; i++) V[i] = b[i] / beta;
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < kmax; j++) {
        if (transpose) slmo_apply_BT(dim, nx, p, sx, sy, V + (long long)j * S, w);
        else slmo_apply_B(dim, nx, p, sx, sy, V + (long long)j * S, w);
        for (int i = 0; i <= j; i++) hcol[i] = dot(S, V + (long long)i * S, w);   /* classical G-S */
        double ww = dot(S, w, w);
        for (int i = 0; i <= j; i++) {
            const double *vi = V + (long long)i * S;
            for (long long t = 0; t < S; t++) w[t] -= hcol[i] * vi[t];
        }
        double hn2 = ww;                             /* Pythagoras */
        for (int i = 0; i <= j; i++) hn2 -= hcol[i] * hcol[i];
        if (!(hn2 >= 1e-3 * ww)) hn2 = dot(S, w, w); /* cancellation: the explicit norm */
        double hn = sqrt(hn2 > 0.0 ? hn2 : 0.0);
        for (int i = 0; i < j; i++) {                /* previous rotations */
            double t0 = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
            double t1 = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
            hcol[i] = t0; hcol[i + 1] = t1;
        }
        double den = sqrt(hcol[j] * hcol[j] + hn * hn);
        cs[j] = hcol[j] / den;
        sn[j] = hn / den;
        hcol[j] = den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        for (int i = 0; i <= j; i++) H[(long long)j * (kmax + 1) + i] = hcol[i];
        k = j + 1;
        if (hn == 0.0) break;                        /* happy breakdown */
        for (long long t = 0; t < S; t++) V[(long long)(j + 1) * S + t] = w[t] / hn;
        if (fabs(g[j + 1]) <= rtol * beta) break;
    }
    for (int i = k - 1; i >= 0; i--) {               /* back substitution */
        double s = g[i];
        for (int t = i + 1; t < k; t++) s -= H[(long long)t * (kmax + 1) + i] * z[t];
        z[i] = s / H[(long long)i * (kmax + 1) + i];
    }
    for (int i = 0; i < k; i++) {
        const double *vi = V + (long long)i * S;
        for (long long t = 0; t < S; t++) y[t] += z[i] * vi[t];
    }
    free(V); free(w); free(H); free(cs); free(sn); free(g); free(hcol); free(z);
    return k;
}

/* Backtracking of a coarse departure point through the m fine sub-steps of
 * a coarse step (Sec. 3.3.1, eq. coarse_depart_interp).  fine[k*nx+i] is the
 * departure point of sub-step k whose characteristic arrives at x_i.  The
 * last sub-step's departure point starts the recursion; each earlier one is
 * the linear interpolant of the sub-step's departure map at the current
 * point.  Reading (periodic mesh): E and W are unwrapped indices of the
 * nodes east and west of c; the departure map at an unwrapped node is the
 * stored one shifted by the same multiple of the period 2. */
void slmo_backtrack_1d(int nx, int m, const double *fine, double *coarse)
{
    double h = 2.0 / nx;
    for (int i = 0; i < nx; i++) {
        double c = fine[(long long)(m - 1) * nx + i];
        for (int k = m - 2; k >= 0; k--) {
            long long E = (long long)ceil((c + 1.0) / h), W = E - 1;
            long long e = pmod(E, nx), w = pmod(W, nx);
            double xE = -1.0 + E * h;
            double fE = fine[(long long)k * nx + e] + (double)(E - e) * h;
            double fW = fine[(long long)k * nx + w] + (double)(W - w) * h;
            c = (fE - fW) / h * (c - xE) + fE;
        }
        coarse[i] = c;
    }
}

/* Linear interpolant p^1d of SM6 eq. (poly_interp_1d). */
static double p1d(double x, double xE, double h, double qE, double qW)
{
    return (qE - qW) / h * (x - xE) + qE;
}

/* Bilinear interpolant p^2d of SM6 eq. (poly_interp_2d) on the cell with
 * north-east corner (xE, yN). */
static double p2d(double x, double y, double xE, double yN, double h,
                  double rNE, double rNW, double rSE, double rSW)
{
    double north = p1d(x, xE, h, rNE, rNW);
    double south = p1d(x, xE, h, rSE, rSW);
    return (north - south) / h * (y - yN) + north;
}

/* 2D backtracking (SM6): the x and y components of the coarse characteristic
 * are each propagated through a bilinear fit of how the four neighbouring
 * fine characteristics map their arrival point to their departure point.
 * fxi/feta are [m][nx*nx]; periodic shifts as in the 1D case. */
void slmo_backtrack_2d(int nx, int m, const double *fxi, const double *feta,
                       double *cxi, double *ceta)
{
    double h = 2.0 / nx;
    long long S = (long long)nx * nx;
    for (long long id = 0; id < S; id++) {
        double cx = fxi[(long long)(m - 1) * S + id];
        double cy = feta[(long long)(m - 1) * S + id];
        for (int k = m - 2; k >= 0; k--) {
            long long E = (long long)ceil((cx + 1.0) / h), W = E - 1;
            long long N = (long long)ceil((cy + 1.0) / h), Sd = N - 1;
            long long e = pmod(E, nx), w = pmod(W, nx), n = pmod(N, nx), s = pmod(Sd, nx);
            double xE = -1.0 + E * h, yN = -1.0 + N * h;
            double sxE = (double)(E - e) * h, sxW = (double)(W - w) * h;
            double syN = (double)(N - n) * h, syS = (double)(Sd - s) * h;
            const double *X = fxi + (long long)k * S, *Y = feta + (long long)k * S;
            double nx_ = p2d(cx, cy, xE, yN, h,
                             X[n * nx + e] + sxE, X[n * nx + w] + sxW,
                             X[s * nx + e] + sxE, X[s * nx + w] + sxW);
            double ny_ = p2d(cx, cy, xE, yN, h,
                             Y[n * nx + e] + syN, Y[n * nx + w] + syN,
                             Y[s * nx + e] + syS, Y[s * nx + w] + syS);
            cx = nx_; cy = ny_;
        }
        cxi[id] = cx; ceta[id] = cy;
    }
}

/* Sequential time-stepping of eq. (one-step) with g = 0: the plain
 * definition of what MGRIT converges to. u_all is [(nt+1)][S]. */
void slmo_seq_fine(const slmo_problem *pr, const double *u0, double *u_all)
{
    long long S = pr->dim == 1 ? pr->nx : (long long)pr->nx * pr->nx;
    double *xi = (double *)malloc(sizeof(double) * S);
    double *eta = (double *)malloc(sizeof(double) * S);
    memcpy(u_all, u0, sizeof(double) * S);
    for (int n = 0; n < pr->nt; n++) {
        slmo_depart_fine(pr, n, xi, eta);
        slmo_interp(pr->dim, pr->nx, pr->p, xi, eta, u_all + (long long)n * S,
                    u_all + (long long)(n + 1) * S);
    }
    free(xi); free(eta);
}

/* ------------------------------------------------------------------------ */
/* Hierarchy, coarse-operator setup and linear MGRIT                         */
/* ------------------------------------------------------------------------ */

struct slmo_ctx {
    slmo_problem pr;
    slmo_term *alpha, *beta;
    slmo_solver sv;
    int *mlist;
    int L;
    int N[SLMO_MAXL], mm[SLMO_MAXL];
    long long M[SLMO_MAXL];                 /* fine steps per level-l step */
    long long S;
    double *dep[SLMO_MAXL][2];              /* departure points [N_l][S] */
    double *sig[SLMO_MAXL][2];              /* sigma vectors, l >= 1 */
    double *v[SLMO_MAXL], *g[SLMO_MAXL];    /* MGRIT iterate and RHS */
    double *t0, *t1;                        /* work slices */
    long long gmres_solves, gmres_iters;
    int adjoint;                            /* 1: reverse-time adjoint system */
};

/* Initial iterate of MGRIT.  Sec. 2.2 starts from a random space-time
 * guess with entries uniform in [0,1) and gives no generator.  Reading: a
 * counter-based draw, so that any implementation can reproduce it without
 * sharing a random stream.  The value at fine time point n and node k is the
 * SplitMix64 output (Steele, Lea & Flood, OOPSLA 2014) for the state
 * seed XOR (n*S + k), keeping its top 53 bits as a fraction of 2^53.
 * SplitMix64's output for a state x: z = x + 0x9e3779b97f4a7c15, then
 * z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9, z = (z ^ (z >> 27)) *
 * 0x94d049bb133111eb, result z ^ (z >> 31). */
uint64_t slmo_splitmix64(uint64_t x)
{
    uint64_t z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double slmo_seeded_value(uint64_t seed, uint64_t idx)
{
    return (double)(slmo_splitmix64(seed ^ idx) >> 11) * (1.0 / 9007199254740992.0);
}

/* u is [(nt+1)][S]; the C-points (time points n = j*m0; every point when
 * m0 <= 1) receive the seeded values, the other entries are left alone. */
void slmo_seeded_iterate(uint64_t seed, int nt, long long S, int m0, double *u)
{
    int step = m0 > 1 ? m0 : 1;
    for (long long n = 0; n <= nt; n += step)
        for (long long k = 0; k < S; k++) u[n * S + k] = slmo_seeded_value(seed, (uint64_t)(n * S + k));
}

/* Level hierarchy (Sec. 2.2 and 3.4): coarsen by m_l while the coarse level
 * keeps at least two time points.  Reading: also stop at max_levels, once a
 * level has no more than coarsest_max_points points, or when N_l is not a
 * multiple of m_l (that level is then solved sequentially). */
int slmo_hierarchy(int nt, const slmo_solver *sv, int *N, int *mm, int cap)
{
    int L = 1;
    N[0] = nt;
    for (int l = 0; l + 1 < cap; l++) {
        int m = sv->m[l < sv->n_m ? l : sv->n_m - 1];
        mm[l] = 0;
        if (l + 1 >= sv->max_levels) break;
        if (N[l] + 1 <= sv->coarsest_max_points) break;
        if (m < 2 || N[l] % m != 0 || N[l] / m < 1) break;
        mm[l] = m;
        N[l + 1] = N[l] / m;
        L = l + 2;
    }
    mm[L - 1] = 0;
    return L;
}

static double *alloc0(long long n) { return (double *)calloc((size_t)n, sizeof(double)); }

slmo_ctx *slmo_setup(const slmo_problem *pr, const slmo_solver *sv)
{
    slmo_ctx *c = (slmo_ctx *)calloc(1, sizeof(slmo_ctx));
    c->pr = *pr;
    c->alpha = (slmo_term *)malloc(sizeof(slmo_term) * (pr->n_alpha > 0 ? pr->n_alpha : 1));
    memcpy(c->alpha, pr->alpha, sizeof(slmo_term) * pr->n_alpha);
    c->pr.alpha = c->alpha;
    c->beta = (slmo_term *)malloc(sizeof(slmo_term) * (pr->n_beta > 0 ? pr->n_beta : 1));
    if (pr->n_beta > 0) memcpy(c->beta, pr->beta, sizeof(slmo_term) * pr->n_beta);
    c->pr.beta = c->beta;
    c->sv = *sv;
    c->mlist = (int *)malloc(sizeof(int) * sv->n_m);
    memcpy(c->mlist, sv->m, sizeof(int) * sv->n_m);
    c->sv.m = c->mlist;
    c->S = pr->dim == 1 ? pr->nx : (long long)pr->nx * pr->nx;
    c->L = slmo_hierarchy(pr->nt, sv, c->N, c->mm, SLMO_MAXL);
    c->M[0] = 1;
    for (int l = 1; l < c->L; l++) c->M[l] = c->M[l - 1] * c->mm[l - 1];
    c->t0 = alloc0(c->S);
    c->t1 = alloc0(c->S);
    int dim = pr->dim, nx = pr->nx, p = pr->p;
    long long S = c->S;
    double h = 2.0 / nx;

    /* level 0: ERK departure points of every fine step */
    c->dep[0][0] = alloc0(S * c->N[0]);
    c->dep[0][1] = dim == 2 ? alloc0(S * c->N[0]) : NULL;
#pragma omp parallel for schedule(dynamic)
    for (int n = 0; n < c->N[0]; n++)
        slmo_depart_fine(pr, n, c->dep[0][0] + n * S, dim == 2 ? c->dep[0][1] + n * S : NULL);

    for (int l = 1; l < c->L; l++) {
        int m = c->mm[l - 1];
        long long Nl = c->N[l];
        if (sv->coarse_op == SLMO_COARSE_IDEAL) continue;
        c->dep[l][0] = alloc0(S * Nl);
        c->dep[l][1] = dim == 2 ? alloc0(S * Nl) : NULL;
        if (sv->coarse_op == SLMO_COARSE_REDISC) {
            /* rediscretised operator: departure points from M_l fine-size ERK
             * steps (Sec. 2.3; Sec. 4.3 locates them this way). */
#pragma omp parallel for schedule(dynamic)
            for (long long n = 0; n < Nl; n++)
                for (long long id = 0; id < S; id++) {
                    double x = -1.0 + (id % nx) * h, y = dim == 2 ? -1.0 + (id / nx) * h : 0.0;
                    for (long long s = c->M[l] - 1; s >= 0; s--) {
                        double t_arr = (n * c->M[l] + s + 1) * pr->dt, xd, yd;
                        slmo_erk_back(pr, x, y, t_arr, pr->dt, &xd, &yd);
                        x = xd; y = yd;
                    }
                    c->dep[l][0][n * S + id] = x;
                    if (dim == 2) c->dep[l][1][n * S + id] = y;
                }
            continue;
        }
        /* modified operator: backtracked departure points (Sec. 3.3.1,
         * recursively across levels, Sec. 3.4; SM6 in 2D), then phi of
         * eq. (varphi_p_multilevel_def) and sigma of eq. (nu_p_def).
         * Reading: the sum over sub-steps is taken node by node; in 2D the
         * x and y coefficient vectors follow the same recursion separately. */
        c->sig[l][0] = alloc0(S * Nl);
        c->sig[l][1] = dim == 2 ? alloc0(S * Nl) : NULL;
        double sgn = (p + 1) % 2 == 0 ? 1.0 : -1.0;
#pragma omp parallel for schedule(dynamic)
        for (long long n = 0; n < Nl; n++) {
            const double *fx = c->dep[l - 1][0] + n * m * S;
            if (dim == 1) slmo_backtrack_1d(nx, m, fx, c->dep[l][0] + n * S);
            else slmo_backtrack_2d(nx, m, fx, c->dep[l - 1][1] + n * m * S,
                                   c->dep[l][0] + n * S, c->dep[l][1] + n * S);
            for (int comp = 0; comp < dim; comp++) {
                const double *dc = c->dep[l][comp] + n * S;
                const double *df = c->dep[l - 1][comp] + n * m * S;
                for (long long id = 0; id < S; id++) {
                    long long E; double eps;
                    slmo_decompose(nx, dc[id], &E, &eps);
                    double fc = slmo_fpoly(p, eps), fs = 0.0;
                    for (int k = 0; k < m; k++) {
                        slmo_decompose(nx, df[k * S + id], &E, &eps);
                        fs += slmo_fpoly(p, eps);
                    }
                    double phi = sgn * (fc - fs);
                    double acc = 0.0;
                    if (l > 1)
                        for (int k = 0; k < m; k++) acc += c->sig[l - 1][comp][(n * m + k) * S + id];
                    c->sig[l][comp][n * S + id] = acc + phi;
                }
            }
        }
    }
    return c;
}

void slmo_free(slmo_ctx *c)
{
    if (!c) return;
    for (int l = 0; l < SLMO_MAXL; l++) {
        free(c->dep[l][0]); free(c->dep[l][1]);
        free(c->sig[l][0]); free(c->sig[l][1]);
        if (l > 0) { free(c->v[l]); free(c->g[l]); }
    }
    free(c->t0); free(c->t1); free(c->alpha); free(c->beta); free(c->mlist);
    free(c);
}

int slmo_levels(const slmo_ctx *c) { return c->L; }
int slmo_level_N(const slmo_ctx *c, int l) { return c->N[l]; }
int slmo_level_m(const slmo_ctx *c, int l) { return c->mm[l]; }
const double *slmo_level_dep(const slmo_ctx *c, int l, int comp) { return c->dep[l][comp]; }
const double *slmo_level_sigma(const slmo_ctx *c, int l, int comp) { return c->sig[l][comp]; }

/* The level-l time-stepper Phi_l for step n (t_n^l -> t_{n+1}^l).
 * l = 0: S_{p,r} (Sec. 2.1).  l >= 1, modified: [I - diag(sigma) D]^{-1}
 * S_{p,r*} (eq. Phi_multilevel; eq. BEOper_2D in 2D) with the inverse
 * approximated by GMRES.  Forward Euler: [I + diag(sigma) D] S_{p,r*}
 * (eq. Fp_def), explicit.  Ideal: the product of the fine steps it spans
 * (Sec. 2.2).  Rediscretised: S_{p,r} with the coarse time-step. */
void slmo_apply_phi(slmo_ctx *c, int l, int n, const double *in, double *out)
{
    const slmo_problem *pr = &c->pr;
    long long S = c->S;
    if (l == 0 || c->sv.coarse_op == SLMO_COARSE_REDISC) {
        slmo_interp(pr->dim, pr->nx, pr->p, c->dep[l][0] + (long long)n * S,
                    pr->dim == 2 ? c->dep[l][1] + (long long)n * S : NULL, in, out);
        return;
    }
    if (c->sv.coarse_op == SLMO_COARSE_IDEAL) {
        double *a = (double *)malloc(sizeof(double) * S), *b = (double *)malloc(sizeof(double) * S);
        memcpy(a, in, sizeof(double) * S);
        for (long long s = 0; s < c->M[l]; s++) {
            long long f = (long long)n * c->M[l] + s;
            slmo_interp(pr->dim, pr->nx, pr->p, c->dep[0][0] + f * S,
                        pr->dim == 2 ? c->dep[0][1] + f * S : NULL, a, b);
            double *t = a; a = b; b = t;
        }
        memcpy(out, a, sizeof(double) * S);
        free(a); free(b);
        return;
    }
    double *tmp = (double *)malloc(sizeof(double) * S);
    slmo_interp(pr->dim, pr->nx, pr->p, c->dep[l][0] + (long long)n * S,
                pr->dim == 2 ? c->dep[l][1] + (long long)n * S : NULL, in, tmp);
    if (c->sv.coarse_op == SLMO_COARSE_FWD) {   /* eq. (Fp_def): explicit correction */
        slmo_apply_F(pr->dim, pr->nx, pr->p, c->sig[l][0] + (long long)n * S,
                     pr->dim == 2 ? c->sig[l][1] + (long long)n * S : NULL, tmp, out);
        free(tmp);
        return;
    }
    int it = slmo_bsolve(pr->dim, pr->nx, pr->p, c->sig[l][0] + (long long)n * S,
                         pr->dim == 2 ? c->sig[l][1] + (long long)n * S : NULL,
                         tmp, out, c->sv.gmres_kmax, c->sv.gmres_rtol);
#pragma omp atomic
    c->gmres_solves++;
#pragma omp atomic
    c->gmres_iters += it;
    free(tmp);
}

/* The level-l one-step operator of the system being solved: Phi_l(n) for
 * the forward system; for the adjoint system in reverse time (step k maps
 * lambda_{N-k} to lambda_{N-k-1}) the transpose of the forward step it
 * mirrors, Phi_l(N_l-1-k)^T. */
static void phi_sys(slmo_ctx *c, int l, int n, const double *in, double *out)
{
    if (c->adjoint) slmo_apply_phi_T(c, l, c->N[l] - 1 - n, in, out);
    else slmo_apply_phi(c, l, n, in, out);
}

/* v[n] = Phi_l(n-1) v[n-1] + g[n]  (eq. one-step at level l) */
static void step_to(slmo_ctx *c, int l, int n)
{
    long long S = c->S;
    double *v = c->v[l];
    phi_sys(c, l, n - 1, v + (long long)(n - 1) * S, v + (long long)n * S);
    if (c->g[l])
        for (long long i = 0; i < S; i++) v[(long long)n * S + i] += c->g[l][(long long)n * S + i];
}

/* F-relaxation (Sec. 2.2): from each C-point across the m-1 F-points after it. */
static void f_relax(slmo_ctx *c, int l)
{
    int m = c->mm[l], nc = c->N[l] / m;
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < nc; j++)
        for (int k = 1; k < m; k++) step_to(c, l, j * m + k);
}

/* C-relaxation (Sec. 2.2): each C-point from the F-point before it. */
static void c_relax(slmo_ctx *c, int l)
{
    int m = c->mm[l], nc = c->N[l] / m;
#pragma omp parallel for schedule(dynamic)
    for (int j = 1; j <= nc; j++) step_to(c, l, j * m);
}

/* C-point residual r_{jm} = g_{jm} + Phi v_{jm-1} - v_{jm} (Sec. 2.2), injected
 * as the right-hand side of level l+1 (eq. one-step-coarse).  Returns its
 * unscaled Euclidean norm over all C-point entries. */
static double residual(slmo_ctx *c, int l)
{
    int m = c->mm[l], nc = c->N[l] / m;
    long long S = c->S;
    double *v = c->v[l], *gc = c->g[l + 1], s2 = 0.0;
#pragma omp parallel for schedule(dynamic)
    for (int j = 1; j <= nc; j++) {
        long long n = (long long)j * m;
        double *t = gc + (long long)j * S;            /* Phi v_{jm-1}, then r_{jm} */
        phi_sys(c, l, (int)n - 1, v + (n - 1) * S, t);
        for (long long i = 0; i < S; i++)
            t[i] = (c->g[l] ? c->g[l][n * S + i] : 0.0) + t[i] - v[n * S + i];
    }
    for (int j = 1; j <= nc; j++)                      /* in index order */
        for (long long i = 0; i < S; i++) s2 += gc[(long long)j * S + i] * gc[(long long)j * S + i];
    return sqrt(s2);
}

static void pre_relax(slmo_ctx *c, int l)
{
    f_relax(c, l);
    if (c->sv.relax == SLMO_RELAX_FCF) { c_relax(c, l); f_relax(c, l); }
}

/* Coarse-grid correction of level l (linear MGRIT, SM2): the coarse unknown
 * is the error, starting from zero; it is solved sequentially on the
 * coarsest level or by a recursive V-cycle, then injected at the C-points. */
static void cycle_from(slmo_ctx *c, int l);

static void coarse_correct(slmo_ctx *c, int l)
{
    long long S = c->S;
    int nc = c->N[l + 1], m = c->mm[l];
    memset(c->v[l + 1], 0, sizeof(double) * S * (nc + 1));
    cycle_from(c, l + 1);
    for (int j = 1; j <= nc; j++)
        for (long long i = 0; i < S; i++) c->v[l][(long long)j * m * S + i] += c->v[l + 1][(long long)j * S + i];
}

static void cycle_from(slmo_ctx *c, int l)
{
    if (l == c->L - 1) {
        for (int n = 1; n <= c->N[l]; n++) step_to(c, l, n);
        return;
    }
    pre_relax(c, l);
    residual(c, l);
    coarse_correct(c, l);
    f_relax(c, l);
}

/* Linear MGRIT driver (Sec. 2.2; SM2).  u is [(nt+1)][S]: on entry its
 * C-points hold the initial iterate (u[0] is overwritten by u0); on exit the
 * approximate solution.  Reading of the stopping test (Sec. 2.2): the
 * residual norm rho_k is measured after cycle k's pre-relaxation (k = 0, 1,
 * ...); iterations stop at the first k with rho_k < tol*rho_0 (relative) or
 * rho_k < tol (absolute), and the iteration count is k+1, the number of
 * cycles begun (this count reproduces the constant-speed columns of Tables
 * 1-3).  DIVERGED only if rho_k is not finite: there is no test on growth,
 * since with the rediscretised coarse operator of Table 3 the residual
 * grows by many orders of magnitude and still converges in the printed
 * number of cycles (rounding added at the peak is damped like any other
 * error of the iterate);
 * NOT_CONVERGED once k reaches max_iter, after that cycle's coarse-grid
 * correction (the returned iterate is where cycle k+1 would start). */
int slmo_mgrit(slmo_ctx *c, const double *u0, double *u, double *hist, int hist_cap,
               slmo_stats *st)
{
    long long S = c->S;
    c->v[0] = u;
    c->g[0] = NULL;                         /* g_n = 0 for n >= 1 */
    memcpy(u, u0, sizeof(double) * S);
    for (int l = 1; l < c->L; l++) {
        if (!c->v[l]) c->v[l] = alloc0(S * (c->N[l] + 1));
        if (!c->g[l]) c->g[l] = alloc0(S * (c->N[l] + 1));
    }
    c->gmres_solves = c->gmres_iters = 0;
    slmo_stats s;
    memset(&s, 0, sizeof(s));
    s.n_levels = c->L;
    if (c->L == 1) {
        for (int n = 1; n <= c->N[0]; n++) step_to(c, 0, n);
        s.status = SLMO_CONVERGED;
    } else {
        double rho0 = 0.0;
        for (int k = 0;; k++) {
            pre_relax(c, 0);
            double rho = residual(c, 0);
            if (k < hist_cap) hist[k] = rho;
            if (k == 0) rho0 = rho;
            s.rho_final = rho;
            s.iterations = k + 1;
            double thr = c->sv.tol_mode == SLMO_TOL_REL ? c->sv.tol * rho0 : c->sv.tol;
            if (rho < thr || rho == 0.0) { s.status = SLMO_CONVERGED; break; }
            if (!isfinite(rho)) { s.status = SLMO_DIVERGED; break; }
            coarse_correct(c, 0);
            f_relax(c, 0);
            /* Reading: a run cut off at max_iter still completes the cycle's
             * coarse-grid correction, so the iterate it leaves is the one the
             * next cycle starts from and a second call resumes exactly. */
            if (k >= c->sv.max_iter) { s.status = SLMO_NOT_CONVERGED; break; }
        }
        s.rho0 = rho0;
    }
    s.gmres_solves = c->gmres_solves;
    s.gmres_iters = c->gmres_iters;
    if (st) *st = s;
    c->v[0] = NULL;
    return s.status;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the one-step system (gradients of a final-time misfit)         */
/* ------------------------------------------------------------------------ */
/* The discrete forward problem is the space-time system A u = g of Sec. 2.2
 * with u_{n+1} = S_n u_n.  For L = 1/2 ||u_nt - u_obs||^2 the adjoint
 * system A^T lambda = dL/du reads lambda_nt = u_nt - u_obs and
 * lambda_n = S_n^T lambda_{n+1}; then dL/du0 = lambda_0 and, for a
 * coefficient theta of the wave-speed terms,
 *     dL/dtheta = sum_n lambda_{n+1}^T (dS_n/dtheta) u_n,
 * where S_n depends on theta through its departure points only. */

/* out = S^T lam: the transpose of slmo_interp, written as the scatter of
 * every node's interpolation weights. */
void slmo_interp_T(int dim, int nx, int p, const double *xi, const double *eta,
                   const double *lam, double *out)
{
    double wx[8], wy[8];
    long long S = dim == 1 ? nx : (long long)nx * nx;
    for (long long k = 0; k < S; k++) out[k] = 0.0;
    if (dim == 1) {
        for (int i = 0; i < nx; i++) {
            long long E; double eps; int ell, rr;
            slmo_decompose(nx, xi[i], &E, &eps);
            slmo_stencil(p, eps, &ell, &rr);
            slmo_weights(p, eps, wx);
            for (int j = -ell; j <= rr; j++) out[pmod(E + j, nx)] += wx[j + ell] * lam[i];
        }
        return;
    }
    for (long long k = 0; k < S; k++) {
        long long E, N; double eps, nu; int lx, rx, ly, ry;
        slmo_decompose(nx, xi[k], &E, &eps);
        slmo_decompose(nx, eta[k], &N, &nu);
        slmo_stencil(p, eps, &lx, &rx);
        slmo_stencil(p, nu, &ly, &ry);
        slmo_weights(p, eps, wx);
        slmo_weights(p, nu, wy);
        for (int b = -ly; b <= ry; b++) {
            long long row = pmod(N + b, nx);
            for (int a = -lx; a <= rx; a++)
                out[row * nx + pmod(E + a, nx)] += wy[b + ly] * wx[a + lx] * lam[k];
        }
    }
}

/* Phi_l(n)^T.  Level 0: S_n^T.  Modified coarse operator (eq.
 * Phi_multilevel / BEOper_2D): (B^{-1} S_l)^T = S_l^T (B^T)^{-1}, the inverse
 * again by GMRES.  Reading: the adjoint uses the same GMRES settings as the
 * forward solve.  Ideal: the product of the transposed fine steps in reverse
 * order.  Rediscretised: S_l^T. */
void slmo_apply_phi_T(slmo_ctx *c, int l, int n, const double *in, double *out)
{
    const slmo_problem *pr = &c->pr;
    long long S = c->S;
    if (l == 0 || c->sv.coarse_op == SLMO_COARSE_REDISC) {
        slmo_interp_T(pr->dim, pr->nx, pr->p, c->dep[l][0] + (long long)n * S,
                      pr->dim == 2 ? c->dep[l][1] + (long long)n * S : NULL, in, out);
        return;
    }
    if (c->sv.coarse_op == SLMO_COARSE_IDEAL) {
        double *a = (double *)malloc(sizeof(double) * S), *b = (double *)malloc(sizeof(double) * S);
        memcpy(a, in, sizeof(double) * S);
        for (long long s = c->M[l] - 1; s >= 0; s--) {
            long long f = (long long)n * c->M[l] + s;
            slmo_interp_T(pr->dim, pr->nx, pr->p, c->dep[0][0] + f * S,
                          pr->dim == 2 ? c->dep[0][1] + f * S : NULL, a, b);
            double *t = a; a = b; b = t;
        }
        memcpy(out, a, sizeof(double) * S);
        free(a); free(b);
        return;
    }
    double *tmp = (double *)malloc(sizeof(double) * S);
    if (c->sv.coarse_op == SLMO_COARSE_FWD) {   /* (F S)^T = S^T F^T */
        slmo_apply_FT(pr->dim, pr->nx, pr->p, c->sig[l][0] + (long long)n * S,
                      pr->dim == 2 ? c->sig[l][1] + (long long)n * S : NULL, in, tmp);
        slmo_interp_T(pr->dim, pr->nx, pr->p, c->dep[l][0] + (long long)n * S,
                      pr->dim == 2 ? c->dep[l][1] + (long long)n * S : NULL, tmp, out);
        free(tmp);
        return;
    }
    int it = slmo_bsolve_T(pr->dim, pr->nx, pr->p, c->sig[l][0] + (long long)n * S,
                           pr->dim == 2 ? c->sig[l][1] + (long long)n * S : NULL,
                           in, tmp, c->sv.gmres_kmax, c->sv.gmres_rtol);
#pragma omp atomic
    c->gmres_solves++;
#pragma omp atomic
    c->gmres_iters += it;
    slmo_interp_T(pr->dim, pr->nx, pr->p, c->dep[l][0] + (long long)n * S,
                  pr->dim == 2 ? c->dep[l][1] + (long long)n * S : NULL, tmp, out);
    free(tmp);
}

/* Sequential adjoint sweep: lam is [(nt+1)][S]; lam[nt] = lamT and
 * lam[n] = S_n^T lam[n+1] (the plain definition of the adjoint solution). */
void slmo_adjoint_seq(const slmo_problem *pr, const double *lamT, double *lam)
{
    long long S = pr->dim == 1 ? pr->nx : (long long)pr->nx * pr->nx;
    double *xi = (double *)malloc(sizeof(double) * S);
    double *eta = (double *)malloc(sizeof(double) * S);
    memcpy(lam + (long long)pr->nt * S, lamT, sizeof(double) * S);
    for (int n = pr->nt - 1; n >= 0; n--) {
        slmo_depart_fine(pr, n, xi, eta);
        slmo_interp_T(pr->dim, pr->nx, pr->p, xi, eta, lam + (long long)(n + 1) * S,
                      lam + (long long)n * S);
    }
    free(xi); free(eta);
}

/* Linear MGRIT on the adjoint system in reverse time: mu_k = lambda_{nt-k},
 * mu_0 = lamT, mu_{k+1} = S_{nt-1-k}^T mu_k.  The level hierarchy, coarse
 * departure points and sigma of the forward context are reused: reverse
 * coarse step K of level l mirrors forward coarse step N_l-1-K, whose
 * transpose is its coarse operator.  Same driver, cycle and stopping test as
 * slmo_mgrit.  mu is [(nt+1)][S]; its C-points are the initial iterate. */
int slmo_mgrit_adjoint(slmo_ctx *c, const double *lamT, double *mu, double *hist, int hist_cap,
                       slmo_stats *st)
{
    c->adjoint = 1;
    int rc = slmo_mgrit(c, lamT, mu, hist, hist_cap, st);
    c->adjoint = 0;
    return rc;
}

/* Derivative of one term cos(kx pi x + px) cos(ky pi y + py) cos(kt pi t + pt)
 * (without its coefficient) with respect to x and y. */
static void term_grad(const slmo_term *t, double x, double y, double time, double *val,
                      double *gx, double *gy)
{
    double ax = t->kx * SLMO_PI * x + t->px, ay = t->ky * SLMO_PI * y + t->py;
    double ct = cos(t->kt * SLMO_PI * time + t->pt);
    *val = cos(ax) * cos(ay) * ct;
    *gx = -t->kx * SLMO_PI * sin(ax) * cos(ay) * ct;
    *gy = -t->ky * SLMO_PI * cos(ax) * sin(ay) * ct;
}

/* Tangent of the backward ERK departure point (slmo_erk_back) with respect
 * to every term coefficient: dxi[q], deta[q] for q = 0..n_alpha-1 (alpha
 * terms) then n_alpha..n_alpha+n_beta-1 (beta terms).  The ERK stages are
 * differentiated exactly (forward-mode through the stage recursion). */
void slmo_erk_back_tangent(const slmo_problem *pr, double x, double y, double t_arr,
                           double dt, double *dxi, double *deta)
{
    double c[6], a[36], b[6], kx[6], ky[6], X[6], Y[6];
    int s = slmo_erk_tableau(pr->r, c, a, b);
    int nq = pr->n_alpha + (pr->dim == 2 ? pr->n_beta : 0);
    double hs = -dt;
    for (int i = 0; i < s; i++) {
        X[i] = x; Y[i] = y;
        for (int j = 0; j < i; j++) {
            X[i] += hs * a[i * 6 + j] * kx[j];
            Y[i] += hs * a[i * 6 + j] * ky[j];
        }
        double ti = t_arr + c[i] * hs;
        kx[i] = slmo_wave(pr->alpha, pr->n_alpha, X[i], Y[i], ti);
        ky[i] = pr->dim == 2 ? slmo_wave(pr->beta, pr->n_beta, X[i], Y[i], ti) : 0.0;
    }
    for (int q = 0; q < nq; q++) {
        double dkx[6], dky[6];
        for (int i = 0; i < s; i++) {
            double dX = 0.0, dY = 0.0;
            for (int j = 0; j < i; j++) {
                dX += hs * a[i * 6 + j] * dkx[j];
                dY += hs * a[i * 6 + j] * dky[j];
            }
            double ti = t_arr + c[i] * hs;
            double ax = 0.0, ay = 0.0, bx = 0.0, by = 0.0, pa = 0.0, pb = 0.0, v, gx, gy;
            for (int k = 0; k < pr->n_alpha; k++) {
                term_grad(&pr->alpha[k], X[i], Y[i], ti, &v, &gx, &gy);
                ax += pr->alpha[k].coef * gx;
                ay += pr->alpha[k].coef * gy;
                if (k == q) pa = v;
            }
            if (pr->dim == 2)
                for (int k = 0; k < pr->n_beta; k++) {
                    term_grad(&pr->beta[k], X[i], Y[i], ti, &v, &gx, &gy);
                    bx += pr->beta[k].coef * gx;
                    by += pr->beta[k].coef * gy;
                    if (pr->n_alpha + k == q) pb = v;
                }
            dkx[i] = ax * dX + (pr->dim == 2 ? ay * dY : 0.0) + pa;
            dky[i] = pr->dim == 2 ? bx * dX + by * dY + pb : 0.0;
        }
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < s; i++) { sx += b[i] * dkx[i]; sy += b[i] * dky[i]; }
        dxi[q] = hs * sx;
        deta[q] = pr->dim == 2 ? hs * sy : 0.0;
    }
}

/* Derivatives of the Lagrange weights of slmo_weights with respect to eps
 * (odd p: the stencil does not change with eps):
 * d/deps w_j(-eps) = -sum_{l != j} prod_{k != j,l} (z - k) / prod_{k != j} (j - k). */
void slmo_weights_deps(int p, double eps, double *dw)
{
    int ell, rr;
    slmo_stencil(p, eps, &ell, &rr);
    double z = -eps;
    for (int j = -ell; j <= rr; j++) {
        double den = 1.0, sum = 0.0;
        for (int k = -ell; k <= rr; k++)
            if (k != j) den *= (double)(j - k);
        for (int l = -ell; l <= rr; l++) {
            if (l == j) continue;
            double prod = 1.0;
            for (int k = -ell; k <= rr; k++)
                if (k != j && k != l) prod *= z - k;
            sum += prod;
        }
        dw[j + ell] = -sum / den;
    }
}

/* dL/dtheta = sum_n lam[n+1]^T (dS_n/dtheta) u[n] for every term
 * coefficient (order of slmo_erk_back_tangent).  u and lam are
 * [(nt+1)][S].  eps = ceil(s) - s with s = (xi+1)/h, so d eps = -d xi / h
 * away from mesh nodes. */
void slmo_grad_theta(const slmo_problem *pr, const double *u, const double *lam, double *grad)
{
    int nx = pr->nx, p = pr->p, dim = pr->dim;
    int nq = pr->n_alpha + (dim == 2 ? pr->n_beta : 0);
    long long S = dim == 1 ? nx : (long long)nx * nx;
    double h = 2.0 / nx;
    double wx[8], wy[8], dwx[8], dwy[8], dxi[2 * 8], deta[2 * 8];
    for (int q = 0; q < nq; q++) grad[q] = 0.0;
    for (int n = 0; n < pr->nt; n++) {
        const double *un = u + (long long)n * S, *ln = lam + (long long)(n + 1) * S;
        double t_arr = (n + 1) * pr->dt;
        for (long long k = 0; k < S; k++) {
            double x = -1.0 + (k % nx) * h, y = dim == 2 ? -1.0 + (k / nx) * h : 0.0;
            double xd, yd;
            slmo_erk_back(pr, x, y, t_arr, pr->dt, &xd, &yd);
            slmo_erk_back_tangent(pr, x, y, t_arr, pr->dt, dxi, deta);
            long long E, N = 0; double eps, nu = 0.0; int lx, rx, ly = 0, ry = 0;
            slmo_decompose(nx, xd, &E, &eps);
            slmo_stencil(p, eps, &lx, &rx);
            slmo_weights(p, eps, wx);
            slmo_weights_deps(p, eps, dwx);
            double gx = 0.0, gy = 0.0;      /* d u_{n+1}[k] / d eps, / d nu */
            if (dim == 1) {
                for (int a = -lx; a <= rx; a++) gx += dwx[a + lx] * un[pmod(E + a, nx)];
            } else {
                slmo_decompose(nx, yd, &N, &nu);
                slmo_stencil(p, nu, &ly, &ry);
                slmo_weights(p, nu, wy);
                slmo_weights_deps(p, nu, dwy);
                for (int b = -ly; b <= ry; b++) {
                    long long row = pmod(N + b, nx);
                    for (int a = -lx; a <= rx; a++) {
                        double uv = un[row * nx + pmod(E + a, nx)];
                        gx += dwx[a + lx] * wy[b + ly] * uv;
                        gy += wx[a + lx] * dwy[b + ly] * uv;
                    }
                }
            }
            for (int q = 0; q < nq; q++)
                grad[q] += ln[k] * (gx * (-dxi[q] / h) + (dim == 2 ? gy * (-deta[q] / h) : 0.0));
        }
    }
}
