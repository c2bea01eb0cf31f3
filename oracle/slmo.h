/*
 * slmo.h -- FP64 CPU oracle for semi-Lagrangian MGRIT on periodic advection.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded reference
 * written from De Sterck, Falgout & Krzysik, "Fast multigrid reduction-in-time
 * for advection via modified semi-Lagrangian coarse-grid operators"
 * (arXiv 2203.13382).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * Every routine cites the passage it follows (section / equation of the
 * paper; "SM" = the paper's supplementary materials).  Where the paper is
 * silent the reading taken is stated next to the code.
 *
 * Conventions
 *   mesh     x_i = -1 + i h, i = 0..nx-1, h = 2/nx (periodic on [-1,1));
 *            2D: same in y, grid index k = j*nx + i (x fastest), Sec. 4.2.
 *   time     t_n = n dt, n = 0..nt.
 *   arrays   space-time arrays are [(N+1)][S] with S = nx^dim.
 *   departure points are stored as POSITIONS (unwrapped, not reduced mod 2).
 */
#ifndef SLMO_H
#define SLMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* wave-speed term: coef*cos(kx*pi*x+px)*cos(ky*pi*y+py)*cos(kt*pi*t+pt) */
typedef struct { double coef, kx, px, ky, py, kt, pt; } slmo_term;

enum { SLMO_RELAX_F = 0, SLMO_RELAX_FCF = 1 };
enum { SLMO_COARSE_MODIFIED = 0, SLMO_COARSE_IDEAL = 1, SLMO_COARSE_REDISC = 2, SLMO_COARSE_FWD = 3 };
enum { SLMO_TOL_ABS = 0, SLMO_TOL_REL = 1 };
enum { SLMO_CONVERGED = 0, SLMO_NOT_CONVERGED = 1, SLMO_DIVERGED = 2 };

typedef struct {
    int dim, nx, nt;
    double dt;
    int p, r;
    const slmo_term *alpha; int n_alpha;
    const slmo_term *beta;  int n_beta;
} slmo_problem;

typedef struct {
    const int *m; int n_m;          /* coarsening factor per level (last repeats) */
    int max_levels;                 /* >= 1 */
    int coarsest_max_points;        /* stop once a level has <= this many points */
    int relax;                      /* SLMO_RELAX_F / SLMO_RELAX_FCF */
    int coarse_op;                  /* SLMO_COARSE_* */
    int gmres_kmax;
    double gmres_rtol;              /* 0 => always gmres_kmax iterations */
    double tol; int tol_mode; int max_iter;
} slmo_solver;

typedef struct {
    int iterations, status, n_levels;
    double rho0, rho_final;
    long long gmres_solves, gmres_iters;
} slmo_stats;

/* ---- threads (OpenMP builds; results do not depend on the count) ---- */
void slmo_set_threads(int n);
int  slmo_get_threads(void);

/* ---- scalar building blocks ---- */
double slmo_wave(const slmo_term *t, int n, double x, double y, double time);
int    slmo_erk_tableau(int r, double *c, double *a, double *b); /* a is 6x6 row-major */
void   slmo_erk_back(const slmo_problem *pr, double x, double y, double t_arr,
                     double dt, double *xd, double *yd);
void   slmo_stencil(int p, double eps, int *ell, int *rr);
void   slmo_weights(int p, double eps, double *w);
double slmo_fpoly(int p, double z);
void   slmo_dop_taps(int p, double *taps);
void   slmo_decompose(int nx, double xi, long long *E, double *eps);

/* ---- vector operators ---- */
void slmo_depart_fine(const slmo_problem *pr, int n, double *xi, double *eta);
void slmo_interp(int dim, int nx, int p, const double *xi, const double *eta,
                 const double *u, double *out);
void slmo_apply_D(int nx, int p, const double *v, double *out);
/* out = [I + diag(sx) D_x + diag(sy) D_y] v: the explicit forward-Euler
 * correction F_{p+1} of eq. (Fp_def). */
void slmo_apply_F(int dim, int nx, int p, const double *sx, const double *sy,
                  const double *v, double *out);
/* out = [I + D_x diag(sx) + D_y diag(sy)] v (its transpose; D symmetric). */
void slmo_apply_FT(int dim, int nx, int p, const double *sx, const double *sy,
                   const double *v, double *out);
void slmo_apply_B(int dim, int nx, int p, const double *sx, const double *sy,
                  const double *v, double *out);
int  slmo_bsolve(int dim, int nx, int p, const double *sx, const double *sy,
                 const double *b, double *y, int kmax, double rtol);
void slmo_backtrack_1d(int nx, int m, const double *fine /* m x nx */, double *coarse);
void slmo_backtrack_2d(int nx, int m, const double *fxi, const double *feta,
                       double *cxi, double *ceta);
void slmo_seq_fine(const slmo_problem *pr, const double *u0, double *u_all);

/* ---- seeded initial iterate (Sec. 2.2: random initial guess) ---- */
uint64_t slmo_splitmix64(uint64_t state);
double   slmo_seeded_value(uint64_t seed, uint64_t idx);
void     slmo_seeded_iterate(uint64_t seed, int nt, long long S, int m0, double *u);

/* ---- hierarchy, setup and MGRIT ---- */
typedef struct slmo_ctx slmo_ctx;
int   slmo_hierarchy(int nt, const slmo_solver *sv, int *N, int *mm, int cap);
slmo_ctx *slmo_setup(const slmo_problem *pr, const slmo_solver *sv);
void  slmo_free(slmo_ctx *c);
int   slmo_levels(const slmo_ctx *c);
int   slmo_level_N(const slmo_ctx *c, int level);
int   slmo_level_m(const slmo_ctx *c, int level);
const double *slmo_level_dep(const slmo_ctx *c, int level, int comp);
const double *slmo_level_sigma(const slmo_ctx *c, int level, int comp);
void  slmo_apply_phi(slmo_ctx *c, int level, int n, const double *in, double *out);
int   slmo_mgrit(slmo_ctx *c, const double *u0, double *u, double *hist, int hist_cap,
                 slmo_stats *st);

/* ---- adjoint (gradient of 1/2 ||u_nt - u_obs||^2) ---- */
void slmo_apply_BT(int dim, int nx, int p, const double *sx, const double *sy,
                   const double *v, double *out);
int  slmo_bsolve_T(int dim, int nx, int p, const double *sx, const double *sy,
                   const double *b, double *y, int kmax, double rtol);
void slmo_interp_T(int dim, int nx, int p, const double *xi, const double *eta,
                   const double *lam, double *out);
void slmo_apply_phi_T(slmo_ctx *c, int level, int n, const double *in, double *out);
void slmo_adjoint_seq(const slmo_problem *pr, const double *lamT, double *lam_all);
int  slmo_mgrit_adjoint(slmo_ctx *c, const double *lamT, double *mu, double *hist, int hist_cap,
                        slmo_stats *st);
void slmo_erk_back_tangent(const slmo_problem *pr, double x, double y, double t_arr,
                           double dt, double *dxi, double *deta);
void slmo_weights_deps(int p, double eps, double *dw);
void slmo_grad_theta(const slmo_problem *pr, const double *u_all, const double *lam_all,
                     double *grad);

#ifdef __cplusplus
}
#endif
#endif
