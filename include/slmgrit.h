/*
 * slmgrit.h -- C ABI of the MI355X (gfx950) semi-Lagrangian MGRIT library.
 *
 * The library solves the one-step system of periodic linear advection
 * (De Sterck, Falgout & Krzysik, arXiv 2203.13382):
 *     u_{n+1} = Phi u_n,  n = 0..nt-1,  u_0 given              (eq. one-step)
 * for u_t + alpha u_x = 0 on [-1,1) (eq. ad) or
 *     u_t + alpha u_x + beta u_y = 0 on [-1,1)^2 (eq. ad_2D),
 * where Phi is a semi-Lagrangian step of order (p, r) (Sec. 2.1 and 4.1),
 * either by sequential stepping or by linear multilevel MGRIT (Sec. 2.2)
 * with the modified coarse-grid operator
 *     Phi_l = [I - diag(sigma_l) D_{p+1}]^{-1} S_{p,r*}(m^l dt)  (eq. Phi_multilevel)
 * whose coarse departure points are backtracked (Sec. 3.3.1; SM6 in 2D).
 *
 * Conventions shared by every call
 *   - Mesh x_i = -1 + i h, h = 2/nx (y likewise); a spatial slice has
 *     S = nx (1D) or nx*nx values (2D), x fastest.
 *   - A space-time array is [(N+1)][S], time index slowest.
 *   - "T" is the bulk element type of a plan: double for SLM_FP64, float for
 *     SLM_FP32_BULK.  Departure-point tracing, backtracking, sigma, GMRES
 *     inner products and residual norms are always FP64.
 *   - Device pointers are caller-owned, in the plan's device memory, and
 *     must stay valid for the duration of the call.  All device work of a
 *     call is enqueued on `stream` (a hipStream_t, 0 = legacy default);
 *     calls that return solver statistics synchronise that stream.
 *   - The library never allocates device memory: the caller provides the
 *     workspace sized by slm_plan_workspace_size().
 *   - Return codes: SLM_OK (0); positive values are solver outcomes; negative
 *     values are errors, with a message in slm_last_error().  No C++
 *     exception crosses this boundary.
 */
#ifndef SLMGRIT_H
#define SLMGRIT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest nt a plan takes: launches put time steps, coarse steps or
 * intervals on grid.y, whose limit HIP reports as 65536 on gfx950.
 * slm_plan_create refuses more with SLM_EUNSUPPORTED, and slm_plan_setup
 * also checks the current device's reported limit. */
#define SLM_MAX_NT 65536

/* One term of a wave-speed field (Sec. 2.1 requires alpha(x,t) computable
 * anywhere): coef*cos(kx*pi*x+px)*cos(ky*pi*y+py)*cos(kt*pi*t+pt).  A field
 * is a sum of at most SLM_MAX_TERMS terms. */
typedef struct { double coef, kx, px, ky, py, kt, pt; } slm_wave_term;
#define SLM_MAX_TERMS 8
#define SLM_MAX_LEVELS 24

enum { SLM_RELAX_F = 0, SLM_RELAX_FCF = 1 };            /* Sec. 2.2 */
enum { SLM_TOL_ABS = 0, SLM_TOL_REL = 1 };
enum { SLM_FP64 = 0, SLM_FP32_BULK = 1 };
/* Coarse-grid operator: the modified SL operator of eq. (Phi_multilevel) /
 * (BEOper_2D), the rediscretized SL operator of Sec. 2.3 (a plain SL step of
 * size m^l dt whose departure points are traced through the m^l fine-size
 * ERK steps it spans, as in Sec. 4.3's comparison), or the explicit
 * forward-Euler operator of eq. (Fp_def), [I + diag(sigma) D_{p+1}] S_{p,r*}
 * with the same departure points and sigma as the modified operator (the
 * paper finds it unstable for larger m, Sec. 3.2). */
enum { SLM_COARSE_MODIFIED = 0, SLM_COARSE_REDISC = 2, SLM_COARSE_FWD_EULER = 3 };

enum {
    SLM_OK = 0,                /* success / converged */
    SLM_NOT_CONVERGED = 1,     /* max_iter cycles without meeting tol */
    SLM_DIVERGED = 2,          /* residual norm not finite (no growth test) */
    SLM_STAGNATED = 3,         /* FP32 bulk: ratio > 0.95 for 3 cycles */
    SLM_EINVAL = -1,           /* invalid argument or descriptor */
    SLM_EUNSUPPORTED = -2,     /* valid but not supported by this library */
    SLM_EWORKSPACE = -3,       /* workspace missing or too small */
    SLM_EHIP = -4,             /* a HIP runtime call failed */
    SLM_ENOTSETUP = -5         /* slm_plan_setup() has not run */
};

/* Problem and solver description.  The library copies everything it needs
 * at slm_plan_create(); the caller keeps ownership of its arrays. */
typedef struct {
    int dim;                   /* 1 or 2 */
    int nx;                    /* nodes per axis, >= 8 (1D: <= 8192, 2D: <= 4096) */
    int nt;                    /* fine time steps, 1..SLM_MAX_NT */
    double dt;                 /* fine time step (> 0) */
    int p;                     /* interpolation degree 1..5 (MGRIT: odd p only) */
    int r;                     /* ERK order 1..5 of the departure trace */
    const slm_wave_term *alpha; int n_alpha;   /* x-speed */
    const slm_wave_term *beta;  int n_beta;    /* y-speed (2D) */
    const int *m; int n_m;     /* coarsening factor per level, the last repeats; >= 2 */
    int max_levels;            /* >= 1; 1 = no coarsening */
    int coarsest_max_points;   /* stop coarsening once a level has <= this many time points */
    int relax;                 /* SLM_RELAX_F or SLM_RELAX_FCF */
    int gmres_kmax;            /* 1..10 GMRES iterations for the B solve (Sec. 3.3) */
    double gmres_rtol;         /* exit once the relative residual <= rtol; 0 = always kmax */
    double tol;                /* stop once rho_k < tol (ABS) or tol*rho_0 (REL), Sec. 2.2 */
    int tol_mode;              /* SLM_TOL_ABS or SLM_TOL_REL */
    int max_iter;              /* cycle cap, >= 1 */
    int precision;             /* SLM_FP64 or SLM_FP32_BULK */
    int adjoint;               /* 1: also size the workspace for slm_adjoint (needs SLM_FP64,
                                  odd p and at least two levels); 0: forward only */
    int coarse_op;             /* SLM_COARSE_MODIFIED; SLM_COARSE_REDISC (SLM_FP64 only, no
                                  adjoint, not in a batch); SLM_COARSE_FWD_EULER (odd p,
                                  SLM_FP64 only, no adjoint, not in a batch) */
} slm_desc;

typedef struct slm_plan slm_plan;

typedef struct {
    int iterations;            /* cycles begun; the last met the tolerance if converged */
    int status;                /* SLM_OK, SLM_NOT_CONVERGED, SLM_DIVERGED, SLM_STAGNATED */
    int n_levels;
    double rho0;               /* residual 2-norm after cycle 0's pre-relaxation */
    double rho_final;          /* the last measured residual 2-norm */
    double solve_ms;           /* host wall time of slm_solve */
    long long point_updates;   /* rows of Phi_l applied (relaxation + residual + output), all levels */
    long long gmres_solves;    /* B solves (coarse steps) */
    long long gmres_iters;     /* total GMRES iterations */
} slm_stats;

/* Validate `desc` and build the level hierarchy (Sec. 2.2, 3.4): coarsen by
 * m_l while the level keeps >= 2 time points, more than
 * coarsest_max_points points, fewer than max_levels levels and N_l is a
 * multiple of m_l.  Host only.  *out receives a new plan or NULL. */
int slm_plan_create(const slm_desc *desc, slm_plan **out);
void slm_plan_destroy(slm_plan *plan);

/* Device bytes the plan needs: departure displacements and sigma on every
 * level, coarse-level iterates and right-hand sides, C-point buffers,
 * reduction scratch. */
int slm_plan_workspace_size(const slm_plan *plan, size_t *bytes);

/* Level structure: *n_levels, and for l < min(n_levels, cap): N[l] time
 * steps and m[l] coarsening factor (0 on the coarsest level). */
int slm_plan_levels(const slm_plan *plan, int *n_levels, int *N, int *m, int cap);

/* Bind the caller's workspace (d_ws, >= workspace_size bytes, 256-byte
 * aligned, kept alive and unmodified by the caller while the plan is used)
 * and enqueue the setup: the fine departure points by one ERK step
 * (Sec. 2.1), then per level the backtracked coarse departure points
 * (eq. coarse_depart_interp; SM6) and sigma (eqs. varphi_p_multilevel_def,
 * nu_p_def).  Departure points are stored as displacements in cells,
 * d = (x_i - xi)/h (and the y analogue). */
int slm_plan_setup(slm_plan *plan, void *d_ws, size_t bytes, void *stream);

/* Device views of level l's setup arrays inside the workspace:
 *   *d_disp : [dim][N_l][S] displacements; double, except level 0 of an
 *             FP32-bulk plan, which is float (*disp_is_f32 = 1);
 *   *d_sigma: [dim][N_l][S] double sigma vectors (NULL on level 0). */
int slm_level_arrays(const slm_plan *plan, int level, const void **d_disp,
                     int *disp_is_f32, const void **d_sigma);

/* Launch-shape autotuner of one plan.  Times the level-0 F+C relaxation
 * sweep (Sec. 2.2) for a few launch shapes and keeps the fastest: in 2D the
 * output tile of the LDS-staged SL step (Sec. 4.1; 64x16, 64x32, 128x16 or
 * 128x32 nodes), in 1D the elements per thread and the slice
 * double-buffering of level-0 sweeps that form no residual.  Every shape
 * computes the same products in the same order, so results are bitwise
 * independent of the choice (residual sweeps keep their built-in layout,
 * whose per-interval sums follow the thread layout).  Needs setup
 * (SLM_ENOTSETUP otherwise); d_ws is the workspace bound at setup or NULL,
 * anything else is SLM_EINVAL; the plan's C-point buffers serve as timing
 * scratch (no solve may run on the plan meanwhile).  With a non-NULL
 * cache_path the choice is read from that text file when a line for this
 * plan's shape exists, else measured and appended (one line per shape).
 * Plans without coarsening, and adjoint plans, keep the built-in shapes.
 * Synchronises `stream`. */
int slm_autotune(slm_plan *plan, void *d_ws, size_t bytes, const char *cache_path, void *stream);

/* Launch shape of level l's relaxation step (the SL step of Sec. 2.1 /
 * 4.1 on level 0, eq. (BEOper_2D) on coarse levels) for a call over
 * `nchains` intervals or slices, for tests and profiling: *tiled = 1 + the
 * tile shape index (see slm_autotune) when the 2D level-0 step stages each
 * tile's source window in LDS (0: the plain gather kernel; always 0 in 1D
 * and on coarse levels); *blocks_per_system =
 * workgroups per slice of the batched 2D kernels, whose per-block partial
 * sums are reduced in a fixed order (1 in 1D).  Either pointer may be NULL.
 * Host only. */
int slm_launch_info(const slm_plan *plan, int level, int nchains, int *tiled, int *blocks_per_system);

/* out[k] = Phi_l(n0+k) in[k] for k < count: one level-l time step applied to
 * `count` independent slices (T, [count][S]); n0+count <= N_l.  Level 0 is
 * the SL step S_{p,r}; level l >= 1 is eq. (Phi_multilevel) / (BEOper_2D)
 * with GMRES per the descriptor. */
int slm_apply_phi(slm_plan *plan, int level, int n0, int count,
                  const void *d_in, void *d_out, void *stream);

/* Batched F/C relaxation sweep on level l (Sec. 2.2), every coarse interval
 * in parallel.  `mode`:
 *   SLM_SWEEP_FC  : from C-values c_in [(nc+1)][S] take m steps per interval
 *                   (F- then C-relaxation); write the new C-values to c_out
 *                   (c_out[0] = c_in[0]).
 *   SLM_SWEEP_RES : from c_in take m-1 steps (F-relaxation) and form the
 *                   C-point residual r_{jm} = g_{jm} + Phi v_{jm-1} - c_in[j]
 *                   into res [(nc+1)][S] (res[0] untouched); *h_norm (if not
 *                   NULL) receives ||r||_2 in FP64 (synchronises the stream).
 *   SLM_SWEEP_F   : F-relaxation writing every point of v [(N+1)][S].
 * g is the level's right-hand side [(N+1)][S] or NULL for zero. */
enum { SLM_SWEEP_FC = 0, SLM_SWEEP_RES = 1, SLM_SWEEP_F = 2 };
int slm_relax(slm_plan *plan, int level, int mode, const void *d_g,
              const void *d_c_in, void *d_c_out, void *d_res, void *d_v,
              double *h_norm, void *stream);

/* slm_relax for callers that cannot allocate device memory or bring a
 * scratch workspace per call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * kernels as slm_relax; the residual partial sums and the norm live in a
 * static device array of the library (one per GPU, (SLM_NOALLOC_MAX_CHAINS
 * + 32) doubles = 128.25 KiB, held until the process ends) instead of the
 * plan's workspace, and the GMRES statistics counters are not updated.  The
 * call allocates nothing.  Limits: 1D plans only (SLM_EUNSUPPORTED
 * otherwise); at most SLM_NOALLOC_MAX_CHAINS intervals on the level
 * (SLM_EINVAL otherwise, nothing launched; a plan has at most 65536 time
 * steps, the grid.y limit, so this covers every m >= 4 and nt <= 32768
 * at m = 2).  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (other streams or host
 * threads) race on it and must be serialised by the caller. */
#define SLM_NOALLOC_MAX_CHAINS 16384
int slm_relax_noalloc(slm_plan *plan, int level, int mode, const void *d_g, const void *d_c_in, void *d_c_out,
                      void *d_res, void *d_v, double *h_norm, void *stream);

/* Sequential time stepping: u_{n+1} = S_{p,r}(t_n) u_n for n = 0..nt-1
 * from d_u0 (T, [S]), i.e. forward substitution through the one-step
 * system (eq. one-step) with the fine SL step of Sec. 2.1 (Sec. 4.1 in 2D);
 * this is the serial time-stepping the paper compares MGRIT against
 * (Sec. 5).  store_all: d_u receives [(nt+1)][S]; otherwise only u_{nt}
 * ([S]).  Needs setup (the fine departure points); asynchronous. */
int slm_step(slm_plan *plan, const void *d_u0, void *d_u, int store_all, void *stream);

/* Seeded initial iterate of MGRIT (Sec. 2.2 starts from a random
 * space-time guess, uniform in [0,1); the paper gives no generator).  Writes
 * the C-points (fine time points n = j*m_0, j = 0..nt/m_0; every time point
 * of a plan without coarsening) of d_u: the value at time point n and node k
 * is the top 53 bits of the SplitMix64 output (Steele, Lea & Flood 2014) for
 * the state seed XOR (n*S + k), as a fraction of 2^53, rounded to T.  It is
 * a pure function of (seed, n, k), so any implementation reproduces it.
 * layout SLM_ITERATE_FULL: d_u is [(nt+1)][S] (slm_solve's iterate);
 * SLM_ITERATE_CPOINTS: d_u is [(nt/m_0)+1][S] (slm_solve_cpoints' iterate).
 * Other entries are not touched.  Slice 0 is overwritten by u_0 in the
 * solve.  Needs no setup; asynchronous on `stream`. */
enum { SLM_ITERATE_FULL = 0, SLM_ITERATE_CPOINTS = 1 };
int slm_seed_iterate(slm_plan *plan, uint64_t seed, void *d_u, int layout, void *stream);

/* Linear MGRIT V-cycles (Sec. 2.2; linear variant of SM2) until the
 * tolerance test of the descriptor.  d_u ([(nt+1)][S], T) is in/out: on
 * entry its C-points (every m_0-th slice) are the initial iterate, on exit
 * it holds the approximation of every time point.  d_u0 is u_0.  The
 * residual history rho_k is written to h_hist[k] for k < hist_cap.  Returns
 * the stats status (>= 0) or an error (< 0).  A run stopped by max_iter
 * (SLM_NOT_CONVERGED) completes its last cycle's coarse-grid correction, so
 * the iterate it leaves in d_u is the one the next cycle would start from:
 * calling slm_solve again on it continues the iteration exactly (resume;
 * the relative tolerance then refers to the new call's first residual). */
int slm_solve(slm_plan *plan, const void *d_u0, void *d_u, slm_stats *stats,
              double *h_hist, int hist_cap, void *stream);

/* Forward MGRIT that keeps only the C-points (every m_0-th time slice), the
 * checkpoints from which slm_adjoint recomputes the F-points.  d_c is
 * [(nt/m_0)+1][S] of T, in/out: on entry the initial iterate at the
 * C-points (slice 0 is overwritten by u_0), on exit the converged C-values
 * (slice nt/m_0 is the approximation of u_nt).  Statistics as slm_solve;
 * the final F-relaxation is not run.  Needs at least two levels. */
int slm_solve_cpoints(slm_plan *plan, const void *d_u0, void *d_c, slm_stats *stats,
                      double *h_hist, int hist_cap, void *stream);

/* Gradient of a final-time misfit L(u_nt) through the one-step system
 * (discrete adjoint of eq. one-step): with lambda_nt = d_lamT (= dL/du_nt,
 * [S] double) the adjoint system lambda_n = S_n^T lambda_{n+1} is solved by
 * linear MGRIT in reverse time on the plan's hierarchy, its coarse operator
 * being the transpose S_l^T [I - D_x diag(sx) - D_y diag(sy)]^{-1} of eq.
 * (Phi_multilevel) / (BEOper_2D), with the descriptor's relaxation, GMRES
 * settings and tolerance.  Then, coarse interval by interval, the F-points
 * of u are recomputed from the checkpoints d_c (slm_solve_cpoints output)
 * and lambda is swept back through them, accumulating
 *     dL/dtheta_q = sum_n lambda_{n+1}^T (dS_n/dtheta_q) u_n
 * for every wave-speed coefficient (the alpha terms' coef, then the beta
 * terms'), with dS_n/dtheta from the Lagrange weights' derivative and the
 * tangent of the ERK departure trace.  Outputs: d_grad_u0 = lambda_0 ([S]
 * double), h_grad_theta[n_alpha + n_beta] (host), statistics and residual
 * history of the adjoint MGRIT.  The transposed interpolation is a gather
 * over an inverse stencil index built once per plan (integer counting
 * sort); floating-point sums run in a fixed order, so results are
 * deterministic.  Needs a plan created with desc.adjoint = 1. */
int slm_adjoint(slm_plan *plan, const void *d_c, const void *d_lamT, void *d_grad_u0,
                double *h_grad_theta, slm_stats *stats, double *h_hist, int hist_cap,
                void *stream);

/* ---- Many independent 1D problems solved together (a batch) --------------
 * The level-0 relaxation sweeps of every problem run as one persistent
 * launch over a work list of (problem, coarse interval) items; coarse-level
 * sweeps are batched per (interpolation order, elements per thread) class;
 * convergence is decided per problem on the device, so one V-cycle of the
 * whole batch can be captured once as a HIP graph and replayed until every
 * problem has stopped.  Every problem keeps the semantics (hierarchy,
 * stopping test, iteration count) of slm_solve on its own descriptor.
 * Constraints: dim = 1, odd p, and all descriptors share precision and
 * relax.  Errors of the slm_batch_* calls are reported by
 * slm_last_error(NULL).  Calls on one batch must not overlap. */
typedef struct slm_batch slm_batch;
int slm_batch_create(const slm_desc *descs, int n, slm_batch **out);
void slm_batch_destroy(slm_batch *batch);
int slm_batch_workspace_size(const slm_batch *batch, size_t *bytes);
/* Binds one caller-owned, 256-byte aligned workspace of at least
 * slm_batch_workspace_size() bytes for all problems, runs every problem's
 * setup (departure points, backtracking, sigma) and uploads the batch's
 * work lists. */
int slm_batch_setup(slm_batch *batch, void *d_ws, size_t bytes, void *stream);
/* Autotuner: times the persistent level-0 kernel for a few launch shapes
 * (workgroups per CU, item order) and keeps the fastest.  With a non-NULL
 * cache_path the choice is read from / appended to that text file, keyed
 * by the batch's shapes.  Calls before setup return SLM_ENOTSETUP. */
int slm_batch_tune(slm_batch *batch, const char *cache_path, void *stream);
/* Solve every problem: d_u0[i] / d_u[i] as for slm_solve (T of the batch).
 * stats[i] receives problem i's statistics; h_hist (optional) is
 * [n][hist_cap].  use_graph != 0 replays one captured V-cycle.  Returns
 * SLM_OK when every problem converged, else the largest status. */
int slm_batch_solve(slm_batch *batch, const void *const *d_u0, void *const *d_u, slm_stats *stats,
                    double *h_hist, int hist_cap, int use_graph, void *stream);

const char *slm_strerror(int code);
const char *slm_last_error(const slm_plan *plan);   /* plan may be NULL */

#ifdef __cplusplus
}
#endif
#endif
