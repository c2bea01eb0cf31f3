// slm_internal.h -- plan structure and kernel launchers (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "slm_common.h"

struct LevelInfo {
    int N = 0;              // time steps on this level
    int m = 0;              // coarsening factor to the next level (0: coarsest)
    size_t disp = 0;        // [dim][N][S] displacements (double; level 0 of bulk: float)
    size_t disp64 = 0;      // level 0 of an FP32-bulk plan: FP64 copy used by setup
    size_t sigma = 0;       // [dim][N][S] double, l >= 1
    size_t sigma32 = 0;     // 2D FP32-bulk plans: [dim][N][S] float copy of sigma for the GMRES matvec
    size_t V = 0;           // [(N+1)][S] T, l >= 1: iterate
    size_t G = 0;           // [(N+1)][S] T, l >= 1: right-hand side
    size_t C = 0;           // [(N/m+1)][S] T: C-point buffer (not on the coarsest level)
    size_t idx_end = 0;     // adjoint: [N][S] int, end of each stencil cell's source list
    size_t idx_perm = 0;    // adjoint: [N][S] int, sources ordered by stencil cell
    size_t idx_eps = 0;     // adjoint: [dim][N][S] double, eps (and nu) of the sources in that order
};

// Per-system Givens state of the batched 2D GMRES.
struct Gs2 {
    double R[SLM_KMAX][SLM_KMAX];    // R[col][row]
    double cs[SLM_KMAX], sn[SLM_KMAX], g[SLM_KMAX + 1], hn[SLM_KMAX];
    double beta;
    int k;                           // iterations done
    int done;
    int need;                        // the step's norm must be reduced from the updated vector
};
#define SLM_NPART2 16

struct slm_plan {
    slm_desc d;                         // copy; pointers below own the arrays
    std::vector<slm_wave_term> alpha, beta;
    std::vector<int> mlist;
    int S = 0;                          // values per spatial slice
    int L = 0;                          // number of levels
    LevelInfo lv[SLM_MAX_LEVELS];
    size_t C0b = 0;                     // second level-0 C-point buffer
    size_t stab = 0;                    // [nt][6 stages][2 fields][SLM_MAX_TERMS] stage factors of the fine trace
    size_t partial = 0;                 // [max intervals] double
    size_t norm = 0;                    // 1 double
    size_t counter = 0;                 // 2 x uint64: gmres solves, iterations
    // 2D: chains per launch batch, ping-pong slices and batched-GMRES state
    int cap2 = 0, capg = 0, nb2 = 0;
    size_t w2 = 0, g2b = 0, g2v = 0, g2w = 0, g2s = 0, g2p = 0, part2 = 0;
    // adjoint: reverse-time mode of the chain kernels, inverse index ready,
    // checkpoint recomputation (gcap chains at a time) and gradient sums
    int adj_mode = 0;
    bool adj_ready = false;
    int gcap = 0, nq = 0;
    size_t lamC = 0, gU = 0, gL = 0, gacc = 0, gout = 0;
    size_t ws_bytes = 0;
    char *ws = nullptr;
    bool ready = false;
    int elem = 8;                       // sizeof(T)
    // launch shapes chosen by slm_autotune (they never change the arithmetic):
    // 2D level-0 tile shape index; 1D level-0 elements per thread and slice
    // double-buffering for sweeps without a residual (0 = built-in choice)
    int tile2d = 0, fine_ept = 0, fine_dbuf = -1;
    std::string err;
    WaveField fa, fb;
};

// Arguments of the batched relaxation ("chain") kernels: every workgroup
// advances one coarse interval j through `nsteps` level steps.
struct ChainArgs {
    int nx, S, m, nsteps, p;
    int n_base;              // global step index of chain 0's first step
    int stride_chain;        // steps between consecutive chains' first steps (= m)
    const void *disp;        // level displacements [dim][N][S]
    const double *sigma;     // [dim][N][S] (coarse levels)
    const void *G;           // [(N+1)][S] or null
    const void *Cin;         // start slices [(nc+1)][S] (chain j starts at Cin[j]) or null => 0
    long long cin_stride;    // elements between consecutive start slices
    void *Vout;              // write every state: Vout[n*S]
    int write_start;         // also write the start slice at Vout[n_first*S]
    int write_last;          // also write the final state into Vout
    void *Cout;              // Cout[(j+cout_shift)*S] = final state
    int cout_shift;          // 1: C-point sweep (chain 0 also writes Cout[0] = start); 0: direct
    const void *Cref;        // residual mode: r = final - Cref[(j+1)*S] (null: zero C-values)
    void *R;                 // residual out R[(j+1)*S]
    double *partial;         // per-chain sum of r^2
    int kmax;
    double rtol;
    unsigned long long *counter;
    int nsmall;              // |displacement| bound < nx - p - 1 (cheap wrap)
    int fpad;                // level 0: periodic copies on each side of the fast sweep's LDS slice
                             // (ceil(|displacement| bound) + p + 2; 0: no padded variant)
    int adj;                 // 1: adjoint system in reverse time (transposed steps)
    int Nl;                  // level steps; step n of the adjoint uses forward step Nl-1-n
    int fwd;                 // coarse level with the explicit forward-Euler operator (eq. Fp_def)
    int ept_hint;            // level 0: elements per thread chosen by the autotuner (0: built-in)
    int dbuf_hint;           // level 0: slice double-buffering chosen by the autotuner (-1: built-in)
};

// launchers (slm_chain1d.hip / slm_setup.hip / slm_misc.hip)
hipError_t launch_trace_1d(const slm_plan &P, hipStream_t st);
hipError_t launch_backtrack_1d(const slm_plan &P, int level, hipStream_t st);
hipError_t launch_trace_redisc(const slm_plan &P, int level, hipStream_t st);
hipError_t launch_chain_1d(const slm_plan &P, int level, int nchains, const ChainArgs &a, hipStream_t st);
hipError_t launch_fine_1d(int nchains, bool f32, const ChainArgs &a, hipStream_t st);
hipError_t launch_trace_2d(const slm_plan &P, hipStream_t st);
hipError_t launch_backtrack_2d(const slm_plan &P, int level, hipStream_t st);
hipError_t launch_chain_2d(const slm_plan &P, int level, int nchains, const ChainArgs &a, hipStream_t st);
int chain2d_blocks(long long S);
int chain2d_tiled(const slm_plan &P, int level, int nchains);
int chain2d_num_tiles();
hipError_t launch_sum_partials(const double *partial, int n, double *out, hipStream_t st);
hipError_t launch_axpy_slices(void *dst, long long dst_stride, const void *src, long long src_stride,
                              int count, int S, int elem, int assign, hipStream_t st);
hipError_t launch_seed_slices(void *u, long long ls, int count, int S, long long nstep, unsigned long long seed,
                              int elem, hipStream_t st);
hipError_t launch_copy_slices(void *dst, long long dst_stride, const void *src, long long src_stride,
                              int count, int S, int elem, hipStream_t st);
// adjoint (slm_adjoint.hip)
hipError_t launch_adj_index(const slm_plan &P, int level, hipStream_t st);
hipError_t launch_stepT(const slm_plan &P, int level, int nch, const double *src, long long src_stride, double *dst,
                        long long dst_stride, long long n_first, int stride, int rev, const double *G, double *Vout,
                        hipStream_t st);
hipError_t launch_step_fwd(const slm_plan &P, int nch, const double *src, long long src_stride, double *dst,
                           long long dst_stride, long long n_first, int stride, hipStream_t st);
hipError_t launch_grad(const slm_plan &P, int nch, const double *U, long long u_stride, const double *lam,
                       long long lam_stride, long long n_first, int stride, double *gacc, hipStream_t st);
hipError_t launch_grad_reduce(const slm_plan &P, int nchains, double *out, hipStream_t st);
hipError_t launch_fill0(double *p, long long n, hipStream_t st);
hipError_t launch_narrow(const double *src, float *dst, long long n, hipStream_t st);

// message returned by slm_last_error(NULL) (slm_plan.hip)
void slm_set_error(const std::string &msg);

inline char *ws_at(const slm_plan &P, size_t off) { return P.ws + off; }

// Per-(interval, block) slot buffers (residual and GMRES partial sums, the
// adjoint's gradient slots) are sized for P.nb2 blocks per interval and a
// fixed number of intervals.  A launcher whose grid would index past them
// returns this code instead of launching; the C ABI reports it as
// SLM_EINVAL.
constexpr hipError_t kSlotMismatch = hipErrorInvalidValue;
inline bool slots_fit(const slm_plan &P, int nb, long long first_interval, long long count, long long capacity)
{
    return nb == P.nb2 && first_interval >= 0 && count >= 0 && first_interval + count <= capacity;
}
