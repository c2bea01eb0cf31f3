// slm_plan.hip -- C ABI of the library: plan validation and level hierarchy,
// workspace layout, setup, sequential stepping and the linear MGRIT V-cycle
// driver (Sec. 2.2; linear variant of SM2).
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>

#include "slm_internal.h"

namespace {

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ == kSlotMismatch)                                                      \
            return fail(P, SLM_EINVAL, std::string(#expr) + ": launch shape does not match the " \
                                       "workspace's per-block slots (nothing launched)"); \
        if (e_ != hipSuccess) return fail(P, SLM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

thread_local std::string g_err;

int fail(slm_plan *P, int code, const std::string &msg)
{
    if (P) P->err = msg;
    g_err = msg;
    return code;
}
int fail(const slm_plan &P, int code, const std::string &msg) { return fail(const_cast<slm_plan *>(&P), code, msg); }

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool fill_field(WaveField &f, const slm_wave_term *t, int n)
{
    std::memset(&f, 0, sizeof(f));
    if (n < 0 || n > SLM_MAX_TERMS || (n > 0 && !t)) return false;
    f.n = n;
    for (int k = 0; k < n; ++k) {
        f.coef[k] = t[k].coef; f.kx[k] = t[k].kx; f.px[k] = t[k].px;
        f.ky[k] = t[k].ky; f.py[k] = t[k].py; f.kt[k] = t[k].kt; f.pt[k] = t[k].pt;
    }
    return true;
}

// Bound on |displacement| in cells of a fine step: dt/h * sum |coef|.
double disp_bound(const slm_plan &P)
{
    double a = 0.0, b = 0.0;
    for (const auto &t : P.alpha) a += std::fabs(t.coef);
    for (const auto &t : P.beta) b += std::fabs(t.coef);
    return P.d.dt / (2.0 / P.d.nx) * (a > b ? a : b);
}

ChainArgs base_args(const slm_plan &P, int level)
{
    ChainArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = P.d.nx;
    a.S = P.S;
    a.p = P.d.p;
    a.m = P.lv[level].m;
    a.stride_chain = P.lv[level].m;
    a.disp = ws_at(P, P.lv[level].disp);
    a.sigma = level > 0 ? (const double *)ws_at(P, P.lv[level].sigma) : nullptr;
    a.cin_stride = P.S;
    a.cout_shift = 1;
    a.kmax = P.d.gmres_kmax;
    a.rtol = P.d.gmres_rtol;
    a.counter = (unsigned long long *)ws_at(P, P.counter);
    a.nsmall = level == 0 && disp_bound(P) + P.d.p + 8 < P.d.nx ? 1 : 0;
    if (level == 0) {
        const double f = std::ceil(disp_bound(P)) + P.d.p + 2;
        a.fpad = f < P.d.nx ? (int)f : 0;
    }
    a.adj = P.adj_mode;
    a.Nl = P.lv[level].N;
    a.fwd = level > 0 && P.d.coarse_op == SLM_COARSE_FWD_EULER ? 1 : 0;
    a.ept_hint = P.fine_ept;
    a.dbuf_hint = P.fine_dbuf;
    return a;
}

// Device sum of the residual partial sums of a sweep over nc chains.
hipError_t sum_norm(const slm_plan &P, int nc, double *out, hipStream_t st)
{
    if (P.d.dim == 2 || P.adj_mode) return launch_sum_partials((const double *)ws_at(P, P.part2), nc * P.nb2, out, st);
    return launch_sum_partials((const double *)ws_at(P, P.partial), nc, out, st);
}

hipError_t chain(const slm_plan &P, int level, int nchains, const ChainArgs &a, hipStream_t st)
{
    return P.d.dim == 1 && !a.adj ? launch_chain_1d(P, level, nchains, a, st) : launch_chain_2d(P, level, nchains, a, st);
}

struct Solver {
    slm_plan &P;
    hipStream_t st;
    long long updates = 0;

    char *T(size_t off) const { return ws_at(P, off); }
    size_t sl() const { return (size_t)P.S * P.elem; }

    // Coarse-grid correction of level l >= 1, which starts from a zero
    // iterate with right-hand side G_l: relax, restrict the C-point
    // residual by injection, recurse, correct by injection, F-relax.
    int cycle(int l)
    {
        LevelInfo &L = P.lv[l];
        const int S = P.S;
        if (l == P.L - 1) {                 // coarsest: sequential stepping
            ChainArgs a = base_args(P, l);
            a.m = a.stride_chain = L.N;
            a.nsteps = L.N;
            a.G = T(L.G);
            a.Vout = T(L.V);
            a.write_start = 1;
            a.write_last = 1;
            HIPCHK(chain(P, l, 1, a, st));
            updates += (long long)L.N * S;
            return 0;
        }
        const int m = L.m, nc = L.N / m;
        const bool fcf = P.d.relax == SLM_RELAX_FCF;
        if (fcf) {                          // F- then C-relaxation from zero C-values
            ChainArgs a = base_args(P, l);
            a.nsteps = m;
            a.G = T(L.G);
            a.Cout = T(L.C);
            HIPCHK(chain(P, l, nc, a, st));
            updates += (long long)L.N * S;
        }
        {                                   // F-relaxation + C-point residual -> G_{l+1}
            ChainArgs a = base_args(P, l);
            a.nsteps = m;
            a.G = T(L.G);
            a.Cin = fcf ? T(L.C) : nullptr;
            a.Cref = fcf ? T(L.C) : nullptr;
            a.R = T(P.lv[l + 1].G);
            a.partial = (double *)T(P.partial);
            HIPCHK(chain(P, l, nc, a, st));
            updates += (long long)L.N * S;
        }
        int rc = cycle(l + 1);
        if (rc) return rc;
        HIPCHK(launch_axpy_slices(T(L.C), S, T(P.lv[l + 1].V), S, nc + 1, S, P.elem, fcf ? 0 : 1, st));
        {                                   // F-relaxation writing every point of V_l
            ChainArgs a = base_args(P, l);
            a.nsteps = m - 1;
            a.G = T(L.G);
            a.Cin = T(L.C);
            a.Vout = T(L.V);
            a.write_start = 1;
            a.write_last = 1;
            HIPCHK(chain(P, l, nc, a, st));
            HIPCHK(launch_copy_slices(T(L.V) + (size_t)L.N * sl(), S, T(L.C) + (size_t)nc * sl(), S, 1, S,
                                      P.elem, st));
            updates += (long long)(L.N - nc) * S;
        }
        return 0;
    }
};


// Linear MGRIT driver shared by slm_solve (d_u: every time point in and
// out), slm_solve_cpoints (d_c: C-points in and out) and the adjoint
// (P.adj_mode: the reverse-time adjoint system, d_c receives its C-values).
int solve_core(slm_plan *P, const void *d_u0, void *d_u, void *d_c, slm_stats *stats, double *h_hist, int hist_cap,
               hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int S = P->S;
    const size_t sl = (size_t)S * P->elem;
    char *u = (char *)d_u;
    slm_stats s;
    std::memset(&s, 0, sizeof(s));
    s.n_levels = P->L;
    HIPCHK(hipMemsetAsync(ws_at(*P, P->counter), 0, 2 * sizeof(unsigned long long), st));
    Solver sv{*P, st};
    if (P->L == 1) {                        // no coarsening: sequential stepping
        int rc = slm_step(P, d_u0, d_u, 1, st);
        if (rc) return rc;
        sv.updates += (long long)P->d.nt * S;
        s.status = SLM_OK;
    } else {
        const int m0 = P->lv[0].m, nc0 = P->d.nt / m0;
        const bool fcf = P->d.relax == SLM_RELAX_FCF;
        char *Ca = ws_at(*P, P->lv[0].C), *Cb = ws_at(*P, P->C0b);
        if (u) HIPCHK(launch_copy_slices(Ca, S, u, (long long)m0 * S, nc0 + 1, S, P->elem, st));
        else HIPCHK(launch_copy_slices(Ca, S, d_c, S, nc0 + 1, S, P->elem, st));
        HIPCHK(launch_copy_slices(Ca, S, d_u0, S, 1, S, P->elem, st));
        double *dn = (double *)ws_at(*P, P->norm);
        double rho0 = 0.0;
        int stag = 0;
        double prev = 0.0;
        for (int k = 0;; ++k) {
            char *Cc = Ca;                 // C-values after pre-relaxation
            if (fcf) {
                ChainArgs a = base_args(*P, 0);
                a.nsteps = m0;
                a.Cin = Ca;
                a.Cout = Cb;
                HIPCHK(chain(*P, 0, nc0, a, st));
                sv.updates += (long long)P->d.nt * S;
                Cc = Cb;
            }
            {
                ChainArgs a = base_args(*P, 0);
                a.nsteps = m0;
                a.Cin = Cc;
                a.Cref = Cc;
                a.R = ws_at(*P, P->lv[1].G);
                a.partial = (double *)ws_at(*P, P->partial);
                HIPCHK(chain(*P, 0, nc0, a, st));
                sv.updates += (long long)P->d.nt * S;
            }
            HIPCHK(sum_norm(*P, nc0, dn, st));
            double v = 0.0;
            HIPCHK(hipMemcpyAsync(&v, dn, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const double rho = std::sqrt(v);
            if (h_hist && k < hist_cap) h_hist[k] = rho;
            if (k == 0) rho0 = rho;
            s.iterations = k + 1;
            s.rho_final = rho;
            const double thr = P->d.tol_mode == SLM_TOL_REL ? P->d.tol * rho0 : P->d.tol;
            bool stop = true, last = false;
            if (rho < thr || rho == 0.0) s.status = SLM_OK;
            else if (!std::isfinite(rho)) s.status = SLM_DIVERGED;
            else if (P->d.precision == SLM_FP32_BULK && k > 0 && (stag = rho > 0.95 * prev ? stag + 1 : 0) >= 3)
                s.status = SLM_STAGNATED;
            else if (k >= P->d.max_iter) {
                // cut off: still apply this cycle's correction, so the iterate
                // left is where the next cycle starts (a later call resumes)
                s.status = SLM_NOT_CONVERGED;
                stop = false;
                last = true;
            } else stop = false;
            prev = rho;
            if (stop) {
                Ca = Cc;
                break;
            }
            int rc = sv.cycle(1);
            if (rc) return rc;
            HIPCHK(launch_axpy_slices(Cc + sl, S, ws_at(*P, P->lv[1].V) + sl, S, nc0, S, P->elem, 0, st));
            if (fcf) std::swap(Ca, Cb);     // the corrected C-values become the next cycle's start
            if (last) break;
        }
        s.rho0 = rho0;
        if (u) {
            // output: F-relaxation from the final C-values writes every point
            ChainArgs a = base_args(*P, 0);
            a.nsteps = m0 - 1;
            a.Cin = Ca;
            a.Vout = u;
            a.write_start = 1;
            a.write_last = 1;
            HIPCHK(chain(*P, 0, nc0, a, st));
            HIPCHK(launch_copy_slices(u + (size_t)P->d.nt * sl, S, Ca + (size_t)nc0 * sl, S, 1, S, P->elem, st));
            sv.updates += (long long)(P->d.nt - nc0) * S;
        } else {
            HIPCHK(launch_copy_slices(d_c, S, Ca, S, nc0 + 1, S, P->elem, st));
        }
    }
    unsigned long long cnt[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(cnt, ws_at(*P, P->counter), sizeof(cnt), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    s.gmres_solves = (long long)cnt[0];
    s.gmres_iters = (long long)cnt[1];
    s.point_updates = sv.updates;
    s.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = s;
    return s.status;
}

}  // namespace

void slm_set_error(const std::string &msg) { g_err = msg; }

// ---------------------------------------------------------------------- ABI
extern "C" {

const char *slm_strerror(int code)
{
    switch (code) {
    case SLM_OK: return "ok";
    case SLM_NOT_CONVERGED: return "not converged within max_iter cycles";
    case SLM_DIVERGED: return "diverged";
    case SLM_STAGNATED: return "stagnated at the FP32 floor";
    case SLM_EINVAL: return "invalid argument";
    case SLM_EUNSUPPORTED: return "unsupported";
    case SLM_EWORKSPACE: return "workspace missing or too small";
    case SLM_EHIP: return "HIP runtime error";
    case SLM_ENOTSETUP: return "plan not set up";
    }
    return "unknown";
}

const char *slm_last_error(const slm_plan *plan) { return plan ? plan->err.c_str() : g_err.c_str(); }

int slm_plan_create(const slm_desc *d, slm_plan **out)
{
    if (!out) return fail(nullptr, SLM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(nullptr, SLM_EINVAL, "desc is NULL");
    if (d->dim != 1 && d->dim != 2) return fail(nullptr, SLM_EUNSUPPORTED, "dim must be 1 or 2");
    if (d->nx < 8 || (d->dim == 1 && d->nx > 8192) || (d->dim == 2 && d->nx > 4096))
        return fail(nullptr, SLM_EUNSUPPORTED, "nx out of range (1D: 8..8192, 2D: 8..4096)");
    if (d->nt < 1 || !(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(nullptr, SLM_EINVAL, "nt >= 1 and dt > 0 required");
    if (d->nt > SLM_MAX_NT) return fail(nullptr, SLM_EUNSUPPORTED, "nt above SLM_MAX_NT (65536, the grid.y limit)");
    if (d->p < 1 || d->p > 5) return fail(nullptr, SLM_EUNSUPPORTED, "p must be 1..5");
    if (d->r < 1 || d->r > 5) return fail(nullptr, SLM_EUNSUPPORTED, "r must be 1..5");
    if (d->n_alpha < 1 || d->n_alpha > SLM_MAX_TERMS || !d->alpha) return fail(nullptr, SLM_EINVAL, "alpha needs 1..8 terms");
    if (d->dim == 2 && (d->n_beta < 0 || d->n_beta > SLM_MAX_TERMS || (d->n_beta > 0 && !d->beta)))
        return fail(nullptr, SLM_EINVAL, "beta needs 0..8 terms");
    if (!d->m || d->n_m < 1) return fail(nullptr, SLM_EINVAL, "m list required");
    for (int k = 0; k < d->n_m; ++k)
        if (d->m[k] < 2) return fail(nullptr, SLM_EINVAL, "coarsening factors must be >= 2");
    if (d->max_levels < 1) return fail(nullptr, SLM_EINVAL, "max_levels >= 1 required");
    if (d->relax != SLM_RELAX_F && d->relax != SLM_RELAX_FCF) return fail(nullptr, SLM_EINVAL, "relax must be F or FCF");
    if (d->gmres_kmax < 1 || d->gmres_kmax > SLM_KMAX) return fail(nullptr, SLM_EINVAL, "gmres_kmax must be 1..10");
    if (!(d->gmres_rtol >= 0.0) || !(d->tol >= 0.0)) return fail(nullptr, SLM_EINVAL, "tolerances must be >= 0");
    if (d->tol_mode != SLM_TOL_ABS && d->tol_mode != SLM_TOL_REL) return fail(nullptr, SLM_EINVAL, "bad tol_mode");
    if (d->max_iter < 1) return fail(nullptr, SLM_EINVAL, "max_iter >= 1 required");
    if (d->precision != SLM_FP64 && d->precision != SLM_FP32_BULK) return fail(nullptr, SLM_EINVAL, "bad precision");
    if (d->adjoint != 0 && d->adjoint != 1) return fail(nullptr, SLM_EINVAL, "adjoint must be 0 or 1");
    if (d->coarse_op != SLM_COARSE_MODIFIED && d->coarse_op != SLM_COARSE_REDISC &&
        d->coarse_op != SLM_COARSE_FWD_EULER)
        return fail(nullptr, SLM_EUNSUPPORTED,
                    "coarse_op must be SLM_COARSE_MODIFIED, SLM_COARSE_REDISC or SLM_COARSE_FWD_EULER");
    if (d->coarse_op == SLM_COARSE_REDISC && (d->precision != SLM_FP64 || d->adjoint))
        return fail(nullptr, SLM_EUNSUPPORTED, "the rediscretized coarse operator needs SLM_FP64 and no adjoint");
    if (d->coarse_op == SLM_COARSE_FWD_EULER && (d->precision != SLM_FP64 || d->adjoint))
        return fail(nullptr, SLM_EUNSUPPORTED, "the forward-Euler coarse operator needs SLM_FP64 and no adjoint");
    if (d->adjoint && (d->precision != SLM_FP64 || d->p % 2 == 0))
        return fail(nullptr, SLM_EUNSUPPORTED, "the adjoint needs SLM_FP64 and odd p");
    if (d->adjoint && d->n_alpha + (d->dim == 2 ? d->n_beta : 0) > 16)
        return fail(nullptr, SLM_EUNSUPPORTED, "the adjoint supports at most 16 wave-speed coefficients");

    slm_plan *P = new (std::nothrow) slm_plan();
    if (!P) return fail(nullptr, SLM_EINVAL, "out of host memory");
    P->d = *d;
    P->alpha.assign(d->alpha, d->alpha + d->n_alpha);
    if (d->dim == 2 && d->n_beta > 0) P->beta.assign(d->beta, d->beta + d->n_beta);
    P->mlist.assign(d->m, d->m + d->n_m);
    P->d.alpha = P->alpha.data();
    P->d.beta = P->beta.empty() ? nullptr : P->beta.data();
    P->d.n_beta = (int)P->beta.size();
    P->d.m = P->mlist.data();
    fill_field(P->fa, P->d.alpha, P->d.n_alpha);
    fill_field(P->fb, P->d.beta, P->d.n_beta);
    P->S = d->dim == 1 ? d->nx : d->nx * d->nx;
    P->elem = d->precision == SLM_FP64 ? 8 : 4;

    // level hierarchy
    P->L = 1;
    P->lv[0].N = d->nt;
    for (int l = 0; l + 1 < SLM_MAX_LEVELS; ++l) {
        const int m = P->mlist[l < d->n_m ? l : d->n_m - 1];
        const int N = P->lv[l].N;
        if (l + 1 >= d->max_levels || N + 1 <= d->coarsest_max_points || N % m != 0 || N / m < 1) break;
        P->lv[l].m = m;
        P->lv[l + 1].N = N / m;
        P->L = l + 2;
    }
    P->lv[P->L - 1].m = 0;
    if (P->L > 1 && (d->p % 2) == 0 && d->coarse_op != SLM_COARSE_REDISC) {
        delete P;
        return fail(nullptr, SLM_EUNSUPPORTED, "MGRIT with the modified or forward-Euler coarse operator needs odd p");
    }
    if (d->adjoint && P->L < 2) {
        delete P;
        return fail(nullptr, SLM_EUNSUPPORTED, "the adjoint needs at least two levels");
    }
    P->nq = d->adjoint ? d->n_alpha + (d->dim == 2 ? d->n_beta : 0) : 0;

    // workspace layout
    const size_t S = P->S, el = P->elem, dim = d->dim;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + (bytes ? bytes : 1)); return o; };
    LevelInfo &L0 = P->lv[0];
    L0.disp = take(dim * (size_t)d->nt * S * (d->precision == SLM_FP32_BULK ? 4 : 8));
    P->stab = take((size_t)d->nt * 6 * 2 * SLM_MAX_TERMS * sizeof(double));
    if (d->precision == SLM_FP32_BULK) L0.disp64 = take(dim * (size_t)d->nt * S * 8);
    size_t maxc = 1;
    if (P->L > 1) {
        L0.C = take(((size_t)d->nt / L0.m + 1) * S * el);
        P->C0b = take(((size_t)d->nt / L0.m + 1) * S * el);
        maxc = d->nt / L0.m;
    }
    for (int l = 1; l < P->L; ++l) {
        LevelInfo &L = P->lv[l];
        L.disp = take(dim * (size_t)L.N * S * 8);
        L.sigma = take(dim * (size_t)L.N * S * 8);
        if (dim == 2 && d->precision == SLM_FP32_BULK && d->coarse_op == SLM_COARSE_MODIFIED)
            L.sigma32 = take(dim * (size_t)L.N * S * 4);
        L.V = take(((size_t)L.N + 1) * S * el);
        L.G = take(((size_t)L.N + 1) * S * el);
        if (L.m) {
            L.C = take(((size_t)L.N / L.m + 1) * S * el);
            if ((size_t)(L.N / L.m) > maxc) maxc = L.N / L.m;
        }
    }
    if (d->dim == 2 || d->adjoint) {
        size_t cap2 = 1, capg = 1;
        for (int l = 0; l < P->L; ++l) {
            const size_t nc = P->lv[l].m ? (size_t)P->lv[l].N / P->lv[l].m : 1;
            if (nc > cap2) cap2 = nc;
            if (l > 0 && nc > capg) capg = nc;
        }
        P->cap2 = (int)cap2;
        P->capg = (int)capg;
        P->nb2 = chain2d_blocks((long long)S);
        P->w2 = take(2 * cap2 * S * el);
        P->part2 = take(cap2 * (size_t)P->nb2 * sizeof(double));
        if (P->L > 1) {
            P->g2b = take(capg * S * el);
            P->g2v = take(capg * (SLM_KMAX + 1) * S * el);
            P->g2w = take(2 * capg * S * el);             // w of two consecutive Arnoldi steps
            P->g2s = take(capg * sizeof(Gs2));
            P->g2p = take((3 * capg * (size_t)P->nb2 * SLM_NPART2 + 3 * capg * SLM_NPART2) * sizeof(double));
        }
    }
    if (d->adjoint) {
        const size_t nc0 = (size_t)d->nt / L0.m;
        for (int l = 0; l < P->L; ++l) {
            P->lv[l].idx_end = take((size_t)P->lv[l].N * S * sizeof(int));
            P->lv[l].idx_perm = take((size_t)P->lv[l].N * S * sizeof(int));
            P->lv[l].idx_eps = take(dim * (size_t)P->lv[l].N * S * sizeof(double));
        }
        P->gcap = (int)(nc0 < 64 ? nc0 : 64);
        P->lamC = take((nc0 + 1) * S * sizeof(double));
        P->gU = take((size_t)P->gcap * L0.m * S * sizeof(double));
        P->gL = take(2 * (size_t)P->gcap * S * sizeof(double));
        P->gacc = take(nc0 * (size_t)P->nb2 * 16 * sizeof(double));
        P->gout = take(16 * sizeof(double));
    }
    P->partial = take(maxc * sizeof(double));
    P->norm = take(sizeof(double));
    P->counter = take(2 * sizeof(unsigned long long));
    P->ws_bytes = off;
    *out = P;
    return SLM_OK;
}

void slm_plan_destroy(slm_plan *plan) { delete plan; }

int slm_plan_workspace_size(const slm_plan *P, size_t *bytes)
{
    if (!P || !bytes) return fail(nullptr, SLM_EINVAL, "NULL argument");
    *bytes = P->ws_bytes;
    return SLM_OK;
}

int slm_plan_levels(const slm_plan *P, int *n_levels, int *N, int *m, int cap)
{
    if (!P || !n_levels) return fail(nullptr, SLM_EINVAL, "NULL argument");
    *n_levels = P->L;
    for (int l = 0; l < P->L && l < cap; ++l) {
        if (N) N[l] = P->lv[l].N;
        if (m) m[l] = P->lv[l].m;
    }
    return SLM_OK;
}

int slm_plan_setup(slm_plan *P, void *d_ws, size_t bytes, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!d_ws || bytes < P->ws_bytes) return fail(P, SLM_EWORKSPACE, "workspace smaller than slm_plan_workspace_size()");
    if (((uintptr_t)d_ws & 255) != 0) return fail(P, SLM_EWORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    // Setup and sweep launches put time steps, coarse steps or intervals on
    // grid.y (at most nt of them); gfx950 takes up to 2^31-1 there, but a
    // device that reports less is refused here rather than at a launch.
    int dev = 0, maxy = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&maxy, hipDeviceAttributeMaxGridDimY, dev));
    if (P->d.nt > maxy)
        return fail(P, SLM_EUNSUPPORTED, "nt exceeds the device's grid.y limit (" + std::to_string(maxy) + ")");
    P->ws = (char *)d_ws;
    P->ready = false;
    P->adj_ready = false;                   // the inverse stencil index follows the departure points
    HIPCHK(P->d.dim == 1 ? launch_trace_1d(*P, st) : launch_trace_2d(*P, st));
    for (int l = 1; l < P->L; ++l) {
        if (P->d.coarse_op == SLM_COARSE_REDISC) HIPCHK(launch_trace_redisc(*P, l, st));
        else HIPCHK(P->d.dim == 1 ? launch_backtrack_1d(*P, l, st) : launch_backtrack_2d(*P, l, st));
    }
    P->ready = true;
    return SLM_OK;
}

int slm_level_arrays(const slm_plan *P, int level, const void **d_disp, int *disp_is_f32, const void **d_sigma)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(*P, SLM_ENOTSETUP, "plan not set up");
    if (level < 0 || level >= P->L) return fail(*P, SLM_EINVAL, "level out of range");
    if (d_disp) *d_disp = ws_at(*P, P->lv[level].disp);
    if (disp_is_f32) *disp_is_f32 = (level == 0 && P->d.precision == SLM_FP32_BULK) ? 1 : 0;
    if (d_sigma) *d_sigma = level > 0 ? ws_at(*P, P->lv[level].sigma) : nullptr;
    return SLM_OK;
}

int slm_launch_info(const slm_plan *P, int level, int nchains, int *tiled, int *blocks_per_system)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (level < 0 || level >= P->L || nchains < 1) return fail(*P, SLM_EINVAL, "level or chain count out of range");
    if (tiled) *tiled = P->d.dim == 2 ? chain2d_tiled(*P, level, nchains) : 0;
    if (blocks_per_system) *blocks_per_system = P->d.dim == 2 ? P->nb2 : 1;
    return SLM_OK;
}

int slm_autotune(slm_plan *P, void *d_ws, size_t bytes, const char *cache_path, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (d_ws && (d_ws != (void *)P->ws || bytes < P->ws_bytes))
        return fail(P, SLM_EINVAL, "d_ws must be the workspace bound at setup (or NULL)");
    hipStream_t st = (hipStream_t)stream;
    char key[256];
    std::snprintf(key, sizeof(key), "plan dim=%d nx=%d nt=%d p=%d r=%d prec=%d m0=%d levels=%d", P->d.dim, P->d.nx,
                  P->d.nt, P->d.p, P->d.r, P->d.precision, P->lv[0].m, P->L);
    // a cached choice for this plan shape
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        const std::string pre = std::string(key) + " |";
        while (std::getline(in, line)) {
            if (line.compare(0, pre.size(), pre) != 0) continue;
            int tile = 0, ept = 0, dbuf = -1;
            if (std::sscanf(line.c_str() + pre.size(), " tile=%d ept=%d dbuf=%d", &tile, &ept, &dbuf) == 3 &&
                tile >= 0 && tile < chain2d_num_tiles() && (ept == 0 || ept == 1 || ept == 2 || ept == 4 || ept == 8) &&
                dbuf >= -1 && dbuf <= 1) {
                P->tile2d = tile;
                P->fine_ept = ept;
                P->fine_dbuf = dbuf;
                return SLM_OK;
            }
        }
    }
    struct Cand { int tile, ept, dbuf; };
    std::vector<Cand> cands;
    if (P->L > 1 && !P->d.adjoint) {
        if (P->d.dim == 2) {
            for (int t = 0; t < chain2d_num_tiles(); ++t) cands.push_back({t, 0, -1});
        } else {
            const Cand c1[] = {{0, 0, -1}, {0, 4, 0}, {0, 4, 1}, {0, 8, 0}, {0, 8, 1}};
            for (const Cand &c : c1)
                if (c.ept == 0 || P->d.nx >= 64 * c.ept) cands.push_back(c);
        }
    }
    if (cands.size() > 1) {
        // time the level-0 F+C sweep (Sec. 2.2) of every candidate shape on
        // the plan's own C-point buffers
        const LevelInfo &L0 = P->lv[0];
        const int nc0 = P->d.nt / L0.m;
        HIPCHK(hipMemsetAsync(ws_at(*P, L0.C), 0, ((size_t)nc0 + 1) * P->S * P->elem, st));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return fail(P, SLM_EHIP, "hipEventCreate failed");
        }
        float best = 0.0f;
        Cand bc = cands[0];
        int rc = SLM_OK;
        for (const Cand &c : cands) {
            P->tile2d = c.tile;
            P->fine_ept = c.ept;
            P->fine_dbuf = c.dbuf;
            ChainArgs a = base_args(*P, 0);
            a.nsteps = L0.m;
            a.Cin = ws_at(*P, L0.C);
            a.Cout = ws_at(*P, P->C0b);
            hipError_t e = chain(*P, 0, nc0, a, st);                 // warm-up
            for (int r = 0; e == hipSuccess && r < 3; ++r) {
                if (r == 0) e = hipEventRecord(e0, st);
                if (e == hipSuccess) e = chain(*P, 0, nc0, a, st);
            }
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(P, SLM_EHIP, std::string("autotune timing: ") + hipGetErrorString(e));
                break;
            }
            if (&c == &cands[0] || ms < best) {
                best = ms;
                bc = c;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        P->tile2d = bc.tile;
        P->fine_ept = bc.ept;
        P->fine_dbuf = bc.dbuf;
        if (rc != SLM_OK) return rc;
    }
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (!out) return fail(P, SLM_EINVAL, std::string("cannot append to ") + cache_path);
        out << key << " | tile=" << P->tile2d << " ept=" << P->fine_ept << " dbuf=" << P->fine_dbuf << "\n";
    }
    return SLM_OK;
}

int slm_apply_phi(slm_plan *P, int level, int n0, int count, const void *d_in, void *d_out, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (level < 0 || level >= P->L || n0 < 0 || count < 0 || n0 + count > P->lv[level].N)
        return fail(P, SLM_EINVAL, "level or step range out of bounds");
    if (count == 0) return SLM_OK;
    if (!d_in || !d_out) return fail(P, SLM_EINVAL, "NULL slice pointer");
    ChainArgs a = base_args(*P, level);
    a.m = 1;
    a.stride_chain = 1;
    a.n_base = n0;
    a.nsteps = 1;
    a.Cin = d_in;
    a.Cout = d_out;
    a.cout_shift = 0;
    HIPCHK(chain(*P, level, count, a, (hipStream_t)stream));
    return SLM_OK;
}

int slm_relax(slm_plan *P, int level, int mode, const void *d_g, const void *d_c_in, void *d_c_out, void *d_res,
              void *d_v, double *h_norm, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (level < 0 || level >= P->L - 1) return fail(P, SLM_EINVAL, "level must have a coarser level below it");
    hipStream_t st = (hipStream_t)stream;
    const LevelInfo &L = P->lv[level];
    const int m = L.m, nc = L.N / m;
    ChainArgs a = base_args(*P, level);
    a.G = d_g;
    a.Cin = d_c_in;
    if (mode == SLM_SWEEP_FC) {
        if (!d_c_out) return fail(P, SLM_EINVAL, "c_out required");
        a.nsteps = m;
        a.Cout = d_c_out;
    } else if (mode == SLM_SWEEP_RES) {
        if (!d_res) return fail(P, SLM_EINVAL, "res required");
        a.nsteps = m;
        a.Cref = d_c_in;
        a.R = d_res;
        a.partial = (double *)ws_at(*P, P->partial);
    } else if (mode == SLM_SWEEP_F) {
        if (!d_v) return fail(P, SLM_EINVAL, "v required");
        a.nsteps = m - 1;
        a.Vout = d_v;
        a.write_start = 1;
        a.write_last = 1;
    } else {
        return fail(P, SLM_EINVAL, "bad mode");
    }
    HIPCHK(chain(*P, level, nc, a, st));
    if (mode == SLM_SWEEP_F && d_c_in) {
        HIPCHK(launch_copy_slices((char *)d_v + (size_t)L.N * P->S * P->elem, P->S,
                                  (const char *)d_c_in + (size_t)nc * P->S * P->elem, P->S, 1, P->S, P->elem, st));
    }
    if (mode == SLM_SWEEP_RES && h_norm) {
        double *dn = (double *)ws_at(*P, P->norm);
        HIPCHK(sum_norm(*P, nc, dn, st));
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, dn, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *h_norm = std::sqrt(v);
    }
    return SLM_OK;
}

// Scratch of slm_relax_noalloc: the per-interval residual partial sums
// (SLM_NOALLOC_MAX_CHAINS doubles) followed by the norm.  Each GPU the
// library runs on holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): it passes the address hipGetSymbolAddress returned
// for the current device.
static __device__ __align__(256) double scratch[SLM_NOALLOC_MAX_CHAINS + 32];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t scratch_on_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (double *)ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

int slm_relax_noalloc(slm_plan *P, int level, int mode, const void *d_g, const void *d_c_in, void *d_c_out,
                      void *d_res, void *d_v, double *h_norm, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (P->d.dim != 1 || P->adj_mode)
        return fail(P, SLM_EUNSUPPORTED, "slm_relax_noalloc supports 1D plans only (2D sweeps stage slices in the workspace)");
    if (level < 0 || level >= P->L - 1) return fail(P, SLM_EINVAL, "level must have a coarser level below it");
    hipStream_t st = (hipStream_t)stream;
    const LevelInfo &L = P->lv[level];
    const int m = L.m, nc = L.N / m;
    if (nc > SLM_NOALLOC_MAX_CHAINS)
        return fail(P, SLM_EINVAL, "slm_relax_noalloc: more than SLM_NOALLOC_MAX_CHAINS (" +
                                   std::to_string(SLM_NOALLOC_MAX_CHAINS) + ") intervals on this level");
    double *scr = nullptr;
    HIPCHK(scratch_on_current_device(&scr));
    ChainArgs a = base_args(*P, level);
    a.counter = nullptr;                    // no GMRES statistics: nothing outside the inputs, outputs and scratch
    a.G = d_g;
    a.Cin = d_c_in;
    if (mode == SLM_SWEEP_FC) {
        if (!d_c_out) return fail(P, SLM_EINVAL, "c_out required");
        a.nsteps = m;
        a.Cout = d_c_out;
    } else if (mode == SLM_SWEEP_RES) {
        if (!d_res) return fail(P, SLM_EINVAL, "res required");
        a.nsteps = m;
        a.Cref = d_c_in;
        a.R = d_res;
        a.partial = scr;                    // every interval overwrites its own slot
    } else if (mode == SLM_SWEEP_F) {
        if (!d_v) return fail(P, SLM_EINVAL, "v required");
        a.nsteps = m - 1;
        a.Vout = d_v;
        a.write_start = 1;
        a.write_last = 1;
    } else {
        return fail(P, SLM_EINVAL, "bad mode");
    }
    HIPCHK(chain(*P, level, nc, a, st));
    if (mode == SLM_SWEEP_F && d_c_in) {
        HIPCHK(launch_copy_slices((char *)d_v + (size_t)L.N * P->S * P->elem, P->S,
                                  (const char *)d_c_in + (size_t)nc * P->S * P->elem, P->S, 1, P->S, P->elem, st));
    }
    if (mode == SLM_SWEEP_RES && h_norm) {
        double *dn = scr + SLM_NOALLOC_MAX_CHAINS;
        HIPCHK(launch_sum_partials(scr, nc, dn, st));
        double v = 0.0;
        HIPCHK(hipMemcpyAsync(&v, dn, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *h_norm = std::sqrt(v);
    }
    return SLM_OK;
}

int slm_step(slm_plan *P, const void *d_u0, void *d_u, int store_all, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (!d_u0 || !d_u) return fail(P, SLM_EINVAL, "NULL pointer");
    ChainArgs a = base_args(*P, 0);
    a.m = a.stride_chain = P->d.nt;
    a.nsteps = P->d.nt;
    a.Cin = d_u0;
    if (store_all) {
        a.Vout = d_u;
        a.write_start = 1;
        a.write_last = 1;
    } else {
        a.Cout = d_u;
        a.cout_shift = 0;
    }
    HIPCHK(chain(*P, 0, 1, a, (hipStream_t)stream));
    return SLM_OK;
}

int slm_seed_iterate(slm_plan *P, uint64_t seed, void *d_u, int layout, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!d_u) return fail(P, SLM_EINVAL, "NULL pointer");
    const int m0 = P->lv[0].m > 1 ? P->lv[0].m : 1, nc = P->d.nt / m0;
    long long ls;
    if (layout == SLM_ITERATE_FULL) ls = (long long)m0 * P->S;
    else if (layout == SLM_ITERATE_CPOINTS) ls = P->S;
    else return fail(P, SLM_EINVAL, "layout must be SLM_ITERATE_FULL or SLM_ITERATE_CPOINTS");
    HIPCHK(launch_seed_slices(d_u, ls, nc + 1, P->S, m0, (unsigned long long)seed, P->elem, (hipStream_t)stream));
    return SLM_OK;
}

int slm_solve(slm_plan *P, const void *d_u0, void *d_u, slm_stats *stats, double *h_hist, int hist_cap,
              void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (!d_u0 || !d_u) return fail(P, SLM_EINVAL, "NULL pointer");
    return solve_core(P, d_u0, d_u, nullptr, stats, h_hist, hist_cap, (hipStream_t)stream);
}

int slm_solve_cpoints(slm_plan *P, const void *d_u0, void *d_c, slm_stats *stats, double *h_hist, int hist_cap,
                      void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (!d_u0 || !d_c) return fail(P, SLM_EINVAL, "NULL pointer");
    if (P->L < 2) return fail(P, SLM_EUNSUPPORTED, "C-point checkpoints need at least two levels");
    return solve_core(P, d_u0, nullptr, d_c, stats, h_hist, hist_cap, (hipStream_t)stream);
}

int slm_adjoint(slm_plan *P, const void *d_c, const void *d_lamT, void *d_grad_u0, double *h_grad_theta,
                slm_stats *stats, double *h_hist, int hist_cap, void *stream)
{
    if (!P) return fail(nullptr, SLM_EINVAL, "plan is NULL");
    if (!P->ready) return fail(P, SLM_ENOTSETUP, "plan not set up");
    if (!P->d.adjoint) return fail(P, SLM_EUNSUPPORTED, "plan was created without desc.adjoint = 1");
    if (!d_c || !d_lamT || !d_grad_u0) return fail(P, SLM_EINVAL, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    const long long S = P->S;
    const int m0 = P->lv[0].m, nc0 = P->d.nt / m0;
    // inverse stencil index of every level (once per setup)
    if (!P->adj_ready) {
        for (int l = 0; l < P->L; ++l) HIPCHK(launch_adj_index(*P, l, st));
        P->adj_ready = true;
    }
    // 1. lambda at the C-points: MGRIT on the adjoint system in reverse time,
    //    from a zero initial iterate (C-point 0 of reverse time = lambda_nt)
    double *lamC = (double *)ws_at(*P, P->lamC);
    HIPCHK(launch_fill0(lamC, (nc0 + 1) * S, st));
    P->adj_mode = 1;
    const int rc = solve_core(P, d_lamT, nullptr, lamC, stats, h_hist, hist_cap, st);
    P->adj_mode = 0;
    if (rc < 0) return rc;
    // 2. per coarse interval: recompute u_n from the checkpoint, sweep lambda
    //    back through the interval and accumulate the gradient
    double *gacc = (double *)ws_at(*P, P->gacc);
    HIPCHK(launch_fill0(gacc, (long long)nc0 * P->nb2 * 16, st));
    double *U = (double *)ws_at(*P, P->gU), *Lb = (double *)ws_at(*P, P->gL);
    const double *C = (const double *)d_c;
    for (int c0 = 0; c0 < nc0; c0 += P->gcap) {
        const int nch = nc0 - c0 < P->gcap ? nc0 - c0 : P->gcap;
        const long long us = (long long)m0 * S;
        HIPCHK(launch_copy_slices(U, us, C + (long long)c0 * S, S, nch, (int)S, 8, st));
        for (int k = 0; k + 1 < m0; ++k)
            HIPCHK(launch_step_fwd(*P, nch, U + k * S, us, U + (k + 1) * S, us, (long long)c0 * m0 + k, m0, st));
        // lambda at forward time (c0+c+1) m0 is reverse-time C-point nc0-(c0+c+1)
        for (int c = 0; c < nch; ++c)
            HIPCHK(launch_copy_slices(Lb + (long long)c * S, S, lamC + (long long)(nc0 - (c0 + c + 1)) * S, S, 1,
                                      (int)S, 8, st));
        double *cur = Lb, *nxt = Lb + (long long)P->gcap * S;
        for (int k = m0 - 1; k >= 0; --k) {
            HIPCHK(launch_grad(*P, nch, U + k * S, us, cur, S, (long long)c0 * m0 + k, m0, gacc, st));
            HIPCHK(launch_stepT(*P, 0, nch, cur, S, nxt, S, (long long)c0 * m0 + k, m0, 0, nullptr, nullptr, st));
            std::swap(cur, nxt);
        }
        if (c0 == 0) HIPCHK(launch_copy_slices(d_grad_u0, S, cur, S, 1, (int)S, 8, st));
    }
    double *gout = (double *)ws_at(*P, P->gout);
    HIPCHK(launch_grad_reduce(*P, nc0, gout, st));
    double g[16];
    HIPCHK(hipMemcpyAsync(g, gout, sizeof(g), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (h_grad_theta)
        for (int q = 0; q < P->nq; ++q) h_grad_theta[q] = g[q];
    return rc;
}

}  // extern "C"
