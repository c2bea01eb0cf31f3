// slm_setup.hip -- plan setup kernels: the fine-grid departure trace and the
// per-level backtracking of coarse departure points with the sigma recursion.
//
// Departure points are stored as displacements in cells, d = (x_i - xi)/h
// (and (y_j - eta)/h in 2D), so that x_E = x_{i - floor(d)} and
// eps = d - floor(d) (eq. depart_decompose).
#include "slm_internal.h"

namespace {

// One ERK step of size dt backwards along the characteristic arriving at
// (x, y) at time t_arr (eq. depart_ODE; eqs. SL2D_char1-2).  Returns the
// displacement of the departure point in cells.
template <int R, int DIM>
__device__ __forceinline__ void erk_back(const WaveField &fa, const WaveField &fb, double x, double y,
                                         double t_arr, double dt, double h, double &dx, double &dy)
{
    const Erk e = erk_tableau(R);
    double kx[6], ky[6];
    const double hs = -dt;
#pragma unroll
    for (int s = 0; s < e.s; ++s) {
        double X = x, Y = y;
#pragma unroll
        for (int q = 0; q < s; ++q) {
            X += hs * e.a[s][q] * kx[q];
            if (DIM == 2) Y += hs * e.a[s][q] * ky[q];
        }
        const double ts = t_arr + e.c[s] * hs;
        kx[s] = wave_eval(fa, X, Y, ts);
        ky[s] = DIM == 2 ? wave_eval(fb, X, Y, ts) : 0.0;
    }
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int s = 0; s < e.s; ++s) {
        sx += e.b[s] * kx[s];
        sy += e.b[s] * ky[s];
    }
    dx = dt * sx / h;
    dy = dt * sy / h;
}

// The wave-speed terms of the fine trace, split into the factor that is the
// same for every node of a stage (coefficient, time factor, and the space
// factors of zero wavenumber; in 1D also the y factor at y = 0) and the
// per-node space factors.  The products are those of wave_eval, taken in a
// different order.
template <int DIM>
__device__ __forceinline__ void stage_factors(const WaveField &f, double ts, double (&u)[SLM_MAX_TERMS])
{
    for (int k = 0; k < f.n; ++k) {
        double v = f.coef[k] * cos(f.kt[k] * SLM_PI * ts + f.pt[k]);
        if (f.kx[k] == 0.0) v *= cos(f.px[k]);
        if (DIM == 1 || f.ky[k] == 0.0) v *= cos(f.ky[k] * SLM_PI * 0.0 + f.py[k]);
        u[k] = v;
    }
}

template <int DIM>
__device__ __forceinline__ double node_eval(const WaveField &f, const double (&u)[SLM_MAX_TERMS], double X, double Y)
{
    double s = 0.0;
    for (int k = 0; k < f.n; ++k) {
        double v = u[k];
        if (f.kx[k] != 0.0) v *= cos(f.kx[k] * SLM_PI * X + f.px[k]);
        if (DIM == 2 && f.ky[k] != 0.0) v *= cos(f.ky[k] * SLM_PI * Y + f.py[k]);
        s += v;
    }
    return s;
}

// The stage factors of every fine step (stage_factors for step n, stage s,
// field f, term k at tab[((n*6 + s)*2 + f)*SLM_MAX_TERMS + k]): the same for
// every node of the step, so they are evaluated once here instead of in
// every thread of the trace.
template <int R, int DIM>
__global__ void stage_table_kernel(int nt, double dt, WaveField fa, WaveField fb, double *tab)
{
    const Erk e = erk_tableau(R);
    const int n = blockIdx.x;
    if (n >= nt) return;
    const double hs = -dt, t_arr = (n + 1) * dt;
    for (int i = threadIdx.x; i < e.s * 2; i += blockDim.x) {
        const int s = i >> 1, f = i & 1;
        const double ts = t_arr + e.c[s] * hs;
        double u[SLM_MAX_TERMS];
        stage_factors<DIM>(f ? fb : fa, ts, u);
        double *o = tab + (((long long)n * 6 + s) * 2 + f) * SLM_MAX_TERMS;
        for (int k = 0; k < (f ? fb.n : fa.n); ++k) o[k] = u[k];
    }
}

// Fine departure trace: trace_npt nodes of one step per thread.
template <int DIM>
constexpr int trace_npt() { return DIM == 1 ? 2 : 1; }

template <int R, int DIM>
__global__ void __launch_bounds__(256) trace_kernel(int nx, long long S, int nt, double dt, double h, WaveField fa,
                                                    WaveField fb, const double *__restrict__ tab, double *out64,
                                                    float *out32)
{
    constexpr int NPT = trace_npt<DIM>();
    const Erk e = erk_tableau(R);
    const int n = blockIdx.y;
    const long long id0 = (long long)blockIdx.x * blockDim.x * NPT + threadIdx.x;
    double x[NPT], y[NPT], kx[NPT][6], ky[NPT][6];
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const long long id = id0 + (long long)j * blockDim.x;
        int i = 0, jy = 0;
        if (id < S) split_xy(id, nx, i, jy);
        x[j] = -1.0 + i * h;
        y[j] = DIM == 2 ? -1.0 + jy * h : 0.0;
    }
    const double hs = -dt, t_arr = (n + 1) * dt;
    double ua[SLM_MAX_TERMS], ub[SLM_MAX_TERMS];
#pragma unroll
    for (int s = 0; s < e.s; ++s) {
        const double *ts = tab + ((long long)n * 6 + s) * 2 * SLM_MAX_TERMS;
        for (int k = 0; k < fa.n; ++k) ua[k] = ts[k];
        if (DIM == 2)
            for (int k = 0; k < fb.n; ++k) ub[k] = ts[SLM_MAX_TERMS + k];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            double X = x[j], Y = y[j];
#pragma unroll
            for (int q = 0; q < s; ++q) {
                X += hs * e.a[s][q] * kx[j][q];
                if (DIM == 2) Y += hs * e.a[s][q] * ky[j][q];
            }
            kx[j][s] = node_eval<DIM>(fa, ua, X, Y);
            ky[j][s] = DIM == 2 ? node_eval<DIM>(fb, ub, X, Y) : 0.0;
        }
    }
    const long long plane = (long long)nt * S;
#pragma unroll
    for (int j = 0; j < NPT; ++j) {
        const long long id = id0 + (long long)j * blockDim.x;
        if (id >= S) continue;
        double sx = 0.0, sy = 0.0;
#pragma unroll
        for (int s = 0; s < e.s; ++s) {
            sx += e.b[s] * kx[j][s];
            sy += e.b[s] * ky[j][s];
        }
        const double dx = dt * sx / h, dy = dt * sy / h;
        const long long o = (long long)n * S + id;
        if (out64) {
            out64[o] = dx;
            if (DIM == 2) out64[plane + o] = dy;
        }
        if (out32) {
            out32[o] = (float)dx;
            if (DIM == 2) out32[plane + o] = (float)dy;
        }
    }
}

// Backtracking of Sec. 3.3.1 in displacement form.  The current point of
// the coarse characteristic is X = i - D (cells).  With E = ceil(X) =
// i - floor(D) and theta = D - floor(D), the linear interpolant of the
// sub-step's departure map moves it to X - [(1-theta) d_E + theta d_W].
// phi (eq. varphi_p_multilevel_def) and sigma (eq. nu_p_def) follow.
__global__ void backtrack1d_kernel(int nx, int m, int Nl, int p, const double *__restrict__ dprev,
                                   const double *__restrict__ sprev, double *__restrict__ dcur,
                                   double *__restrict__ scur)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (i >= nx || n >= Nl) return;
    const long long base = (long long)n * m;
    double D = dprev[(base + m - 1) * nx + i];
    for (int k = m - 2; k >= 0; --k) {
        const double fl = floor(D), th = D - fl;
        const int E = i - (int)fl;
        const int e = wrap_mod(E, nx), w = wrap_mod(E - 1, nx);
        const double *dk = dprev + (base + k) * nx;
        D = D + (1.0 - th) * dk[e] + th * dk[w];
    }
    dcur[(long long)n * nx + i] = D;
    const double sgn = ((p + 1) & 1) ? -1.0 : 1.0;
    double fs = 0.0, acc = 0.0;
    for (int k = 0; k < m; ++k) {
        const double dk = dprev[(base + k) * nx + i];
        fs += fpoly_odd(p, dk - floor(dk));
        if (sprev) acc += sprev[(base + k) * nx + i];
    }
    scur[(long long)n * nx + i] = acc + sgn * (fpoly_odd(p, D - floor(D)) - fs);
}

// 2D backtracking (SM6): bilinear fit over the cell (W..E) x (S..N) around
// the current point of how the four neighbouring fine characteristics move
// their arrival point, separately for the x and y components.  With
// theta_x = Dx - floor(Dx), theta_y = Dy - floor(Dy) the fit is the tensor
// product of the 1D weights (1-theta, theta) on (E, W) and (N, S).
__global__ void backtrack2d_kernel(int nx, int m, int Nl, int p, const double *__restrict__ dprev,
                                   const double *__restrict__ sprev, double *__restrict__ dcur,
                                   double *__restrict__ scur, long long plane_prev, long long plane_cur)
{
    const long long S = (long long)nx * nx;
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (id >= S || n >= Nl) return;
    int i, jy;
    split_xy(id, nx, i, jy);
    const long long base = (long long)n * m;
    const double *px = dprev, *py = dprev + plane_prev;
    double Dx = px[(base + m - 1) * S + id], Dy = py[(base + m - 1) * S + id];
    for (int k = m - 2; k >= 0; --k) {
        const double fx = floor(Dx), tx = Dx - fx, fy = floor(Dy), ty = Dy - fy;
        const int E = wrap_mod(i - (int)fx, nx), W = wrap_mod(i - (int)fx - 1, nx);
        const int N = wrap_mod(jy - (int)fy, nx), Sd = wrap_mod(jy - (int)fy - 1, nx);
        const double *ax = px + (base + k) * S, *ay = py + (base + k) * S;
        const long long NE = (long long)N * nx + E, NW = (long long)N * nx + W;
        const long long SE = (long long)Sd * nx + E, SW = (long long)Sd * nx + W;
        const double wNE = (1.0 - tx) * (1.0 - ty), wNW = tx * (1.0 - ty);
        const double wSE = (1.0 - tx) * ty, wSW = tx * ty;
        const double ddx = wNE * ax[NE] + wNW * ax[NW] + wSE * ax[SE] + wSW * ax[SW];
        const double ddy = wNE * ay[NE] + wNW * ay[NW] + wSE * ay[SE] + wSW * ay[SW];
        Dx += ddx;
        Dy += ddy;
    }
    dcur[(long long)n * S + id] = Dx;
    dcur[plane_cur + (long long)n * S + id] = Dy;
    const double sgn = ((p + 1) & 1) ? -1.0 : 1.0;
    double fsx = 0.0, fsy = 0.0, ax = 0.0, ay = 0.0;
    for (int k = 0; k < m; ++k) {
        const double dkx = px[(base + k) * S + id], dky = py[(base + k) * S + id];
        fsx += fpoly_odd(p, dkx - floor(dkx));
        fsy += fpoly_odd(p, dky - floor(dky));
        if (sprev) {
            ax += sprev[(base + k) * S + id];
            ay += sprev[plane_prev + (base + k) * S + id];
        }
    }
    scur[(long long)n * S + id] = ax + sgn * (fpoly_odd(p, Dx - floor(Dx)) - fsx);
    scur[plane_cur + (long long)n * S + id] = ay + sgn * (fpoly_odd(p, Dy - floor(Dy)) - fsy);
}

// Rediscretized coarse operator (Sec. 2.3): the departure point of a level-l
// step of size M dt (M = m^l fine steps) traced through the M fine-size ERK
// steps it spans, the position carried from one to the next (unwrapped).
template <int R, int DIM>
__global__ void trace_redisc_kernel(int nx, long long S, int Nl, int M, double dt, double h, WaveField fa,
                                    WaveField fb, double *out)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = blockIdx.y;
    if (id >= S || n >= Nl) return;
    int i, jy;
    split_xy(id, nx, i, jy);
    const double x0 = -1.0 + i * h, y0 = DIM == 2 ? -1.0 + jy * h : 0.0;
    double x = x0, y = y0;
    for (int s = M - 1; s >= 0; --s) {
        double dx, dy;
        erk_back<R, DIM>(fa, fb, x, y, ((double)n * M + s + 1) * dt, dt, h, dx, dy);
        x -= dx * h;
        if (DIM == 2) y -= dy * h;
    }
    out[(long long)n * S + id] = (x0 - x) / h;
    if (DIM == 2) out[(long long)Nl * S + (long long)n * S + id] = (y0 - y) / h;
}

template <int DIM>
hipError_t trace_dispatch(const slm_plan &P, hipStream_t st)
{
    const LevelInfo &L0 = P.lv[0];
    const bool f32 = P.d.precision == SLM_FP32_BULK;
    double *o64 = (double *)ws_at(P, f32 ? L0.disp64 : L0.disp);
    float *o32 = f32 ? (float *)ws_at(P, L0.disp) : nullptr;
    const double h = 2.0 / P.d.nx;
    constexpr int NPT = trace_npt<DIM>();
    double *tab = (double *)ws_at(P, P.stab);
    dim3 grid((unsigned)((P.S + 256 * NPT - 1) / (256 * NPT)), (unsigned)P.d.nt);
#define TR(RR) do { \
        hipLaunchKernelGGL((stage_table_kernel<RR, DIM>), dim3((unsigned)P.d.nt), dim3(64), 0, st, P.d.nt, P.d.dt, \
                           P.fa, P.fb, tab); \
        hipLaunchKernelGGL((trace_kernel<RR, DIM>), grid, dim3(256), 0, st, P.d.nx, (long long)P.S, P.d.nt, P.d.dt, \
                           h, P.fa, P.fb, (const double *)tab, o64, o32); \
    } while (0)
    switch (P.d.r) {
    case 1: TR(1); break;
    case 2: TR(2); break;
    case 3: TR(3); break;
    case 4: TR(4); break;
    default: TR(5); break;
    }
#undef TR
    return hipGetLastError();
}

// FP64 displacement array of level l as read by setup.
const double *setup_disp(const slm_plan &P, int l)
{
    if (l == 0 && P.d.precision == SLM_FP32_BULK) return (const double *)ws_at(P, P.lv[0].disp64);
    return (const double *)ws_at(P, P.lv[l].disp);
}

}  // namespace

hipError_t launch_trace_1d(const slm_plan &P, hipStream_t st) { return trace_dispatch<1>(P, st); }
hipError_t launch_trace_2d(const slm_plan &P, hipStream_t st) { return trace_dispatch<2>(P, st); }

hipError_t launch_trace_redisc(const slm_plan &P, int l, hipStream_t st)
{
    int M = 1;
    for (int k = 0; k < l; ++k) M *= P.lv[k].m;
    const LevelInfo &cur = P.lv[l];
    const double h = 2.0 / P.d.nx;
    dim3 grid((unsigned)((P.S + 255) / 256), (unsigned)cur.N);
    double *out = (double *)ws_at(P, cur.disp);
#define RD(RR, DD) hipLaunchKernelGGL((trace_redisc_kernel<RR, DD>), grid, dim3(256), 0, st, P.d.nx, (long long)P.S, \
                                      cur.N, M, P.d.dt, h, P.fa, P.fb, out)
#define RDR(DD) switch (P.d.r) { case 1: RD(1, DD); break; case 2: RD(2, DD); break; case 3: RD(3, DD); break; \
                                 case 4: RD(4, DD); break; default: RD(5, DD); break; }
    if (P.d.dim == 1) RDR(1) else RDR(2)
#undef RDR
#undef RD
    return hipGetLastError();
}

hipError_t launch_backtrack_1d(const slm_plan &P, int l, hipStream_t st)
{
    const LevelInfo &prev = P.lv[l - 1], &cur = P.lv[l];
    dim3 grid((unsigned)((P.d.nx + 255) / 256), (unsigned)cur.N);
    hipLaunchKernelGGL(backtrack1d_kernel, grid, dim3(256), 0, st, P.d.nx, prev.m, cur.N, P.d.p,
                       setup_disp(P, l - 1), l > 1 ? (const double *)ws_at(P, prev.sigma) : nullptr,
                       (double *)ws_at(P, cur.disp), (double *)ws_at(P, cur.sigma));
    return hipGetLastError();
}

hipError_t launch_backtrack_2d(const slm_plan &P, int l, hipStream_t st)
{
    const LevelInfo &prev = P.lv[l - 1], &cur = P.lv[l];
    dim3 grid((unsigned)((P.S + 255) / 256), (unsigned)cur.N);
    hipLaunchKernelGGL(backtrack2d_kernel, grid, dim3(256), 0, st, P.d.nx, prev.m, cur.N, P.d.p,
                       setup_disp(P, l - 1), l > 1 ? (const double *)ws_at(P, prev.sigma) : nullptr,
                       (double *)ws_at(P, cur.disp), (double *)ws_at(P, cur.sigma),
                       (long long)prev.N * P.S, (long long)cur.N * P.S);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !cur.sigma32) return e;
    // FP32 bulk: the GMRES matvec reads sigma rounded to float (sigma itself
    // stays FP64 and feeds the next level's recursion)
    return launch_narrow((const double *)ws_at(P, cur.sigma), (float *)ws_at(P, cur.sigma32),
                         2LL * cur.N * P.S, st);
}
