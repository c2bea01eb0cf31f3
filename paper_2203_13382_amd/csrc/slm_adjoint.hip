// slm_adjoint.hip -- kernels of the discrete adjoint (gradient of a
// final-time misfit through the one-step system u_{n+1} = S_n u_n).
//
// Transposed interpolation.  S_n^T scatters every node's interpolation
// weights onto the p+1 (1D) or (p+1)^2 (2D) nodes of its stencil.  The
// scatter is turned into a gather: for each level step an inverse index
// lists, per stencil cell (the node x_E east of the departure point), the
// nodes whose departure points fall in that cell, in ascending order.  A
// target node then visits the p+1 cells per axis whose stencils cover it
// and sums the weights of their sources.  The index is a counting sort with
// integer atomics; the floating-point sums use no atomics and run in a
// fixed order, so every result is deterministic.
//
// Gradient.  dL/dtheta_q = sum_n lambda_{n+1}^T (dS_n/dtheta_q) u_n with
// dS_n/dtheta_q u_n = sum_stencil (w'(eps) deps/dtheta_q w(nu) + w(eps)
// w'(nu) dnu/dtheta_q) u_n, where eps, nu move with the departure point:
// deps/dtheta = -dxi/dtheta / h, and dxi/dtheta is the tangent of the ERK
// trace (Sec. 2.1) differentiated through its stages.
#include "slm_internal.h"

namespace {

constexpr int TPB = 256;
constexpr int NQ = 16;              // gradient slots per block (n_alpha + n_beta <= 16)

int nblk(long long S)
{
    long long b = (S + TPB - 1) / TPB;
    return (int)(b < 1024 ? b : 1024);
}

// Stencil cell of source k at a step: the (wrapped) node east of its
// departure point, E = k - floor(d) per axis.
__device__ __forceinline__ int cell_of(long long k, int nx, int dim, double dx, double dy)
{
    int ix, iy;
    split_xy(k, nx, ix, iy);
    const int ex = wrap_mod(ix - (int)floor(dx), nx);
    if (dim == 1) return ex;
    const int ey = wrap_mod(iy - (int)floor(dy), nx);
    return ey * nx + ex;
}

__global__ void __launch_bounds__(TPB) idx_clear(int *end, long long n)
{
    for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < n; i += (long long)gridDim.x * TPB) end[i] = 0;
}

__global__ void __launch_bounds__(TPB) idx_count(const double *__restrict__ disp, long long plane, long long S, int nx,
                                                 int dim, int *end)
{
    const long long n = blockIdx.y;
    for (long long k = (long long)blockIdx.x * TPB + threadIdx.x; k < S; k += (long long)gridDim.x * TPB) {
        const double dx = disp[n * S + k], dy = dim == 2 ? disp[plane + n * S + k] : 0.0;
        atomicAdd(&end[n * S + cell_of(k, nx, dim, dx, dy)], 1);
    }
}

// Exclusive prefix sum of one step's S counts, in place (one workgroup per
// step; each thread scans a contiguous chunk).
__global__ void __launch_bounds__(1024) idx_scan(int *cnt, long long S)
{
    __shared__ int tot[1024];
    int *c = cnt + (long long)blockIdx.x * S;
    const long long ch = (S + 1023) / 1024;
    const long long lo = threadIdx.x * ch, hi = lo + ch < S ? lo + ch : S;
    int s = 0;
    for (long long i = lo; i < hi; ++i) s += c[i];
    tot[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int v = tot[t];
            tot[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int run = tot[threadIdx.x];
    for (long long i = lo; i < hi; ++i) {
        const int v = c[i];
        c[i] = run;
        run += v;
    }
}

// Place every source at the next free slot of its cell; afterwards end[c]
// holds the end of cell c's list (= the start of cell c+1).
__global__ void __launch_bounds__(TPB) idx_fill(const double *__restrict__ disp, long long plane, long long S, int nx,
                                                int dim, int *end, int *perm)
{
    const long long n = blockIdx.y;
    for (long long k = (long long)blockIdx.x * TPB + threadIdx.x; k < S; k += (long long)gridDim.x * TPB) {
        const double dx = disp[n * S + k], dy = dim == 2 ? disp[plane + n * S + k] : 0.0;
        const int pos = atomicAdd(&end[n * S + cell_of(k, nx, dim, dx, dy)], 1);
        perm[n * S + pos] = (int)k;
    }
}

// Sort each cell's (short) list ascending: the summation order of the
// gather no longer depends on the order of the atomics.
__global__ void __launch_bounds__(TPB) idx_sort(const int *__restrict__ end, int *perm, long long S)
{
    const long long n = blockIdx.y;
    for (long long c = (long long)blockIdx.x * TPB + threadIdx.x; c < S; c += (long long)gridDim.x * TPB) {
        const int lo = c ? end[n * S + c - 1] : 0, hi = end[n * S + c];
        int *q = perm + n * S;
        for (int i = lo + 1; i < hi; ++i) {
            const int v = q[i];
            int j = i - 1;
            while (j >= lo && q[j] > v) {
                q[j + 1] = q[j];
                --j;
            }
            q[j + 1] = v;
        }
    }
}

// Fractional parts of the sources' displacements in index order, so the
// gather reads them contiguously.
__global__ void __launch_bounds__(TPB) idx_eps(const double *__restrict__ disp, long long plane, long long S,
                                               int dim, const int *__restrict__ perm, double *eps, long long eplane)
{
    const long long n = blockIdx.y;
    for (long long q = (long long)blockIdx.x * TPB + threadIdx.x; q < S; q += (long long)gridDim.x * TPB) {
        const int k = perm[n * S + q];
        const double dx = disp[n * S + k];
        eps[n * S + q] = dx - floor(dx);
        if (dim == 2) {
            const double dy = disp[plane + n * S + k];
            eps[eplane + n * S + q] = dy - floor(dy);
        }
    }
}

// Lagrange weights and their derivatives with respect to eps at the
// departure point (odd p: stencil nodes E-l .. E+r, fixed in eps).
template <int P>
__device__ __forceinline__ void weights_eps(double eps, double (&w)[P + 1], double (&dw)[P + 1])
{
    const double z = -eps + (double)((P + 1) / 2);     // shifted variable, nodes 0..P
    lagrange_weights<P, double>(z, w);
    constexpr double fact[6] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0};
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l <= P; ++l) {
            if (l == j) continue;
            double pr = 1.0;
#pragma unroll
            for (int k = 0; k <= P; ++k)
                if (k != j && k != l) pr *= z - (double)k;
            s += pr;
        }
        const double inv = ((P - j) & 1 ? -1.0 : 1.0) / (fact[j] * fact[P - j]);
        dw[j] = -s * inv;                                 // d/deps = -d/dz
    }
}

// One Lagrange weight of the stencil: node j (0..P) at the shifted point z,
// prod_{k != j} (z - k) / prod_{k != j} (j - k).
template <int P>
__device__ __forceinline__ double lweight(double z, int j)
{
    double pr = 1.0;
#pragma unroll
    for (int k = 0; k <= P; ++k)
        if (k != j) pr *= z - (double)k;
    // 1 / prod_{k != j} (j - k) = (-1)^{P-j} / (j! (P-j)!)
    constexpr double f[6] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0};
    double inv = 1.0;
#pragma unroll
    for (int t = 0; t <= P; ++t)
        if (t == j) inv = ((P - t) & 1 ? -1.0 : 1.0) / (f[t] * f[P - t]);
    return pr * inv;
}

// dst[c] = S^T(step) src[c] (+ G[n+1]); step = n, or Nl-1-n when rev.
// Target t visits the p+1 cells per axis whose stencils cover it; the cell
// fixes t's node index in each source's stencil, so a source costs its
// loads and two single Lagrange weights (no index arithmetic per source).
template <int P>
__global__ void __launch_bounds__(TPB) stepT_kernel(const double *__restrict__ src, long long src_stride,
                                                    double *__restrict__ dst, long long dst_stride,
                                                    const double *__restrict__ eps, long long eplane,
                                                    const int *__restrict__ end, const int *__restrict__ perm,
                                                    int nx, int dim, long long S, long long n_first, int stride,
                                                    int rev, int Nl, const double *__restrict__ G,
                                                    double *__restrict__ Vout)
{
    constexpr int ell = (P + 1) / 2;
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const long long nd = rev ? Nl - 1 - n : n;
    const double *lam = src + c * src_stride;
    const double *exs = eps + nd * S, *eys = eps + eplane + nd * S;
    const int *en = end + nd * S, *pm = perm + nd * S;
    // Each block takes a contiguous run of targets, and consecutive runs go
    // to the same XCD (the dispatcher deals blocks to the 8 XCDs in turn):
    // neighbouring target rows read overlapping cell lists, which then meet
    // in one L2 instead of being fetched once per XCD.
    const long long nb = gridDim.x, per = (S + nb - 1) / nb, lb = xcd_block(blockIdx.x, nb);
    const long long t_end = (lb + 1) * per < S ? (lb + 1) * per : S;
    for (long long t = lb * per + threadIdx.x; t < t_end; t += TPB) {
        int tx, ty;
        split_xy(t, nx, tx, ty);
        if (dim != 2) ty = 0;
        double acc = 0.0;
        const int nby = dim == 2 ? P : 0;
        // the source ranges of all the target's cells first (independent
        // loads), then the sources cell by cell in the same order as before
        int lo[P + 1][P + 1], hi[P + 1][P + 1];
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            int ey = 0;
            if (dim == 2) {
                ey = ty + ell - b;
                ey += ey < 0 ? nx : 0;
                ey -= ey >= nx ? nx : 0;
            }
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                int ex = tx + ell - a;
                ex += ex < 0 ? nx : 0;
                ex -= ex >= nx ? nx : 0;
                const long long cell = (long long)ey * nx + ex;
                lo[b][a] = (b <= nby && cell) ? en[cell - 1] : 0;
                hi[b][a] = b <= nby ? en[cell] : 0;
            }
        }
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            if (b > nby) break;
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                for (int q = lo[b][a]; q < hi[b][a]; ++q) {
                    double wv = lweight<P>(-exs[q] + (double)ell, a);
                    if (dim == 2) wv *= lweight<P>(-eys[q] + (double)ell, b);
                    acc += wv * lam[pm[q]];
                }
            }
        }
        if (G) acc += G[(n + 1) * S + t];
        dst[c * dst_stride + t] = acc;
        if (Vout) Vout[(n + 1) * S + t] = acc;
    }
}

// Forward level-0 step in 1D or 2D (recomputation of F-points):
// dst[c] = S_n src[c], n = n_first + c*stride.
template <int P>
__global__ void __launch_bounds__(TPB) stepF_kernel(const double *__restrict__ src, long long src_stride,
                                                    double *__restrict__ dst, long long dst_stride,
                                                    const double *__restrict__ disp, long long plane, int nx,
                                                    int dim, long long S, long long n_first, int stride)
{
    constexpr int ell = (P + 1) / 2;
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const double *u = src + c * src_stride;
    for (long long t = (long long)blockIdx.x * TPB + threadIdx.x; t < S; t += (long long)gridDim.x * TPB) {
        int tx, ty;
        split_xy(t, nx, tx, ty);
        if (dim != 2) ty = 0;
        const double dx = disp[n * S + t];
        const double fx = floor(dx);
        double wx[P + 1];
        lagrange_weights<P, double>(-(dx - fx) + (double)ell, wx);
        const int bx = wrap_mod(tx - (int)fx - ell, nx);
        double acc = 0.0;
        if (dim == 1) {
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                int col = bx + a;
                col -= col >= nx ? nx : 0;
                acc += wx[a] * u[col];
            }
        } else {
            const double dy = disp[plane + n * S + t];
            const double fy = floor(dy);
            double wy[P + 1];
            lagrange_weights<P, double>(-(dy - fy) + (double)ell, wy);
            const int by = wrap_mod(ty - (int)fy - ell, nx);
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                int row = by + b;
                row -= row >= nx ? nx : 0;
                double ar = 0.0;
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    int col = bx + a;
                    col -= col >= nx ? nx : 0;
                    ar += wx[a] * u[(long long)row * nx + col];
                }
                acc += wy[b] * ar;
            }
        }
        dst[c * dst_stride + t] = acc;
    }
}

// Value and x/y partial derivatives of one wave term without its coefficient.
__device__ __forceinline__ void term_d(const WaveField &f, int k, double x, double y, double t, double &v, double &gx,
                                       double &gy)
{
    const double ax = f.kx[k] * SLM_PI * x + f.px[k], ay = f.ky[k] * SLM_PI * y + f.py[k];
    const double ct = cos(f.kt[k] * SLM_PI * t + f.pt[k]);
    const double cx = cos(ax), cy = cos(ay);
    v = cx * cy * ct;
    gx = -f.kx[k] * SLM_PI * sin(ax) * cy * ct;
    gy = -f.ky[k] * SLM_PI * cx * sin(ay) * ct;
}

// Stages of the backward ERK trace of one node (positions, times and the
// velocity gradients there), shared by the tangents of every coefficient.
template <int R>
struct ErkStages {
    double X[6], Y[6], T[6], ax[6], ay[6], bx[6], by[6];
};

template <int R, int DIM>
__device__ __forceinline__ void erk_stages(const WaveField &fa, const WaveField &fb, double x, double y, double t_arr,
                                           double dt, ErkStages<R> &st)
{
    const Erk e = erk_tableau(R);
    const double hs = -dt;
    double kx[6], ky[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        if (s >= e.s) break;
        double X = x, Y = y;
#pragma unroll
        for (int j = 0; j < s; ++j) {
            X += hs * e.a[s][j] * kx[j];
            if (DIM == 2) Y += hs * e.a[s][j] * ky[j];
        }
        const double ts = t_arr + e.c[s] * hs;
        double va = 0.0, gxa = 0.0, gya = 0.0, vb = 0.0, gxb = 0.0, gyb = 0.0;
        for (int k = 0; k < fa.n; ++k) {
            double v, gx, gy;
            term_d(fa, k, X, Y, ts, v, gx, gy);
            va += fa.coef[k] * v;
            gxa += fa.coef[k] * gx;
            gya += fa.coef[k] * gy;
        }
        if (DIM == 2)
            for (int k = 0; k < fb.n; ++k) {
                double v, gx, gy;
                term_d(fb, k, X, Y, ts, v, gx, gy);
                vb += fb.coef[k] * v;
                gxb += fb.coef[k] * gx;
                gyb += fb.coef[k] * gy;
            }
        kx[s] = va;
        ky[s] = vb;
        st.X[s] = X;
        st.Y[s] = Y;
        st.T[s] = ts;
        st.ax[s] = gxa;
        st.ay[s] = gya;
        st.bx[s] = gxb;
        st.by[s] = gyb;
    }
}

// Tangent of the backward ERK departure point with respect to coefficient q
// (alpha terms first, then beta terms), differentiated through the stage
// recursion, in cells: d(d)/dtheta_q for the displacements d = (x - xi)/h.
template <int R, int DIM>
__device__ __forceinline__ void erk_tangent(const WaveField &fa, const WaveField &fb, const ErkStages<R> &st,
                                            double dt, double h, int q, double &ddx, double &ddy)
{
    const Erk e = erk_tableau(R);
    const double hs = -dt;
    const bool qa = q < fa.n;
    const WaveField &f = qa ? fa : fb;
    const int k = qa ? q : q - fa.n;
    double dkx[6], dky[6], sx = 0.0, sy = 0.0;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        if (s >= e.s) break;
        double dX = 0.0, dY = 0.0;
#pragma unroll
        for (int j = 0; j < s; ++j) {
            dX += hs * e.a[s][j] * dkx[j];
            dY += hs * e.a[s][j] * dky[j];
        }
        const double tv = cos(f.kx[k] * SLM_PI * st.X[s] + f.px[k]) * cos(f.ky[k] * SLM_PI * st.Y[s] + f.py[k]) *
                          cos(f.kt[k] * SLM_PI * st.T[s] + f.pt[k]);
        dkx[s] = st.ax[s] * dX + (DIM == 2 ? st.ay[s] * dY : 0.0) + (qa ? tv : 0.0);
        dky[s] = DIM == 2 ? st.bx[s] * dX + st.by[s] * dY + (qa ? 0.0 : tv) : 0.0;
        sx += e.b[s] * dkx[s];
        sy += e.b[s] * dky[s];
    }
    // xi = x + hs*sum(b k)  =>  d(xi) = hs*sum(b dk);  d = (x - xi)/h
    ddx = -hs * sx / h;
    ddy = -hs * sy / h;
}

// Gradient contributions of one level-0 step for every chain:
// gacc[(c0+c)*nb + block][q] += sum_nodes lam[n+1] (dS_n/dtheta_q u_n).
template <int P, int R, int DIM>
__global__ void __launch_bounds__(TPB) grad_kernel(const double *__restrict__ U, long long u_stride,
                                                   const double *__restrict__ lam, long long lam_stride,
                                                   const double *__restrict__ disp, long long plane, int nx,
                                                   long long S, long long n_first, int stride, double dt, double h,
                                                   WaveField fa, WaveField fb, int nq, double *gacc, int c0)
{
    __shared__ double red[SLM_RED_DOUBLES];
    constexpr int ell = (P + 1) / 2;
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const double *u = U + c * u_stride, *lm = lam + c * lam_stride;
    double g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = 0.0;
    for (long long t = (long long)blockIdx.x * TPB + threadIdx.x; t < S; t += (long long)gridDim.x * TPB) {
        const double l = lm[t];
        if (l == 0.0) continue;
        int tx, ty;
        split_xy(t, nx, tx, ty);
        if (DIM != 2) ty = 0;
        const double dx = disp[n * S + t], fx = floor(dx);
        double wx[P + 1], dwx[P + 1];
        weights_eps<P>(dx - fx, wx, dwx);
        const int bx = wrap_mod(tx - (int)fx - ell, nx);
        double gx = 0.0, gy = 0.0;                // d out / d eps, d out / d nu
        if (DIM == 1) {
#pragma unroll
            for (int a = 0; a <= P; ++a) {
                int col = bx + a;
                col -= col >= nx ? nx : 0;
                gx += dwx[a] * u[col];
            }
        } else {
            const double dy = disp[plane + n * S + t], fy = floor(dy);
            double wy[P + 1], dwy[P + 1];
            weights_eps<P>(dy - fy, wy, dwy);
            const int by = wrap_mod(ty - (int)fy - ell, nx);
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                int row = by + b;
                row -= row >= nx ? nx : 0;
                double sw = 0.0, sd = 0.0;
#pragma unroll
                for (int a = 0; a <= P; ++a) {
                    int col = bx + a;
                    col -= col >= nx ? nx : 0;
                    const double uv = u[(long long)row * nx + col];
                    sw += wx[a] * uv;
                    sd += dwx[a] * uv;
                }
                gx += sd * wy[b];
                gy += sw * dwy[b];
            }
        }
        const double x = -1.0 + tx * h, y = DIM == 2 ? -1.0 + ty * h : 0.0;
        ErkStages<R> es;
        erk_stages<R, DIM>(fa, fb, x, y, (double)(n + 1) * dt, dt, es);
        for (int q = 0; q < nq; ++q) {
            double ddx, ddy;
            erk_tangent<R, DIM>(fa, fb, es, dt, h, q, ddx, ddy);
            // eps = d - floor(d): d eps / d theta = d(d) / d theta
            const double v = l * (gx * ddx + (DIM == 2 ? gy * ddy : 0.0));
#pragma unroll
            for (int qq = 0; qq < NQ; ++qq)
                if (qq == q) g[qq] += v;
        }
    }
    block_sum<NQ>(g, red, 0);
    if (threadIdx.x < nq) gacc[((long long)(c0 + c) * gridDim.x + blockIdx.x) * NQ + threadIdx.x] += g[threadIdx.x];
}

// Fixed-order sum of the gradient slots of every (chain, block): one
// workgroup, each thread a strided subset, then the workgroup tree.
__global__ void __launch_bounds__(TPB) grad_reduce(const double *__restrict__ gacc, long long nslots, int nq,
                                                  double *out)
{
    __shared__ double red[SLM_RED_DOUBLES];
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = 0.0;
    for (long long i = threadIdx.x; i < nslots; i += TPB)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < nq) v[q] += gacc[i * NQ + q];
    block_sum<NQ>(v, red, 0);
    if (threadIdx.x < nq) out[threadIdx.x] = v[threadIdx.x];
}

__global__ void __launch_bounds__(TPB) fill0(double *p, long long n)
{
    for (long long i = (long long)blockIdx.x * TPB + threadIdx.x; i < n; i += (long long)gridDim.x * TPB) p[i] = 0.0;
}

}  // namespace

// ------------------------------------------------------------ launchers
hipError_t launch_adj_index(const slm_plan &P, int level, hipStream_t st)
{
    const LevelInfo &L = P.lv[level];
    const long long S = P.S, N = L.N;
    const double *disp = (const double *)ws_at(P, L.disp);
    int *end = (int *)ws_at(P, L.idx_end), *perm = (int *)ws_at(P, L.idx_perm);
    const long long plane = N * S;
    const int nb = nblk(S);
    for (long long n0 = 0; n0 < N; n0 += 65535) {          // grid.y limit
        const int nn = (int)(N - n0 < 65535 ? N - n0 : 65535);
        int *e = end + n0 * S, *pm = perm + n0 * S;
        const double *d = disp + n0 * S;
        hipLaunchKernelGGL(idx_clear, dim3(1024), dim3(TPB), 0, st, e, (long long)nn * S);
        hipLaunchKernelGGL(idx_count, dim3(nb, nn), dim3(TPB), 0, st, d, plane, S, P.d.nx, P.d.dim, e);
        hipLaunchKernelGGL(idx_scan, dim3(nn), dim3(1024), 0, st, e, S);
        hipLaunchKernelGGL(idx_fill, dim3(nb, nn), dim3(TPB), 0, st, d, plane, S, P.d.nx, P.d.dim, e, pm);
        hipLaunchKernelGGL(idx_sort, dim3(nb, nn), dim3(TPB), 0, st, e, pm, S);
        hipLaunchKernelGGL(idx_eps, dim3(nb, nn), dim3(TPB), 0, st, d, plane, S, P.d.dim, pm,
                           (double *)ws_at(P, L.idx_eps) + n0 * S, N * S);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_stepT(const slm_plan &P, int level, int nch, const double *src, long long src_stride, double *dst,
                        long long dst_stride, long long n_first, int stride, int rev, const double *G, double *Vout,
                        hipStream_t st)
{
    const LevelInfo &L = P.lv[level];
    const long long S = P.S;
    const double *disp = (const double *)ws_at(P, L.disp);
    const int *end = (const int *)ws_at(P, L.idx_end), *perm = (const int *)ws_at(P, L.idx_perm);
    const double *eps = (const double *)ws_at(P, L.idx_eps);
    (void)disp;
    const dim3 grid(nblk(S), nch);
#define ST(PP) hipLaunchKernelGGL((stepT_kernel<PP>), grid, dim3(TPB), 0, st, src, src_stride, dst, dst_stride, eps, \
                                  (long long)L.N * S, end, perm, P.d.nx, P.d.dim, S, n_first, stride, rev, L.N, G, Vout)
    switch (P.d.p) {
    case 1: ST(1); break;
    case 3: ST(3); break;
    case 5: ST(5); break;
    default: return hipErrorInvalidValue;
    }
#undef ST
    return hipGetLastError();
}

hipError_t launch_step_fwd(const slm_plan &P, int nch, const double *src, long long src_stride, double *dst,
                           long long dst_stride, long long n_first, int stride, hipStream_t st)
{
    const LevelInfo &L = P.lv[0];
    const long long S = P.S;
    const double *disp = (const double *)ws_at(P, L.disp);
    const dim3 grid(nblk(S), nch);
#define SF(PP) hipLaunchKernelGGL((stepF_kernel<PP>), grid, dim3(TPB), 0, st, src, src_stride, dst, dst_stride, disp, \
                                  (long long)L.N * S, P.d.nx, P.d.dim, S, n_first, stride)
    switch (P.d.p) {
    case 1: SF(1); break;
    case 3: SF(3); break;
    case 5: SF(5); break;
    default: return hipErrorInvalidValue;
    }
#undef SF
    return hipGetLastError();
}

hipError_t launch_grad(const slm_plan &P, int nch, const double *U, long long u_stride, const double *lam,
                       long long lam_stride, long long n_first, int stride, double *gacc, hipStream_t st)
{
    const long long S = P.S;
    const double *disp = (const double *)ws_at(P, P.lv[0].disp);
    const dim3 grid(P.nb2, nch);                 // gacc holds P.nb2 slots per interval
    const double h = 2.0 / P.d.nx;
    const int c0 = (int)(n_first / stride);
    if (!slots_fit(P, (int)grid.x, c0, nch, P.lv[0].N / P.lv[0].m)) return kSlotMismatch;
#define GK(PP, RR, DD) hipLaunchKernelGGL((grad_kernel<PP, RR, DD>), grid, dim3(TPB), 0, st, U, u_stride, lam, \
                                          lam_stride, disp, (long long)P.lv[0].N * S, P.d.nx, S, n_first, stride, \
                                          P.d.dt, h, P.fa, P.fb, P.nq, gacc, c0)
#define GKR(PP, DD) switch (P.d.r) { case 1: GK(PP, 1, DD); break; case 2: GK(PP, 2, DD); break; \
                                     case 3: GK(PP, 3, DD); break; case 4: GK(PP, 4, DD); break; default: GK(PP, 5, DD); break; }
#define GKP(DD) switch (P.d.p) { case 1: GKR(1, DD); break; case 3: GKR(3, DD); break; default: GKR(5, DD); break; }
    if (P.d.dim == 1) GKP(1) else GKP(2)
#undef GKP
#undef GKR
#undef GK
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const slm_plan &P, int nchains, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(grad_reduce, dim3(1), dim3(TPB), 0, st, (const double *)ws_at(P, P.gacc),
                       (long long)nchains * P.nb2, P.nq, out);
    return hipGetLastError();
}

hipError_t launch_fill0(double *p, long long n, hipStream_t st)
{
    hipLaunchKernelGGL(fill0, dim3(1024), dim3(TPB), 0, st, p, n);
    return hipGetLastError();
}
