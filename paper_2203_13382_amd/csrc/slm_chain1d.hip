// slm_chain1d.hip -- batched F/C relaxation on a periodic 1D mesh.
//
// One workgroup advances one coarse time interval through its level steps
// (Sec. 2.2: F-relaxation steps from each C-point across the m-1 F-points
// after it; C-relaxation takes one more step).  All intervals of a level run
// concurrently.  The spatial slice stays resident in LDS across the steps of
// an interval, so HBM traffic per point-update is the stored displacement
// (and the right-hand side on coarse levels) plus the slices a sweep must
// write.
//
// One level step is the semi-Lagrangian step of Sec. 2.1 (level 0) or the
// modified coarse operator of eq. (Phi_multilevel):
//     v <- [I - diag(sigma) D_{p+1}]^{-1} S_{p,r*} v,
// with the inverse applied by GMRES inside the workgroup (Sec. 3.3 / 3.4):
// zero initial guess, Arnoldi with classical Gram-Schmidt applied twice,
// Givens rotations, exit once |g_{j+1}| <= rtol*||b|| or after kmax
// iterations.  Inner products and the Givens recurrence are FP64; the Krylov
// basis lives in registers (EPT values per thread per vector).
#include "slm_internal.h"

#include <type_traits>

namespace {

// Interpolate the LDS slice `s` at the departure point of node i whose
// displacement is d cells (xi = x_i - d h): x_E = x_{i - floor(d)},
// eps = d - floor(d) (eq. depart_decompose).
template <int P, typename T, typename TD>
__device__ __forceinline__ T interp1(const T *__restrict__ s, int i, TD d, int nx, int nsmall)
{
    const TD fl = floor(d);
    const T eps = T(d - fl);
    const int first = stencil_first<T>(P, eps);
    int base = i - int(fl) + first;
    if (nsmall) {
        base += base < 0 ? nx : 0;
        base -= base >= nx ? nx : 0;
    } else {
        base = wrap_mod(base, nx);
    }
    T w[P + 1];
    lagrange_weights<P, T>(-eps - T(first), w);
    T acc = T(0);
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        int idx = base + j;
        idx -= idx >= nx ? nx : 0;
        acc += w[j] * s[idx];
    }
    return acc;
}

// LDS scalars used by thread 0 for the Givens recurrence.
struct GmresScalars {
    double R[SLM_KMAX][SLM_KMAX];   // R[col][row]
    double cs[SLM_KMAX], sn[SLM_KMAX], g[SLM_KMAX + 1], z[SLM_KMAX];
    int flag;
};

template <typename T, int P, int EPT>
struct Gmres1D {
    T V[SLM_KMAX + 1][EPT];
    T w[EPT];
    int k;

    // One Arnoldi step JJ.  Returns true when the iteration must stop
    // before step JJ is taken.
    template <int JJ>
    __device__ __forceinline__ bool step(const double (&sg)[EPT], T *xb, double *red, int &rb,
                                          GmresScalars *gs, int kmax, double rtol, double beta, int nx)
    {
        const int tid = threadIdx.x, B = blockDim.x;
        if (JJ >= kmax) return true;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            if (i < nx) xb[i] = V[JJ][e];
        }
        __syncthreads();
        if (JJ > 0 && gs->flag) return true;
        // w = V_JJ - sigma .* (D_{p+1} V_JJ)
        constexpr int q = DTaps<P>::q;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            double dv = 0.0;
            if (i < nx) {
#pragma unroll
                for (int t = -q; t <= q; ++t) {
                    int idx = i + t;
                    idx += idx < 0 ? nx : 0;
                    idx -= idx >= nx ? nx : 0;
                    dv += DTaps<P>::t[t + q] * double(xb[idx]);
                }
                w[e] = T(double(V[JJ][e]) - sg[e] * dv);
            } else {
                w[e] = T(0);
            }
        }
        // classical Gram-Schmidt, twice
        double hc[JJ + 1];
#pragma unroll
        for (int i = 0; i <= JJ; ++i) hc[i] = 0.0;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            double h[JJ + 1];
#pragma unroll
            for (int i = 0; i <= JJ; ++i) {
                double s = 0.0;
#pragma unroll
                for (int e = 0; e < EPT; ++e) s += double(V[i][e]) * double(w[e]);
                h[i] = s;
            }
            block_sum<JJ + 1>(h, red, rb);
            rb ^= 1;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                double t = double(w[e]);
#pragma unroll
                for (int i = 0; i <= JJ; ++i) t -= h[i] * double(V[i][e]);
                w[e] = T(t);
            }
#pragma unroll
            for (int i = 0; i <= JJ; ++i) hc[i] += h[i];
        }
        double nn[1] = {0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) nn[0] += double(w[e]) * double(w[e]);
        block_sum<1>(nn, red, rb);
        rb ^= 1;
        const double hn = sqrt(nn[0]);
        if (tid == 0) {
#pragma unroll
            for (int i = 0; i < JJ; ++i) {          // previous rotations
                const double t0 = gs->cs[i] * hc[i] + gs->sn[i] * hc[i + 1];
                const double t1 = -gs->sn[i] * hc[i] + gs->cs[i] * hc[i + 1];
                hc[i] = t0;
                hc[i + 1] = t1;
            }
            const double den = sqrt(hc[JJ] * hc[JJ] + hn * hn);
            const double c = hc[JJ] / den, s = hn / den;
            gs->cs[JJ] = c;
            gs->sn[JJ] = s;
            hc[JJ] = den;
            gs->g[JJ + 1] = -s * gs->g[JJ];
            gs->g[JJ] = c * gs->g[JJ];
#pragma unroll
            for (int i = 0; i <= JJ; ++i) gs->R[JJ][i] = hc[i];
            gs->flag = (hn == 0.0) || (fabs(gs->g[JJ + 1]) <= rtol * beta);
        }
        k = JJ + 1;
        const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) V[JJ + 1][e] = T(double(w[e]) * inv);
        return false;
    }

    // Solve [I - diag(sg) D_{p+1}] y = x in place.  Returns iterations.
    __device__ __forceinline__ int solve(T (&x)[EPT], const double (&sg)[EPT], T *xb, double *red, int &rb,
                                         GmresScalars *gs, int kmax, double rtol, int nx)
    {
        const int tid = threadIdx.x;
        double bb[1] = {0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) bb[0] += double(x[e]) * double(x[e]);
        if (tid == 0) gs->flag = 0;
        block_sum<1>(bb, red, rb);
        rb ^= 1;
        const double beta = sqrt(bb[0]);
        if (beta == 0.0 || kmax <= 0) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) x[e] = T(0);
            return 0;
        }
        if (tid == 0) {
            gs->g[0] = beta;
            for (int i = 1; i <= SLM_KMAX; ++i) gs->g[i] = 0.0;
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) V[0][e] = T(double(x[e]) / beta);
        k = 0;
        step<0>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) || step<1>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) ||
            step<2>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) || step<3>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) ||
            step<4>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) || step<5>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) ||
            step<6>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) || step<7>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) ||
            step<8>(sg, xb, red, rb, gs, kmax, rtol, beta, nx) || step<9>(sg, xb, red, rb, gs, kmax, rtol, beta, nx);
        // back substitution R z = g (thread 0), then y = V z
        if (tid == 0) {
            for (int i = k - 1; i >= 0; --i) {
                double s = gs->g[i];
                for (int t = i + 1; t < k; ++t) s -= gs->R[t][i] * gs->z[t];
                gs->z[i] = s / gs->R[i][i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            double y = 0.0;
#pragma unroll
            for (int i = 0; i < SLM_KMAX; ++i)
                if (i < k) y += gs->z[i] * double(V[i][e]);
            x[e] = T(y);
        }
        return k;
    }
};

template <typename T, typename TD, int P, int EPT, bool COARSE, bool DBUF>
__global__ void __launch_bounds__(SLM_MAXB) chain1d(ChainArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x, B = blockDim.x, nx = a.nx;
    const long long S = a.S;
    const int j = blockIdx.x;
    T *sl0 = reinterpret_cast<T *>(smem);
    T *sl1 = DBUF ? sl0 + nx : sl0;
    const size_t off = ((size_t)(DBUF ? 2 : 1) * nx * sizeof(T) + 15) & ~size_t(15);
    double *red = reinterpret_cast<double *>(smem + off);
    GmresScalars *gs = reinterpret_cast<GmresScalars *>(red + SLM_RED_DOUBLES);

    const T *Cin = static_cast<const T *>(a.Cin);
    const T *G = static_cast<const T *>(a.G);
    const TD *disp = static_cast<const TD *>(a.disp);
    T *Vout = static_cast<T *>(a.Vout);
    T *Cout = static_cast<T *>(a.Cout);
    const long long n_first = a.n_base + (long long)j * a.stride_chain;

    T val[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid + e * B;
        T s = T(0);
        if (i < nx) {
            if (Cin) s = Cin[(long long)j * a.cin_stride + i];
            sl0[i] = s;
            if (Vout && a.write_start) Vout[n_first * S + i] = s;
            if (Cout && j == 0 && a.cout_shift) Cout[i] = s;
        }
        val[e] = s;
    }
    __syncthreads();

    TD dn[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid + e * B;
        dn[e] = (i < nx && a.nsteps > 0) ? disp[n_first * S + i] : TD(0);
    }
    int cur = 0, rb = 0;
    Gmres1D<T, P, EPT> gm;
    unsigned long long nsolve = 0, niter = 0;
    for (int k = 0; k < a.nsteps; ++k) {
        const long long n = n_first + k;
        TD dc[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) dc[e] = dn[e];
        if (k + 1 < a.nsteps) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = tid + e * B;
                if (i < nx) dn[e] = disp[(n + 1) * S + i];
            }
        }
        T gv[EPT];
        double sg[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            gv[e] = (G && i < nx) ? G[(n + 1) * S + i] : T(0);
            sg[e] = (COARSE && i < nx) ? a.sigma[n * S + i] : 0.0;
        }
        const T *src = cur ? sl1 : sl0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            val[e] = i < nx ? interp1<P, T, TD>(src, i, dc[e], nx, a.nsmall) : T(0);
        }
        if constexpr (COARSE) {
            __syncthreads();                     // every read of the slice is done
            const int it = gm.solve(val, sg, sl0, red, rb, gs, a.kmax, a.rtol, nx);
            ++nsolve;
            niter += it;
        } else if constexpr (!DBUF) {
            __syncthreads();
        }
        T *dst = DBUF ? (cur ? sl0 : sl1) : sl0;
        const bool wv = Vout && (k + 1 < a.nsteps || a.write_last);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            val[e] += gv[e];
            if (i < nx) {
                dst[i] = val[e];
                if (wv) Vout[(n + 1) * S + i] = val[e];
            }
        }
        if (DBUF) cur ^= 1;
        __syncthreads();
    }
    if (Cout) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            if (i < nx) Cout[(long long)(j + a.cout_shift) * S + i] = val[e];
        }
    }
    if (a.R) {
        const T *Cref = static_cast<const T *>(a.Cref);
        T *R = static_cast<T *>(a.R);
        double acc[1] = {0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            if (i < nx) {
                const T r = Cref ? T(val[e] - Cref[(long long)(j + 1) * S + i]) : val[e];
                R[(long long)(j + 1) * S + i] = r;
                acc[0] += double(r) * double(r);
            }
        }
        block_sum<1>(acc, red, rb);
        if (tid == 0) a.partial[j] = acc[0];
    }
    if (COARSE && tid == 0 && a.counter) {
        atomicAdd(a.counter, nsolve);
        atomicAdd(a.counter + 1, niter);
    }
}

template <typename T, typename TD, int P, int EPT, bool COARSE, bool DBUF>
hipError_t launch_one(const ChainArgs &a, int nchains, int block, hipStream_t st)
{
    const size_t sl = ((size_t)(DBUF ? 2 : 1) * a.nx * sizeof(T) + 15) & ~size_t(15);
    const size_t lds = sl + SLM_RED_DOUBLES * sizeof(double) + sizeof(GmresScalars);
    auto k = chain1d<T, TD, P, EPT, COARSE, DBUF>;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(nchains), dim3(block), lds, st, a);
    return hipGetLastError();
}

template <typename T, typename TD, int P, bool COARSE, bool DBUF>
hipError_t dispatch_ept(const ChainArgs &a, int nchains, hipStream_t st)
{
    const int block = a.nx >= SLM_MAXB ? SLM_MAXB : ((a.nx + 63) / 64) * 64;
    const int ept = (a.nx + block - 1) / block;
    switch (ept) {
    case 1: return launch_one<T, TD, P, 1, COARSE, DBUF>(a, nchains, block, st);
    case 2: return launch_one<T, TD, P, 2, COARSE, DBUF>(a, nchains, block, st);
    case 3:
    case 4: return launch_one<T, TD, P, 4, COARSE, DBUF>(a, nchains, block, st);
    default: return launch_one<T, TD, P, 8, COARSE, DBUF>(a, nchains, block, st);
    }
}

template <typename T, typename TD, bool COARSE, bool DBUF>
hipError_t dispatch_p(const ChainArgs &a, int nchains, hipStream_t st)
{
    switch (a.p) {
    case 1: return dispatch_ept<T, TD, 1, COARSE, DBUF>(a, nchains, st);
    case 3: return dispatch_ept<T, TD, 3, COARSE, DBUF>(a, nchains, st);
    case 5: return dispatch_ept<T, TD, 5, COARSE, DBUF>(a, nchains, st);
    case 2: if constexpr (!COARSE) return dispatch_ept<T, TD, 2, COARSE, DBUF>(a, nchains, st); break;
    case 4: if constexpr (!COARSE) return dispatch_ept<T, TD, 4, COARSE, DBUF>(a, nchains, st); break;
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_chain_1d(const slm_plan &P, int level, int nchains, const ChainArgs &a, hipStream_t st)
{
    if (nchains <= 0) return hipSuccess;
    const bool coarse = level > 0;
    const bool f32 = P.d.precision == SLM_FP32_BULK;
    // double-buffer the slice when two copies fit in the workgroup's LDS
    static int lds_max = -1;
    if (lds_max < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds_max = 65536;
    }
    const size_t extra = SLM_RED_DOUBLES * sizeof(double) + sizeof(GmresScalars) + 16;
    const bool dbuf = 2ull * a.nx * (f32 ? 4 : 8) + extra <= (size_t)lds_max;
    if (coarse) {
        return f32 ? dispatch_p<float, double, true, false>(a, nchains, st)
                   : dispatch_p<double, double, true, false>(a, nchains, st);
    }
    if (f32) return dbuf ? dispatch_p<float, float, false, true>(a, nchains, st)
                         : dispatch_p<float, float, false, false>(a, nchains, st);
    return dbuf ? dispatch_p<double, double, false, true>(a, nchains, st)
                : dispatch_p<double, double, false, false>(a, nchains, st);
}
