// slm_misc.hip -- small device utilities: deterministic residual-norm
// reduction, slice-wise axpy (coarse-grid correction by injection) and
// strided slice copies.
#include "slm_internal.h"

namespace {

// Sum of n partial sums in a fixed order (one workgroup): deterministic.
__global__ void __launch_bounds__(1024) sum_partials_kernel(const double *__restrict__ p, int n,
                                                           double *__restrict__ out)
{
    __shared__ double red[SLM_RED_DOUBLES];
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < n; i += blockDim.x) v[0] += p[i];
    block_sum<1>(v, red, 0);
    if (threadIdx.x == 0) *out = v[0];
}

// dst[c*dst_stride + s] (+)= src[c*src_stride + s], c < count, s < S.
template <typename T>
__global__ void axpy_kernel(T *__restrict__ dst, long long ds, const T *__restrict__ src, long long ss,
                            int count, long long S, int assign)
{
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long c = blockIdx.y;
    if (id >= S || c >= count) return;
    const T v = src[c * ss + id];
    if (assign) dst[c * ds + id] = v;
    else dst[c * ds + id] += v;
}

// SplitMix64 output for the state x (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x)
{
    unsigned long long z = x + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Seeded random initial iterate: slice c of u (stride ls elements) is fine
// time point n = (c0 + c) * nstep and receives, at node k, the top 53 bits of
// splitmix64(seed ^ (n*S + k)) as a fraction of 2^53 (rounded to T).
template <typename T>
__global__ void seed_kernel(T *__restrict__ u, long long ls, int c0, int count, long long S, long long nstep,
                            unsigned long long seed)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= S || c >= count) return;
    const unsigned long long idx = (unsigned long long)((long long)(c0 + c) * nstep * S + k);
    const double v = (double)(splitmix64(seed ^ idx) >> 11) * (1.0 / 9007199254740992.0);
    u[(long long)(c0 + c) * ls + k] = T(v);
}

// dst[i] = float(src[i]), i < n.
__global__ void narrow_kernel(const double *__restrict__ src, float *__restrict__ dst, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

}  // namespace

hipError_t launch_narrow(const double *src, float *dst, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    long long nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)nb), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_seed_slices(void *u, long long ls, int count, int S, long long nstep, unsigned long long seed,
                              int elem, hipStream_t st)
{
    for (int c0 = 0; c0 < count; c0 += 65535) {           // grid.y limit
        const int cnt = count - c0 < 65535 ? count - c0 : 65535;
        dim3 grid((unsigned)((S + 255) / 256), (unsigned)cnt);
        if (elem == 8)
            hipLaunchKernelGGL(seed_kernel<double>, grid, dim3(256), 0, st, (double *)u, ls, c0, cnt, (long long)S,
                               nstep, seed);
        else
            hipLaunchKernelGGL(seed_kernel<float>, grid, dim3(256), 0, st, (float *)u, ls, c0, cnt, (long long)S,
                               nstep, seed);
    }
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partial, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, st, partial, n, out);
    return hipGetLastError();
}

hipError_t launch_axpy_slices(void *dst, long long ds, const void *src, long long ss, int count, int S,
                              int elem, int assign, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    dim3 grid((unsigned)((S + 255) / 256), (unsigned)count);
    if (elem == 8)
        hipLaunchKernelGGL(axpy_kernel<double>, grid, dim3(256), 0, st, (double *)dst, ds, (const double *)src, ss,
                           count, (long long)S, assign);
    else
        hipLaunchKernelGGL(axpy_kernel<float>, grid, dim3(256), 0, st, (float *)dst, ds, (const float *)src, ss,
                           count, (long long)S, assign);
    return hipGetLastError();
}

hipError_t launch_copy_slices(void *dst, long long ds, const void *src, long long ss, int count, int S, int elem,
                              hipStream_t st)
{
    return launch_axpy_slices(dst, ds, src, ss, count, S, elem, 1, st);
}
