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

}  // namespace

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
