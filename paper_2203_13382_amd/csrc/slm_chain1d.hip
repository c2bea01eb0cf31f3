// slm_chain1d.hip -- batched F/C relaxation on a periodic 1D mesh.
//
// One workgroup advances one coarse time interval through its level steps
// (Sec. 2.2: F-relaxation steps from each C-point across the m-1 F-points
// after it; C-relaxation takes one more step).  All intervals of a level run
// concurrently.  The spatial slice stays resident in LDS across the steps of
// an interval, so HBM traffic per point-update is the stored displacement
// (and the right-hand side on coarse levels) plus the slices a sweep writes.
//
// Level 0 applies the semi-Lagrangian step of Sec. 2.1; its kernel streams
// the displacements through a prefetch ring PF steps deep (launchers in
// slm_fine1d.hip, a translation unit of its own).  Coarse levels
// apply the modified operator of eq. (Phi_multilevel),
//     v <- [I - diag(sigma) D_{p+1}]^{-1} S_{p,r*} v,
// with the inverse applied by GMRES inside the workgroup (Sec. 3.3 / 3.4):
// zero initial guess, Arnoldi with classical Gram-Schmidt (one pass) whose
// reduction also carries ||w||^2, so that the new vector's norm follows by
// Pythagoras (reduced from the updated vector where that would cancel),
// Givens rotations, exit once |g_{j+1}| <= rtol*||b|| or after kmax
// iterations.  Inner products and the Givens recurrence are FP64.  The
// Krylov basis lives in registers (EPT values per thread per vector), so
// coarse workgroups use at most 512 threads to get 256 VGPRs per lane.
#include "slm_kernels1d.h"

#include <type_traits>

namespace {

using namespace slmk;

// ------------------------------------------------------------------ launchers
int lds_limit()
{
    static int v = -1;
    if (v < 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            v = 65536;
    }
    return v;
}

template <typename K>
hipError_t launch(K kern, int nchains, int block, size_t lds, const ChainArgs &a, hipStream_t st)
{
    if (lds > (size_t)lds_limit()) return hipErrorInvalidConfiguration;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(nchains), dim3(block), lds, st, a);
    return hipGetLastError();
}

template <typename T, int P, int EPT>
hipError_t coarse_launch(const ChainArgs &a, int nchains, hipStream_t st)
{
    size_t o1, o2, o3;
    const size_t lds = coarse_lds_parts<T, EPT>(a.nx, &o1, &o2, &o3);
    const int block = ((a.nx + EPT - 1) / EPT + 63) / 64 * 64;
    if constexpr (std::is_same<T, double>::value) {   // the forward-Euler operator is FP64 only
        if (a.fwd) {
            if (a.nx == EPT * block) return launch(coarse1d<T, P, EPT, true, true>, nchains, block, lds, a, st);
            return launch(coarse1d<T, P, EPT, false, true>, nchains, block, lds, a, st);
        }
    }
    if (a.nx == EPT * block) return launch(coarse1d<T, P, EPT, true>, nchains, block, lds, a, st);
    return launch(coarse1d<T, P, EPT, false>, nchains, block, lds, a, st);
}

// Elements per thread: the smallest power of two that keeps the workgroup at
// or below COARSE_MAXB threads.
template <typename T, int P>
hipError_t coarse_ept(const ChainArgs &a, int nchains, hipStream_t st)
{
    if (a.nx <= COARSE_MAXB) return coarse_launch<T, P, 1>(a, nchains, st);
    if (a.nx <= 2 * COARSE_MAXB) return coarse_launch<T, P, 2>(a, nchains, st);
    if (a.nx <= 4 * COARSE_MAXB) return coarse_launch<T, P, 4>(a, nchains, st);
    if (a.nx <= 8 * COARSE_MAXB) return coarse_launch<T, P, 8>(a, nchains, st);
    return coarse_launch<T, P, 16>(a, nchains, st);
}

template <typename T>
hipError_t coarse_p(const ChainArgs &a, int nchains, hipStream_t st)
{
    switch (a.p) {
    case 1: return coarse_ept<T, 1>(a, nchains, st);
    case 3: return coarse_ept<T, 3>(a, nchains, st);
    case 5: return coarse_ept<T, 5>(a, nchains, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_chain_1d(const slm_plan &P, int level, int nchains, const ChainArgs &a, hipStream_t st)
{
    if (nchains <= 0) return hipSuccess;
    const bool f32 = P.d.precision == SLM_FP32_BULK;
    if (level > 0 && P.d.coarse_op != SLM_COARSE_REDISC)
        return f32 ? coarse_p<float>(a, nchains, st) : coarse_p<double>(a, nchains, st);
    return launch_fine_1d(nchains, f32, a, st);
}
