// slm_fine1d.hip -- launchers of the level-0 sweep and sequential-stepping
// kernels of the 1D path (Sec. 2.1 steps, chained per coarse interval as in
// Sec. 2.2).  The kernels live in slm_kernels1d.h; this unit only chooses
// the instantiation: elements per thread, double buffering, prefetch depth,
// and the fast variant for slices that fill the workgroup exactly and whose
// displacements need a one-sided wrap only.
#include "slm_kernels1d.h"

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

// The autotuner's elements per thread apply to sweeps over many intervals
// (the shape it timed) that form no residual: with a residual the per-chain
// sum of squares follows the thread layout, so those sweeps keep the
// built-in shape and the norms stay bitwise fixed.
template <typename T, typename TD, int P, bool DBUF>
hipError_t fine_ept(const ChainArgs &a, int nchains, hipStream_t st)
{
    int block = fine_block(a.nx, nchains);
    if (a.ept_hint > 0 && !a.R && nchains >= 64) {
        const int b = ((a.nx + a.ept_hint - 1) / a.ept_hint + 63) / 64 * 64;
        if (b <= SLM_MAXB) block = b;
    }
    const int ept = (a.nx + block - 1) / block;
    // the fast variant: the slice fills the workgroup and the displacement
    // bound gives a pad that the threads of one row can write
    const bool fast_ok = a.fpad > 0 && a.fpad <= block;
    auto lds_for = [&](bool fast) {
        const size_t slen = fast ? fast_slice_len(a.nx, a.fpad) : fine_slice_len(a.nx);
        return (((size_t)(DBUF ? 2 : 1) * slen * sizeof(T) + 15) & ~size_t(15)) + SLM_RED_DOUBLES * sizeof(double);
    };
#define FL(E) (fast_ok && a.nx == (E) * block                                                                      \
                   ? launch(fine1d<T, TD, P, E, DBUF, pf_depth<TD, E>(), true>, nchains, block, lds_for(true), a, st) \
                   : launch(fine1d<T, TD, P, E, DBUF, pf_depth<TD, E>(), false>, nchains, block, lds_for(false), a, st))
    switch (ept) {
    case 1: return FL(1);
    case 2: return FL(2);
    case 3:
    case 4: return FL(4);
    default: return FL(8);
    }
#undef FL
}

template <typename T, typename TD, bool DBUF>
hipError_t fine_p(const ChainArgs &a, int nchains, hipStream_t st)
{
    switch (a.p) {
    case 1: return fine_ept<T, TD, 1, DBUF>(a, nchains, st);
    case 2: return fine_ept<T, TD, 2, DBUF>(a, nchains, st);
    case 3: return fine_ept<T, TD, 3, DBUF>(a, nchains, st);
    case 4: return fine_ept<T, TD, 4, DBUF>(a, nchains, st);
    default: return fine_ept<T, TD, 5, DBUF>(a, nchains, st);
    }
}

}  // namespace

hipError_t launch_fine_1d(int nchains, bool f32, const ChainArgs &a, hipStream_t st)
{
    // Double-buffer the slice when two copies fit in the workgroup's LDS,
    // except for FP64 sweeps over many intervals: with one slice buffer
    // three workgroups share a CU instead of two (LDS 3 x 33 KB for 4096
    // points), which keeps more displacement loads in flight and outweighs
    // the extra barrier per step (level-0 sweep of the 1D workload: 152 ->
    // 142 us).
    const size_t extra = SLM_RED_DOUBLES * sizeof(double) + 16;
    const size_t slen = a.fpad > 0 && fast_slice_len(a.nx, a.fpad) > fine_slice_len(a.nx) ? fast_slice_len(a.nx, a.fpad)
                                                                                            : fine_slice_len(a.nx);
    const bool fits = 2ull * slen * (f32 ? 4 : 8) + extra <= (size_t)lds_limit();
    bool dbuf = fits && (f32 || nchains < 512);
    if (a.dbuf_hint >= 0 && !a.R && nchains >= 64) dbuf = fits && a.dbuf_hint;
    if (f32) return dbuf ? fine_p<float, float, true>(a, nchains, st) : fine_p<float, float, false>(a, nchains, st);
    return dbuf ? fine_p<double, double, true>(a, nchains, st) : fine_p<double, double, false>(a, nchains, st);
}
