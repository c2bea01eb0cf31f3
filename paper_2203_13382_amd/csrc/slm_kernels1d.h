// slm_kernels1d.h -- device code of the 1D relaxation chains, shared by the
// per-level launches (slm_chain1d.hip) and the persistent batch kernels
// (slm_batch.hip).  See slm_chain1d.hip for the method.  Internal header.
#pragma once

#include "slm_internal.h"

namespace slmk {

constexpr int COARSE_MAXB = 512;

// Workgroup size of the level-0 chain kernel for an nx-point slice and a
// sweep of `nchains` chains.  Up to 2047 points, or when the sweep has too
// few chains to give every CU two of them: one node per thread (at most 1024
// threads), the shortest step latency.  Otherwise, from 2048 points: eight
// nodes per thread, so a 4096-point chain runs in 512 threads and two chains
// share a CU (LDS and registers allow it), overlapping one chain's barriers
// and start-up with the other's steps.
__host__ __device__ inline int fine_block(int nx, long long nchains)
{
    if (nx >= 2048 && nchains >= 512)
        return ((nx / 8 + 63) / 64) * 64 < SLM_MAXB ? ((nx / 8 + 63) / 64) * 64 : SLM_MAXB;
    return nx >= SLM_MAXB ? SLM_MAXB : ((nx + 63) / 64) * 64;
}

// Interpolate the LDS slice `s` at the departure point of node i whose
// displacement is d cells (xi = x_i - d h): x_E = x_{i - floor(d)},
// eps = d - floor(d) (eq. depart_decompose).  The coarse-level kernels call
// this one; it keeps the general product form of the weights, which needs
// fewer live registers than interp_weights in kernels that hold a Krylov
// basis in registers.
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

// Level-0 slices in LDS carry a periodic tail: entries nx .. nx+SLM_SLICE_PAD-1
// repeat nodes 0, 1, ... (mod nx), so the p+1 taps of a stencil that starts
// inside the slice are read at base, base+1, ... without a per-tap wrap.
constexpr int SLM_SLICE_PAD = 8;
__host__ __device__ inline size_t fine_slice_len(int nx) { return (size_t)nx + SLM_SLICE_PAD; }

// interp1 on a padded slice: one wrap of the stencil start, then p+1
// consecutive LDS reads (same products and summation order as
// interp1_nowrap, so every level-0 variant rounds alike).
template <int P, typename T, typename TD>
__device__ __forceinline__ T interp1_padded(const T *__restrict__ s, int i, TD d, int nx, int nsmall)
{
    static_assert(P < SLM_SLICE_PAD, "the periodic tail must cover p taps past the last node");
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
    interp_weights<P, T>(eps, w);
    const T *sp = s + base;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j <= P; ++j) acc += w[j] * sp[j];
    return acc;
}

// Write the periodic tail of a padded slice from the registers that hold
// nodes 0 .. nx-1 in the strided layout (thread t holds node t in val[0]).
template <typename T>
__device__ __forceinline__ void pad_slice(T *sl, T v0, int nx)
{
    const int tid = threadIdx.x;
    if (tid < nx)
        for (int t = tid; t < SLM_SLICE_PAD; t += nx) sl[nx + t] = v0;
}

// The fast level-0 sweep (nx = EPT * blockDim) keeps fpad periodic copies on
// each side of its LDS slice: sl[-fpad .. -1] repeat nodes nx-fpad .. nx-1
// and sl[nx .. nx+fpad-1] nodes 0 .. fpad-1.  With fpad >= ceil(|d|) + p + 2
// every stencil start i - floor(d) + first lies in [-fpad, nx+fpad-p-1], so
// the taps are read with no wrap at all (same products and summation order
// as interp1_padded).
__host__ __device__ inline size_t fast_slice_len(int nx, int fpad) { return (size_t)nx + 2 * (size_t)fpad; }

template <int P, typename T, typename TD>
__device__ __forceinline__ T interp1_nowrap(const T *__restrict__ s, int i, TD d)
{
    const TD fl = floor(d);
    const T eps = T(d - fl);
    T w[P + 1];
    interp_weights<P, T>(eps, w);
    const T *sp = s + (i - int(fl) + stencil_first<T>(P, eps));
    T acc = T(0);
#pragma unroll
    for (int j = 0; j <= P; ++j) acc += w[j] * sp[j];
    return acc;
}

// Both pads of a fast slice from the strided registers: thread t holds node
// t in val[0] and node (EPT-1) * blockDim + t = nx - blockDim + t in
// val[EPT-1]; fpad <= blockDim.
template <typename T, int EPT>
__device__ __forceinline__ void pad_fast(T *sl, const T (&val)[EPT], int nx, int fpad)
{
    const int tid = threadIdx.x, B = blockDim.x;
    if (tid < fpad) sl[nx + tid] = val[0];
    if (tid >= B - fpad) sl[tid - B] = val[EPT - 1];
}

// Load the chain's start slice into LDS (and registers); optionally copy it
// to the full-iterate output and, for chain 0 of a C-point sweep, to Cout[0].
template <typename T, int EPT>
__device__ __forceinline__ void chain_start(const ChainArgs &a, int j, T *sl, T (&val)[EPT], long long n_first)
{
    const int tid = threadIdx.x, B = blockDim.x, nx = a.nx;
    const T *Cin = static_cast<const T *>(a.Cin);
    T *Vout = static_cast<T *>(a.Vout);
    T *Cout = static_cast<T *>(a.Cout);
    // all loads first, then the stores (a store to Vout or Cout could alias
    // Cin, so interleaving them would serialise the loads)
#pragma unroll
    for (int e = 0; e < EPT; ++e) val[e] = T(0);
    if (Cin) {
        const T *c = Cin + (long long)j * a.cin_stride;
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            if (tid + e * B < nx) val[e] = c[tid + e * B];
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = tid + e * B;
        if (i < nx) {
            sl[i] = val[e];
            if (Vout && a.write_start) Vout[n_first * a.S + i] = val[e];
            if (Cout && j == 0 && a.cout_shift) Cout[i] = val[e];
        }
    }
}

// Write the chain's final state (Cout) and/or its C-point residual (R) with
// the per-chain partial sum of squares.
template <typename T, int EPT>
__device__ __forceinline__ void chain_finish(const ChainArgs &a, int j, const T (&val)[EPT], double *red, int rb)
{
    const int tid = threadIdx.x, B = blockDim.x, nx = a.nx;
    const long long S = a.S;
    T *Cout = static_cast<T *>(a.Cout);
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
        T cv[EPT];                               // Cref in one batch of loads
#pragma unroll
        for (int e = 0; e < EPT; ++e) cv[e] = T(0);
        if (Cref) {
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                if (tid + e * B < nx) cv[e] = Cref[(long long)(j + 1) * S + tid + e * B];
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            if (i < nx) {
                const T r = Cref ? T(val[e] - cv[e]) : val[e];
                R[(long long)(j + 1) * S + i] = r;
                acc[0] += double(r) * double(r);
            }
        }
        block_sum<1>(acc, red, rb);
        if (tid == 0) a.partial[j] = acc[0];
    }
}

// ------------------------------------------------------------------ level 0 (and sequential stepping)
// FAST: nx == EPT * blockDim and 0 < a.fpad <= blockDim (no node guards; the
// slice carries periodic pads on both sides, so no stencil wraps).
template <typename T, typename TD, int P, int EPT, bool DBUF, int PF, bool FAST = false>
__device__ __forceinline__ void fine_chain(const ChainArgs &a, int j, unsigned char *smem)
{
    constexpr bool FULL = FAST;
    const int tid = threadIdx.x, B = blockDim.x, nx = a.nx;
    const long long S = a.S;
    const int lp = FAST ? a.fpad : 0;
    const size_t slen = FAST ? fast_slice_len(nx, lp) : fine_slice_len(nx);
    T *sl0 = reinterpret_cast<T *>(smem) + lp;
    T *sl1 = DBUF ? sl0 + slen : sl0;
    const size_t off = ((size_t)(DBUF ? 2 : 1) * slen * sizeof(T) + 15) & ~size_t(15);
    double *red = reinterpret_cast<double *>(smem + off);
    const TD *disp = static_cast<const TD *>(a.disp);
    const T *G = static_cast<const T *>(a.G);
    T *Vout = static_cast<T *>(a.Vout);
    const long long n_first = a.n_base + (long long)j * a.stride_chain;
    const int ns = a.nsteps;

    T val[EPT];
    chain_start<T, EPT>(a, j, sl0, val, n_first);
    if constexpr (FAST)
        pad_fast<T, EPT>(sl0, val, nx, lp);
    else
        pad_slice(sl0, val[0], nx);
    TD ring[PF][EPT];                           // displacements of the next PF steps
#pragma unroll
    for (int u = 0; u < PF; ++u)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = tid + e * B;
            ring[u][e] = (u < ns && (FULL || i < nx)) ? disp[(n_first + u) * S + i] : TD(0);
        }
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < ns; k0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int k = k0 + u;
            if (k >= ns) break;
            const long long n = n_first + k;
            // Refill for step k+PF into separate registers, issued before
            // this step's arithmetic and kept there by the scheduling
            // barrier; the refill is unconditional (the last PF steps
            // re-read their own row, which is cached), so the loads stay in
            // straight-line code and are waited for only at their use.
            const TD *drow = disp + (k + PF < ns ? n + PF : n) * S;   // uniform row base
            TD nxt[EPT];
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = tid + e * B;
                nxt[e] = (FULL || i < nx) ? drow[i] : TD(0);
            }
            __builtin_amdgcn_sched_barrier(0);
            const T *src = cur ? sl1 : sl0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = tid + e * B;
                if constexpr (FAST)
                    val[e] = interp1_nowrap<P, T, TD>(src, i, ring[u][e]);
                else
                    val[e] = i < nx ? interp1_padded<P, T, TD>(src, i, ring[u][e], nx, a.nsmall) : T(0);
                ring[u][e] = nxt[e];
            }
            if constexpr (!DBUF) __syncthreads();
            T *dst = DBUF ? (cur ? sl0 : sl1) : sl0;
            const bool wv = Vout && (k + 1 < ns || a.write_last);
            const T *grow = G ? G + (n + 1) * S : nullptr;
            T *vrow = wv ? Vout + (n + 1) * S : nullptr;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = tid + e * B;
                if (FULL || i < nx) {
                    if (grow) val[e] += grow[i];
                    dst[i] = val[e];
                    if (vrow) vrow[i] = val[e];
                }
            }
            if constexpr (FAST)
                pad_fast<T, EPT>(dst, val, nx, lp);
            else
                pad_slice(dst, val[0], nx);
            if (DBUF) cur ^= 1;
            __syncthreads();
        }
    }
    chain_finish<T, EPT>(a, j, val, red, 0);
}

template <typename T, typename TD, int P, int EPT, bool DBUF, int PF, bool FAST>
__global__ void __launch_bounds__(SLM_MAXB) fine1d(ChainArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    fine_chain<T, TD, P, EPT, DBUF, PF, FAST>(a, blockIdx.x, smem);
}

// ------------------------------------------------------------------ coarse levels
// Element layout of the coarse kernel: thread t owns the EPT contiguous
// nodes t*EPT .. t*EPT+EPT-1, so the D_{p+1} stencil needs only q neighbours
// on each side from other threads.  Those come through an LDS exchange
// buffer with one pad word per EPT nodes (no bank conflicts).
template <int EPT>
__device__ __forceinline__ int pidx(int i) { return i + i / EPT; }

// LDS scalars used by thread 0 for the Givens recurrence.
struct GmresScalars {
    double R[SLM_KMAX][SLM_KMAX];   // R[col][row]
    double cs[SLM_KMAX], sn[SLM_KMAX], g[SLM_KMAX + 1], z[SLM_KMAX];
    int flag;
};

// FULL: the slice fills the workgroup exactly (nx == EPT * blockDim), so no
// node guard or ragged-tail wrap is needed.
template <typename T, int P, int EPT, bool FULL = false>
struct Gmres1D {
    T V[SLM_KMAX + 1][EPT];
    T w[EPT];
    int k;

    // One Arnoldi step JJ.  Returns true when the iteration stops before
    // step JJ is taken.  xp: padded exchange buffer; sgp: sigma, padded.
    template <int JJ>
    __device__ __forceinline__ bool step(const double *sgp, T *xp, double *red, int &rb,
                                          GmresScalars *gs, int kmax, double rtol, double beta, int nx)
    {
        int tid = threadIdx.x;
        // Opaque per step: addresses derived from tid are recomputed in every
        // Arnoldi step instead of being hoisted and held across all of them.
        __asm__ volatile("" : "+v"(tid));
        if (JJ >= kmax) return true;
        const int i0 = tid * EPT;
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            if (FULL || i0 + e < nx) xp[pidx<EPT>(i0 + e)] = V[JJ][e];
        __syncthreads();
        if (JJ > 0 && gs->flag) return true;
        // w = V_JJ - sigma .* (D_{p+1} V_JJ) over the window i0-q .. i0+EPT-1+q
        constexpr int q = DTaps<P>::q;
        T win[EPT + 2 * q];
#pragma unroll
        for (int t = 0; t < q; ++t) {
            int il = i0 - q + t;
            il += il < 0 ? nx : 0;
            int ir = i0 + EPT + t;
            ir -= ir >= nx ? nx : 0;             // periodic (ragged tails wrap too)
            win[t] = (FULL || i0 < nx) ? xp[pidx<EPT>(il)] : T(0);
            win[EPT + q + t] = (FULL || i0 < nx) ? xp[pidx<EPT>(ir)] : T(0);
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) win[q + e] = V[JJ][e];
        // ragged tail: neighbours past nx wrap to the start of the slice
        if (!FULL && i0 + EPT > nx) {
#pragma unroll
            for (int e = 0; e < EPT + q; ++e) {
                const int i = i0 + e;
                if (i >= nx && i - nx < nx) win[q + e] = xp[pidx<EPT>(i - nx)];
            }
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            if (FULL || i0 + e < nx) {
                double dv = 0.0;
#pragma unroll
                for (int t = 0; t <= 2 * q; ++t) dv += DTaps<P>::t[t] * double(win[e + t]);
                w[e] = T(double(V[JJ][e]) - sgp[pidx<EPT>(i0 + e)] * dv);
            } else {
                w[e] = T(0);
            }
        }
        // classical Gram-Schmidt (every coefficient projects the same w) and
        // ||w||^2 in one reduction; the new vector's norm then follows by
        // Pythagoras, ||w - V h||^2 = ||w||^2 - sum h_i^2, unless cancellation
        // would cost more than three digits: then a second reduction takes it
        // from the updated vector.  Inner products are wave-uniform.
        double h1[JJ + 2];
#pragma unroll
        for (int i = 0; i <= JJ; ++i) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) s += double(V[i][e] * w[e]);   // FP32 bulk: product in T
            h1[i] = s;
        }
        {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) s += double(w[e] * w[e]);
            h1[JJ + 1] = s;
        }
        block_sum_u<JJ + 2>(h1, red, rb);
        rb ^= 1;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            T t = w[e];
#pragma unroll
            for (int i = 0; i <= JJ; ++i) t -= T(h1[i]) * V[i][e];
            w[e] = t;
        }
        double hn2 = h1[JJ + 1];
#pragma unroll
        for (int i = 0; i <= JJ; ++i) hn2 -= h1[i] * h1[i];
        if (!(hn2 >= 1e-3 * h1[JJ + 1])) {
            double nn[1] = {0.0};
#pragma unroll
            for (int e = 0; e < EPT; ++e) nn[0] += double(w[e] * w[e]);
            block_sum_u<1>(nn, red, rb);
            rb ^= 1;
            hn2 = nn[0];
        }
        const double hn = sqrt(hn2 > 0.0 ? hn2 : 0.0);
        if (tid == 0) {
            double hc[JJ + 1];
#pragma unroll
            for (int i = 0; i <= JJ; ++i) hc[i] = h1[i];
#pragma unroll
            for (int i = 0; i < JJ; ++i) {          // previous rotations
                const double ci = gs->cs[i], si = gs->sn[i];
                const double t0 = ci * hc[i] + si * hc[i + 1];
                const double t1 = -si * hc[i] + ci * hc[i + 1];
                hc[i] = t0;
                hc[i + 1] = t1;
            }
            const double den = sqrt(hc[JJ] * hc[JJ] + hn * hn);
            const double c = hc[JJ] / den, sv = hn / den;
            gs->cs[JJ] = c;
            gs->sn[JJ] = sv;
            hc[JJ] = den;
            const double gj = gs->g[JJ];
            gs->g[JJ + 1] = -sv * gj;
            gs->g[JJ] = c * gj;
#pragma unroll
            for (int i = 0; i <= JJ; ++i) gs->R[JJ][i] = hc[i];
            gs->flag = (hn == 0.0) || (fabs(sv * gj) <= rtol * beta);
        }
        k = JJ + 1;
        const double inv = hn > 0.0 ? 1.0 / hn : 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) V[JJ + 1][e] = w[e] * T(inv);
        return false;
    }

    // Solve [I - diag(sigma) D_{p+1}] y = x in place.  Returns iterations.
    __device__ __forceinline__ int solve(T (&x)[EPT], const double *sgp, T *xp, double *red, int &rb,
                                         GmresScalars *gs, int kmax, double rtol, int nx)
    {
        const int tid = threadIdx.x;
        double bb[1] = {0.0};
#pragma unroll
        for (int e = 0; e < EPT; ++e) bb[0] += double(x[e]) * double(x[e]);
        if (tid == 0) gs->flag = 0;
        block_sum_u<1>(bb, red, rb);
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
        step<0>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) || step<1>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) ||
            step<2>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) || step<3>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) ||
            step<4>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) || step<5>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) ||
            step<6>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) || step<7>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) ||
            step<8>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx) || step<9>(sgp, xp, red, rb, gs, kmax, rtol, beta, nx);
        // back substitution R z = g (thread 0), then y = V z
        if (tid == 0) {
            for (int i = k - 1; i >= 0; --i) {
                double s = gs->g[i];
                for (int t = i + 1; t < k; ++t) s -= gs->R[t][i] * gs->z[t];
                gs->z[i] = s / gs->R[i][i];
            }
        }
        __syncthreads();
        double y[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) y[e] = 0.0;
#pragma unroll
        for (int i = 0; i < SLM_KMAX; ++i)
            if (i < k) {
                const double zi = gs->z[i];
#pragma unroll
                for (int e = 0; e < EPT; ++e) y[e] += zi * double(V[i][e]);
            }
#pragma unroll
        for (int e = 0; e < EPT; ++e) x[e] = T(y[e]);
        return k;
    }
};

// Explicit forward-Euler correction of eq. (Fp_def) in place:
// x <- x + sigma .* (D_{p+1} x), with the same halo exchange through the
// padded LDS buffer as the GMRES stencil.  Ends with a barrier, so the
// buffer (aliased with the slice) may be rewritten afterwards.
template <typename T, int P, int EPT, bool FULL>
__device__ __forceinline__ void fwd_euler_apply(T (&x)[EPT], const double *sgp, T *xp, int nx)
{
    const int tid = threadIdx.x, i0 = tid * EPT;
#pragma unroll
    for (int e = 0; e < EPT; ++e)
        if (FULL || i0 + e < nx) xp[pidx<EPT>(i0 + e)] = x[e];
    __syncthreads();
    constexpr int q = DTaps<P>::q;
    T win[EPT + 2 * q];
#pragma unroll
    for (int t = 0; t < q; ++t) {
        int il = i0 - q + t;
        il += il < 0 ? nx : 0;
        int ir = i0 + EPT + t;
        ir -= ir >= nx ? nx : 0;
        win[t] = (FULL || i0 < nx) ? xp[pidx<EPT>(il)] : T(0);
        win[EPT + q + t] = (FULL || i0 < nx) ? xp[pidx<EPT>(ir)] : T(0);
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) win[q + e] = x[e];
    if (!FULL && i0 + EPT > nx) {
#pragma unroll
        for (int e = 0; e < EPT + q; ++e) {
            const int i = i0 + e;
            if (i >= nx && i - nx < nx) win[q + e] = xp[pidx<EPT>(i - nx)];
        }
    }
    T y[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        if (FULL || i0 + e < nx) {
            double dv = 0.0;
#pragma unroll
            for (int t = 0; t <= 2 * q; ++t) dv += DTaps<P>::t[t] * double(win[e + t]);
            y[e] = T(double(x[e]) + sgp[pidx<EPT>(i0 + e)] * dv);
        } else {
            y[e] = T(0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; ++e) x[e] = y[e];
}

// LDS layout of the coarse kernel: slice (natural order) aliased with the
// padded exchange buffer (the slice is dead while GMRES runs) | sigma
// (padded) | reduction scratch | Givens scalars.
template <typename T, int EPT>
__host__ __device__ inline size_t coarse_lds_parts(int nx, size_t *o_sg, size_t *o_red, size_t *o_gs)
{
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    const size_t np = (size_t)nx + nx / EPT + 1;
    size_t o = al(np * sizeof(T));
    *o_sg = o;
    o = al(o + np * sizeof(double));
    *o_red = o;
    o = al(o + SLM_RED_DOUBLES * sizeof(double));
    *o_gs = o;
    return o + sizeof(GmresScalars);
}

// FWD: the explicit forward-Euler correction replaces the GMRES solve (a
// variant of its own, so the GMRES kernel's register allocation is untouched).
template <typename T, int P, int EPT, bool FULL = false, bool FWD = false>
__device__ __forceinline__ void coarse_chain(const ChainArgs &a, int j, unsigned char *smem)
{
    const int tid = threadIdx.x, nx = a.nx;
    const long long S = a.S;
    size_t osg, ored, ogs;
    coarse_lds_parts<T, EPT>(nx, &osg, &ored, &ogs);
    T *sl = reinterpret_cast<T *>(smem);
    T *xp = sl;
    double *sgp = reinterpret_cast<double *>(smem + osg);
    double *red = reinterpret_cast<double *>(smem + ored);
    GmresScalars *gs = reinterpret_cast<GmresScalars *>(smem + ogs);
    const double *disp = static_cast<const double *>(a.disp);
    const T *Cin = static_cast<const T *>(a.Cin);
    const T *G = static_cast<const T *>(a.G);
    T *Vout = static_cast<T *>(a.Vout);
    T *Cout = static_cast<T *>(a.Cout);
    const long long n_first = a.n_base + (long long)j * a.stride_chain;
    const int i0 = tid * EPT;

    T val[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = i0 + e;
        T s = T(0);
        if (FULL || i < nx) {
            if (Cin) s = Cin[(long long)j * a.cin_stride + i];
            sl[i] = s;
            if (Vout && a.write_start) Vout[n_first * S + i] = s;
            if (Cout && j == 0 && a.cout_shift) Cout[i] = s;
        }
        val[e] = s;
    }
    __syncthreads();
    int rb = 0;
    Gmres1D<T, P, EPT, FULL> gm;
    unsigned long long nsolve = 0, niter = 0;
    // Displacements and sigma of the next step are loaded right after the
    // current step's solve, next to its G(n+1) loads: the step pays one
    // memory latency instead of two, and the registers are only live while
    // the Krylov basis is not.
    double dnx[EPT], snx[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = i0 + e;
        dnx[e] = (FULL || i < nx) && a.nsteps > 0 ? disp[n_first * S + i] : 0.0;
        snx[e] = (FULL || i < nx) && a.nsteps > 0 ? a.sigma[n_first * S + i] : 0.0;
    }
    for (int k = 0; k < a.nsteps; ++k) {
        const long long n = n_first + k;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = i0 + e;
            if (FULL || i < nx) sgp[pidx<EPT>(i)] = snx[e];
            val[e] = (FULL || i < nx) ? interp1<P, T, double>(sl, i, dnx[e], nx, 0) : T(0);
        }
        __syncthreads();                         // every read of the slice is done, sigma staged
        if constexpr (FWD) {
            fwd_euler_apply<T, P, EPT, FULL>(val, sgp, xp, nx);
        } else {
            niter += gm.solve(val, sgp, xp, red, rb, gs, a.kmax, a.rtol, nx);
            ++nsolve;
        }
        const long long nn = k + 1 < a.nsteps ? n + 1 : n;    // the last step re-reads its own (cached) rows
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = i0 + e;
            dnx[e] = (FULL || i < nx) ? disp[nn * S + i] : 0.0;
            snx[e] = (FULL || i < nx) ? a.sigma[nn * S + i] : 0.0;
        }
        // G(n+1) in one batch of loads (a per-node test of G would issue and
        // wait for them one at a time)
        T gv[EPT];
#pragma unroll
        for (int e = 0; e < EPT; ++e) gv[e] = T(0);
        if (G) {
            const T *gn = G + (n + 1) * S;
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                if (FULL || i0 + e < nx) gv[e] = gn[i0 + e];
        }
        const bool wv = Vout && (k + 1 < a.nsteps || a.write_last);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = i0 + e;
            if (FULL || i < nx) {
                if (G) val[e] += gv[e];
                sl[i] = val[e];
                if (wv) Vout[(n + 1) * S + i] = val[e];
            }
        }
        __syncthreads();
    }
    if (Cout) {
#pragma unroll
        for (int e = 0; e < EPT; ++e)
            if (FULL || i0 + e < nx) Cout[(long long)(j + a.cout_shift) * S + i0 + e] = val[e];
    }
    if (a.R) {
        const T *Cref = static_cast<const T *>(a.Cref);
        T *R = static_cast<T *>(a.R);
        double acc[1] = {0.0};
        T cv[EPT];                               // Cref in one batch of loads
#pragma unroll
        for (int e = 0; e < EPT; ++e) cv[e] = T(0);
        if (Cref) {
#pragma unroll
            for (int e = 0; e < EPT; ++e)
                if (FULL || i0 + e < nx) cv[e] = Cref[(long long)(j + 1) * S + i0 + e];
        }
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = i0 + e;
            if (FULL || i < nx) {
                const T r = Cref ? T(val[e] - cv[e]) : val[e];
                R[(long long)(j + 1) * S + i] = r;
                acc[0] += double(r) * double(r);
            }
        }
        block_sum<1>(acc, red, rb);
        if (tid == 0) a.partial[j] = acc[0];
    }
    if (tid == 0 && a.counter) {
        atomicAdd(a.counter, nsolve);
        atomicAdd(a.counter + 1, niter);
    }
}

template <typename T, int P, int EPT, bool FULL, bool FWD = false>
__global__ void __launch_bounds__(COARSE_MAXB) coarse1d(ChainArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    coarse_chain<T, P, EPT, FULL, FWD>(a, blockIdx.x, smem);
}

// Prefetch depth of the displacement ring: about 64 bytes per lane in
// flight, between 1 and 4 steps.
template <typename TD, int EPT>
constexpr int pf_depth()
{
    return 64 / ((int)sizeof(TD) * EPT) < 1 ? 1 : (64 / ((int)sizeof(TD) * EPT) > 4 ? 4 : 64 / ((int)sizeof(TD) * EPT));
}

}  // namespace slmk
