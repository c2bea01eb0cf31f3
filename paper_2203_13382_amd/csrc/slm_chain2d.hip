// slm_chain2d.hip -- relaxation sweeps on a periodic 2D mesh (and the
// sweeps of the adjoint system, 1D and 2D).
//
// A 2D slice (nx*nx values) does not fit in one CU's LDS, so a sweep over m
// level steps is a sequence of launches, one per step index, each advancing
// every coarse interval ("chain") of the sweep at once: the grid spans the
// points of a slice times the chains.  Slices in flight live in a
// ping-pong work buffer in HBM.
//
// Level 0 applies the tensor-product semi-Lagrangian step (Sec. 4.1).
// Coarse levels apply eq. (BEOper_2D) with the multilevel sigma of Sec. 4.3:
//     v <- [I - diag(sx) D_x - diag(sy) D_y]^{-1} S_{p,r*} v,
// D_x = I (x) D_{p+1}, D_y = D_{p+1} (x) I.  The inverse is applied by GMRES
// (zero guess, classical Gram-Schmidt in one pass with the new vector's norm
// reduced from the vector, Givens, exit at rtol or kmax),
// batched over the chains: every Arnoldi phase is one launch over all
// systems, inner products are per-block FP64 partial sums reduced in a fixed
// order, and a one-thread-per-system kernel runs the Givens recurrence.
// Converged systems skip their work through a per-system flag.
//
// Adjoint mode (ChainArgs.adj) runs the same sweeps on the reverse-time
// adjoint system: level 0 applies S_n^T of the mirrored forward step, the
// coarse levels S_l^T [I - D_x diag(sx) - D_y diag(sy)]^{-1}: the GMRES
// right-hand side is the incoming slice, the matvec the transposed one, and
// the transposed interpolation follows the solve.
#include <climits>
#include <cmath>
#include <type_traits>

#include "slm_internal.h"

namespace {

constexpr int TPB = 256;            // threads per block of the point kernels
constexpr int NPART = 16;           // partial-sum slots per block
constexpr int WWS = SLM_KMAX + 1;   // slot of ||w||^2 beside the projections 0..j

// ------------------------------------------------------------ interpolation
template <int P, typename T, typename TD>
__device__ __forceinline__ T interp2(const T *__restrict__ s, int i, int j, TD dx, TD dy, int nx)
{
    const TD fx = floor(dx), fy = floor(dy);
    const T ex = T(dx - fx), ey = T(dy - fy);
    const int firstx = stencil_first<T>(P, ex), firsty = stencil_first<T>(P, ey);
    const int bx = wrap_mod(i - int(fx) + firstx, nx);
    const int by = wrap_mod(j - int(fy) + firsty, nx);
    T wx[P + 1], wy[P + 1];
    interp_weights<P, T>(ex, wx);
    interp_weights<P, T>(ey, wy);
    T acc = T(0);
#pragma unroll
    for (int b = 0; b <= P; ++b) {
        int row = by + b;
        row -= row >= nx ? nx : 0;
        const T *sr = s + (long long)row * nx;
        T ar = T(0);
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            int col = bx + a;
            col -= col >= nx ? nx : 0;
            ar += wx[a] * sr[col];
        }
        acc += wy[b] * ar;
    }
    return acc;
}

// One level step for every chain c: dst[c] = S(n_c) src[c] (+ G[n_c+1]).
// n_c = n_first + c*stride.  src may be null (zero start).
template <typename T, typename TD, int P>
__global__ void __launch_bounds__(TPB) step2d_kernel(const T *__restrict__ src, long long src_stride,
                                                     T *__restrict__ dst, long long dst_stride,
                                                     const TD *__restrict__ disp, long long plane, int nx,
                                                     long long n_first, int stride, const T *__restrict__ G,
                                                     T *__restrict__ Vout)
{
    const long long S = (long long)nx * nx;
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const T *s = src ? src + c * src_stride : nullptr;
    T *d = dst + c * dst_stride;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        int i, j;
        split_xy(id, nx, i, j);
        T v = s ? interp2<P, T, TD>(s, i, j, disp[n * S + id], disp[plane + n * S + id], nx) : T(0);
        if (G) v += G[(n + 1) * S + id];
        d[id] = v;
        if (Vout) Vout[(n + 1) * S + id] = v;
    }
}

// Level-0 step with the source window staged in LDS.  A workgroup computes a
// TX x TY tile of outputs; every departure point of the tile lies within F
// cells of its node (F bounds |floor(d)| from the wave speed), so the tile's
// stencils read only the window [x0 - F - LO, x0 + TX - 1 + F + HI] x (same in
// y), loaded once with coalesced reads.  The (p+1)^2-tap gathers then hit LDS
// instead of the texture path.  A stencil outside the window (not expected)
// falls back to global reads, so the result never depends on F, and every
// output is formed by the same products in the same order whatever the tile
// shape (the autotuner's choice, slm_autotune).
struct TileShape { int tx, ty; };
constexpr TileShape kTiles[] = {{64, 16}, {64, 32}, {128, 16}, {128, 32}};
constexpr int kNumTiles = 4;

template <typename T, typename TD, int P, int TX, int TY, bool PRE>
__global__ void __launch_bounds__(TPB) step2d_tile_kernel(const T *__restrict__ src, long long src_stride,
                                                          T *__restrict__ dst, long long dst_stride,
                                                          const TD *__restrict__ disp, long long plane, int nx,
                                                          long long n_first, int stride, const T *__restrict__ G,
                                                          T *__restrict__ Vout, int F, unsigned inv_wx)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *win = reinterpret_cast<T *>(smem_raw);
    constexpr int LO = P / 2 + 1, HI = P / 2;      // node offsets around x_E, any p
    const long long S = (long long)nx * nx;
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const T *s = src + c * src_stride;
    const int ntx = (nx + TX - 1) / TX;
    const int x0 = (int)(blockIdx.x % ntx) * TX, y0 = (int)(blockIdx.x / ntx) * TY;
    const int wx = TX + 2 * F + LO + HI, wy = TY + 2 * F + LO + HI;
    const int ox = x0 - F - LO, oy = y0 - F - LO;   // window origin (unwrapped)
    // PRE (launches of a few hundred workgroups, e.g. sequential stepping,
    // where each CU waits on its own loads): this thread's outputs are nodes
    // threadIdx.x + u * TPB of the tile, and their displacements are
    // requested before the window is staged so the loads overlap it.  Big
    // sweeps keep the registers for occupancy instead.
    constexpr int NPT = TX * TY / TPB;
    static_assert(TX * TY % TPB == 0, "a tile is a whole number of workgroup rows");
    TD dxr[NPT], dyr[NPT];
    if constexpr (PRE) {
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int k = threadIdx.x + u * TPB, ly = k / TX, lx = k - ly * TX;
            const int i = x0 + lx, j = y0 + ly;
            const long long id = (long long)j * nx + i;
            const bool in = i < nx && j < nx;
            dxr[u] = in ? disp[n * S + id] : TD(0);
            dyr[u] = in ? disp[plane + n * S + id] : TD(0);
        }
    }
    // Every window coordinate lies in (-nx, 2 nx) (checked on the host), so
    // one conditional add or subtract wraps it; k / wx is a multiply by a
    // 24-bit reciprocal, exact for k < wx * wy.
    for (int k = threadIdx.x; k < wx * wy; k += TPB) {
        const int r = (int)(((unsigned long long)(unsigned)k * inv_wx) >> 24), q = k - r * wx;
        int gy = oy + r, gx = ox + q;
        gy += gy < 0 ? nx : 0;
        gy -= gy >= nx ? nx : 0;
        gx += gx < 0 ? nx : 0;
        gx -= gx >= nx ? nx : 0;
        win[k] = s[(long long)gy * nx + gx];
    }
    __syncthreads();
    // output k of the tile from its displacement (dx, dy)
    auto output = [&](int k, TD dx, TD dy) {
        const int ly = k / TX, lx = k - ly * TX;
        const int i = x0 + lx, j = y0 + ly;
        const long long id = (long long)j * nx + i;
        const TD fx = floor(dx), fy = floor(dy);
        const T ex = T(dx - fx), ey = T(dy - fy);
        const int firstx = stencil_first<T>(P, ex), firsty = stencil_first<T>(P, ey);
        const int bx = i - int(fx) + firstx - ox, by = j - int(fy) + firsty - oy;   // window coordinates
        T v;
        if (bx >= 0 && by >= 0 && bx + P < wx && by + P < wy) {
            T wxv[P + 1], wyv[P + 1];
            interp_weights<P, T>(ex, wxv);
            interp_weights<P, T>(ey, wyv);
            T acc = T(0);
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                const T *row = win + (by + b) * wx + bx;
                T ar = T(0);
#pragma unroll
                for (int a = 0; a <= P; ++a) ar += wxv[a] * row[a];
                acc += wyv[b] * ar;
            }
            v = acc;
        } else {
            v = interp2<P, T, TD>(s, i, j, dx, dy, nx);
        }
        if (G) v += G[(n + 1) * S + id];
        dst[c * dst_stride + id] = v;
        if (Vout) Vout[(n + 1) * S + id] = v;
    };
    if constexpr (PRE) {
        // opaque thread index: the output addresses are formed again here
        // rather than kept live from the loads above
        int t = threadIdx.x;
        __asm__ volatile("" : "+v"(t));
#pragma unroll
        for (int u = 0; u < NPT; ++u) {
            const int k = t + u * TPB, ly = k / TX, lx = k - ly * TX;
            if (x0 + lx < nx && y0 + ly < nx) output(k, dxr[u], dyr[u]);
        }
    } else {
        for (int k = threadIdx.x; k < TX * TY; k += TPB) {
            const int ly = k / TX, lx = k - ly * TX;
            const int i = x0 + lx, j = y0 + ly;
            if (i >= nx || j >= nx) continue;
            const long long id = (long long)j * nx + i;
            output(k, disp[n * S + id], disp[plane + n * S + id]);
        }
    }
}

// Coarse-level step with a per-tile window: a workgroup computes a WX x WY
// tile of outputs.  It first reads the tile's departure points, then stages
// in LDS the bounding box of all their stencils (periodically wrapped), so
// the (p+1)^2-tap gathers hit LDS.  Coarse displacements are large but vary
// slowly across a tile, so the box stays a small multiple of the tile.  A
// tile whose box exceeds the LDS budget or the mesh gathers from global
// memory instead.  Both paths form every output from interp2's products in
// interp2's order, so the result never depends on the path.
constexpr int WX = 64, WY = 16;
constexpr int WIN_LDS_BYTES = 24 * 1024;

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int o = SLM_WAVE / 2; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = SLM_WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

template <typename T, typename TD, int P>
__global__ void __launch_bounds__(TPB) step2d_win_kernel(const T *__restrict__ src, long long src_stride,
                                                         T *__restrict__ dst, long long dst_stride,
                                                         const TD *__restrict__ disp, long long plane, int nx,
                                                         long long n_first, int stride, const T *__restrict__ G,
                                                         T *__restrict__ Vout)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *win = reinterpret_cast<T *>(smem_raw);
    __shared__ int mm[4][TPB / SLM_WAVE];
    constexpr int K = WX * WY / TPB;
    const long long S = (long long)nx * nx;
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const T *s = src + c * src_stride;
    const int ntx = (nx + WX - 1) / WX;
    const int x0 = (int)(blockIdx.x % ntx) * WX, y0 = (int)(blockIdx.x / ntx) * WY;
    TD dxs[K], dys[K];
    T ex[K], ey[K];
    int gx[K], gy[K];
    int xlo = INT_MAX, xhi = INT_MIN, ylo = INT_MAX, yhi = INT_MIN;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int e = threadIdx.x + k * TPB, i = x0 + e % WX, j = y0 + e / WX;
        gx[k] = INT_MIN;
        if (i < nx && j < nx) {
            const long long id = (long long)j * nx + i;
            const TD dx = disp[n * S + id], dy = disp[plane + n * S + id];
            dxs[k] = dx;
            dys[k] = dy;
            const TD fx = floor(dx), fy = floor(dy);
            ex[k] = T(dx - fx);
            ey[k] = T(dy - fy);
            gx[k] = i - int(fx) + stencil_first<T>(P, ex[k]);     // unwrapped stencil origin
            gy[k] = j - int(fy) + stencil_first<T>(P, ey[k]);
            xlo = min(xlo, gx[k]);
            xhi = max(xhi, gx[k]);
            ylo = min(ylo, gy[k]);
            yhi = max(yhi, gy[k]);
        }
    }
    const int wid = threadIdx.x / SLM_WAVE, lane = threadIdx.x % SLM_WAVE;
    xlo = wave_min_i(xlo);
    xhi = wave_max_i(xhi);
    ylo = wave_min_i(ylo);
    yhi = wave_max_i(yhi);
    if (lane == 0) {
        mm[0][wid] = xlo;
        mm[1][wid] = xhi;
        mm[2][wid] = ylo;
        mm[3][wid] = yhi;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < TPB / SLM_WAVE; ++w) {
        xlo = min(xlo, mm[0][w]);
        xhi = max(xhi, mm[1][w]);
        ylo = min(ylo, mm[2][w]);
        yhi = max(yhi, mm[3][w]);
    }
    // box of every stencil of the tile (the tile always holds a mesh node)
    const long long bw = (long long)xhi - xlo + P + 1, bh = (long long)yhi - ylo + P + 1;
    const bool staged = bw <= nx && bh <= nx && bw * bh * (long long)sizeof(T) <= WIN_LDS_BYTES;
    if (staged) {
        const int w = (int)bw, hgt = (int)bh;
        int ox = xlo % nx, oy = ylo % nx;
        ox += ox < 0 ? nx : 0;
        oy += oy < 0 ? nx : 0;
        for (int r = wid; r < hgt; r += TPB / SLM_WAVE) {          // one wave per box row
            int gyy = oy + r;
            gyy -= gyy >= nx ? nx : 0;
            const T *row = s + (long long)gyy * nx;
            for (int q = lane; q < w; q += SLM_WAVE) {
                int gxx = ox + q;
                gxx -= gxx >= nx ? nx : 0;
                win[r * w + q] = row[gxx];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (gx[k] == INT_MIN) continue;
        const int e = threadIdx.x + k * TPB, i = x0 + e % WX, j = y0 + e / WX;
        const long long id = (long long)j * nx + i;
        T v;
        if (staged) {
            const int w = (int)bw;
            const int bx = gx[k] - xlo, by = gy[k] - ylo;
            T wxv[P + 1], wyv[P + 1];
            interp_weights<P, T>(ex[k], wxv);
            interp_weights<P, T>(ey[k], wyv);
            T acc = T(0);
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                const T *row = win + (by + b) * w + bx;
                T ar = T(0);
#pragma unroll
                for (int a = 0; a <= P; ++a) ar += wxv[a] * row[a];
                acc += wyv[b] * ar;
            }
            v = acc;
        } else {
            v = interp2<P, T, TD>(s, i, j, dxs[k], dys[k], nx);
        }
        if (G) v += G[(n + 1) * S + id];
        dst[c * dst_stride + id] = v;
        if (Vout) Vout[(n + 1) * S + id] = v;
    }
}

// Chain epilogue: Cout[c+shift] = last[c]; or residual R[c+1] = last[c] - Cref[c+1]
// with per-(chain, block) partial sums of squares.
template <typename T>
__global__ void __launch_bounds__(TPB) finish2d_kernel(const T *__restrict__ last, long long S, T *Cout, int shift,
                                                       const T *__restrict__ Cref, T *R, double *partial)
{
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.y;
    double acc[1] = {0.0};
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        const T v = last[c * S + id];
        if (Cout) Cout[(c + shift) * S + id] = v;
        if (R) {
            const T r = Cref ? T(v - Cref[(c + 1) * S + id]) : v;
            R[(c + 1) * S + id] = r;
            acc[0] += double(r) * double(r);
        }
    }
    if (R) {
        block_sum<1>(acc, red, 0);
        if (threadIdx.x == 0) partial[(long long)c * gridDim.x + blockIdx.x] = acc[0];
    }
}

// Start slices: dst[c] = src[c*stride] or 0; optional Vout[n_first(c)] and Cout[0].
template <typename T>
__global__ void __launch_bounds__(TPB) start2d_kernel(const T *__restrict__ Cin, long long cin_stride, T *dst,
                                                      long long S, T *Vout, long long n_first, int stride,
                                                      T *Cout0)
{
    const int c = blockIdx.y;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        const T v = Cin ? Cin[c * cin_stride + id] : T(0);
        dst[c * S + id] = v;
        if (Vout) Vout[(n_first + (long long)c * stride) * S + id] = v;
        if (Cout0 && c == 0) Cout0[id] = v;
    }
}

// ------------------------------------------------------------ batched GMRES
// (per-system Givens state Gs2 is declared in slm_internal.h)

template <int NV>
__device__ __forceinline__ void write_parts(double (&v)[NV], double *red, double *part, int c)
{
    block_sum<NV>(v, red, 0);
    if (threadIdx.x < NV) part[((long long)c * gridDim.x + blockIdx.x) * NPART + threadIdx.x] = v[threadIdx.x];
}

// partials of b.b
template <typename T>
__global__ void __launch_bounds__(TPB) g2_norm0(const T *__restrict__ b, long long S, double *part)
{
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.y;
    double v[1] = {0.0};
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        const double x = b[c * S + id];
        v[0] += x * x;
    }
    write_parts<1>(v, red, part, c);
}

// Fixed-order reduction of the per-block partials of system c: one
// workgroup sums the nb blocks' slots q < nv (each thread a strided subset,
// then a deterministic workgroup tree); every thread receives the totals.
template <int NV>
__device__ __forceinline__ void sum_parts(const double *part, int nb, int nv, int c, double (&v)[NV], double *red,
                                          int buf)
{
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nb; b += TPB) {
        const double *pp = part + ((long long)c * nb + b) * NPART;
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q < nv) v[q] += pp[q];
    }
    block_sum_rs<NV>(v, red, buf);
}

// Totals of the per-block partials, one workgroup per system, into
// out[c][q] (q < nv).  Systems already converged are skipped when gs is given.
__global__ void __launch_bounds__(TPB) g2_sum(const double *__restrict__ part, int nb, int nv, const Gs2 *gs,
                                              double *__restrict__ out)
{
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.x;
    if (gs && gs[c].done) return;
    double v[SLM_KMAX + 1];
    sum_parts(part, nb, nv, c, v, red, 0);
    if (threadIdx.x < nv) out[(long long)c * NPART + threadIdx.x] = v[threadIdx.x];
}

// beta = ||b|| from the reduced b.b, V0 = b / beta
template <typename T>
__global__ void __launch_bounds__(TPB) g2_start(const T *__restrict__ b, long long S, const double *bb, T *V,
                                                 Gs2 *gs, int kmax)
{
    const int c = blockIdx.y;
    const double beta = sqrt(bb[(long long)c * NPART]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Gs2 &g = gs[c];
        g.beta = beta;
        g.k = 0;
        g.done = (beta == 0.0 || kmax <= 0) ? 1 : 0;
        g.g[0] = beta;
        for (int i = 1; i <= SLM_KMAX; ++i) g.g[i] = 0.0;
    }
    if (beta == 0.0) return;
    const double inv = 1.0 / beta;
    T *V0 = V + (long long)c * (SLM_KMAX + 1) * S;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB)
        V0[id] = T(double(b[c * S + id]) * inv);
}

// Arnoldi step j of every system c (blockIdx.y):
//   v = V_0 (j = 0) or w_{j-1} / hn_{j-1}, the previous step's vector
//       normalised here (and stored as V_j) rather than in a launch of its own;
//   w = v - sx .* (D_x v) - sy .* (D_y v), or for the adjoint system
//       (transpose) w = v - D_x (sx .* v) - D_y (sy .* v), where the
//       difference sums run over w_{j-1} and take the factor 1/hn_{j-1} once;
// then the partials of the projections V_i . w (i <= j, zero above) and of
// w . w (slot WWS).  1D slices have no y term.  The sigma of step n (or of Nl-1-n when rev) is read in TS: FP64,
// or its float copy for FP32 bulk.
template <typename T, typename TS, int P>
__global__ void __launch_bounds__(TPB) g2_matvec(T *__restrict__ V, const T *__restrict__ Wsrc, T *__restrict__ Wdst,
                                                  long long S, int nx, const TS *__restrict__ sig, long long plane,
                                                  long long n_first, int stride, int j, const Gs2 *gs, double *part,
                                                  int dim, int transpose, int rev, int Nl)
{
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.y;
    if (gs[c].done) return;
    const long long n0 = n_first + (long long)c * stride;
    const long long n = rev ? Nl - 1 - n0 : n0;
    T *Vc = V + (long long)c * (SLM_KMAX + 1) * S;
    const T *src = j == 0 ? Vc : Wsrc + (long long)c * S;
    double inv = 1.0;
    if (j > 0) {
        const double hn = gs[c].hn[j - 1];
        inv = hn > 0.0 ? 1.0 / hn : 0.0;
    }
    const TS *sx = sig + n * S, *sy = sig + plane + n * S;
    constexpr int q = DTaps<P>::q;
    double h[WWS + 1];
#pragma unroll
    for (int i = 0; i <= WWS; ++i) h[i] = 0.0;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        int i, jr;
        split_xy(id, nx, i, jr);
        if (dim != 2) jr = 0;
        double dxv = 0.0, dyv = 0.0;
#pragma unroll
        for (int t = -q; t <= q; ++t) {
            int ii = i + t;
            ii += ii < 0 ? nx : 0;
            ii -= ii >= nx ? nx : 0;
            const long long ix = (long long)jr * nx + ii;
            dxv += DTaps<P>::t[t + q] * (transpose ? double(sx[ix]) * double(src[ix]) : double(src[ix]));
            if (dim == 2) {
                int jj = jr + t;
                jj += jj < 0 ? nx : 0;
                jj -= jj >= nx ? nx : 0;
                const long long iy = (long long)jj * nx + i;
                dyv += DTaps<P>::t[t + q] * (transpose ? double(sy[iy]) * double(src[iy]) : double(src[iy]));
            }
        }
        dxv *= inv;
        dyv *= inv;
        const T vj = T(double(src[id]) * inv);             // V_j at this node
        if (j > 0) Vc[(long long)j * S + id] = vj;
        const double yterm = dim == 2 ? (transpose ? dyv : double(sy[id]) * dyv) : 0.0;
        const T w = T(double(vj) - (transpose ? dxv : double(sx[id]) * dxv) - yterm);
        Wdst[c * S + id] = w;
#pragma unroll
        for (int k = 0; k <= SLM_KMAX; ++k)
            if (k <= j) h[k] += double(k == j ? vj : Vc[(long long)k * S + id]) * double(w);
        h[WWS] += double(w) * double(w);
    }
    block_sum_rs<WWS + 1>(h, red, 0);
    if (threadIdx.x <= WWS) part[((long long)c * gridDim.x + blockIdx.x) * NPART + threadIdx.x] = h[threadIdx.x];
}

// The same Arnoldi matvec for a 2D system whose mesh splits exactly into
// the blocks' WX x WY tiles: the block stages its tile of w_{j-1} (or V_0)
// with q cells of halo on every side in LDS, so the 2(2q+1) difference taps
// of a node read LDS instead of the cache hierarchy.  The adjoint operator
// (TRANS) differences sigma .* v: it stages the products sx .* v and
// sy .* v, rounded as the untiled kernel rounds them.  Per node the
// arithmetic is the untiled kernel's; only the nodes each block's partial
// projections gather differ.
template <typename T, typename TS, int P, bool TRANS>
__global__ void __launch_bounds__(TPB) g2_matvec_tile(T *__restrict__ V, const T *__restrict__ Wsrc,
                                                       T *__restrict__ Wdst, long long S, int nx,
                                                       const TS *__restrict__ sig, long long plane, long long n_first,
                                                       int stride, int j, const Gs2 *gs, double *part, int rev, int Nl)
{
    constexpr int q = DTaps<P>::q;
    constexpr int HX = WX + 2 * q, HY = WY + 2 * q;
    using TT = typename std::conditional<TRANS, double, T>::type;   // staged type
    __shared__ TT tile[TRANS ? 2 : 1][HY * HX];
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.y;
    if (gs[c].done) return;
    const long long n0 = n_first + (long long)c * stride;
    const long long n = rev ? Nl - 1 - n0 : n0;
    T *Vc = V + (long long)c * (SLM_KMAX + 1) * S;
    const T *src = j == 0 ? Vc : Wsrc + (long long)c * S;
    double inv = 1.0;
    if (j > 0) {
        const double hn = gs[c].hn[j - 1];
        inv = hn > 0.0 ? 1.0 / hn : 0.0;
    }
    const TS *sx = sig + n * S, *sy = sig + plane + n * S;
    const int ntx = nx / WX;
    const int x0 = (int)(blockIdx.x % ntx) * WX, y0 = (int)(blockIdx.x / ntx) * WY;
    for (int k = threadIdx.x; k < HX * HY; k += TPB) {
        const int r = k / HX, cc = k - r * HX;
        int gy = y0 - q + r, gx = x0 - q + cc;
        gy += gy < 0 ? nx : 0;
        gy -= gy >= nx ? nx : 0;
        gx += gx < 0 ? nx : 0;
        gx -= gx >= nx ? nx : 0;
        const long long g = (long long)gy * nx + gx;
        if constexpr (TRANS) {
            tile[0][k] = double(sx[g]) * double(src[g]);
            tile[1][k] = double(sy[g]) * double(src[g]);
        } else {
            tile[0][k] = src[g];
        }
    }
    __syncthreads();
    double h[WWS + 1];
#pragma unroll
    for (int i = 0; i <= WWS; ++i) h[i] = 0.0;
#pragma unroll
    for (int k = 0; k < WX * WY / TPB; ++k) {
        const int e = threadIdx.x + k * TPB, lx = e % WX, ly = e / WX;
        const long long id = (long long)(y0 + ly) * nx + x0 + lx;
        const int co = (ly + q) * HX + lx + q;
        double dxv = 0.0, dyv = 0.0;
#pragma unroll
        for (int t = -q; t <= q; ++t) {
            dxv += DTaps<P>::t[t + q] * double(tile[0][co + t]);
            dyv += DTaps<P>::t[t + q] * double(tile[TRANS ? 1 : 0][co + t * HX]);
        }
        dxv *= inv;
        dyv *= inv;
        const T vj = T(double(src[id]) * inv);
        if (j > 0) Vc[(long long)j * S + id] = vj;
        const T w = TRANS ? T(double(vj) - dxv - dyv)
                          : T(double(vj) - double(sx[id]) * dxv - double(sy[id]) * dyv);
        Wdst[c * S + id] = w;
#pragma unroll
        for (int kk = 0; kk <= SLM_KMAX; ++kk)
            if (kk <= j) h[kk] += double(kk == j ? vj : Vc[(long long)kk * S + id]) * double(w);
        h[WWS] += double(w) * double(w);
    }
    block_sum_rs<WWS + 1>(h, red, 0);
    if (threadIdx.x <= WWS) part[((long long)c * gridDim.x + blockIdx.x) * NPART + threadIdx.x] = h[threadIdx.x];
}

// Givens recurrence of system g after Arnoldi step j: h = the Gram-Schmidt
// coefficients, hn the norm of the orthogonalised vector (Sec. 3.3 GMRES,
// same arithmetic order as the 1D kernel).  One thread.
__device__ __forceinline__ void givens_step(Gs2 &g, int j, const double *h1, double hn, double rtol, int kmax)
{
    double hc[SLM_KMAX + 1];
    for (int i = 0; i <= j; ++i) hc[i] = h1[i];
    for (int i = 0; i < j; ++i) {
        const double t0 = g.cs[i] * hc[i] + g.sn[i] * hc[i + 1];
        const double t1 = -g.sn[i] * hc[i] + g.cs[i] * hc[i + 1];
        hc[i] = t0;
        hc[i + 1] = t1;
    }
    const double den = sqrt(hc[j] * hc[j] + hn * hn);
    const double cc = hc[j] / den, ss = hn / den;
    g.cs[j] = cc;
    g.sn[j] = ss;
    hc[j] = den;
    const double gj = g.g[j];
    g.g[j + 1] = -ss * gj;
    g.g[j] = cc * gj;
    for (int i = 0; i <= j; ++i) g.R[j][i] = hc[i];
    g.hn[j] = hn;
    g.k = j + 1;
    if (hn == 0.0 || fabs(ss * gj) <= rtol * g.beta || j + 1 >= kmax) g.done = 1;
}

// w -= sum_i h_i V_i with the reduced h (i <= j), then the partials of w . w.
template <typename T>
__global__ void __launch_bounds__(TPB) g2_update(const T *__restrict__ V, T *__restrict__ W, long long S, int j,
                                                  const Gs2 *gs, const double *__restrict__ hin, double *part)
{
    __shared__ double red[SLM_RED_DOUBLES];
    __shared__ double hs[SLM_KMAX + 1];
    const int c = blockIdx.y;
    if (gs[c].done) return;
    const int nb = gridDim.x;
    if (threadIdx.x <= j) hs[threadIdx.x] = hin[(long long)c * NPART + threadIdx.x];
    __syncthreads();
    const T *Vc = V + (long long)c * (SLM_KMAX + 1) * S;
    double h[SLM_KMAX + 1];
#pragma unroll
    for (int i = 0; i <= SLM_KMAX; ++i) h[i] = 0.0;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        double t = double(W[c * S + id]);
        for (int k = 0; k <= j; ++k) t -= hs[k] * double(Vc[(long long)k * S + id]);
        const T w = T(t);
        W[c * S + id] = w;
        h[0] += double(w) * double(w);
    }
    block_sum_rs<SLM_KMAX + 1>(h, red, 0);
    if (threadIdx.x == 0) part[((long long)c * nb + blockIdx.x) * NPART] = h[0];
}

// Totals of the matvec's partials (projections h and ||w||^2, one workgroup
// per system, fixed order) into h1; the new vector's norm by Pythagoras,
// ||w - V h||^2 = ||w||^2 - sum h_i^2, and the Givens step, unless that
// difference is below 1e-3 ||w||^2: then the system is marked to take its
// norm from the updated vector (g2_norm_givens).
__global__ void __launch_bounds__(TPB) g2_sum_givens(const double *__restrict__ part, int nb, Gs2 *gs, int j,
                                                     double *__restrict__ h1, double rtol, int kmax)
{
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.x;
    if (gs[c].done) return;
    double v[WWS + 1];
    sum_parts(part, nb, WWS + 1, c, v, red, 0);
    if (threadIdx.x <= j) h1[(long long)c * NPART + threadIdx.x] = v[threadIdx.x];
    if (threadIdx.x == 0) {
        const double ww = v[WWS];
        double hn2 = ww;
        for (int i = 0; i <= j; ++i) hn2 -= v[i] * v[i];
        Gs2 &g = gs[c];
        g.need = !(hn2 >= 1e-3 * ww);
        if (!g.need) givens_step(g, j, v, sqrt(hn2 > 0.0 ? hn2 : 0.0), rtol, kmax);
    }
}

// The explicit norm for the systems g2_sum_givens marked: ||w|| from the
// update's partials (one workgroup per system, fixed order), then the Givens
// step.  h1: the reduced projections.
__global__ void __launch_bounds__(TPB) g2_norm_givens(const double *__restrict__ part, int nb, Gs2 *gs, int j,
                                                      const double *__restrict__ h1, double rtol, int kmax)
{
    __shared__ double red[SLM_RED_DOUBLES];
    const int c = blockIdx.x;
    if (gs[c].done || !gs[c].need) return;
    double v[SLM_KMAX + 1];
    sum_parts(part, nb, 1, c, v, red, 0);
    if (threadIdx.x == 0) givens_step(gs[c], j, h1 + (long long)c * NPART, sqrt(v[0]), rtol, kmax);
}

// y = V z (back substitution per block), then dst[c] = y (+ G[n+1]), Vout.
template <typename T>
__global__ void __launch_bounds__(TPB) g2_combine(const T *__restrict__ V, long long S, const Gs2 *gs, T *dst,
                                                   long long dst_stride, long long n_first, int stride,
                                                   const T *__restrict__ G, T *Vout)
{
    __shared__ double z[SLM_KMAX];
    const int c = blockIdx.y;
    const Gs2 &g = gs[c];
    const int k = g.k;
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double s = g.g[i];
            for (int t = i + 1; t < k; ++t) s -= g.R[t][i] * z[t];
            z[i] = s / g.R[i][i];
        }
    }
    __syncthreads();
    const long long n = n_first + (long long)c * stride;
    const T *Vc = V + (long long)c * (SLM_KMAX + 1) * S;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        double y = 0.0;
        for (int i = 0; i < k; ++i) y += z[i] * double(Vc[(long long)i * S + id]);
        T v = T(y);
        if (G) v += G[(n + 1) * S + id];
        dst[c * dst_stride + id] = v;
        if (Vout) Vout[(n + 1) * S + id] = v;
    }
}

// Explicit forward-Euler correction of eq. (Fp_def) on the interpolated
// slices b (one per chain): dst = b + sx .* (D_x b) + sy .* (D_y b), plus
// G(n+1), also written to Vout.
template <typename T, int P>
__global__ void __launch_bounds__(TPB) fwd2d_kernel(const T *__restrict__ B, long long S, int nx,
                                                    const double *__restrict__ sig, long long plane, long long n_first,
                                                    int stride, int dim, T *dst, long long dst_stride,
                                                    const T *__restrict__ G, T *Vout)
{
    const int c = blockIdx.y;
    const long long n = n_first + (long long)c * stride;
    const T *b = B + (long long)c * S;
    const double *sx = sig + n * S, *sy = sig + plane + n * S;
    constexpr int q = DTaps<P>::q;
    for (long long id = (long long)blockIdx.x * TPB + threadIdx.x; id < S; id += (long long)gridDim.x * TPB) {
        int i, jr;
        split_xy(id, nx, i, jr);
        if (dim != 2) jr = 0;
        double dxv = 0.0, dyv = 0.0;
#pragma unroll
        for (int t = -q; t <= q; ++t) {
            int ii = i + t;
            ii += ii < 0 ? nx : 0;
            ii -= ii >= nx ? nx : 0;
            dxv += DTaps<P>::t[t + q] * double(b[(long long)jr * nx + ii]);
            if (dim == 2) {
                int jj = jr + t;
                jj += jj < 0 ? nx : 0;
                jj -= jj >= nx ? nx : 0;
                dyv += DTaps<P>::t[t + q] * double(b[(long long)jj * nx + i]);
            }
        }
        double y = double(b[id]) + sx[id] * dxv;
        if (dim == 2) y += sy[id] * dyv;
        T v = T(y);
        if (G) v += G[(n + 1) * S + id];
        dst[c * dst_stride + id] = v;
        if (Vout) Vout[(n + 1) * S + id] = v;
    }
}

__global__ void g2_count(const Gs2 *gs, int nsys, unsigned long long *counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long it = 0;
        for (int c = 0; c < nsys; ++c) it += gs[c].k;
        counter[0] += nsys;
        counter[1] += it;
    }
}

// ------------------------------------------------------------ host side
// Blocks per system of the batched kernels: about four nodes per thread, so
// the per-block partial sums (up to 11 values) are amortised over several
// nodes; at most 1024.  Every per-block buffer (part2, the GMRES partials,
// the adjoint's gradient slots) is sized and indexed with this count.
int nblocks(long long S)
{
    long long b = (S + 4 * TPB - 1) / (4 * TPB);
    return (int)(b < 1024 ? b : 1024);
}

template <typename T, typename TD>
hipError_t launch_step(int p, dim3 grid, hipStream_t st, const T *src, long long ss, T *dst, long long ds,
                       const TD *disp, long long plane, int nx, long long n_first, int stride, const T *G, T *Vout)
{
#define STEP2D(PP) hipLaunchKernelGGL((step2d_kernel<T, TD, PP>), grid, dim3(TPB), 0, st, src, ss, dst, ds, disp, \
                                      plane, nx, n_first, stride, G, Vout)
    switch (p) {
    case 1: STEP2D(1); break;
    case 2: STEP2D(2); break;
    case 3: STEP2D(3); break;
    case 4: STEP2D(4); break;
    default: STEP2D(5); break;
    }
#undef STEP2D
    return hipGetLastError();
}

// Coarse-level step with per-tile stencil windows (step2d_win_kernel).
template <typename T, typename TD>
hipError_t launch_step_win(int p, int nch, hipStream_t st, const T *src, long long ss, T *dst, long long ds,
                           const TD *disp, long long plane, int nx, long long n_first, int stride, const T *G,
                           T *Vout)
{
    const dim3 grid(((nx + WX - 1) / WX) * ((nx + WY - 1) / WY), nch);
#define STEPW(PP) hipLaunchKernelGGL((step2d_win_kernel<T, TD, PP>), grid, dim3(TPB), WIN_LDS_BYTES, st, src, ss, dst, \
                                     ds, disp, plane, nx, n_first, stride, G, Vout)
    switch (p) {
    case 1: STEPW(1); break;
    case 2: STEPW(2); break;
    case 3: STEPW(3); break;
    case 4: STEPW(4); break;
    default: STEPW(5); break;
    }
#undef STEPW
    return hipGetLastError();
}

// Level-0 step, LDS-tiled when the window of a tile fits (F from the bound
// on the displacement); the plain gather kernel otherwise.
// Halo F (cells) of the LDS-tiled level-0 step with tile shape `tile` for a
// launch over nch chains, or 0 when the plain gather kernel runs instead:
// every window coordinate must wrap onto the mesh with one add or subtract,
// the window fit in 48 KB, and the launch have enough tiles to fill the GPU.
int step0_tile_halo(const slm_plan &P, int tile, int nch, size_t *lds_bytes, int *wx_out)
{
    const int nx = P.d.nx, p = P.d.p;
    const TileShape ts = kTiles[tile >= 0 && tile < kNumTiles ? tile : 0];
    double a = 0.0, b = 0.0;
    for (const auto &t : P.alpha) a += std::fabs(t.coef);
    for (const auto &t : P.beta) b += std::fabs(t.coef);
    const double dbound = P.d.dt / (2.0 / nx) * (a > b ? a : b);
    const int F = (int)std::ceil(dbound) + 1;
    const int wx = ts.tx + 2 * F + p / 2 + 1 + p / 2, wy = ts.ty + 2 * F + p / 2 + 1 + p / 2;
    const size_t lds = (size_t)wx * wy * P.elem;
    const int ntx = (nx + ts.tx - 1) / ts.tx, nty = (nx + ts.ty - 1) / ts.ty;
    const long long ntiles = (long long)ntx * nty;
    if (lds_bytes) *lds_bytes = lds;
    if (wx_out) *wx_out = wx;
    // every window coordinate lies in (-nx, 2 nx), so the kernel wraps it
    // with one conditional add or subtract
    const int lo = p / 2 + 1, hi = p / 2;
    const bool one_wrap = F + lo < nx && ntx * ts.tx + F + hi < 2 * nx && nty * ts.ty + F + hi < 2 * nx;
    if (F > 16 || !one_wrap || lds > 48 * 1024 || ntiles * nch < 256) return 0;
    return F;
}

template <typename T, typename TD>
hipError_t launch_step0(const slm_plan &P, int nch, hipStream_t st, const T *src, long long ss, T *dst, long long ds,
                        const TD *disp, long long plane, long long n_first, int stride, const T *G, T *Vout)
{
    const int nx = P.d.nx, p = P.d.p;
    size_t lds = 0;
    int wx = 1;
    const int tile = P.tile2d >= 0 && P.tile2d < kNumTiles ? P.tile2d : 0;
    const int F = step0_tile_halo(P, tile, nch, &lds, &wx);
    if (F == 0) {
        const dim3 grid(nblocks((long long)nx * nx), nch);
        return launch_step<T, TD>(p, grid, st, src, ss, dst, ds, disp, plane, nx, n_first, stride, G, Vout);
    }
    const TileShape ts = kTiles[tile];
    const dim3 grid(((nx + ts.tx - 1) / ts.tx) * ((nx + ts.ty - 1) / ts.ty), nch);
    const unsigned inv_wx = (unsigned)(((1u << 24) + wx - 1) / wx);     // ceil(2^24 / wx)
    // small launches prefetch each thread's displacements (see the kernel)
    const bool pre = (long long)grid.x * grid.y < 1024;
#define STEPT(PP, TXX, TYY)                                                                                         \
    if (pre)                                                                                                        \
        hipLaunchKernelGGL((step2d_tile_kernel<T, TD, PP, TXX, TYY, true>), grid, dim3(TPB), lds, st, src, ss, dst,  \
                           ds, disp, plane, nx, n_first, stride, G, Vout, F, inv_wx);                                \
    else                                                                                                            \
        hipLaunchKernelGGL((step2d_tile_kernel<T, TD, PP, TXX, TYY, false>), grid, dim3(TPB), lds, st, src, ss, dst, \
                           ds, disp, plane, nx, n_first, stride, G, Vout, F, inv_wx)
#define STEPP(TXX, TYY)                                       \
    switch (p) {                                              \
    case 1: STEPT(1, TXX, TYY); break;                        \
    case 2: STEPT(2, TXX, TYY); break;                        \
    case 3: STEPT(3, TXX, TYY); break;                        \
    case 4: STEPT(4, TXX, TYY); break;                        \
    default: STEPT(5, TXX, TYY); break;                       \
    }
    switch (tile) {
    case 1: STEPP(64, 32); break;
    case 2: STEPP(128, 16); break;
    case 3: STEPP(128, 32); break;
    default: STEPP(64, 16); break;
    }
#undef STEPP
#undef STEPT
    return hipGetLastError();
}

// The LDS-tiled matvec applies when the 2D mesh splits exactly into the
// grid's WX x WY tiles, one per block.
bool matvec_tiled(int dim, int nx, int nb)
{
    return dim == 2 && nx % WX == 0 && nx % WY == 0 && (nx / WX) * (nx / WY) == nb;
}

template <typename T, typename TS>
hipError_t launch_matvec(int p, dim3 grid, hipStream_t st, T *V, const T *Wsrc, T *Wdst, long long S, int nx,
                         const TS *sig, long long plane, long long n_first, int stride, int j, const Gs2 *gs,
                         double *part, int dim, int transpose, int rev, int Nl)
{
    if (matvec_tiled(dim, nx, (int)grid.x)) {
#define MVT(PP, TR) hipLaunchKernelGGL((g2_matvec_tile<T, TS, PP, TR>), grid, dim3(TPB), 0, st, V, Wsrc, Wdst, S, nx, \
                                       sig, plane, n_first, stride, j, gs, part, rev, Nl)
        if (transpose) {
            switch (p) {
            case 1: MVT(1, true); break;
            case 3: MVT(3, true); break;
            case 5: MVT(5, true); break;
            default: return hipErrorInvalidValue;
            }
        } else {
            switch (p) {
            case 1: MVT(1, false); break;
            case 3: MVT(3, false); break;
            case 5: MVT(5, false); break;
            default: return hipErrorInvalidValue;
            }
        }
#undef MVT
        return hipGetLastError();
    }
#define MV(PP) hipLaunchKernelGGL((g2_matvec<T, TS, PP>), grid, dim3(TPB), 0, st, V, Wsrc, Wdst, S, nx, sig, plane, \
                                  n_first, stride, j, gs, part, dim, transpose, rev, Nl)
    switch (p) {
    case 1: MV(1); break;
    case 3: MV(3); break;
    case 5: MV(5); break;
    default: return hipErrorInvalidValue;
    }
#undef MV
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fwd2d(int p, dim3 grid, hipStream_t st, const T *B, long long S, int nx, const double *sig,
                        long long plane, long long n_first, int stride, int dim, T *dst, long long dst_stride,
                        const T *G, T *Vout)
{
#define FW(PP) hipLaunchKernelGGL((fwd2d_kernel<T, PP>), grid, dim3(TPB), 0, st, B, S, nx, sig, plane, n_first, \
                                  stride, dim, dst, dst_stride, G, Vout)
    switch (p) {
    case 1: FW(1); break;
    case 3: FW(3); break;
    case 5: FW(5); break;
    default: return hipErrorInvalidValue;
    }
#undef FW
    return hipGetLastError();
}

// One batch of chains [c0, c0+nch) of a sweep, all in the same level.
template <typename T>
hipError_t chain_batch(const slm_plan &P, int level, const ChainArgs &a, int c0, int nch, hipStream_t st)
{
    using TD0 = T;   // level-0 displacement type follows the bulk type
    const long long S = a.S;
    const int nx = a.nx;
    const LevelInfo &L = P.lv[level];
    const long long plane = (long long)L.N * S;
    T *Wb = (T *)ws_at(P, P.w2);
    T *bufs[2] = {Wb, Wb + (long long)P.cap2 * S};
    const int nb = nblocks(S);
    dim3 grid(nb, nch);
    // slots: the residual partials (part2) hold cap2 intervals, the GMRES
    // partials capg systems
    if ((a.R && !slots_fit(P, nb, c0, nch, P.cap2)) || (level > 0 && !slots_fit(P, nb, 0, nch, P.capg)))
        return kSlotMismatch;
    const long long n_first0 = a.n_base + (long long)c0 * a.stride_chain;
    const T *Cin = a.Cin ? (const T *)a.Cin + (long long)c0 * a.cin_stride : nullptr;
    T *Vout = (T *)a.Vout;
    T *Cout = (T *)a.Cout;
    hipError_t e;
    // start slices
    hipLaunchKernelGGL(start2d_kernel<T>, grid, dim3(TPB), 0, st, Cin, a.cin_stride, bufs[0], S,
                       a.write_start ? Vout : nullptr, n_first0, a.stride_chain,
                       (Cout && a.cout_shift && c0 == 0) ? Cout : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int cur = 0;
    for (int k = 0; k < a.nsteps; ++k) {
        const bool last = k + 1 == a.nsteps;
        T *vo = (Vout && (!last || a.write_last)) ? Vout : nullptr;
        if (a.adj && level == 0) {
            // adjoint: transposed SL step of the mirrored forward step
            e = launch_stepT(P, 0, nch, (const double *)bufs[cur], S, (double *)bufs[cur ^ 1], S, n_first0 + k,
                             a.stride_chain, 1, (const double *)a.G, (double *)vo, st);
            if (e != hipSuccess) return e;
        } else if (level > 0 && P.d.coarse_op == SLM_COARSE_REDISC) {
            // rediscretized coarse operator: a plain SL step at the level's departure points
            e = launch_step_win<T, double>(P.d.p, nch, st, bufs[cur], S, bufs[cur ^ 1], S,
                                           (const double *)ws_at(P, L.disp), plane, nx, n_first0 + k, a.stride_chain,
                                           (const T *)a.G, vo);
            if (e != hipSuccess) return e;
        } else if (level == 0) {
            // level-0 displacements have the bulk type (FP32 bulk is T = float)
            if ((P.d.precision == SLM_FP32_BULK) != std::is_same<T, float>::value) return hipErrorInvalidValue;
            e = launch_step0<T, T>(P, nch, st, bufs[cur], S, bufs[cur ^ 1], S, (const T *)ws_at(P, L.disp), plane,
                                   n_first0 + k, a.stride_chain, (const T *)a.G, vo);
            if (e != hipSuccess) return e;
        } else {
            // forward: interpolation into the GMRES right-hand side; adjoint:
            // the incoming slice is the right-hand side of the transposed solve
            T *bb = (T *)ws_at(P, P.g2b);
            const T *rhs = bb;
            if (a.adj) {
                rhs = bufs[cur];
            } else {
                e = launch_step_win<T, double>(P.d.p, nch, st, bufs[cur], S, bb, S, (const double *)ws_at(P, L.disp),
                                               plane, nx, n_first0 + k, a.stride_chain, nullptr, nullptr);
                if (e != hipSuccess) return e;
            }
            if (a.fwd) {                         // explicit correction, no linear solve
                e = launch_fwd2d<T>(P.d.p, grid, st, rhs, S, nx, (const double *)ws_at(P, L.sigma), plane,
                                    n_first0 + k, a.stride_chain, P.d.dim, bufs[cur ^ 1], S, (const T *)a.G, vo);
                if (e != hipSuccess) return e;
                cur ^= 1;
                continue;
            }
            T *V = (T *)ws_at(P, P.g2v);
            T *Wb2[2] = {(T *)ws_at(P, P.g2w), (T *)ws_at(P, P.g2w) + (long long)P.capg * S};
            Gs2 *gs = (Gs2 *)ws_at(P, P.g2s);
            double *pa = (double *)ws_at(P, P.g2p), *pb = pa + (long long)P.capg * nb * NPART;
            double *pc = pb + (long long)P.capg * nb * NPART;
            double *r1 = pc + (long long)P.capg * nb * NPART, *r2 = r1 + (long long)P.capg * NPART;
            double *r3 = r2 + (long long)P.capg * NPART;
            hipLaunchKernelGGL(g2_norm0<T>, grid, dim3(TPB), 0, st, rhs, S, pa);
            hipLaunchKernelGGL(g2_sum, dim3(nch), dim3(TPB), 0, st, pa, nb, 1, (const Gs2 *)nullptr, r3);
            hipLaunchKernelGGL(g2_start<T>, grid, dim3(TPB), 0, st, rhs, S, r3, V, gs, a.kmax);
            // Arnoldi step j: the matvec (normalising w_{j-1} on the fly) with
            // the partial projections and ||w||^2; their totals, the norm by
            // Pythagoras and the Givens step; classical Gram-Schmidt
            // w -= V h with the partials of ||w - V h||^2; the explicit norm
            // and Givens step where Pythagoras would cancel.  w alternates
            // between two buffers so the matvec's stencil reads w_{j-1} while
            // it writes w_j.
            for (int j = 0; j < a.kmax; ++j) {
                T *Wsrc = Wb2[(j + 1) & 1], *Wdst = Wb2[j & 1];
                bool done = false;
                if constexpr (std::is_same<T, float>::value) {
                    if (L.sigma32) {                // FP32 bulk: sigma rounded to float
                        e = launch_matvec<T, float>(P.d.p, grid, st, V, Wsrc, Wdst, S, nx,
                                                    (const float *)ws_at(P, L.sigma32), plane, n_first0 + k,
                                                    a.stride_chain, j, gs, pa, P.d.dim, a.adj, a.adj, L.N);
                        done = true;
                    }
                }
                if (!done)
                    e = launch_matvec<T, double>(P.d.p, grid, st, V, Wsrc, Wdst, S, nx,
                                                 (const double *)ws_at(P, L.sigma), plane, n_first0 + k,
                                                 a.stride_chain, j, gs, pa, P.d.dim, a.adj, a.adj, L.N);
                if (e != hipSuccess) return e;
                hipLaunchKernelGGL(g2_sum_givens, dim3(nch), dim3(TPB), 0, st, pa, nb, gs, j, r1, a.rtol, a.kmax);
                hipLaunchKernelGGL(g2_update<T>, grid, dim3(TPB), 0, st, V, Wdst, S, j, gs, r1, pc);
                hipLaunchKernelGGL(g2_norm_givens, dim3(nch), dim3(TPB), 0, st, pc, nb, gs, j, r1, a.rtol, a.kmax);
            }
            if (a.adj) {
                // y = (B^T)^{-1} rhs, then the transposed interpolation S_l^T y
                hipLaunchKernelGGL(g2_combine<T>, grid, dim3(TPB), 0, st, V, S, gs, bb, S, n_first0 + k,
                                   a.stride_chain, (const T *)nullptr, (T *)nullptr);
                if ((e = hipGetLastError()) != hipSuccess) return e;
                e = launch_stepT(P, level, nch, (const double *)bb, S, (double *)bufs[cur ^ 1], S, n_first0 + k,
                                 a.stride_chain, 1, (const double *)a.G, (double *)vo, st);
                if (e != hipSuccess) return e;
            } else {
                hipLaunchKernelGGL(g2_combine<T>, grid, dim3(TPB), 0, st, V, S, gs, bufs[cur ^ 1], S, n_first0 + k,
                                   a.stride_chain, (const T *)a.G, vo);
            }
            if (a.counter) hipLaunchKernelGGL(g2_count, dim3(1), dim3(64), 0, st, gs, nch, a.counter);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        cur ^= 1;
    }
    if (Cout || a.R) {
        double *part = (double *)ws_at(P, P.part2) + (long long)c0 * nb;
        hipLaunchKernelGGL(finish2d_kernel<T>, grid, dim3(TPB), 0, st, bufs[cur], S,
                           Cout ? Cout + (long long)c0 * S : nullptr, a.cout_shift,
                           a.Cref ? (const T *)a.Cref + (long long)c0 * S : nullptr,
                           a.R ? (T *)a.R + (long long)c0 * S : nullptr, part);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

int chain2d_blocks(long long S) { return nblocks(S); }

int chain2d_tiled(const slm_plan &P, int level, int nchains)
{
    if (level != 0 || P.adj_mode) return 0;
    const int cap = P.cap2 > 0 ? P.cap2 : 1;
    const int tile = P.tile2d >= 0 && P.tile2d < kNumTiles ? P.tile2d : 0;
    return step0_tile_halo(P, tile, nchains < cap ? nchains : cap, nullptr, nullptr) > 0 ? 1 + tile : 0;
}

int chain2d_num_tiles() { return kNumTiles; }

hipError_t launch_chain_2d(const slm_plan &P, int level, int nchains, const ChainArgs &a, hipStream_t st)
{
    const int cap = level > 0 ? P.capg : P.cap2;
    for (int c0 = 0; c0 < nchains; c0 += cap) {
        const int nch = nchains - c0 < cap ? nchains - c0 : cap;
        hipError_t e = P.d.precision == SLM_FP32_BULK ? chain_batch<float>(P, level, a, c0, nch, st)
                                                      : chain_batch<double>(P, level, a, c0, nch, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
