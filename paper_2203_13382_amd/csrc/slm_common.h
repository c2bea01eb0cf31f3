// slm_common.h -- device building blocks shared by the gfx950 kernels of the
// semi-Lagrangian MGRIT library (arXiv 2203.13382).  Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "slmgrit.h"

#define SLM_PI 3.14159265358979323846
#define SLM_KMAX 10          // GMRES iterations, upper bound (Sec. 3.3)
#define SLM_WAVE 64          // CDNA wavefront width
#define SLM_MAXB 1024        // largest workgroup

// ---------------------------------------------------------------- problem data
// A wave-speed field as a sum of separable cosine terms (the ABI's term list).
struct WaveField {
    int n;
    double coef[SLM_MAX_TERMS], kx[SLM_MAX_TERMS], px[SLM_MAX_TERMS];
    double ky[SLM_MAX_TERMS], py[SLM_MAX_TERMS], kt[SLM_MAX_TERMS], pt[SLM_MAX_TERMS];
};

__device__ __forceinline__ double wave_eval(const WaveField &f, double x, double y, double t)
{
    double s = 0.0;
    for (int k = 0; k < f.n; ++k)
        s += f.coef[k] * cos(f.kx[k] * SLM_PI * x + f.px[k]) * cos(f.ky[k] * SLM_PI * y + f.py[k]) *
             cos(f.kt[k] * SLM_PI * t + f.pt[k]);
    return s;
}

// Explicit Runge-Kutta tableaux for the backward departure trace (Sec. 2.1).
// r=1 forward Euler, r=2 Heun, r=3 Kutta's third-order method, r=4 the
// classical fourth-order method, r=5 Butcher's six-stage fifth-order method.
struct Erk {
    int s;
    double c[6], b[6], a[6][6];
};

__host__ __device__ inline Erk erk_tableau(int r)
{
    Erk e = {};
    switch (r) {
    case 1: e.s = 1; e.b[0] = 1.0; break;
    case 2: e.s = 2; e.c[1] = 1.0; e.a[1][0] = 1.0; e.b[0] = 0.5; e.b[1] = 0.5; break;
    case 3:
        e.s = 3; e.c[1] = 0.5; e.c[2] = 1.0;
        e.a[1][0] = 0.5; e.a[2][0] = -1.0; e.a[2][1] = 2.0;
        e.b[0] = 1.0 / 6.0; e.b[1] = 2.0 / 3.0; e.b[2] = 1.0 / 6.0;
        break;
    case 4:
        e.s = 4; e.c[1] = 0.5; e.c[2] = 0.5; e.c[3] = 1.0;
        e.a[1][0] = 0.5; e.a[2][1] = 0.5; e.a[3][2] = 1.0;
        e.b[0] = 1.0 / 6.0; e.b[1] = 1.0 / 3.0; e.b[2] = 1.0 / 3.0; e.b[3] = 1.0 / 6.0;
        break;
    default:
        e.s = 6; e.c[1] = 0.25; e.c[2] = 0.25; e.c[3] = 0.5; e.c[4] = 0.75; e.c[5] = 1.0;
        e.a[1][0] = 0.25;
        e.a[2][0] = 0.125; e.a[2][1] = 0.125;
        e.a[3][1] = -0.5; e.a[3][2] = 1.0;
        e.a[4][0] = 3.0 / 16.0; e.a[4][3] = 9.0 / 16.0;
        e.a[5][0] = -3.0 / 7.0; e.a[5][1] = 2.0 / 7.0; e.a[5][2] = 12.0 / 7.0;
        e.a[5][3] = -12.0 / 7.0; e.a[5][4] = 8.0 / 7.0;
        e.b[0] = 7.0 / 90.0; e.b[2] = 32.0 / 90.0; e.b[3] = 12.0 / 90.0;
        e.b[4] = 32.0 / 90.0; e.b[5] = 7.0 / 90.0;
        break;
    }
    return e;
}

// ---------------------------------------------------------------- stencils
// Offset of the first of the p+1 interpolation nodes relative to the node
// x_E east of the departure point: -l(p), with the even-p bias of Sec. 2.1
// (the extra node goes west when eps > 1/2).
template <typename F>
__device__ __forceinline__ int stencil_first(int p, F eps)
{
    if (p & 1) return -((p + 1) >> 1);
    return eps > F(0.5) ? -((p >> 1) + 1) : -(p >> 1);
}

// Lagrange weights of the nodes first+j, j = 0..p, evaluated at -eps, in the
// shifted variable z = -eps - first (nodes 0..p):
//   w_j = prod_{k != j} (z - k) / (j - k).
template <int P, typename F>
__device__ __forceinline__ void lagrange_weights(F z, F (&w)[P + 1])
{
    // 1 / prod_{k != j} (j - k) = (-1)^{P-j} / (j! (P-j)!)
    constexpr double fact[6] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0};
    F pre[P + 1], suf[P + 1];
    pre[0] = F(1);
#pragma unroll
    for (int j = 1; j <= P; ++j) pre[j] = pre[j - 1] * (z - F(j - 1));
    suf[P] = F(1);
#pragma unroll
    for (int j = P - 1; j >= 0; --j) suf[j] = suf[j + 1] * (z - F(j + 1));
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        const F inv = F(((P - j) & 1 ? -1.0 : 1.0) / (fact[j] * fact[P - j]));
        w[j] = pre[j] * suf[j] * inv;
    }
}

// Weights of the interpolation stencil at the departure point, from eps
// (w[j] for the node first+j, first = stencil_first(P, eps)): the same
// Lagrange polynomials as lagrange_weights(-eps - first), evaluated in fewer
// operations for odd p.  There the p+1 nodes sit symmetrically about the
// midpoint of the departure cell; with s the departure point's offset from
// that midpoint (s = 1/2 - eps, in cells) and Q = s^2, node pairs +-c give
// the factor (s - c)(s + c) = Q - c^2, so every weight is a product of such
// factors times one linear factor:
//   p = 3 (nodes at s = -3/2, -1/2, 1/2, 3/2):
//     w = { -a (s - 3/2), b (s - 1/2), -b (s + 1/2), a (s + 3/2) },
//     a = (Q - 1/4) / 6, b = (Q - 9/4) / 2;
//   p = 5 (nodes at s = -5/2 .. 5/2):
//     w = { -a (s - 5/2), b (s - 3/2), -c (s - 1/2), c (s + 1/2), -b (s + 3/2), a (s + 5/2) },
//     a = (Q - 9/4)(Q - 1/4) / 120, b = (Q - 25/4)(Q - 1/4) / 24, c = (Q - 25/4)(Q - 9/4) / 12;
//   p = 1: w = { eps, 1 - eps }.
// Even p keeps the general product form.
template <int P, typename F>
__device__ __forceinline__ void interp_weights(F eps, F (&w)[P + 1])
{
    if constexpr (P == 1) {
        w[0] = eps;
        w[1] = F(1) - eps;
    } else if constexpr (P == 3) {
        const F s = F(0.5) - eps, q = s * s;
        const F a = fma(q, F(1.0 / 6.0), F(-1.0 / 24.0));
        const F b = fma(q, F(0.5), F(-1.125));
        const F a3 = F(1.5) * a, b1 = F(0.5) * b;
        w[0] = fma(-a, s, a3);
        w[1] = fma(b, s, -b1);
        w[2] = fma(-b, s, -b1);
        w[3] = fma(a, s, a3);
    } else if constexpr (P == 5) {
        const F s = F(0.5) - eps, q = s * s;
        const F p25 = q - F(6.25);
        const F p15 = fma(q, F(1.0 / 12.0), F(-2.25 / 12.0));     // (Q - 9/4) / 12
        const F p05 = fma(q, F(1.0 / 24.0), F(-0.25 / 24.0));     // (Q - 1/4) / 24
        const F c = p25 * p15, b = p25 * p05, a = F(2.4) * (p15 * p05);
        const F a5 = F(2.5) * a, b3 = F(1.5) * b, c1 = F(0.5) * c;
        w[0] = fma(-a, s, a5);
        w[1] = fma(b, s, -b3);
        w[2] = fma(-c, s, c1);
        w[3] = fma(c, s, c1);
        w[4] = fma(-b, s, -b3);
        w[5] = fma(a, s, a5);
    } else {
        lagrange_weights<P, F>(-eps - F(stencil_first<F>(P, eps)), w);
    }
}

// f_{p+1}(z) of eq. (fpoly_def), odd p: (1/(p+1)!) prod_{q=-l}^{r} (q + z).
__device__ __forceinline__ double fpoly_odd(int p, double z)
{
    const int l = (p + 1) >> 1, r = (p - 1) >> 1;
    double prod = 1.0, fact = 1.0;
    for (int q = -l; q <= r; ++q) prod *= (double)q + z;
    for (int k = 2; k <= p + 1; ++k) fact *= (double)k;
    return prod / fact;
}

// Taps of D_{p+1} = (central second difference)^{(p+1)/2}, odd p
// (eq. Dp+1_def with a second-order rule): [1,-2,1], [1,-4,6,-4,1],
// [1,-6,15,-20,15,-6,1].
template <int P>
struct DTaps;
template <> struct DTaps<1> { static constexpr int q = 1; static constexpr double t[3] = {1, -2, 1}; };
template <> struct DTaps<3> { static constexpr int q = 2; static constexpr double t[5] = {1, -4, 6, -4, 1}; };
template <> struct DTaps<5> { static constexpr int q = 3; static constexpr double t[7] = {1, -6, 15, -20, 15, -6, 1}; };
// Even p has no D_{p+1} correction (MGRIT uses odd p only); placeholders keep
// the stepping-only instantiations well formed.
template <> struct DTaps<2> { static constexpr int q = 1; static constexpr double t[3] = {0, 0, 0}; };
template <> struct DTaps<4> { static constexpr int q = 1; static constexpr double t[3] = {0, 0, 0}; };

// Column i and row j of point id of an nx-wide slice, in 32-bit arithmetic
// (a slice holds fewer than 2^31 points; 64-bit division is a long software
// sequence on the GPU).
__device__ __forceinline__ void split_xy(long long id, int nx, int &i, int &j)
{
    const unsigned u = (unsigned)id, n = (unsigned)nx;
    const unsigned q = u / n;
    j = (int)q;
    i = (int)(u - q * n);
}

__device__ __forceinline__ int wrap_mod(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------- reductions
// DPP lane permutations (quad_perm xor1, quad_perm xor2, row_half_mirror,
// row_mirror) applied to both 32-bit halves of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const unsigned long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffull), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// DPP broadcast of a double: lanes in the rows of ROWMASK receive the value
// of the lane CTRL selects (row_bcast:15 / row_bcast:31), the others 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_bcast_f64(double x)
{
    const unsigned long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffull), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wavefront, all in DPP (no LDS traffic): four
// in-row steps leave every lane with its 16-lane row's sum, then
// row_bcast:15 and row_bcast:31 carry the row sums up.  The total is exact
// in lane 63 only (the other lanes hold partial sums).
__device__ __forceinline__ double wave_sum_last(double x)
{
    x += dpp_f64<0xB1>(x);    // lanes i ^ 1
    x += dpp_f64<0x4E>(x);    // lanes i ^ 2
    x += dpp_f64<0x141>(x);   // the other quad of the 8-lane half row
    x += dpp_f64<0x140>(x);   // the other half of the 16-lane row
    x += dpp_bcast_f64<0x142, 0xA>(x);   // rows 1, 3 += last lane of rows 0, 2
    x += dpp_bcast_f64<0x143, 0xC>(x);   // rows 2, 3 += lane 31
    return x;
}

// Sum NV values over the workgroup; every thread receives the totals.
// `red` is LDS scratch of 2 * (SLM_MAXB/64) * NV doubles; `buf` alternates
// between consecutive calls so one barrier per call suffices.  The order of
// the cross-wave sum is fixed, so results are deterministic and identical in
// every thread.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *red, int buf)
{
    const int lane = threadIdx.x & (SLM_WAVE - 1), wid = threadIdx.x / SLM_WAVE;
    const int nw = blockDim.x / SLM_WAVE;
    double *r = red + buf * (SLM_MAXB / SLM_WAVE) * 16;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum_last(v[i]);
    if (lane == SLM_WAVE - 1) {
#pragma unroll
        for (int i = 0; i < NV; ++i) r[wid * 16 + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += r[w * 16 + i];
        v[i] = s;
    }
}

#define SLM_RED_DOUBLES (2 * (SLM_MAXB / SLM_WAVE) * 16)

// The blocks of one grid row are dealt to the 8 XCDs in turn: with n blocks
// per row (a multiple of 8) block b runs on XCD b % 8.  xcd_block maps the
// physical index to a logical one so that each XCD takes a contiguous run of
// logical blocks, and data shared by neighbouring blocks meets in one L2.
// A bijection on [0, n); the identity when n is not a multiple of 8.
__device__ __forceinline__ long long xcd_block(long long b, long long n)
{
    return (n & 7) ? b : (b & 7) * (n >> 3) + (b >> 3);
}

__device__ __forceinline__ double readlane_f64(double x, int lane)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Exchange of two doubles between lane halves (v_permlane32_swap on both
// 32-bit words): afterwards a = (a lanes 0-31 | b lanes 0-31) and
// b = (a lanes 32-63 | b lanes 32-63).
__device__ __forceinline__ void swap32_f64(double &a, double &b)
{
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// Same between 16-lane rows (v_permlane16_swap): afterwards a holds rows
// (a0, b0, a2, b2) and b rows (a1, b1, a3, b3).
__device__ __forceinline__ void swap16_f64(double &a, double &b)
{
    const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
    a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// Wave sums of NV values as a reduce-scatter: the values are padded to 4Q
// (zeros); a half-wave exchange pairs value j with j + 2Q and a row exchange
// pairs j with j + Q, so that each register then carries four values, one
// per 16-lane row, each summed over four lanes; four in-row DPP steps finish
// the sums.  Value m + kQ ends in every lane of row k of register m; lane
// 16k writes it to r[m + kQ].  About 5 instructions per value instead of 18
// for NV separate all-lane sums.
template <int NV>
__device__ __forceinline__ void wave_sums_to_lds(const double (&v)[NV], double *r)
{
    constexpr int Q = (NV + 3) / 4;
    double a[4 * Q];
#pragma unroll
    for (int i = 0; i < 4 * Q; ++i) a[i] = i < NV ? v[i] : 0.0;
#pragma unroll
    for (int j = 0; j < 2 * Q; ++j) {
        swap32_f64(a[j], a[j + 2 * Q]);
        a[j] += a[j + 2 * Q];                   // lanes 0-31: value j, 32-63: value j+2Q
    }
#pragma unroll
    for (int m = 0; m < Q; ++m) {
        swap16_f64(a[m], a[m + Q]);
        a[m] += a[m + Q];                       // row k: value m + kQ
        a[m] += dpp_f64<0xB1>(a[m]);
        a[m] += dpp_f64<0x4E>(a[m]);
        a[m] += dpp_f64<0x141>(a[m]);
        a[m] += dpp_f64<0x140>(a[m]);
    }
    const int lane = threadIdx.x & (SLM_WAVE - 1);
    if ((lane & 15) == 0) {
        const int k = lane >> 4;
#pragma unroll
        for (int m = 0; m < Q; ++m) r[m + k * Q] = a[m];
    }
}

// block_sum with the reduce-scatter wave stage (fewer instructions for many
// values; used by the batched 2D kernels, whose blocks each reduce up to
// SLM_KMAX+1 partial inner products).  Every thread receives the totals,
// summed over the waves in a fixed order.
template <int NV>
__device__ __forceinline__ void block_sum_rs(double (&v)[NV], double *red, int buf)
{
    const int wid = threadIdx.x / SLM_WAVE;
    const int nw = blockDim.x / SLM_WAVE;
    double *r = red + buf * (SLM_MAXB / SLM_WAVE) * 16;
    wave_sums_to_lds<NV>(v, r + wid * 16);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += r[w * 16 + i];
        v[i] = s;
    }
}

// block_sum variant whose totals come back as wave-uniform values (scalar
// registers): each wave reduce-scatters its partial sums into LDS, then lane
// l < NV adds up value l over the waves in a fixed order and each total is
// read from its lane.  Same determinism as block_sum.
template <int NV>
__device__ __forceinline__ void block_sum_u(double (&v)[NV], double *red, int buf)
{
    static_assert(NV <= 16, "at most 16 values");
    const int lane = threadIdx.x & (SLM_WAVE - 1), wid = threadIdx.x / SLM_WAVE;
    const int nw = blockDim.x / SLM_WAVE;
    double *r = red + buf * (SLM_MAXB / SLM_WAVE) * 16;
    wave_sums_to_lds<NV>(v, r + wid * 16);
    __syncthreads();
    double t = 0.0;
    if (lane < NV)
        for (int w = 0; w < nw; ++w) t += r[w * 16 + lane];
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = readlane_f64(t, i);
}
