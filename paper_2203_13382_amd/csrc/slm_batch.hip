// slm_batch.hip -- many independent 1D problems solved together.
//
// Every problem keeps its own plan (hierarchy, setup arrays, workspace
// slice).  One V-cycle of the whole batch is a fixed program of launches:
//   * level-0 sweeps of every problem as persistent launches (one per
//     interpolation order p) whose workgroups pull (problem, coarse
//     interval) items from a work list, the slice resident in LDS as in the
//     per-level kernels;
//   * coarse sweeps per (p, elements-per-thread) class, also persistent;
//   * a control kernel that applies the stopping test of Sec. 2.2 per
//     problem on the device;
//   * batched slice copies and injections.
// Every kernel skips the problems whose control flag says they stopped, so
// the program can be captured once as a HIP graph and replayed; the host
// reads one counter per cycle.  Per problem the arithmetic and the order of
// operations are those of slm_solve (linear V-cycle, Sec. 2.2).
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "slm_kernels1d.h"

namespace {

using namespace slmk;

struct BItem {
    ChainArgs a;
    int j;        // chain index inside its sweep
    int prob;     // problem index
};

struct BCtl {     // per-problem control state
    int active, status, iterations, stag;
    double rho0, prev, rho_last;
    double tol;
    int tol_mode, max_iter, fp32, nparts;
    const double *partial;
    double *hist;
};

struct BCopy {    // dst[c*ds + s] (+)= src[c*ss + s], c < count, s < S
    void *dst;
    const void *src;
    long long ds, ss;
    int count, S, assign, prob;
};

constexpr int CTL_THREADS = 1024;

// ------------------------------------------------------------------ kernels
// Work-list counter of a persistent sweep: next[0] hands out items, next[1]
// counts the workgroups that have left.  A workgroup leaves after its first
// failed claim, so when the last one arrives no claim is pending and it sets
// both back to zero for the next launch (which sees them at the kernel
// boundary).  No launch is needed to reset them.
__device__ __forceinline__ void leave_items(unsigned int *next)
{
    if (threadIdx.x == 0 && atomicAdd(next + 1, 1u) == gridDim.x - 1) {
        atomicExch(next, 0u);
        atomicExch(next + 1, 0u);
    }
}

// Next work item of the workgroup (uniform).
__device__ __forceinline__ int next_item(unsigned int *next)
{
    __shared__ int item;
    if (threadIdx.x == 0) item = (int)atomicAdd(next, 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(item);
    __syncthreads();
    return it;
}

// Persistent level-0 sweep: every workgroup takes items until the list is
// exhausted, so every wave reaches the exit.  One launch per order p keeps
// the register budget of the per-level kernel.
template <typename T, typename TD, int P, int EPT, bool DBUF, int PF>
__global__ void __launch_bounds__(SLM_MAXB) fine_batch(const BItem *items, int n, unsigned int *next,
                                                       const BCtl *ctl)
{
    extern __shared__ __align__(16) unsigned char smem[];
    for (;;) {
        const int it = next_item(next);
        if (it >= n) break;
        if (!ctl[items[it].prob].active) continue;
        const ChainArgs a = items[it].a;
        fine_chain<T, TD, P, EPT, DBUF, PF>(a, items[it].j, smem);
        __syncthreads();
    }
    leave_items(next);
}

template <typename T, int P, int EPT>
__global__ void __launch_bounds__(COARSE_MAXB) coarse_batch(const BItem *items, int n, unsigned int *next,
                                                            const BCtl *ctl)
{
    extern __shared__ __align__(16) unsigned char smem[];
    for (;;) {
        const int it = next_item(next);
        if (it >= n) break;
        if (!ctl[items[it].prob].active) continue;
        const ChainArgs a = items[it].a;
        coarse_chain<T, P, EPT>(a, items[it].j, smem);
        __syncthreads();
    }
    leave_items(next);
}

// Stopping test of one active problem per workgroup; the residual norm is
// summed in the order of the single-problem driver.  `remaining` counts the
// problems still running.
__global__ void __launch_bounds__(CTL_THREADS) batch_control(BCtl *ctl, int hist_cap, int *remaining)
{
    __shared__ double red[SLM_RED_DOUBLES];
    BCtl &c = ctl[blockIdx.x];
    if (!c.active) return;                      // uniform over the workgroup
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < c.nparts; i += blockDim.x) v[0] += c.partial[i];
    block_sum<1>(v, red, 0);
    if (threadIdx.x != 0) return;
    const double rho = sqrt(v[0]);
    const int k = c.iterations;                 // cycles finished before this test
    if (c.hist && k < hist_cap) c.hist[k] = rho;
    if (k == 0) c.rho0 = rho;
    c.iterations = k + 1;
    c.rho_last = rho;
    const double thr = c.tol_mode == SLM_TOL_REL ? c.tol * c.rho0 : c.tol;
    int stop = 1;
    if (rho < thr || rho == 0.0) c.status = SLM_OK;
    else if (!isfinite(rho)) c.status = SLM_DIVERGED;
    else if (c.fp32 && k > 0 && (c.stag = rho > 0.95 * c.prev ? c.stag + 1 : 0) >= 3) c.status = SLM_STAGNATED;
    else if (k >= c.max_iter) c.status = SLM_NOT_CONVERGED;
    else stop = 0;
    c.prev = rho;
    if (stop) {
        c.active = 0;
        atomicSub(remaining, 1);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) batch_copy(const BCopy *ops, const BCtl *ctl, int check)
{
    const BCopy o = ops[blockIdx.y];
    if (check && !ctl[o.prob].active) return;
    const long long tot = (long long)o.count * o.S;
    T *d = static_cast<T *>(o.dst);
    const T *s = static_cast<const T *>(o.src);
    for (long long id = (long long)blockIdx.x * 256 + threadIdx.x; id < tot; id += (long long)gridDim.x * 256) {
        const long long c = id / o.S, x = id - c * o.S;
        const T v = s[c * o.ss + x];
        if (o.assign) d[c * o.ds + x] = v;
        else d[c * o.ds + x] += v;
    }
}

int ept_class(int nx)
{
    return nx <= COARSE_MAXB ? 1 : nx <= 2 * COARSE_MAXB ? 2 : nx <= 4 * COARSE_MAXB ? 4 : nx <= 8 * COARSE_MAXB ? 8 : 16;
}

template <typename T>
size_t coarse_lds(int nx, int ept)
{
    size_t a, b, c;
    switch (ept) {
    case 1: return coarse_lds_parts<T, 1>(nx, &a, &b, &c);
    case 2: return coarse_lds_parts<T, 2>(nx, &a, &b, &c);
    case 4: return coarse_lds_parts<T, 4>(nx, &a, &b, &c);
    case 8: return coarse_lds_parts<T, 8>(nx, &a, &b, &c);
    default: return coarse_lds_parts<T, 16>(nx, &a, &b, &c);
    }
}

}  // namespace

// ------------------------------------------------------------------ host state
struct slm_batch {
    struct Op {
        int kind;             // 0 fine, 1 coarse, 2 control, 3 checked copy, 4 unchecked copy
        int group;            // ops of one sweep split by launch shape run concurrently (0: alone)
        int p, ept;           // coarse class
        size_t off;           // device offset of the op's items / copy descriptors
        int n;                // items / descriptors
        int block;
        size_t lds;
        long long maxelems;   // copies: largest count*S; level-0 sweeps: largest slice
    };
    int n = 0;
    std::vector<slm_plan *> plans;
    std::vector<size_t> poff;           // plan workspaces inside the batch workspace
    size_t ws_bytes = 0;
    char *ws = nullptr;
    bool ready = false;
    int fp32 = 0, relax = SLM_RELAX_FCF, nx_max = 8;
    size_t o_ctl = 0, o_counter = 0, o_remaining = 0, o_hist = 0, o_items = 0, o_sitems = 0;
    size_t items_cap = 0, sitems_cap = 0;
    int hist_cap = 512;
    std::vector<Op> cycle;
    int grid_mult = 2, order_desc = 1, cus = 256;   // launch shape (autotuned)
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<hipStream_t> side;      // streams for the concurrent ops of a group
    std::vector<hipEvent_t> ev;         // fork event + one join event per side stream
    // host staging that must outlive asynchronous copies until the next sync
    std::vector<unsigned char> blob, blob2;
    std::vector<BCtl> hctl, hon;
    std::string err;
};

namespace {

int bfail(slm_batch *B, int code, const std::string &m)
{
    if (B) B->err = m;
    slm_set_error(m);
    return code;
}

#define BCHK(...)                                                                                          \
    do {                                                                                                   \
        hipError_t e_ = (__VA_ARGS__);                                                                     \
        if (e_ != hipSuccess) return bfail(B, SLM_EHIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

// Arguments shared by every sweep of a level (as the single-problem driver).
ChainArgs level_args(const slm_plan &P, int level)
{
    ChainArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nx = P.d.nx;
    a.S = P.S;
    a.p = P.d.p;
    a.m = P.lv[level].m;
    a.stride_chain = P.lv[level].m;
    a.disp = ws_at(P, P.lv[level].disp);
    a.sigma = level > 0 ? (const double *)ws_at(P, P.lv[level].sigma) : nullptr;
    a.cin_stride = P.S;
    a.cout_shift = 1;
    a.kmax = P.d.gmres_kmax;
    a.rtol = P.d.gmres_rtol;
    a.counter = (unsigned long long *)ws_at(P, P.counter);
    double amax = 0.0;
    for (const auto &t : P.alpha) amax += std::fabs(t.coef);
    a.nsmall = level == 0 && P.d.dt / (2.0 / P.d.nx) * amax + P.d.p + 8 < P.d.nx ? 1 : 0;
    return a;
}

// Collects the items and copy descriptors of a program of ops.
struct Builder {
    const slm_batch &B;
    std::vector<BItem> items;
    std::vector<BCopy> copies;
    struct Pending { int kind, p, ept, first, n, block; size_t lds; long long maxe; int group = 0; };
    std::vector<Pending> pend;
    int next_group = 1;

    explicit Builder(const slm_batch &b) : B(b) {}

    // Level-0 items are grouped by (p, workgroup size, elements per thread)
    // of their slice, the shape the per-level kernel would use.
    static void fine_shape(int nx, long long nitems, int &block, int &ept)
    {
        block = fine_block(nx, nitems);
        const int e = (nx + block - 1) / block;
        ept = e <= 1 ? 1 : e <= 2 ? 2 : e <= 4 ? 4 : 8;
    }
    void fine(const std::vector<BItem> &v)
    {
        std::vector<std::array<int, 3>> keys;
        for (const auto &it : v) {
            int b, e;
            fine_shape(it.a.nx, (long long)v.size(), b, e);
            const std::array<int, 3> k{it.a.p, b, e};
            if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
        }
        std::sort(keys.begin(), keys.end());
        for (const auto &k : keys) {
            std::vector<BItem> g;
            int nxg = 0;
            for (const auto &it : v) {
                int b, e;
                fine_shape(it.a.nx, (long long)v.size(), b, e);
                if (it.a.p == k[0] && b == k[1] && e == k[2]) {
                    g.push_back(it);
                    nxg = std::max(nxg, it.a.nx);
                }
            }
            if (B.order_desc)     // largest items first: the tail of the list is short work
                std::stable_sort(g.begin(), g.end(), [](const BItem &x, const BItem &y) {
                    return (long long)x.a.nx * x.a.nsteps > (long long)y.a.nx * y.a.nsteps;
                });
            pend.push_back(Pending{0, k[0], k[2], (int)items.size(), (int)g.size(), k[1], 0, nxg, next_group});
            items.insert(items.end(), g.begin(), g.end());
        }
        ++next_group;
    }
    void coarse(const std::vector<BItem> &v)
    {
        for (int p : {1, 3, 5})
            for (int e : {1, 2, 4, 8, 16}) {
                std::vector<BItem> g;
                int block = 64;
                size_t lds = 0;
                for (const auto &it : v) {
                    if (it.a.p != p || ept_class(it.a.nx) != e) continue;
                    g.push_back(it);
                    block = std::max(block, ((it.a.nx + e - 1) / e + 63) / 64 * 64);
                    lds = std::max(lds, B.fp32 ? coarse_lds<float>(it.a.nx, e) : coarse_lds<double>(it.a.nx, e));
                }
                if (g.empty()) continue;
                pend.push_back(Pending{1, p, e, (int)items.size(), (int)g.size(), block, lds, 0, next_group});
                items.insert(items.end(), g.begin(), g.end());
            }
        ++next_group;
    }
    void control() { pend.push_back(Pending{2, 0, 0, 0, 0, 0, 0, 0}); }
    void copy(const std::vector<BCopy> &v, bool checked)
    {
        if (v.empty()) return;
        long long maxe = 0;
        for (const auto &c : v) maxe = std::max(maxe, (long long)c.count * c.S);
        pend.push_back(Pending{checked ? 3 : 4, 0, 0, (int)copies.size(), (int)v.size(), 256, 0, maxe});
        copies.insert(copies.end(), v.begin(), v.end());
    }
    // Items at device offset `base`, copies after them; returns the bytes.
    size_t finish(size_t base, std::vector<unsigned char> &blob, std::vector<slm_batch::Op> &ops) const
    {
        const size_t ib = items.size() * sizeof(BItem);
        blob.resize(ib + copies.size() * sizeof(BCopy));
        if (ib) std::memcpy(blob.data(), items.data(), ib);
        if (!copies.empty()) std::memcpy(blob.data() + ib, copies.data(), copies.size() * sizeof(BCopy));
        ops.clear();
        for (const auto &pd : pend) {
            slm_batch::Op o{};
            o.kind = pd.kind;
            o.group = pd.group;
            o.p = pd.p;
            o.ept = pd.ept;
            o.n = pd.n;
            o.block = pd.block;
            o.lds = pd.lds;
            o.maxelems = pd.maxe;
            if (pd.kind <= 1) o.off = base + (size_t)pd.first * sizeof(BItem);
            else if (pd.kind >= 3) o.off = base + ib + (size_t)pd.first * sizeof(BCopy);
            ops.push_back(o);
        }
        return blob.size();
    }
};

int lds_cap()
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
hipError_t plaunch(K k, int grid, int block, size_t lds, hipStream_t st, const BItem *items, int n, unsigned *next,
                   const BCtl *ctl)
{
    if (lds > (size_t)lds_cap()) return hipErrorInvalidConfiguration;
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, st, items, n, next, ctl);
    return hipGetLastError();
}

// Level-0 launch of one (p, workgroup size, elements per thread) group;
// LDS is sized for the group's largest slice.  Workgroups per CU come from
// slm_batch_tune.
template <typename T>
hipError_t fine_launch(const slm_batch &B, const slm_batch::Op &o, hipStream_t st, unsigned *next)
{
    const BItem *items = (const BItem *)(B.ws + o.off);
    const BCtl *ctl = (const BCtl *)(B.ws + B.o_ctl);
    const long long nxg = o.maxelems;
    const bool dbuf = 2ull * fine_slice_len((int)nxg) * sizeof(T) + SLM_RED_DOUBLES * sizeof(double) + 16 <= (size_t)lds_cap();
    const size_t lds = (((size_t)(dbuf ? 2 : 1) * fine_slice_len((int)nxg) * sizeof(T) + 15) & ~size_t(15)) +
                       SLM_RED_DOUBLES * sizeof(double);
    const int grid = std::max(1, std::min(o.n, B.grid_mult * B.cus * (SLM_MAXB / o.block)));
    const int block = o.block;
#define FB(PP, E, D) plaunch(fine_batch<T, T, PP, E, D, pf_depth<T, E>()>, grid, block, lds, st, items, o.n, next, ctl)
#define FBE(PP, D) switch (o.ept) { case 1: return FB(PP, 1, D); case 2: return FB(PP, 2, D); case 4: return FB(PP, 4, D); default: return FB(PP, 8, D); }
#define FBP(D) switch (o.p) { case 1: FBE(1, D); case 3: FBE(3, D); default: FBE(5, D); }
    if (dbuf) FBP(true);
    FBP(false);
#undef FBP
#undef FBE
#undef FB
}

template <typename T>
hipError_t coarse_launch(const slm_batch &B, const slm_batch::Op &o, hipStream_t st, unsigned *next)
{
    const BItem *items = (const BItem *)(B.ws + o.off);
    const BCtl *ctl = (const BCtl *)(B.ws + B.o_ctl);
    const int grid = std::max(1, std::min(o.n, B.cus));
#define CB(PP, E) return plaunch(coarse_batch<T, PP, E>, grid, o.block, o.lds, st, items, o.n, next, ctl)
#define CBP(PP) switch (o.ept) { case 1: CB(PP, 1); case 2: CB(PP, 2); case 4: CB(PP, 4); case 8: CB(PP, 8); default: CB(PP, 16); }
    switch (o.p) {
    case 1: CBP(1);
    case 3: CBP(3);
    default: CBP(5);
    }
#undef CBP
#undef CB
}

// One op on `st`; persistent sweeps pull items through counter slot `slot`.
int run_op(slm_batch *B, const slm_batch::Op &o, hipStream_t st, int slot)
{
    unsigned *cnt = (unsigned *)(B->ws + B->o_counter) + 2 * slot;     // (next item, workgroups out)
    int *rem = (int *)(B->ws + B->o_remaining);
    BCtl *ctl = (BCtl *)(B->ws + B->o_ctl);
    if (o.kind == 0 || o.kind == 1) {
        if (o.kind == 0) BCHK(B->fp32 ? fine_launch<float>(*B, o, st, cnt) : fine_launch<double>(*B, o, st, cnt));
        else BCHK(B->fp32 ? coarse_launch<float>(*B, o, st, cnt) : coarse_launch<double>(*B, o, st, cnt));
    } else if (o.kind == 2) {
        hipLaunchKernelGGL(batch_control, dim3(B->n), dim3(CTL_THREADS), 0, st, ctl, B->hist_cap, rem);
        BCHK(hipGetLastError());
    } else {
        const long long g = std::max(1LL, std::min(4096LL, (o.maxelems + 255) / 256));
        const BCopy *c = (const BCopy *)(B->ws + o.off);
        const int chk = o.kind == 3 ? 1 : 0;
        if (B->fp32) hipLaunchKernelGGL(batch_copy<float>, dim3((unsigned)g, o.n), dim3(256), 0, st, c, ctl, chk);
        else hipLaunchKernelGGL(batch_copy<double>, dim3((unsigned)g, o.n), dim3(256), 0, st, c, ctl, chk);
        BCHK(hipGetLastError());
    }
    return SLM_OK;
}

// Side streams and events for the largest group of `ops` (created outside
// any stream capture).
int ensure_side(slm_batch *B, const std::vector<slm_batch::Op> &ops)
{
    int most = 1;
    for (size_t i = 0; i < ops.size();) {
        size_t j = i + 1;
        if (ops[i].group)
            while (j < ops.size() && ops[j].group == ops[i].group) ++j;
        most = std::max(most, (int)(j - i));
        i = j;
    }
    while ((int)B->side.size() < most - 1) {
        hipStream_t s2 = nullptr;
        BCHK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        B->side.push_back(s2);
    }
    while ((int)B->ev.size() < most) {
        hipEvent_t e = nullptr;
        BCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        B->ev.push_back(e);
    }
    return SLM_OK;
}

// Enqueue a program of ops on `st` (also used under stream capture).  The
// ops of one group (a sweep split by launch shape) are independent: they
// fork onto side streams and join back, so a long chain of one shape does
// not wait behind another shape's tail.
int run_ops(slm_batch *B, const std::vector<slm_batch::Op> &ops, hipStream_t st)
{
    for (size_t i = 0; i < ops.size();) {
        size_t j = i + 1;
        if (ops[i].group)
            while (j < ops.size() && ops[j].group == ops[i].group) ++j;
        const int cnt = (int)(j - i);
        if (cnt == 1) {
            const int rc = run_op(B, ops[i], st, 0);
            if (rc) return rc;
            i = j;
            continue;
        }
        if (cnt > 63) return bfail(B, SLM_EUNSUPPORTED, "too many launch shapes in one batch sweep");
        if ((int)B->side.size() < cnt - 1 || (int)B->ev.size() < cnt)
            return bfail(B, SLM_EINVAL, "side streams not prepared for this program");
        BCHK(hipEventRecord(B->ev[0], st));
        for (int k = 1; k < cnt; ++k) {
            BCHK(hipStreamWaitEvent(B->side[k - 1], B->ev[0], 0));
            const int rc = run_op(B, ops[i + k], B->side[k - 1], k);
            if (rc) return rc;
        }
        const int rc = run_op(B, ops[i], st, 0);
        if (rc) return rc;
        for (int k = 1; k < cnt; ++k) {
            BCHK(hipEventRecord(B->ev[k], B->side[k - 1]));
            BCHK(hipStreamWaitEvent(st, B->ev[k], 0));
        }
        i = j;
    }
    return SLM_OK;
}

// One V-cycle of every problem, levels in lockstep: level-0 F- and
// C-relaxation, residual and stopping test; per coarse level the
// relaxation and residual sweeps (or the sequential coarsest solve); then
// upward the injected corrections and F-relaxations; finally the level-0
// correction (for FCF the corrected C-values are copied back as the next
// cycle's start).
void build_cycle(const slm_batch &B, Builder &bd)
{
    const bool fcf = B.relax == SLM_RELAX_FCF;
    int Lmax = 1;
    for (auto *P : B.plans) Lmax = std::max(Lmax, P->L);
    std::vector<BItem> fc, res;
    for (int p = 0; p < B.n; ++p) {
        const slm_plan &P = *B.plans[p];
        if (P.L < 2) continue;
        const int nc = P.d.nt / P.lv[0].m;
        char *Ca = ws_at(P, P.lv[0].C), *Cb = ws_at(P, P.C0b);
        for (int j = 0; j < nc; ++j) {
            if (fcf) {
                BItem it{level_args(P, 0), j, p};
                it.a.nsteps = P.lv[0].m;
                it.a.Cin = Ca;
                it.a.Cout = Cb;
                fc.push_back(it);
            }
            BItem r{level_args(P, 0), j, p};
            r.a.nsteps = P.lv[0].m;
            r.a.Cin = fcf ? Cb : Ca;
            r.a.Cref = fcf ? Cb : Ca;
            r.a.R = ws_at(P, P.lv[1].G);
            r.a.partial = (double *)ws_at(P, P.partial);
            res.push_back(r);
        }
    }
    bd.fine(fc);
    bd.fine(res);
    bd.control();
    for (int l = 1; l < Lmax; ++l) {
        std::vector<BItem> vfc, vres, vseq;
        for (int p = 0; p < B.n; ++p) {
            const slm_plan &P = *B.plans[p];
            if (l >= P.L) continue;
            const LevelInfo &L = P.lv[l];
            if (l == P.L - 1) {
                BItem it{level_args(P, l), 0, p};
                it.a.m = it.a.stride_chain = L.N;
                it.a.nsteps = L.N;
                it.a.G = ws_at(P, L.G);
                it.a.Vout = ws_at(P, L.V);
                it.a.write_start = 1;
                it.a.write_last = 1;
                vseq.push_back(it);
                continue;
            }
            for (int j = 0; j < L.N / L.m; ++j) {
                if (fcf) {
                    BItem it{level_args(P, l), j, p};
                    it.a.nsteps = L.m;
                    it.a.G = ws_at(P, L.G);
                    it.a.Cout = ws_at(P, L.C);
                    vfc.push_back(it);
                }
                BItem r{level_args(P, l), j, p};
                r.a.nsteps = L.m;
                r.a.G = ws_at(P, L.G);
                r.a.Cin = fcf ? ws_at(P, L.C) : nullptr;
                r.a.Cref = fcf ? ws_at(P, L.C) : nullptr;
                r.a.R = ws_at(P, P.lv[l + 1].G);
                r.a.partial = (double *)ws_at(P, P.partial);
                vres.push_back(r);
            }
        }
        bd.coarse(vfc);
        bd.coarse(vres);
        bd.coarse(vseq);
    }
    for (int l = Lmax - 2; l >= 1; --l) {
        std::vector<BCopy> corr, last;
        std::vector<BItem> post;
        for (int p = 0; p < B.n; ++p) {
            const slm_plan &P = *B.plans[p];
            if (l >= P.L - 1) continue;
            const LevelInfo &L = P.lv[l];
            const int nc = L.N / L.m;
            const size_t sl = (size_t)P.S * P.elem;
            corr.push_back(BCopy{ws_at(P, L.C), ws_at(P, P.lv[l + 1].V), P.S, P.S, nc + 1, P.S, fcf ? 0 : 1, p});
            for (int j = 0; j < nc; ++j) {
                BItem it{level_args(P, l), j, p};
                it.a.nsteps = L.m - 1;
                it.a.G = ws_at(P, L.G);
                it.a.Cin = ws_at(P, L.C);
                it.a.Vout = ws_at(P, L.V);
                it.a.write_start = 1;
                it.a.write_last = 1;
                post.push_back(it);
            }
            last.push_back(BCopy{ws_at(P, L.V) + (size_t)L.N * sl, ws_at(P, L.C) + (size_t)nc * sl, P.S, P.S, 1, P.S, 1, p});
        }
        bd.copy(corr, true);
        bd.coarse(post);
        bd.copy(last, true);
    }
    std::vector<BCopy> c0, back;
    for (int p = 0; p < B.n; ++p) {
        const slm_plan &P = *B.plans[p];
        if (P.L < 2) continue;
        const int nc = P.d.nt / P.lv[0].m;
        const size_t sl = (size_t)P.S * P.elem;
        char *Cc = fcf ? ws_at(P, P.C0b) : ws_at(P, P.lv[0].C);
        c0.push_back(BCopy{Cc + sl, ws_at(P, P.lv[1].V) + sl, P.S, P.S, nc, P.S, 0, p});
        if (fcf) back.push_back(BCopy{ws_at(P, P.lv[0].C), ws_at(P, P.C0b), P.S, P.S, nc + 1, P.S, 1, p});
    }
    bd.copy(c0, true);
    bd.copy(back, true);
}

int upload_cycle(slm_batch *B, hipStream_t st)
{
    Builder bd(*B);
    build_cycle(*B, bd);
    const size_t bytes = bd.finish(B->o_items, B->blob, B->cycle);
    if (bytes > B->items_cap) return bfail(B, SLM_EWORKSPACE, "batch work-list region too small");
    if (const int rc = ensure_side(B, B->cycle)) return rc;
    if (bytes) BCHK(hipMemcpyAsync(B->ws + B->o_items, B->blob.data(), bytes, hipMemcpyHostToDevice, st));
    BCHK(hipStreamSynchronize(st));
    if (B->gexec) {
        (void)hipGraphExecDestroy(B->gexec);
        B->gexec = nullptr;
    }
    return SLM_OK;
}

// Point updates of slm_solve for a given number of cycles (statistics).
long long updates_of(const slm_plan &P, int iterations)
{
    const bool fcf = P.d.relax == SLM_RELAX_FCF;
    if (P.L == 1) return (long long)P.d.nt * P.S;
    std::vector<long long> coarse(P.L, 0);
    for (int l = P.L - 1; l >= 1; --l) {
        const long long N = P.lv[l].N;
        coarse[l] = l == P.L - 1 ? N : (fcf ? N : 0) + N + coarse[l + 1] + (N - N / P.lv[l].m);
    }
    const long long N0 = P.d.nt;
    long long tot = 0;
    for (int k = 0; k < iterations; ++k) tot += (fcf ? N0 : 0) + N0 + (k + 1 < iterations ? coarse[1] : 0);
    return (tot + N0 - N0 / P.lv[0].m) * P.S;
}

// Run a one-off program (solve start / single-level problems / output)
// from the solve-time item region.
int run_once(slm_batch *B, const Builder &bd, hipStream_t st)
{
    std::vector<slm_batch::Op> ops;
    const size_t bytes = bd.finish(B->o_sitems, B->blob2, ops);
    if (bytes > B->sitems_cap) return bfail(B, SLM_EWORKSPACE, "batch solve work-list region too small");
    if (const int rc = ensure_side(B, ops)) return rc;
    if (bytes) BCHK(hipMemcpyAsync(B->ws + B->o_sitems, B->blob2.data(), bytes, hipMemcpyHostToDevice, st));
    int rc = run_ops(B, ops, st);
    if (rc) return rc;
    BCHK(hipStreamSynchronize(st));     // the staging blob is reused by the next program
    return SLM_OK;
}

}  // namespace

// ------------------------------------------------------------------ ABI
extern "C" {

int slm_batch_create(const slm_desc *descs, int n, slm_batch **out)
{
    if (!out) return bfail(nullptr, SLM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!descs || n < 1) return bfail(nullptr, SLM_EINVAL, "descs and n >= 1 required");
    slm_batch *B = new (std::nothrow) slm_batch();
    if (!B) return bfail(nullptr, SLM_EINVAL, "out of host memory");
    auto drop = [&](int rc, const std::string &m) {
        for (auto *P : B->plans) slm_plan_destroy(P);
        delete B;
        return m.empty() ? rc : bfail(nullptr, rc, m);
    };
    B->n = n;
    B->fp32 = descs[0].precision == SLM_FP32_BULK;
    B->relax = descs[0].relax;
    size_t off = 0;
    long long nitems = 0, nseq = 0;
    for (int i = 0; i < n; ++i) {
        const slm_desc &d = descs[i];
        if (d.dim != 1 || d.precision != descs[0].precision || d.relax != descs[0].relax)
            return drop(SLM_EUNSUPPORTED, "a batch holds 1D problems of one precision and one relax type");
        if (d.p % 2 == 0) return drop(SLM_EUNSUPPORTED, "a batch needs odd p");
        if (d.coarse_op != SLM_COARSE_MODIFIED || d.adjoint)
            return drop(SLM_EUNSUPPORTED, "a batch uses the modified coarse operator and no adjoint");
        slm_plan *P = nullptr;
        const int rc = slm_plan_create(&d, &P);
        if (rc) return drop(rc, "");
        B->plans.push_back(P);
        B->poff.push_back(off);
        off = al256(off + P->ws_bytes);
        B->nx_max = std::max(B->nx_max, d.nx);
        for (int l = 0; l < P->L; ++l) nitems += P->lv[l].m ? 3LL * (P->lv[l].N / P->lv[l].m) : 1;
        nseq += P->L > 1 ? P->d.nt / P->lv[0].m : 1;
    }
    B->o_ctl = off;
    off = al256(off + n * sizeof(BCtl));
    B->o_counter = off;
    off = al256(off + 2 * 64 * sizeof(unsigned));
    B->o_remaining = off;
    off = al256(off + sizeof(int));
    B->o_hist = off;
    off = al256(off + (size_t)n * B->hist_cap * sizeof(double));
    B->items_cap = (size_t)nitems * sizeof(BItem) + (size_t)n * (2 * SLM_MAX_LEVELS + 2) * sizeof(BCopy);
    B->o_items = off;
    off = al256(off + B->items_cap);
    B->sitems_cap = (size_t)nseq * sizeof(BItem) + (size_t)n * 3 * sizeof(BCopy);
    B->o_sitems = off;
    off = al256(off + B->sitems_cap);
    B->ws_bytes = off;
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        cu > 0)
        B->cus = cu;
    *out = B;
    return SLM_OK;
}

void slm_batch_destroy(slm_batch *B)
{
    if (!B) return;
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    for (auto s2 : B->side) (void)hipStreamDestroy(s2);
    for (auto e : B->ev) (void)hipEventDestroy(e);
    for (auto *P : B->plans) slm_plan_destroy(P);
    delete B;
}

int slm_batch_workspace_size(const slm_batch *B, size_t *bytes)
{
    if (!B || !bytes) return bfail(nullptr, SLM_EINVAL, "NULL argument");
    *bytes = B->ws_bytes;
    return SLM_OK;
}

int slm_batch_setup(slm_batch *B, void *d_ws, size_t bytes, void *stream)
{
    if (!B) return bfail(nullptr, SLM_EINVAL, "batch is NULL");
    if (!d_ws || bytes < B->ws_bytes || ((uintptr_t)d_ws & 255))
        return bfail(B, SLM_EWORKSPACE, "workspace smaller than slm_batch_workspace_size() or not 256-byte aligned");
    B->ready = false;
    B->ws = (char *)d_ws;
    for (int i = 0; i < B->n; ++i) {
        const int rc = slm_plan_setup(B->plans[i], B->ws + B->poff[i], B->plans[i]->ws_bytes, stream);
        if (rc) return bfail(B, rc, "setup of problem " + std::to_string(i) + ": " + B->plans[i]->err);
    }
    const int rc = upload_cycle(B, (hipStream_t)stream);
    if (rc) return rc;
    B->ready = true;
    return SLM_OK;
}

int slm_batch_tune(slm_batch *B, const char *cache_path, void *stream)
{
    if (!B) return bfail(nullptr, SLM_EINVAL, "batch is NULL");
    if (!B->ready) return bfail(B, SLM_ENOTSETUP, "batch not set up");
    hipStream_t st = (hipStream_t)stream;
    std::ostringstream key;
    key << "n" << B->n << (B->fp32 ? "f" : "d") << (B->relax == SLM_RELAX_FCF ? "fcf" : "f") << "cu" << B->cus;
    for (auto *P : B->plans) key << "_" << P->d.nx << "x" << P->d.nt << "p" << P->d.p;
    const std::string k = key.str();
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string kk;
        int gm, od;
        double ms;
        while (in >> kk >> gm >> od >> ms)
            if (kk == k && gm >= 1 && gm <= 8 && (od == 0 || od == 1)) {
                B->grid_mult = gm;
                B->order_desc = od;
                return upload_cycle(B, st);
            }
    }
    // Candidates: workgroups per CU x item order, timed on the level-0
    // sweeps of the cycle (up to its stopping test) with every problem
    // active.  They read and write only the batch's own buffers.
    B->hon.assign(B->n, BCtl{});
    for (auto &c : B->hon) c.active = 1;
    BCHK(hipMemcpyAsync(B->ws + B->o_ctl, B->hon.data(), B->n * sizeof(BCtl), hipMemcpyHostToDevice, st));
    hipEvent_t e0, e1;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    double best = 1e30;
    int bg = B->grid_mult, bo = B->order_desc, rc = SLM_OK;
    for (int od : {0, 1}) {
        for (int gm : {1, 2, 4}) {
            B->grid_mult = gm;
            B->order_desc = od;
            if ((rc = upload_cycle(B, st))) break;
            std::vector<slm_batch::Op> first;
            for (const auto &o : B->cycle) {
                if (o.kind != 0) break;
                first.push_back(o);
            }
            if ((rc = run_ops(B, first, st))) break;
            float ms = 0.f;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = bfail(B, SLM_EHIP, "hipEventRecord"); break; }
            for (int r = 0; r < 3 && !rc; ++r) rc = run_ops(B, first, st);
            if (rc) break;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = bfail(B, SLM_EHIP, "event timing failed");
                break;
            }
            if (ms < best) { best = ms; bg = gm; bo = od; }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    B->grid_mult = bg;
    B->order_desc = bo;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << k << " " << bg << " " << bo << " " << best / 3.0 << "\n";
    }
    return upload_cycle(B, st);
}

int slm_batch_solve(slm_batch *B, const void *const *d_u0, void *const *d_u, slm_stats *stats, double *h_hist,
                    int hist_cap, int use_graph, void *stream)
{
    if (!B) return bfail(nullptr, SLM_EINVAL, "batch is NULL");
    if (!B->ready) return bfail(B, SLM_ENOTSETUP, "batch not set up");
    if (!d_u0 || !d_u) return bfail(B, SLM_EINVAL, "NULL pointer arrays");
    for (int p = 0; p < B->n; ++p)
        if (!d_u0[p] || !d_u[p]) return bfail(B, SLM_EINVAL, "NULL pointer for problem " + std::to_string(p));
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    const bool fcf = B->relax == SLM_RELAX_FCF;
    int rc = SLM_OK;

    // control state of every problem; single-level problems never run cycles
    B->hctl.assign(B->n, BCtl{});
    int remaining = 0, maxit = 0;
    for (int p = 0; p < B->n; ++p) {
        const slm_plan &P = *B->plans[p];
        BCtl &c = B->hctl[p];
        c.active = P.L > 1;
        c.tol = P.d.tol;
        c.tol_mode = P.d.tol_mode;
        c.max_iter = P.d.max_iter;
        c.fp32 = B->fp32;
        c.nparts = P.L > 1 ? P.d.nt / P.lv[0].m : 0;
        c.partial = (const double *)ws_at(P, P.partial);
        c.hist = (double *)(B->ws + B->o_hist) + (size_t)p * B->hist_cap;
        remaining += c.active;
        maxit = std::max(maxit, P.d.max_iter);
        BCHK(hipMemsetAsync(ws_at(P, P.counter), 0, 2 * sizeof(unsigned long long), st));
    }
    // work-list counters start at zero; every persistent sweep leaves them so
    BCHK(hipMemsetAsync(B->ws + B->o_counter, 0, 2 * 64 * sizeof(unsigned), st));
    // start: C-point initial iterate (u_0 at C-point 0) and single-level
    // problems' sequential stepping, with every flag on
    B->hon = B->hctl;
    for (auto &c : B->hon) c.active = 1;
    BCHK(hipMemcpyAsync(B->ws + B->o_ctl, B->hon.data(), B->n * sizeof(BCtl), hipMemcpyHostToDevice, st));
    {
        Builder pre(*B);
        std::vector<BCopy> init0, init1;
        std::vector<BItem> seq;
        for (int p = 0; p < B->n; ++p) {
            const slm_plan &P = *B->plans[p];
            if (P.L == 1) {
                BItem it{level_args(P, 0), 0, p};
                it.a.m = it.a.stride_chain = P.d.nt;
                it.a.nsteps = P.d.nt;
                it.a.Cin = d_u0[p];
                it.a.Vout = d_u[p];
                it.a.write_start = 1;
                it.a.write_last = 1;
                seq.push_back(it);
                continue;
            }
            const int m0 = P.lv[0].m, nc = P.d.nt / m0;
            const size_t sl = (size_t)P.S * P.elem;
            char *Ca = ws_at(P, P.lv[0].C);
            init0.push_back(BCopy{Ca + sl, (const char *)d_u[p] + (size_t)m0 * sl, P.S, (long long)m0 * P.S, nc, P.S, 1, p});
            init1.push_back(BCopy{Ca, d_u0[p], P.S, P.S, 1, P.S, 1, p});
        }
        pre.copy(init0, false);
        pre.copy(init1, false);
        pre.fine(seq);
        if ((rc = run_once(B, pre, st))) return rc;
    }
    BCHK(hipMemcpyAsync(B->ws + B->o_ctl, B->hctl.data(), B->n * sizeof(BCtl), hipMemcpyHostToDevice, st));
    BCHK(hipMemcpyAsync(B->ws + B->o_remaining, &remaining, sizeof(int), hipMemcpyHostToDevice, st));
    BCHK(hipStreamSynchronize(st));

    // V-cycles until every problem has stopped (each stops after at most
    // max_iter + 1 stopping tests)
    if (use_graph && !B->gexec && remaining > 0) {
        if (!B->cap_stream) BCHK(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        BCHK(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeRelaxed));
        rc = run_ops(B, B->cycle, B->cap_stream);
        const hipError_t ee = hipStreamEndCapture(B->cap_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        BCHK(ee);
        const hipError_t ei = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        BCHK(ei);
    }
    for (int cyc = 0; remaining > 0 && cyc <= maxit + 1; ++cyc) {
        if (use_graph) BCHK(hipGraphLaunch(B->gexec, st));
        else if ((rc = run_ops(B, B->cycle, st))) return rc;
        BCHK(hipMemcpyAsync(&remaining, B->ws + B->o_remaining, sizeof(int), hipMemcpyDeviceToHost, st));
        BCHK(hipStreamSynchronize(st));
    }
    if (remaining > 0) return bfail(B, SLM_EHIP, "batch control did not stop every problem");

    // output: F-relaxation from each problem's final C-values
    BCHK(hipMemcpyAsync(B->hctl.data(), B->ws + B->o_ctl, B->n * sizeof(BCtl), hipMemcpyDeviceToHost, st));
    BCHK(hipStreamSynchronize(st));
    B->hon = B->hctl;
    for (auto &c : B->hon) c.active = 1;
    BCHK(hipMemcpyAsync(B->ws + B->o_ctl, B->hon.data(), B->n * sizeof(BCtl), hipMemcpyHostToDevice, st));
    {
        Builder post(*B);
        std::vector<BItem> outF;
        std::vector<BCopy> lastc;
        for (int p = 0; p < B->n; ++p) {
            const slm_plan &P = *B->plans[p];
            if (P.L == 1) continue;
            const int m0 = P.lv[0].m, nc = P.d.nt / m0;
            const size_t sl = (size_t)P.S * P.elem;
            char *Cf = fcf ? ws_at(P, P.C0b) : ws_at(P, P.lv[0].C);
            for (int j = 0; j < nc; ++j) {
                BItem it{level_args(P, 0), j, p};
                it.a.nsteps = m0 - 1;
                it.a.Cin = Cf;
                it.a.Vout = d_u[p];
                it.a.write_start = 1;
                it.a.write_last = 1;
                outF.push_back(it);
            }
            lastc.push_back(BCopy{(char *)d_u[p] + (size_t)P.d.nt * sl, Cf + (size_t)nc * sl, P.S, P.S, 1, P.S, 1, p});
        }
        post.fine(outF);
        post.copy(lastc, false);
        if ((rc = run_once(B, post, st))) return rc;
    }

    // statistics
    std::vector<double> hist((size_t)B->n * B->hist_cap);
    BCHK(hipMemcpyAsync(hist.data(), B->ws + B->o_hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    std::vector<unsigned long long> cnt(2 * (size_t)B->n);
    for (int p = 0; p < B->n; ++p)
        BCHK(hipMemcpyAsync(&cnt[2 * p], ws_at(*B->plans[p], B->plans[p]->counter), 2 * sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, st));
    BCHK(hipStreamSynchronize(st));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = SLM_OK;
    for (int p = 0; p < B->n; ++p) {
        const slm_plan &P = *B->plans[p];
        const BCtl &c = B->hctl[p];
        slm_stats s;
        std::memset(&s, 0, sizeof(s));
        s.n_levels = P.L;
        s.iterations = P.L > 1 ? c.iterations : 0;
        s.status = P.L > 1 ? c.status : SLM_OK;
        s.rho0 = c.rho0;
        s.rho_final = c.rho_last;
        s.solve_ms = ms;
        s.point_updates = updates_of(P, s.iterations);
        s.gmres_solves = (long long)cnt[2 * p];
        s.gmres_iters = (long long)cnt[2 * p + 1];
        if (stats) stats[p] = s;
        if (h_hist)
            for (int k = 0; k < hist_cap; ++k)
                h_hist[(size_t)p * hist_cap + k] =
                    k < B->hist_cap && k < s.iterations ? hist[(size_t)p * B->hist_cap + k] : 0.0;
        worst = std::max(worst, s.status);
    }
    return worst;
}

}  // extern "C"
