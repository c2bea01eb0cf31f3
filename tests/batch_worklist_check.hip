// Host-side bounds check of the batch work list (test infrastructure, no GPU
// needed): builds the cycle program of a created batch against a fake
// workspace base, exactly as setup and the tuner build it, and checks that
// every item's pointers (over the rows and slices the sweep touches) lie in
// its own problem's workspace region and every copy descriptor in the batch
// workspace.  With `shrink` > 0 the first problem's region is taken to end
// `shrink` bytes before the highest byte its items touch, which lets a test
// confirm that the check fails when an extent does not fit.
// It includes the library source for the internal types and the program
// builder, and launches nothing.
#include "slm_batch.hip"
#include <cstdio>

// findings are printed only when asked (verbose)
#define REPORT(...) \
    do {                \
        if (verbose) printf(__VA_ARGS__); \
    } while (0)

extern "C" int check_batch(void *handle, int verbose, long long shrink)
{
    slm_batch *B = (slm_batch *)handle;
    char *base = (char *)0x100000000000ULL;
    B->ws = base;
    for (int i = 0; i < B->n; ++i) B->plans[i]->ws = base + B->poff[i];
    int bad = 0;
    const size_t T = B->fp32 ? 4 : 8;
    for (int od : {0, 1})
        for (int gm : {1, 2, 4}) {
            B->grid_mult = gm;
            B->order_desc = od;
            Builder bd(*B);
            build_cycle(*B, bd);
            size_t top0 = 0;     // highest byte (offset) the first problem's items touch
            auto touch = [&](const slm_plan &P, const void *p, size_t hi) {
                if (p && &P == B->plans[0]) top0 = std::max(top0, (size_t)((const char *)p + hi - P.ws));
            };
            std::vector<slm_batch::Op> ops;
            const size_t bytes = bd.finish(B->o_items, B->blob, ops);
            if (bytes > B->items_cap) { REPORT("items %zu > cap %zu\n", bytes, B->items_cap); ++bad; }
            auto inside = [&](const slm_plan &P, const void *p, size_t lo, size_t hi, const char *what, int it) {
                if (!p) return;
                const char *c = (const char *)p;
                const size_t cap = (&P == B->plans[0] && shrink > 0) ? top0 - (size_t)shrink : P.ws_bytes;
                if (c + lo < P.ws || c + hi > P.ws + cap) {
                    if (bad < 20)
                        REPORT("item %d %s out of plan ws: [%lld, %lld) of %zu\n", it, what,
                               (long long)(c + lo - P.ws), (long long)(c + hi - P.ws), cap);
                    ++bad;
                }
            };
            for (const BItem &it : bd.items) {
                const slm_plan &P = *B->plans[it.prob];
                const ChainArgs &a = it.a;
                const long long S = a.S, nf = (long long)a.n_base + (long long)it.j * a.stride_chain;
                touch(P, a.G, (nf + a.nsteps + 1) * S * T);
                touch(P, a.Vout, (nf + a.nsteps + 1) * S * T);
                touch(P, a.Cin, ((size_t)it.j * a.cin_stride + S) * T);
                touch(P, a.Cout, ((size_t)(it.j + a.cout_shift) + 1) * S * T);
            }
            for (size_t k = 0; k < bd.items.size(); ++k) {
                const BItem &it = bd.items[k];
                const slm_plan &P = *B->plans[it.prob];
                const ChainArgs &a = it.a;
                const int j = it.j;
                const long long S = a.S, nf = (long long)a.n_base + (long long)j * a.stride_chain;
                int lev = -1;
                for (int l = 0; l < P.L; ++l)
                    if ((const char *)a.disp == ws_at(P, P.lv[l].disp)) lev = l;
                if (lev < 0) { REPORT("item %zu: disp matches no level\n", k); ++bad; continue; }
                const size_t TD = (lev == 0 && B->fp32) ? 4 : 8;
                if (nf < 0 || nf + a.nsteps > P.lv[lev].N) { REPORT("item %zu: steps [%lld,%lld) of N=%d\n", k, nf, nf + a.nsteps, P.lv[lev].N); ++bad; }
                inside(P, a.disp, nf * S * TD, (nf + a.nsteps) * S * TD, "disp", (int)k);
                inside(P, a.sigma, nf * S * 8, (nf + a.nsteps) * S * 8, "sigma", (int)k);
                inside(P, a.G, (nf + 1) * S * T, (nf + a.nsteps + 1) * S * T, "G", (int)k);
                inside(P, a.Cin, (size_t)j * a.cin_stride * T, ((size_t)j * a.cin_stride + S) * T, "Cin", (int)k);
                inside(P, a.Vout, nf * S * T, (nf + a.nsteps + 1) * S * T, "Vout", (int)k);
                inside(P, a.Cout, 0, ((size_t)(j + a.cout_shift) + 1) * S * T, "Cout", (int)k);
                inside(P, a.Cref, (size_t)(j + 1) * S * T, (size_t)(j + 2) * S * T, "Cref", (int)k);
                inside(P, a.R, (size_t)(j + 1) * S * T, (size_t)(j + 2) * S * T, "R", (int)k);
                inside(P, a.partial, (size_t)j * 8, (size_t)(j + 1) * 8, "partial", (int)k);
                inside(P, a.counter, 0, 16, "counter", (int)k);
                if (a.nx != P.d.nx || a.S != P.S || a.p != P.d.p) { REPORT("item %zu: shape mismatch\n", k); ++bad; }
            }
            for (size_t k = 0; k < bd.copies.size(); ++k) {
                const BCopy &c = bd.copies[k];
                const char *wsb = B->ws, *wse = B->ws + B->ws_bytes;
                const size_t ext_d = ((size_t)(c.count - 1) * c.ds + c.S) * T, ext_s = ((size_t)(c.count - 1) * c.ss + c.S) * T;
                if (c.dst && ((const char *)c.dst < wsb || (const char *)c.dst + ext_d > wse)) { REPORT("copy %zu dst out\n", k); ++bad; }
                if (c.src && ((const char *)c.src < wsb || (const char *)c.src + ext_s > wse)) { REPORT("copy %zu src out\n", k); ++bad; }
            }
            // ops: items and descriptors inside the item region
            for (const auto &o : ops) {
                if (o.kind <= 1 && o.off + (size_t)o.n * sizeof(BItem) > B->o_items + bytes) { REPORT("op items out\n"); ++bad; }
                if (o.kind >= 3 && o.off + (size_t)o.n * sizeof(BCopy) > B->o_items + bytes) { REPORT("op copies out\n"); ++bad; }
            }
            if (verbose) REPORT("od=%d gm=%d: %zu items, %zu copies, %zu ops, %zu bytes (cap %zu)\n", od, gm,
                                bd.items.size(), bd.copies.size(), ops.size(), bytes, B->items_cap);
        }
    B->ws = nullptr;
    for (int i = 0; i < B->n; ++i) B->plans[i]->ws = nullptr;
    return bad;
}
