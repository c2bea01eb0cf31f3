#!/usr/bin/env python3
"""Benchmark: semi-Lagrangian MGRIT for 1D variable-speed advection on one
MI355X (nx = 4096, nt = 16384, dt = 4h, p = r = 3, m = 8 multilevel V-cycles
down to <= 16 coarse points, FCF relaxation, FP64, relative tolerance 1e-10).

One step = one pass of the whole hot path on resident inputs: plan setup
(fine ERK departure trace, backtracked coarse departure points, sigma on
every level) followed by MGRIT from the seeded initial iterate to the
tolerance, including the final F-relaxation that writes every time point.

value = space-time point-updates (rows of Phi_l applied in relaxation,
residual and output on all levels) per second of step time.  Beside it:
GPU sequential semi-Lagrangian stepping (the speed-up denominator), the
FP32-bulk variant, the dominant kernel against the HBM roofline (HIP events
on the launch stream), and the FP64 CPU oracle on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "space-time point-updates/s in relaxation + MGRIT time-to-1e-10 vs GPU seq. stepping"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-bulk variant")
    ap.add_argument("--cpu-nt", type=int, default=4096, help="time steps of the CPU oracle sample")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the level-0 F+C sweep kernel (FP64 and FP32 bulk in 1D; FP32 bulk and one "
                         "level-1 sweep with --workload 2d) and a 1 GiB device copy (for counter runs)")
    ap.add_argument("--workload", choices=["1d", "batch", "adjoint", "2d", "paper"], default="1d",
                    help="1d: the single 1D problem (default line); batch: 64 drawn 1D problems solved together; "
                         "adjoint: gradient of a final-time misfit for the 2D 256^2 problem; "
                         "2d: the 2D 512^2 FP32-bulk problem")
    return ap.parse_args()


def batch_bench(args):
    """64 independent 1D problems of drawn (nx, nt, p, amplitude), FP32 bulk
    with FP64 tracing and norms, solved together: persistent work-list
    sweeps, device-side stopping test, one captured V-cycle replayed.  One
    step = setup of every problem + the batched solve.  The sequential
    baseline steps all 64 problems concurrently (one persistent launch over
    the problems)."""
    import torch
    from paper_2203_13382_amd import Batch
    from paper_2203_13382_amd import inputs as I
    from paper_2203_13382_amd import workloads as W
    probs, prec = W.batch_config()
    dt = np.float32 if prec == "fp32" else np.float64
    b = Batch(probs, prec).setup()
    t0 = time.perf_counter()
    b.tune()
    tune_s = time.perf_counter() - t0
    u0s = [torch.from_numpy(I.initial_condition(pr, 10 + i).astype(dt)).cuda() for i, (pr, sv) in enumerate(probs)]
    uis = [torch.from_numpy(I.initial_iterate(pr.nt, pr.S, sv.m[0], 20 + i).astype(dt)).cuda()
           for i, (pr, sv) in enumerate(probs)]
    us = [torch.empty_like(u) for u in uis]
    last = {}

    def one_step():
        b.setup()
        for u, ui in zip(us, uis):
            u.copy_(ui)
        last["st"], _ = b.solve(u0s, us, use_graph=True)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.steps):
        e0.record(stream)
        one_step()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))
    st = last["st"]
    upd = sum(s["point_updates"] for s in st)
    its = [s["iterations"] for s in st]
    # sequential stepping of every problem, all problems concurrently
    seq = Batch([(pr, W.Solver(m=[2], max_levels=1)) for pr, sv in probs], prec).setup()
    useq = [torch.empty_like(u) for u in uis]

    def seq_step():
        seq.setup()
        seq.solve(u0s, useq, use_graph=False)
    seq_ms = timed(torch, seq_step, max(1, args.steps))
    err = max(float((u.double() - v.double()).abs().max() / v.double().abs().max()) for u, v in zip(us, useq))
    # the same problems stepped in FP64 (the GPU stepping equals the oracle's
    # to 1e-11): the FP32-bulk MGRIT error against FP64
    seq64 = Batch([(pr, W.Solver(m=[2], max_levels=1)) for pr, sv in probs], "fp64").setup()
    u064 = [torch.from_numpy(I.initial_condition(pr, 10 + i)).cuda() for i, (pr, sv) in enumerate(probs)]
    u64 = [torch.empty(u.shape, dtype=torch.float64, device="cuda") for u in uis]
    seq64.solve(u064, u64, use_graph=False)
    torch.cuda.synchronize()
    err64 = max(float((u.double() - v).abs().max() / v.abs().max()) for u, v in zip(us, u64))
    del seq64, u064, u64
    pts = sum(pr.nt * pr.S for pr, sv in probs)
    out = {
        "metric": METRIC, "value": upd / (ms * 1e-3), "unit": "point-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch of {len(probs)} 1D problems, nx 256..8192, nt 1024..16384, p in 1/3/5, "
                               f"dt=0.85h, alpha amplitudes U[0.2,0.8] (seed 4), m=8 to <=16 points, FCF, "
                               f"FP32 bulk + FP64 tracing/norms, rel. tol 1e-6",
                   "problems": len(probs), "space_time_points": pts, "precision": prec},
        "mgrit": {"time_to_tol_ms": ms, "point_updates": upd, "iterations_min": min(its),
                  "iterations_max": max(its), "statuses": sorted(set(s["status"] for s in st)),
                  "max_rel_err_vs_seq": err, "max_rel_err_vs_fp64_seq": err64, "tune_s": tune_s},
        "seq": {"total_ms": seq_ms, "point_updates_per_s": pts / (seq_ms * 1e-3)},
        "speedup_vs_seq": seq_ms / ms,
    }
    print(json.dumps(out))


def kernel_only(args):
    """The dominant HBM kernel alone (level-0 F+C sweep of the 1D workload,
    or with --workload 2d the 2D one, plus one level-1 sweep whose batched
    GMRES kernels the counters also cover), each plan autotuned as in the
    bench line, and a plain copy of known size whose counter readings
    calibrate FETCH_SIZE / WRITE_SIZE."""
    import torch
    from paper_2203_13382_amd import Plan
    from paper_2203_13382_amd import inputs as I
    from paper_2203_13382_amd import workloads as W
    if args.workload == "2d":
        pr, sv, prec = W.config(3)
        dt = torch.float32
    else:
        pr, sv, _ = W.config(2)
        prec, dt = "fp64", torch.float64
    el = 8 if prec == "fp64" else 4
    plan = Plan(pr, sv, prec).setup().autotune()
    ui = torch.from_numpy(I.initial_iterate(pr.nt, pr.S, sv.m[0], 1)).to(device="cuda", dtype=dt)
    cin = ui[::sv.m[0]].contiguous()
    cout = torch.empty_like(cin)
    ms = timed(torch, lambda: plan.relax_into(0, "FC", c_in=cin, c_out=cout), args.kernel_reps)
    nc = pr.nt // sv.m[0]
    out = {"kernel": "level-0 F+C sweep", "workload": args.workload, "launch_ms": ms,
           "launch_info": plan.launch_info(0, nc)}
    if pr.dim == 1:
        out["bytes_per_launch"] = el * pr.S * (pr.nt + 2 * nc + 1)
        # the FP32-bulk plan's level-0 sweep (float displacements and slices)
        p32 = Plan(pr, sv, "fp32").setup().autotune()
        c32, o32 = cin.float(), torch.empty_like(cin, dtype=torch.float32)
        out["fp32_launch_ms"] = timed(torch, lambda: p32.relax_into(0, "FC", c_in=c32, c_out=o32), args.kernel_reps)
        out["fp32_bytes_per_launch"] = 4 * pr.S * (pr.nt + 2 * nc + 1)
    else:
        out["bytes_per_launch"] = el * pr.S * (4 * pr.nt + 2 * nc)
        N1, m1 = plan.N[1], plan.m[1]
        c1 = torch.randn(N1 // m1 + 1, pr.S, dtype=dt, device="cuda")
        g1 = torch.randn(N1 + 1, pr.S, dtype=dt, device="cuda") * 1e-3
        o1 = torch.empty_like(c1)
        out["level1_sweep_ms"] = timed(torch, lambda: plan.relax_into(1, "FC", c_in=c1, g=g1, c_out=o1), 1, warm=0)
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)   # 1 GiB
    dst = torch.empty_like(src)
    out["copy_ms"] = timed(torch, lambda: dst.copy_(src), 3)
    out["copy_bytes_each_way"] = src.numel() * 8
    print(json.dumps(out))


def adjoint_bench(args):
    """2D adjoint workload (256^2, nt = 2048, dt = 2h, p = r = 3, m = 4 to
    <= 16 points, FCF, FP64): one step = plan setup + forward MGRIT keeping
    the C-point checkpoints + the adjoint (inverse stencil index, reverse-time
    adjoint MGRIT, F-point recomputation and gradient accumulation).  The
    sequential baseline is GPU sequential stepping of the forward problem."""
    import ctypes as C
    import torch
    from paper_2203_13382_amd import Plan
    from paper_2203_13382_amd import _native as N
    from paper_2203_13382_amd import inputs as I
    from paper_2203_13382_amd import workloads as W
    from paper_2203_13382_amd.autograd import with_theta
    pr, sv, theta, theta_true = W.adjoint_config()
    stream = torch.cuda.current_stream()
    u0 = torch.from_numpy(I.initial_condition(pr, 0)).cuda()
    seq_plan = Plan(with_theta(pr, theta_true), W.Solver(m=[2], max_levels=1), "fp64").setup()
    u_obs = torch.empty(pr.S, dtype=torch.float64, device="cuda")
    N.check(N.lib().slm_step(seq_plan.h, C.c_void_p(u0.data_ptr()), C.c_void_p(u_obs.data_ptr()), 0,
                             C.c_void_p(stream.cuda_stream)), seq_plan.h)
    plan = Plan(pr, sv, "fp64", adjoint=True)
    m0 = sv.m[0]
    c_init = torch.from_numpy(I.initial_iterate(pr.nt, pr.S, m0, 1)[::m0].copy()).cuda()
    c = torch.empty_like(c_init)
    r = {}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def one_step():
        ev[0].record(stream)
        plan.setup()
        c.copy_(c_init)
        r["f"], _ = plan.solve_cpoints(u0, c)
        ev[1].record(stream)
        r["g0"], r["gth"], r["a"], _ = plan.adjoint(c, c[-1] - u_obs)
        ev[2].record(stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    tot, fwd, adj = [], [], []
    for _ in range(args.steps):
        one_step()
        torch.cuda.synchronize()
        tot.append(ev[0].elapsed_time(ev[2]))
        fwd.append(ev[0].elapsed_time(ev[1]))
        adj.append(ev[1].elapsed_time(ev[2]))
    ms = float(np.mean(tot))
    upd = r["f"]["point_updates"] + r["a"]["point_updates"]
    pl1 = Plan(pr, W.Solver(m=[2], max_levels=1), "fp64")
    useq = torch.empty(pr.S, dtype=torch.float64, device="cuda")

    def seq_step():
        pl1.setup()
        N.check(N.lib().slm_step(pl1.h, C.c_void_p(u0.data_ptr()), C.c_void_p(useq.data_ptr()), 0,
                                 C.c_void_p(stream.cuda_stream)), pl1.h)
    seq_ms = timed(torch, seq_step, max(1, args.steps))
    out = {
        "metric": METRIC, "value": upd / (ms * 1e-3), "unit": "point-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"adjoint of 2D advection, nx=ny={pr.nx}, nt={pr.nt}, dt=2h, p=r=3, m=4 to <=16 "
                               f"points, FCF, FP64, loss 1/2||u(T)-u_obs||^2, gradient wrt u0 and 4 wave-speed "
                               f"coefficients, C-point checkpoints", "precision": "fp64"},
        "adjoint": {"time_to_gradient_ms": ms, "forward_ms": float(np.mean(fwd)), "adjoint_ms": float(np.mean(adj)),
                    "forward_iterations": r["f"]["iterations"], "adjoint_iterations": r["a"]["iterations"],
                    "point_updates": upd, "grad_theta": [float(v) for v in r["gth"]],
                    "grad_u0_norm": float(r["g0"].norm())},
        "seq": {"forward_ms": seq_ms},
        "forward_speedup_vs_seq": seq_ms / float(np.mean(fwd)),
    }
    print(json.dumps(out))


def twod_bench(args):
    """2D workload: nx = ny = 512, nt = 4096, dt = 2h, p = r = 5, m = 8 to
    <= 16 points, FCF, FP32 bulk (FP64 tracing, sigma and norms), relative
    tolerance 1e-6.  One step = setup + MGRIT + final F-relaxation; beside it
    GPU sequential stepping and the FP32-vs-FP64 error at the final time."""
    import ctypes as C
    import torch
    from paper_2203_13382_amd import Plan
    from paper_2203_13382_amd import _native as N
    from paper_2203_13382_amd import inputs as I
    from paper_2203_13382_amd import workloads as W
    pr, sv, prec = W.config(3)
    stream = torch.cuda.current_stream()
    u0 = torch.from_numpy(I.initial_condition(pr, 0)).cuda()
    ui = torch.from_numpy(I.initial_iterate(pr.nt, pr.S, sv.m[0], 1).astype(np.float32)).cuda()
    plan = Plan(pr, sv, prec).setup().autotune()
    u = torch.empty_like(ui)
    u032 = u0.float()
    r = {}

    def one_step():
        plan.setup()
        u.copy_(ui)
        r["st"], _ = plan.solve(u032, u)

    for _ in range(args.warmup):
        one_step()
    ms = timed(torch, one_step, max(1, args.steps), warm=0)
    st = r["st"]
    seq = Plan(pr, W.Solver(m=[2], max_levels=1), "fp64")
    useq = torch.empty(pr.S, dtype=torch.float64, device="cuda")

    def seq_step():
        seq.setup()
        N.check(N.lib().slm_step(seq.h, C.c_void_p(u0.data_ptr()), C.c_void_p(useq.data_ptr()), 0,
                                 C.c_void_p(stream.cuda_stream)), seq.h)
    seq_ms = timed(torch, seq_step, max(1, args.steps))
    seq32 = Plan(pr, W.Solver(m=[2], max_levels=1), "fp32")
    useq32 = torch.empty(pr.S, dtype=torch.float32, device="cuda")

    def seq32_step():
        seq32.setup()
        N.check(N.lib().slm_step(seq32.h, C.c_void_p(u032.data_ptr()), C.c_void_p(useq32.data_ptr()), 0,
                                 C.c_void_p(stream.cuda_stream)), seq32.h)
    seq32_ms = timed(torch, seq32_step, max(1, args.steps))
    err = float((u[-1].double() - useq).abs().max() / useq.abs().max())
    out = {
        "metric": METRIC, "value": st["point_updates"] / (ms * 1e-3), "unit": "point-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"2D advection alpha=(cos(pi y)cos(pi t), sin(pi x)), nx=ny={pr.nx}, nt={pr.nt}, "
                               f"dt=2h, p=r=5 tensor product, m=8 to <=16 points, FCF, FP32 bulk + FP64 "
                               f"tracing/norms, rel. tol 1e-6", "precision": prec},
        "mgrit": {"time_to_tol_ms": ms, "iterations": st["iterations"], "status": st["status"],
                  "rho_final_over_rho0": st["rho_final"] / st["rho0"], "point_updates": st["point_updates"],
                  "gmres_solves": st["gmres_solves"], "gmres_iters": st["gmres_iters"],
                  "max_rel_err_vs_fp64_seq_at_T": err},
        "seq": {"fp64_ms": seq_ms, "fp32_ms": seq32_ms},
        "speedup_vs_fp32_seq": seq32_ms / ms,
    }
    levels = level_table(torch, plan, pr, prec, 5)
    l0 = levels[0]
    tiled, nb = plan.launch_info(0, plan.N[0] // plan.m[0])
    out["levels"] = levels
    out["roofline"] = {"kernel": f"level-0 F+C sweep (LDS-tiled SL steps, tile choice {plan.tile_choice()})"
                                 if tiled else "level-0 F+C sweep (gather SL steps)",
                       "bound": "hbm", "achieved": l0["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": l0["frac"],
                       "traffic": measured_traffic("cfg3_2d_kernels.md", ("slm_chain2d.hip", "slm_common.h")),
                       "launch_ms": l0["sweep_us"] * 1e-3,
                       "bytes_per_launch": l0["bytes"]}
    cr = copy_rate(torch)
    out["roofline"].update({"copy_GBps": cr, "frac_of_copy": l0["GBps"] / cr})
    print(json.dumps(out))


def paper_bench(args):
    """The paper's Sec. 5 problems on one GPU, FP64: 1D alpha =
    cos(2 pi t)cos(2 pi x) on 2^12 x 2^14 and 2D with the time-dependent
    field on (2^9)^2 x 2^13, dt = 0.85h, u0 = sin^4 / sin^2, p = r = 1, 3, 5,
    m = 16 on the first level and 4 below, GMRES(10, 1e-2), relative tolerance
    1e-10.  Each run: setup + MGRIT keeping C-points only, next to GPU
    sequential stepping of the same problem.  The JSON value is the 1D p = 3
    run; the 1D iteration counts are printed in the paper (13, 19, 24)."""
    import ctypes as C
    import sys
    import torch
    from paper_2203_13382_amd import Plan
    from paper_2203_13382_amd import _native as N
    from paper_2203_13382_amd import workloads as W
    stream = torch.cuda.current_stream()
    printed = {1: 13, 3: 19, 5: 24}
    runs = {}
    for dim, field, nx, nt in ((1, "a4", 4096, 16384), (2, "var", 512, 8192)):
        for p in (1, 3, 5):
            pr = W.paper_problem(dim, field, p, nx, nt)
            u0n = W.paper_initial_condition(dim, nx)
            sv = W.Solver(m=[16, 4], coarsest_max_points=2, gmres_kmax=10, gmres_rtol=1e-2, max_iter=300)
            plan = Plan(pr, sv, "fp64")
            u0 = torch.from_numpy(u0n).cuda()
            g = torch.Generator(device="cuda")
            g.manual_seed(5)
            c_init = torch.rand((pr.nt // 16 + 1, pr.S), generator=g, dtype=torch.float64, device="cuda")
            c = torch.empty_like(c_init)
            r = {}

            def one_step():
                plan.setup()
                c.copy_(c_init)
                r["st"], _ = plan.solve_cpoints(u0, c)
            ms = timed(torch, one_step, max(1, args.steps), warm=args.warmup)
            seq = Plan(pr, W.Solver(m=[2], max_levels=1), "fp64")
            useq = torch.empty(pr.S, dtype=torch.float64, device="cuda")

            def seq_step():
                seq.setup()
                N.check(N.lib().slm_step(seq.h, C.c_void_p(u0.data_ptr()), C.c_void_p(useq.data_ptr()), 0,
                                         C.c_void_p(stream.cuda_stream)), seq.h)
            seq_ms = timed(torch, seq_step, max(1, args.steps))
            st = r["st"]
            runs[f"{dim}d_p{p}"] = {"time_to_tol_ms": ms, "iterations": st["iterations"],
                                    "iterations_printed": printed[p] if dim == 1 else None,
                                    "status": st["status"], "seq_ms": seq_ms, "speedup_vs_seq": seq_ms / ms,
                                    "point_updates": st["point_updates"],
                                    "max_rel_err_vs_seq_at_T": float((c[-1] - useq).abs().max() / useq.abs().max())}
            del plan, seq
            print(f"# {dim}d p={p}: {ms:.1f} ms, {st['iterations']} cycles, seq {seq_ms:.1f} ms",
                  file=sys.stderr, flush=True)
    main_run = runs["1d_p3"]
    out = {
        "metric": METRIC, "value": main_run["point_updates"] / (main_run["time_to_tol_ms"] * 1e-3),
        "unit": "point-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_run["time_to_tol_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Sec. 5 problems: 1D alpha=cos(2 pi t)cos(2 pi x), 2^12 x 2^14 and 2D time-dependent "
                               "field, (2^9)^2 x 2^13; dt=0.85h, p=r=1,3,5, m=16 then 4, GMRES(10, 1e-2), rel. tol "
                               "1e-10, FP64; value = 1D p=3"},
        "runs": runs,
    }
    print(json.dumps(out))


def measured_traffic(profile="cfg2_kernels.md",
                     sources=("slm_kernels1d.h", "slm_chain1d.hip", "slm_fine1d.hip", "slm_common.h")):
    """HBM bytes per launch of a workload's level-0 sweep from its committed
    counter summary, or None once the kernel sources (device code of the
    sweep and its helpers) differ from the ones profiled."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", profile)
    csrc = os.path.join(ROOT, "paper_2203_13382_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in sources]
    try:
        kv = dict(line.split(": ", 1) for line in open(prof).read().splitlines() if ": " in line
                  and line.split(": ", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_sha256_16"))
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in srcs)).hexdigest()[:16]
        return int(kv["traffic_bytes_per_launch"]) if kv.get("kernel_source_sha256_16", "").strip() == sha else None
    except (OSError, KeyError, ValueError):
        return None


def copy_rate(torch):
    """Read + write rate of a plain 1 GiB device-to-device copy (GB/s): the
    practical ceiling a streaming kernel meets on this GPU, reported beside
    the roofline fraction of the nominal peak."""
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ms = timed(torch, lambda: dst.copy_(src), 5)
    rate = 2 * src.numel() * 8 / (ms * 1e-3) / 1e9
    del src, dst
    return rate


def timed(torch, fn, reps, warm=1):
    st = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def updates_of(N, m, iterations, fcf, L):
    """Point-updates of the V-cycle schedule used by the library, in units
    of spatial slices (multiply by S)."""
    tot = 0
    if L == 1:
        return N[0]

    def coarse(l):
        if l == L - 1:
            return N[l]
        nc = N[l] // m[l]
        return (N[l] if fcf else 0) + N[l] + coarse(l + 1) + (N[l] - nc)
    for k in range(iterations):
        tot += (N[0] if fcf else 0) + N[0]
        if k < iterations - 1:
            tot += coarse(1)
    return tot + N[0] - N[0] // m[0]


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU time-slab sharding "
                                   "is a design note only (--gpus must be 1)"}))
        sys.exit(2)
    import torch
    from paper_2203_13382_amd import Plan
    from paper_2203_13382_amd import inputs as I
    from paper_2203_13382_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.kernel_only:
        return kernel_only(args)
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "adjoint":
        return adjoint_bench(args)
    if args.workload == "paper":
        return paper_bench(args)
    if args.workload == "2d":
        return twod_bench(args)
    dev = torch.device("cuda")

    pr, sv, _ = W.config(2)
    workload = (f"1D periodic advection alpha=1+0.5 sin(pi x)cos(2 pi t), nx={pr.nx}, nt={pr.nt}, dt=4h, "
                f"p=r={pr.p}, multilevel V-cycles m={sv.m[0]} to <={sv.coarsest_max_points} points, FCF, "
                f"GMRES(10, 1e-2), rel. tol {sv.tol:g}")
    u0 = torch.from_numpy(I.initial_condition(pr, 0)).to(dev)
    ui = torch.from_numpy(I.initial_iterate(pr.nt, pr.S, sv.m[0], 1)).to(dev)

    # ---------------------------------------------------------------- FP64 MGRIT
    plan = Plan(pr, sv, "fp64").setup().autotune()
    u = torch.empty_like(ui)
    last = {}

    def one_step():
        plan.setup()
        u.copy_(ui)
        last["st"], last["hist"] = plan.solve(u0, u)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    st_ = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_steps = []
    for _ in range(args.steps):
        e0.record(st_)
        one_step()
        e1.record(st_)
        torch.cuda.synchronize()
        ms_steps.append(e0.elapsed_time(e1))
    ms = float(np.mean(ms_steps))
    stats = last["st"]
    setup_ms = timed(torch, lambda: plan.setup(), 3)
    upd = stats["point_updates"]
    value = upd / (ms * 1e-3)

    # ---------------------------------------------------------------- sequential stepping
    seq_plan = Plan(pr, W.Solver(m=[2], max_levels=1), "fp64").setup()
    useq = torch.empty_like(ui)
    from paper_2203_13382_amd import _native as N
    import ctypes as C

    def seq_step():
        N.check(N.lib().slm_step(seq_plan.h, C.c_void_p(u0.data_ptr()), C.c_void_p(useq.data_ptr()), 1,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream)), seq_plan.h)
    trace_ms = timed(torch, lambda: seq_plan.setup(), 3)
    seq_ms = timed(torch, seq_step, 3)
    err = float((u - useq).abs().max() / useq.abs().max())

    # ---------------------------------------------------------------- dominant kernel
    nc = pr.nt // sv.m[0]
    cin = ui[::sv.m[0]].contiguous()
    cout = torch.empty_like(cin)
    k_ms = timed(torch, lambda: plan.relax_into(0, "FC", c_in=cin, c_out=cout), args.kernel_reps)
    k_bytes = 8 * pr.S * (pr.nt + 2 * nc + 1)
    k_gbs = k_bytes / (k_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC, "value": value, "unit": "point-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "nx": pr.nx, "nt": pr.nt, "p": pr.p, "m": sv.m[0],
                   "levels": plan.N, "precision": "fp64"},
        "mgrit": {"iterations": stats["iterations"], "status": stats["status"],
                  "rho0": stats["rho0"], "rho_final": stats["rho_final"],
                  "time_to_tol_ms": ms, "setup_ms": setup_ms, "solve_ms": ms - setup_ms,
                  "point_updates": upd, "gmres_solves": stats["gmres_solves"],
                  "gmres_iters": stats["gmres_iters"], "max_rel_err_vs_seq": err},
        "seq": {"trace_ms": trace_ms, "step_ms": seq_ms, "total_ms": trace_ms + seq_ms,
                "point_updates_per_s": pr.nt * pr.S / ((trace_ms + seq_ms) * 1e-3)},
        "speedup_vs_seq": (trace_ms + seq_ms) / ms,
        "roofline": {"kernel": "level-0 F+C relaxation sweep (chain1d, FP64)", "bound": "hbm",
                     "achieved": k_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": k_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(), "launch_ms": k_ms, "bytes_per_launch": k_bytes},
    }

    cr = copy_rate(torch)
    out["roofline"].update({"copy_GBps": cr, "frac_of_copy": k_gbs / cr})

    # ---------------------------------------------------------------- FP32 bulk
    if not args.no_fp32:
        import dataclasses
        sv32 = dataclasses.replace(sv, tol=1e-6)
        p32 = Plan(pr, sv32, "fp32").setup().autotune()
        u32 = torch.empty(ui.shape, dtype=torch.float32, device=dev)
        ui32 = ui.float()
        u032 = u0.float()
        r = {}

        def step32():
            p32.setup()
            u32.copy_(ui32)
            r["st"], _ = p32.solve(u032, u32)
        step32()
        ms32 = timed(torch, step32, max(1, args.steps), warm=0)
        st32 = r["st"]
        out["fp32_bulk"] = {"time_to_tol_ms": ms32, "iterations": st32["iterations"], "status": st32["status"],
                            "tol_rel": sv32.tol, "rho_final_over_rho0": st32["rho_final"] / st32["rho0"],
                            "value": st32["point_updates"] / (ms32 * 1e-3),
                            "max_rel_err_vs_fp64_seq": float((u32.double() - useq).abs().max() / useq.abs().max()),
                            "speedup_vs_fp64_seq": (trace_ms + seq_ms) / ms32}

    # ---------------------------------------------------------------- per-level sweeps
    out["levels"] = level_table(torch, plan, pr, "fp64", args.kernel_reps)

    # ---------------------------------------------------------------- CPU oracle baseline
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pr, sv, args.cpu_nt)
    print(json.dumps(out))


def level_table(torch, plan, pr, prec, reps):
    """One F+C sweep on every level but the coarsest, timed with HIP events
    on the launch stream: microseconds per sweep, point-updates per second,
    and for level 0 the HBM rate of its algorithmic bytes (the displacement
    of every update, the start C-points read and the new C-points written;
    the slice stays on chip).  Coarse levels are latency-bound (GMRES with a
    workgroup barrier per reduction), so their update rate is the figure."""
    el = 8 if prec == "fp64" else 4
    dt = torch.float64 if prec == "fp64" else torch.float32
    rows = []
    for l in range(plan.L - 1):
        Nl, m = plan.N[l], plan.m[l]
        nc = Nl // m
        cin = torch.randn(nc + 1, pr.S, dtype=dt, device="cuda")
        g = None if l == 0 else torch.randn(Nl + 1, pr.S, dtype=dt, device="cuda") * 1e-3
        cout = torch.empty_like(cin)
        us = timed(torch, lambda: plan.relax_into(l, "FC", c_in=cin, g=g, c_out=cout), reps) * 1e3
        row = {"level": l, "steps": Nl, "intervals": nc, "sweep_us": us,
               "point_updates_per_s": Nl * pr.S / (us * 1e-6)}
        if l == 0:
            if pr.dim == 1:     # displacement per update; start and new C-point per interval
                b = el * pr.S * (Nl + 2 * nc + 1)
            else:               # two displacements, the previous slice and the new one per update
                b = el * pr.S * (4 * Nl + 2 * nc)
            row.update({"bound": "hbm", "bytes": b, "GBps": b / (us * 1e-6) / 1e9,
                        "frac": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS})
        else:
            row["bound"] = "latency"
        rows.append(row)
    return rows


def cpu_threads():
    """Host threads the oracle may use: the CPUs this process may run on,
    at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(pr, sv, cpu_nt):
    """The FP64 oracle (unchanged) on a bounded sample of the same workload:
    the same PDE and solver with nt = cpu_nt, setup + MGRIT to the
    tolerance, once on one thread and once on every host thread it may use
    (intervals in parallel, fixed-order sums; identical results)."""
    from oracle import oracle as O
    from paper_2203_13382_amd import inputs as I
    from paper_2203_13382_amd import workloads as W
    O.build(force=False)
    prc = W.scaled(pr, pr.nx, cpu_nt, 4.0)
    u0c = I.initial_condition(prc, 0)
    uic = I.initial_iterate(prc.nt, prc.S, sv.m[0], 1)
    res = {}
    nthr = cpu_threads()
    keep = O.get_threads()
    try:
        for n in (1, nthr):
            O.set_threads(n)
            t0 = time.perf_counter()
            ctx = O.Context(prc, sv)
            _, stc, _ = ctx.mgrit(u0c, uic)
            res[n] = (time.perf_counter() - t0, stc, ctx)
    finally:
        O.set_threads(keep)
    tc, stc, ctx = res[nthr]
    updc = updates_of(ctx.N, ctx.m, stc["iterations"], sv.relax == "FCF", ctx.L) * prc.S
    t1 = res[1][0]
    return {"value": updc / tc, "unit": "point-updates/s", "cores": nthr, "kind": "oracle",
            "single_thread_value": updc / t1, "cpu_model": cpu_model(),
            "sample": f"same PDE and solver with nt={prc.nt} (1/{pr.nt // prc.nt} of the time domain): setup + "
                      f"MGRIT to rel. 1e-10, {stc['iterations']} iterations; {tc:.1f} s on {nthr} threads, "
                      f"{t1:.1f} s on 1 thread; updates counted with the GPU schedule"}


if __name__ == "__main__":
    main()
