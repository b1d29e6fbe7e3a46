"""Throughput benchmark of the spectral Monte Carlo hot path on one MI355X.

A step is one residual iteration (reconstruction, time contraction, Monte Carlo
sampling of every node, reduction and update) of one interval of the 2-D
long-time workload (24 x 24 Jacobi-Gauss nodes x 16 Lobatto times per unit
interval, u_t = Lap u + sin u + s), run as the sampling slice
samples 0 .. m-1 of every node (the per-sample work does not depend on M, so
the node-sample rate of the slice is that of the full sample count).

Prints ONE JSON line: node-samples/s of the FP32-sampling form (value), the
FP64 form on the same slice (the throughput ratio and the time to each error
decade against the exact solution), the speedup at equal accuracy -- FP32
sampling that hands over to FP64 for the last digits against FP64 alone, both
solved to Algorithm 1's tolerance 1e-10 -- the roofline of the dominant kernel
(the sampling kernel, measured with HIP events on its own stream) and the CPU
oracle's rate on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--m-slice m] [--no-cpu] [--no-fp64] [--no-switch]
    python bench.py --workload c1|c3|c4|c5|...   (the other workloads, one line each)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

os.environ.setdefault("HPSMC_TUNE_VERBOSE", "1")   # the tuner reports each trial on stderr
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3   # published MI355X FP32: dense matrix cores, and the vector units with packed FMA
FP64_PEAK_TFLOPS = 78.6    # published MI355X vector FP64
METRIC = "node-samples/sec at fixed error vs exact; FP32-batched vs FP64 speedup"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "advance_mma_kernel_c2_fp32_m1024_traffic.json")
# the matrix-core round kernel's sources (its unit and the device helpers it includes)
KERNEL_SRC = [os.path.join(ROOT, "paper_2608_22190_amd", "csrc", f) for f in ("hpsmc_kern_mma.hip", "hpsmc_device.h")]


def measured_traffic(launch):
    """HBM bytes per launch of the sampling kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by the copy-kernel calibration),
    or None when the kernel source or launch shape changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        h = hashlib.sha256()
        for f in KERNEL_SRC:
            h.update(open(f, "rb").read())
        sha = h.hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != sha or list(rec.get("launch", [])) != list(launch):
        return None
    return 1024.0 * (rec["fetch_kib_per_launch"] * rec["fetch_factor"] + rec["write_kib_per_launch"] * rec["write_factor"])


def flops_per_eval(dim, P, picard=False):
    """Algorithmic FP operations of one residual evaluation: the nested
    tensor-product contraction of the u and v slabs (2 polynomials x 2 flops x
    (P^d + P^{d-1} + ... + P) multiply-adds) plus the three-term recurrences of
    the d coordinates (3 flops per new Legendre value).  The Picard-form
    integrand f(u*) + s needs the u slab only (one polynomial)."""
    cont = sum(P ** k for k in range(1, dim + 1))
    return (2 if picard else 4) * cont + 3 * dim * (P - 2)


def run_gpu(wl, steps, warmup, launch, torch, tune_cache=None, m_tune=256, exact_fn=None):
    """Warm up, then time `steps` residual iterations of interval 1 from the
    replicated initial data.  With `exact_fn` (grid -> nodal values of the exact
    solution), every timed iteration also records (seconds so far, max error against it,
    max node standard error, max|eps|), read after its own timing stops."""
    from paper_2608_22190_amd import hpsmc
    stream = torch.cuda.Stream()
    with hpsmc.Plan(wl) as plan:
        exact = exact_fn(plan.hpsmc_grid(0)) if exact_fn else None
        if launch:
            plan.hpsmc_set_launch(*launch)
        elif tune_cache:
            t0 = time.perf_counter()
            plan.hpsmc_tune(0, m_tune, tune_cache, stream=stream)
            print(f"[bench] {wl.precision} launch {plan.hpsmc_get_launch()} ({time.perf_counter() - t0:.1f}s)",
                  file=sys.stderr, flush=True)
        plan.hpsmc_start_interval(0, stream=stream)
        for w in range(warmup):
            plan.hpsmc_iterate(0, w, stream=stream)
            stream.synchronize()
            print(f"[bench] {wl.precision} warmup {w + 1}/{warmup}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        plan.hpsmc_reset_stats(stream=stream)
        plan.hpsmc_start_interval(0, stream=stream)
        torch.cuda.synchronize()
        traj, busy = [], 0.0
        t0 = time.perf_counter()
        for k in range(steps):
            ts = time.perf_counter()
            plan.hpsmc_iterate(0, k, stream=stream)
            if steps > 1 or exact is not None:
                stream.synchronize()
                busy += time.perf_counter() - ts
                print(f"[bench] {wl.precision} step {k + 1}/{steps} {busy:.2f}s", file=sys.stderr, flush=True)
            if exact is not None:
                Uk = plan.hpsmc_get_nodes(0, stream=stream)[0]
                ek, sk = plan.hpsmc_get_increment(0, stream=stream)
                sig_k = float(np.sqrt(np.maximum(sk / wl.M - ek ** 2, 0.0) / wl.M).max())
                traj.append([busy, float(np.max(np.abs(Uk - exact))), sig_k, float(np.max(np.abs(ek)))])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if exact is not None:
            t1 = t0 + busy                 # the reads of the trajectory are not timed
        st = plan.hpsmc_stats(stream=stream)
        U = plan.hpsmc_get_nodes(0, stream=stream)
        grid = plan.hpsmc_grid(0)
        eps, ssq = plan.hpsmc_get_increment(0, stream=stream)
        lau = plan.hpsmc_get_launch()
        mma = plan.hpsmc_get_option("sample_mfma_active")
    sig = float(np.sqrt(np.maximum(ssq / wl.M - eps ** 2, 0.0) / wl.M).max())
    return {"seconds": t1 - t0, "stats": st, "U": U, "sigma": sig, "launch": lau, "mma": mma, "grid": grid,
            "trajectory": traj}


def run_switched_solve(wl, tol, switch_tol, torch, tune_cache=None):
    """Algorithm 1 on interval 1 with the loop condition max|eps| < tol, FP32
    sampling until max|eps| < switch_tol and FP64 after (one timed solve);
    switch_tol None: FP64 throughout."""
    from paper_2608_22190_amd import hpsmc
    stream = torch.cuda.Stream()
    wl = (wl.with_(precision="fp64", tol=tol) if switch_tol is None else
          wl.with_(precision="fp32_then_fp64", switch_tol=switch_tol, tol=tol))
    with hpsmc.Plan(wl) as plan:
        if tune_cache:
            plan.hpsmc_tune(0, 256, tune_cache, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status = plan.hpsmc_solve(stream=stream)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        rec = plan.hpsmc_stats(stream=stream)["max_eps"]
        U = plan.hpsmc_get_nodes(0, stream=stream)[0]
        eps, ssq = plan.hpsmc_get_increment(0, stream=stream)
        grid = plan.hpsmc_grid(0)
    used = int(np.count_nonzero(rec))
    switch = None if switch_tol is None else next((k + 1 for k, e in enumerate(rec[:used]) if e < switch_tol), None)
    print(f"[bench] {'FP64' if switch_tol is None else 'switched'} solve to tolerance: {used} iterations "
          f"({switch} in FP32), {sec:.1f}s", file=sys.stderr, flush=True)
    return {"seconds": sec, "status": int(status), "iterations": used, "fp32_iterations": switch, "U": U,
            "grid": grid, "sigma": float(np.sqrt(np.maximum(ssq / wl.M - eps ** 2, 0.0) / wl.M).max()),
            "max_eps": [float(e) for e in rec[:used]]}


def time_to_error(traj, target, col=1):
    """seconds until the first iteration whose column `col` (1: error against the
    exact solution, 3: max|eps|) is below `target`, or None"""
    for t, *vals in traj:
        if vals[col - 1] < target:
            return t
    return None


def long_time_exact(wl, grid):
    """The 2-D long-time workload's manufactured solution at the nodes of
    interval 1: prod_i (1 - x_i^2) sin(x_0 + x_1) e^{cos t} / (1 + t^2)."""
    x, t = grid
    X0, X1 = np.meshgrid(x, x, indexing="ij")
    sp = ((1 - X0 ** 2) * (1 - X1 ** 2) * np.sin(X0 + X1)).reshape(-1)
    tf = np.exp(np.cos(t)) / (1 + t ** 2)
    return sp[:, None] * tf[None, :]


def exact_nodes(name, wl, grid):
    """Nodal values of the manufactured exact solution of a workload (None when
    it has none): C1 e^{-t} sin(pi x); C4 e^{-t} prod cos(pi x_i / 2); the 2-D
    long-time solution for the Picard and ball-point lines."""
    x, t = grid
    if name == "c1":
        return np.sin(np.pi * x)[:, None] * np.exp(-t)[None, :]
    if name == "c4":
        c = np.cos(0.5 * np.pi * x)
        sp = c
        for _ in range(wl.dim - 1):
            sp = np.multiply.outer(sp, c)
        return sp.reshape(-1)[:, None] * np.exp(-t)[None, :]
    if name in ("c2p", "c2b"):
        return long_time_exact(wl, grid)
    return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_other(name, args, torch):
    """Measured line for the other workload shapes (one step each):
    c1 a whole solve (graph-captured), c3 one sweep over all 12 intervals,
    c4 one iteration, c5 forward + adjoint of the batched misfit."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    stream = torch.cuda.Stream()
    m = args.m_slice
    if name == "compare":
        return run_compare(args, torch)
    if name == "aitken":
        return run_aitken(args, torch)
    if name == "ballcmp":
        return run_ballcmp(args, torch)
    if name == "frac":
        return run_frac(args, torch)
    if name == "fraccmp":
        return run_fraccmp(args, torch)
    if name == "fracexp":
        return run_fracexp(args, torch)
    if name == "ex1":
        return run_ex1(args, torch)
    if name == "c1":
        wl = W.c1_single_step()
    elif name == "c2p":
        wl = W.c2_long_time(M=m, iters=args.steps + args.warmup, n_intervals=1, estimator="picard")
    elif name == "c2b":
        wl = W.c2_long_time(M=m, iters=args.steps + args.warmup, n_intervals=1, quad="ball")
    elif name == "c3":
        wl = W.c3_initial_singularity(M=m, sweeps=args.steps + args.warmup)
    elif name == "c4":
        wl = W.c4_five_dim(M=m, iters=args.steps + args.warmup)
    else:
        wl = W.c5_batched_gradient(M=m)
    nodes = wl.nodes_per_sweep * wl.n_instances
    with hpsmc.Plan(wl) as plan:
        if args.launch:
            plan.hpsmc_set_launch(*(int(v) for v in args.launch.split(",")))
        elif args.tune_cache and name in ("c1", "c2p", "c2b", "c3", "c4", "c5"):
            t0 = time.perf_counter()
            # tuned on the slice it times (c1: all its samples, c4: its 16 per node), else a short trial
            plan.hpsmc_tune(0, 256 if name in ("c2p", "c2b") else wl.M if name in ("c1", "c4") else min(wl.M, 4),
                            args.tune_cache, stream=stream)
            print(f"[bench] {name} launch {plan.hpsmc_get_launch()} ({time.perf_counter() - t0:.1f}s)",
                  file=sys.stderr, flush=True)
        def step(k):
            if name == "c1":
                plan.hpsmc_solve(stream=stream)
            elif name in ("c2p", "c2b"):
                plan.hpsmc_iterate(0, k, stream=stream)
            elif name == "c3":
                plan.hpsmc_sweep(k, stream=stream)
            elif name == "c4":
                plan.hpsmc_iterate(0, k, stream=stream)
            else:
                plan.hpsmc_loss_grad_c0(W.c5_target(wl.n_instances, wl.nsp, seed=1), stream=stream)
        if name == "c1":
            plan.hpsmc_set_option("graph", 1)
        for w in range(args.warmup):
            step(w)
            stream.synchronize()
            print(f"[bench] {name} warmup {w + 1}", file=sys.stderr, flush=True)
        plan.hpsmc_reset_stats(stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(args.warmup + k)
            stream.synchronize()
            print(f"[bench] {name} step {k + 1} {time.perf_counter() - t0:.2f}s", file=sys.stderr, flush=True)
        sec = time.perf_counter() - t0
        st = plan.hpsmc_stats(stream=stream)
        st_k = st
        if name == "c1":
            # graph replays record no per-launch events: the round kernel's launch times come
            # from one eager solve after the timed region (the same kernels and work; the solve
            # restarts from the initial data, so the iterate is the graph's, bit for bit)
            plan.hpsmc_set_option("graph", 0)
            plan.hpsmc_reset_stats(stream=stream)
            step(args.warmup + args.steps)
            stream.synchronize()
            st_k = plan.hpsmc_stats(stream=stream)
        plan_launch = plan.hpsmc_get_launch()
        mma = plan.hpsmc_get_option("sample_mfma_active")
        # accuracy of the iterate after the run (outside the timed region)
        acc = None
        if name in ("c1", "c4", "c2p", "c2b"):
            ex = exact_nodes(name, wl, plan.hpsmc_grid(0))
            U = plan.hpsmc_get_nodes(0, stream=stream)[0]
            eps, ssq = plan.hpsmc_get_increment(0, stream=stream)
            acc = {"error_vs_exact": float(np.max(np.abs(U - ex))),
                   "max_node_std_error": float(np.sqrt(np.maximum(ssq / wl.M - eps ** 2, 0.0) / wl.M).max()),
                   "iterations": int(args.warmup + args.steps) if name != "c1" else int(wl.iters),
                   "note": ("max over all nodes of the interval against the manufactured solution after the "
                            "run's iterations from the replicated initial data, with the samples of the slice")}
        elif name == "c3":
            U32 = [plan.hpsmc_get_nodes(iv, stream=stream)[0] for iv in range(wl.n_intervals)]
    if name == "c3":
        # the FP64 sweeps on the same Philox words, for the FP32 result's error against them
        with hpsmc.Plan(wl.with_(precision="fp64")) as p64:
            if args.tune_cache:
                p64.hpsmc_tune(0, min(wl.M, 4), args.tune_cache, stream=stream)
            for k in range(args.warmup + args.steps):
                p64.hpsmc_sweep(k, stream=stream)
            stream.synchronize()
            U64 = [p64.hpsmc_get_nodes(iv, stream=stream)[0] for iv in range(wl.n_intervals)]
            sig = 0.0
            for iv in range(wl.n_intervals):
                eps, ssq = p64.hpsmc_get_increment(iv, stream=stream)
                sig = max(sig, float(np.sqrt(np.maximum(ssq / wl.M - eps ** 2, 0.0) / wl.M).max()))
        acc = {"max_abs_u32_minus_u64": max(float(np.max(np.abs(a - b))) for a, b in zip(U32, U64)),
               "max_node_std_error_fp64": sig, "sweeps": int(args.warmup + args.steps),
               "note": "no exact solution: the FP32 sweeps against the FP64 sweeps on the same Philox words, "
                       "all 12 intervals, after the run's sweeps"}
    per_step = nodes * wl.M * (wl.iters if name in ("c1", "c5") else 1)
    P = wl.n + 2
    fpe = flops_per_eval(wl.dim, P, picard=wl.estimator == "picard")
    k_ms = st_k["sample_ms"] / max(1, st_k["sample_launches"])
    launches = max(1, st_k["advance_launches"] or st_k["sample_launches"])
    desc = {"c1": "c1_1d_single_step: whole solve (5 iterations, 256 nodes x M=4096), FP64, hipGraph replay",
            "c2p": f"c2_2d_long_time interval 1, one Picard-form (classical Monte Carlo, eq. uast) iteration, "
                   f"{nodes} nodes x samples 0..{m - 1} of M=65536, FP32 sampling",
            "c2b": f"c2_2d_long_time interval 1, one residual iteration with the ball-point path quadrature, "
                   f"{nodes} nodes x samples 0..{m - 1} of M=65536, FP32 sampling",
            "c3": f"c3_2d_initial_singularity: one sweep over all 12 geometric intervals ({nodes} nodes, "
                  f"degrees 4..26) x samples 0..{m - 1} of M=32768, FP32",
            "c4": f"c4_5d: one residual iteration, {nodes} nodes (8^5 x 8) x samples 0..{m - 1} of M=16384, FP32",
            "c5": f"c5_2d_batched_gradient: forward (6 iterations) + adjoint, 256 instances x {wl.nsp * 12} nodes "
                  f"x samples 0..{m - 1} of M=8192, FP32"}[name]
    out = {"metric": METRIC, "value": per_step * args.steps / sec, "unit": "node-samples/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64" if wl.precision == "fp64" else "f32",
           "data": "synthetic", "config": {"workload": desc, "max_nstar": int(hpsmc.resolve_nstar(wl)[0].max()),
                                           "launch": list(plan_launch)}}
    if name != "c5":
        out["roofline"] = {"bound": "mfma" if mma else "alu", "achieved": fpe * st_k["path_steps"] / launches / max(1e-9, k_ms * 1e-3) / 1e12
                           if st_k["sample_launches"] else None,
                           "peak": FP64_PEAK_TFLOPS if wl.precision == "fp64" else FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "avg_launch_ms": k_ms, "flops_per_eval": fpe,
                           "lane_utilization": st["path_steps"] / max(1, st["lane_steps"])}
        if out["roofline"]["achieved"] is not None:
            out["roofline"]["frac"] = out["roofline"]["achieved"] / out["roofline"]["peak"]
    else:
        # the dominant kernel is the adjoint: it replays every forward evaluation and forms, per
        # evaluation, u* (2 (P + P^2) flops), the Legendre values at both coordinates (3 flops
        # each) and the two weighted outer products L(x_0) (x) L(x_1) (2 P^2 multiply-adds each)
        fadj = 2 * (P + P * P) + 3 * 2 * (P - 2) + 4 * P * P
        adj_ms = st["adjoint_ms"]
        fwd_ms = st["sample_ms"]
        achieved = fadj * st["path_steps"] / max(1e-9, adj_ms * 1e-3) / 1e12
        out["roofline"] = {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
                           "kernel": (f"adjoint_mma2_kernel<{(P + 1) // 2}> (u* on v_mfma_f32_32x32x2f32, the "
                                      f"outer products on v_mfma_f32_16x16x4f32)" if P <= 20 else
                                      "adjoint_kernel<float,2,PMAX,true> (outer products on v_mfma_f32_32x32x2f32)"),
                           "flops_per_eval": fadj,
                           "evals_per_launch": st["path_steps"] / max(1, st["adjoint_launches"]),
                           "avg_launch_ms": adj_ms / max(1, st["adjoint_launches"]),
                           "adjoint_ms_per_step": adj_ms / args.steps,
                           "forward_round_kernel_ms_per_step": fwd_ms / args.steps,
                           "adjoint_over_forward": adj_ms / max(1e-9, fwd_ms)}
    out["path_steps_per_s"] = st["path_steps"] / sec
    out["mean_path_length"] = st["path_steps"] / max(1, st["node_samples"])
    if acc is not None:
        out["accuracy"] = acc
    print(json.dumps(out), flush=True)


def run_compare(args, torch):
    """The paper's contrast between the classical (Picard-form) Monte Carlo
    estimator and the residual form, on one partition: the 1-D long-time
    problem u_t = u_xx + sin u + s to T = 10 in unit intervals (u_ex =
    (1-x^2) sin x e^{cos t}/(1+t^2)), 16 nodes, degree 16 in time, M = 4096,
    6 iterations per interval, FP64; error against u_ex at every node."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    tb = [float(k) for k in range(11)]
    base = W._mk("long_time_1d", 1, 16, tb, [16] * 10, f="sin", src="longtime", ic="exact", M=4096, iters=6,
                 seed=0, precision="fp64")
    out = {}
    for est in ("residual", "picard"):
        wl = base.with_(estimator=est)
        with hpsmc.Plan(wl) as plan:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.hpsmc_solve()
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            errs = []
            for iv in range(10):
                x, t = plan.hpsmc_grid(iv)
                ex = ((1 - x ** 2) * np.sin(x))[:, None] * (np.exp(np.cos(t)) / (1 + t ** 2))[None, :]
                errs.append(float(np.max(np.abs(plan.hpsmc_get_nodes(iv)[0] - ex))))
        out[est] = {"seconds": sec, "max_error_per_interval": errs, "max_error": max(errs)}
        print(f"[bench] compare {est}: {sec:.2f}s, max error {max(errs):.3e}", file=sys.stderr, flush=True)
    ns = base.nodes_per_sweep * base.M * base.iters
    line = {"metric": METRIC, "value": ns / out["residual"]["seconds"], "unit": "node-samples/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": 1e3 * out["residual"]["seconds"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "1-D long-time problem to T=10 in unit intervals, residual form against the "
                                   "Picard (classical Monte Carlo) form, 16 x 16 nodes per interval, M=4096, "
                                   "6 iterations per interval, FP64"},
            "comparison": out}
    print(json.dumps(line), flush=True)


def flops_per_eval_frac(P, K, fp32):
    """Algorithmic FP operations of one step of the fractional walk: the Newton
    inverse of the incomplete beta (a start interpolated from a table, ~10, then
    one iteration of a 26- or 60-term series at 3 flops a term, plus ~30 for
    the logarithms and the update), the Jacobi recurrence with three
    contractions over P modes (9 flops a mode) and the source series over K
    modes (4 flops a mode), ~40 for w, f and the source."""
    nit, nt = (1, 26) if fp32 else (1, 60)
    return 10 + nit * (3 * nt + 30) + 9 * P + 4 * K + 40


def run_frac(args, torch):
    """Ex. 2's fractional long-time problem: alpha = 0.4, 11 Gauss-Jacobi nodes
    x 6 node times per interval, h = 0.5 to T = 10, M = 8192, 10 iterations per
    interval, whole solve (both precisions on the same Philox words), error
    against the exact solution (1-x^2)^{0.2} sin x e^{cos t}/(1+t^2)."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    res = {}
    stream = torch.cuda.Stream()
    for prec in ("fp64", "fp32"):
        wl = W.frac_long_time(iters=10, precision=prec)
        with hpsmc.Plan(wl) as plan:
            if args.tune_cache:   # tuned on the full sample count: one interval-iteration is small
                plan.hpsmc_tune(0, wl.M, args.tune_cache, stream=stream)
            plan.hpsmc_set_option("graph", 1)
            plan.hpsmc_solve(stream=stream)       # warm-up solve (code loading, graph capture)
            stream.synchronize()
            plan.hpsmc_reset_stats(stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.hpsmc_solve(stream=stream)
            stream.synchronize()
            sec = time.perf_counter() - t0
            st = plan.hpsmc_stats(stream=stream)
            errs = []
            for iv in range(wl.n_intervals):
                x, t = plan.hpsmc_grid(iv)
                ex = ((1 - x ** 2) ** (wl.alpha / 2) * np.sin(x))[:, None] * (np.exp(np.cos(t)) / (1 + t ** 2))[None, :]
                errs.append(float(np.max(np.abs(plan.hpsmc_get_nodes(iv)[0] - ex))))
            launch = plan.hpsmc_get_launch()
            # the round kernel's own launch time, from eager iterations of the
            # first interval (a graph replay records no per-launch events)
            plan.hpsmc_set_option("graph", 0)
            plan.hpsmc_start_interval(0, stream=stream)
            plan.hpsmc_reset_stats(stream=stream)
            for k in range(4):
                plan.hpsmc_iterate(0, k, stream=stream)
            stream.synchronize()
            sk = plan.hpsmc_stats(stream=stream)
        ns = wl.nodes_per_sweep * wl.M * wl.iters
        k_ms = sk["sample_ms"] / max(1, sk["sample_launches"])
        fpe = flops_per_eval_frac(wl.n, 40, prec == "fp32")
        res[prec] = {"seconds": sec, "node_samples_per_s": ns / sec, "max_error": max(errs),
                     "error_per_interval": errs, "path_steps": st["path_steps"],
                     "mean_path_length": st["path_steps"] / max(1, st["node_samples"]),
                     "avg_launch_ms": k_ms,
                     "achieved_tflops": fpe * sk["path_steps"] / max(1, sk["sample_launches"]) / max(1e-9, k_ms * 1e-3) / 1e12,
                     "lane_utilization": st["path_steps"] / max(1, st["lane_steps"]), "launch": list(launch)}
        print(f"[bench] frac {prec}: {sec:.2f}s {ns / sec / 1e6:.2f} M node-samples/s, max error {max(errs):.3e}",
              file=sys.stderr, flush=True)
    r32, r64 = res["fp32"], res["fp64"]
    line = {"metric": METRIC, "value": r32["node_samples_per_s"], "unit": "node-samples/s", "n_gpus": 1, "steps": 1,
            "warmup": 1, "ms_per_step": 1e3 * r32["seconds"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "fractional long-time problem (Ex. 2 shape): alpha = 0.4, 1-D, 11 Gauss-Jacobi "
                                   "nodes x 6 node times per interval, h = 0.5 to T = 10, M = 8192, 10 iterations "
                                   "per interval, whole solve"},
            "roofline": {"bound": "alu", "achieved": r32["achieved_tflops"], "peak": FP32_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": r32["achieved_tflops"] / FP32_PEAK_TFLOPS,
                         "flops_per_eval": flops_per_eval_frac(11, 40, True)},
            "speedup_fp32_vs_fp64": r64["seconds"] / r32["seconds"], "results": res}
    print(json.dumps(line), flush=True)


def run_fraccmp(args, torch):
    """The paper's long-time contrast on its fractional problem (Ex. 2): the
    residual form against the Picard (classical Monte Carlo) form, alpha = 0.4,
    11 x 6 nodes per interval, h = 0.5 to T = 50, M = 8192, 10 iterations per
    interval, FP64, the same walks; error against the exact solution per
    interval, absolute and relative to max |u_ex| on the interval."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    out = {}
    stream = torch.cuda.Stream()
    for est in ("residual", "picard"):
        wl = W.frac_long_time(iters=10, n_intervals=100, precision="fp64", estimator=est)
        with hpsmc.Plan(wl) as plan:
            if args.tune_cache:
                plan.hpsmc_tune(0, wl.M, args.tune_cache, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.hpsmc_solve(stream=stream)
            stream.synchronize()
            sec = time.perf_counter() - t0
            err, rel = [], []
            for iv in range(wl.n_intervals):
                x, t = plan.hpsmc_grid(iv)
                ex = ((1 - x ** 2) ** (wl.alpha / 2) * np.sin(x))[:, None] * (np.exp(np.cos(t)) / (1 + t ** 2))[None, :]
                e = float(np.max(np.abs(plan.hpsmc_get_nodes(iv)[0] - ex)))
                err.append(e)
                rel.append(e / float(np.max(np.abs(ex))))
        out[est] = {"seconds": sec, "max_error": max(err), "final_error": err[-1], "final_relative_error": rel[-1],
                    "error_at_T": {str(T): err[int(2 * T) - 1] for T in (1, 5, 10, 25, 50)},
                    "relative_error_at_T": {str(T): rel[int(2 * T) - 1] for T in (1, 5, 10, 25, 50)}}
        print(f"[bench] fraccmp {est}: {sec:.2f}s, max error {max(err):.3e}, relative error at T=50 {rel[-1]:.3e}",
              file=sys.stderr, flush=True)
    wl = W.frac_long_time(iters=10, n_intervals=100)
    ns = wl.nodes_per_sweep * wl.M * wl.iters
    line = {"metric": METRIC, "value": ns / out["residual"]["seconds"], "unit": "node-samples/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": 1e3 * out["residual"]["seconds"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "fractional long-time problem (Ex. 2 shape) to T = 50: residual form against the "
                                   "Picard (classical Monte Carlo) form, alpha = 0.4, 11 x 6 nodes per interval, "
                                   "h = 0.5, M = 8192, 10 iterations per interval, FP64"},
            "comparison": out}
    print(json.dumps(line), flush=True)


def run_ex1(args, torch):
    """Ex. 1's convergence studies on the GPU (FP64, one interval [0, 0.5], f = u sin u,
    exact solution e^{-t} sin(pi x)): (a) error against n (spatial nodes) with
    M_1 = 6; (b) against M_1 with n = 19; both with M = 4096 and 30 iterations;
    (c) error after K = 1..30 iterations for M = 100, 1000, 10000 (n = 11, M_1 = 6)."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    stream = torch.cuda.Stream()

    def run(n, deg, M, iters):
        wl = W._mk("ex1", 1, n, [0.0, 0.5], [deg], f="u_sin_u", src="sin_decay", ic="exact", M=M, iters=iters,
                   seed=0, precision="fp64")
        with hpsmc.Plan(wl) as plan:
            plan.hpsmc_solve(stream=stream)
            stream.synchronize()
            x, t = plan.hpsmc_grid(0)
            ex = np.sin(np.pi * x)[:, None] * np.exp(-t)[None, :]
            return float(np.max(np.abs(plan.hpsmc_get_nodes(0)[0] - ex)))

    t0 = time.perf_counter()
    res = {"error_vs_n": {}, "error_vs_M1": {}, "error_vs_K": {}}
    for n in (4, 6, 8, 10, 12, 14, 16, 19):
        res["error_vs_n"][str(n)] = run(n, 6, 4096, 30)
    for deg in (2, 3, 4, 5, 6, 8, 10):
        res["error_vs_M1"][str(deg)] = run(19, deg, 4096, 30)
    for M in (100, 1000, 10000):
        res["error_vs_K"][str(M)] = [run(11, 6, M, K) for K in (1, 2, 4, 8, 12, 16, 20, 30)]
    sec = time.perf_counter() - t0
    for k, v in res.items():
        print(f"[bench] ex1 {k}: {v}", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "value": None, "unit": "node-samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "convergence studies of Ex. 1 (1-D, one interval, f = u sin u): error against n, "
                                   "against the temporal degree, and against the iteration count for several M"},
            "results": res}
    print(json.dumps(line), flush=True)


def run_fracexp(args, torch):
    """Accuracy studies of the fractional examples, FP64, M = 8192:
    (a) Ex. 2 to T = 25 with step sizes h = 1, 0.5, 0.2, 0.1 (M_n = 6, 11
        nodes, 10 iterations per interval; at most 255 intervals, the
        counter's interval field): max error over all nodes;
    (b) Ex. 3 (rho = 0.51, T = 0.5): the geometric mesh t_n = T 0.2^{N-n} with
        degrees M_1 = 1, M_n = floor(1.5 n), N = 2..8, against uniform steps
        h = T/N with the same largest degree; 12 iterations per interval."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    stream = torch.cuda.Stream()

    def solve_err(wl, exact):
        with hpsmc.Plan(wl) as plan:
            if args.tune_cache:
                plan.hpsmc_tune(0, min(wl.M, 1024), args.tune_cache, stream=stream)
            t0 = time.perf_counter()
            plan.hpsmc_solve(stream=stream)
            stream.synchronize()
            sec = time.perf_counter() - t0
            err = 0.0
            for iv in range(wl.n_intervals):
                x, t = plan.hpsmc_grid(iv)
                err = max(err, float(np.max(np.abs(plan.hpsmc_get_nodes(iv)[0] - exact(x, t)))))
        return err, sec

    a = wl_alpha = 0.4
    ex2 = lambda x, t: ((1 - x ** 2) ** (a / 2) * np.sin(x))[:, None] * (np.exp(np.cos(t)) / (1 + t ** 2))[None, :]
    ex3 = lambda x, t: ((1 - x ** 2) ** (a / 2) * np.cos(x ** 3 + 1) / (10 * x ** 2 + 1))[:, None] * (t ** 0.51)[None, :]
    res = {"ex2_step_size": {}, "ex3_geometric": {}, "ex3_uniform": {}}
    total = 0.0
    for h in (1.0, 0.5, 0.2, 0.1):
        wl = W.frac_long_time(iters=10, n_intervals=int(round(25 / h)), h=h, alpha=wl_alpha)
        e, sec = solve_err(wl, ex2)
        total += sec
        res["ex2_step_size"][str(h)] = e
        print(f"[bench] fracexp Ex.2 h={h}: max error {e:.3e} ({sec:.1f}s)", file=sys.stderr, flush=True)
    for N in range(2, 9):
        wg = W.frac_singular(iters=12, N=N, T=0.5, alpha=wl_alpha, rho=0.51)
        eg, sec = solve_err(wg, ex3)
        total += sec
        tb = [0.5 * k / N for k in range(N + 1)]
        wu = W._mk("frac_singular_uniform", 1, 11, tb, [max(wg.degree)] * N, f="u_minus_u3", src="frac_singular",
                   src_param=[0.51, 0, 0, 0, 0, 0, 0, 0], ic="exact", M=8192, iters=12, seed=0, precision="fp64",
                   alpha=wl_alpha)
        eu, sec = solve_err(wu, ex3)
        total += sec
        res["ex3_geometric"][str(N)] = eg
        res["ex3_uniform"][str(N)] = eu
        print(f"[bench] fracexp Ex.3 N={N}: geometric {eg:.3e}, uniform {eu:.3e}", file=sys.stderr, flush=True)
    line = {"metric": METRIC, "value": None, "unit": "node-samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * total, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "accuracy studies of the fractional examples (Ex. 2 step sizes to T = 25, Ex. 3 "
                                   "geometric against uniform meshes), FP64, M = 8192"},
            "results": res}
    print(json.dumps(line), flush=True)


def run_ballcmp(args, torch):
    """Centre-point (eq. interIQ) against ball-point path quadrature on the
    single-step problem (1-D, u = e^{-t} sin(pi x), 16 x 16 nodes, M = 4096,
    FP64, fresh samples): error against the exact solution after K = 1..8
    iterations, time of the whole 8-iteration solve."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    out = {}
    for quad in ("centre", "ball"):
        errs, secs = [], 0.0
        for k in range(1, 9):
            wl = W.c1_single_step(iters=k).with_(quad=quad)
            with hpsmc.Plan(wl) as plan:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan.hpsmc_solve()
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
                x, t = plan.hpsmc_grid(0)
                ex = np.sin(np.pi * x)[:, None] * np.exp(-t)[None, :]
                errs.append(float(np.max(np.abs(plan.hpsmc_get_nodes(0)[0] - ex))))
        out[quad] = {"error_after_k": errs, "seconds_8_iterations": secs}
        print(f"[bench] ballcmp {quad}: {secs:.2f}s for 8 iterations, errors "
              f"{', '.join(f'{e:.2e}' for e in errs)}", file=sys.stderr, flush=True)
    wl = W.c1_single_step(iters=8)
    line = {"metric": METRIC, "value": wl.nodes_per_sweep * wl.M * 8 / out["ball"]["seconds_8_iterations"],
            "unit": "node-samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": 1e3 * out["ball"]["seconds_8_iterations"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "c1_1d_single_step, 8 iterations, ball-point against centre-point path "
                                   "quadrature, fresh samples"},
            "comparison": out}
    print(json.dumps(line), flush=True)


def run_aitken(args, torch):
    """What the Aitken relaxation (the remark after Algorithm 1) buys on the
    single-step problem (1-D, u = e^{-t} sin(pi x), 16 x 16 nodes, M = 4096,
    FP64): (a) common random numbers, so the iteration map is deterministic:
    iterations until max|eps| < 1e-10; (b) fresh samples each iteration (the
    paper's setting): error against the exact solution after each iteration
    count 1..8."""
    from paper_2608_22190_amd import hpsmc, workloads as W
    out = {}
    for accel in ("none", "aitken"):
        wl = W.c1_single_step(iters=60).with_(fresh_per_iter=False, tol=1e-10, accel=accel)
        with hpsmc.Plan(wl) as plan:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            status = plan.hpsmc_solve()
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            st = plan.hpsmc_stats()
        hist = list(st["max_eps"][:st["n_records"]])
        errs = []
        for k in range(1, 9):
            wlf = W.c1_single_step(iters=k).with_(accel=accel)
            with hpsmc.Plan(wlf) as plan:
                plan.hpsmc_solve()
                x, t = plan.hpsmc_grid(0)
                ex = np.sin(np.pi * x)[:, None] * np.exp(-t)[None, :]
                errs.append(float(np.max(np.abs(plan.hpsmc_get_nodes(0)[0] - ex))))
        out[accel] = {"crn_iterations_to_1e-10": len(hist), "crn_status": int(status), "crn_seconds": sec,
                      "crn_max_eps": hist, "fresh_error_after_k": errs}
        print(f"[bench] aitken {accel}: {len(hist)} iterations to 1e-10 ({sec:.2f}s), fresh errors "
              f"{', '.join(f'{e:.2e}' for e in errs)}", file=sys.stderr, flush=True)
    wl = W.c1_single_step()
    ns = wl.nodes_per_sweep * wl.M * out["aitken"]["crn_iterations_to_1e-10"]
    line = {"metric": METRIC, "value": ns / out["aitken"]["crn_seconds"], "unit": "node-samples/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": 1e3 * out["aitken"]["crn_seconds"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "c1_1d_single_step with common random numbers, solved to max|eps| < 1e-10, "
                                   "Aitken-relaxed against plain iteration; then fresh samples, K = 1..8"},
            "iterations_saved": 1 - out["aitken"]["crn_iterations_to_1e-10"] / out["none"]["crn_iterations_to_1e-10"],
            "comparison": out}
    print(json.dumps(line), flush=True)


def cpu_baseline(wl, budget_s=20.0):
    """The FP64 oracle on a bounded sample: random nodes of the same interval,
    the first samples of each, one residual iteration from the same iterate."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle as O
    pb = O.Problem(wl)
    rng = np.random.default_rng(123)
    nn = wl.nsp * wl.degree[0]
    U0 = np.repeat(pb.ic_nodes()[:, None], wl.degree[0] + 1, axis=1).reshape(-1)
    done, t_used, nodes_used = 0, 0.0, 0
    m = 2
    while t_used < budget_s:
        nodes = rng.choice(nn, size=O.num_threads(), replace=False)
        t0 = time.perf_counter()
        pb.estimate(U0, nodes=nodes, m_lo=0, m_hi=m)
        t_used += time.perf_counter() - t0
        done += len(nodes) * m
        nodes_used += len(nodes)
        if t_used < 1.0:
            m *= 2
    return {"value": done / t_used, "unit": "node-samples/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{nodes_used} random nodes of interval 1 x first samples ({done} node-samples, "
                      f"one residual iteration from the replicated initial data), {t_used:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m-slice", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-switch", action="store_true", help="skip the solve with the FP32 -> FP64 switch")
    ap.add_argument("--workload", type=str, default="c2", choices=["c1", "c2", "c2p", "c2b", "c3", "c4", "c5", "compare", "aitken",
                                                              "ballcmp", "frac", "fraccmp", "fracexp", "ex1"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain device copy of 512 MiB (calibrates HBM byte counters)")
    ap.add_argument("--launch", type=str, default="",
                    help="samples_per_lane,waves_per_block,blocks_per_cu,round_steps (skips the tuner)")
    ap.add_argument("--tune-cache", type=str, default=os.path.join(ROOT, "paper_2608_22190_amd", "tuned_launch.json"),
                    help="autotuner cache (looked up; tuned and written when the entry is missing)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (one process, one device).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_22190_amd import hpsmc, workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "c2":
        run_other(args.workload, args, torch)
        return

    base = W.c2_long_time(M=args.m_slice, iters=args.steps, n_intervals=1)
    P = base.n + 2
    nodes = base.nsp * base.degree[0]
    exact_fn = (lambda grid: long_time_exact(base, grid))
    r32 = run_gpu(base.with_(precision="fp32"), args.steps, args.warmup, launch, torch, args.tune_cache,
                  exact_fn=exact_fn)
    ns_step = nodes * base.M
    value = ns_step * args.steps / r32["seconds"]
    st = r32["stats"]
    fpe = flops_per_eval(base.dim, P)
    k_ms = st["sample_ms"] / max(1, st["sample_launches"])
    evals_per_launch = st["path_steps"] / max(1, st["advance_launches"])
    achieved = fpe * evals_per_launch / (k_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "node-samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * r32["seconds"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c2_2d_long_time interval 1 (t in [0,1]), one residual iteration per step, "
                               f"all {nodes} nodes (24x24 JG(1,1) x 16 LGL times) x samples 0..{base.M - 1} "
                               f"of M=65536; FP32 sampling, FP64 reconstruction/update",
                   "dim": 2, "n": 24, "temporal_degree": 16, "nodes": nodes, "samples_per_node": base.M,
                   "max_nstar": int(hpsmc.resolve_nstar(base)[0].max()), "launch": list(r32["launch"])},
        "roofline": {"bound": "mfma" if r32["mma"] else "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": measured_traffic(r32["launch"]),
                     "kernel": (f"advance_mma_kernel<{(P + 1) // 2},0> (v_mfma_f32_32x32x2f32)"
                                if r32["mma"] else "advance_kernel<float,2,28,NS,0,0> (vector units)"),
                     "flops_per_eval": fpe,
                     "evals_per_launch": evals_per_launch, "avg_launch_ms": k_ms,
                     "lane_utilization": st["path_steps"] / max(1, st["lane_steps"])},
        "path_steps_per_s": st["path_steps"] / r32["seconds"],
        "mean_path_length": st["path_steps"] / max(1, st["node_samples"]),
        "reconstruction_ms_per_step": st["recon_ms"] / max(1, st["recon_launches"]),
        "slab_ms_per_step": st["slab_ms"] / args.steps,
        "sampling_span_ms_per_step": st["sampling_span_ms"] / args.steps,
        "advance_launches_per_step": st["advance_launches"] / args.steps,
    }
    if args.no_fp64:
        # FP32 alone: its error against the exact solution after every timed iteration
        t32 = r32["trajectory"]
        out["accuracy"] = {
            "e32_vs_exact": t32[-1][1], "max_node_std_error_fp32": t32[-1][2],
            "trajectory_fp32": [[round(t, 4), e, s_, m] for t, e, s_, m in t32],
            "note": "rows: [seconds so far, max error against the exact solution, max node standard error, "
                    "max|eps|] after each timed iteration from the replicated initial data"}
    else:
        r64 = run_gpu(base.with_(precision="fp64"), args.steps, args.warmup, launch, torch, args.tune_cache,
                      exact_fn=exact_fn)
        v64 = ns_step * args.steps / r64["seconds"]
        s64 = r64["stats"]
        k64 = s64["sample_ms"] / max(1, s64["sample_launches"])
        a64 = fpe * s64["path_steps"] / max(1, s64["advance_launches"]) / (k64 * 1e-3) / 1e12
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["seconds"] / args.steps,
                       "roofline_achieved_tflops": a64, "roofline_frac": a64 / FP64_PEAK_TFLOPS}
        out["fp32_over_fp64_rate_ratio"] = value / v64
        ex = long_time_exact(base, r64["grid"])
        t32, t64 = r32["trajectory"], r64["trajectory"]
        # time to a given error against the exact solution, each precision from the replicated
        # initial data on the same Philox words; the speedup at equal accuracy is quoted at the
        # tightest decade both precisions reach
        tte = {}
        for j in range(1, 13):
            target = 10.0 ** -j
            a, b = time_to_error(t32, target), time_to_error(t64, target)
            tte[f"1e-{j}"] = {"fp32_s": a, "fp64_s": b, "speedup": (b / a) if a and b else None}
        common = [k for k, v in tte.items() if v["speedup"] is not None]
        e32, e64, sig = t32[-1][1], t64[-1][1], t64[-1][2]
        out["fp32_over_fp64_speedup"] = tte[common[-1]]["speedup"] if common else None
        out["accuracy"] = {
            "equal_accuracy_target": common[-1] if common else None,
            "time_to_error": tte,
            "e32_vs_exact": e32, "e64_vs_exact": e64, "max_node_std_error_fp64": sig,
            "max_abs_u32_minus_u64": float(np.max(np.abs(r32["U"] - r64["U"]))),
            "r24_pass": bool(e32 <= e64 + 3 * sig),
            "trajectory_fp32": [[round(t, 4), e, s_, m] for t, e, s_, m in t32],
            "trajectory_fp64": [[round(t, 4), e, s_, m] for t, e, s_, m in t64],
            "note": "rows: [seconds so far, max error against the exact solution, max node standard error, "
                    "max|eps|] after each timed iteration from the replicated initial data; same Philox words in "
                    "both precisions.  FP32 sampling levels off at its rounding floor, so the speedup at equal "
                    "accuracy is quoted at the tightest error both reach; r24_pass is reading R24 after the last "
                    "iteration (e32 <= e64 + 3 sigma)"}
        if not args.no_switch:
            # Algorithm 1's loop condition at the paper's long-time tolerance: FP64 alone (its
            # trajectory), and FP32 sampling that hands over to FP64 once max|eps| < switch_tol
            tol, sw = 1e-10, 1e-6
            rs = run_switched_solve(base.with_(iters=max(args.steps, 30)), tol, sw, torch, args.tune_cache)
            es = float(np.max(np.abs(rs["U"] - long_time_exact(base, rs["grid"]))))
            t64_tol = time_to_error(t64, tol, col=3)
            f64 = {"seconds": t64_tol, "iterations": next((k + 1 for k, r in enumerate(t64) if r[3] < tol), None),
                   "error_vs_exact": next((r[1] for r in t64 if r[3] < tol), None), "max_node_std_error": sig}
            if t64_tol is None:
                # the timed FP64 iterations stopped short of the tolerance: FP64 alone to it
                r64t = run_switched_solve(base.with_(iters=max(args.steps, 30)), tol, None, torch, args.tune_cache)
                f64 = {"seconds": r64t["seconds"], "iterations": r64t["iterations"],
                       "error_vs_exact": float(np.max(np.abs(r64t["U"] - long_time_exact(base, r64t["grid"])))),
                       "max_node_std_error": r64t["sigma"]}
            sp = f64["seconds"] / rs["seconds"] if f64["seconds"] else None
            r24 = bool(es <= f64["error_vs_exact"] + 3 * f64["max_node_std_error"]) if f64["seconds"] else None
            out["accuracy"]["to_tolerance"] = {
                "tol": tol, "switch_tol": sw, "fp64": f64,
                "fp32": {"reached": time_to_error(t32, tol, col=3) is not None, "min_max_eps": min(r[3] for r in t32)},
                "fp32_then_fp64": {"seconds": rs["seconds"], "iterations": rs["iterations"],
                                   "fp32_iterations": rs["fp32_iterations"], "status": rs["status"],
                                   "error_vs_exact": es, "max_node_std_error": rs["sigma"],
                                   "r24_pass_vs_fp64": r24},
                "speedup_vs_fp64": sp}
            if sp is not None and r24:
                # the headline: FP32-batched sampling (switching to FP64 for the last digits) against
                # FP64, both solved to Algorithm 1's tolerance, at equal accuracy (R24 holds)
                out["fp32_over_fp64_speedup"] = sp
                out["accuracy"]["speedup_basis"] = (f"time to max|eps| < {tol:g} (Algorithm 1's loop condition): FP32 "
                                                    f"sampling until max|eps| < {sw:g}, then FP64, against FP64 alone; "
                                                    "errors against the exact solution within R24")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(base.with_(precision="fp64"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
