"""Benchmark of the implicit SPH radiation-diffusion hot path on one MI355X.

One step = the whole path on one synthetic batch, inputs resident in HBM:
neighbour lists (cell sort + search), per-step frozen data and CSR assembly
with the aggregation-AMG set-up, then the outer iterations of the
nonlinear-elimination loop (right-hand side, diffusion solve warm-started
from E^l, per-particle material Newton, convergence measures).

Default workload: the 3-D Marshak-like front on 256^3 = 16,777,216 particles
from greedy dart throwing (~58 neighbours), one time step dt = 1e-3 with
exactly five outer iterations, FP32 inner PCG with FP64 iterative refinement
to ||r||/||b|| <= 1e-10.  value = particle-updates/s = interior particles x
outer iterations / wall time per step.  The plain-FP64 solve of the same
systems is timed afterwards for the mixed-vs-FP64 ratio; the SpMV roofline
uses HIP events recorded around every SpMV launch on the library's stream.
The CPU baseline times the oracle on a smaller instance of the same recipe.

Other workloads (--workload): densitystep3d and wendland3d (one step of the
same path on those recipes), ensemble (a batch of independent problems), and
coswave3d / coswave2d (the manufactured problem of Sec. 4.3, time stepped
with per-step sources; --steps 1000 runs one full cycle).
"""
from __future__ import annotations

import argparse
import contextlib
import gc
from concurrent.futures import ThreadPoolExecutor
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# The timed solve: Jacobi-preconditioned CG, stopped when ||b - A x|| <= 1e-10
# ||b|| and max_i |b - A x|_i / (a_ii |x_i|) <= 1e-10 (every particle's E to
# about 1e-10 relative, also far ahead of the front); mixed precision asks each
# FP32 inner solve for a reduction of 1e-4.  Five outer iterations per step.
BENCH_TOL = 1e-10
BENCH_CW_TOL = 1e-10
BENCH_INNER_TOL = 1e-4
BENCH_OUTER = 5


def bench_solve_opts(precision, precond=0, tol=BENCH_TOL, cw_tol=BENCH_CW_TOL,
                     inner_tol=BENCH_INNER_TOL):
    from paper_2001_11606_amd import rt
    return rt.solve_opts(precision, precond, tol, 5000, inner_tol, 30, cw_tol)


METRIC = "diffusion solve particle-updates/s + SpMV HBM GB/s; mixed vs FP64 @1e-10"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_problem(workload: str, n: int):
    import synth
    if workload == "marshak3d":
        return synth.config4(n=n)
    if workload == "densitystep3d":
        return synth.config3(n=n)
    if workload == "wendland3d":
        return synth.wendland_lattice(3, n)
    raise SystemExit(f"unknown workload {workload}")


@contextlib.contextmanager
def paused_gc():
    """The interpreter's cyclic garbage collector off while steps are timed,
    after one collection: a full pass over the problem generators' objects
    once stalled the host for about 50 ms between two library calls."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def run_step(ctx, dp, solve, outer, amg, shapes=None):
    """One pass of the whole hot path; returns (e, E, A, report, nb)."""
    from paper_2001_11606_amd import driver
    nb = ctx.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
    e, E, A, rep = driver.time_step(ctx, dp, nb, amg=amg, solve=solve, fixed_outer=outer,
                                    shapes=shapes)
    return e, E, A, rep, nb


def release(ctx, nb, A):
    from paper_2001_11606_amd import rt
    rt.rt_matrix_free(A)
    rt.rt_neighbors_free(nb.handle)
    ctx._owned = [o for o in ctx._owned if o[1] not in (A, nb.handle)]


def spmv_bytes(vbytes: int, nnz_off: int, n: int, tile_cols: int) -> float:
    """Algorithmic bytes of one Krylov-loop product y = A x (values in vbytes
    bytes): off-diagonal values and column indices (16-bit tile-local ones
    plus the tiles' 32-bit column lists when tiled, else 32-bit), the row
    pointers (8 B), diagonal, x read once and y written once."""
    if tile_cols:
        idx = 2.0 * nnz_off + 4.0 * tile_cols
    else:
        idx = 4.0 * nnz_off
    return vbytes * nnz_off + idx + 8.0 * (n + 1) + 3.0 * vbytes * n


def resid_bytes(nnz_off: int, n: int, tile_cols: int, with_w32: bool) -> float:
    """Algorithmic bytes of one FP64 residual product r = b - A x of the
    refinement loop: FP64 values and 16-bit tile-local columns (or 32-bit
    columns untiled) per off-diagonal entry, the tiles' column lists, row
    pointers, and per row the diagonal, x and b read, r written in FP64 and
    in FP32 (the inner solve's right-hand side), and the FP32 weights of the
    componentwise test when it is on."""
    idx = (2.0 * nnz_off + 4.0 * tile_cols) if tile_cols else 4.0 * nnz_off
    per_row = 8.0 * 4 + 4.0 + (4.0 if with_w32 else 0.0)
    return 8.0 * nnz_off + idx + 8.0 * (n + 1) + per_row * n


COUNTERS = os.path.join(ROOT, "profiles", "k_spmv_tiled_marshak3d_16.8M_counters.md")


def profiled_traffic(workload: str, n: int, kernel: str):
    """HBM bytes per launch of a product kernel (FETCH_SIZE and WRITE_SIZE,
    each scaled by its reading for a plain copy of known size) from the
    committed counter summary -- only for the workload it was taken on, a
    kernel instance it lists, and while the kernel source is unchanged (hash);
    else None."""
    import hashlib
    if workload != "marshak3d" or n != 256 or not os.path.exists(COUNTERS):
        return None
    sha, traffic = None, {}
    for line in open(COUNTERS):
        line = line.strip()
        if line.startswith("spmv_source_sha256: "):
            sha = line.split(": ", 1)[1]
        elif line.startswith("traffic ") and ": " in line:
            name, _, v = line[len("traffic "):].rpartition(": ")
            traffic[name] = float(v)
    src = os.path.join(ROOT, "paper_2001_11606_amd", "csrc", "spmv.h")
    if sha != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return traffic.get(kernel)


def copy_bandwidth(nbytes: int = 2 << 30, reps: int = 5) -> float:
    """Device-to-device stream copy rate (GB/s, read + write bytes) of a plain
    elementwise kernel over nbytes; the same launch serves as the known-size
    reference when HBM counters are read under a profiler."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    ev1.record()
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1e3 / reps
    del src, dst
    return 2.0 * nbytes / sec / 1e9


def host_cpu():
    """(logical CPUs this process may run on, CPU model name)."""
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return ncpu, model


def cpu_baseline(workload: str, n_sample: int, outer: int, tol: float, cw_tol: float):
    """The oracle (plain FP64 numpy/scipy) on a smaller instance of the recipe,
    its linear solves to the bench's tolerances: once with BLAS/OpenMP pools
    held to one thread, once with every pool free to use all host CPUs.  The
    all-CPU leg's `cores` is what it used: process CPU time over wall time
    (numpy's element-wise and scipy's sparse kernels run on one thread, so it
    stays near one)."""
    from threadpoolctl import threadpool_limits
    from oracle import linsolve, step as ostep
    solver = lambda A, b, x0: linsolve.solve(A, b, x0, max(tol, cw_tol))
    legs = {}
    for name, limit in (("one_core", 1), ("all_cores", None)):
        prob = make_problem(workload, n_sample)
        with threadpool_limits(limits=limit):
            c0, t0 = time.process_time(), time.perf_counter()
            ostep.time_step(prob, fixed_outer=outer, solver=solver)
            wall = time.perf_counter() - t0
            cpu = time.process_time() - c0
        legs[name] = (prob.n_interior * outer / wall, wall, cpu / wall)
    ncpu, model = host_cpu()
    best = max(legs, key=lambda k: legs[k][0])
    v, wall, used = legs[best]
    return {"value": v, "unit": "particle-updates/s",
            "cores": 1 if best == "one_core" else max(1, round(used, 1)),
            "kind": "oracle",
            "sample": f"{workload} recipe at n={n_sample} ({prob.n_interior} interior particles), "
                      f"one time step with {outer} outer iterations, {wall:.1f} s",
            "legs": {k: {"value": round(lv[0], 1), "wall_s": round(lv[1], 2),
                         "cpu_time_over_wall": round(lv[2], 2)} for k, lv in legs.items()},
            "host_cpus": ncpu, "cpu_model": model}


def ensemble_vcycle_leg(ctx, dps, ntot, args):
    """The batched V-cycle on the ensemble: every problem assembled with its
    own aggregation hierarchy, the batch concatenating them level by level;
    mixed solves of b = 1 with the V-cycle (iterations launched one by one,
    and replayed from graphs) against Jacobi (graphs) on that batch, and
    with the V-cycle on a batch whose problems each take the depth the
    depth tuner chose on their own solve, and at the depth the batch's own
    tuner keeps; outside the timed steps."""
    import torch
    from paper_2001_11606_amd import rt
    amg = rt.amg_opts(build_fp32=1)
    built = []
    for dp in dps:
        nb = ctx.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
        A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=amg)
        built.append((nb, A))
    levels = [ctx.matrix_info(A).levels for _, A in built]
    opts = rt.solve_opts(rt.RT_PREC_MIXED, 1, args.tol, 5000, args.inner_tol, 30)
    B = rt.rt_batch_create(ctx.handle, [A for _, A in built])
    # each problem's depth tuned on its own solve of b = 1, then a second
    # batch built from the tuned matrices
    depths = []
    for (nb, A), dp in zip(built, dps):
        bq = torch.ones(dp.n_interior, dtype=torch.float64, device=ctx.device)
        depths.append(ctx.tune_depth(A, bq, torch.zeros_like(bq), opts, 2).chosen)
    BT = rt.rt_batch_create(ctx.handle, [A for _, A in built])
    ctx.free(*[h for nb, A in built for h in (A, nb)])
    for b_ in (B, BT):
        rep = rt.rt_batch_tune(ctx.handle, b_, 3)
        rt.rt_batch_set_spmv_shape(b_, rt.RT_PREC_FP64, rep.chosen[0][0])
        rt.rt_batch_set_spmv_shape(b_, rt.RT_PREC_MIXED, rep.chosen[0][1])
        rt.rt_batch_set_spmv_shape(b_, rt.RT_PRODUCT_RESIDUAL, rep.chosen[0][2])
    res = {}
    runs = ((B, 1, 0), (B, 1, args.graph_iters), (B, 0, args.graph_iters), (BT, 1, 0))
    for b_, precond, graph in runs + runs:   # the second round is timed
        bt = torch.ones(ntot, dtype=torch.float64, device=ctx.device)
        xt = torch.zeros_like(bt)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        s, sst = rt.rt_batch_solve(ctx.handle, b_, len(dps), bt.data_ptr(), xt.data_ptr(),
                                   rt.solve_opts(rt.RT_PREC_MIXED, precond, args.tol, 5000,
                                                 args.inner_tol, 30), graph)
        torch.cuda.synchronize()
        if s != rt.RT_OK:
            raise RuntimeError(f"ensemble V-cycle leg: status {s}")
        res[(b_, precond, graph)] = (time.perf_counter() - ta,
                                     max(sst[q].iterations for q in range(len(dps))))
    # the depth timed inside the batch
    bt = torch.ones(ntot, dtype=torch.float64, device=ctx.device)
    rep = rt.rt_batch_tune_depth(ctx.handle, B, bt.data_ptr(), torch.zeros_like(bt).data_ptr(),
                                 opts, 0, 1)
    for k in range(2):   # the second run is timed
        xt = torch.zeros_like(bt)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        s, sst = rt.rt_batch_solve(ctx.handle, B, len(dps), bt.data_ptr(), xt.data_ptr(), opts, 0)
        torch.cuda.synchronize()
        if s != rt.RT_OK:
            raise RuntimeError(f"ensemble V-cycle leg: status {s}")
    vb = (time.perf_counter() - ta, max(sst[q].iterations for q in range(len(dps))))
    rt.rt_batch_free(B)
    rt.rt_batch_free(BT)
    v0, vg, jg, vt = (res[k] for k in runs)
    hist = {d: depths.count(d) for d in sorted(set(depths))}
    return {"levels_min": min(levels), "levels_max": max(levels),
            "solve_s_vcycle": round(v0[0], 5), "solve_s_vcycle_graph": round(vg[0], 5),
            "solve_s_jacobi": round(jg[0], 5), "graph_iters": args.graph_iters,
            "solve_s_vcycle_tuned_depths": round(vt[0], 5),
            "tuned_depth_counts": {str(d): c for d, c in hist.items()},
            "krylov_max_vcycle": v0[1], "krylov_max_jacobi": jg[1],
            "krylov_max_vcycle_tuned_depths": vt[1],
            "batch_depth_ms": [round(1e3 * rep.seconds[d], 2) for d in range(rep.depths)],
            "batch_depth_chosen": rep.chosen, "solve_s_vcycle_batch_depth": round(vb[0], 5),
            "krylov_max_vcycle_batch_depth": vb[1],
            "ratio_jacobi_over_vcycle": round(jg[0] / min(v0[0], vg[0], vt[0], vb[0]), 3)}


def run_ensemble(args):
    """The ensemble workload: 96 independent problems (2-D / 3-D, log-uniform
    sizes 8k-500k, about 1.1e7 particles), one step = per-problem neighbour
    lists and assembly, the block-diagonal batch, and one batched outer
    iteration of Algorithm 1 (initial material solve, right-hand side, mixed
    solve to the tolerance, material update) for every problem at once."""
    import torch
    import synth
    from paper_2001_11606_amd import driver, rt
    t0 = time.perf_counter()
    probs = synth.config5(args.nprob, args.scale)
    nin = [pr.n_interior for pr in probs]
    ntot = int(sum(nin))
    log(f"[bench] ensemble of {len(probs)} problems, {ntot} particles, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    ctx = rt.Context(0)
    dps = [driver.upload(pr, ctx.device) for pr in probs]
    amg = rt.amg_opts(max_levels=1, build_fp32=1)
    e0 = torch.cat([dp.arrays["e"][:dp.n_interior] for dp in dps])
    E0 = torch.cat([dp.arrays["E"][:dp.n_interior] for dp in dps])
    torch.cuda.synchronize()
    tuned = None
    # The per-problem neighbour lists and matrices are independent: they are
    # built by a few host threads, each with its own context on its own
    # stream, so that one problem's host round trips overlap another's kernels.
    nthreads = max(1, args.build_streams)
    wctx = []
    for _ in range(nthreads):
        with torch.cuda.stream(torch.cuda.Stream()):
            wctx.append(rt.Context(0))
    order = sorted(range(len(dps)), key=lambda q: -dps[q].n_interior)
    parts = [order[w::nthreads] for w in range(nthreads)]

    def build_part(w):
        c = wctx[w]
        out = []
        for q in parts[w]:
            dp = dps[q]
            nb = c.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
            A = c.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                           dp.limiter_k, amg=amg)
            out.append((q, nb, A))
        return out

    def step(precision, keep=False):
        nonlocal tuned
        built = [None] * len(dps)
        with ThreadPoolExecutor(nthreads) as pool:
            for part in pool.map(build_part, range(nthreads)):
                for q, nb, A in part:
                    built[q] = (nb, A)
        torch.cuda.synchronize()   # every worker stream has finished
        nbs = [nb for nb, _ in built]
        mats = [A for _, A in built]
        B = rt.rt_batch_create(ctx.handle, mats)
        if tuned is None:   # tuned on the first batch (warm-up), outside the timed steps
            tuned = rt.rt_batch_tune(ctx.handle, B, 5)
        rt.rt_batch_set_spmv_shape(B, rt.RT_PREC_FP64, tuned.chosen[0][0])
        rt.rt_batch_set_spmv_shape(B, rt.RT_PREC_MIXED, tuned.chosen[0][1])
        rt.rt_batch_set_spmv_shape(B, rt.RT_PRODUCT_RESIDUAL, tuned.chosen[0][2])
        e, E = e0.clone(), E0.clone()
        nopts = rt.newton_opts(rt.solve_opts(precision, 0, args.tol, 5000, args.inner_tol, 30))
        s, st = rt.rt_batch_newton_step(ctx.handle, B, len(probs), e.data_ptr(), E.data_ptr(), 0,
                                        nopts, args.graph_iters)
        torch.cuda.synchronize()
        for A, nb in zip(mats, nbs):
            rt.rt_matrix_free(A)
            rt.rt_neighbors_free(nb.handle)
        for c in wctx:
            c._owned.clear()
        if keep:
            return e, E, st, B
        rt.rt_batch_free(B)
        return e, E, st, None

    for w in range(max(1, args.warmup)):
        log(f"[bench] warmup step {w}")
        step(rt.RT_PREC_MIXED)
    with paused_gc():
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            e, E, st, _ = step(rt.RT_PREC_MIXED)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t1) / args.steps
    value = ntot / (ms * 1e-3)
    # batched solve alone, mixed vs FP64, on one kept batch
    e, E, st, B = step(rt.RT_PREC_MIXED, keep=True)
    rows, nnz, tcols = rt.rt_batch_get_info(B)
    solve_t = {}
    for prec in (rt.RT_PREC_MIXED, rt.RT_PREC_FP64):
        bt = torch.ones(ntot, dtype=torch.float64, device=ctx.device)
        xt = torch.zeros_like(bt)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        s, sst = rt.rt_batch_solve(ctx.handle, B, len(probs), bt.data_ptr(), xt.data_ptr(),
                                   rt.solve_opts(prec, 0, args.tol, 5000, args.inner_tol, 30),
                                   args.graph_iters)
        torch.cuda.synchronize()
        solve_t[prec] = time.perf_counter() - ta
    rt.rt_batch_free(B)
    vleg = None if args.no_vcycle else ensemble_vcycle_leg(ctx, dps, ntot, args)
    sh = tuned.chosen[0][1]
    shapes = rt.rt_spmv_shapes()
    us32 = tuned.us[0][1][sh]
    bytes32 = spmv_bytes(4, nnz, rows, tcols if shapes[sh][2] else 0)
    achieved = bytes32 / (us32 * 1e-6) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"ensemble of {len(probs)} problems ({ntot} particles), one outer "
                               f"iteration each, batched mixed FP32/FP64 to {args.tol:g}",
                   "particles": ntot, "rows_padded": rows, "nnz": nnz},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"batched SpMV shape {shapes[sh]} (tuner timing)",
                     "bytes_per_launch": bytes32, "avg_launch_us": round(us32, 2)},
        "cpu_baseline": None,
        "mixed_vs_fp64": {"solve_s_mixed": round(solve_t[rt.RT_PREC_MIXED], 5),
                          "solve_s_fp64": round(solve_t[rt.RT_PREC_FP64], 5),
                          "ratio_fp64_over_mixed": round(solve_t[rt.RT_PREC_FP64] /
                                                         solve_t[rt.RT_PREC_MIXED], 3)},
        "krylov_max": max(s.solve.iterations for s in st),
    }
    if vleg is not None:
        out["vcycle"] = vleg
    out["config"]["build_threads"] = nthreads
    print(json.dumps(out), flush=True)
    for c in wctx:
        c.close()
    ctx.close()


def run_coswave(args):
    """The manufactured problem of Sec. 4.3 in 3-D (coswave3d) or 2-D
    (coswave2d): periodic box, Wendland kernel at h = 4 spacings (a few
    hundred neighbours per row in 3-D, about 50 in 2-D), time
    stepped as the paper runs it: dt = t_end/1000, outer iterations to 1e-8,
    FP64 radiation solves to 1e-12 (CG, --precond 0 Jacobi or 1 the
    aggregation V-cycle), sources
    evaluated on the device before every step.  Warm-up steps run first on
    their own copy of the state; the timed region is --steps consecutive steps
    from t = 0 (--steps 1000 is the whole cycle, then the energy drift and the
    L1 errors against the manufactured solution are reported as well).
    value = particles x steps / wall time."""
    import numpy as np
    import torch
    import synth
    from paper_2001_11606_amd import driver, rt
    ctx = rt.Context(0)
    dim = 3 if args.workload == "coswave3d" else 2
    log(f"[bench] generating {args.workload} n={args.n}")
    prob = synth.cos_wave_mms(dim, args.n)
    pos = torch.as_tensor(prob.pos, dtype=torch.float64, device=ctx.device)
    src = synth.CosWaveSources(pos, prob.meta["consts"], xp=torch)
    sources = lambda t: src(t)[2:]
    prec = rt.RT_PREC_MIXED if args.mixed else rt.RT_PREC_FP64
    solve = rt.solve_opts(prec, args.precond, 1e-12, 2000, args.inner_tol, 50)
    # Jacobi needs no coarse levels (the hierarchy is then not built per
    # step), and FP64 solves need no FP32 copy of the matrix
    amg = rt.amg_opts(max_levels=1 if args.precond == 0 else 8, build_fp32=int(args.mixed))
    kw = dict(sources=sources, solve=solve, amg=amg, eps_e=1e-8, eps_E=1e-8, material_tol=1e-12)
    if args.warmup > 0:
        dpw = driver.upload(prob, ctx.device)
        driver.run_fixed(ctx, dpw, prob.dt, args.warmup, **kw)
        del dpw
    dp = driver.upload(prob, ctx.device)
    nin = prob.n_interior
    V = prob.m / prob.rho
    start = float(np.sum(prob.m * prob.e) + np.sum(V * prob.E))
    done = [0]

    def progress(t, e, E):
        done[0] += 1
        if done[0] % 100 == 0:
            log(f"[bench] step {done[0]} t={t:.3e}")

    with paused_gc():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t, reps = driver.run_fixed(ctx, dp, prob.dt, args.steps, callback=progress, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    log(f"[bench] {args.steps} steps in {wall:.2f} s")
    out = {
        "metric": "particle-updates/s", "value": nin * args.steps / wall,
        "unit": "particle-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if args.mixed else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload} {args.n}^{dim} ({nin} particles, periodic), Sec. 4.3 "
                               f"manufactured problem, dt = t_end/{prob.meta['steps']}, outer "
                               f"tolerance 1e-8, {'mixed FP32/FP64' if args.mixed else 'FP64'} "
                               f"CG + {('Jacobi', 'AMG')[args.precond]} to 1e-12",
                   "particles": nin, "precond": ("jacobi", "amg")[args.precond]},
        "outer_per_step": float(np.mean([r.outer for r in reps])),
        "krylov_per_outer": float(np.mean([k for r in reps for k in r.krylov])),
        "projected_cycle_s": wall / args.steps * prob.meta["steps"],
    }
    if args.steps == prob.meta["steps"]:
        e = dp.arrays["e"].cpu().numpy()
        E = dp.arrays["E"].cpu().numpy()
        em, Em, _, _ = prob.mms(t)
        out["energy_drift"] = abs(float(np.sum(prob.m * e) + np.sum(V * E)) - start) / start
        out["l1_e"] = float(np.sum(np.abs(e - em)) / np.sum(em))
        out["l1_E"] = float(np.sum(np.abs(E - Em)) / np.sum(Em))
    print(json.dumps(out), flush=True)
    ctx.close()


def run_config2(args):
    """The 3-D manufactured problem of the 64^3 configuration: ten time steps
    of inexact Newton with nonlinear elimination (outer iterations until both
    relative changes are below 1e-8), every diffusion solve AMG-preconditioned
    CG in FP64 to 1e-10 (normwise and componentwise), sources and ghost values
    of the manufactured solution loaded before every step.  The neighbour
    lists are built once (the particles do not move); every step re-assembles
    the matrix and its hierarchy.  value = interior particles x outer
    iterations / wall time of the ten steps."""
    import numpy as np
    import torch
    import synth
    from paper_2001_11606_amd import driver, rt
    ctx = rt.Context(0)
    prob = synth.config2_mms(n=args.n)
    nin = prob.n_interior
    precond = args.precond
    amg = rt.amg_opts(max_levels=8 if precond == 1 else 1, build_fp32=0)
    solve = rt.solve_opts(0, precond, args.tol, 5000, args.inner_tol, 30, args.cw_tol)

    def run(steps):
        dp = driver.upload(prob, ctx.device)
        host = prob.copy()
        nb = ctx.build_neighbors(dp.pos, dp.h, nin, prob.kernel)
        A, reps = 0, []
        for s in range(steps):
            host.set_time((s + 1) * prob.dt)
            for k in ("Q_e", "Q_E"):
                dp.arrays[k].copy_(torch.as_tensor(getattr(host, k)))
            for k in ("e", "E"):
                dp.arrays[k][nin:] = torch.as_tensor(getattr(host, k)[nin:])
            e, E, A, rep = driver.time_step(ctx, dp, nb, A=A, amg=amg, solve=solve, eps_e=1e-8,
                                            eps_E=1e-8, material_tol=1e-14)
            driver.advance(dp, e, E)
            reps.append(rep)
        torch.cuda.synchronize()
        return reps, dp

    for w in range(max(1, args.warmup)):
        log(f"[bench] config2 warmup run {w}")
        run(2)
    log(f"[bench] timing {args.steps} steps")
    with paused_gc():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps, dp = run(args.steps)
        wall = time.perf_counter() - t0
    outer = sum(r.outer for r in reps)
    nm = prob.copy()
    nm.set_time(args.steps * prob.dt)
    em, Em = nm.mms(args.steps * prob.dt)[:2]
    E = dp.arrays["E"][:nin].cpu().numpy()
    e = dp.arrays["e"][:nin].cpu().numpy()
    out = {
        "metric": METRIC, "value": nin * outer / wall, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"config2 manufactured {args.n}^3 ({nin} particles, "
                               f"{prob.n_ghost} ghosts), {args.steps} steps dt={prob.dt}, outer "
                               f"to 1e-8, FP64 CG + {('Jacobi', 'AMG')[precond]} to "
                               f"{args.tol:g} (componentwise {args.cw_tol:g})",
                   "particles": nin, "precond": ("jacobi", "amg")[precond]},
        "outer_per_step": [r.outer for r in reps],
        "krylov_per_solve": [k for r in reps for k in r.krylov],
        "l1_rel_err_vs_exact": {"e": float(np.sum(np.abs(e - em[:nin])) / np.sum(em[:nin])),
                                "E": float(np.sum(np.abs(E - Em[:nin])) / np.sum(Em[:nin]))},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="marshak3d")
    ap.add_argument("--n", type=int, default=256, help="particles per axis")
    ap.add_argument("--outer", type=int, default=BENCH_OUTER)
    ap.add_argument("--tol", type=float, default=BENCH_TOL, help="normwise solve tolerance")
    ap.add_argument("--cw-tol", type=float, default=BENCH_CW_TOL,
                    help="componentwise solve tolerance (0: normwise test only)")
    ap.add_argument("--precond", type=int, default=None,
                    help="0 Jacobi, 1 AMG V-cycle (default: 1 for config2, else 0)")
    ap.add_argument("--inner-tol", type=float, default=BENCH_INNER_TOL,
                    help="relative reduction asked of each FP32 inner solve")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison step")
    ap.add_argument("--mixed", action="store_true",
                    help="coswave3d: FP32 inner CG with FP64 refinement instead of FP64 CG")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-vcycle", action="store_true",
                    help="ensemble: skip the batched V-cycle leg")
    ap.add_argument("--no-densitystep", action="store_true",
                    help="marshak3d: skip the mixed-vs-FP64 leg on the density-step recipe")
    ap.add_argument("--cpu-n", type=int, default=64)
    ap.add_argument("--nprob", type=int, default=96, help="ensemble: number of problems")
    ap.add_argument("--scale", type=float, default=1.0, help="ensemble: size factor")
    ap.add_argument("--build-streams", type=int, default=4,
                    help="ensemble: host threads (each with its own stream) building the problems")
    ap.add_argument("--graph-iters", type=int, default=8,
                    help="ensemble: PCG iterations per replayed HIP graph (0: none)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default SpMV shapes instead of tuning them during warm-up")
    ap.add_argument("--shapes", default=None,
                    help="fine-level SpMV shape indices FP64,FP32,RESIDUAL (rt_spmv_shapes order) "
                         "used instead of tuning, e.g. to profile the tuned run's kernels")
    args = ap.parse_args()
    if args.precond is None:
        args.precond = 1 if args.workload == "config2" else 0

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2001_11606_amd import driver, rt

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.workload == "ensemble":
        run_ensemble(args)
        return
    if args.workload in ("coswave3d", "coswave2d"):
        run_coswave(args)
        return
    if args.workload == "config2":
        if args.n == 256:
            args.n = 64
        run_config2(args)
        return
    run_single(args)


def _fp64_reference(ctx, dp, outer, amg):
    """The same step solved to 1e-14 in both measures in FP64: the reference of
    the accuracy figures."""
    from paper_2001_11606_amd import rt
    e, E, A, rep, nb = run_step(ctx, dp, rt.solve_opts(0, 0, 1e-14, 20000, 1e-4, 60, 1e-14),
                                outer, amg)
    release(ctx, nb, A)
    return e, E


def _max_rel(a, ref):
    return float(((a - ref).abs() / ref.abs()).max())


def _kernel_roof(name, nbytes, calls, seconds):
    if not calls:
        return None
    us = 1e6 * seconds / calls
    gbs = nbytes / (seconds / calls) / 1e9
    return {"kernel": name, "bytes_per_launch": nbytes, "avg_launch_us": round(us, 2),
            "launches": calls, "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "device_ms": round(1e3 * seconds, 3)}


def precond_leg(ctx, dp, args, ref, steps=2):
    """The same step with the aggregation V-cycle (strength-based aggregates,
    up to eight levels) in place of Jacobi, mixed and FP64 at the same
    tolerances: hierarchy sizes, iterations, mean solve time per step and the
    largest relative difference from the 1e-14 FP64 step `ref` (e, E)."""
    import torch
    from paper_2001_11606_amd import rt
    amg = rt.amg_opts(max_levels=8, build_fp32=1)
    out = {}
    for prec, key in ((rt.RT_PREC_MIXED, "mixed"), (rt.RT_PREC_FP64, "fp64")):
        solve = bench_solve_opts(prec, 1, args.tol, args.cw_tol, args.inner_tol)
        e, E, A, rep, nb = run_step(ctx, dp, solve, args.outer, amg)   # warm-up
        release(ctx, nb, A)
        t = []
        for _ in range(steps):
            e, E, A, rep, nb = run_step(ctx, dp, solve, args.outer, amg)
            t.append(rep.solve_seconds)
            info = ctx.matrix_info(A)
            release(ctx, nb, A)
        torch.cuda.synchronize()
        out["levels"] = info.levels
        out["level_n"] = list(info.level_n[:info.levels])
        out[f"solve_s_{key}"] = round(sum(t) / len(t), 5)
        out[f"krylov_{key}"] = rep.krylov
        out[f"max_rel_err_E_{key}"] = _max_rel(E, ref[1])
        out[f"max_rel_err_e_{key}"] = _max_rel(e, ref[0])
    return out


def densitystep_leg(ctx, args, steps=3):
    """Mixed against FP64 on the density-step recipe at 128^3 (2,097,152
    particles, tens of Krylov iterations per solve), same options as the main
    workload: mean solve time per step of each, and both results' largest
    relative difference from the 1e-14 FP64 step."""
    import torch
    from paper_2001_11606_amd import driver, rt
    prob = make_problem("densitystep3d", 128)
    dp = driver.upload(prob, ctx.device)
    amg = rt.amg_opts(max_levels=1, build_fp32=1)
    out = {"workload": f"densitystep3d 128^3 ({prob.n_interior} particles), {args.outer} outer "
                       f"iterations, Jacobi, tol {args.tol:g}, componentwise {args.cw_tol:g}"}
    eR, ER = _fp64_reference(ctx, dp, args.outer, amg)
    res = {}
    for prec, key in ((rt.RT_PREC_MIXED, "mixed"), (rt.RT_PREC_FP64, "fp64")):
        solve = bench_solve_opts(prec, 0, args.tol, args.cw_tol, args.inner_tol)
        e, E, A, rep, nb = run_step(ctx, dp, solve, args.outer, amg)   # warm-up
        release(ctx, nb, A)
        t = []
        for _ in range(steps):
            e, E, A, rep, nb = run_step(ctx, dp, solve, args.outer, amg)
            t.append(rep.solve_seconds)
            release(ctx, nb, A)
        torch.cuda.synchronize()
        res[key] = sum(t) / len(t)
        out[f"solve_s_{key}"] = round(res[key], 5)
        out[f"krylov_{key}"] = rep.krylov
        out[f"max_rel_err_E_{key}"] = _max_rel(E, ER)
        out[f"max_rel_err_e_{key}"] = _max_rel(e, eR)
    out["ratio_fp64_over_mixed"] = round(res["fp64"] / res["mixed"], 3)
    out["vcycle"] = precond_leg(ctx, dp, args, (eR, ER))
    del dp
    out["depth_tune"] = depth_leg(ctx, args)
    return out


def depth_leg(ctx, args, reps=3):
    """The V-cycle depth tuner on the density-step matrix at 128^3: FP64 CG
    to the bench's tolerances on b = 1 from zero at every depth (1 = Jacobi),
    at the configuration's dt and at dt = 0.025 (diffusion number about 9,
    where the hierarchy pays); mean solve times, iterations and the depth
    kept."""
    import torch
    from paper_2001_11606_amd import driver, rt
    out = {}
    for dt in (None, 0.025):
        prob = make_problem("densitystep3d", 128)
        if dt:
            prob.dt = dt
        dp = driver.upload(prob, ctx.device)
        nb = ctx.build_neighbors(dp.pos, dp.h, prob.n_interior, prob.kernel)
        A = ctx.assemble(nb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                         dp.limiter_k, amg=rt.amg_opts(max_levels=8))
        nin = prob.n_interior
        b = torch.ones(nin, dtype=torch.float64, device=ctx.device)
        x0 = torch.zeros(nin, dtype=torch.float64, device=ctx.device)
        rep = ctx.tune_depth(A, b, x0, bench_solve_opts(rt.RT_PREC_FP64, 1, args.tol, args.cw_tol,
                                                        args.inner_tol), reps=reps)
        out[f"dt_{prob.dt:g}"] = {
            "levels": rep.depths,
            "solve_ms": [round(1e3 * rep.seconds[d], 3) for d in range(rep.depths)],
            "iterations": list(rep.iterations[:rep.depths]),
            "chosen_depth": rep.chosen}
        ctx.free(A, nb)
        del dp
    return out


def run_single(args):
    """One problem (marshak3d, densitystep3d or wendland3d), the whole path
    per step; see the module docstring."""
    import torch
    from paper_2001_11606_amd import driver, rt
    log(f"[bench] generating {args.workload} n={args.n}")
    t0 = time.perf_counter()
    prob = make_problem(args.workload, args.n)
    log(f"[bench] generated {prob.n_interior} interior + {prob.n_ghost} ghosts in "
        f"{time.perf_counter() - t0:.1f} s")
    ctx = rt.Context(0)
    dp = driver.upload(prob, ctx.device)
    amg = rt.amg_opts(max_levels=8 if args.precond == 1 else 1, build_fp32=1)
    torch.cuda.synchronize()
    copy_gbs = copy_bandwidth()
    log(f"[bench] stream copy {copy_gbs:.0f} GB/s")
    solve32 = bench_solve_opts(rt.RT_PREC_MIXED, args.precond, args.tol, args.cw_tol,
                               args.inner_tol)
    solve64 = bench_solve_opts(rt.RT_PREC_FP64, args.precond, args.tol, args.cw_tol,
                               args.inner_tol)

    shapes = None
    tune = None
    if args.shapes:
        shapes = [[int(v) for v in args.shapes.split(",")]]
        tune = {"shapes": rt.rt_spmv_shapes(), "chosen": shapes, "pinned": True}
        args.no_tune = True

    def one(solve, profile=False):
        ctx.set_profiling(profile)
        out = run_step(ctx, dp, solve, args.outer, amg, shapes)
        ctx.set_profiling(False)
        return out

    for w in range(args.warmup):
        log(f"[bench] warmup step {w}")
        e, E, A, rep, nb = one(solve32)
        if w == 0 and not args.no_tune:
            # SpMV shapes are tuned once per problem, outside the timed region
            tune = ctx.tune(A, reps=5)
            shapes = tune["chosen"]
            log(f"[bench] tuned SpMV shapes {[[tune['shapes'][c] if c >= 0 else None for c in ch] for ch in shapes]}")
        release(ctx, nb, A)
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    reps = []
    with paused_gc():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            e, E, A, rep, nb = one(solve32, profile=True)
            reps.append(rep)
            info = ctx.matrix_info(A)
            if s + 1 < args.steps:
                release(ctx, nb, A)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    nin = prob.n_interior
    value = nin * args.outer * args.steps / elapsed
    log(f"[bench] {ms_step:.1f} ms/step, krylov {reps[-1].krylov}, refinements "
        f"{reps[-1].refinements}, status {reps[-1].status}")
    # the backward-Euler residual G (Sec. 2.2) of the last timed step's final
    # state (after the timed region: one more FP64 product)
    g_last = ctx.newton_residual(A, e, E, 0)
    newton_residual = {"rad_rel": g_last.rad_rel, "rad_norm": g_last.rad_norm,
                       "mat_rel": g_last.mat_rel,
                       "starting_rad_rel": [round(v, 16) for v in reps[-1].init_rel_residual]}
    release(ctx, nb, A)

    # per-kernel rooflines of the products, from the HIP events of the timed steps
    n_rows = info.n
    nnz_off = info.nnz - info.n
    tile_cols = info.level_tile_cols[0]
    sh = tune["shapes"] if tune else None
    s64, s32, sres = (shapes[0] if shapes else (None, None, None))
    if sres is not None and sres < 0:
        sres = s64
    tiled32 = bool(tile_cols) and (sh is None or sh[s32][2])
    tiled64 = bool(tile_cols) and (sh is None or sh[s64][2])
    tiledr = bool(tile_cols) and (sh is None or sh[sres][2])
    k32 = (("k_spmv_tiled<float, %d, %d, SP_DOT>" % tuple(sh[s32][:2])) if tiled32 and sh
           else "k_spmv_tiled<float> (default shape)" if tiled32 else "k_spmv<float> (plain CSR)")
    k64r = (("k_spmv_tiled<double, %d, %d, SP_RESID>" % tuple(sh[sres][:2])) if tiledr and sh
            else "k_spmv_tiled<double> SP_RESID" if tiledr else "k_spmv<double> SP_RESID")
    roof32 = _kernel_roof(k32, spmv_bytes(4, nnz_off, n_rows, tile_cols if tiled32 else 0),
                          sum(r.spmv32_calls for r in reps), sum(r.spmv32_seconds for r in reps))
    roof_res = _kernel_roof(k64r, resid_bytes(nnz_off, n_rows, tile_cols if tiledr else 0,
                                              args.cw_tol > 0),
                            sum(r.resid_calls for r in reps), sum(r.resid_seconds for r in reps))
    kernels = [k for k in (roof_res, roof32) if k]
    for k in kernels:
        k["traffic"] = profiled_traffic(args.workload, args.n, k["kernel"])
    roof = None
    if kernels:
        dom = max(kernels, key=lambda k: k["device_ms"])   # most device time per step
        roof = {"bound": "hbm", "achieved": dom["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["frac"], "traffic": dom["traffic"],
                "kernel": dom["kernel"], "bytes_per_launch": dom["bytes_per_launch"],
                "avg_launch_us": dom["avg_launch_us"], "launches": dom["launches"],
                "stream_copy_gbs": round(copy_gbs, 1), "tile_cols": tile_cols,
                "kernels": kernels}
    solve_mixed = sum(r.solve_seconds for r in reps) / len(reps)

    cmp = None
    if not args.no_fp64:
        log("[bench] FP64 comparison step and the 1e-14 reference")
        e64, E64, A64, rep64, nb64 = one(solve64, profile=True)
        release(ctx, nb64, A64)
        eR, ER = _fp64_reference(ctx, dp, args.outer, amg)
        torch.cuda.synchronize()
        cmp = {"solve_s_mixed": round(solve_mixed, 5), "solve_s_fp64": round(rep64.solve_seconds, 5),
               "ratio_fp64_over_mixed": round(rep64.solve_seconds / max(solve_mixed, 1e-12), 3),
               "krylov_mixed": reps[-1].krylov, "krylov_fp64": rep64.krylov,
               "refinements_mixed": reps[-1].refinements,
               "max_rel_err_E_mixed": _max_rel(E, ER), "max_rel_err_e_mixed": _max_rel(e, eR),
               "max_rel_err_E_fp64": _max_rel(E64, ER), "max_rel_err_e_fp64": _max_rel(e64, eR),
               "reference": "the same step in FP64 to 1e-14, normwise and componentwise"}
        k64 = (("k_spmv_tiled<double, %d, %d, SP_DOT>" % tuple(sh[s64][:2])) if tiled64 and sh
               else "FP64 SP_DOT product")
        r64 = _kernel_roof(k64, spmv_bytes(8, nnz_off, n_rows, tile_cols if tiled64 else 0),
                           rep64.spmv64_calls, rep64.spmv64_seconds)
        if r64:
            cmp["fp64_cg_product"] = r64
    amg_leg = None
    if not args.no_fp64 and args.precond == 0:
        log("[bench] V-cycle leg")
        amg_leg = precond_leg(ctx, dp, args, (eR, ER))
    c3 = None
    if args.workload == "marshak3d" and not args.no_densitystep:
        log("[bench] density-step leg (mixed vs FP64 at 128^3)")
        c3 = densitystep_leg(ctx, args)

    # phase breakdown (one extra, synchronised step; not part of the timed region)
    log("[bench] phase breakdown step")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nbb = ctx.build_neighbors(dp.pos, dp.h, dp.n_interior, dp.kernel)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    Ab = ctx.assemble(nbb, dp.arrays, dp.dt, dp.c, dp.a, dp.opacity_exponent, dp.limiter,
                      dp.limiter_k, amg=amg)
    for lvl, chosen in enumerate((shapes or [])[:ctx.matrix_info(Ab).levels]):
        for prod, sh_ in zip((rt.RT_PREC_FP64, rt.RT_PREC_MIXED, rt.RT_PRODUCT_RESIDUAL), chosen):
            rt.rt_matrix_set_spmv_shape(Ab, lvl, prod, sh_)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    eb = torch.empty(nin, dtype=torch.float64, device=ctx.device)
    Eb = torch.empty_like(eb)
    rt.rt_to_sorted(ctx.handle, nbb.handle, dp.arrays["e"].data_ptr(), eb.data_ptr())
    rt.rt_to_sorted(ctx.handle, nbb.handle, dp.arrays["E"].data_ptr(), Eb.data_ptr())
    nopts = rt.newton_opts(solve32, state_order=1)
    solve_b = 0.0
    for ell in range(args.outer):
        _, stb = ctx.newton_step(Ab, eb, Eb, ell, nopts)
        solve_b += stb.solve.seconds
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    phases = {"neighbors_ms": round(1e3 * (t2 - t1), 2), "assemble_ms": round(1e3 * (t3 - t2), 2),
              "outer_iterations_ms": round(1e3 * (t4 - t3), 2),
              "of_which_solves_ms": round(1e3 * solve_b, 2)}
    release(ctx, nbb, Ab)
    log(f"[bench] phases {phases}")
    solve_rate = nin * args.outer / (solve_mixed if solve_mixed > 0 else float("inf"))

    cpu = None
    if not args.no_cpu:
        log(f"[bench] CPU oracle baseline at n={args.cpu_n}")
        cpu = cpu_baseline(args.workload, args.cpu_n, args.outer, args.tol, args.cw_tol)

    rule = (f"mixed FP32/FP64 to ||r|| <= {args.tol:g} ||b|| and max_i |r_i|/(a_ii |x_i|) <= "
            f"{args.cw_tol:g} (inner {args.inner_tol:g})")
    out = {
        "metric": METRIC, "value": value, "unit": "particle-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} {args.n}^3 ({nin} particles, {prob.n_ghost} ghosts), "
                               f"1 step dt={prob.dt}, {args.outer} outer iterations, {rule}",
                   "particles": nin, "nnz": info.nnz, "amg_levels": info.levels,
                   "precond": "amg" if args.precond == 1 else "jacobi",
                   "tol": args.tol, "cw_tol": args.cw_tol, "inner_tol": args.inner_tol},
        "roofline": roof, "cpu_baseline": cpu, "mixed_vs_fp64": cmp,
        "vcycle": amg_leg, "mixed_vs_fp64_densitystep3d": c3, "phases": phases,
        "solve_particle_updates_per_s": solve_rate,
        "newton_residual": newton_residual,
        "spmv_tune": None if tune is None else (
            {"shapes_g_e": tune["shapes"], "chosen": tune["chosen"], "pinned": True}
            if tune.get("pinned") else {
                "shapes_g_e": tune["shapes"], "chosen": tune["chosen"],
                "level0_us_fp64": [round(t, 1) for t in tune["us"][0][0]],
                "level0_us_fp32": [round(t, 1) for t in tune["us"][0][1]],
                "level0_us_fp64_residual": [round(t, 1) for t in tune["us"][0][2]]}),
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
