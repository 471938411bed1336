#!/usr/bin/env python3
"""Benchmark of the GMG hot path on one MI355X.

One step = one complete solve of the periodic Q2 Poisson problem on 256^3 elements
(512^3 DoFs) with a Gaussian-random-field source (power spectrum |k|^-alpha,
alpha ~ U[2, 4]; the held-out evaluation seeds 30000-30004 in turn) to a relative
true FP64 residual of 1e-8, with the learned smoother: FP32 V-cycles whose smoothing
phases end with a learned correction (per-cycle fallback to the plain cycle) inside
FP64 flexible CG.  Inputs (sources, buffers, hierarchy) are resident in HBM before
the timed region.  The plain FP64 solve (CG on FP64 V-cycles) and the FP32 solve
without the net run the same sources next to it, the operator apply is timed alone
(GDoF/s), and the other workloads (the 256^3-DoF Gaussian and sharp Q2/Q4 problems,
the octree, the sharp layer, the FFT methods) are reported as extras.

Prints one JSON line (stdout).  --gpus > 1 is not supported: this build runs on a
single GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GMG time to 1e-8 rel. residual (learned+FP32 vs plain FP64); apply GDoF/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def apply_rate(ctx, prec, reps=20):
    """Average duration of the finest-level apply kernel: `reps` back-to-back launches between
    two HIP events recorded on the context's stream (torch's current stream, which the context
    was built on), so no event sits between two launches."""
    import torch
    from paper_1408_6497_amd import GMG_FP32
    n = ctx.num_dofs()
    dt = torch.float32 if prec == GMG_FP32 else torch.float64
    g = torch.Generator(device="cuda").manual_seed(1)
    x = torch.randn(n, device="cuda", dtype=dt, generator=g)
    y = torch.empty_like(x)
    assert ctx.stream == torch.cuda.current_stream()
    for _ in range(3):
        ctx.apply(-1, x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.apply(-1, x, y)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    bytes_per = 2 * n * x.element_size()
    return {"dofs": n, "launches": reps, "sec": sec, "gdofs": n / sec * 1e-9, "gbs": bytes_per / sec * 1e-9,
            "hbm_frac": bytes_per / sec * 1e-9 / HBM_PEAK_GBS}


def smoother_roofline(ctx, order):
    """Achieved bandwidth of the FP32 smoother-step kernel instance
    k_apply_col<float, q, 1, Cheb> -- the one launched on every level with at
    least 64 element columns in x -- over all its launches since the last timing
    reset: algorithmic bytes of those launches over their duration, measured with
    HIP events on the library stream around each run of consecutive smoother
    steps (4 or 6 launches of this kernel per smoothing phase)."""
    from paper_1408_6497_amd import Context, GMG_FP32
    launches, sec, algo_bytes = 0, 0.0, 0.0
    per_level = []
    for l in range(ctx.levels):
        nl = ctx.num_dofs(l)
        if ctx.lattice(l) // order < 64:
            continue
        lv_l, lv_s, lv_b = 0, 0.0, 0.0
        for kind, vals in ((Context.KIND_SMOOTH0, 3), (Context.KIND_SMOOTH, 4)):
            c, s_ = ctx.timing(l, kind, GMG_FP32)
            lv_l += c
            lv_s += s_
            lv_b += c * vals * 4 * nl
        launches += lv_l
        sec += lv_s
        algo_bytes += lv_b
        if lv_l:
            per_level.append({"level": l, "dofs": nl, "launches": lv_l, "avg_us": lv_s / lv_l * 1e6,
                              "gbs": lv_b / lv_s * 1e-9 if lv_s > 0 else None})
    return launches, sec, algo_bytes, per_level


def traffic_record():
    """HBM traffic per launch of the roofline kernel, from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary; None if the kernel source changed since the
    counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_apply_col_f32_q2_c4_learned_traffic.md")
    src = os.path.join(ROOT, "paper_1408_6497_amd", "csrc", "gmg_apply.hip")
    try:
        rec = None
        for line in open(path):
            if line.startswith("traffic_record: "):
                rec = json.loads(line[len("traffic_record: "):])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if rec and rec.get("source_sha256_16") == sha:
            return rec
    except OSError:
        pass
    return None


EVAL_SEEDS = (30000, 30001, 30002, 30003, 30004)
# the learned configuration of the headline: nets on depths 2 and coarser (the two finest
# levels keep the polynomial, where one net application costs several Chebyshev ones)
LEARNED_OPTS = dict(use_learned=1, learned_min_depth=2)


def load_nets(ctx):
    """Install every shipped net (weights/q2_depth<d>.gmgw) on its depth; returns the depths."""
    import glob
    import re
    from paper_1408_6497_amd import train as T
    depths = []
    for path in sorted(glob.glob(os.path.join(ROOT, "paper_1408_6497_amd", "weights", "q2_depth*.gmgw"))):
        d = int(re.search(r"q2_depth(\d+)\.gmgw$", path).group(1))
        if d < ctx.levels - 1:
            ctx.net_set_weights(d, T.load(path)["w"])
            depths.append(d)
    return depths


def host_info():
    """CPU model and core counts of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "cpus_in_affinity_mask": affinity}


def cpu_baseline(n_sample=64, n_full=256, seed=EVAL_SEEDS[0]):
    """The oracle (numpy/scipy, FP64, Kronecker form, as it stands) on the headline workload.

    Sample: the oracle's whole solve (CG preconditioned by its Chebyshev V-cycle, to 1e-8) of
    the same kind of source (GRF, evaluation seed) at Q2 n_sample^3 elements, timed; plus one
    oracle operator apply at the full 512^3-DoF size and one at the sample size, timed.  The
    value is the sample solve scaled by the ratio of the two applies (the solve's work is
    a fixed number of applies per iteration and the iteration count does not grow with the
    mesh; the measured ratio carries the oracle's growing cost per DoF at the full size)."""
    import numpy as np
    from oracle import multigrid as mg, krylov
    from oracle import operator as op
    from workloads import grf
    q = 2
    N = q * n_sample
    f = grf(N, seed)[0].numpy()
    H = mg.Hierarchy(q, n_sample, int(math.log2(n_sample)) - 1, mg.Options(seed=0), form="kron")
    b = mg.rhs(q, n_sample, f, form="kron")
    t0 = time.perf_counter()
    u, info = krylov.pcg(H.finest.A, b, H.vcycle, 1e-8)
    t = time.perf_counter() - t0
    x = np.random.default_rng(1).standard_normal(N ** 3)
    t0 = time.perf_counter()
    H.finest.A @ x
    t_apply_sample = time.perf_counter() - t0
    del x, u, H
    A = op.KroneckerOperator(q, n_full)
    x = np.random.default_rng(2).standard_normal((q * n_full) ** 3)
    t0 = time.perf_counter()
    A @ x
    t_apply_full = time.perf_counter() - t0
    del x
    dof_ratio = (n_full / n_sample) ** 3
    # the oracle's cost per DoF grows with the size (its sparse products leave the caches), so
    # the sample is scaled by the measured ratio of its own applies at the two sizes, not by
    # the DoF count
    ratio = t_apply_full / t_apply_sample
    return {"value": t * ratio, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle FP64 CG + Chebyshev(3) V(2,2) cycle (Kronecker 1D-CSR form, scipy sparse products, "
                       f"single-threaded) on a GRF source (seed {seed}) at Q2 {n_sample}^3 elements "
                       f"({N ** 3} DoFs): {info.iters} iterations to 1e-8 in {t:.2f} s; one oracle operator apply "
                       f"takes {t_apply_sample:.3f} s there and {t_apply_full:.2f} s at the full 512^3 DoFs "
                       f"({dof_ratio:.0f}x the DoFs), and the solve is scaled by that measured ratio "
                       f"{ratio:.1f} (the iteration count does not grow with the mesh)"),
            "sample_seconds": t, "sample_iters": info.iters, "apply_sample_s": t_apply_sample,
            "apply_full_s": t_apply_full, "scale": ratio, "dof_ratio": dof_ratio, "host": host_info()}


def c4_solves(steps, warmup, n=256, seeds=EVAL_SEEDS):
    """The headline workload: Q2 on n^3 elements, GRF sources of the evaluation seeds; the
    learned FP32 cycle (shipped nets, per-cycle fallback), the FP32 cycle without the net and
    plain FP64 CG, each to 1e-8; step i solves seed i mod len(seeds).  Seconds per solve."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64
    from workloads import grf
    N = 2 * n
    sources = [grf(N, sd, device="cuda")[0] for sd in seeds]
    out = {"workload": f"Q2, {n}^3 elements ({N ** 3} DoFs), GRF |k|^-alpha sources, seeds "
                       f"{seeds[0]}..{seeds[-1]} in turn, to 1e-8", "seeds": list(seeds)}
    for name, kw in (("learned_fp32", LEARNED_OPTS), ("fp32", dict(vcycle_prec=GMG_FP32)),
                     ("plain_fp64", dict(vcycle_prec=GMG_FP64))):
        ctx = Context(2, n, 0, seed=0, **kw)
        if name.startswith("learned"):
            out["net_depths"] = load_nets(ctx)
        u = torch.empty_like(sources[0])
        for i in range(max(warmup, 1)):
            ctx.solve(sources[i % len(seeds)], u, 1e-8)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for i in range(steps):
            infos.append(ctx.solve(sources[i % len(seeds)], u, 1e-8))
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        out[name] = {"s": t, "iters": [x.inner_iters for x in infos[:len(seeds)]],
                     "fallbacks": [x.fallbacks for x in infos[:len(seeds)]],
                     "max_rel_residual_f64": max(x.rel_residual_f64 for x in infos)}
        log(f"[bench] C4 {name}: {t * 1e3:.2f} ms/solve {out[name]}")
        ctx.close()
        del ctx, u
        torch.cuda.empty_cache()
    del sources
    torch.cuda.empty_cache()
    return out


def c4_roofline(n=256, seed=EVAL_SEEDS[0]):
    """Per-kernel durations of one learned solve of the headline workload, from the library's
    HIP events (timing=1: the same kernels and arguments, launched eagerly): the dominant
    kernel, the FP32 smoother step k_apply_col<float, 2, 1, Cheb> on the levels that keep the
    polynomial, and the learned corrections."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32
    from workloads import grf
    ctx = Context(2, n, 0, seed=0, timing=1, **LEARNED_OPTS)
    load_nets(ctx)
    f = grf(2 * n, seed, device="cuda")[0]
    u = torch.empty_like(f)
    ctx.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    ctx.timing_reset()
    info = ctx.solve(f, u, 1e-8)
    launches, sec, algo_bytes, per_level = smoother_roofline(ctx, 2)
    learned = []
    for l in range(ctx.levels):
        c, s_ = ctx.timing(l, Context.KIND_LEARNED, GMG_FP32)
        if c:
            learned.append({"level": l, "lattice": ctx.lattice(l), "corrections": c, "avg_us": s_ / c * 1e6})
    ctx.close()
    del f, u
    torch.cuda.empty_cache()
    return launches, sec, algo_bytes, per_level, learned, info


def c1_workload(steps=20):
    """C1: Q1 on 32^3 elements, 4 levels, f = 12 pi^2 sin sin sin, plain FP64 to 1e-10; the
    solve launched through the captured HIP graphs and eagerly; the amplitude of the solution
    against the closed-form discrete one (0.99679344074)."""
    import numpy as np
    import torch
    from paper_1408_6497_amd import Context
    from workloads import sin_exact, sin_source
    out = {"workload": "Q1, 32^3 elements, 4 levels, 12 pi^2 sin sin sin, plain FP64 to 1e-10"}
    for name, kw in (("graph", {}), ("no_graph", dict(no_graphs=1))):
        ctx = Context(1, 32, 4, seed=0, **kw)
        x1 = ctx.dof_coords_1d()
        f = sin_source(x1, device="cuda")
        u = torch.empty_like(f)
        ctx.solve(f, u, 1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = ctx.solve(f, u, 1e-10)
        torch.cuda.synchronize()
        ue = sin_exact(x1)
        amp = float(np.dot(u.cpu().numpy(), ue) / np.dot(ue, ue))
        out[name] = {"s": (time.perf_counter() - t0) / steps, "iters": info.inner_iters,
                     "rel_residual_f64": info.rel_residual_f64, "amplitude": amp,
                     "amplitude_err": abs(amp - 0.99679344074) / 0.99679344074}
        ctx.close()
    log(f"[bench] C1: {out}")
    return out


def spectral_workload(sizes=(256, 512), steps=5):
    """The paper's FFT Poisson method (Section 2.1): the spectral solve on the N^3 grid, test
    case 1 of Section 3 at frequency N/4 (u = sin sin sin, exact on the grid); seconds per solve
    and the max error."""
    import torch
    from paper_1408_6497_amd import SpectralSolver
    out = {"workload": "spectral FFT Poisson solve (own transforms), f = 12 pi^2 k^2 sss at k = N/4"}
    for N in sizes:
        k = N // 4
        x = torch.arange(N, dtype=torch.float64, device="cuda") / N
        s = torch.sin(2 * math.pi * k * x)
        ue = (s[:, None, None] * s[None, :, None] * s[None, None, :]).reshape(-1)
        f = 12 * math.pi ** 2 * k * k * ue
        u = torch.empty_like(f)
        sp = SpectralSolver(N)
        sp.solve(f, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sp.solve(f, u)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        out[f"N{N}"] = {"s": t, "max_err": float((u - ue).abs().max()), "gbs_at_144B_per_point": 144 * N ** 3 / t * 1e-9}
        sp.close()
        del f, u, ue, s
        torch.cuda.empty_cache()
    log(f"[bench] spectral: {out}")
    return out


def c2_workload(steps, warmup):
    """Q2 on 128^3 elements (256^3 DoFs), 32 Gaussians (sigma U[0.02, 0.1], seed 0): FP32 cycles in
    FP64 flexible CG against plain FP64 CG, to 1e-8, and the FP32 smoother step's bandwidth on
    its 256^3- and 128^3-node levels (HIP events in an eager repeat)."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64
    from workloads import gaussian_params, gaussian_source
    q, n = 2, 128
    out = {"workload": "Q2, 128^3 elements (256^3 DoFs), 32 Gaussians sigma U[0.02, 0.1], seed 0, to 1e-8"}
    f = None
    for name, kw in (("fp32", dict(vcycle_prec=GMG_FP32)), ("plain_fp64", dict(vcycle_prec=GMG_FP64))):
        ctx = Context(q, n, 0, seed=0, **kw)
        if f is None:
            f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(0, 32, 0.02, 0.1), device="cuda")
            u = torch.empty_like(f)
        for _ in range(max(warmup, 1)):
            ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        out[name] = {"s": (time.perf_counter() - t0) / steps, "iters": info.inner_iters,
                     "rel_residual_f64": info.rel_residual_f64}
        ctx.close()
    ctxt = Context(q, n, 0, seed=0, vcycle_prec=GMG_FP32, timing=1)
    ctxt.solve(f, u, 1e-8)
    torch.cuda.synchronize()
    ctxt.timing_reset()
    ctxt.solve(f, u, 1e-8)
    launches, sec, algo_bytes, per_level = smoother_roofline(ctxt, q)
    out["smoother_step"] = {"launches": launches, "avg_us": sec / max(launches, 1) * 1e6,
                            "gbs": algo_bytes / sec * 1e-9 if sec > 0 else None, "per_level": per_level}
    ctxt.close()
    log(f"[bench] c2 workload: {out}")
    return out


def q4_workload(steps=5):
    """Q4 on 64^3 elements (256^3 DoFs), 8 Gaussians with sigma log-uniform in [1e-3, 1e-2]
    (seed 0): plain FP64 CG vs FP32 cycles in FP64 flexible CG, to 1e-8."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64
    from workloads import gaussian_params, gaussian_source
    params = gaussian_params(0, 8, 1e-3, 1e-2, log_uniform=True)
    out = {"workload": "Q4, 64^3 elements (256^3 DoFs), 8 Gaussians sigma log-uniform [1e-3, 1e-2], seed 0, to 1e-8"}
    for name, kw in (("plain_fp64", dict(vcycle_prec=GMG_FP64)), ("fp32", dict(vcycle_prec=GMG_FP32))):
        ctx = Context(4, 64, 0, seed=0, **kw)
        f = gaussian_source(ctx.dof_coords_1d(), params, device="cuda")
        u = torch.empty_like(f)
        ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        out[name] = {"s": (time.perf_counter() - t0) / steps, "iters": info.inner_iters,
                     "rel_residual_f64": info.rel_residual_f64}
        ctx.close()
        del f, u
        torch.cuda.empty_cache()
    log(f"[bench] q4 workload: {out}")
    return out


def orders_workload(steps=3):
    """The orders on the generic kernels (q = 3 and 5-16: Tables 7 and 10, Section 3's GMG-16) near
    256^3 DoFs each: the finest-level apply in both precisions (algorithmic bytes: x read, y
    written) and FP32 cycles in FP64 flexible CG on 32 Gaussians (sigma U[0.02, 0.1], seed 0) to
    1e-8."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64
    from workloads import gaussian_params, gaussian_source
    params = gaussian_params(0, 32, 0.02, 0.1)
    out = {"workload": "orders 3, 5, 6, 8, 14, 16 near 256^3 DoFs: apply rates, FP32 cycles in FP64 flexible CG "
                       "on 32 Gaussians (sigma U[0.02, 0.1], seed 0) to 1e-8"}
    for q, n in ((3, 64), (5, 32), (6, 32), (8, 32), (14, 16), (16, 16)):
        ctx = Context(q, n, 0, seed=0, vcycle_prec=GMG_FP32)
        rec = {"dofs": ctx.num_dofs(), "levels": ctx.levels,
               "apply_fp32": apply_rate(ctx, GMG_FP32, reps=10), "apply_fp64": apply_rate(ctx, GMG_FP64, reps=10)}
        f = gaussian_source(ctx.dof_coords_1d(), params, device="cuda")
        u = torch.empty_like(f)
        ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        rec["fp32_cycles"] = {"s": (time.perf_counter() - t0) / steps, "iters": info.inner_iters,
                              "rel_residual_f64": info.rel_residual_f64}
        out[f"q{q}_n{n}"] = rec
        ctx.close()
        del f, u
        torch.cuda.empty_cache()
    log(f"[bench] orders workload: {out}")
    return out


def octree_workload(steps=5):
    """The adaptive workload: Q2 on the octree refined from level 3 to 9 around 4 Gaussians
    (sigma 1e-3, seed 0); plain FP64 CG vs FP32 cycles in FP64 flexible CG, to 1e-8, plus the
    octree apply launch time on the finest level."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64, octree_refine_gaussians
    from workloads import gaussian_params, gaussian_source_points
    p = gaussian_params(0, 4, 1e-3, 1e-3)
    t0 = time.perf_counter()
    leaves = octree_refine_gaussians(3, 9, p["centres"], p["sigma"], p["amps"])
    t_tree = time.perf_counter() - t0
    out = {"workload": "Q2 octree, leaf levels 3..9 refined on a gradient bound around 4 Gaussians "
                       "(sigma 1e-3, seed 0), hanging nodes, to 1e-8", "leaves": int(leaves[0].size),
           "tree_build_s": t_tree}
    for name, kw in (("plain_fp64", dict(vcycle_prec=GMG_FP64)), ("fp32", dict(vcycle_prec=GMG_FP32)),
                     ("learned_fp32", LEARNED_OPTS)):
        ctx = Context(2, 0, leaves=leaves, seed=0, **kw)
        if name.startswith("learned"):
            load_nets(ctx)
        f = torch.from_numpy(gaussian_source_points(ctx.dof_coords(), p)).cuda()
        u = torch.empty_like(f)
        ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = ctx.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        out[name] = {"s": (time.perf_counter() - t0) / steps, "iters": info.inner_iters,
                     "rel_residual_f64": info.rel_residual_f64, "setup_s": info.t_setup,
                     "fallbacks": info.fallbacks}
        out["dofs"] = ctx.num_dofs()
        out["levels"] = ctx.levels
        ctx.close()
    ctxt = Context(2, 0, leaves=leaves, seed=0)
    for prec in (GMG_FP32, GMG_FP64):
        r = apply_rate(ctxt, prec)
        out["apply_" + ("fp32" if prec == GMG_FP32 else "fp64")] = {"us": r["sec"] * 1e6, "gdofs": r["gdofs"]}
    ctxt.close()
    log(f"[bench] octree workload: {out}")
    return out


def sharp_layer_workload(alpha=40.0, radius=0.25, tops=(6, 7, 8), steps=3, tol=1e-10):
    """Time to accuracy for the sharp-layer solution u = exp(-(r/R)^alpha) (R 0.25, centre of
    the unit torus), f = -Laplace(u) in closed form: octrees refined on the gradient of f from
    level 2 to each maximum level, Q1 and Q2, FP32 cycles in FP64 flexible CG to the residual
    tol; reports DoFs, the nodal max-norm error modulo a constant and the solve time."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, octree_refine_sharp_layer
    from workloads import sharp_layer
    out = {"workload": f"sharp layer exp(-(r/R)^alpha), alpha {alpha:g}, R {radius:g}, octree levels 2..L "
                       f"refined on h max|f'| > 1e-2 max|f|, FP32 cycles in FP64 flexible CG to {tol:g}",
           "runs": []}
    for top in tops:
        t0 = time.perf_counter()
        leaves = octree_refine_sharp_layer(2, top, (0.5, 0.5, 0.5), radius, alpha, 1e-2)
        t_tree = time.perf_counter() - t0
        for q in (1, 2):
            ctx = Context(q, 0, leaves=leaves, seed=0, vcycle_prec=GMG_FP32)
            ue, f = sharp_layer(ctx.dof_coords(), radius=radius, alpha=alpha)
            fd = torch.from_numpy(f).cuda()
            u = torch.empty_like(fd)
            ctx.solve(fd, u, tol, raise_on_noconv=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                info = ctx.solve(fd, u, tol, raise_on_noconv=False)
            torch.cuda.synchronize()
            t_solve = (time.perf_counter() - t0) / steps
            e = u.cpu().numpy() - ue
            run = {"q": q, "L": top, "leaves": int(leaves[0].size), "dofs": ctx.num_dofs(),
                   "linf_err": float(0.5 * (e.max() - e.min())), "solve_s": t_solve,
                   "iters": info.inner_iters, "rel_residual_f64": info.rel_residual_f64,
                   "setup_s": info.t_setup, "tree_build_s": t_tree}
            log(f"[bench] sharp layer {run}")
            out["runs"].append(run)
            ctx.close()
            del fd, u
            torch.cuda.empty_cache()
    return out


def fft_workload(n=256, steps=5, q=1):
    """Uniform Q_q on n^3 elements ((q n)^3 DoFs), 32-Gaussian source (seed 0): the exact FFT
    solve of the finite-element system against FP32 cycles in FP64 flexible CG to 1e-8, same
    load vector (the paper's Table 7 comparison of FFT and GMG on a smooth, uniform problem)."""
    import torch
    from paper_1408_6497_amd import Context, GMG_FP32
    from workloads import gaussian_params, gaussian_source
    ctx = Context(q, n, 0, seed=0, vcycle_prec=GMG_FP32)
    f = gaussian_source(ctx.dof_coords_1d(), gaussian_params(0, 32, 0.02, 0.1), device="cuda")
    b = torch.empty_like(f)
    ctx.rhs(f, b)
    uf, ug = torch.empty_like(b), torch.empty_like(b)
    out = {"workload": f"Q{q}, {n}^3 elements ({q * n}^3 DoFs), 32 Gaussians seed 0: FFT exact solve vs multigrid to 1e-8"}
    for name, call in (("fft", lambda: ctx.fft_solve(b, uf)), ("gmg_fp32_cycles", lambda: ctx.solve_rhs(b, ug, 1e-8))):
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call()
        torch.cuda.synchronize()
        out[name + "_s"] = (time.perf_counter() - t0) / steps
    out["rel_difference"] = (uf - ug).norm().item() / ug.norm().item()
    log(f"[bench] fft workload: {out}")
    ctx.close()
    return out


NET_FLOPS_PER_VOXEL = 2 * (432 + 6912 + 432)  # multiply-adds of layers 1, 2 and 3 per voxel, x 2
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak


def net_rate(n=256, reps=10):
    """One learned correction (the FP32 residual scaled by D^-1 and its RMS, the 3-layer BF16 net,
    u += s y) on the finest level of Q2 on n^3 elements ((2n)^3-voxel lattice), the shipped
    depth-0 net: `reps` back-to-back corrections between two HIP events on the context's stream."""
    import torch
    from paper_1408_6497_amd import Context
    from paper_1408_6497_amd import train as T
    ctx = Context(2, n, 0, seed=0, lambda_override=1.0)
    ctx.net_set_weights(0, T.load(os.path.join(ROOT, "paper_1408_6497_amd", "weights", "q2_depth0.gmgw"))["w"])
    top = ctx.levels - 1
    nv = ctx.num_dofs(top)
    g = torch.Generator(device="cuda").manual_seed(5)
    r = torch.randn(nv, device="cuda", dtype=torch.float32, generator=g)
    e = torch.empty_like(r)
    assert ctx.stream == torch.cuda.current_stream()
    for _ in range(2):
        ctx.net_correction(top, r, e)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.net_correction(top, r, e)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    ctx.close()
    del r, e
    torch.cuda.empty_cache()
    tf = NET_FLOPS_PER_VOXEL * nv / sec * 1e-12
    return {"lattice": 2 * n, "voxels": nv, "us": sec * 1e6, "tflops": tf, "frac_bf16_peak": tf / BF16_PEAK_TFLOPS}


def apply512_probe(reps=5):
    """For rocprofv3 counter runs: a 256 MiB device copy three times (the counters' calibration),
    then `reps` applies, restrictions onto the next level and prolongations from it, FP32 and FP64,
    of Q1 on 512^3 elements and Q2 on 256^3 elements (512^3 DoFs)."""
    import torch
    from paper_1408_6497_amd import Context
    a = torch.ones(64 << 20, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    del a, b
    out = {}
    for q, n in ((1, 512), (2, 256)):
        ctx = Context(q, n, 0, seed=0, lambda_override=1.0)
        for dt in (torch.float32, torch.float64):
            g = torch.Generator(device="cuda").manual_seed(3)
            x = torch.randn(ctx.num_dofs(), device="cuda", dtype=dt, generator=g)
            y = torch.empty_like(x)
            xc = torch.randn(ctx.num_dofs(ctx.levels - 2), device="cuda", dtype=dt, generator=g)
            for _ in range(reps):
                ctx.apply(-1, x, y)
            for _ in range(reps):
                ctx.restrict(-1, x, xc)
            for _ in range(reps):
                ctx.prolong(-1, xc, y)
            torch.cuda.synchronize()
            out[f"q{q}_{str(dt).split('.')[-1]}"] = {"dofs": ctx.num_dofs(), "coarse_dofs": ctx.num_dofs(ctx.levels - 2)}
            del x, y, xc
        ctx.close()
        torch.cuda.empty_cache()
    return out


def q4apply512_probe(reps=5):
    """For rocprofv3 counter runs: a 256 MiB device copy three times (the counters' calibration),
    then on Q4 with 128^3 elements (512^3 DoFs) `reps` applies, residuals, smoother applications
    from a guess (three Chebyshev steps each) and from zero (the fused first two steps and one
    more): FP32 in the vector form and in the matrix-core form (option q4_mfma), then FP64."""
    import torch
    from paper_1408_6497_amd import Context
    a = torch.ones(64 << 20, device="cuda", dtype=torch.float32)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    del a, b
    out = {}
    for name, dt, mf in (("fp32_vector", torch.float32, 0), ("fp32_mfma", torch.float32, 1),
                         ("fp64_vector", torch.float64, 0)):
        ctx = Context(4, 128, 0, seed=0, lambda_override=2.199326, q4_mfma=mf)
        g = torch.Generator(device="cuda").manual_seed(3)
        x = torch.randn(ctx.num_dofs(), device="cuda", dtype=dt, generator=g)
        rhs = torch.randn(ctx.num_dofs(), device="cuda", dtype=dt, generator=g)
        y = torch.empty_like(x)
        for _ in range(reps):
            ctx.apply(-1, x, y)
        for _ in range(reps):
            ctx.residual(-1, rhs, x, y)
        for _ in range(reps):
            ctx.smooth(-1, rhs, x, 1)
        for _ in range(reps):
            ctx.smooth_zero(-1, rhs, y, 1)
        torch.cuda.synchronize()
        out[name] = {"dofs": ctx.num_dofs(),
                     "shape_smooth": ctx.launch_shape(-1, 1 if dt == torch.float32 else 0, "smooth")}
        del x, rhs, y
        ctx.close()
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-apply-bench", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (Q2/Q4 on 256^3 DoFs, octree, sharp layer, C1, FFT methods)")
    ap.add_argument("--profile-workload", choices=("learned", "q4", "octree", "c2", "spectral", "c4roofline",
                                                   "apply512", "net512", "q4apply512", "orders"), default=None,
                    help="for profilers: run only this workload and print its JSON (no timed bench step); "
                         "c4roofline is the bench's own per-launch measurement of the learned solve, apply512 "
                         "a 256 MiB copy (counter calibration) then five Q1 and Q2 applies, restrictions and "
                         "prolongations of each precision on 512^3 DoFs, net512 five learned corrections on the 512^3 and "
                         "256^3 lattices, q4apply512 the same copy then five Q4 applies, residuals and smoother "
                         "applications on 512^3 DoFs in each form (FP32 vector, FP32 matrix cores, FP64), orders the "
                         "generic-kernel orders near 256^3 DoFs (apply rates and FP32-cycle solves)")
    ap.add_argument("--profile-n", type=int, default=256,
                    help="elements per direction of the learned workload under --profile-workload")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="for rocprofv3 --pmc runs: a 256 MiB device copy (counter calibration), then one eager "
                         "learned solve of the headline problem; prints nothing on stdout")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1408_6497_amd import Context, GMG_FP32, GMG_FP64
    from workloads import gaussian_params, gaussian_source, grf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.profile_workload:
        if args.profile_workload == "learned":
            res = c4_solves(2, 1, n=args.profile_n, seeds=EVAL_SEEDS[:2])
        elif args.profile_workload == "q4":
            res = q4_workload()
        elif args.profile_workload == "c2":
            res = c2_workload(3, 1)
        elif args.profile_workload == "spectral":
            res = spectral_workload(sizes=(512,), steps=3)
        elif args.profile_workload == "c4roofline":
            launches, sec, algo_bytes, per_level, learned_apps, info_t = c4_roofline()
            res = {"launches": launches, "avg_launch_us": sec / max(launches, 1) * 1e6,
                   "achieved_gbs": algo_bytes / sec * 1e-9, "per_level": per_level}
        elif args.profile_workload == "apply512":
            res = apply512_probe()
        elif args.profile_workload == "q4apply512":
            res = q4apply512_probe()
        elif args.profile_workload == "orders":
            res = orders_workload()
        elif args.profile_workload == "net512":
            res = {"net_512": net_rate(256, reps=5), "net_256": net_rate(128, reps=5)}
        else:
            res = octree_workload()
        print(json.dumps(res), flush=True)
        return
    if args.traffic_probe:
        a = torch.ones(64 << 20, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)          # reads and writes 256 MiB each
        torch.cuda.synchronize()
        ctxp = Context(2, 256, 0, seed=0, no_graphs=1, **LEARNED_OPTS)
        load_nets(ctxp)
        f = grf(512, EVAL_SEEDS[0], device="cuda")[0]
        u = torch.empty_like(f)
        ctxp.solve(f, u, 1e-8)
        torch.cuda.synchronize()
        log("[bench] traffic probe done")
        return

    # ---- timed region: K learned solves of the headline workload (and the same sources
    # with the FP32 cycle without the net and with plain FP64 CG)
    log("[bench] headline: Q2 on 256^3 elements, GRF evaluation seeds")
    c4 = c4_solves(args.steps, args.warmup)
    t_learned = c4["learned_fp32"]["s"]

    # ---- per-launch durations of the dominant kernel inside the same (learned) solve
    launches, sec, algo_bytes, per_level, learned_apps, info_t = c4_roofline()
    avg_dur = sec / max(launches, 1)
    achieved = algo_bytes / sec * 1e-9 if sec > 0 else 0.0
    log(f"[bench] smoother kernel: {launches} launches, avg {avg_dur * 1e6:.2f} us, {achieved:.0f} GB/s")

    apply = {}
    if not args.no_apply_bench:
        # 512^3 DoFs for every order (Q1 on 512^3, Q2 on 256^3, Q4 on 128^3 elements)
        for qq, nn in ((2, 256), (1, 512), (4, 128)):
            big = Context(qq, nn, 0, seed=0, lambda_override=1.0)
            apply[f"q{qq}_512cubed_fp32"] = apply_rate(big, GMG_FP32)
            apply[f"q{qq}_512cubed_fp64"] = apply_rate(big, GMG_FP64)
            big.close()
            del big
            torch.cuda.empty_cache()
        log(f"[bench] apply {json.dumps(apply)}")

    extra = {}
    if not args.no_extra:
        extra["learned_net"] = {"per_application_512cubed": net_rate(256), "per_application_256cubed": net_rate(128),
                                "flops_per_voxel": NET_FLOPS_PER_VOXEL, "peak_tflops": BF16_PEAK_TFLOPS}
        extra["c2_gaussians"] = c2_workload(args.steps, 1)
        extra["q4_sharp"] = q4_workload()
        extra["orders"] = orders_workload()
        extra["octree"] = octree_workload()
        extra["c1"] = c1_workload()
        extra["sharp_layer"] = sharp_layer_workload()
        extra["spectral_fft"] = spectral_workload()
        extra["fft_q1"] = fft_workload()
        extra["fft_q2"] = fft_workload(n=128, q=2)
        extra["fft_q4"] = fft_workload(n=64, q=4)

    traffic = traffic_record()
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline()
        log(f"[bench] cpu baseline {cpu['value']:.1f} s (sample {cpu['sample_seconds']:.1f} s)")

    out = {
        "metric": METRIC,
        "value": t_learned,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_learned * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32+f64",
        "data": "synthetic",
        "config": {
            "workload": ("Q2 periodic Poisson, uniform 256^3 elements (512^3 DoFs), Gaussian-random-field sources "
                         "(|k|^-alpha, alpha ~ U[2,4], evaluation seeds 30000-30004 in turn), learned smoother "
                         "(BF16 3-layer conv net on depths >= 2, per-cycle fallback) in FP32 Chebyshev(3) V(2,2) "
                         "cycles preconditioning FP64 flexible CG, to 1e-8"),
            "order": 2, "elements_per_dim": 256, "dofs": (2 * 256) ** 3, "learned": True,
            "learned_min_depth": LEARNED_OPTS["learned_min_depth"], "net_depths": c4.get("net_depths"),
        },
        "solve": {
            "learned_fp32_s": t_learned, "fp32_s": c4["fp32"]["s"], "plain_fp64_s": c4["plain_fp64"]["s"],
            "speedup_learned_vs_plain_fp64": c4["plain_fp64"]["s"] / t_learned,
            "speedup_learned_vs_fp32": c4["fp32"]["s"] / t_learned,
            "speedup_fp32_vs_plain_fp64": c4["plain_fp64"]["s"] / c4["fp32"]["s"],
            "detail": c4,
        },
        "apply": apply,
        "roofline": {
            "kernel": ("k_apply_col<float, 2, 1, Cheb>: the FP32 smoother step on the 512^3-, 256^3- and 128^3-node "
                       "levels of the learned solve"),
            "measured": ("HIP events on the library stream around each run of consecutive launches of this "
                         "kernel (one smoothing phase) in an eager repeat of a timed learned solve (seed 30000)"),
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (traffic["traffic_bytes_per_launch"] if traffic else None),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE and WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": algo_bytes / max(launches, 1),
            "launches": launches, "avg_launch_us": avg_dur * 1e6, "per_level": per_level,
            "learned_corrections": learned_apps,
        },
        "cpu_baseline": cpu,
        "workloads": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
