"""Benchmark: time to a 1e-7 residual for the preconditioned combined-field BIE
solve on 27 unit spheres (3x3x3 lattice, spacing 3, kappa = 4 pi, 20 panels x
10 Gauss nodes, |m| <= 40, N = 437,400 unknowns, one plane wave along
(1,1,1)/sqrt 3), on one MI355X.

A step is one whole solve -- incident field at the nodes already in HBM ->
sigma with FP64 residual <= 1e-7 -- in mixed precision (FP32 inter-body sum,
DFTs and modal applies inside FP64 flexible GMRES).  Plain FP64 GMRES on the
same problem is timed beside it.  The precomputation of the scattering
matrices (FP64, on the GPU) is timed separately and is not part of a step.

Prints one JSON line.  The roofline object is for the dominant kernel, the
FP32 inter-body sum: 39 flop per (target, source) pair on different bodies,
timed with HIP events on the library's stream.  Beside the step the line
carries
  - `skeleton`: the same problem through the ring skeletonization of Sec. 5
    (and, in `skeleton.points`, through point skeletons from the randomized ID);
  - `c5`: the largest workload (64 mixed bodies in a 24^3 box, kappa = 4 pi,
    N = 1,351,890, 16 plane waves): one mixed and one FP64 batched solve to
    1e-7, iterations and explicit FP64 residuals, and in
    `c5.skeleton_points` the same 16 rhs through point skeletons at eps 1e-10
    (one randomized ID per body shape);
  - `warm_start`: the learned warm start on the 8 mixed bodies (network trained
    on 4,096 of the method's own solves, k in [1.5 pi, 2.5 pi]), 512 held-out
    (k, direction) pairs solved from three initial guesses: zero, the
    single-body responses -D^{-1} v, and those plus the network's
    multiple-scattering part.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_PAIR = 39.0            # algorithmic flops of one kernel evaluation + complex MAC
FLOP_PER_EXTRA_RHS = 8.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
FP64_VECTOR_PEAK_TFLOPS = 78.6
# HBM bytes per launch of the default FP32 inter-body kernel on this workload,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE passes scaled by a calibration copy
# (profiles/interbody_sphere_lattice_27_k4pi_pmc.md); valid only for the kernel
# source they were taken on (source_fingerprint: code, not comments).
TRAFFIC_BYTES = 115.16e6
TRAFFIC_SOURCE_SHA = "c2b78089b674c037"


def source_fingerprint(path):
    """First 16 hex digits of the sha256 of a C/HIP source with its comments
    removed and its whitespace collapsed: any change of code changes it, an
    edit of comments or layout does not."""
    import hashlib
    import re
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(wl, iters_fp64, seconds_budget=15.0):
    """The FP64 reference inter-body sum on sampled rows, on the host cores,
    extrapolated to one full solve: (N / rows) x t_rows x FP64 iterations."""
    import numpy as np
    from oracle.multibody import System, apply_B_c, num_threads
    t0 = time.time()
    S = System.__new__(System)
    # node geometry only (no modal matrices needed for the inter-body sum)
    from oracle.multibody import Body
    from oracle.nystrom import Shape
    shapes = {}
    bodies = []
    for bs in wl.bodies:
        key = id(bs.contour)
        if key not in shapes:
            c = bs.contour
            shapes[key] = Shape(c.rz, c.drz, c.gw, c.n_panels, c.p, wl.kappa, wl.eta, bs.M)
        bodies.append(Body(shapes[key], bs.centre, bs.rot))
    S.__init__(bodies)
    rng = np.random.default_rng(0)
    sig = rng.standard_normal(S.N) + 1j * rng.standard_normal(S.N)
    rows = 64
    tt = 0.0
    while True:
        sel = rng.choice(S.N, size=rows, replace=False).astype(np.int64)
        t1 = time.time()
        apply_B_c(S, sig, sel)
        tt = time.time() - t1
        if tt > 0.25 * seconds_budget or rows >= S.N // 4:
            break
        rows = min(S.N // 4, rows * 4)
    per_row = tt / rows
    full = per_row * S.N
    log(f"cpu baseline: {rows} rows in {tt:.2f} s -> {full:.1f} s per operator, setup {time.time()-t0:.1f} s")
    return {
        "value": full * iters_fp64,
        "unit": "s",
        "cores": num_threads(),
        "kind": "oracle",
        "extrapolated": True,
        "rows_fraction": rows / S.N,
        "sample": (f"FP64 reference inter-body sum (C/OpenMP) on {rows} random rows of N={S.N}: "
                   f"{tt:.2f} s; x N/rows = {full:.1f} s per operator application, x {iters_fp64} "
                   f"(the FP64 GPU GMRES iteration count, one operator application each); the per-body preconditioner "
                   f"(< 0.1% of the work) and Arnoldi are not included"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--small", action="store_true", help="two-sphere workload (quick check)")
    ap.add_argument("--no-c5", action="store_true", help="leave out the 64-body leg")
    ap.add_argument("--no-c5-points", dest="c5_points", action="store_false",
                    help="leave out the 64-body leg's point-skeleton solve")
    ap.add_argument("--no-warm-start", action="store_true", help="leave out the learned warm-start leg")
    ap.add_argument("--learned", action="store_true",
                    help="learned warm start on the 8 mixed bodies: 64 wavenumbers x 64 directions of "
                         "training solves, 8 x 64 held out")
    ap.add_argument("--autotune", action="store_true", help="autotune the inter-body launch shape first")
    ap.add_argument("--batched", action="store_true",
                    help="8 uneven bodies (3 spheres, 3 spheroids, 2 bowls), kappa = 2 pi, 64 plane waves "
                         "solved as one batched multi-rhs solve")
    ap.add_argument("--many", action="store_true",
                    help="64 mixed bodies in a 24^3 box, kappa = 4 pi, N = 1.35 million, 16 plane waves: "
                         "one mixed and one FP64 batched solve (several minutes; progress on stderr)")
    ap.add_argument("--laplace", action="store_true",
                    help="zero frequency: 125 spheroids 2 x 1 x 1 on a 5^3 lattice (tips 0.05 apart), "
                         "10,100 nodes each, interior point sources; FP64 GMRES with and without the "
                         "preconditioner, mixed FGMRES, error of the exterior field")
    ap.add_argument("--laplace-table", action="store_true",
                    help="the rows of the paper's 125-ellipsoid Laplace table (Sec. 6.1; tests/golden/"
                         "laplace_125_spheroids_table.txt): FP64 GMRES to 1e-9 with and without the "
                         "preconditioner at each (N_G, N_F), field error at 10 exterior targets")
    ap.add_argument("--cavities", action="store_true",
                    help="the paper's cavity and ellipsoid experiments (Sec. 6.2, Examples 3 and 4): 8 bowls "
                         "2 and 5 wavelengths across, 8 spheroids 10 wavelengths long; FP64 GMRES to 1e-9 with "
                         "and without the preconditioner (at most 300 iterations), field error at 10 exterior "
                         "targets")
    ap.add_argument("--shard", action="store_true",
                    help="one GPU's share of the 64-body inter-body sum (16 rhs): the bodies split into 8 "
                         "contiguous groups, equal in body count or balanced by pair count; each group's rows "
                         "against all sources, FP32 and FP64, next to the full sum")
    ap.add_argument("--uniform-sources", action="store_true",
                    help="with --laplace-table: interior point sources uniform in each body's volume")
    ap.add_argument("--modal-probe", action="store_true",
                    help="time the per-mode scattering applies (MFMA GEMM) with HIP events: 27 spheres "
                         "with 1 and 16 rhs, 8 mixed bodies with 64 rhs, FP32 and FP64; also the launches "
                         "the matrix-core counter passes measure")
    ap.add_argument("--skeleton", action="store_true",
                    help="the 27-sphere benchmark through the ring skeletonization of Sec. 5: ID time, "
                         "ranks, compressed mixed and FP64 solves, full-system residual of the lifted density")
    ap.add_argument("--many-points", action="store_true",
                    help="the 64-body workload (16 plane waves) through point skeletons only: ID at eps "
                         "1e-10, one warm-up and one timed mixed solve, full-system residual")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="launch only what the hardware-counter passes measure: a 512 MiB device copy "
                         "(calibration), then two FP32 and one FP64 inter-body sums on the 27 spheres, "
                         "and FP32 64-rhs sums on the 8 mixed bodies: two with FP32 MFMAs, two with the FP16 "
                         "multiply-accumulate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "its decomposition over several GPUs is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1406_0236_amd import FP32, FP64, SOLVE_FP64, SOLVE_MIXED, Context
    from workloads import configs

    if args.learned:
        return learned(args)
    if args.pmc_probe:
        return pmc_probe()
    if args.modal_probe:
        return modal_probe()
    if args.batched:
        return batched(args)
    if args.many:
        return many(args)
    if args.laplace:
        return laplace(args)
    if args.laplace_table:
        return laplace_table(args)
    if args.cavities:
        return cavities(args)
    if args.shard:
        return shard(args)
    if args.skeleton:
        return skeleton(args)
    if args.many_points:
        return many_points(args)

    t_start = time.time()
    wl = configs.two_spheres() if args.small else configs.sphere_lattice()
    log(f"workload {wl.name}: N={wl.N}, pairs={wl.pairs:.4g}")
    torch.cuda.init()
    ctx = Context(0).add_workload(wl)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.precompute_scattering()
    torch.cuda.synchronize()
    t_pre = time.time() - t0
    log(f"precompute (FP64, GPU) {t_pre:.2f} s")
    v = ctx.incident_plane_waves(wl.dirs)
    torch.cuda.synchronize()
    tuned = None
    if args.autotune:
        from paper_1406_0236_amd import autotune
        tuned = {}
        for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
            cfg, tim = autotune.tune(ctx, prec, 1, ctx.max_nf, x=v, reps=1, cache_path=None,
                                     verbose=True)
            tuned[name] = {"config": cfg, "ms": min(tim.values())}
        log(f"autotuned: {tuned}")

    infos = []
    for w in range(args.warmup):
        _, info = ctx.solve(v, mode=SOLVE_MIXED, tol=args.tol)
        log(f"warmup {w}: {info[0]}")
    torch.cuda.synchronize()
    t0 = time.time()
    for s in range(args.steps):
        sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=args.tol)
        infos.append(info[0])
    torch.cuda.synchronize()
    t_mixed = (time.time() - t0) / args.steps
    log(f"mixed: {t_mixed:.3f} s/solve, {infos[-1]}")
    # the explicit FP64 residual of the returned sigma (one more application, untimed)
    b_ = ctx.apply_precond(v, FP64)
    explicit_res = float(torch.linalg.norm(ctx.apply_matvec(sol, FP64) + b_) / torch.linalg.norm(b_))
    log(f"mixed: explicit FP64 residual of the returned solution {explicit_res:.3e}")

    fp64 = None
    if not args.no_fp64:
        torch.cuda.synchronize()
        t0 = time.time()
        sol64, info64 = ctx.solve(v, mode=SOLVE_FP64, tol=args.tol)
        torch.cuda.synchronize()
        t64 = time.time() - t0
        fp64 = {"s": t64, **info64[0]}
        diff = float(torch.linalg.norm(sol - sol64) / torch.linalg.norm(sol64))
        fp64["rel_diff_vs_mixed"] = diff
        log(f"fp64: {t64:.3f} s/solve, {info64[0]}, |mixed - fp64|/|fp64| = {diff:.2e}")

    # dominant kernel: FP32 inter-body sum, HIP events on the library stream
    shape32, shape64 = ctx.interbody_launch_shape(FP32), ctx.interbody_launch_shape(FP64)
    kname = {1: "interbody_kernel<float>", 2: "interbody_ring_kernel<float>",
             3: "interbody_mfma_kernel"}[shape32[0]]
    ctx.set_timing(True)
    x = sol.clone()
    ms = []
    for _ in range(4):
        ctx.apply_interbody(x, FP32)
        ms.append(ctx.last_timing()["interbody"])
    ms64 = []
    for _ in range(2):
        ctx.apply_interbody(x, FP64)
        ms64.append(ctx.last_timing()["interbody"])
    variants = {}
    for prec, pname in ((FP32, "fp32"), (FP64, "fp64")):
        for var, vname in ((1, "points"), (2, "rings"), (3, "mfma")):
            if var == 3 and prec != FP32:
                continue
            ctx.set_interbody_config(prec, var, 0, 0, 0)
            t = []
            for _ in range(2):
                ctx.apply_interbody(x, prec)
                t.append(ctx.last_timing()["interbody"])
            variants[f"{pname}_{vname}_ms"] = float(np.min(t))
        ctx.set_interbody_config(prec, 0, 0, 0, 0)
    log(f"inter-body sum by source order: {variants}")
    # far-field pattern of the solution in 4096 Fibonacci directions (FP64)
    from workloads import geometry as geo_
    xh = geo_.fibonacci_directions(4096)
    ctx.far_field(sol, xh)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.far_field(sol, xh)
    torch.cuda.synchronize()
    t_ff = time.time() - t0
    far = {"directions": 4096, "ms": t_ff * 1e3, "gevals_per_s": 4096 * wl.N / t_ff / 1e9}
    log(f"far field: {far}")
    ctx.apply_matvec(x, FP32)
    stage32 = ctx.last_timing()
    ctx.apply_matvec(x, FP64)
    stage64 = ctx.last_timing()
    ctx.set_timing(False)
    t_ib = float(np.median(ms)) * 1e-3
    t_ib64 = float(np.median(ms64)) * 1e-3
    pairs = wl.pairs
    flops = FLOP_PER_PAIR * pairs
    sha = source_fingerprint(os.path.join(ROOT, "paper_1406_0236_amd", "csrc", "interbody.hip"))
    traffic = TRAFFIC_BYTES if (sha == TRAFFIC_SOURCE_SHA and not args.small and tuned is None) else None
    achieved = flops / t_ib / 1e12
    log(f"interbody fp32 {t_ib*1e3:.2f} ms ({pairs / t_ib / 1e9:.1f} Gpairs/s, {achieved:.2f} TFLOP/s); "
        f"fp64 {t_ib64*1e3:.2f} ms; stages fp32 {stage32} fp64 {stage64}")

    # the same problem through the ring skeletonization of Sec. 5 (reported
    # beside the step; the step itself is the uncompressed solve)
    skel = None
    if not args.small:
        torch.cuda.synchronize()
        t0 = time.time()
        ns = ctx.skeletonize(1e-8, 2.0)
        torch.cuda.synchronize()
        t_id = time.time() - t0
        ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=args.tol)     # warm-up
        torch.cuda.synchronize()
        t0 = time.time()
        sk, info_sk = ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=args.tol)
        torch.cuda.synchronize()
        t_sk = time.time() - t0
        b_ = ctx.apply_precond(v, FP64)
        res_sk = float(torch.linalg.norm(ctx.apply_matvec(sk, FP64) + b_) / torch.linalg.norm(b_))
        skel = {"eps": 1e-8, "rings": list(ctx.skeleton_rank(0)), "unknowns": ns, "skeletonize_s": t_id,
                "mixed_s": t_sk, "outer": info_sk[0]["iterations"], "inner": info_sk[0]["inner_iterations"],
                "full_rel_residual": res_sk}
        log(f"skeleton: {skel}")
        # point skeletons (the randomized ID of single nodes); eps 1e-10 keeps the
        # lifted density's full-system residual below the 1e-7 target
        skel["points"] = point_skeleton_leg(ctx, v, args.tol, 1e-10, sol)

    cpu = None
    if not args.no_cpu_baseline:
        iters = fp64["iterations"] if fp64 else 30
        cpu = cpu_baseline(wl, iters)

    out = {
        # the headline metric as stated for this benchmark family; on this
        # workload no learned guess is trained (config.warm_start), so "mixed"
        # is the mixed-precision solve from the zero guess
        "metric": "s to 1e-7 residual (mixed+warm vs FP64); far-field Gpairs/s; % VALU peak",
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "bodies": len(wl.bodies), "N": wl.N, "kappa": wl.kappa,
                   "modes": wl.bodies[0].M, "nodes_per_contour": wl.bodies[0].contour.NG, "nrhs": 1,
                   "tol": args.tol, "warm_start": False},
        "mixed": {"s": t_mixed, **infos[-1], "explicit_rel_residual": explicit_res,
                  "residual": "GMRES least squares in the FP64 Arnoldi basis"},
        "fp64": fp64,
        "speedup_mixed_vs_fp64": (fp64["s"] / t_mixed) if fp64 else None,
        "precompute_s": t_pre,
        "interbody_pairs": pairs,
        "gpairs_per_s_fp32": pairs / t_ib / 1e9,
        "gpairs_per_s_fp64": pairs / t_ib64 / 1e9,
        "pct_fp32_valu_peak": 100.0 * achieved / FP32_VECTOR_PEAK_TFLOPS,
        "interbody_ms_by_variant": variants,
        "interbody_launch_shape": {"fp32": list(shape32), "fp64": list(shape64)},
        "far_field": far,
        "stage_ms_fp32": stage32,
        "stage_ms_fp64": stage64,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": f"{kname} (FP32 inter-body sum), launch shape {list(shape32)}",
                     "flop_per_launch": flops, "launch_ms": t_ib * 1e3},
        "skeleton": skel,
        "cpu_baseline": cpu,
        "autotuned": tuned,
    }
    ctx.close()
    del ctx, v, sol, x
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # the other legs, each only if the run stays well inside ten minutes
    # (estimates from measured runs: 64 bodies about 200 s, warm start about 60 s)
    if not args.small and not args.no_c5:
        left = 600.0 - (time.time() - t_start)
        out["c5"] = c5_leg(args) if left > 330.0 else {"skipped": f"{left:.0f} s left of a 600 s run"}
        torch.cuda.empty_cache()
    if not args.small and not args.no_warm_start:
        left = 600.0 - (time.time() - t_start)
        out["warm_start"] = warm_start_leg() if left > 120.0 else {"skipped": f"{left:.0f} s left of a 600 s run"}
    out["wall_s"] = time.time() - t_start
    print(json.dumps(out), flush=True)


def c5_leg(args):
    """64 mixed bodies, 16 plane waves: one mixed and one FP64 batched solve to
    args.tol from the zero guess (no network is trained for this geometry),
    library default launch shapes; explicit FP64 residuals of both solutions."""
    import torch
    from paper_1406_0236_amd import FP64, SOLVE_FP64, SOLVE_MIXED, Context
    from workloads import configs
    wl = configs.mixed_many()
    r = len(wl.dirs)
    log(f"c5: workload {wl.name}: N={wl.N}, pairs={wl.pairs:.4g}, rhs={r}")
    ctx = Context(0).add_workload(wl)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.precompute_scattering()
    torch.cuda.synchronize()
    t_pre = time.time() - t0
    v = ctx.incident_plane_waves(wl.dirs)
    b_ = ctx.apply_precond(v, FP64)
    bn = torch.linalg.norm(b_, dim=1)
    res = {}
    ref = None
    for mode, name in ((SOLVE_MIXED, "mixed"), (SOLVE_FP64, "fp64")):
        torch.cuda.synchronize()
        t0 = time.time()
        sol, info = ctx.solve(v, mode=mode, tol=args.tol)
        torch.cuda.synchronize()
        dt = time.time() - t0
        expl = (torch.linalg.norm(ctx.apply_matvec(sol, FP64) + b_, dim=1) / bn).max().item()
        res[name] = {"s": dt, "outer": max(i["iterations"] for i in info),
                     "inner": max(i["inner_iterations"] for i in info),
                     "max_rel_residual": max(i["rel_residual"] for i in info),
                     "max_explicit_rel_residual": expl, "converged": all(i["converged"] for i in info)}
        log(f"c5 {name}: {dt:.1f} s, {res[name]}")
        if name == "mixed":
            ref = sol
        del sol
    # the same 16 rhs through point skeletons of Sec. 5 (one ID per body shape)
    points = point_skeleton_leg(ctx, v, args.tol, 1e-10, ref) if args.c5_points else None
    del ref
    ctx.close()
    out = {"workload": wl.name, "bodies": len(wl.bodies), "N": wl.N, "kappa": wl.kappa, "nrhs": r,
           "tol": args.tol, "precompute_s": t_pre, "interbody_pairs": wl.pairs, **res,
           "speedup_mixed_vs_fp64": res["fp64"]["s"] / res["mixed"]["s"],
           "initial_guess": "zero (the learned warm start is trained for the 8-body geometry only)"}
    if points is not None:
        out["skeleton_points"] = points
    return out


def warm_start_leg(n_k=64, n_d=64, held_k=8, held_d=64, epochs=200, log_fn=None):
    """The learned warm start on the 8 mixed bodies: training set of n_k
    wavenumbers x n_d directions (seed 4), held out held_k x held_d (seed 40)."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import Context
    from paper_1406_0236_amd import warmstart as W
    from workloads import configs
    log_fn = log_fn or log
    wl_at = lambda k: configs.mixed_bodies(kappa=k, disc_kappa=W.K_MAX, n_dirs=1)
    rng = np.random.default_rng(4)
    ks = rng.uniform(W.K_MIN, W.K_MAX, n_k)
    dirs = [W.random_directions(n_d, rng) for _ in ks]
    t0 = time.time()
    X, Y = W.generate(wl_at, ks, dirs, mmax=8, tol=1e-8)
    t_gen = time.time() - t0
    log_fn(f"warm start: training set {X.shape[0]} solves, {Y.shape[1]} outputs, {t_gen:.1f} s")
    dev = Context(0)
    ws = W.WarmStart(dev, Y.shape[1], width=512, depth=4)
    hist = ws.train(X, Y, epochs=epochs, batch=256, lr=1e-3, log=log_fn)
    del X, Y
    rng2 = np.random.default_rng(40)
    hk = rng2.uniform(W.K_MIN, W.K_MAX, held_k)
    hd = [W.random_directions(held_d, rng2) for _ in hk]
    rows = W.evaluate(ws, wl_at, hk, hd, tol=1e-7, log=log_fn)
    agg = W.summarise(rows)
    wl = wl_at(W.K_MAX)
    out = {"workload": "mixed8_seed3 at k in [1.5 pi, 2.5 pi], discretised at 2.5 pi", "N": wl.N,
           "train_solves": n_k * n_d, "held_out": held_k * held_d, "m_max": 8,
           "mlp": ws.mlp.sizes, "epochs": epochs, "batch": 256,
           "train_loss_first_last": [hist[0], hist[-1]], "train_s": ws.train_seconds, "generate_s": t_gen,
           "held_out_mean": agg,
           "learned_vs_single_body": {
               "guess_residual_ratio": agg["learned"]["guess_rel_residual"] / agg["single_body"]["guess_rel_residual"],
               "fp64_iters_saved": agg["single_body"]["fp64_iters"] - agg["learned"]["fp64_iters"],
               "mixed_s_ratio": agg["learned"]["mixed_s"] / agg["single_body"]["mixed_s"]},
           "seconds_note": "per 64-rhs solve, mean over the held-out wavenumbers; the learned guess includes "
                           "its prediction"}
    ws.mlp.close()
    dev.close()
    torch.cuda.empty_cache()
    return out


def learned(args):
    """The warm-start leg alone, as its own JSON line."""
    out = warm_start_leg()
    a = out["held_out_mean"]["learned"]
    print(json.dumps({
        "metric": "s to 1e-7 residual with the learned warm start (64 rhs per solve)",
        "value": a["mixed_s"], "unit": "s", "n_gpus": 1, "steps": out["held_out"] // 64, "warmup": 0,
        "ms_per_step": a["mixed_s"] * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic", "config": {"workload": out["workload"], "N": out["N"]},
        "warm_start": out}), flush=True)


def pmc_probe():
    """Known-size copy for counter calibration, then the dominant kernels."""
    import torch
    from paper_1406_0236_amd import FP32, FP64, Context
    from workloads import configs
    n = 512 * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log("calibration copy: 512 MiB read + 512 MiB written")
    wl = configs.sphere_lattice()
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    v = ctx.incident_plane_waves(wl.dirs)
    for prec in (FP32, FP32, FP64):
        ctx.apply_interbody(v, prec)
        torch.cuda.synchronize()
    log("inter-body sums done")
    ctx.close()
    # the MFMA order with 16-rhs groups: 8 mixed bodies, 64 plane waves
    wl = configs.mixed_bodies()
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    v = ctx.incident_plane_waves(wl.dirs)
    # the FP32 MFMA order, then the default (FP16 multiply-accumulate), twice each
    for variant in (3, 3, 0, 0):
        ctx.set_interbody_config(FP32, variant, 0, 0, 0)
        ctx.apply_interbody(v, FP32)
        torch.cuda.synchronize()
        log(f"64-rhs inter-body sum done ({ctx.interbody_launch_shape(FP32, len(wl.dirs))})")
    ctx.close()


def many(args):
    """One mixed and one FP64 solve of 16 plane waves on the 64-body workload,
    library default launch shapes (for 16 rhs: in FP32 the MFMA order with the FP16
    multiply-accumulate, in FP64 the MFMA order)."""
    import numpy as np
    import torch
    os.environ.setdefault("AXS_VERBOSE", "1")     # one progress line per iteration
    from paper_1406_0236_amd import FP32, FP64, SOLVE_FP64, SOLVE_MIXED, Context
    from workloads import configs
    wl = configs.mixed_many()
    r = len(wl.dirs)
    log(f"workload {wl.name}: N={wl.N}, pairs={wl.pairs:.4g}, rhs={r}")
    ctx = Context(0).add_workload(wl)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.precompute_scattering()
    torch.cuda.synchronize()
    t_pre = time.time() - t0
    log(f"precompute {t_pre:.1f} s")
    v = ctx.incident_plane_waves(wl.dirs)
    ctx.set_timing(True)
    ctx.apply_interbody(v, FP32)
    t_ib = ctx.last_timing()["interbody"] * 1e-3
    ctx.apply_interbody(v, FP64)
    t_ib64 = ctx.last_timing()["interbody"] * 1e-3
    ctx.set_timing(False)
    log(f"inter-body sum, {r} rhs: FP32 {t_ib:.3f} s ({wl.pairs * r / t_ib / 1e9:.0f} G pair-rhs/s), "
        f"FP64 {t_ib64:.3f} s")
    torch.cuda.synchronize()
    t0 = time.time()
    sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=args.tol)
    torch.cuda.synchronize()
    t_mixed = time.time() - t0
    log(f"mixed {t_mixed:.1f} s (outer {info[0]['iterations']}, inner {info[0]['inner_iterations']})")
    t0 = time.time()
    sol64, info64 = ctx.solve(v, mode=SOLVE_FP64, tol=args.tol)
    torch.cuda.synchronize()
    t64 = time.time() - t0
    log(f"fp64 {t64:.1f} s (iterations {max(i['iterations'] for i in info64)})")
    b_ = ctx.apply_precond(v, FP64)
    res = (torch.linalg.norm(ctx.apply_matvec(sol, FP64) + b_, dim=1) / torch.linalg.norm(b_, dim=1)).max().item()
    # the same solve through the ring skeletonization of Sec. 5
    torch.cuda.synchronize()
    t0 = time.time()
    ns = ctx.skeletonize(1e-8, 2.0)
    torch.cuda.synchronize()
    t_id = time.time() - t0
    t0 = time.time()
    sk, info_sk = ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=args.tol)
    torch.cuda.synchronize()
    t_sk = time.time() - t0
    res_sk = (torch.linalg.norm(ctx.apply_matvec(sk, FP64) + b_, dim=1) / torch.linalg.norm(b_, dim=1)).max().item()
    log(f"skeleton: {ns} of {wl.N} unknowns, ID {t_id:.1f} s, mixed solve {t_sk:.1f} s, full residual {res_sk:.2e}")
    flops = wl.pairs * (FLOP_PER_PAIR + FLOP_PER_EXTRA_RHS * (r - 1))
    out = {
        "metric": "s to 1e-7 residual, 16 rhs batched (mixed vs FP64 GMRES)",
        "value": t_mixed, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": t_mixed * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "bodies": len(wl.bodies), "N": wl.N, "kappa": wl.kappa, "nrhs": r,
                   "tol": args.tol},
        "mixed": {"s": t_mixed, "outer": max(i["iterations"] for i in info),
                  "inner": max(i["inner_iterations"] for i in info),
                  "max_rel_residual": max(i["rel_residual"] for i in info),
                  "max_explicit_rel_residual": res},
        "fp64": {"s": t64, "iterations": max(i["iterations"] for i in info64),
                 "max_rel_residual": max(i["rel_residual"] for i in info64)},
        "speedup_mixed_vs_fp64": t64 / t_mixed,
        "precompute_s": t_pre,
        "interbody_s": {"fp32": t_ib, "fp64": t_ib64},
        "interbody_launch_shape": {"fp32": list(ctx.interbody_launch_shape(FP32, r)),
                                   "fp64": list(ctx.interbody_launch_shape(FP64, r))},
        "tflops_fp32_algorithmic": flops / t_ib / 1e12,
        "skeleton": {"unknowns": ns, "skeletonize_s": t_id, "mixed_s": t_sk,
                     "outer": max(i["iterations"] for i in info_sk),
                     "inner": max(i["inner_iterations"] for i in info_sk), "max_full_rel_residual": res_sk},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def laplace(args):
    """The zero-frequency problem of the paper's first Laplace example (Sec. 6.1):
    the same solve with and without the block-diagonal preconditioner, and the
    error of the exterior field against the exact one of the interior sources."""
    import numpy as np
    import torch
    os.environ.setdefault("AXS_VERBOSE", "1")
    from paper_1406_0236_amd import FP32, FP64, SOLVE_FP64, SOLVE_MIXED, Context
    from workloads import configs
    wl = configs.laplace_ellipsoids()
    tol = 1e-9
    log(f"workload {wl.name}: N={wl.N}, pairs={wl.pairs:.4g}")
    ctx = Context(0).add_workload(wl)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.precompute_scattering()
    torch.cuda.synchronize()
    t_pre = time.time() - t0
    src = configs.point_sources(wl, seed=11)
    amp = np.random.default_rng(12).standard_normal(len(src))
    v = ctx.incident_point_sources(src, amp)
    ctx.set_timing(True)
    ib = {}
    for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
        t = []
        for _ in range(2):
            ctx.apply_interbody(v, prec)
            t.append(ctx.last_timing()["interbody"])
        ib[name] = {"ms": min(t), "gpairs_per_s": wl.pairs / min(t) / 1e6,
                    "launch_shape": list(ctx.interbody_launch_shape(prec))}
    ctx.set_timing(False)
    log(f"inter-body sum: {ib}")
    runs = {}
    for name, mode, pre in (("fp64", SOLVE_FP64, True), ("fp64_unpreconditioned", SOLVE_FP64, False),
                            ("mixed", SOLVE_MIXED, True)):
        torch.cuda.synchronize()
        t0 = time.time()
        sol, info = ctx.solve(v, mode=mode, tol=tol, precondition=pre)
        torch.cuda.synchronize()
        dt = time.time() - t0
        xt = configs.exterior_targets(wl, 10, seed=12)
        u = ctx.eval_field(sol, xt).cpu().numpy()[0]
        d = xt[:, None, :] - src[None, :, :]
        exact = -(1.0 / (4.0 * math.pi * np.linalg.norm(d, axis=-1))) @ amp
        err = float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))
        runs[name] = {"s": dt, "iterations": info[0]["iterations"], "inner": info[0]["inner_iterations"],
                      "rel_residual": info[0]["rel_residual"], "field_rel_err": err}
        log(f"{name}: {runs[name]}")
    out = {
        "metric": "s to 1e-9 residual at zero frequency (Laplace), with / without preconditioner",
        "value": runs["mixed"]["s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": runs["mixed"]["s"] * 1e3, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "bodies": len(wl.bodies), "N": wl.N, "kappa": 0.0, "eta": 1.0,
                   "tol": tol},
        "solves": runs, "interbody": ib, "precompute_s": t_pre,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def laplace_table(args):
    """The paper's 125-ellipsoid Laplace table, row by row, on the lattice
    reading of its geometry: FP64 GMRES to 1e-9 with and without the
    block-diagonal preconditioner, and the relative l-infinity error of the
    exterior field at 10 targets against the exact field of the interior point
    sources, printed next to the paper's values (its times are other hardware's
    and not compared)."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import SOLVE_FP64, Context
    from workloads import configs
    rows = np.loadtxt(os.path.join(ROOT, "tests", "golden", "laplace_125_spheroids_table.txt"))
    out_rows = []
    for N, NG, NF, i_pre, i_no, e_paper in rows:
        NG, NF = int(NG), int(NF)
        wl = configs.laplace_ellipsoids(n_panels=NG // 10, p=10, M=(NF - 1) // 2)
        assert wl.N == int(N), (wl.N, N)
        ctx = Context(0).add_workload(wl)
        ctx.precompute_scattering()
        # sources near each centre (the default reading), or anywhere in the
        # body's volume (--uniform-sources), whose fields on the surface need
        # more Fourier modes and panels
        src = configs.point_sources(wl, seed=11, uniform=args.uniform_sources)
        amp = np.random.default_rng(12).standard_normal(len(src))
        v = ctx.incident_point_sources(src, amp)
        res = {}
        for name, pre in (("pre", True), ("nopre", False)):
            torch.cuda.synchronize()
            t0 = time.time()
            sol, info = ctx.solve(v, mode=SOLVE_FP64, tol=1e-9, precondition=pre)
            torch.cuda.synchronize()
            res[name] = {"s": time.time() - t0, "iterations": info[0]["iterations"]}
            if pre:
                xt = configs.exterior_targets(wl, 10, seed=12)
                u = ctx.eval_field(sol, xt).cpu().numpy()[0]
                d = xt[:, None, :] - src[None, :, :]
                exact = -(1.0 / (4.0 * math.pi * np.linalg.norm(d, axis=-1))) @ amp
                res["e_inf"] = float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))
        ctx.close()
        row = {"workload": wl.name, "N": wl.N, "N_G": NG, "N_F": NF,
               "iterations_pre": res["pre"]["iterations"], "iterations_nopre": res["nopre"]["iterations"],
               "e_inf": res["e_inf"], "s_pre": res["pre"]["s"], "s_nopre": res["nopre"]["s"],
               "paper": {"iterations_pre": int(i_pre), "iterations_nopre": int(i_no), "e_inf": e_paper}}
        log(f"{wl.name} {NG} x {NF}: N = {wl.N}, iterations {row['iterations_pre']} / {row['iterations_nopre']} "
            f"(paper {int(i_pre)} / {int(i_no)}), E_inf {res['e_inf']:.3e} (paper {e_paper:.3e}), "
            f"FP64 solves {res['pre']['s']:.1f} / {res['nopre']['s']:.1f} s")
        out_rows.append(row)
    out = {"metric": "the paper's 125-ellipsoid Laplace table: iterations to 1e-9 with / without the "
                     "preconditioner and field error", "unit": "rows", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "laplace_ellipsoids_125", "kappa": 0.0, "eta": 1.0, "tol": 1e-9,
                      "sources": "one per body, " + ("uniform in its volume" if args.uniform_sources
                                                     else "within half the inradius of its centre")
                                 + " (seed 11)"},
           "rows": out_rows}
    print(json.dumps(out), flush=True)


def cavities(args):
    """8 bowl cavities with interior point sources: the paper's observation that
    for cavities the block-diagonal preconditioner is essential (without it
    GMRES does not converge); and 8 ellipsoids 10 wavelengths long, where it
    halves the iteration count.  FP64 GMRES to 1e-9 with and without it, capped
    at 300 iterations, and the field error at 10 exterior targets against the
    exact field of the sources."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import SOLVE_FP64, SOLVE_MIXED, Context
    from workloads import configs
    rows = []
    cases = [configs.cavities_8(kappa=2 * math.pi, panels_per_unit=20.0 / math.pi, M=25),
             configs.cavities_8(kappa=5 * math.pi, panels_per_unit=50.0 / math.pi, M=50),
             # the paper's Example 3: 8 ellipsoids 10 wavelengths long, where the
             # preconditioner halves the iterations
             configs.ellipsoids_8(n_panels=10, M=50), configs.ellipsoids_8(n_panels=20, M=100)]
    for wl in cases:
        kappa, M = wl.kappa, wl.bodies[0].M
        ctx = Context(0).add_workload(wl)
        torch.cuda.synchronize()
        t0 = time.time()
        ctx.precompute_scattering()
        torch.cuda.synchronize()
        t_pre = time.time() - t0
        src = configs.point_sources(wl, seed=11)
        amp = np.random.default_rng(12).standard_normal(len(src))
        v = ctx.incident_point_sources(src, amp)
        xt = configs.exterior_targets(wl, 10, seed=12)
        d = xt[:, None, :] - src[None, :, :]
        dist = np.linalg.norm(d, axis=-1)
        exact = -(np.exp(1j * kappa * dist) / (4.0 * math.pi * dist)) @ amp
        row = {"workload": wl.name, "N": wl.N, "N_G": wl.bodies[0].contour.NG, "N_F": 2 * M + 1,
               "precompute_s": t_pre}
        for name, mode, pre in (("fp64", SOLVE_FP64, True), ("fp64_unpreconditioned", SOLVE_FP64, False),
                                ("mixed", SOLVE_MIXED, True)):
            torch.cuda.synchronize()
            t0 = time.time()
            sol, info = ctx.solve(v, mode=mode, tol=1e-9, max_iters=300, precondition=pre)
            torch.cuda.synchronize()
            u = ctx.eval_field(sol, xt).cpu().numpy()[0]
            row[name] = {"s": time.time() - t0, "iterations": info[0]["iterations"],
                         "inner": info[0]["inner_iterations"], "converged": bool(info[0]["converged"]),
                         "rel_residual": info[0]["rel_residual"],
                         "e_inf": float(np.max(np.abs(u - exact)) / np.max(np.abs(exact)))}
            log(f"{wl.name} N={wl.N}: {name} {row[name]}")
        ctx.close()
        rows.append(row)
    out = {"metric": "GMRES iterations to 1e-9 on 8 cavities and 8 ellipsoids with / without the preconditioner",
           "unit": "rows", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "cavities8, ellipsoids8", "sources": "one inside each body (seed 11)",
                      "tol": 1e-9},
           "rows": rows}
    print(json.dumps(out), flush=True)


def shard(args, n_gpus=8):
    """The inter-body sum of the 64-body workload (16 rhs) cut by block rows as
    it would be over n_gpus GPUs: each share is a contiguous group of bodies
    whose targets meet every source (axs_set_target_bodies).  Two cuts: equal
    body counts, and contiguous groups balanced by pairs n_b (N - n_b).  Each
    share is timed on this GPU with HIP events; the largest share bounds the
    sharded sum (before the all-gather of the staged densities)."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import FP32, FP64, Context
    from workloads import configs
    wl = configs.mixed_many()
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    n = np.array([b.n_nodes for b in wl.bodies], dtype=np.int64)
    N = int(n.sum())
    pairs = n * (N - n)
    B = len(n)
    equal = [(i * B // n_gpus, (i + 1) * B // n_gpus) for i in range(n_gpus)]
    # contiguous groups with the smallest largest pair count: bisection on the
    # bound L, greedy filling decides whether n_gpus groups suffice

    def greedy(L):
        cuts, acc = [0], 0
        for i, p_ in enumerate(pairs):
            if acc + p_ > L and acc > 0:
                cuts.append(i)
                acc = 0
            acc += p_
        return cuts + [B]

    lo_, hi_ = float(pairs.max()), float(pairs.sum())
    for _ in range(60):
        mid = 0.5 * (lo_ + hi_)
        if len(greedy(mid)) - 1 <= n_gpus:
            hi_ = mid
        else:
            lo_ = mid
    cuts = greedy(hi_)
    while len(cuts) - 1 < n_gpus:   # split the largest group until there are n_gpus
        k = max(range(len(cuts) - 1), key=lambda g: cuts[g + 1] - cuts[g])
        cuts.insert(k + 1, (cuts[k] + cuts[k + 1]) // 2)
    balanced = [(cuts[i], cuts[i + 1]) for i in range(n_gpus)]
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.standard_normal((16, N)) + 1j * rng.standard_normal((16, N))).to("cuda:0")
    ctx.set_timing(True)

    def timed():
        ctx.apply_interbody(x, prec)
        return ctx.last_timing()["interbody"]

    out_prec = {}
    for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
        full = timed()
        res = {"full_ms": full, "launch_shape": list(ctx.interbody_launch_shape(prec, 16))}
        for cut_name, cut in (("equal_bodies", equal), ("balanced_pairs", balanced)):
            ms = []
            for b0, b1 in cut:
                ctx.set_target_bodies(b0, b1 - b0)
                ms.append(timed())
            ctx.set_target_bodies(0, 0)
            share = [float(pairs[b0:b1].sum() / pairs.sum()) for b0, b1 in cut]
            res[cut_name] = {"bodies": cut, "ms": ms, "pair_share": share, "max_ms": max(ms),
                             "ideal_ms": full / n_gpus, "efficiency": full / n_gpus / max(ms)}
            log(f"{name} {cut_name}: full {full:.1f} ms, shares {[round(v, 1) for v in ms]} ms, "
                f"largest {max(ms):.1f} ms vs ideal {full / n_gpus:.1f} ms")
        out_prec[name] = res
    ctx.set_timing(False)
    ctx.close()
    q_bytes = 16 * N * 8
    out = {"metric": f"inter-body sum of one GPU's share of the block rows ({n_gpus} shares), 16 rhs",
           "unit": "ms", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": wl.name, "N": N, "bodies": B, "nrhs": 16, "shares": n_gpus},
           "allgather_bytes_per_application_fp32": q_bytes, "results": out_prec}
    print(json.dumps(out), flush=True)


def modal_probe():
    """Per-mode scattering applies alone (axs_apply_precond: forward DFT, the
    S_m GEMMs on MFMA, inverse DFT), timed per stage with the library's HIP
    events.  Algorithmic flops of the GEMM stage: 8 NG^2 per column (four real
    products per complex one), columns = 2 modes (+-m, one for m = 0) x bodies
    x rhs per shape and mode."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import FP32, FP64, Context
    from workloads import configs
    rows = []
    for wl, nrs in ((configs.sphere_lattice(), (1, 16)), (configs.mixed_bodies(), (64,))):
        ctx = Context(0).add_workload(wl)
        ctx.precompute_scattering()
        shapes = {}
        for b in wl.bodies:
            key = (id(b.contour), b.M)
            shapes.setdefault(key, [b.contour.NG, b.M, 0])[2] += 1
        for r in nrs:
            flops = sum(8.0 * NG * NG * nb * (2 * M + 1) * r for NG, M, nb in shapes.values())
            g = torch.Generator(device="cuda:0").manual_seed(3)
            x = torch.randn((r, wl.N), dtype=torch.complex128, device="cuda:0", generator=g)
            for prec, pname, peak in ((FP32, "fp32", 157.3), (FP64, "fp64", 78.6)):
                ctx.set_timing(True)
                ms = []
                for _ in range(5):
                    ctx.apply_precond(x, prec)
                    ms.append(ctx.last_timing()["modal_apply"])
                ctx.set_timing(False)
                t = float(np.median(ms))
                row = {"workload": wl.name, "nrhs": r, "precision": pname, "gemm_ms": t,
                       "gemm_tflops": flops / t / 1e9, "mfma_frac": flops / t / 1e9 / peak}
                rows.append(row)
                log(f"modal GEMM {row}")
        ctx.close()
    print(json.dumps({"modal_gemm": rows}), flush=True)


def point_skeleton_leg(ctx, v, tol, eps=1e-8, ref=None):
    """The same problem through point skeletons (single-node index sets, the
    randomized ID): ID time, unknowns, one mixed solve after a warm-up, the
    full-system residual of the lifted density."""
    import torch
    from paper_1406_0236_amd import FP64, SOLVE_MIXED
    torch.cuda.synchronize()
    t0 = time.time()
    ns = ctx.skeletonize_points(eps, 2.0, 0, 1)
    torch.cuda.synchronize()
    t_id = time.time() - t0
    k, n = ctx.skeleton_rank(0)
    log(f"point skeletons (eps {eps}): {t_id:.2f} s, {k} of {n} nodes per body, {ns} unknowns")
    ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=tol)          # warm-up
    torch.cuda.synchronize()
    t0 = time.time()
    sol, info = ctx.solve_skeleton(v, mode=SOLVE_MIXED, tol=tol)
    torch.cuda.synchronize()
    t_s = time.time() - t0
    b_ = ctx.apply_precond(v, FP64)
    res = float((torch.linalg.norm(ctx.apply_matvec(sol, FP64) + b_, dim=1) / torch.linalg.norm(b_, dim=1)).max())
    out = {"eps": eps, "nodes": [k, n], "unknowns": ns, "skeletonize_s": t_id, "mixed_s": t_s,
           "outer": max(i["iterations"] for i in info), "inner": max(i["inner_iterations"] for i in info),
           "full_rel_residual": res}
    if ref is not None:
        out["rel_diff_vs_uncompressed"] = float(torch.linalg.norm(sol - ref) / torch.linalg.norm(ref))
    log(f"point skeleton solve: {out}")
    return out


def many_points(args, eps=1e-10):
    """The 64-body workload's 16 plane waves through point skeletons only (one
    randomized ID per body shape): the leg `c5.skeleton_points` of the default
    line, on its own (for kernel traces)."""
    import torch
    from paper_1406_0236_amd import Context
    from workloads import configs
    wl = configs.mixed_many()
    log(f"workload {wl.name}: N={wl.N}, rhs={len(wl.dirs)}")
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    v = ctx.incident_plane_waves(wl.dirs)
    torch.cuda.synchronize()
    pts = point_skeleton_leg(ctx, v, args.tol, eps)
    ctx.close()
    print(json.dumps({"metric": "s to 1e-7 residual of the compressed system (Sec. 5 point skeletons), 16 rhs",
                      "value": pts["mixed_s"], "unit": "s", "higher_is_better": False,
                      "config": {"workload": wl.name, "N": wl.N, "nrhs": len(wl.dirs), "tol": args.tol},
                      "skeleton_points": pts}), flush=True)


def skeleton(args, eps=1e-8):
    """The benchmark problem solved through the compressed system of Sec. 5."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import FP32, FP64, SOLVE_FP64, SOLVE_MIXED, Context
    from workloads import configs
    wl = configs.sphere_lattice()
    ctx = Context(0).add_workload(wl)
    ctx.precompute_scattering()
    v = ctx.incident_plane_waves(wl.dirs)
    torch.cuda.synchronize()
    t0 = time.time()
    ns = ctx.skeletonize(eps, 2.0)
    torch.cuda.synchronize()
    t_id = time.time() - t0
    k, ng = ctx.skeleton_rank(0)
    log(f"skeletonize (eps {eps}): {t_id:.2f} s, rings {k} of {ng}, {ns} of {wl.N} unknowns")
    runs = {}
    for name, mode in (("mixed", SOLVE_MIXED), ("fp64", SOLVE_FP64)):
        ctx.solve_skeleton(v, mode=mode, tol=args.tol)          # warm-up
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.time()
            sol, info = ctx.solve_skeleton(v, mode=mode, tol=args.tol)
            torch.cuda.synchronize()
            ts.append(time.time() - t0)
        b_ = ctx.apply_precond(v, FP64)
        full_res = float(torch.linalg.norm(ctx.apply_matvec(sol, FP64) + b_) / torch.linalg.norm(b_))
        runs[name] = {"s": float(np.median(ts)), "iterations": info[0]["iterations"],
                      "inner": info[0]["inner_iterations"], "compressed_rel_residual": info[0]["rel_residual"],
                      "full_rel_residual": full_res}
        log(f"{name}: {runs[name]}")
    ref, info_ref = ctx.solve(v, mode=SOLVE_MIXED, tol=args.tol)
    diff = float(torch.linalg.norm(sol - ref) / torch.linalg.norm(ref))
    points = [point_skeleton_leg(ctx, v, args.tol, e, ref) for e in (1e-8, 1e-9, 1e-10)]
    out = {
        "metric": "s to 1e-7 residual of the compressed system (Sec. 5 skeletonization), 27 spheres",
        "value": runs["mixed"]["s"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": runs["mixed"]["s"] * 1e3, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "N": wl.N, "eps": eps, "proxy_factor": 2.0, "tol": args.tol},
        "skeletonize_s": t_id, "rings": [k, ng], "skeleton_unknowns": ns, "solves": runs,
        "rel_diff_vs_uncompressed_mixed": diff, "points": points,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def batched(args):
    """One batched solve of 64 right-hand sides on 8 bodies of three shapes (and
    the same through point skeletons at eps 1e-10)."""
    import numpy as np
    import torch
    from paper_1406_0236_amd import FP32, FP64, SOLVE_FP64, SOLVE_MIXED, Context, autotune
    from workloads import configs
    wl = configs.mixed_bodies()
    r = len(wl.dirs)
    log(f"workload {wl.name}: N={wl.N}, pairs={wl.pairs:.4g}, rhs={r}")
    ctx = Context(0).add_workload(wl)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.precompute_scattering()
    torch.cuda.synchronize()
    t_pre = time.time() - t0
    v = ctx.incident_plane_waves(wl.dirs)
    tuned = {}
    for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
        cfg, tim = autotune.tune(ctx, prec, r, ctx.max_nf, x=v, reps=1, cache_path=None)
        tuned[name] = {"config": cfg, "ms": min(tim.values())}
    log(f"autotuned: {tuned}")
    for _ in range(args.warmup):
        ctx.solve(v, mode=SOLVE_MIXED, tol=args.tol)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        sol, info = ctx.solve(v, mode=SOLVE_MIXED, tol=args.tol)
    torch.cuda.synchronize()
    t_mixed = (time.time() - t0) / args.steps
    t0 = time.time()
    sol64, info64 = ctx.solve(v, mode=SOLVE_FP64, tol=args.tol)
    torch.cuda.synchronize()
    t64 = time.time() - t0
    log(f"mixed {t_mixed:.3f} s (outer {info[0]['iterations']}, inner {info[0]['inner_iterations']}); "
        f"fp64 {t64:.3f} s (iterations {max(i['iterations'] for i in info64)})")
    ctx.set_timing(True)
    ms = []
    for _ in range(3):
        ctx.apply_interbody(v, FP32)
        ms.append(ctx.last_timing()["interbody"])
    ctx.set_timing(False)
    t_ib = float(np.median(ms)) * 1e-3
    flops = wl.pairs * (FLOP_PER_PAIR + FLOP_PER_EXTRA_RHS * (r - 1))
    achieved = flops / t_ib / 1e12
    log(f"interbody fp32, {r} rhs: {t_ib*1e3:.2f} ms, {wl.pairs * r / t_ib / 1e9:.1f} G pair-rhs/s, "
        f"{achieved:.1f} TFLOP/s")
    points = point_skeleton_leg(ctx, v, args.tol, 1e-10, sol)
    out = {
        "metric": "s to 1e-7 residual, 64 rhs batched (mixed vs FP64 GMRES); far-field TFLOP/s",
        "value": t_mixed, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": wl.name, "bodies": len(wl.bodies), "N": wl.N, "kappa": wl.kappa, "nrhs": r,
                   "tol": args.tol},
        "mixed": {"s": t_mixed, "outer": max(i["iterations"] for i in info),
                  "inner": max(i["inner_iterations"] for i in info),
                  "max_rel_residual": max(i["rel_residual"] for i in info)},
        "fp64": {"s": t64, "iterations": max(i["iterations"] for i in info64),
                 "max_rel_residual": max(i["rel_residual"] for i in info64)},
        "speedup_mixed_vs_fp64": t64 / t_mixed,
        "precompute_s": t_pre,
        "autotuned": tuned,
        "point_skeleton": points,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "kernel": f"FP32 inter-body sum, {r} rhs, launch shape "
                               f"{list(ctx.interbody_launch_shape(FP32, r))}",
                     "flop_per_launch": flops, "launch_ms": t_ib * 1e3,
                     # variant 4 does the 8 flop per extra rhs on the FP16 matrix
                     # cores (split operands), so 157.3 is the FP32 reference
                     # rate, not a ceiling; the issue counters of the kernel are
                     # in the VALU profile
                     "note": "multiply-accumulate on the matrix cores; peak = FP32 vector reference"},
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
