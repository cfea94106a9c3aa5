#!/usr/bin/env python3
"""RASPEN solve throughput on one MI355X.

A step is one whole solve (Algorithm 2: local Newton solves with eps-continuation,
RAS restriction/prolongation, outer Newton-GMRES) of the 255x255 workload:
phi = y^3, f = 0, y_d = 8 seeded Gaussian bumps, nu = 1e-3, mu = 5e-3, eps 1 -> 1e-8
halving, 8x8 subdomains (32x32 each) with overlap 4, GMRES(30) rtol 1e-10, outer
tolerance 1e-10, inner tolerance 1e-8.  Inputs are resident in HBM before timing.

Prints one JSON line: solves/s, per-solve latency percentiles, the roofline of the
dominant kernel (HIP-event durations measured during the timed solves, algorithmic
bytes or flops per launch), and the CPU oracle timed on a bounded sample of the same
workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector (and FP64 matrix) peak
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (and FP32 matrix) peak
BOUND = {"factor": ("alu", FP64_PEAK_TFLOPS, "TFLOP/s"), "block_solve": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "newton_refine": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "solve_bwd": ("hbm", HBM_PEAK_GBS, "GB/s"), "gmres_ortho": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "linesearch": ("hbm", HBM_PEAK_GBS, "GB/s"), "prolong": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "ring_rhs": ("hbm", HBM_PEAK_GBS, "GB/s"), "restrict_halo": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "newton_init": ("hbm", HBM_PEAK_GBS, "GB/s"), "global_residual": ("hbm", HBM_PEAK_GBS, "GB/s")}
KERNEL_SOURCES = {"factor": "kernels_factor.hip", "block_solve": "kernels_factor.hip",
                  "solve_bwd": "kernels_factor.hip"}


def workload(name, precision="fp64", max_refine=0):
    import synth
    prob = synth.config_by_name(name)
    opts = synth.Options(precision=1 if precision == "mixed" else 0, max_refine=max_refine)
    return prob, opts


def describe(prob, opts):
    return {"workload": "raspen_%dx%d_phi%d_%dx%d_ov%d" % (prob.nx, prob.ny, prob.phi, prob.sx, prob.sy,
                                                          prob.overlap),
            "grid": [prob.nx, prob.ny], "phi": ["0", "y^3", "exp(y)-1", "kappa(y^3+exp(kappa y))"][prob.phi],
            "nu": prob.nu, "mu": prob.mu, "eps": [prob.eps0, prob.eps_min], "gamma": prob.gamma,
            "subdomains": [prob.sx, prob.sy], "overlap": prob.overlap, "gmres": [opts.gmres_restart, opts.gmres_rtol],
            "tol_outer": opts.tol_outer, "tol_inner": opts.tol_inner,
            "precision": ("fp32 line factors, fp64 residuals / Newton / GMRES, %d extra refinement step(s) "
                          "per local solve" % opts.max_refine) if opts.precision == 1 else "fp64",
            "seed": prob.seed, "unknowns": 2 * prob.nx * prob.ny}


def traffic_for(kernel, launches):
    """HBM bytes per launch from committed rocprofv3 counters, if they were taken on
    the current source of the kernel (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    src = KERNEL_SOURCES.get(kernel)
    if not os.path.exists(path) or src is None:
        return None
    data = json.load(open(path))
    ent = data.get(kernel)
    if not ent:
        return None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2411_00546_amd", "csrc", src), "rb").read()).hexdigest()
    if ent.get("source_sha256") != sha:
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(prob, opts, hist):
    """Oracle cost per solve from a bounded sample of the same workload: local Newton
    iterations of the first evaluation on every 2nd subdomain, sparse LU factorisations and
    solves of local Jacobians, and Gram-Schmidt steps on full-size vectors; each unit
    cost times the counts of the same solve (the oracle runs the same algorithm)."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    from oracle.schwarz import Raspen
    yd, f = prob.inputs()
    with threadpool_limits(limits=1):
        ora = Raspen(prob, opts, yd, f)
        n = ora.n
        x0 = np.zeros(2 * n)
        sample = list(range(0, len(ora.subs), 2))     # corner, edge and interior tiles
        t0 = time.perf_counter()
        iters = 0
        for i in sample:
            c, info = ora.local_solve(i, x0, prob.eps0)
            iters += info.iterations
        t_iter = (time.perf_counter() - t0) / iters
        t0 = time.perf_counter()
        lus = [spla.splu(ora.local_jacobian(i, x0, np.zeros(2 * ora.subs[i].rows.size), prob.eps_min))
               for i in sample]
        t_factor = (time.perf_counter() - t0) / len(sample)
        rng = np.random.default_rng(0)
        d = rng.standard_normal(2 * n)
        ora.x_loc = [x0] * len(ora.subs)
        t0 = time.perf_counter()
        reps = 30
        for _ in range(reps):
            for k, i in enumerate(sample):
                sub = ora.subs[i]
                rhs = ora.sys.jacobian_rows_apply(x0, prob.eps_min, sub.rows, ora.A_rows[i], d)
                lus[k].solve(rhs)
        t_apply_sub = (time.perf_counter() - t0) / (reps * len(sample))
        V = rng.standard_normal((16, 2 * n))
        t0 = time.perf_counter()
        for _ in range(reps):
            w = d.copy()
            for i in range(16):
                h = float(np.dot(w, V[i]))
                w = w - h * V[i]
        t_mgs = (time.perf_counter() - t0) / reps
        sample_s = t_iter * iters + t_factor * len(sample) + (t_apply_sub * len(sample) + t_mgs) * reps
    S = hist["subdomains"]
    inner = hist["newton_iterations"]                              # local Newton iterations
    fac_extra = hist["factorizations"] - inner                    # factorisations at x^(i)
    per_solve = (inner * t_iter + fac_extra * t_factor + hist["jac_applies"] * S * t_apply_sub
                 + hist["gmres_total"] * t_mgs)
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "seconds_per_solve": per_solve,
            "sample": ("NumPy/SciPy oracle, 1 thread: first-evaluation local Newton solves of %d of the %d "
                       "subdomains (%d iterations, %.2f ms each), %d sparse LU factorisations (%.1f ms), "
                       "%d local Jacobian solves (%.2f ms), %d Gram-Schmidt sweeps of 16 vectors (%.1f ms); "
                       "scaled by this solve's counts (%d local Newton iterations, %d extra factorisations, "
                       "%d RASPEN Jacobian products); %.1f s of CPU work"
                       % (len(sample), S, iters, 1e3 * t_iter, len(sample), 1e3 * t_factor, reps * len(sample),
                          1e3 * t_apply_sub, reps, 1e3 * t_mgs, inner, fac_extra, hist["jac_applies"],
                          sample_s))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="plain", choices=["plain", "small", "precision"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"],
                    help="mixed: FP32 line factors + FP64 refinement (the FP64 path is timed beside it)")
    ap.add_argument("--max-refine", type=int, default=0,
                    help="FP64 refinement steps per FP32 local solve (the local Newton iteration "
                         "refines against its FP64 residual in any case)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phases", type=int, default=0,
                    help="profiling mode: run N residual evaluations with continuation at x = 0 "
                         "and 20 Jacobian actions of the workload instead of whole solves")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2411_00546_amd import raspen as R
    R.load()
    prob, opts = workload(args.workload, args.precision, args.max_refine)
    _, opts64 = workload(args.workload, "fp64")
    yd, f = prob.inputs()
    dev = torch.device("cuda:0")
    ydt = torch.as_tensor(yd, dtype=torch.float64, device=dev).contiguous()
    ft = torch.as_tensor(f, dtype=torch.float64, device=dev).contiguous()
    y, p, u = (torch.empty_like(ydt) for _ in range(3))
    P, O, O64 = R.make_problem(prob), R.make_options(opts), R.make_options(opts64)
    ctx = R.rsp_context_create(0)
    if args.phases:
        try:
            R.rsp_setup(ctx, P, O, ydt, ft)
            n = prob.nx * prob.ny
            x = torch.zeros(2 * n, dtype=torch.float64, device=dev)
            out = torch.zeros_like(x)
            for r in range(args.phases):
                t = time.perf_counter()
                st, nrm = R.rsp_eval(ctx, x, 1, out)
                print("evaluation %d: status %d |F| %.6e  %.3f s" % (r, st, nrm, time.perf_counter() - t),
                      flush=True)
            d = torch.randn(2 * n, dtype=torch.float64, device=dev)
            for _ in range(20):
                R.rsp_jac_apply(ctx, d, out)
            torch.cuda.synchronize()
            print("20 Jacobian actions done", flush=True)
        finally:
            R.rsp_context_destroy(ctx)
        return

    def solves(opt, steps, warmup, profile):
        for _ in range(warmup):
            R.rsp_solve(ctx, P, opt, ydt, ft, None, None, y, p, u)
        if profile:
            R.rsp_set_profiling(ctx, True)
            R.rsp_reset_kernel_stats(ctx)
        torch.cuda.synchronize()
        lat, hist = [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            st, hist = R.rsp_solve(ctx, P, opt, ydt, ft, None, None, y, p, u)
            lat.append(time.perf_counter() - ts)
            if st != 0:
                raise RuntimeError("solve ended with status %d" % st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stats = R.rsp_kernel_stats(ctx) if profile else None
        R.rsp_set_profiling(ctx, False)
        x = torch.cat([y.reshape(-1), p.reshape(-1)]).cpu().numpy()
        return el, lat, hist, stats, x

    try:
        elapsed, lat, hist, stats, x = solves(O, args.steps, args.warmup, True)
        cmp64 = None
        if opts.precision == 1:
            el64, lat64, hist64, _, x64 = solves(O64, args.steps, 1, False)
            err = float(np.abs(x - x64).max() / np.abs(x64).max())
            cmp64 = {"value": args.steps / el64, "unit": "solves/s", "ms_per_step": 1e3 * el64 / args.steps,
                     "latency_ms": {"p50": float(np.percentile(np.array(lat64) * 1e3, 50)),
                                    "p99": float(np.percentile(np.array(lat64) * 1e3, 99))},
                     "rel_err_mixed_vs_fp64": err, "outer": hist64["outer"]}
            if not err <= 1e-8:
                raise RuntimeError("mixed-precision solution differs from FP64 by %.3e > 1e-8" % err)
    finally:
        R.rsp_context_destroy(ctx)

    value = args.steps / elapsed
    kern = {k: v for k, v in stats.items() if v["launches"] > 0}
    single = {k: v for k, v in kern.items() if k != "gmres_ortho"}
    dom = max(single, key=lambda k: single[k]["ms"])
    d = kern[dom]
    bound, peak, unit = BOUND[dom]
    if dom == "factor" and opts.precision == 1:
        peak = FP32_PEAK_TFLOPS
    avg_s = d["ms"] / d["launches"] / 1e3
    if bound == "hbm":
        achieved = d["bytes"] / d["launches"] / avg_s / 1e9
    else:
        achieved = d["flops"] / d["launches"] / avg_s / 1e12
    tb = traffic_for(dom, d["launches"])
    roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": tb,
            "avg_launch_us": avg_s * 1e6, "launches": d["launches"],
            "algorithmic_per_launch": (d["bytes"] if bound == "hbm" else d["flops"]) / d["launches"]}
    kernels = {k: {"launches": v["launches"], "ms_total": round(v["ms"], 3),
                   "avg_us": round(1e3 * v["ms"] / v["launches"], 2),
                   "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                   "GFLOPps": round(v["flops"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None}
               for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["ms"])}
    cpu = None if args.no_cpu_baseline else cpu_baseline(prob, opts, hist)
    lat_ms = np.array(lat) * 1e3
    out = {"metric": "solves/s at 1e-8 rel err (mixed vs FP64); p50/p99 solve latency",
           "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64+f32" if opts.precision == 1 else "f64",
           "data": "synthetic (seeded Gaussian-bump y_d)",
           "config": describe(prob, opts),
           "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
           "gflops": hist["flops"] / (elapsed / args.steps) / 1e9,
           "solve": {"outer": hist["outer"], "gmres_its": hist["gmres_its"], "inner_max": hist["inner_max"],
                     "residual_final": hist["residual_final"], "norm": hist["norm"][-1]},
           "fp64": cmp64, "roofline": roof, "kernels": kernels, "cpu_baseline": cpu}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
