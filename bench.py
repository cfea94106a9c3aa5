#!/usr/bin/env python3
"""RASPEN solve throughput on one MI355X.

A step is one whole solve (Algorithm 2: local Newton solves with eps-continuation,
RAS restriction/prolongation, outer Newton-GMRES) of the 511x511 precision workload
(the default): phi = exp(y) - 1, f = 0, y_d = 8 seeded Gaussian bumps, nu = 1e-3,
mu = 5e-3, eps 1 -> 1e-8 halving, 16x16 subdomains (32x32 each) with overlap 4,
GMRES(30) rtol 1e-10 with at most 300 products per outer step, outer tolerance 1e-10,
inner tolerance 1e-8; FP32 line factors on the matrix cores, FP64 everything else.
By default the outer Newton systems take the second level (coarse correction), with
the paper's one-level method timed beside it.  Inputs are resident in HBM before timing.

Prints one JSON line: solves/s, per-solve latency percentiles, the FP64 solve timed
beside it, each result's error against the oracle's stored solution of the same
workload and tolerances, the error of every eps step of the first evaluation against
the oracle on sampled subdomains, the roofline of the dominant kernel (HIP-event
durations measured during the timed solves, algorithmic bytes or flops per launch),
and the CPU oracle timed on a bounded sample of the same workload.
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
# the line factorisation is a chain of dense 80 x 80 inversions on the matrix cores
BOUND = {"factor": ("mfma", FP64_PEAK_TFLOPS, "TFLOP/s"), "block_solve": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "newton_refine": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "solve_bwd": ("hbm", HBM_PEAK_GBS, "GB/s"), "gmres_ortho": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "linesearch": ("hbm", HBM_PEAK_GBS, "GB/s"), "prolong": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "ring_rhs": ("hbm", HBM_PEAK_GBS, "GB/s"), "restrict_halo": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "newton_init": ("hbm", HBM_PEAK_GBS, "GB/s"), "global_residual": ("hbm", HBM_PEAK_GBS, "GB/s"),
         "ras_precond": ("hbm", HBM_PEAK_GBS, "GB/s"), "global_jacobian": ("hbm", HBM_PEAK_GBS, "GB/s")}


def workload(name, precision="fp64", max_refine=0, coarse=0, coef=0):
    import synth
    prob = synth.config_by_name(name)
    prob.coef = coef
    opts = synth.Options(precision=1 if precision == "mixed" else 0, max_refine=max_refine, coarse=coarse)
    return prob, opts


def describe(prob, opts):
    coef = getattr(prob, "coef", 0)
    return {"workload": "raspen_%dx%d_phi%d_%dx%d_ov%d%s" % (prob.nx, prob.ny, prob.phi, prob.sx, prob.sy,
                                                            prob.overlap, "_coef" if coef else ""),
            "operator": ("-d/dx(a1 d/dx) - d/dy(a2 d/dy) + a0, seeded smooth coefficients "
                         "(synth.coefficient_fields)") if coef else "-Laplacian (5-point)",
            "grid": [prob.nx, prob.ny], "phi": ["0", "y^3", "exp(y)-1", "kappa(y^3+exp(kappa y))"][prob.phi],
            "nu": prob.nu, "mu": prob.mu, "eps": [prob.eps0, prob.eps_min], "gamma": prob.gamma,
            "subdomains": [prob.sx, prob.sy], "overlap": prob.overlap,
            "gmres": [opts.gmres_restart, opts.gmres_rtol, opts.max_gmres],
            "tol_outer": opts.tol_outer, "tol_inner": opts.tol_inner,
            "precision": ("fp32 line factors, fp64 residuals / Newton / GMRES, %d extra refinement step(s) "
                          "per local solve" % opts.max_refine) if opts.precision == 1 else "fp64",
            "seed": prob.seed, "unknowns": 2 * prob.nx * prob.ny}


def traffic_for(kernel, fp32, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size)
    from the committed rocprofv3 counters, when they were taken on this workload, on the
    current source of the kernel and for the same factor precision (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    if data.get("workload") != workload:
        return None
    ent = data.get(kernel + ("/fp32" if fp32 else "/fp64")) or data.get(kernel)
    if not ent:
        return None
    src = os.path.join(ROOT, "paper_2411_00546_amd", "csrc", ent["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != ent.get("source_sha256"):
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(prob, opts, hist, max_sub=64):
    """Oracle cost per solve from a bounded sample of the same workload (10-30 s of one
    core): the local Newton iterations of the first evaluation on up to max_sub
    subdomains (every subdomain up to 64, else an even spread), sparse LU factorisations
    and solves of their local Jacobians, and Gram-Schmidt steps on full-size vectors;
    each unit cost times the counts of the same solve (the oracle runs the same
    algorithm).  A whole oracle solve of the 511^2 workload takes about 12 minutes of
    one core, beyond the time of a bench run."""
    import numpy as np
    import scipy.sparse.linalg as spla
    from threadpoolctl import threadpool_limits
    from oracle.schwarz import Raspen
    yd, f = prob.inputs()
    with threadpool_limits(limits=1):
        ora = Raspen(prob, opts, yd, f)
        n = ora.n
        x0 = np.zeros(2 * n)
        S_all = len(ora.subs)
        step = max(1, -(-S_all // max_sub))
        sample = list(range(0, S_all, step))           # corner, edge and interior tiles
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
        # second level: the oracle's coarse correction per product (F'(x) v, the coarse solve)
        t_coarse = 0.0
        if getattr(opts, "coarse", 0):
            Z = ora.coarse_basis()
            J = ora.sys.jacobian(x0, prob.eps_min)
            A0 = ora.coarse_operator(x0, Z)
            t0 = time.perf_counter()
            creps = 5
            for _ in range(creps):
                Z @ np.linalg.solve(A0, Z.T @ (J @ d))
            t_coarse = (time.perf_counter() - t0) / creps
            sample_s += t_coarse * creps
    S = hist["subdomains"]
    inner = hist["newton_iterations"]                              # local Newton iterations
    fac_extra = hist["factorizations"] - inner                    # factorisations at x^(i)
    per_solve = (inner * t_iter + fac_extra * t_factor + hist["jac_applies"] * S * t_apply_sub
                 + hist["gmres_total"] * t_mgs + hist["jac_applies"] * t_coarse)
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1,
            "cores_available": len(os.sched_getaffinity(0)), "kind": "oracle",
            "seconds_per_solve": per_solve, "extrapolated_from_sample": True,
            "units": {"t_iter": t_iter, "t_factor": t_factor, "t_apply_sub": t_apply_sub, "t_mgs": t_mgs,
                      "t_coarse": t_coarse},
            "sample": ("NumPy/SciPy oracle, 1 thread: first-evaluation local Newton solves of %d of the %d "
                       "subdomains (%d iterations, %.2f ms each), %d sparse LU factorisations (%.1f ms), "
                       "%d local Jacobian solves (%.2f ms), %d Gram-Schmidt sweeps of 16 vectors (%.1f ms); "
                       "scaled by this solve's counts (%d local Newton iterations, %d extra factorisations, "
                       "%d RASPEN Jacobian products%s); %.1f s of CPU work"
                       % (len(sample), S, iters, 1e3 * t_iter, len(sample), 1e3 * t_factor, reps * len(sample),
                          1e3 * t_apply_sub, reps, 1e3 * t_mgs, inner, fac_extra, hist["jac_applies"],
                          ", each with a coarse correction of %.1f ms" % (1e3 * t_coarse) if t_coarse else "",
                          sample_s))}


ORACLE_REFS = {"plain": "plain_cfg", "precision": "precision_cfg", "plain_coef": "plain_coef_cfg"}


def oracle_reference(work):
    """The oracle's solution of this workload at its own tolerances, stored by
    tests/golden/make_oracle_refs.py (which runs the oracle alone), or None."""
    import numpy as np
    if work not in ORACLE_REFS:
        return None
    path = os.path.join(ROOT, "tests", "golden", "oracle_%s.npz" % ORACLE_REFS[work])
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return {"x": z["x"], "outer": int(z["outer"]), "seconds": float(z["seconds"]),
                "name": os.path.relpath(path, ROOT)}


def sample_subdomains(prob, count=6):
    """Corner, edge and interior subdomains of the partition (row-major numbering)."""
    S = prob.sx * prob.sy
    return sorted({0, prob.sx - 1, S - prob.sx, S - 1, (prob.sy // 2) * prob.sx + prob.sx // 2,
                   min(S - 1, prob.sx + 1)})[:count]


def eps_step_errors(ora, prob, snaps, count):
    """Error of each eps step of the first evaluation against the oracle: snapshot k
    (x^0 + sum_i P~_i c_i^(k), x^0 = 0) on the cores of sampled subdomains against the
    oracle's local Newton iterates c_i^(k) there (the oracle solves one subdomain at a
    time), relative to the largest |c_i| of the converged local solutions.  snaps:
    {subdomain: [count][2 core] host array}."""
    import numpy as np
    n = prob.nx * prob.ny
    per_k = np.zeros(count)
    for i, got in snaps.items():
        sub = ora.subs[i]
        rec = []
        ora.local_solve(i, np.zeros(2 * n), prob.eps0, record=rec)
        m = sub.rows.size
        scale = max(np.abs(rec[-1]).max(), 1e-300)
        for k in range(count):
            c = rec[min(k, len(rec) - 1)]
            want = np.concatenate([c[:m][sub.core_local], c[m:][sub.core_local]])
            per_k[k] = max(per_k[k], float(np.abs(got[k] - want).max() / scale))
    return [float(e) for e in per_k]


def dominant(stats):
    """The single-pass kernel class with the largest device time (the GMRES
    orthogonalisation is a chain of kernels, not one)."""
    single = {k: v for k, v in stats.items() if v["launches"] > 0 and k != "gmres_ortho"}
    return max(single, key=lambda k: single[k]["ms"])


def kernel_table(stats):
    return {k: {"launches": v["launches"], "ms_total": round(v["ms"], 3),
                "avg_us": round(1e3 * v["ms"] / v["launches"], 2),
                "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                "GFLOPps": round(v["flops"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None}
            for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["ms"]) if v["launches"] > 0}


TIME_EVERY = [1]   # launch sequences per timed one in the timed solves (--time-every)


def solve_roofline(stats, fp32, ms_per_solve):
    """Solve-level roofline: sum over the kernel classes of one solve (every class timed)
    of max(algorithmic bytes / HBM peak, algorithmic flops / peak of the class), over the
    measured time of a solve.  The FP32 line factorisation takes the FP32 matrix peak,
    every other class the FP64 one."""
    bound_s = 0.0
    for name, v in stats.items():
        if v["launches"] == 0:
            continue
        peak = (FP32_PEAK_TFLOPS if (name == "factor" and fp32) else FP64_PEAK_TFLOPS) * 1e12
        bound_s += max(v["bytes"] / (HBM_PEAK_GBS * 1e9), v["flops"] / peak)
    return {"bound_ms": 1e3 * bound_s, "measured_ms": ms_per_solve, "frac": 1e3 * bound_s / ms_per_solve}


def kernel_roofline(stats, fp32, workload):
    """Roofline object of the dominant single-pass kernel from rsp_kernel_stats output."""
    kern = {k: v for k, v in stats.items() if v["launches"] > 0}
    dom = dominant(kern)
    d = kern[dom]
    bound, peak, unit = BOUND[dom]
    if dom == "factor" and fp32:
        peak = FP32_PEAK_TFLOPS
    avg_s = d["ms"] / d["launches"] / 1e3
    if bound == "hbm":
        achieved = d["bytes"] / d["launches"] / avg_s / 1e9
    else:
        achieved = d["flops"] / d["launches"] / avg_s / 1e12
    roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic_for(dom, fp32, workload),
            "avg_launch_us": avg_s * 1e6, "launches": d["launches"], "timed_every": TIME_EVERY[0],
            "algorithmic_per_launch": (d["bytes"] if bound == "hbm" else d["flops"]) / d["launches"]}
    return roof


def pct(lat_s):
    import numpy as np
    a = np.array(lat_s) * 1e3
    return {"p50": float(np.percentile(a, 50)), "p99": float(np.percentile(a, 99))}


class Instances:
    """Device inputs and outputs of a list of problems (allocated once, before timing)."""

    def __init__(self, probs):
        import torch
        self.probs = probs
        self.yd, self.f, self.y, self.p, self.u = [], [], [], [], []
        for pr in probs:
            yd, f = pr.inputs()
            self.yd.append(torch.as_tensor(yd, dtype=torch.float64, device="cuda:0").contiguous())
            self.f.append(torch.as_tensor(f, dtype=torch.float64, device="cuda:0").contiguous())
            for lst in (self.y, self.p, self.u):
                lst.append(torch.empty((pr.ny, pr.nx), dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()

    def x(self, q):
        import torch
        return torch.cat([self.y[q].reshape(-1), self.p[q].reshape(-1)]).cpu().numpy()


def rel_errs(xs, refs):
    """Max-norm relative error of each solution against its FP64 reference."""
    import numpy as np
    return [float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(xs, refs)]


def err_report(errs):
    """A solve counts toward solves/s when it is within 1e-8 of the FP64 solution."""
    import numpy as np
    e = np.array(errs)
    return {"max": float(e.max()), "median": float(np.median(e)), "within_1e-8": int((e <= 1e-8).sum()),
            "count": len(errs)}


def batch_cpu_baseline(probs, opts, hists):
    """Oracle cost of the batch: unit costs measured (bounded sample) on the largest
    instance, scaled by every instance's own counts; Gram-Schmidt cost scaled by size."""
    big = max(range(len(probs)), key=lambda q: probs[q].nx * probs[q].ny)
    one = cpu_baseline(probs[big], opts, hists[big])
    n_big = probs[big].nx * probs[big].ny
    u = one["units"]
    total = 0.0
    for pr, h in zip(probs, hists):
        S = h["subdomains"]
        inner = h["newton_iterations"]
        total += (inner * u["t_iter"] + (h["factorizations"] - inner) * u["t_factor"]
                  + h["jac_applies"] * S * u["t_apply_sub"]
                  + h["gmres_total"] * u["t_mgs"] * (pr.nx * pr.ny) / n_big)
    return {"value": len(probs) / total, "unit": "solves/s", "cores": 1,
            "cores_available": len(os.sched_getaffinity(0)), "kind": "oracle",
            "seconds_per_batch": total, "extrapolated_from_sample": True,
            "sample": "unit costs from the bounded oracle sample of the %dx%d instance (%s), scaled by the "
                      "counts of all %d instances" % (probs[big].nx, probs[big].ny, one["sample"], len(probs))}


def serve_cpu_baseline(probs, opts, hists, count=32):
    """Oracle cost of the request stream: unit costs measured (bounded sample) on the
    largest of the first `count` requests, scaled by the counts of every request."""
    out = batch_cpu_baseline(probs[:count], opts, hists[:count])
    out["sample"] = "the first %d requests: %s" % (count, out["sample"])
    out["seconds_per_request"] = 1.0 / out["value"]
    return out


def apply_tuning(R, ctx, args, prob, opts, yd, f):
    """--tune 1: the autotuner picks the execution settings on this workload's problem
    (graphs, Arnoldi chunk; the partition stays the workload's); else --graphs and
    --gm-chunk.  Returns the settings as a dict."""
    if args.tune:
        t = R.rsp_autotune(ctx, prob, opts, yd, f, flags=0)
    else:
        R.rsp_set_tuning(ctx, graphs=args.graphs, gm_chunk=args.gm_chunk)
        t = R.rsp_get_tuning(ctx)
    return {"graphs": t.graphs, "gm_chunk": t.gm_chunk, "jac_form": t.jac_form, "autotuned": bool(args.tune),
            "tuner_solves_per_s": t.solves_per_s if args.tune else None}


def run_batch_workload(args, R):
    """64 uneven instances per step through rsp_solve_batch (FP32 line factors), checked
    against the FP64 batch, with plain FP64 one-at-a-time solves timed beside it."""
    import numpy as np
    import synth
    import torch
    probs = synth.batch_instances(args.count)
    opts = synth.Options(precision=1 if args.precision == "mixed" else 0, max_refine=args.max_refine,
                         coarse=args.coarse)
    opts64 = synth.Options(coarse=args.coarse)
    inst = Instances(probs)
    P = [R.make_problem(pr) for pr in probs]
    O, O64 = R.make_options(opts), R.make_options(opts64)
    ctx = R.rsp_context_create(0)
    try:
        big = max(range(len(probs)), key=lambda q: probs[q].nx * probs[q].ny)
        tuning = apply_tuning(R, ctx, args, P[big], O, inst.yd[big], inst.f[big])

        def batch(o, steps, warm, profile):
            for _ in range(warm):
                R.rsp_solve_batch(ctx, P, o, inst.yd, inst.f, None, None, inst.y, inst.p, inst.u)
            breakdown = None
            if profile:
                # an untimed batch with every kernel class timed, then events around the
                # dominant kernel only in the timed batches
                R.rsp_set_profiling_filter(ctx, None)
                R.rsp_set_profiling(ctx, True)
                R.rsp_reset_kernel_stats(ctx)
                R.rsp_solve_batch(ctx, P, o, inst.yd, inst.f, None, None, inst.y, inst.p, inst.u)
                breakdown = R.rsp_kernel_stats(ctx)
                R.rsp_set_profiling_filter(ctx, dominant(breakdown))
                R.rsp_set_profiling_sample(ctx, args.time_every)
                R.rsp_reset_kernel_stats(ctx)
            torch.cuda.synchronize()
            lat = []
            t0 = time.perf_counter()
            for _ in range(steps):
                ts = time.perf_counter()
                st, hists = R.rsp_solve_batch(ctx, P, o, inst.yd, inst.f, None, None, inst.y, inst.p, inst.u)
                lat.append(time.perf_counter() - ts)
                if st != 0:
                    raise RuntimeError("batch ended with status %d" % st)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            stats = R.rsp_kernel_stats(ctx) if profile else None
            R.rsp_set_profiling(ctx, False)
            R.rsp_set_profiling_filter(ctx, None)
            R.rsp_set_profiling_sample(ctx, 1)
            return el, lat, hists, (stats, breakdown), [inst.x(q) for q in range(len(probs))]

        el, lat, hists, stats, xs = batch(O, args.steps, args.warmup, True)
        el64b, _, hists64, _, x64 = batch(O64, 1, 0, False)
        errs = err_report(rel_errs(xs, x64))
        # plain FP64, one instance at a time
        t0 = time.perf_counter()
        lat1 = []
        for q in range(len(probs)):
            ts = time.perf_counter()
            st, _ = R.rsp_solve(ctx, P[q], O64, inst.yd[q], inst.f[q], None, None, inst.y[q], inst.p[q],
                                inst.u[q])
            lat1.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t0
    finally:
        R.rsp_context_destroy(ctx)
    stats, breakdown = stats
    roof = kernel_roofline(stats, opts.precision == 1, None)
    kernels = kernel_table(breakdown)
    flops = sum(h["flops"] for h in hists)
    sizes = sorted({(pr.nx, pr.ny) for pr in probs})
    cpu = None if args.no_cpu_baseline else batch_cpu_baseline(probs, opts, hists)
    return {"metric": "solves/s at 1e-8 rel err (mixed vs FP64); p50/p99 solve latency",
            "value": errs["within_1e-8"] * args.steps / el, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32" if opts.precision == 1 else "f64",
            "data": "synthetic (seeded Gaussian-bump y_d)",
            "config": {"workload": "raspen_batch%d_grids63-255_32x32subdomains_ov4" % len(probs),
                       "instances": len(probs), "grids": sizes, "step": "one rsp_solve_batch of every instance",
                       "precision": "fp32 line factors" if opts.precision == 1 else "fp64",
                       "levels": 2 if args.coarse else 1},
            "latency_ms": pct([l / 1.0 for l in lat]),
            "per_instance_latency_ms": {"p50": float(np.percentile([h["ms_total"] for h in hists], 50)),
                                        "p99": float(np.percentile([h["ms_total"] for h in hists], 99))},
            "gflops": flops / (el / args.steps) / 1e9,
            "rel_err_mixed_vs_fp64": errs, "all_solves_per_s": len(probs) * args.steps / el,
            "fp64_batch": {"value": len(probs) / el64b, "unit": "solves/s"},
            "fp64_one_at_a_time": {"value": len(probs) / el1, "unit": "solves/s", "latency_ms": pct(lat1)},
            "outer": [h["outer"] for h in hists], "tuning": tuning, "roofline": roof, "kernels": kernels,
            "cpu_baseline": cpu}


def run_serve_workload(args, R):
    """Poisson request stream through rsp_server_*: closed-loop capacity first, then an
    open-loop stream at 0.8 of it; every result checked against plain FP64 solves."""
    import numpy as np
    import synth
    import torch
    # grids up to 511x511 (256 subdomains): the GMRES iterations of an outer step grow with the
    # subdomain count, so the cap on products per outer step is raised for this stream
    opts = synth.Options(precision=1 if args.precision == "mixed" else 0, max_refine=args.max_refine,
                         max_gmres=1500, coarse=args.coarse)
    _, probs = synth.request_stream(args.count, 1.0)
    inst = Instances(probs)
    P = [R.make_problem(pr) for pr in probs]
    O, O64 = R.make_options(opts), R.make_options(synth.Options(max_gmres=1500, coarse=args.coarse))

    # execution settings for the server's context, tuned on a median-size request
    mid = sorted(range(len(probs)), key=lambda q: probs[q].nx * probs[q].ny)[len(probs) // 2]
    ctx = R.rsp_context_create(0)
    try:
        tuning = apply_tuning(R, ctx, args, P[mid], O, inst.yd[mid], inst.f[mid])
        tune = R.rsp_get_tuning(ctx)
    finally:
        R.rsp_context_destroy(ctx)

    def serve(arrivals, profile=False):
        srv = R.rsp_server_create(O, tune=tune, profile_every=args.time_every if profile else 0)
        try:
            t0 = time.perf_counter()
            tickets = []
            for q in range(len(probs)):
                if arrivals is not None:
                    dt = t0 + arrivals[q] - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                tickets.append(R.rsp_server_submit(srv, P[q], inst.yd[q], inst.f[q], inst.y[q], inst.p[q],
                                                   inst.u[q]))
            hists = []
            for t in tickets:
                st, h = R.rsp_server_wait(srv, t)
                if st != 0:
                    raise RuntimeError("request ended with status %d" % st)
                hists.append(h)
            el = time.perf_counter() - t0
            stats = R.rsp_server_stats(srv)
            kstats = R.rsp_server_kernel_stats(srv) if profile else None
        finally:
            R.rsp_server_destroy(srv)
        return el, hists, (stats, kstats)

    serve(None)                                     # warm-up (code objects, allocations)
    el_c, _, (st_c, _) = serve(None)
    capacity = len(probs) / el_c
    rate = 0.8 * capacity
    arrivals, _ = synth.request_stream(args.count, rate)
    el_o, hists, (st_o, kst) = serve(arrivals, profile=True)
    xs = [inst.x(q) for q in range(len(probs))]
    ctx = R.rsp_context_create(0)
    try:
        lat1 = []
        t0 = time.perf_counter()
        for q in range(len(probs)):
            ts = time.perf_counter()
            R.rsp_solve(ctx, P[q], O64, inst.yd[q], inst.f[q], None, None, inst.y[q], inst.p[q], inst.u[q])
            lat1.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t0
    finally:
        R.rsp_context_destroy(ctx)
    errs = err_report(rel_errs(xs, [inst.x(q) for q in range(len(probs))]))
    return {"metric": "solves/s at 1e-8 rel err (mixed vs FP64); p50/p99 solve latency",
            "value": st_o["solves_per_s"] * errs["within_1e-8"] / len(probs), "unit": "solves/s", "n_gpus": 1,
            "steps": len(probs), "warmup": 1,
            "ms_per_step": 1e3 * el_o / len(probs), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64+f32" if opts.precision == 1 else "f64",
            "data": "synthetic (seeded Gaussian-bump y_d, Poisson arrivals)",
            "config": {"workload": "raspen_serve%d_grids127-511_poisson" % len(probs), "requests": len(probs),
                       "rate_per_s": rate, "load": 0.8, "grids": sorted({(pr.nx, pr.ny) for pr in probs})},
            "latency_ms": {"p50": st_o["p50_ms"], "p99": st_o["p99_ms"], "mean": st_o["mean_ms"]},
            "mean_batch": st_o["mean_batch"],
            "closed_loop": {"solves_per_s": capacity, "p50_ms": st_c["p50_ms"], "p99_ms": st_c["p99_ms"],
                            "mean_batch": st_c["mean_batch"]},
            "rel_err_mixed_vs_fp64": errs, "all_solves_per_s": st_o["solves_per_s"],
            "fp64_one_at_a_time": {"value": len(probs) / el1, "unit": "solves/s", "latency_ms": pct(lat1)},
            "tuning": tuning, "roofline": kernel_roofline(kst, opts.precision == 1, None) if kst else None,
            "levels": 2 if args.coarse else 1,
            "cpu_baseline": None if args.no_cpu_baseline else serve_cpu_baseline(probs, opts, hists)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="precision", choices=["plain", "small", "precision", "batch", "serve"],
                    help="precision: 511x511 exp (default); plain: 255x255; small: 63x63; batch: 64 uneven "
                         "instances per step; serve: Poisson request stream through the server")
    ap.add_argument("--count", type=int, default=64, help="instances (batch) or requests (serve)")
    ap.add_argument("--tune", type=int, default=1, choices=[0, 1],
                    help="1: rsp_autotune picks graphs and the Arnoldi chunk on the workload first")
    ap.add_argument("--graphs", type=int, default=0, choices=[0, 1],
                    help="with --tune 0: capture Arnoldi chunks and continuation runs into hipGraphs")
    ap.add_argument("--gm-chunk", type=int, default=32, help="with --tune 0: Arnoldi steps between GMRES "
                                                             "header reads")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"],
                    help="mixed: FP32 line factors + FP64 refinement (the FP64 path is timed beside it)")
    ap.add_argument("--max-refine", type=int, default=0,
                    help="FP64 refinement steps per FP32 local solve (the local Newton iteration "
                         "refines against its FP64 residual in any case)")
    ap.add_argument("--time-every", type=int, default=4,
                    help="in the timed solves, HIP events around the dominant kernel in one of every "
                         "N launch sequences (Arnoldi chunks); the others run untimed, as graphs when on")
    ap.add_argument("--method", default="raspen", choices=["raspen", "newton_ras", "newton"],
                    help="plain/small/precision workloads: RASPEN (Algorithm 2, the default), the "
                         "linearly RAS-preconditioned Newton with eps-continuation (rsp_solve_newton_ras) "
                         "or the unpreconditioned one (rsp_solve_newton)")
    ap.add_argument("--coarse", type=int, default=1, choices=[0, 1],
                    help="RASPEN: 1 (default) the two-level method (coarse correction of the outer "
                         "Newton systems), with the paper's one-level method timed beside it; 0 one level")
    ap.add_argument("--coef", type=int, default=0, choices=[0, 1],
                    help="1: the workload with the seeded variable coefficients of A")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eps-errors", action="store_true",
                    help="skip the per-eps-step comparison with the oracle on sampled subdomains")
    ap.add_argument("--phases", type=int, default=0,
                    help="profiling mode: run N residual evaluations with continuation at x = 0, "
                         "20 Jacobian actions of the workload and 3 plain 64 MiB device copies "
                         "(traffic-counter calibration) instead of whole solves")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.time_every < 1:
        ap.error("--time-every must be >= 1")
    TIME_EVERY[0] = args.time_every

    import numpy as np
    import torch
    from paper_2411_00546_amd import raspen as R
    R.load()
    if args.workload in ("batch", "serve"):
        run = run_batch_workload if args.workload == "batch" else run_serve_workload
        print(json.dumps(run(args, R)))
        return
    coarse = args.coarse if args.method == "raspen" else 0
    prob, opts = workload(args.workload, args.precision, args.max_refine, coarse, args.coef)
    _, opts64 = workload(args.workload, "fp64", 0, coarse)
    _, opts_one = workload(args.workload, args.precision, args.max_refine, 0)
    yd, f = prob.inputs()
    dev = torch.device("cuda:0")
    ydt = torch.as_tensor(yd, dtype=torch.float64, device=dev).contiguous()
    ft = torch.as_tensor(f, dtype=torch.float64, device=dev).contiguous()
    y, p, u = (torch.empty_like(ydt) for _ in range(3))
    coef_t = None
    if args.coef:
        import synth
        coef_t = torch.as_tensor(synth.pack_coefficients(*prob.coefficients()), dtype=torch.float64, device=dev)
    P, O, O64 = R.make_problem(prob, coef_t), R.make_options(opts), R.make_options(opts64)
    O1 = R.make_options(opts_one)
    ctx = R.rsp_context_create(0)
    tuning = None
    if not args.phases:
        tuning = apply_tuning(R, ctx, args, P, O, ydt, ft)
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
            # a plain device copy of 64 MiB, the calibration of the HBM traffic counters
            src = torch.ones(8 << 20, dtype=torch.float64, device=dev)
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            print("3 copies of %d bytes done" % (src.numel() * 8), flush=True)
        finally:
            R.rsp_context_destroy(ctx)
        return

    # the method timed: RASPEN (Algorithm 2), or the linearly RAS-preconditioned Newton
    # of Section 4.1 on the same workload
    solve_fn = {"raspen": R.rsp_solve, "newton_ras": R.rsp_solve_newton_ras,
                "newton": R.rsp_solve_newton}[args.method]

    def solves(opt, steps, warmup, profile):
        for _ in range(warmup):
            solve_fn(ctx, P, opt, ydt, ft, None, None, y, p, u)
        breakdown = None
        if profile:
            # one untimed solve with every kernel class timed: the per-kernel table and
            # the choice of the dominant kernel; the timed solves then carry events
            # around that kernel only
            R.rsp_set_profiling_filter(ctx, None)
            R.rsp_set_profiling(ctx, True)
            R.rsp_reset_kernel_stats(ctx)
            solve_fn(ctx, P, opt, ydt, ft, None, None, y, p, u)
            breakdown = R.rsp_kernel_stats(ctx)
            R.rsp_set_profiling_filter(ctx, dominant(breakdown))
            R.rsp_set_profiling_sample(ctx, args.time_every)
            R.rsp_reset_kernel_stats(ctx)
        torch.cuda.synchronize()
        lat, hist = [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            ts = time.perf_counter()
            st, hist = solve_fn(ctx, P, opt, ydt, ft, None, None, y, p, u)
            lat.append(time.perf_counter() - ts)
            if st != 0:
                raise RuntimeError("solve ended with status %d" % st)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        stats = R.rsp_kernel_stats(ctx) if profile else None
        R.rsp_set_profiling(ctx, False)
        R.rsp_set_profiling_filter(ctx, None)
        R.rsp_set_profiling_sample(ctx, 1)
        x = torch.cat([y.reshape(-1), p.reshape(-1)]).cpu().numpy()
        return el, lat, hist, (stats, breakdown), x

    def snapshot_cores(opt, sample, K=48):
        """One untimed solve recording the first evaluation's eps steps; the cores of
        the sampled subdomains of each snapshot, as host arrays."""
        o = type(opt).from_buffer_copy(opt)
        o.record_eps_snapshots = K
        buf = torch.empty((K, 2, prob.ny, prob.nx), dtype=torch.float64, device=dev)
        o.eps_snapshots = buf.data_ptr()
        st, h = solve_fn(ctx, P, o, ydt, ft, None, None, y, p, u)
        if st != 0:
            raise RuntimeError("snapshot solve ended with status %d" % st)
        k = h["snapshots"]
        out = {}
        for i in sample:
            x0, x1, y0, y1 = part[i][4:]
            out[i] = torch.cat([buf[:k, 0, y0:y1, x0:x1].reshape(k, -1),
                                buf[:k, 1, y0:y1, x0:x1].reshape(k, -1)], 1).cpu().numpy()
        return out, k, h["snapshot_eps"]

    ref = oracle_reference(args.workload + ("_coef" if args.coef else "")) if args.method == "raspen" else None
    sample = sample_subdomains(prob)
    part = R.rsp_partition(P)[3]
    try:
        elapsed, lat, hist, stats, x = solves(O, args.steps, args.warmup, True)
        cmp64 = None
        if opts.precision == 1:
            el64, lat64, hist64, _, x64 = solves(O64, args.steps, 1, False)
            err = float(np.abs(x - x64).max() / np.abs(x64).max())
            cmp64 = {"value": args.steps / el64, "unit": "solves/s", "ms_per_step": 1e3 * el64 / args.steps,
                     "latency_ms": {"p50": float(np.percentile(np.array(lat64) * 1e3, 50)),
                                    "p99": float(np.percentile(np.array(lat64) * 1e3, 99))},
                     "rel_err_mixed_vs_fp64": err, "outer": hist64["outer"],
                     "rel_err_vs_oracle": (float(np.abs(x64 - ref["x"]).max() / np.abs(ref["x"]).max())
                                           if ref is not None else None)}
            if not err <= 1e-8:
                raise RuntimeError("mixed-precision solution differs from FP64 by %.3e > 1e-8" % err)
        one_level = None
        if coarse:
            # the paper's one-level method on the same workload, timed beside it
            el1, lat1, hist1, _, x1 = solves(O1, args.steps, 1, False)
            one_level = {"value": args.steps / el1, "unit": "solves/s", "ms_per_step": 1e3 * el1 / args.steps,
                         "latency_ms": {"p50": float(np.percentile(np.array(lat1) * 1e3, 50)),
                                        "p99": float(np.percentile(np.array(lat1) * 1e3, 99))},
                         "outer": hist1["outer"], "gmres_its": hist1["gmres_its"],
                         "rel_err_vs_oracle": (float(np.abs(x1 - ref["x"]).max() / np.abs(ref["x"]).max())
                                               if ref is not None else None)}
        snaps = None
        if args.method == "raspen" and not args.no_eps_errors:
            snaps = {"mixed" if opts.precision == 1 else "fp64": snapshot_cores(O, sample)}
            if opts.precision == 1:
                snaps["fp64"] = snapshot_cores(O64, sample)
    finally:
        R.rsp_context_destroy(ctx)

    vs_oracle = None
    if ref is not None:
        vs_oracle = {"reference": ref["name"], "oracle_outer": ref["outer"],
                     "rel_err": float(np.abs(x - ref["x"]).max() / np.abs(ref["x"]).max()),
                     "oracle_full_solve_s_on_build_host": ref["seconds"]}
    ora = None
    eps_err = None
    if snaps is not None:
        from threadpoolctl import threadpool_limits
        from oracle.schwarz import Raspen
        with threadpool_limits(limits=1):
            ora = Raspen(prob, opts64, yd, f)
            eps_err = {"sampled_subdomains": sample, "unit": "max-norm error on the sampled cores / max |c_i|"}
            for key, (cores, k, eps_k) in snaps.items():
                e = eps_step_errors(ora, prob, cores, k)
                eps_err[key] = {"per_step": e, "max": max(e), "last": e[-1], "eps": eps_k}

    value = args.steps / elapsed
    stats, breakdown = stats
    desc = describe(prob, opts)
    roof = kernel_roofline(stats, opts.precision == 1, desc["workload"])
    kernels = kernel_table(breakdown)
    # the CPU baseline is the RASPEN oracle's sample; none for the comparison method
    cpu = None if args.no_cpu_baseline or args.method != "raspen" else cpu_baseline(prob, opts, hist)
    lat_ms = np.array(lat) * 1e3
    out = {"metric": "solves/s at 1e-8 rel err (mixed vs FP64); p50/p99 solve latency",
           "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64+f32" if opts.precision == 1 else "f64",
           "data": "synthetic (seeded Gaussian-bump y_d)",
           "config": dict(desc, method=args.method + (" two-level (coarse correction of the outer Newton "
                                                       "systems; the one-level method under one_level)"
                                                       if coarse else "")),
           "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
           "gflops": hist["flops"] / (elapsed / args.steps) / 1e9,
           "solve": {"outer": hist["outer"], "gmres_its": hist["gmres_its"], "inner_max": hist["inner_max"],
                     "residual_final": hist["residual_final"], "norm": hist["norm"][-1]},
           "fp64": cmp64, "one_level": one_level, "vs_oracle": vs_oracle, "eps_step_errors": eps_err,
           "tuning": tuning,
           "roofline": roof,
           "solve_roofline": solve_roofline(breakdown, opts.precision == 1, 1e3 * elapsed / args.steps),
           "kernels": kernels, "cpu_baseline": cpu}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
