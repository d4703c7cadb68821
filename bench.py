"""Benchmark: (l, grad l) evaluations per second at n = 40,000 on one MI355X.

Workload (the configuration the headline metric is quoted on): 40,000
locations uniform on [0,1]^2 (seed 0), Matern theta = (1, 0.1, 1.0), tile
size 768, z drawn from the same field with the library's simulator (untimed);
one step = one exact FP64 evaluation of l(theta) and its gradient, every
kernel of the path included (ordering, generation, Cholesky, solves,
reductions, inverse, fused LAUUM + score contraction).

Prints ONE JSON line.  Extra keys: POTRF TFLOP/s (n^3/3 + n^2/2 + n/6 over
the Cholesky phase time) and the fraction of the FP64 MFMA peak, per-phase
times, the roofline of the dominant kernel (the trailing-update GEMM,
timed with HIP events on the library's stream around every launch), and
the CPU oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the trailing-update kernel from two rocprofv3 --pmc
# passes over this workload (profiles/k_chol_update_n40000_ts768_counters.md):
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors that make a plain 1 GiB
# device copy read and write 1 GiB.  Valid only for the kernel source the
# counters were taken on: the shared GEMM core (common.h) and the text of
# k_chol_update and of its launcher (fingerprint below); otherwise null.
TRAFFIC_BYTES_PER_LAUNCH = (4.9837e6 * 2.0 + 1.0333e6 * 1.0) * 1024
TRAFFIC_FILES = ("paper_1908_06936_amd/csrc/common.h",)
TRAFFIC_FUNCTIONS = ("paper_1908_06936_amd/csrc/k_gemm.hip", ("k_chol_update", "launch_chol_update"))
TRAFFIC_FINGERPRINT = "75b22615e038699458018ddce2e921c3b65fd274"


def _function_text(src: str, name: str) -> str:
    """Source text of the function `name` (signature to its closing brace)."""
    i = src.index(f" {name}(")
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        depth += {"{": 1, "}": -1}.get(src[k], 0)
        if depth == 0:
            return src[i:k + 1]
    raise ValueError(name)


def traffic_fingerprint() -> str:
    import hashlib

    h = hashlib.sha1()
    for f in TRAFFIC_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    path, names = TRAFFIC_FUNCTIONS
    with open(os.path.join(ROOT, path)) as fh:
        src = fh.read()
    for name in names:
        h.update(_function_text(src, name).encode())
    return h.hexdigest()


def traffic_bytes():
    return TRAFFIC_BYTES_PER_LAUNCH if traffic_fingerprint() == TRAFFIC_FINGERPRINT else None


def set_map(ctx, mp):
    """Mixed-precision map of a context: 'default' (the library's correlation
    map with one refinement step), 'fp32' (distance map without BF16 or FP64
    tiles) or 'bf16_3beta' (BF16 beyond 3 beta), the last two unrefined."""
    if mp in (None, "default"):
        ctx.set_mixed_correlation()
        ctx.set_mixed_refinement(1)
    else:
        ctx.set_mixed_policy(0.0 if mp == "fp32" else 3.0, 0.0)
        ctx.set_mixed_refinement(0)


def cpu_baseline(n_full: int, theta, sizes=(400, 700, 1000)) -> dict:
    """The oracle (CPU, FP64) timed on one host core, extrapolated to n_full.

    Runs before any GPU call, in this process: the process is pinned to one
    CPU of its allowed set and the oracle to one OpenMP thread, both restored
    afterwards.  One (l, grad l) per size on the workload's own recipe (U[0,1]^2
    locations, seed 0, the same theta; z standard normal, which costs the same
    as a simulated field).  At these sizes the O(n^2) Bessel-derivative
    quadratures weigh as much as the O(n^3) factorisation and inverse, so the
    times are fitted by t = a n^2 + b n^3 (least squares) and the fit is
    evaluated at n_full; the result is an extrapolation and says so.
    """
    import numpy as np

    import inputgen
    import oracle

    oracle._load()
    host_cores = os.cpu_count()
    aff = os.sched_getaffinity(0)
    threads = oracle.num_threads()
    os.sched_setaffinity(0, {min(aff)})
    oracle.set_threads(1)
    pts = []
    try:
        for n in sizes:
            x, y = inputgen.uniform(n, seed=0)
            z = inputgen.normals(n, seed=0)
            t0 = time.perf_counter()
            oracle.loglik_grad(x, y, z, theta)
            pts.append((n, time.perf_counter() - t0))
            print(f"[bench] cpu oracle n={n}: {pts[-1][1]:.2f} s", file=sys.stderr, flush=True)
    finally:
        oracle.set_threads(threads)
        os.sched_setaffinity(0, aff)
    A = np.array([[float(n) ** 2, float(n) ** 3] for n, _ in pts])
    t = np.array([dt for _, dt in pts])
    (a, b), *_ = np.linalg.lstsq(A, t, rcond=None)
    resid = float(np.max(np.abs(A @ np.array([a, b]) - t) / t))
    t_full = a * n_full ** 2 + b * n_full ** 3
    return {"value": 1.0 / t_full, "unit": "evals/s", "cores": 1, "host_cores": host_cores, "kind": "oracle",
            "extrapolated": True,
            "sample": f"one oracle (l, grad l) at n = {', '.join(str(n) for n, _ in pts)} (U[0,1]^2, seed 0) on one "
                      f"pinned core, one thread; times {', '.join(f'{dt:.2f}' for _, dt in pts)} s; fit "
                      f"t = {a:.3e} n^2 + {b:.3e} n^3 s (max relative residual {resid:.1%}); value = 1 / t({n_full}) "
                      f"= 1 / {t_full:.4g} s, extrapolated",
            "fit": {"a_n2_s": a, "b_n3_s": b, "max_rel_residual": resid, "points": pts,
                    "t_extrapolated_s": t_full}}


def mle_study(args) -> int:
    """Wall clock of the estimators (one JSON line).

    * n = 400 (20 x 20 jittered grid, theta = (1, 0.1, 0.5)): one l and the
      derivative-free MLE from the lower bound, as in the paper's example.
    * n = 40,000 (200 x 200 jittered grid, true theta = (1, 0.1, 0.5) and
      (1, 0.1, 0.8), start (0.5, 0.3, 0.5)): FP64 derivative-free vs FP64
      L-BFGS-B and the mixed-precision L-BFGS-B search with an FP64 finish
      (--mle-all adds plain mixed L-BFGS-B and mixed derivative-free), wall
      clock, theta-hat and l(theta-hat) re-evaluated in FP64.
    * n = side^2 (default 160,000): one FP64 l, one FP64 (l, grad l) and one
      mixed (l, grad l) at the true theta (the full estimators at this size
      take hours of derivative-free evaluations).
    """
    import torch

    import inputgen
    import paper_1908_06936_amd as exa

    dev = torch.device("cuda:0")
    out = {"study": "mle", "data": "synthetic"}

    def field(m, th, seed, ts):
        x, y = inputgen.jittered_grid(m, seed=seed)
        e = inputgen.normals(x.size, seed=seed)
        X, Y, E = (torch.as_tensor(a, device=dev) for a in (x, y, e))
        ctx = exa.Context(ts=ts)
        Z = ctx.simulate(X, Y, th, E)
        torch.cuda.synchronize()
        return ctx, X, Y, Z

    # n = 400, one tile
    th1 = [1.0, 0.1, 0.5]
    ctx, X, Y, Z = field(20, th1, 0, 512)
    ctx.loglik(X, Y, Z, th1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l1 = ctx.loglik(X, Y, Z, th1)
    t1 = time.perf_counter()
    lb, ub = [0.001, 0.001, 0.001], [5.0, 5.0, 5.0]
    th_hat, l_hat, st = ctx.mle(X, Y, Z, lb, ub, tol=1e-4, method="dfo")
    out["n400"] = {"loglik_at_true": l1, "loglik_ms": 1e3 * (t1 - t0), "dfo_theta_hat": th_hat, "dfo_loglik": l_hat,
                   "dfo_stats": st}
    print(f"[mle] n=400 done: {st}", file=sys.stderr, flush=True)
    ctx.close()
    del ctx

    # n = 40,000: estimators compared, for a rough (nu = 0.5) and a smoother
    # (nu = 0.8) field; evaluation caps keep each run within a few minutes.
    # Mixed precision uses the library's default map (tiles by correlation
    # bound, one FP64 refinement step of Sigma^-1 z).
    lb, ub, th0 = [0.01, 0.01, 0.1], [5.0, 2.0, 3.0], [0.5, 0.3, 0.5]
    out["n40000_grid"] = {}
    all_est = {"fp64_dfo": ("dfo", "fp64", 400), "fp64_lbfgsb": ("lbfgsb", "fp64", 80),
               "mixed_lbfgsb": ("lbfgsb", "mixed", 80), "mixed_lbfgsb_fp64_finish": ("lbfgsb_fp64_finish", "mixed", 80),
               "mixed_dfo": ("dfo", "mixed", 400)}
    chosen = args.mle_estimators or ["fp64_dfo", "fp64_lbfgsb", "mixed_lbfgsb", "mixed_lbfgsb_fp64_finish"]
    for th_true in [[1.0, 0.1, nu] for nu in (args.mle_nus if not args.mle_skip_40k else [])]:
        ctx, X, Y, Z = field(200, th_true, 1, 768)
        runs = {}
        for label in chosen:
            meth, prec, cap = all_est[label]
            t0 = time.perf_counter()
            try:
                th_hat, l_hat, st = ctx.mle(X, Y, Z, lb, ub, theta0=th0, tol=1e-4, max_iters=cap, method=meth,
                                            precision=prec)
            except exa.ExaGeoError as err:
                runs[label] = {"error": str(err)}
                continue
            wall = time.perf_counter() - t0
            l64 = ctx.loglik_status(X, Y, Z, th_hat, "fp64")[1]
            runs[label] = {"theta_hat": th_hat, "loglik_reported": l_hat, "loglik_fp64_at_theta_hat": l64,
                           "wall_s": wall, "max_evals": cap, "stats": st,
                           "mixed_policy": "default correlation map, 1 refinement step" if prec == "mixed" else None}
            print(f"[mle] n=40000 nu={th_true[2]} {label}: {wall:.1f} s, theta {th_hat}, {st}", file=sys.stderr,
                  flush=True)
        refl = "fp64_dfo" if "fp64_dfo" in runs else "fp64_lbfgsb"
        ref = runs.get(refl, {}).get("loglik_fp64_at_theta_hat")
        for label, d in runs.items():
            if ref is not None and "loglik_fp64_at_theta_hat" in d:
                d[f"rel_dl_vs_{refl}"] = abs(d["loglik_fp64_at_theta_hat"] - ref) / abs(ref)
                d[f"speedup_vs_{refl}"] = runs[refl]["wall_s"] / d["wall_s"]
        out["n40000_grid"][f"nu={th_true[2]}"] = {"theta_true": th_true, "theta0": th0, "lb": lb, "ub": ub,
                                                  "runs": runs}
        ctx.close()
        del ctx
        torch.cuda.empty_cache()
    th_true = [1.0, 0.1, 0.8]

    # large n: single evaluations
    m = args.big_n_side
    if m <= 0:
        print(json.dumps(out))
        return 0
    ctx, X, Y, Z = field(m, th_true, 2, 768)
    big = {"n": m * m, "mixed_policy": "default correlation map, 1 refinement step"}
    for label, prec, grad in (("fp64_loglik", "fp64", False), ("fp64_loglik_grad", "fp64", True),
                              ("mixed_loglik_grad", "mixed", True)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if grad:
            st_, v, info = ctx.loglik_status(X, Y, Z, th_true, prec)
            if st_ == 0:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                v, g = ctx.loglik_grad(X, Y, Z, th_true, prec)
            else:
                g = None
        else:
            st_, v, info = ctx.loglik_status(X, Y, Z, th_true, prec)
            g = None
        torch.cuda.synchronize()
        big[label] = {"status": exa.STATUS_NAMES.get(st_, st_), "s": time.perf_counter() - t0, "loglik": v, "grad": g}
        print(f"[mle] n={m * m} {label}: {big[label]['s']:.1f} s status {big[label]['status']}", file=sys.stderr,
              flush=True)
    out["large"] = big
    print(json.dumps(out))
    return 0


def mle_large(args) -> int:
    """One estimator on an m x m jittered grid (default 300 x 300, n = 90,000;
    --big-n-side 400 gives n = 160,000), true theta = (1, --mle-beta,
    --mle-nu), start (0.5, 0.3, 0.5) or --theta0, tile 768 (one JSON line;
    progress lines on stderr, one per evaluation).  Estimators: fp64_lbfgsb,
    fp64_dfo, mixed_lbfgsb, mixed_dfo, mixed_lbfgsb_fp64_finish; mixed map
    --mle-policy: default (the library's correlation map with one refinement
    step), fp32 (FP32 off-diagonal tiles) or bf16_3beta (BF16 beyond 3 beta).
    theta-hat and l(theta-hat) re-evaluated in FP64 are reported so that runs
    of different estimators compare directly."""
    import torch

    import inputgen
    import paper_1908_06936_amd as exa

    dev = torch.device("cuda:0")
    m, beta = args.big_n_side, args.mle_beta
    x, y = inputgen.jittered_grid(m, seed=0)
    e = inputgen.normals(x.size, seed=0)
    X, Y, E = (torch.as_tensor(a, device=dev) for a in (x, y, e))
    ctx = exa.Context(ts=768)
    th_true = [1.0, beta, args.mle_nu]
    t_sim = time.perf_counter()
    Z = ctx.simulate(X, Y, th_true, E)
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t_sim
    lb, ub = [0.01, 0.001, 0.1], [5.0, 2.0, 3.0]
    # a later segment of a long estimation restarts from an earlier one's
    # best point (the quasi-Newton curvature pairs are not carried over)
    th0 = list(args.theta0) if args.theta0 else [0.5, 0.3, 0.5]
    meth, prec = {"fp64_lbfgsb": ("lbfgsb", "fp64"), "fp64_dfo": ("dfo", "fp64"), "mixed_dfo": ("dfo", "mixed"),
                  "mixed_lbfgsb": ("lbfgsb", "mixed"),
                  "mixed_lbfgsb_fp64_finish": ("lbfgsb_fp64_finish", "mixed")}[args.mle_estimator]
    if args.mle_policy == "default":
        ctx.set_mixed_correlation()  # the library's default map
    else:
        ctx.set_mixed_policy(3.0 if args.mle_policy == "bf16_3beta" else 0.0)
        ctx.set_mixed_refinement(0)
    ctx.set_verbose(True)
    print(f"[mle-large] n={x.size} beta={beta} {args.mle_estimator} policy={args.mle_policy} cap={args.mle_cap}",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    th_hat, l_hat, st = ctx.mle(X, Y, Z, lb, ub, theta0=th0, tol=1e-4, max_iters=args.mle_cap, method=meth,
                                precision=prec)
    wall = time.perf_counter() - t0
    ctx.set_verbose(False)
    l64 = ctx.loglik_status(X, Y, Z, th_hat, "fp64")[1]
    out = {"study": "mle_large", "n": int(x.size), "grid": f"{m}x{m} jittered, seed 0", "data": "synthetic",
           "simulate_s": t_sim, "segment_start": "restart" if args.theta0 else "initial",
           "theta_true": th_true, "theta0": th0, "lb": lb, "ub": ub, "estimator": args.mle_estimator,
           "mixed_policy": args.mle_policy if prec == "mixed" else None, "max_evals": args.mle_cap,
           "theta_hat": th_hat, "loglik_reported": l_hat, "loglik_fp64_at_theta_hat": l64, "wall_s": wall,
           "stats": st}
    print(json.dumps(out))
    return 0


PRECISION_POLICIES = {
    # label: (kind, parameters, refinement steps)
    "corr_0.3_1e-4": ("corr", (0.3, 1e-4), 1),
    "corr_0.3_1e-4_norefine": ("corr", (0.3, 1e-4), 0),
    "corr_0.3_1e-4_refine2": ("corr", (0.3, 1e-4), 2),
    "corr_0.5_1e-3": ("corr", (0.5, 1e-3), 1),
    "corr_0.1_1e-5": ("corr", (0.1, 1e-5), 1),
    "corr_0.3_nobf16": ("corr", (0.3, 0.0), 1),
    "dist_fp32_only": ("dist", (0.0, 0.0), 0),
    "dist_bf16_3beta": ("dist", (3.0, 0.0), 0),
    "dist_fp32_fp64band_0.5beta": ("dist", (0.0, 0.5), 0),
}


def _apply_policy(ctx, label):
    kind, prm, refine = PRECISION_POLICIES[label]
    if kind == "corr":
        ctx.set_mixed_correlation(*prm)
    else:
        ctx.set_mixed_policy(*prm)
    ctx.set_mixed_refinement(refine)


def precision_study(args) -> int:
    """l (and, where asked, (l, grad l)) in FP64 and under several mixed-
    precision maps (one JSON line): the relative error of l against the FP64
    path split into its log-det and quadratic-form parts, the score error per
    component relative to max |g|, tile fractions, and times.

    Fields (tile 768): the 300 x 300 jittered grid (n = 90,000, theta = (1,
    beta, 0.5), beta in {0.03, 0.1}); the 200 x 200 jittered grid (n = 40,000,
    beta in {0.03, 0.1}, nu in {0.5, 1.0}, with scores); the n = 40,000
    uniform field of the headline workload (nu = 1); sorted points on a line
    with mean gap 5e-4 (n = 40,000, beta = 0.1, nu = 0.5), whose exact l is
    the O(n) Markov closed form.  --precision-policies picks the maps."""
    import math

    import numpy as np
    import torch

    import inputgen
    import paper_1908_06936_amd as exa

    dev = torch.device("cuda:0")
    ctx = exa.Context(ts=768)
    labels = args.precision_policies or list(PRECISION_POLICIES)
    out = {"study": "precision", "data": "synthetic", "policies": {k: PRECISION_POLICIES[k] for k in labels}}

    def run(name, X, Y, Z, th, with_grad, exact=None):
        res = {}
        for label in ["fp64"] + labels:
            prec = "fp64" if label == "fp64" else "mixed"
            if label != "fp64":
                _apply_policy(ctx, label)
            st, v, info = ctx.loglik_status(X, Y, Z, th, prec)  # warm-up / status
            if st != 0:
                res[label] = {"status": exa.STATUS_NAMES.get(st, st), "info": info}
                print(f"[precision] {name} {label}: status {res[label]['status']}", file=sys.stderr, flush=True)
                continue
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v = ctx.loglik(X, Y, Z, th, prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            tm = ctx.timings()
            d = {"status": "OK", "loglik": v, "loglik_s": t1 - t0, "logdet": tm["logdet"], "quad_form": tm["quad_form"],
                 "frac_bf16": tm.get("frac_bf16"), "frac_fp64": tm.get("frac_fp64"), "frac_fp32": tm.get("frac_fp32")}
            if with_grad:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, g = ctx.loglik_grad(X, Y, Z, th, prec)
                torch.cuda.synchronize()
                d["grad"] = g
                d["loglik_grad_s"] = time.perf_counter() - t0
            res[label] = d
            print(f"[precision] {name} {label}: l {v:.12g} ({d['loglik_s']:.3f} s) bf16 {d['frac_bf16']} "
                  f"fp64 {d['frac_fp64']}", file=sys.stderr, flush=True)
        ref = res["fp64"]
        for label, d in res.items():
            if d.get("status") != "OK":
                continue
            if exact is not None:
                d["rel_err_vs_exact"] = abs(d["loglik"] - exact) / abs(exact)
            if label == "fp64" or ref.get("status") != "OK":
                continue
            L = abs(ref["loglik"])
            d["rel_err_vs_fp64"] = abs(d["loglik"] - ref["loglik"]) / L
            d["rel_err_logdet_part"] = 0.5 * abs(d["logdet"] - ref["logdet"]) / L
            d["rel_err_quad_part"] = 0.5 * abs(d["quad_form"] - ref["quad_form"]) / L
            d["speedup_l"] = ref["loglik_s"] / d["loglik_s"]
            if with_grad:
                gmax = max(abs(q) for q in ref["grad"])
                d["grad_err_over_max_abs_grad"] = [abs(a - b) / gmax for a, b in zip(d["grad"], ref["grad"])]
                d["grad_rel_err_per_component"] = [abs(a - b) / abs(b) for a, b in zip(d["grad"], ref["grad"])]
                d["speedup_l_grad"] = ref["loglik_grad_s"] / d["loglik_grad_s"]
        out[name] = res

    # config 4: 300 x 300 jittered grid
    if not args.precision_skip_90k:
        x, y = inputgen.jittered_grid(300, seed=0)
        X, Y = torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev)
        E = torch.as_tensor(inputgen.normals(x.size, seed=0), device=dev)
        for beta in (0.03, 0.1):
            th = [1.0, beta, 0.5]
            Z = ctx.simulate(X, Y, th, E)
            run(f"grid300_beta{beta}_nu0.5", X, Y, Z, th, False)
        del X, Y, E, Z
    # 200 x 200 jittered grid with scores
    x, y = inputgen.jittered_grid(200, seed=0)
    X, Y = torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev)
    E = torch.as_tensor(inputgen.normals(x.size, seed=0), device=dev)
    for beta, nu in ((0.03, 0.5), (0.1, 0.5), (0.1, 1.0)):
        th = [1.0, beta, nu]
        Z = ctx.simulate(X, Y, th, E)
        run(f"grid200_beta{beta}_nu{nu}", X, Y, Z, th, True)
    # the headline field: 40,000 uniform points, nu = 1
    x, y = inputgen.uniform(40000, seed=0)
    X, Y = torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev)
    th = [1.0, 0.1, 1.0]
    Z = ctx.simulate(X, Y, th, E)
    run("uniform40000_beta0.1_nu1.0", X, Y, Z, th, True)
    # Markov line: exact l in O(n)
    n, s2, beta = 40000, 1.0, 0.1
    t, y0 = inputgen.collinear(n, mean_gap=5e-4, seed=11)
    e = inputgen.normals(n, seed=11)
    rho = np.exp(-np.diff(t) / beta)
    z = np.empty(n)
    z[0] = math.sqrt(s2) * e[0]
    for i in range(1, n):
        z[i] = rho[i - 1] * z[i - 1] + math.sqrt(s2 * (1 - rho[i - 1] ** 2)) * e[i]
    v = s2 * (1 - rho ** 2)
    exact = -0.5 * (math.log(2 * math.pi) + math.log(s2) + z[0] ** 2 / s2)
    exact += float(np.sum(-0.5 * (math.log(2 * math.pi) + np.log(v) + (z[1:] - rho * z[:-1]) ** 2 / v)))
    X, Y, Z = (torch.as_tensor(a, device=dev) for a in (t, y0, z))
    run("markov_line40000_gap5e-4", X, Y, Z, [s2, beta, 0.5], False, exact=exact)
    print(json.dumps(out))
    return 0


def profile_mixed(args) -> int:
    """A short run to profile under rocprofv3: --profile-steps (l, grad l)
    evaluations in --profile-precision (mixed: the library's default map) on
    the m x m jittered grid (--big-n-side, default 200: n = 40,000), theta =
    (1, --mle-beta, --profile-nu), or with --profile-field uniform on the
    headline workload (n = m^2 uniform points, theta = (1, 0.1, 1.0)), tile
    768, after one warm-up, with the BF16 targets on --profile-bf16-block
    blocks; one JSON line with the per-phase times and tile fractions."""
    import torch

    import inputgen
    import paper_1908_06936_amd as exa

    dev = torch.device("cuda:0")
    m = args.big_n_side
    if args.profile_field == "uniform":
        # the headline workload: n = m^2 uniform points, theta = (1, 0.1, 1.0)
        x, y = inputgen.uniform(m * m, seed=0)
        th = [1.0, 0.1, 1.0]
    else:
        x, y = inputgen.jittered_grid(m, seed=0)
        th = [1.0, args.mle_beta, args.profile_nu]
    X, Y = torch.as_tensor(x, device=dev), torch.as_tensor(y, device=dev)
    E = torch.as_tensor(inputgen.normals(x.size, seed=0), device=dev)
    ctx = exa.Context(ts=768)
    ctx.set_mixed_bf16_block(args.profile_bf16_block)
    Z = ctx.simulate(X, Y, th, E)
    prec = args.profile_precision
    ctx.loglik_grad(X, Y, Z, th, prec)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.profile_steps):
        ll, g = ctx.loglik_grad(X, Y, Z, th, prec)
        print(f"[profile] step {s + 1}/{args.profile_steps} l={ll:.10g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.profile_steps
    tm = ctx.timings()
    print(json.dumps({"study": "profile", "n": int(x.size), "theta": th, "precision": prec, "s_per_step": dt,
                      "timings": tm}))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=40000)
    ap.add_argument("--ts", type=int, default=768)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the n = 10,000 and n = 400 studies (profiles of the n = 40,000 kernels alone)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the l-only and FP64-vs-mixed sections (profiling runs of the headline step)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--mle-study", action="store_true",
                    help="instead of the throughput step: the MLE comparisons (FP64 derivative-free vs "
                         "gradient-based and mixed precision) and single evaluations at n = 160,000")
    ap.add_argument("--big-n-side", type=int, default=400,
                    help="grid side of the large single evaluations (0: skip them)")
    ap.add_argument("--mle-estimators", nargs="+", default=None,
                    choices=["fp64_dfo", "fp64_lbfgsb", "mixed_lbfgsb", "mixed_lbfgsb_fp64_finish", "mixed_dfo"],
                    help="estimators of --mle-study at n = 40,000 (default: all but mixed_dfo)")
    ap.add_argument("--mle-nus", type=float, nargs="+", default=[0.5, 0.8], help="true nu of the n = 40,000 fields")
    ap.add_argument("--mle-skip-40k", action="store_true", help="--mle-study without the n = 40,000 estimators")
    ap.add_argument("--mle-large", action="store_true",
                    help="instead of the throughput step: one estimator on the --big-n-side grid (see mle_large)")
    ap.add_argument("--mle-beta", type=float, default=0.03)
    ap.add_argument("--mle-nu", type=float, default=0.5, help="true nu of --mle-large")
    ap.add_argument("--theta0", type=float, nargs=3, default=None,
                    help="start of --mle-large (default (0.5, 0.3, 0.5)); a restart point for a second segment")
    ap.add_argument("--mle-estimator", default="fp64_lbfgsb",
                    choices=["fp64_lbfgsb", "fp64_dfo", "mixed_dfo", "mixed_lbfgsb", "mixed_lbfgsb_fp64_finish"])
    ap.add_argument("--mle-policy", default="default", choices=["default", "fp32", "bf16_3beta"])
    ap.add_argument("--mle-cap", type=int, default=60, help="evaluation cap of --mle-large")
    ap.add_argument("--precision-study", action="store_true",
                    help="instead of the throughput step: FP64 vs mixed-precision l and scores under several "
                         "precision maps (see precision_study)")
    ap.add_argument("--precision-policies", nargs="+", choices=sorted(PRECISION_POLICIES), default=None)
    ap.add_argument("--precision-skip-90k", action="store_true")
    ap.add_argument("--profile-mixed", action="store_true",
                    help="instead of the throughput step: a short (l, grad l) run to profile (see profile_mixed)")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--profile-nu", type=float, default=0.5)
    ap.add_argument("--profile-precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--profile-field", default="grid", choices=["grid", "uniform"])
    ap.add_argument("--profile-bf16-block", type=int, default=256, choices=[128, 256],
                    help="output block edge of the BF16 targets' update in --profile-mixed")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch

        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8}))
        return 0

    if args.profile_mixed:
        if args.big_n_side == 400 and "--big-n-side" not in sys.argv:
            args.big_n_side = 200
        if "--mle-beta" not in sys.argv:
            args.mle_beta = 0.1
        return profile_mixed(args)
    if args.mle_study:
        return mle_study(args)
    if args.precision_study:
        return precision_study(args)
    if args.mle_large:
        if args.big_n_side == 400 and "--big-n-side" not in sys.argv:
            args.big_n_side = 300
        return mle_large(args)

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "this path runs on one GPU; its multi-GPU sharding is not built.", file=sys.stderr)
        return 2

    n, ts = args.n, args.ts
    theta = [1.0, 0.1, 1.0]
    # the CPU oracle first, before anything touches the GPU
    cpu = None if args.no_cpu else cpu_baseline(n, theta)

    import torch

    import inputgen
    import paper_1908_06936_amd as exa

    dev = torch.device("cuda:0")
    x, y = inputgen.uniform(n, seed=0)
    e = inputgen.normals(n, seed=0)
    X = torch.as_tensor(x, device=dev)
    Y = torch.as_tensor(y, device=dev)
    E = torch.as_tensor(e, device=dev)
    ctx = exa.Context(ts=ts, device=0)
    Z = ctx.simulate(X, Y, theta, E)  # untimed input preparation
    torch.cuda.synchronize()
    print(f"[bench] n={n} ts={ts} data ready", file=sys.stderr, flush=True)

    for w in range(args.warmup):
        ctx.loglik_grad(X, Y, Z, theta)
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    per = []
    lls = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        ll, g = ctx.loglik_grad(X, Y, Z, theta)
        per.append(ctx.timings())
        lls.append((ll, g))
        print(f"[bench] step {s + 1}/{args.steps} loglik={ll:.10g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    def avg(key):
        return sum(p[key] for p in per) / len(per)

    ms_step = 1000.0 * elapsed / args.steps
    chol_ms = avg("chol_ms")
    chol_tflops = avg("chol_flops") / (chol_ms * 1e-3) / 1e12
    upd_ms = avg("update_kernel_ms")
    upd_flops = avg("update_flops")
    upd_launch = avg("update_launches")
    achieved = upd_flops / (upd_ms * 1e-3) / 1e12
    result = {
        # value: FP64 (l, grad l) evaluations/s on the headline workload; the
        # mixed-precision rates (that field does not factor in FP32, so they
        # are measured on the 200 x 200 grid) and POTRF TFLOP/s are the keys
        # "fp64_vs_mixed_jittered_grid_200x200", "mixed_summary", "potrf_*"
        "metric": "loglik+grad evals/s at n=40K (FP64 vs mixed); POTRF TFLOP/s vs MFMA peak",
        "value": args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"exact FP64 (l, grad l), n={n} U[0,1]^2 locations seed 0, "
                               f"Matern theta=(1, 0.1, 1.0), tile {ts}, z simulated from the same field",
                   "n": n, "ts": ts, "theta": theta},
        "roofline": {"bound": "mfma", "kernel": "k_chol_update (trailing SYRK/GEMM of the tile Cholesky)",
                     "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": traffic_bytes(),
                     "traffic_unit": "bytes per launch (HBM fetch + write)",
                     "flops_per_launch": upd_flops / max(upd_launch, 1),
                     "avg_launch_ms": upd_ms / max(upd_launch, 1)},
        "potrf_tflops": chol_tflops,
        "potrf_frac_of_fp64_mfma_peak": chol_tflops / FP64_MFMA_PEAK_TFLOPS,
        "phases_ms": {k: avg(k) for k in ("prep_ms", "gen_ms", "chol_ms", "solve_ms", "grad_ms", "total_ms")},
        "gen_bessel_evals_per_s": (n * (n + 1) / 2) / (avg("gen_ms") * 1e-3),
        # generation writes the lower tiles once; the forward solve reads them once
        "gen_hbm_write_gbs": ((n + ts - 1) // ts) * (((n + ts - 1) // ts) + 1) / 2 * ts * ts * 8
                             / (avg("gen_ms") * 1e-3) / 1e9,
        "solve_hbm_read_gbs": ((n + ts - 1) // ts) * (((n + ts - 1) // ts) + 1) / 2 * ts * ts * 8
                              / (avg("solve_ms") * 1e-3) / 1e9,
        "loglik": lls[-1][0],
        "grad": lls[-1][1],
    }
    if not args.no_studies:
        # the two small studies of the workload list: n = 10,000 (100 x 100
        # jittered grid, tile 512, six (beta, nu)), one l each; n = 400 (20 x 20
        # jittered grid, theta = (1, 0.1, 0.5)), one l and the derivative-free MLE
        # from the lower bound (0.001, 0.001, 0.001) with tolerance 1e-4
        x2, y2 = inputgen.jittered_grid(100, seed=0)
        X2, Y2 = torch.as_tensor(x2, device=dev), torch.as_tensor(y2, device=dev)
        E2 = torch.as_tensor(inputgen.normals(x2.size, seed=0), device=dev)
        ctx2 = exa.Context(ts=512, device=0)
        c2 = {}
        for nu in (0.5, 1.0):
            for beta in (0.03, 0.1, 0.3):
                th2 = [1.0, beta, nu]
                Z2 = ctx2.simulate(X2, Y2, th2, E2)
                ctx2.loglik(X2, Y2, Z2, th2)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                l2 = ctx2.loglik(X2, Y2, Z2, th2)
                torch.cuda.synchronize()
                c2[f"beta={beta},nu={nu}"] = {"loglik": l2, "ms": 1e3 * (time.perf_counter() - t1)}
        result["n10000_grid_ts512_one_loglik"] = c2
        x1, y1 = inputgen.jittered_grid(20, seed=0)
        X1, Y1 = torch.as_tensor(x1, device=dev), torch.as_tensor(y1, device=dev)
        E1 = torch.as_tensor(inputgen.normals(x1.size, seed=0), device=dev)
        th1 = [1.0, 0.1, 0.5]
        Z1 = ctx2.simulate(X1, Y1, th1, E1)
        ctx2.loglik(X1, Y1, Z1, th1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        l1 = ctx2.loglik(X1, Y1, Z1, th1)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        th1_hat, l1_hat, st1 = ctx2.mle(X1, Y1, Z1, [0.001] * 3, [5.0] * 3, tol=1e-4, method="dfo")
        result["n400_grid"] = {"loglik": l1, "loglik_ms": 1e3 * (t2 - t1), "dfo_theta_hat": th1_hat,
                               "dfo_loglik": l1_hat, "dfo_wall_s": st1["total_s"], "dfo_evals": st1["n_evals"],
                               "dfo_per_eval_ms": 1e3 * st1["per_eval_s"], "dfo_status": st1["status"]}
        ctx2.close()
        print("[bench] n = 10,000 and n = 400 studies done", file=sys.stderr, flush=True)
    # kriging at 1,000 new points from the same data (factorisation included)
    xq, yq = inputgen.uniform(1000, seed=5)
    Xq, Yq = torch.as_tensor(xq, device=dev), torch.as_tensor(yq, device=dev)
    ctx.predict(X, Y, Z, theta, Xq, Yq, with_mse=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.predict(X, Y, Z, theta, Xq, Yq, with_mse=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.predict(X, Y, Z, theta, Xq, Yq, with_mse=True)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    result["kriging_m1000"] = {"mean_ms": 1e3 * (t2 - t1), "mean_and_mse_ms": 1e3 * (t3 - t2),
                               "note": "factorisation of the n = 40,000 covariance included"}
    # Fisher information at theta (FP64; factorisation and L^-1 included)
    ctx.fisher(X, Y, theta)  # warm-up (allocates its 3 n^2 doubles per call)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fish = ctx.fisher(X, Y, theta)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tf = ctx.timings()
    result["fisher_information"] = {
        "call_ms": 1e3 * (t2 - t1), "fisher_phase_ms": tf["grad_ms"], "product_flops": tf["fisher_flops"],
        "phase_tflops": tf["fisher_flops"] / (tf["grad_ms"] * 1e-3) / 1e12,
        "note": "phase = L^-1, the two derivative matrices, B_j = L^-1 dSigma_j L^-T, the reduction",
        "I": fish.tolist()}
    print("[bench] Fisher done", file=sys.stderr, flush=True)
    if cpu is not None:
        result["cpu_baseline"] = cpu
    if args.no_mixed:
        print(json.dumps(result))
        return 0
    # l(theta) alone, FP64 and mixed precision on the same inputs: the
    # library's default map (tiles by correlation bound, one FP64 refinement
    # step) and, for the record, the distance maps FP32-only and BF16 beyond
    # 3 beta without refinement (this smooth nu = 1 field on uniform points
    # does not factor with FP32 tiles next to the diagonal: ENOTPD)
    ctx.set_profiling(False)
    ll_only = {}
    for label, prec, mp in (("fp64", "fp64", None), ("mixed_default_map", "mixed", "default"),
                               ("mixed_fp32_only", "mixed", "fp32"), ("mixed_bf16_3beta", "mixed", "bf16_3beta")):
        set_map(ctx, mp)
        st, v, info = ctx.loglik_status(X, Y, Z, theta, prec)  # warm-up / status
        if st != 0:
            ll_only[label] = {"status": exa.STATUS_NAMES.get(st, st), "info": info}
            print(f"[bench] loglik-only {label}: status {st}", file=sys.stderr, flush=True)
            continue
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            v = ctx.loglik(X, Y, Z, theta, prec)
        torch.cuda.synchronize()
        rate = args.steps / (time.perf_counter() - t1)
        tmo = ctx.timings()
        ll_only[label] = {"status": "OK", "evals_per_s": rate, "loglik": v,
                          "frac_bf16_tiles": tmo.get("frac_bf16"), "frac_fp64_tiles": tmo.get("frac_fp64")}
        if label == "mixed_default_map":
            # (l, grad l) in mixed precision on the headline field
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                lg, gg = ctx.loglik_grad(X, Y, Z, theta, prec)
            torch.cuda.synchronize()
            ll_only[label]["loglik_grad_evals_per_s"] = args.steps / (time.perf_counter() - t1)
            ll_only[label]["grad"] = gg
            g64 = result["grad"]
            gmax = max(abs(q) for q in g64)
            ll_only[label]["grad_err_vs_fp64_over_max_abs_grad"] = [abs(a - b) / gmax for a, b in zip(gg, g64)]
        print(f"[bench] loglik-only {label}: {rate:.3f} evals/s", file=sys.stderr, flush=True)
    set_map(ctx, "default")
    l64 = ll_only["fp64"].get("loglik")
    for label, d in ll_only.items():
        if label != "fp64" and "loglik" in d and l64 is not None:
            d["rel_err_vs_fp64"] = abs(d["loglik"] - l64) / abs(l64)
    result["loglik_only"] = ll_only

    # FP64 vs mixed precision, l alone and (l, grad l), on a 200 x 200
    # jittered grid (n = 40,000), where the minimum spacing keeps the
    # lower-precision tiles positive definite
    xg, yg = inputgen.jittered_grid(200, seed=0)
    Xg, Yg = torch.as_tensor(xg, device=dev), torch.as_tensor(yg, device=dev)
    grid = {}
    for th_g in ([1.0, 0.1, 0.5], [1.0, 0.03, 0.5]):
        Zg = ctx.simulate(Xg, Yg, th_g, E)
        key = f"beta={th_g[1]},nu={th_g[2]}"
        grid[key] = {}
        for label, prec, mp in (("fp64", "fp64", None), ("mixed_default_map", "mixed", "default"),
                               ("mixed_fp32_only", "mixed", "fp32"), ("mixed_bf16_3beta", "mixed", "bf16_3beta")):
            set_map(ctx, mp)
            st, v, info = ctx.loglik_status(Xg, Yg, Zg, th_g, prec)
            if st != 0:
                grid[key][label] = {"status": exa.STATUS_NAMES.get(st, st), "info": info}
                continue
            ctx.set_profiling(True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                v = ctx.loglik(Xg, Yg, Zg, th_g, prec)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tm = ctx.timings()
            ctx.set_profiling(False)
            for _ in range(args.steps):
                lg, gg = ctx.loglik_grad(Xg, Yg, Zg, th_g, prec)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            # trailing update: achieved rate against the peak weighted by the
            # precision of its flops, 1 / sum(share_p / peak_p)
            fl = [tm["update_flops_fp32"], tm["update_flops_bf16"], tm["update_flops_fp64"]]
            wpeak = sum(fl) / sum(f / pk for f, pk in zip(fl, (157.3, 2500.0, FP64_MFMA_PEAK_TFLOPS)))
            upd = tm["update_flops"] / (tm["update_kernel_ms"] * 1e-3) / 1e12
            grid[key][label] = {"status": "OK", "loglik_evals_per_s": args.steps / (t2 - t1),
                                "loglik_grad_evals_per_s": args.steps / (t3 - t2), "loglik": v, "grad": gg,
                                "frac_bf16_tiles": tm.get("frac_bf16"), "frac_fp64_tiles": tm.get("frac_fp64"),
                                "update_flop_shares_fp32_bf16_fp64": [f / sum(fl) for f in fl],
                                "update_tflops": upd, "update_weighted_peak_tflops": wpeak,
                                "update_frac_of_weighted_peak": upd / wpeak}
        ref = grid[key]["fp64"]
        for label, d in grid[key].items():
            if label != "fp64" and "loglik" in d and "loglik" in ref:
                d["rel_err_loglik_vs_fp64"] = abs(d["loglik"] - ref["loglik"]) / abs(ref["loglik"])
                gmax = max(abs(q) for q in ref["grad"])
                d["grad_err_vs_fp64_over_max_abs_grad"] = [abs(a - b) / gmax for a, b in zip(d["grad"], ref["grad"])]
                d["loglik_grad_speedup_vs_fp64"] = d["loglik_grad_evals_per_s"] / ref["loglik_grad_evals_per_s"]
        print(f"[bench] jittered grid {key} done", file=sys.stderr, flush=True)
    set_map(ctx, "default")
    result["fp64_vs_mixed_jittered_grid_200x200"] = grid
    g03 = grid.get("beta=0.03,nu=0.5", {})
    result["mixed_summary"] = {
        "workload": "n=40,000 200x200 jittered grid, theta=(1, 0.03, 0.5), tile 768",
        **{f"{label}_loglik_grad_evals_per_s": d.get("loglik_grad_evals_per_s") for label, d in g03.items()},
        **{f"{label}_rel_err_loglik": d.get("rel_err_loglik_vs_fp64") for label, d in g03.items() if label != "fp64"}}

    # DST approximation (tiles |I - J| >= band set to zero) on the same grid,
    # theta = (1, 0.005, 0.5): l alone, rate and difference from the exact l.
    # Zeroing tiles can leave an indefinite matrix: at beta = 0.01 and above
    # every band here fails the factorisation on this grid (pairs of adjacent
    # points across the Z-curve's quadrant seams are dropped), at 0.005 all pass
    th_d = [1.0, 0.005, 0.5]
    Zd = ctx.simulate(Xg, Yg, th_d, E)
    dst = {}
    for band in (0, 26, 16, 8, 4, 2):
        ctx.set_dst_band(band)
        st, v, info = ctx.loglik_status(Xg, Yg, Zd, th_d)
        if st != 0:
            dst[f"band={band}"] = {"status": exa.STATUS_NAMES.get(st, st)}
            continue
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            v = ctx.loglik(Xg, Yg, Zd, th_d)
        torch.cuda.synchronize()
        dst[f"band={band}"] = {"status": "OK", "loglik_evals_per_s": args.steps / (time.perf_counter() - t1),
                               "loglik": v}
    ctx.set_dst_band(0)
    exact = dst["band=0"]
    for d in dst.values():
        if "loglik" in d:
            d["rel_dl_vs_exact"] = abs(d["loglik"] - exact["loglik"]) / abs(exact["loglik"])
            d["speedup_vs_exact"] = d["loglik_evals_per_s"] / exact["loglik_evals_per_s"]
    result["dst_jittered_grid_200x200_beta0.005"] = dst
    print("[bench] DST done", file=sys.stderr, flush=True)
    print(json.dumps(result))
    return 0


if __name__ == "__main__":
    sys.exit(main())
