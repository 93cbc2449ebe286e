"""Marginal-likelihood gradient steps per second on one MI355X.

Workload (the precision workload the metric is quoted on): n = 434,874 inputs
x ~ U[-1, 1]^3, targets from a 2,048-feature random-Fourier Matern-3/2 draw
with length scales U[0.05, 0.2] plus noise sigma = 0.05; s = 64 probe vectors.
One step = one marginal-likelihood optimisation step of the paper's method:
pathwise right-hand sides from fixed random features (1,000 sin/cos pairs),
warm-started CG with a pivoted-Cholesky preconditioner (App. B; rank 32000 by
default, the paper's experiments use 100; by default the factor built in the first
step serves the whole run, with sigma^2 I + L^T L refactored in every step) to
relative residual 1e-2 (both mean and probe criteria, accepted on the FP32 true
residual), the gradient estimate and one Adam step (lr 0.03, softplus).  Inputs are
resident in HBM before the timed region.  The first W steps (the first one cold,
from U = 0) run as untimed warm-up; the next K steps, warm-started from the
previous solution as in the paper's optimisation runs, are timed.

Forms:
  bf16x3+adjoint  products on bf16 MFMA with hi/lo splitting, FP32 true-residual
                  acceptance, one fused adjoint pass for the gradient (the value).
  fp32-plain      FP32 products, d+1 separate derivative-kernel passes for the
                  gradient; by default one step of each form is timed after
                  the timed region, from the same state, for the ratio.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects).
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# the solver prints a progress line on stderr every 30 s of a long solve
os.environ.setdefault("GPMI_PROGRESS", "30")

METRIC = "MLL-grad steps/s at n=434,874, BF16+adjoint vs FP32 plain, rel-res 1e-2"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3
# VALU issue model of the chip: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-slots/s;
# an FP32 FMA is one slot (2 flops); v_sqrt_f32 / v_exp_f32 are half rate on gfx950
# (measured: 8.5 vs 4.6 SIMD cycles per wave64 instruction), i.e. 2 slots each.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
# Vector-ALU instructions the dominant kernel issues per kernel entry, from its
# counters (SQ_INSTS_VALU - SQ_INSTS_MFMA, SQ_INSTS_VALU_TRANS_F32, per wave-step
# of 64 rows x 32 columns): simple ops, and transcendentals (sqrt, exp2).
VALU_SIMPLE_PER_ENTRY = 5.5
VALU_TRANS_PER_ENTRY = 2.0
# contraction length of the squared-distance MFMA at d <= 3 ([-2x, |x|^2] . [x, 1])
XT_KDIM = 4
# HBM bytes per launch of the dominant kernel from two counter passes (FETCH_SIZE,
# then WRITE_SIZE) over `bench.py --kernel-only 2`, each scaled by the same
# counter's reading for the plain 1 GiB device copy of `bench.py --copy-probe 1024`
# (FETCH_SIZE counted 524,300 per GiB read, WRITE_SIZE 1,048,576 per GiB written).
# The figure belongs to the kernel sources it was taken on: when their hash
# differs, the traffic is reported as null.
TRAFFIC = {"sources_sha256": "4d5ab6df0c99541950927944ac58b299eae299b15373d6366433cb64fee062f2",
           "fetch_bytes": 8.5089e+09, "write_bytes": 2.7837e+08}
TRAFFIC_SOURCES = ("fwd.hip", "dispatch.hip", "gpk.h")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", choices=["bf16x3+adjoint", "fp32-plain"], default="bf16x3+adjoint")
    ap.add_argument("--compare-steps", type=int, default=1,
                    help="after the timed region, time this many steps of both forms from the "
                         "same state (warm start, Adam moments, cached factor) for the metric's "
                         "bf16x3+adjoint / fp32-plain ratio (0 = skip)")
    ap.add_argument("--n", type=int, default=None, help="override n (smaller runs; not the metric)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=1024)
    ap.add_argument("--cpu-rows-1core", type=int, default=128)
    ap.add_argument("--kernel-only", type=int, default=0, metavar="K",
                    help="only time K launches of the forward product on the bench inputs "
                         "(65 columns, same launch configuration); for profilers")
    ap.add_argument("--precision", choices=["bf16x3", "fp32", "bf16"], default="bf16x3",
                    help="product precision for --kernel-only")
    ap.add_argument("--precond-reuse", type=int, default=1000,
                    help="later steps that may reuse a pivoted-Cholesky factor (0 = rebuild in "
                         "every step; default 1000: the factor built in the first step serves "
                         "the whole run)")
    ap.add_argument("--compare-after-s", type=float, default=520.0,
                    help="skip the comparison steps when the run has already taken this long "
                         "(keeps the whole run within a 600 s limit)")
    ap.add_argument("--precond-rank", type=int, default=32000,
                    help="rank of CG's pivoted-Cholesky preconditioner (the paper uses 100; the "
                         "library allows up to 32768; 0 = none)")
    ap.add_argument("--probe-scaling", action="store_true",
                    help="only time the forward product at 1..256 columns on the bench inputs "
                         "(cost of adding probe vectors)")
    ap.add_argument("--theta0", choices=["true", "heuristic"], default="true",
                    help="starting hyperparameters of the timed run: the data-generating theta, "
                         "or the initial-hyperparameter heuristic of the large data sets "
                         "(App. B; computed before the timed region and reported)")
    ap.add_argument("--init-heuristic", action="store_true",
                    help="time the initial-hyperparameter heuristic instead (own JSON line)")
    ap.add_argument("--init-centres", type=int, default=10)
    ap.add_argument("--init-steps", type=int, default=100)
    ap.add_argument("--init-m", type=int, default=10_000)
    ap.add_argument("--init-single", type=int, default=10,
                    help="single evaluations timed for the roofline of the heuristic line")
    ap.add_argument("--early-stop", action="store_true",
                    help="the early-stopping workload instead (n = 2,049,280, d = 11): pathwise "
                         "steps with a budget of 10 solver epochs each, warm-started and cold, "
                         "true relative residual of every budgeted solution (own JSON line)")
    ap.add_argument("--es-steps", type=int, default=3, help="steps per leg of --early-stop")
    ap.add_argument("--es-epochs", type=float, default=10.0)
    ap.add_argument("--es-solver", choices=["cg", "ap", "sgd"], default="cg")
    ap.add_argument("--es-rank", type=int, default=100,
                    help="pivoted-Cholesky rank of --early-stop (the paper's CG uses 100)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 3 plain device copies of MIB MiB (calibrates the HBM "
                         "byte counters of a profiler against a known traffic)")
    return ap.parse_args()


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "launches": 3}), flush=True)


def kernel_only(args):
    import torch
    from paper_2405_18457_amd import api
    ctx = api.Context(0)
    inp, _, dev = make_inputs(args.n)
    n = inp["n"]
    prec = {"bf16x3": api.GP_BF16X3, "fp32": api.GP_FP32, "bf16": api.GP_BF16}[args.precision]
    V = dev(np.random.default_rng(1).standard_normal((n, inp["w"].s + 1)).astype(np.float32))
    out = torch.empty_like(V)
    api.gp_kmatvec(ctx, inp["X"], inp["X"], inp["theta_true"], V, prec, True, out)  # warm
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.kernel_only):
        api.gp_kmatvec(ctx, inp["X"], inp["X"], inp["theta_true"], V, prec, True, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, cnt = ctx.profile_read(4 if prec == api.GP_FP32 else 0)
    ctx.profile_enable(False)
    print(json.dumps({"kernel_only": args.precision, "n": n, "launches": cnt,
                      "avg_kernel_ms": round(ms / max(cnt, 1), 3),
                      "avg_call_ms": round(1e3 * wall / max(args.kernel_only, 1), 3),
                      "kernel_entries_per_s": float(n) * n / (ms / max(cnt, 1) / 1e3)}),
          flush=True)


def probe_scaling(args):
    """Forward-product time against the number of columns c = s + 1 (the kernel values
    are computed once per entry and shared by all columns of a 128-column pass)."""
    import torch
    from paper_2405_18457_amd import api
    ctx = api.Context(0)
    inp, _, dev = make_inputs(args.n)
    n = inp["n"]
    prec = {"bf16x3": api.GP_BF16X3, "fp32": api.GP_FP32, "bf16": api.GP_BF16}[args.precision]
    base = None
    for c in (1, 9, 17, 33, 65, 129, 257):
        V = dev(np.random.default_rng(c).standard_normal((n, c)).astype(np.float32))
        out = torch.empty_like(V)
        api.gp_kmatvec(ctx, inp["X"], inp["X"], inp["theta_true"], V, prec, True, out)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        for _ in range(2):
            api.gp_kmatvec(ctx, inp["X"], inp["X"], inp["theta_true"], V, prec, True, out)
        ms, cnt = ctx.profile_read(4 if prec == api.GP_FP32 else 0)
        ctx.profile_enable(False)
        per = ms / cnt * (cnt // 2)  # kernel time of one product (all of its column passes)
        base = per if c == 1 else base
        print(json.dumps({"probe_scaling": args.precision, "n": n, "columns": c,
                          "product_ms": round(per, 3), "relative_to_1_column": round(per / base, 3)}),
              flush=True)


def init_heuristic(args):
    """The initial-hyperparameter heuristic of the large-data experiments (App. B) on the
    precision workload: m nearest rows around each centroid row, Adam on the exact
    likelihood (lr 0.1 from theta = 1), mean theta.  One JSON line; the unit of work is
    one exact-likelihood gradient evaluation at m rows."""
    import torch
    import workloads as wl
    from paper_2405_18457_amd import api
    torch.cuda.init()
    ctx = api.Context(0)
    inp, tr, dev = make_inputs(args.n)
    y = build_targets(ctx, inp, tr, dev)
    w, n, d, m = inp["w"], inp["n"], inp["w"].d, args.init_m
    centres = wl.draw_centroids(w, count=args.init_centres, n=n)
    # warm-up: one selection and one evaluation (workspace allocation)
    idx = api.gp_nearest(ctx, inp["X"], int(centres[0]), m)
    api.gp_exact_mll(ctx, inp["X"], y, np.ones(d + 2), idx=idx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    theta, each = api.gp_init_heuristic(ctx, inp["X"], y, centres, m, steps=args.init_steps,
                                        lr=0.1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = len(centres) * args.init_steps
    # the dominant kernels, timed live with HIP events on single evaluations (the
    # heuristic itself runs its centroid subsets concurrently on separate streams)
    ctx.profile_enable(True)
    for _ in range(args.init_single):
        api.gp_exact_mll(ctx, inp["X"], y, np.ones(d + 2), idx=idx)
    torch.cuda.synchronize()
    prof = {k: ctx.profile_read(k) for k in (6, 7, 8)}
    ctx.profile_enable(False)
    fac_ms, fac_n = prof[7]
    # algorithmic FP64 work of one factorisation: Cholesky m^3/3, triangular inverse m^3/3,
    # H^-1 = W^T W (symmetric) m^3/3
    flops = float(m) ** 3
    avg_s = fac_ms / max(fac_n, 1) / 1e3
    achieved = flops / avg_s / 1e12 if fac_n else 0.0
    rec = {
        "metric": "exact-likelihood gradient evaluations/s in the initial-hyperparameter "
                  f"heuristic (m = {m:,} nearest rows)",
        "value": round(evals / wall, 4), "unit": "evaluations/s", "n_gpus": 1, "steps": evals,
        "warmup": 1, "ms_per_step": round(1e3 * wall / max(evals, 1), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"initial-hyperparameter heuristic on the precision workload: "
                               f"n={n}, d={d}, m={m}, {len(centres)} centroid rows, "
                               f"{args.init_steps} Adam steps (lr 0.1, softplus) from theta = 1",
                   "n": n, "d": d, "m": m, "centres": len(centres), "adam_steps": args.init_steps},
        "heuristic_s": round(wall, 3),
        "heuristic_tflops": round(flops * evals / wall / 1e12, 3),  # m^3 per evaluation, wall clock
        "theta": [round(float(v), 6) for v in theta],
        "single_evaluation_ms": {"factor": round(fac_ms / max(fac_n, 1), 3),
                                 "finish": round(prof[8][0] / max(prof[8][1], 1), 3),
                                 "evaluations": fac_n},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_MFMA_PEAK_TFLOPS, 4), "traffic": None,
                     "kernel": "kex_gemm<FP64 MFMA> + kex_leaf (exact-likelihood factorisation)",
                     "avg_launch_ms": round(avg_s * 1e3, 3), "launches": fac_n,
                     "flops_per_launch": flops},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline_exact(inp["Xh"], y.cpu().numpy(), int(centres[0]), m)
    print(json.dumps(rec), flush=True)


def early_stop(args):
    """Early stopping at scale (Sec. 5 "The Effects of Early Stopping"; App. B: a budget
    of 10 solver epochs per outer step on the large data sets): the pathwise estimator
    with CG stopped after `--es-epochs` epochs, once warm-started from the previous
    step's solution and once from zero, each for `--es-steps` Adam steps (lr 0.03) from
    the data-generating theta.  Reports every budgeted solution's FP32 true relative
    residual (mean and probe criteria), whose average over the steps is the paper's
    comparison (Tables 8-11), and the step times."""
    import torch
    import workloads as wl
    from paper_2405_18457_amd import api
    torch.cuda.init()
    ctx = api.Context(0)
    w = wl.WORKLOADS["E"]
    n = w.n if args.n is None else args.n
    X = wl.draw_inputs(w, n=n)
    tr = wl.truth_draws(w, n=n)
    md = wl.model_pathwise_draws(w, n=n)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    inp = {"w": w, "n": n, "X": dev(X), "t": dev(md["t"]), "W": dev(md["W"]),
           "w_eps": dev(md["w_eps"]),
           "theta_true": np.concatenate([tr["ell"], [1.0, w.sigma]])}
    y = build_targets(ctx, inp, tr, dev)
    torch.cuda.synchronize()
    legs = {}
    for leg in ("warm", "cold"):
        solver = {"cg": api.GP_CG, "ap": api.GP_AP, "sgd": api.GP_SGD}[args.es_solver]
        cfg = api.solver_cfg(solver=solver, tol=1e-2, max_epochs=args.es_epochs,
                             precision=api.GP_BF16X3,
                             precond_rank=args.es_rank if solver == api.GP_CG else 0,
                             ap_block=1000, sgd_batch=500, sgd_lr=50.0, sgd_momentum=0.9,
                             sgd_seed=8)
        trn = api.Trainer(ctx, inp["X"], y, inp["theta_true"], api.GP_PATHWISE, cfg, lr=0.03,
                          s=w.s, transform=api.GP_SOFTPLUS, warm=leg == "warm", rff_t=inp["t"],
                          rff_W=inp["W"], w_eps=inp["w_eps"])
        log = []
        for k in range(args.es_steps):
            t0 = time.perf_counter()
            th, _, st = trn.step()
            torch.cuda.synchronize()
            log.append({"s": round(time.perf_counter() - t0, 3), **_brief(st, th)})
            print(f"[bench] early-stop {leg} step {k}: {log[-1]}", file=sys.stderr, flush=True)
        legs[leg] = {"per_step": log,
                     "avg_relres_y": float(np.mean([r["relres_y"] for r in log])),
                     "avg_relres_z": float(np.mean([r["relres_z"] for r in log])),
                     "s_per_step": float(np.mean([r["s"] for r in log]))}
    rec = {
        "metric": "true relative residual of budgeted solves (10 epochs per step), "
                  "warm-started vs cold, early-stopping workload",
        "value": round(legs["cold"]["avg_relres_z"] / max(legs["warm"]["avg_relres_z"], 1e-30), 4),
        "unit": "cold / warm average probe residual", "n_gpus": 1, "steps": args.es_steps,
        "higher_is_better": True, "dtype": "bf16x3", "data": "synthetic",
        "config": {"workload": f"early-stopping workload: n={n}, d={w.d}, x~N(0,I), "
                               f"ell~U[0.3,3], sigma={w.sigma}, s={w.s}, pathwise, "
                               f"{args.es_solver.upper()} with a budget of {args.es_epochs:g} "
                               f"epochs" + (f", pivoted-Cholesky rank {args.es_rank}"
                                            if args.es_solver == "cg" else "") +
                               ", Adam lr 0.03 from the data-generating theta",
                   "n": n, "d": w.d, "s": w.s},
        "legs": legs,
    }
    print(json.dumps(rec), flush=True)


def cpu_baseline_exact(Xh, yh, centre, m, m_sample=5000):
    """The oracle's exact-likelihood gradient on a smaller nearest subset, scaled by m^3."""
    from oracle import init_heuristic as ih
    from oracle import mll
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas_threads = os.cpu_count() or 1
    idx = ih.nearest(Xh, centre, m_sample)
    Xs, ys = Xh[idx].astype(np.float64), yh[idx].astype(np.float64)
    theta = np.ones(Xh.shape[1] + 2)
    t0 = time.perf_counter()
    mll.mll_grad_exact(Xs, ys, theta)
    dt = time.perf_counter() - t0
    t_eval = dt * (m / m_sample) ** 3
    return {"value": float(f"{1.0 / t_eval:.4g}"), "unit": "evaluations/s",
            "cores": int(blas_threads), "kind": "oracle",
            "sample": f"FP64 exact-likelihood gradient (dense Cholesky) on {m_sample} nearest rows "
                      f"took {dt:.2f} s; scaled by (m / {m_sample})^3 to {t_eval:.1f} s at m = {m}"}


def make_inputs(n=None):
    import torch
    import workloads as wl
    from paper_2405_18457_amd import api
    w = wl.WORKLOADS["D"]
    n = w.n if n is None else n
    X = wl.draw_inputs(w, n=n)
    tr = wl.truth_draws(w, n=n)
    md = wl.model_pathwise_draws(w, n=n)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    inp = {"w": w, "n": n, "X": dev(X), "t": dev(md["t"]), "W": dev(md["W"]),
           "w_eps": dev(md["w_eps"]), "Xh": X, "ell": tr["ell"]}
    theta_true = np.concatenate([tr["ell"], [1.0, w.sigma]])
    inp["theta_true"] = theta_true
    return inp, tr, dev


def build_targets(ctx, inp, tr, dev):
    """y = f(x) + sigma * noise, f the data-generating random-feature draw (GPU)."""
    from paper_2405_18457_amd import api
    w = inp["w"]
    F = api.gp_prior_sample(ctx, inp["X"], inp["theta_true"], dev(tr["t"]), dev(tr["w"][:, None]))
    y = (F[:, 0] + w.sigma * dev(tr["noise"])).contiguous()
    return y


def run_form(ctx, inp, y, form, steps, warmup, precond_rank, precond_reuse=0):
    import torch
    from paper_2405_18457_amd import api
    cfg, mode = _form_cfg(form, precond_rank, precond_reuse)
    tr = api.Trainer(ctx, inp["X"], y, inp["theta_true"], api.GP_PATHWISE, cfg, lr=0.03,
                     s=inp["w"].s, transform=api.GP_SOFTPLUS, warm=True, rff_t=inp["t"],
                     rff_W=inp["W"], w_eps=inp["w_eps"], adjoint_mode=mode)
    log = []
    for k in range(warmup):
        t0 = time.perf_counter()
        th, _, st = tr.step()
        torch.cuda.synchronize()
        log.append({"phase": "warmup", "s": time.perf_counter() - t0, **_brief(st, th)})
        print(f"[bench] {form} warmup {k}: {log[-1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # the state the timed steps start from (warm-start solution, Adam moments), kept for
    # the comparison of the two forms on the same step
    tr.snapshot = (tr.U.clone(), copy.deepcopy(tr.state))
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        th, _, st = tr.step()
        log.append({"phase": "timed", "s": time.perf_counter() - ts, **_brief(st, th)})
        print(f"[bench] {form} step {k}: {log[-1]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {k: ctx.profile_read(k) for k in range(6)}
    ctx.profile_enable(False)
    return elapsed, log, prof, tr


def _form_cfg(form, precond_rank, precond_reuse):
    from paper_2405_18457_amd import api
    prec = api.GP_BF16X3 if form == "bf16x3+adjoint" else api.GP_FP32
    mode = api.GP_ADJ_FUSED if form == "bf16x3+adjoint" else api.GP_ADJ_PER_PARAM
    return api.solver_cfg(solver=api.GP_CG, tol=1e-2, precision=prec, precond_rank=precond_rank,
                          precond_reuse=precond_reuse), mode


def compare_forms(ctx, inp, y, trainer, steps, precond_rank):
    """The metric's comparison on identical marginal-likelihood steps: from the state
    the timed region started from (warm-start solution and Adam moments after the
    warm-up steps; the cached pivoted-Cholesky factor, which both forms reuse without
    rebuilding), `steps` steps of the bf16x3+adjoint form and then the same steps of
    the fp32-plain form (FP32 products, d+1 separate derivative passes for the
    gradient)."""
    import torch
    from paper_2405_18457_amd import api
    U0, state0 = trainer.snapshot
    res = {}
    for form in ("bf16x3+adjoint", "fp32-plain"):
        cfg, mode = _form_cfg(form, precond_rank, 1 << 30)
        tr = api.Trainer(ctx, inp["X"], y, trainer.theta, api.GP_PATHWISE, cfg, lr=0.03,
                         s=inp["w"].s, transform=api.GP_SOFTPLUS, warm=True, rff_t=inp["t"],
                         rff_W=inp["W"], w_eps=inp["w_eps"], adjoint_mode=mode)
        tr.U.copy_(U0)
        tr.state = copy.deepcopy(state0)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        log = []
        t0 = time.perf_counter()
        for k in range(steps):
            ts = time.perf_counter()
            th, _, st = tr.step()
            log.append({"phase": "compare", "s": time.perf_counter() - ts, **_brief(st, th)})
            print(f"[bench] compare {form} step {k}: {log[-1]}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        prof = {k: ctx.profile_read(k) for k in range(6)}
        ctx.profile_enable(False)
        res[form] = {"value": round(steps / elapsed, 6), "unit": "steps/s",
                     "ms_per_step": round(1e3 * elapsed / steps, 1), "per_step": log,
                     "kernel_ms": {"fwd_bf16": prof[0], "adjoint": prof[1], "fwd_fp32": prof[4],
                                   "precond": prof[5]}}
    return res


def _brief(st, theta=None):
    extra = {} if theta is None else {"theta": [round(float(v), 5) for v in theta]}
    return {**extra, "iters": st["iterations"], "matvecs": st["matvecs"], "refine": st["refinements"],
            "precond_rank": st["precond_rank"],
            "relres_y": round(st["true_relres_y"], 5) if st["true_relres_y"] == st["true_relres_y"]
            else round(st["relres_y"], 5),
            "relres_z": round(st["true_relres_z"], 5) if st["true_relres_z"] == st["true_relres_z"]
            else round(st["relres_z"], 5),
            "converged": st["converged"],
            **({"fp32_iters": st["fp32_iterations"]} if st.get("fp32_iterations") else {})}


def traffic_per_launch():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_18457_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sources_sha256"]:
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]


def roofline(n, d, c, prof):
    """Dominant kernel: the bf16x3 forward product (profile class 0).

    `achieved` is the algorithmic K*V work of one product, 2 c n^2 flops with
    c = s + 1 columns (every kernel entry multiplies every column once), over the
    average launch time, against the bf16 matrix-core peak.  The kernel issues
    three bf16 passes per tile (hi*hi + hi*lo + lo*hi) over 80 padded columns and
    the squared distances on the FP32 matrix cores; `mfma_issued` reports that
    busy time, and `valu` the vector-ALU work the kernel issues per entry."""
    ms, cnt = prof[0]
    if cnt == 0:
        return None
    avg_s = ms / cnt / 1e3
    entries = float(n) * n
    kv_flops = 2.0 * c * entries
    achieved = kv_flops / avg_s / 1e12
    c_pad = 16 * ((c + 15) // 16)
    t_bf16 = 3 * 2.0 * c_pad * entries / (BF16_PEAK_TFLOPS * 1e12)
    t_xt = 2.0 * XT_KDIM * entries / (FP32_MFMA_PEAK_TFLOPS * 1e12)
    slots = entries * (VALU_SIMPLE_PER_ENTRY + 2.0 * VALU_TRANS_PER_ENTRY)
    return {
        "bound": "mfma",
        "achieved": round(achieved, 2),
        "peak": BF16_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
        "traffic": traffic_per_launch(),
        "kernel": "kfwd_bf16_xt<BF16X3, CT=5, RS=4>",
        "flops_per_launch": kv_flops,
        "avg_launch_ms": round(avg_s * 1e3, 3),
        "launches": cnt,
        "kernel_entries_per_s": round(entries / avg_s, 1),
        "mfma_issued": {"bf16_passes": 3, "columns_padded": c_pad,
                        "busy_ms_at_peak": round(1e3 * (t_bf16 + t_xt), 2),
                        "busy_frac": round((t_bf16 + t_xt) / avg_s, 4)},
        "valu": {"slots_per_entry": VALU_SIMPLE_PER_ENTRY + 2.0 * VALU_TRANS_PER_ENTRY,
                 "achieved_slots_per_s": round(slots / avg_s, 1),
                 "peak_slots_per_s": VALU_SLOTS_PER_S,
                 "frac": round(slots / avg_s / VALU_SLOTS_PER_S, 4)},
    }


def cpu_baseline(inp, iters_per_step, rows, rows_1core):
    """The oracle's matrix-free FP64 product on a bounded row sample, scaled to a step:
    once with every BLAS thread the host gives it, once on one core."""
    import oracle.kernel as ok
    from threadpoolctl import threadpool_info, threadpool_limits
    blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    X = inp["Xh"]
    n = X.shape[0]
    theta = inp["theta_true"]
    V = np.random.default_rng(0).standard_normal((n, inp["w"].s + 1))

    def timed(r):
        t0 = time.perf_counter()
        ok.k_matvec(X[:r], X, theta, V)
        return time.perf_counter() - t0

    def per_step(dt, r):
        t_matvec = dt * n / r
        # per step: iterations + initial/true-residual products + one adjoint (~ one product)
        return t_matvec, (iters_per_step + 3) * t_matvec

    dt = timed(rows)
    t_mv, t_step = per_step(dt, rows)
    with threadpool_limits(limits=1):
        dt1 = timed(rows_1core)
    t_mv1, t_step1 = per_step(dt1, rows_1core)
    return {"value": float(f"{1.0 / t_step:.4g}"), "unit": "steps/s", "cores": int(blas_threads),
            "kind": "oracle",
            "sample": f"FP64 matrix-free H*V on {rows} of {n} rows x 65 columns took {dt:.2f} s; "
                      f"full product extrapolated to {t_mv:.1f} s; step = (CG iterations "
                      f"{iters_per_step:.1f} + 3) products",
            "one_core": {"value": float(f"{1.0 / t_step1:.4g}"), "unit": "steps/s", "cores": 1,
                         "sample": f"{rows_1core} rows on one BLAS thread took {dt1:.2f} s; "
                                   f"full product extrapolated to {t_mv1:.1f} s"}}


T_START = time.perf_counter()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "row-sharded design is documented with the library and not run here.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.kernel_only:
        kernel_only(args)
        return
    if args.probe_scaling:
        probe_scaling(args)
        return
    if args.init_heuristic:
        init_heuristic(args)
        return
    if args.early_stop:
        early_stop(args)
        return
    import torch
    from paper_2405_18457_amd import api
    torch.cuda.init()
    ctx = api.Context(0)
    inp, tr, dev = make_inputs(args.n)
    y = build_targets(ctx, inp, tr, dev)
    torch.cuda.synchronize()
    n, d, s = inp["n"], inp["w"].d, inp["w"].s

    theta0_info = {"kind": "data-generating theta"}
    if args.theta0 == "heuristic":
        import workloads as wl
        centres = wl.draw_centroids(inp["w"], count=args.init_centres, n=n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th0, _ = api.gp_init_heuristic(ctx, inp["X"], y, centres, args.init_m,
                                       steps=args.init_steps, lr=0.1)
        torch.cuda.synchronize()
        theta0_info = {"kind": "initial-hyperparameter heuristic (App. B)", "s": round(
            time.perf_counter() - t0, 3), "theta0": [round(float(v), 6) for v in th0],
            "centres": len(centres), "m": args.init_m, "adam_steps": args.init_steps}
        print(f"[bench] heuristic theta0 {theta0_info}", file=sys.stderr, flush=True)
        inp["theta_true"] = th0
    elapsed, log, prof, trainer = run_form(ctx, inp, y, args.form, args.steps, args.warmup,
                                           args.precond_rank, args.precond_reuse)
    value = args.steps / elapsed
    timed = [r for r in log if r["phase"] == "timed"]
    iters = float(np.mean([r["iters"] for r in timed])) if timed else 0.0
    rec = {
        "metric": METRIC, "value": round(value, 6), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3" if args.form == "bf16x3+adjoint" else "fp32",
        "data": "synthetic",
        "config": {"workload": f"precision workload: n={n}, d={d}, x~U[-1,1]^3, ell~U[0.05,0.2], "
                               f"sigma=0.05, s={s}, pathwise + warm start, CG to rel-res 1e-2, "
                               "Adam lr 0.03, theta0 = " + (
                                   "the initial-hyperparameter heuristic" if args.theta0 ==
                                   "heuristic" else "data-generating theta"),
                   "form": args.form, "n": n, "d": d, "s": s, "solver": "cg", "tol": 1e-2,
                   "precond": (f"pivoted Cholesky rank {args.precond_rank}, factor reused by up to "
                               f"{args.precond_reuse} later steps (built in the first warm-up "
                               "step)") if args.precond_rank
                   else "none"},
        "theta0": theta0_info,
        "per_step": timed,
        "warmup_log": [r for r in log if r["phase"] == "warmup"],
    }
    if args.form == "bf16x3+adjoint":
        rec["roofline"] = roofline(n, d, s + 1, prof)
    # the FP32 fused product (the true-residual products of every step) on its own peak
    f32_ms, f32_n = prof[4]
    if f32_n:
        t = f32_ms / f32_n / 1e3
        tf = 2.0 * (s + 1) * float(n) * n / t / 1e12
        rec["fp32_product_mfma"] = {"kernel": "kfwd_f32_xt<CT=5, RS=4>",
                                    "avg_launch_ms": round(t * 1e3, 3), "launches": f32_n,
                                    "achieved": round(tf, 2), "peak": FP32_MFMA_PEAK_TFLOPS,
                                    "unit": "TFLOP/s", "frac": round(tf / FP32_MFMA_PEAK_TFLOPS, 4)}
    rec["kernel_ms"] = {"fwd_bf16": prof[0], "adjoint": prof[1], "rff": prof[2], "cg_vec": prof[3],
                        "fwd_fp32": prof[4], "precond": prof[5]}
    if args.compare_steps > 0 and time.perf_counter() - T_START > args.compare_after_s:
        rec["compare"] = {"skipped": f"the run had taken {time.perf_counter() - T_START:.0f} s"}
    elif args.compare_steps > 0:
        cmp = compare_forms(ctx, inp, y, trainer, args.compare_steps, args.precond_rank)
        rec["compare"] = {
            "note": "the same marginal-likelihood step(s) in both forms, from the state the "
                    "timed region started from, both reusing the cached preconditioner factor",
            **cmp,
            "bf16x3_adjoint_over_fp32_plain": round(cmp["bf16x3+adjoint"]["value"]
                                                    / cmp["fp32-plain"]["value"], 3)}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(inp, iters, args.cpu_rows, args.cpu_rows_1core)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
