"""The 16,384-point workload (d = 24, s = 64): 50 Adam steps of marginal-likelihood
optimisation (pathwise estimator, warm start, lr 0.1, softplus, theta0 = 1) with each
of the three solvers of App. B stopped at tau = 1e-2 -- CG, alternating projections
(b = 1,000) and SGD (b = 500, momentum 0.9, learning rate from the paper's grid) --
against the oracle's trajectory with exact Cholesky solves and the same random
features (tests/golden/config_b_exact_trajectory.json, written by
tests/golden/make_config_b_trajectory.py).  Bound: every step's nu within 0.05 of
the oracle's (half an Adam step at lr 0.1)."""
import json
import os

import numpy as np
import pytest

import workloads as wl
from gpu_common import announce, dev, require_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "config_b_exact_trajectory.json")
SGD_GRID = [5, 10, 20, 30, 50, 60, 70, 80, 90, 100]


@pytest.fixture(scope="module")
def case():
    require_gpu()
    if not os.path.exists(GOLDEN):
        pytest.skip("golden trajectory not generated")
    from paper_2405_18457_amd import api
    from oracle import rff
    w = wl.WORKLOADS["B"]
    X = wl.draw_inputs(w)
    tr = wl.truth_draws(w)
    y = rff.truth_targets_rff(X, tr["ell"], 1.0, w.sigma, tr["t"], tr["w"],
                              tr["noise"]).astype(np.float32)
    dr = wl.model_pathwise_draws(w)
    gold = json.load(open(GOLDEN))
    ctx = api.Context(0)
    yield dict(w=w, X=dev(X), y=dev(y), dr={k: dev(v) for k, v in dr.items()}, gold=gold, ctx=ctx)
    ctx.close()


def _trajectory(case, cfg, steps):
    from paper_2405_18457_amd import api
    w = case["w"]
    t = api.Trainer(case["ctx"], case["X"], case["y"], np.ones(w.d + 2), api.GP_PATHWISE, cfg,
                    lr=0.1, s=w.s, transform=api.GP_SOFTPLUS, warm=True, rff_t=case["dr"]["t"],
                    rff_W=case["dr"]["W"], w_eps=case["dr"]["w_eps"])
    nus, stats = [t.state["nu"].copy()], []
    for _ in range(steps):
        _, _, st = t.step()
        nus.append(t.state["nu"].copy())
        stats.append(st)
    return np.array(nus), stats


def _sgd_learning_rate(case):
    """The paper's rule (App. B, SGD paragraph): the largest rate of the grid whose
    solve on the first outer step does not diverge (here: stays finite and ends with a
    smaller residual estimate than it started with, within 50 epochs)."""
    from paper_2405_18457_amd import api
    import torch
    w = case["w"]
    ok = None
    for lr in SGD_GRID:
        U = torch.zeros((w.n, w.s + 1), device="cuda")
        cfg = api.solver_cfg(solver=api.GP_SGD, tol=1e-2, max_epochs=50, sgd_batch=500,
                             sgd_lr=float(lr), sgd_momentum=0.9, sgd_seed=8)
        try:
            _, st = api.gp_mll_grad(case["ctx"], case["X"], case["y"], np.ones(w.d + 2),
                                    api.GP_PATHWISE, U, cfg, rff_t=case["dr"]["t"],
                                    rff_W=case["dr"]["W"], w_eps=case["dr"]["w_eps"])
        except api.GPError:
            break
        if not (np.isfinite(st["relres_z"]) and st["relres_z"] < 1.0):
            break
        ok = lr
    return ok


@pytest.mark.parametrize("solver", ["cg", "ap", "sgd"])
def test_trajectory_matches_exact_solves(case, solver):
    from paper_2405_18457_amd import api
    gold = case["gold"]
    steps = gold["steps"]
    ref = np.array(gold["nu"])
    if solver == "cg":
        cfg = api.solver_cfg(tol=1e-2, precision=api.GP_FP32)
    elif solver == "ap":
        cfg = api.solver_cfg(solver=api.GP_AP, tol=1e-2, ap_block=1000, precision=api.GP_FP32)
    else:
        lr = _sgd_learning_rate(case)
        print(f"[gpu-case] SGD learning rate from the grid: {lr}", flush=True)
        assert lr is not None
        cfg = api.solver_cfg(solver=api.GP_SGD, tol=1e-2, sgd_batch=500, sgd_lr=float(lr),
                             sgd_momentum=0.9, sgd_seed=8, max_epochs=200, precision=api.GP_FP32)
    announce("config B trajectory", solver)
    import time
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nus, stats = _trajectory(case, cfg, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_per_step = np.max(np.abs(nus - ref), axis=1)
    its = [s["iterations"] for s in stats]
    conv = sum(bool(s["converged"]) for s in stats)
    print(f"[gpu-case] {solver}: max |nu - nu_exact| per step {np.round(dev_per_step, 4).tolist()}; "
          f"iterations {its}; converged {conv}/{steps}; {wall:.1f} s for {steps} steps", flush=True)
    assert float(dev_per_step.max()) <= 0.05
