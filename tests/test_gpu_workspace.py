"""Workspace planning (gp_workspace_size / gp_workspace_reserve / gp_workspace_held):
after a reservation, calls of the planned size allocate nothing more, and the
reservation is what the size query said."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import announce, dev, problem, require_gpu

pytestmark = pytest.mark.gpu


def _cfgs(api):
    return {
        "cg-bf16x3": api.solver_cfg(tol=1e-2, precision=api.GP_BF16X3),
        "cg-pc": api.solver_cfg(tol=1e-2, precision=api.GP_BF16X3, precond_rank=40),
        "ap": api.solver_cfg(solver=api.GP_AP, tol=1e-2, ap_block=300, max_epochs=1),
        "sgd": api.solver_cfg(solver=api.GP_SGD, tol=1e-2, sgd_batch=200, sgd_lr=5.0,
                              max_epochs=1, precision=api.GP_FP32),
    }


@pytest.mark.parametrize("name", ["cg-bf16x3", "cg-pc", "ap", "sgd"])
def test_reserved_solve_allocates_nothing(name):
    require_gpu()
    from paper_2405_18457_amd import api
    import torch
    n, d, c = 1500, 3, 17
    X, B, theta = problem(n, d, c, seed=31, dist="uniform", sigma=0.1, ell_scale=(0.2, 0.5))
    cfg = _cfgs(api)[name]
    ctx = api.Context(0)
    try:
        announce("workspace solve", name)
        want = api.gp_workspace_size(api.GP_WS_SOLVE, n, d, c, cfg)
        api.gp_workspace_reserve(ctx, api.GP_WS_SOLVE, n, d, c, cfg)
        held = api.gp_workspace_held(ctx)
        assert held == want, (held, want)
        api.gp_solve(ctx, dev(X), theta, dev(B), torch.zeros((n, c), device="cuda"), cfg)
        assert api.gp_workspace_held(ctx) == held
        # a smaller problem fits the same reservation
        api.gp_solve(ctx, dev(X[:700]), theta, dev(B[:700, :9]),
                     torch.zeros((700, 9), device="cuda"), cfg)
        assert api.gp_workspace_held(ctx) == held
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_reserved_product_and_gradient_allocate_nothing(prec):
    require_gpu()
    from paper_2405_18457_amd import api
    import torch
    w = wl.WORKLOADS["A"]
    X, V, theta = problem(w.n, w.d, w.s + 1, seed=32)
    y = np.random.default_rng(33).standard_normal(w.n).astype(np.float32)
    dr = wl.model_pathwise_draws(w)
    Z = np.random.default_rng(34).standard_normal((w.n, w.s)).astype(np.float32)
    cfg = api.solver_cfg(tol=1e-2, precision=prec, precond_rank=50)
    M = dr["t"].shape[0]
    ctx = api.Context(0)
    try:
        announce("workspace product+gradient", prec)
        want = api.gp_workspace_size(api.GP_WS_MLL_GRAD, w.n, w.d, w.s + 1, cfg, M)
        assert want >= api.gp_workspace_size(api.GP_WS_KMATVEC, w.n, w.d, w.s + 1, cfg)
        api.gp_workspace_reserve(ctx, api.GP_WS_MLL_GRAD, w.n, w.d, w.s + 1, cfg, M)
        held = api.gp_workspace_held(ctx)
        assert held == want, (held, want)
        Xd = dev(X)  # one buffer: the planned product is H V with X1 == X2
        api.gp_kmatvec(ctx, Xd, Xd, theta, dev(V), prec, add_noise=True)
        assert api.gp_workspace_held(ctx) == held
        for est, mode in ((api.GP_PATHWISE, api.GP_ADJ_FUSED), (api.GP_STANDARD, api.GP_ADJ_PER_PARAM)):
            U = torch.zeros((w.n, w.s + 1), device="cuda")
            api.gp_mll_grad(ctx, Xd, dev(y), theta, est, U, cfg, Z=dev(Z), rff_t=dev(dr["t"]),
                            rff_W=dev(dr["W"]), w_eps=dev(dr["w_eps"]), adjoint_mode=mode)
            assert api.gp_workspace_held(ctx) == held, (est, mode)
    finally:
        ctx.close()
