"""Differentiable product and the optimisation loop on the GPU against the FP64
oracle: the autograd function around gp_kmatvec (hand-written backward: H grad for
V, the fused adjoint for theta) against the oracle's derivatives and central
finite differences; and Adam trajectories of the pathwise, warm-started iterative
method against the oracle run with exact solves (Sec. 2 "Hierarchical View",
App. B "Iterative Optimiser")."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import announce, dev, host, problem, require_gpu
from oracle import kernel, rff, train

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    require_gpu()
    from paper_2405_18457_amd import api
    ctx = api.Context(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("prec,tol", [(0, 2e-5), (1, 5e-5)], ids=["fp32", "bf16x3"])
def test_kmatvec_autograd_matches_oracle_and_finite_differences(gp, prec, tol):
    from paper_2405_18457_amd import api
    import torch
    X, V, theta = problem(600, 3, 5, seed=21, dist="uniform", ell_scale=(0.2, 0.5))
    Wt = np.random.default_rng(22).standard_normal(V.shape).astype(np.float32)
    announce("autograd", prec)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    Vd = dev(V).requires_grad_(True)
    out = api.KMatvec.apply(dev(X), th, Vd, gp, prec)
    loss = (out * dev(Wt)).sum()
    loss.backward()
    # forward and dL/dV = H W (H symmetric)
    ref_out = kernel.h_matvec(X, theta, V)
    assert np.linalg.norm(host(out) - ref_out) / np.linalg.norm(ref_out) <= tol
    ref_dV = kernel.h_matvec(X, theta, Wt)
    assert np.linalg.norm(host(Vd.grad) - ref_dV) / np.linalg.norm(ref_dV) <= tol
    # dL/dtheta_k = sum_c W_c^T (dH/dtheta_k) V_c
    ref_dth = kernel.adjoint(X, theta, Wt, V, np.ones(V.shape[1]))
    g = th.grad.numpy()
    assert np.linalg.norm(g - ref_dth) / np.linalg.norm(ref_dth) <= 10 * tol
    # central differences of the FP64 loss, relative step 1e-5
    fd = np.zeros_like(theta)
    for k in range(theta.size):
        h = 1e-5 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (np.sum(Wt * kernel.h_matvec(X, tp, V)) - np.sum(Wt * kernel.h_matvec(X, tm, V))) / (2 * h)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) <= 10 * tol + 1e-6


def test_adam_trajectory_matches_oracle_with_exact_solves(gp):
    """Ten Adam steps (lr 0.1, log transform, theta0 = 1) of the pathwise estimator
    with warm-started CG at tau = 1e-2 on the GPU, against the oracle's run with
    exact Cholesky solves and the same random features: the log-hyperparameter
    trajectories stay within half an Adam step (0.05)."""
    from paper_2405_18457_amd import api
    import torch
    w = wl.WORKLOADS["A"]
    X = wl.draw_inputs(w)
    tr = wl.truth_draws(w)
    y = rff.truth_targets_exact(X, tr["ell"], 1.0, w.sigma, tr["w"], tr["noise"]).astype(np.float32)
    dr = wl.model_pathwise_draws(w)
    theta0 = np.ones(w.d + 2)
    announce("trajectory")
    cfg = api.solver_cfg(tol=1e-2, precision=api.GP_BF16X3)
    tg = api.Trainer(gp, dev(X), dev(y), theta0, api.GP_PATHWISE, cfg, lr=0.1, s=w.s,
                     transform=api.GP_LOG, warm=True, rff_t=dev(dr["t"]), rff_W=dev(dr["W"]),
                     w_eps=dev(dr["w_eps"]))
    to = train.Trainer(X, y, theta0, "pathwise", dr, lr=0.1, transform="log", solver="exact")
    worst = 0.0
    for _ in range(10):
        tg.step()
        to.step()
        worst = max(worst, float(np.max(np.abs(tg.state["nu"] - to.nu))))
    print("max |nu_gpu - nu_oracle| over 10 steps:", worst)
    assert worst <= 0.05
    for h in tg.history:
        assert h["stats"]["converged"]
