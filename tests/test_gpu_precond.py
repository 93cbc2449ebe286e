"""Pivoted-Cholesky preconditioner of CG (App. B: Algorithm 1 with P(.), rank 100
in the paper) on the GPU against the FP64 oracle: the greedy factor itself
(pivot sequence and factor columns), and preconditioned CG (step-for-step under
a budget, to tolerance, with bf16x3 products and inside the gradient step)."""
import numpy as np
import pytest

import workloads as wl
from gpu_common import announce, dev, host, problem, require_gpu
from oracle import kernel, mll, precond, rff, solvers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gp():
    require_gpu()
    from paper_2405_18457_amd import api
    ctx = api.Context(0)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("n,d,k,dist", [(700, 3, 40, "uniform"), (513, 8, 64, "normal"),
                                        (300, 1, 25, "normal"), (20, 3, 50, "uniform")])
def test_pivoted_cholesky_matches_oracle(gp, n, d, k, dist):
    from paper_2405_18457_amd import api
    X, _, theta = problem(n, d, 1, seed=11 * n + d, dist=dist,
                          ell_scale=(0.2, 0.5) if dist == "uniform" else None)
    announce("pivchol", n, d, k)
    L, piv = api.gp_pivoted_cholesky(gp, dev(X), theta, k)
    Lo, po = precond.pivoted_cholesky(X, theta, k)
    assert L.shape[0] == len(po) == min(k, n)
    assert list(host(piv).astype(int)) == po
    np.testing.assert_allclose(host(L).T, Lo, rtol=0, atol=1e-9)


def test_pivoted_cholesky_empty_and_invalid(gp):
    from paper_2405_18457_amd import api
    X, _, theta = problem(50, 3, 1, seed=2)
    L, piv = api.gp_pivoted_cholesky(gp, dev(X), theta, 0)
    assert L.shape[0] == 0 and piv.shape[0] == 0
    with pytest.raises(api.GPError):
        api.gp_pivoted_cholesky(gp, dev(X), theta, 40000)


# The larger case spans many 64-row factor tiles and several row chunks of the
# products, with ragged tails in n, k and the columns.  Storing the factor in
# FP32 (as the library does) moves the oracle's iterates by about 1e-7 relative
# at this size, so the tolerance is set by the products.  The four iterates of
# the larger case are far more sensitive to them: a symmetric random relative
# perturbation eps of every kernel entry moves the oracle's own U by about
# 218 eps of max|U| there (3.6 eps in the smaller case).  bf16x3 drops terms of
# relative size 2^-16 per entry, hence 218 * 2^-16 = 3.3e-3, bounded by 5e-3.
# With 65 columns (64 probes and the mean column, the column count whose
# preconditioner apply runs the 65th column on the vector ALU) a 2^-16 error per
# entry moves the oracle's U by 8.1e-5 (900 rows) and 3.6e-3 (4000 rows) of
# max|U|, against 5.6e-5 and 3.3e-3 with 9 columns (tests/test_tolerances.py),
# inside the same bounds.
ATOL_FRAC = {(900, 0): 2e-4, (900, 1): 2e-4, (4000, 0): 2e-4, (4000, 1): 5e-3}


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("n,k,seed,c", [(900, 60, 31, 9), (900, 60, 31, 65), (4000, 1000, 57, 9),
                                        (4000, 1000, 57, 65)])
def test_pcg_steps_match_oracle_under_a_budget(gp, prec, n, k, seed, c):
    from paper_2405_18457_amd import api
    import torch
    X, B, theta = problem(n, 3, c, seed=seed, dist="uniform", sigma=0.05, ell_scale=(0.2, 0.5))
    op = solvers.DenseOperator(X, theta)
    P = precond.preconditioner(X, theta, k)
    announce("pcg-budget", prec, n, k, c)
    U = torch.zeros((n, c), device="cuda")
    st = api.gp_solve(gp, dev(X), theta, dev(B), U,
                      api.solver_cfg(tol=1e-8, max_epochs=4, precision=prec, precond_rank=k))
    assert st["iterations"] == 4 and not st["converged"] and st["precond_rank"] == k
    Uo, so = solvers.cg(op, B, tol=1e-8, max_epochs=4, precond=P)
    np.testing.assert_allclose(host(U), Uo, rtol=2e-3, atol=ATOL_FRAC[n, prec] * np.abs(Uo).max())
    assert st["relres_y"] == pytest.approx(so["relres_y"], rel=2e-3)
    assert st["relres_z"] == pytest.approx(so["relres_z"], rel=2e-3)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("n,d,c,sigma,k", [(2000, 3, 65, 0.05, 100), (1500, 8, 17, 0.2, 50)])
def test_pcg_reaches_tolerance_in_fewer_iterations(gp, n, d, c, sigma, k, prec):
    from paper_2405_18457_amd import api
    import torch
    X, B, theta = problem(n, d, c, seed=n + 7 * c, dist="uniform" if d == 3 else "normal",
                          sigma=sigma, ell_scale=(0.2, 0.5) if d == 3 else None)
    op = solvers.DenseOperator(X, theta)
    announce("pcg-tol", n, d, c, k, prec)
    U0 = torch.zeros((n, c), device="cuda")
    s0 = api.gp_solve(gp, dev(X), theta, dev(B), U0, api.solver_cfg(tol=1e-2, precision=prec))
    U = torch.zeros((n, c), device="cuda")
    st = api.gp_solve(gp, dev(X), theta, dev(B), U,
                      api.solver_cfg(tol=1e-2, precision=prec, precond_rank=k))
    ry, rz = solvers.true_relres(op, B, host(U))
    assert st["converged"] and ry <= 1.02e-2 and rz <= 1.02e-2, (st, ry, rz)
    Uo, so = solvers.cg(op, B, tol=1e-2, precond=precond.preconditioner(X, theta, k))
    print("iterations plain / preconditioned / oracle:", s0["iterations"], st["iterations"],
          so["iterations"])
    assert 0.7 * so["iterations"] - 2 <= st["iterations"] <= 1.5 * so["iterations"] + 6, (st, so)
    assert st["iterations"] < s0["iterations"]


def test_precond_rank_validation(gp):
    from paper_2405_18457_amd import api
    import torch
    X, B, theta = problem(100, 3, 3, seed=5)
    U = torch.zeros((100, 3), device="cuda")
    with pytest.raises(api.GPError):
        api.gp_solve(gp, dev(X), theta, dev(B), U, api.solver_cfg(precond_rank=40000))
    with pytest.raises(api.GPError):
        api.gp_solve(gp, dev(X), theta, dev(B), U,
                     api.solver_cfg(solver=api.GP_AP, precond_rank=10, ap_block=50))
    # rank above n is capped at n (P = H: one iteration)
    st = api.gp_solve(gp, dev(X), theta, dev(B), U, api.solver_cfg(tol=1e-4, precond_rank=500))
    assert st["precond_rank"] == 100 and st["converged"] and st["iterations"] <= 2


def test_pathwise_gradient_with_preconditioner(gp):
    """Gradient estimate with preconditioned CG stopped at tau = 1e-2 against the
    oracle estimator with exact solves and the same random features (workload A
    shape).  The bound is the one the unpreconditioned solve meets: at tau = 1e-2
    the solve error itself is of order 1e-3 to 1e-2 in the gradient."""
    from paper_2405_18457_amd import api
    import torch
    w = wl.WORKLOADS["A"]
    X = wl.draw_inputs(w)
    tr = wl.truth_draws(w)
    y = rff.truth_targets_exact(X, tr["ell"], 1.0, w.sigma, tr["w"], tr["noise"]).astype(np.float32)
    dr = wl.model_pathwise_draws(w)
    theta = np.concatenate([tr["ell"], [1.0, w.sigma]])
    U = torch.zeros((w.n, w.s + 1), device="cuda")
    cfg = api.solver_cfg(tol=1e-2, precision=api.GP_BF16X3, precond_rank=100)
    announce("grad-tau-precond")
    g, st = api.gp_mll_grad(gp, dev(X), dev(y), theta, api.GP_PATHWISE, U, cfg,
                            rff_t=dev(dr["t"]), rff_W=dev(dr["W"]), w_eps=dev(dr["w_eps"]))
    B = rff.pathwise_rhs(X, y, theta, dr["t"], dr["W"], dr["w_eps"])
    ref = mll.pathwise_estimate(X, y, theta, B[:, 1:])
    err = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    # the same algorithm in FP64: preconditioned CG stopped at the same tau
    op = solvers.DenseOperator(X, theta)
    Uo, so = solvers.cg(op, B, tol=1e-2, precond=precond.preconditioner(X, theta, 100))
    go = mll.pathwise_estimate(X, y, theta, B[:, 1:], solutions=Uo)
    err_o = float(np.linalg.norm(go - ref) / np.linalg.norm(ref))
    print("gradient relative error at tau=1e-2, rank-100 preconditioning: gpu", err, "oracle", err_o,
          st, so["iterations"])
    assert st["converged"] and st["precond_rank"] == 100
    assert st["true_relres_y"] <= 1e-2 and st["true_relres_z"] <= 1e-2
    assert err <= max(2.0 * err_o, 1e-3)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_reused_factor(gp, prec):
    """precond_reuse: at the same theta a reused factor gives the very same solve as a
    fresh one; at a moved theta (a later outer step) the reused factor still defines
    an SPD preconditioner, so the solve meets the tolerance against the FP64 operator."""
    from paper_2405_18457_amd import api
    import torch
    n, c, k = 1500, 17, 80
    X, B, theta = problem(n, 3, c, seed=77, dist="uniform", sigma=0.05, ell_scale=(0.2, 0.5))
    Xd, Bd = dev(X), dev(B)
    fresh = api.solver_cfg(tol=1e-2, precision=prec, precond_rank=k)
    reuse = api.solver_cfg(tol=1e-2, precision=prec, precond_rank=k, precond_reuse=2)
    announce("pcg-reuse same theta", prec)
    U1 = torch.zeros((n, c), device="cuda")
    s1 = api.gp_solve(gp, Xd, theta, Bd, U1, fresh)     # builds and keeps the factor
    U2 = torch.zeros((n, c), device="cuda")
    s2 = api.gp_solve(gp, Xd, theta, Bd, U2, reuse)     # reuses it
    U3 = torch.zeros((n, c), device="cuda")
    s3 = api.gp_solve(gp, Xd, theta, Bd, U3, fresh)     # rebuilds
    assert s1["iterations"] == s2["iterations"] == s3["iterations"]
    np.testing.assert_array_equal(host(U2), host(U1))
    np.testing.assert_array_equal(host(U3), host(U1))
    # the same pointer with other contents is not taken for the same inputs
    X2 = X.copy()
    X2[:, 0] = X2[::-1, 0]
    Xd.copy_(dev(X2))
    U4 = torch.zeros((n, c), device="cuda")
    s4 = api.gp_solve(gp, Xd, theta, Bd, U4, reuse)
    s4f = api.gp_solve(gp, Xd, theta, Bd, torch.zeros((n, c), device="cuda"), fresh)
    assert s4["iterations"] == s4f["iterations"]
    Xd.copy_(dev(X))
    announce("pcg-reuse moved theta", prec)
    api.gp_solve(gp, Xd, theta, Bd, torch.zeros((n, c), device="cuda"), fresh)  # factor at theta
    moved = theta * np.array([1.05, 0.95, 1.04, 1.03, 0.96])
    U5 = torch.zeros((n, c), device="cuda")
    s5 = api.gp_solve(gp, Xd, moved, Bd, U5, reuse)     # reuses the factor of theta
    ry, rz = solvers.true_relres(solvers.DenseOperator(X, moved), B, host(U5))
    assert s5["converged"] and ry <= 1.02e-2 and rz <= 1.02e-2, (s5, ry, rz)
    U6 = torch.zeros((n, c), device="cuda")
    s6 = api.gp_solve(gp, Xd, moved, Bd, U6, fresh)
    print("iterations fresh / reused at moved theta:", s6["iterations"], s5["iterations"])
    assert s5["iterations"] <= 2 * s6["iterations"] + 5
    with pytest.raises(api.GPError):
        api.gp_solve(gp, Xd, theta, Bd, U6, api.solver_cfg(precond_rank=k, precond_reuse=-1))


def test_full_size_precision_workload_solve_residual_rows(gp):
    """Precision workload at full size (n = 434,874, d = 3, 65 columns) in the
    configuration the bench times (bf16x3 products, rank-8000 pivoted-Cholesky
    preconditioner): a cold solve at the data-generating theta, then a solve at a
    moved theta (every hyperparameter moved by about one Adam step, lr 0.03)
    warm-started from the first solution and reusing its factor.  On 192 sampled
    rows the oracle recomputes B - H U in FP64 from the same U; the library's FP32
    residual (its FP32 product) must agree entry by entry to the FP32 product's
    accuracy, and the residual norms the library reports must agree with the
    sampled-row estimate."""
    import torch
    from paper_2405_18457_amd import api
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w)
    tr = wl.truth_draws(w)
    md = wl.model_pathwise_draws(w)
    theta = np.concatenate([tr["ell"], [1.0, w.sigma]])
    Xd = dev(X)
    announce("full-D rhs")
    # right-hand sides of the pathwise system: targets from the data-generating
    # random-feature draw, probes f(x) + sigma eps from the model's fixed features
    y = api.gp_prior_sample(gp, Xd, theta, dev(tr["t"]), dev(tr["w"][:, None]))[:, 0]
    y = y + w.sigma * dev(tr["noise"])
    xi = api.gp_prior_sample(gp, Xd, theta, dev(md["t"]), dev(md["W"])) + w.sigma * dev(md["w_eps"])
    Bd = torch.cat([y[:, None], xi], dim=1).contiguous()
    U = torch.zeros_like(Bd)
    announce("full-D cold solve")
    s1 = api.gp_solve(gp, Xd, theta, Bd, U, api.solver_cfg(
        tol=1e-2, precision=api.GP_BF16X3, precond_rank=8000, precond_reuse=1))
    moved = theta * np.array([1.03, 0.97, 1.03, 0.97, 1.03])
    announce("full-D warm solve")
    s2 = api.gp_solve(gp, Xd, moved, Bd, U, api.solver_cfg(
        tol=1e-2, precision=api.GP_BF16X3, precond_rank=8000, precond_reuse=1))
    print(f"[gpu-case] cold {s1['iterations']} iterations, warm {s2['iterations']}", flush=True)
    assert s1["converged"] and s2["converged"] and s2["iterations"] < s1["iterations"]
    HU = api.gp_kmatvec(gp, Xd, Xd, moved, U, precision=api.GP_FP32, add_noise=True)
    rows = np.sort(np.random.default_rng(16).choice(w.n, 192, replace=False))
    ri = torch.from_numpy(rows).cuda()
    R_lib = host((Bd - HU)[ri])
    Uh = host(U)
    HU_ref = (kernel.k_matvec(X[rows], X, moved, Uh) + moved[-1] ** 2 * Uh[rows])
    R_ref = host(Bd[ri]) - HU_ref
    # Entry by entry the FP32 residual inherits the FP32 product's rounding, which is
    # relative to the magnitudes of the terms, S_i = a^2 sum_j k_ij |u_j| + sigma^2 |u_i|,
    # not to the residual: the solution's components along small eigenvalues are
    # large and cancel in H U.  Bound per entry: the squared-distance cancellation of
    # the norm expansion, |d r^2| <= 3u (|x^_i|^2 + |x^_j|^2), moves the Matern value
    # by at most (ln 2)^2 / 2 |d r^2| of itself, plus 64 units for the evaluation and
    # the FP32 accumulation (u = 2^-24).
    u32 = 2.0 ** -24
    S = kernel.k_matvec(X[rows], X, moved, np.abs(Uh)) + moved[-1] ** 2 * np.abs(Uh[rows])
    scl = np.sqrt(3.0) / np.log(2.0) / moved[:3]
    nrm = ((X.astype(np.float64) * scl) ** 2).sum(1)
    per_entry = (np.log(2.0) ** 2 / 2 * 3 * u32 * (nrm[rows] + nrm.max()) + 64 * u32)[:, None]
    units = float(np.max(np.abs(R_lib - R_ref) / (per_entry * S)))
    ent = float(np.max(np.abs(R_lib - R_ref)) / np.max(np.abs(R_ref)))
    assert units <= 1.0, units
    # norms: the library's true residual against the oracle's sampled-row estimate
    nb = np.linalg.norm(host(Bd), axis=0)
    est = np.sqrt(np.sum(R_ref ** 2, axis=0) * w.n / len(rows)) / nb
    est_y, est_z = float(est[0]), float(np.mean(est[1:]))
    print(f"[gpu-case] relres library ({s2['true_relres_y']:.4f}, {s2['true_relres_z']:.4f}), "
          f"sampled oracle rows ({est_y:.4f}, {est_z:.4f}); entry error {ent:.2e} of max |R|, "
          f"{units:.3f} of the per-entry bound", flush=True)
    # 192 rows estimate a mean square to about 1/sqrt(192 / 2) = 10 % (chi-square), so
    # 25 % on the norm of a single column and 10 % on the mean over 64 columns
    assert abs(est_y - s2["true_relres_y"]) <= 0.25 * s2["true_relres_y"]
    assert abs(est_z - s2["true_relres_z"]) <= 0.10 * s2["true_relres_z"]
    assert est_z <= 1.1e-2
