"""Pins for the FP64 oracle: each check is against something other than the
oracle itself -- a library routine, a closed form, finite differences, an
invariant, brute force, or a Monte Carlo expectation with an exact standard
error -- chosen so that a dropped term, a wrong sign/index or a transposed
operand in the oracle fails at least one of them."""
import numpy as np
import pytest
import scipy.stats
import torch

import workloads as wl
from oracle import kernel, mll, optim, rff, solvers, train


def _data(n, d, seed, ell_lo=0.5, ell_hi=2.0, scale=1.0):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d)) * scale
    ell = g.uniform(ell_lo, ell_hi, d)
    return X, ell


# ---------------------------------------------------------------- kernel

def test_kernel_matches_sklearn_matern32():
    from sklearn.gaussian_process.kernels import Matern
    X, ell = _data(40, 5, 0)
    Y, _ = _data(30, 5, 1)
    a = 1.7
    ref = a * a * Matern(length_scale=ell, nu=1.5)(X, Y)
    np.testing.assert_allclose(kernel.kernel_matrix(X, Y, ell, a), ref, rtol=1e-12, atol=1e-14)


def test_kernel_closed_forms():
    a = 1.3
    # K_ii = a^2; k(r = 1/sqrt(3)) = 2 a^2 / e; d = 1, n = 2 hand value.
    ell = np.array([0.7])
    X = np.array([[0.0], [0.7 / np.sqrt(3.0)]])
    K = kernel.kernel_matrix(X, X, ell, a)
    assert K[0, 0] == pytest.approx(a * a, rel=1e-15)
    assert K[0, 1] == pytest.approx(2 * a * a / np.e, rel=1e-14)
    X2 = np.array([[0.0], [1.0]])
    K2 = kernel.kernel_matrix(X2, X2, np.array([1.0]), 1.0)
    assert K2[0, 1] == pytest.approx((1 + np.sqrt(3)) * np.exp(-np.sqrt(3)), rel=1e-14)
    assert K2[0, 1] == pytest.approx(0.48335772, rel=1e-7)


def test_kernel_symmetry_translation_psd():
    X, ell = _data(60, 3, 2)
    theta = np.concatenate([ell, [0.9, 0.2]])
    H = kernel.h_matrix(X, theta)
    np.testing.assert_array_equal(H, H.T)
    H2 = kernel.h_matrix(X + np.array([3.0, -1.0, 0.5]), theta)
    np.testing.assert_allclose(H, H2, atol=1e-12)
    assert np.linalg.eigvalsh(H).min() >= 0.2 ** 2 * (1 - 1e-9)


def test_dk_matches_sklearn_gradient():
    from sklearn.gaussian_process.kernels import Matern
    X, ell = _data(25, 4, 3)
    a = 1.4
    theta = np.concatenate([ell, [a, 0.3]])
    _, gK = Matern(length_scale=ell, nu=1.5)(X, eval_gradient=True)  # d/dlog(ell_k) of K/a^2
    dH = kernel.dh_dtheta(X, theta)
    for k in range(4):
        np.testing.assert_allclose(dH[k], a * a * gK[:, :, k] / ell[k], rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(dH[4], 2 * a * Matern(length_scale=ell, nu=1.5)(X), rtol=1e-12)
    np.testing.assert_allclose(dH[5], 2 * 0.3 * np.eye(25))


def test_matvec_matrix_free_equals_dense_and_rectangular():
    X, ell = _data(50, 3, 4)
    Q, _ = _data(7, 3, 5)
    theta = np.concatenate([ell, [1.1, 0.4]])
    V = np.random.default_rng(6).standard_normal((50, 5))
    np.testing.assert_allclose(kernel.h_matvec(X, theta, V), kernel.h_matrix(X, theta) @ V,
                               rtol=1e-12, atol=1e-12)
    from sklearn.gaussian_process.kernels import Matern
    ref = 1.1 ** 2 * Matern(length_scale=ell, nu=1.5)(Q, X) @ V
    np.testing.assert_allclose(kernel.k_matvec(Q, X, theta, V), ref, rtol=1e-12, atol=1e-12)


def test_adjoint_vs_central_differences():
    X, ell = _data(30, 3, 7)
    theta = np.concatenate([ell, [1.2, 0.35]])
    g = np.random.default_rng(8)
    U = g.standard_normal((30, 4))
    W = g.standard_normal((30, 4))
    w = np.array([0.5, -0.2, 0.3, -0.1])
    adj = kernel.adjoint(X, theta, U, W, w)

    def bilinear(th):
        return float(np.sum(w * np.einsum("ic,ic->c", U, kernel.h_matvec(X, th, W))))

    for k in range(len(theta)):
        h = 1e-5 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (bilinear(tp) - bilinear(tm)) / (2 * h)
        assert adj[k] == pytest.approx(fd, rel=1e-6, abs=1e-9), k


# ---------------------------------------------------------------- marginal likelihood

def test_mll_matches_scipy_logpdf():
    X, ell = _data(40, 2, 9)
    theta = np.concatenate([ell, [0.8, 0.25]])
    y = np.random.default_rng(10).standard_normal(40)
    H = kernel.h_matrix(X, theta)
    ref = scipy.stats.multivariate_normal(mean=np.zeros(40), cov=H).logpdf(y)
    assert mll.log_marginal_likelihood(X, y, theta) == pytest.approx(ref, rel=1e-10)


def test_mll_n1_closed_form():
    X = np.array([[0.3, -0.2]])
    theta = np.array([0.7, 1.9, 1.3, 0.4])
    y = np.array([0.9])
    v = 1.3 ** 2 + 0.4 ** 2
    ref = -0.5 * 0.81 / v - 0.5 * np.log(v) - 0.5 * np.log(2 * np.pi)
    assert mll.log_marginal_likelihood(X, y, theta) == pytest.approx(ref, rel=1e-14)


def test_mll_grad_vs_central_differences():
    X, ell = _data(35, 3, 11)
    theta = np.concatenate([ell, [1.1, 0.3]])
    y = np.random.default_rng(12).standard_normal(35)
    g = mll.mll_grad_exact(X, y, theta)
    for k in range(len(theta)):
        h = 1e-5 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mll.log_marginal_likelihood(X, y, tp) - mll.log_marginal_likelihood(X, y, tm)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-8), k


# ---------------------------------------------------------------- estimators (App. A variances)

def _small_problem(seed=13, n=30):
    X, ell = _data(n, 2, seed)
    theta = np.concatenate([ell, [1.0, 0.5]])
    y = np.random.default_rng(seed + 1).standard_normal(n)
    return X, y, theta


def test_standard_estimator_unbiased_with_exact_variance():
    X, y, theta = _small_problem()
    n, s, M = 30, 8, 400
    H = kernel.h_matrix(X, theta)
    Hinv = np.linalg.inv(H)
    exact = mll.mll_grad_exact(X, y, theta)
    g = np.random.default_rng(14)
    est = np.array([mll.standard_estimate(X, y, theta, g.standard_normal((n, s))) for _ in range(M)])
    for k, dH in enumerate(kernel.dh_dtheta(X, theta)):
        A = Hinv @ dH
        var = np.trace(A @ (A + A.T)) / (4 * s)          # App. A, standard-estimator variance
        se = np.sqrt(var / M)
        assert abs(est[:, k].mean() - exact[k]) < 4 * se + 1e-12, k
        # the empirical variance matches the closed form (chi-square-ish ratio bound)
        assert 0.75 < est[:, k].var() / var < 1.3, k


def test_pathwise_estimator_unbiased_exact_prior_and_variance():
    X, y, theta = _small_problem(15)
    n, s, M = 30, 8, 400
    H = kernel.h_matrix(X, theta)
    L = np.linalg.cholesky(H)
    Hinv = np.linalg.inv(H)
    exact = mll.mll_grad_exact(X, y, theta)
    g = np.random.default_rng(16)
    est = np.array([mll.pathwise_estimate(X, y, theta, L @ g.standard_normal((n, s)))
                    for _ in range(M)])
    for k, dH in enumerate(kernel.dh_dtheta(X, theta)):
        var = 2 * np.trace(dH @ Hinv @ dH @ Hinv) / (4 * s)   # App. A, pathwise variance
        se = np.sqrt(var / M)
        assert abs(est[:, k].mean() - exact[k]) < 4 * se + 1e-12, k
        assert 0.75 < est[:, k].var() / var < 1.3, k


def test_equal_variance_for_noise_scale():
    X, y, theta = _small_problem(17)
    H = kernel.h_matrix(X, theta)
    Hinv = np.linalg.inv(H)
    dH = kernel.dh_dtheta(X, theta)[-1]            # 2 sigma I commutes with H
    A = Hinv @ dH
    assert np.trace(A @ (A + A.T)) == pytest.approx(2 * np.trace(dH @ Hinv @ dH @ Hinv), rel=1e-12)
    dHl = kernel.dh_dtheta(X, theta)[0]            # a length scale does not commute
    A = Hinv @ dHl
    assert abs(np.trace(A @ (A + A.T)) - 2 * np.trace(dHl @ Hinv @ dHl @ Hinv)) > 1e-6


def test_pathwise_rff_expectation_closed_form():
    # With the frequencies fixed, E over W, w_eps of the pathwise trace term is
    # tr(H^-1 (Phi Phi^T + sigma^2 I) H^-1 dH).
    X, y, theta = _small_problem(18, n=20)
    n, d = X.shape
    t = wl.draw_spectral_t3(np.random.default_rng(19), 50, d).astype(np.float64)
    Phi = rff.rff_features(X, t, theta[:d], theta[d])
    H = kernel.h_matrix(X, theta)
    Hinv = np.linalg.inv(H)
    C = Phi @ Phi.T + theta[-1] ** 2 * np.eye(n)
    g = np.random.default_rng(20)
    s, M = 16, 300
    samples = []
    for _ in range(M):
        B = rff.pathwise_rhs(X, y, theta, t, g.standard_normal((100, s)), g.standard_normal((n, s)))
        Z = np.linalg.solve(H, B[:, 1:])
        samples.append([np.mean(np.einsum("ij,ij->j", Z, dH @ Z)) for dH in kernel.dh_dtheta(X, theta)])
    samples = np.array(samples)
    for k, dH in enumerate(kernel.dh_dtheta(X, theta)):
        expect = np.trace(Hinv @ C @ Hinv @ dH)
        se = samples[:, k].std() / np.sqrt(M)
        assert abs(samples[:, k].mean() - expect) < 4 * se, k


def test_initial_distance_identities():
    # E[z^T H^-1 z] = tr H^-1 (standard) and E[xi^T H^-1 xi] = n (pathwise), Sec. 3.
    X, y, theta = _small_problem(21, n=25)
    H = kernel.h_matrix(X, theta)
    Hinv = np.linalg.inv(H)
    L = np.linalg.cholesky(H)
    g = np.random.default_rng(22)
    Z = g.standard_normal((25, 20000))
    q = np.einsum("ij,ij->j", Z, Hinv @ Z)
    assert abs(q.mean() - np.trace(Hinv)) < 4 * q.std() / np.sqrt(q.size)
    Xi = L @ g.standard_normal((25, 20000))
    q = np.einsum("ij,ij->j", Xi, Hinv @ Xi)
    assert abs(q.mean() - 25) < 4 * q.std() / np.sqrt(q.size)


# ---------------------------------------------------------------- random features

def test_rff_spectral_measure_reproduces_matern():
    g = np.random.default_rng(23)
    d = 3
    X = g.standard_normal((6, d))
    ell = np.array([0.7, 1.3, 2.0])
    a = 1.2
    M = 200_000
    t = wl.draw_spectral_t3(g, M, d).astype(np.float64)
    Phi = rff.rff_features(X, t, ell, a)
    approx = Phi @ Phi.T
    K = kernel.kernel_matrix(X, X, ell, a)
    omega = t / ell
    for i in range(6):
        for j in range(6):
            c = np.cos((X[i] - X[j]) @ omega.T) * a * a
            se = c.std() / np.sqrt(M)
            assert abs(approx[i, j] - K[i, j]) < 5 * se + 1e-12, (i, j)


def test_rff_prior_covariance_is_phi_phi_t():
    g = np.random.default_rng(24)
    X = g.standard_normal((5, 2))
    t = wl.draw_spectral_t3(g, 10, 2).astype(np.float64)
    theta = np.array([0.8, 1.5, 1.1, 0.1])
    F = rff.prior_sample(X, t, g.standard_normal((20, 100000)), theta)
    Phi = rff.rff_features(X, t, theta[:2], theta[2])
    np.testing.assert_allclose(np.cov(F, bias=True), Phi @ Phi.T, atol=0.03)


def test_posterior_samples_mean_and_covariance_exact_prior():
    # Pathwise conditioning (Sec. 2) with exact joint prior draws reproduces the
    # closed-form posterior mean and covariance (Sec. 2, eq. gp_posterior).
    g = np.random.default_rng(25)
    X = g.standard_normal((12, 2))
    Q = g.standard_normal((4, 2))
    theta = np.array([1.0, 0.8, 1.1, 0.3])
    y = g.standard_normal(12)
    Z = np.vstack([Q, X])
    Kzz = kernel.kernel_matrix(Z, Z, theta[:2], theta[2])
    L = np.linalg.cholesky(Kzz + 1e-10 * np.eye(16))
    S = 200_000
    F = L @ g.standard_normal((16, S))
    fq, fx = F[:4], F[4:]
    eps = theta[3] * g.standard_normal((12, S))
    H = kernel.h_matrix(X, theta)
    Kqx = kernel.kernel_matrix(Q, X, theta[:2], theta[2])
    post = fq + Kqx @ np.linalg.solve(H, y[:, None] - (fx + eps))
    mu = Kqx @ np.linalg.solve(H, y)
    cov = kernel.kernel_matrix(Q, Q, theta[:2], theta[2]) - Kqx @ np.linalg.solve(H, Kqx.T)
    np.testing.assert_allclose(post.mean(1), mu, atol=5 * np.sqrt(np.diag(cov).max() / S))
    np.testing.assert_allclose(np.cov(post, bias=True), cov, atol=0.02)


def test_rff_posterior_samples_mean_is_exact_posterior_mean():
    g = np.random.default_rng(26)
    X = g.standard_normal((15, 2))
    Q = g.standard_normal((3, 2))
    theta = np.array([1.1, 0.9, 1.0, 0.4])
    y = g.standard_normal(15)
    t = wl.draw_spectral_t3(g, 30, 2).astype(np.float64)
    S = 20000
    W = g.standard_normal((60, S))
    B = rff.pathwise_rhs(X, y, theta, t, W, g.standard_normal((15, S)))
    sol = mll.exact_solve(X, theta, B)
    post = rff.posterior_samples(Q, X, theta, t, W, sol[:, 0], sol[:, 1:])
    mu = kernel.kernel_matrix(Q, X, theta[:2], theta[2]) @ np.linalg.solve(kernel.h_matrix(X, theta), y)
    se = post.std(1) / np.sqrt(S)
    assert np.all(np.abs(post.mean(1) - mu) < 5 * se)


# ---------------------------------------------------------------- solvers (App. B, Algs. 1-3)

def _spd_problem(n=40, d=2, s=3, seed=27, sigma=0.3):
    X, ell = _data(n, d, seed)
    theta = np.concatenate([ell, [1.0, sigma]])
    B = np.random.default_rng(seed + 1).standard_normal((n, s + 1))
    return X, theta, B


def test_cg_finite_termination_tiny():
    X, theta, B = _spd_problem(n=12, sigma=0.8)
    op = solvers.DenseOperator(X, theta)
    U, st = solvers.cg(op, B, tol=1e-11, max_epochs=40)
    np.testing.assert_allclose(U, np.linalg.solve(op.H, B), rtol=1e-7, atol=1e-9)
    assert st["iterations"] <= 12 + 3


def test_cg_iterate_is_krylov_optimal():
    # After k CG steps from 0, u_k minimises ||u - u*||_H over span{b, Hb, .., H^{k-1} b}.
    X, theta, B = _spd_problem(n=30)
    op = solvers.DenseOperator(X, theta)
    b = B[:, :1]
    H = op.H
    for k in (1, 2, 5):
        U, st = solvers.cg(op, b, tol=0.0, max_epochs=k)
        assert st["iterations"] == k
        K = np.hstack([np.linalg.matrix_power(H, i) @ b for i in range(k)])
        Q, _ = np.linalg.qr(K)
        u_opt = Q @ np.linalg.solve(Q.T @ H @ Q, Q.T @ b)
        np.testing.assert_allclose(U, u_opt, rtol=1e-6, atol=1e-9)


def test_cg_tolerance_budget_and_warm_start():
    X, theta, B = _spd_problem(n=60, sigma=0.1)
    op = solvers.DenseOperator(X, theta)
    U, st = solvers.cg(op, B, tol=1e-2)
    assert st["converged"]
    ry, rz = solvers.true_relres(op, B, U)
    assert ry <= 1.0001e-2 and rz <= 1.0001e-2
    U2, st2 = solvers.cg(op, B, tol=1e-8, max_epochs=3)
    assert st2["iterations"] == 3 and not st2["converged"]
    exact = np.linalg.solve(op.H, B)
    U3, st3 = solvers.cg(op, B, tol=1e-2, U0=exact)
    assert st3["iterations"] == 0
    # linearity: scaling b by a power of two scales u (same iterations on a
    # well-conditioned system; an ill-conditioned one amplifies rounding)
    X, theta, B = _spd_problem(n=60, sigma=0.7)
    op = solvers.DenseOperator(X, theta)
    U, st = solvers.cg(op, B, tol=1e-2)
    U4, st4 = solvers.cg(op, 8.0 * B, tol=1e-2)
    assert st4["iterations"] == st["iterations"]
    np.testing.assert_allclose(U4, 8.0 * U, rtol=1e-8, atol=1e-10)


def test_cg_nonfinite_and_breakdown():
    X, theta, B = _spd_problem(n=10)
    op = solvers.DenseOperator(X, theta)
    Bn = B.copy()
    Bn[3, 1] = np.nan
    with pytest.raises(solvers.SolverError) as e:
        solvers.cg(op, Bn)
    assert e.value.code == "nonfinite"
    op.H = -op.H
    with pytest.raises(solvers.SolverError) as e:
        solvers.cg(op, B)
    assert e.value.code == "breakdown"


def test_ap_full_block_is_exact_in_one_step():
    X, theta, B = _spd_problem(n=25)
    op = solvers.DenseOperator(X, theta)
    U, st = solvers.ap(op, B, block=25, tol=1e-3)
    assert st["iterations"] == 1
    np.testing.assert_allclose(U, np.linalg.solve(op.H, B), rtol=1e-9, atol=1e-10)


def test_ap_projection_zeroes_selected_block_and_converges():
    X, theta, B = _spd_problem(n=47)
    op = solvers.DenseOperator(X, theta)
    for steps in range(1, 6):
        U, st = solvers.ap(op, B, block=10, tol=0.0, max_epochs=(steps - 0.5) * 10 / 47)
        assert st["iterations"] == steps
        k = st["chosen"][-1]
        I = np.arange(k * 10, min(k * 10 + 10, 47))
        Rtrue = B - op.H @ U
        assert np.abs(Rtrue[I]).max() < 1e-9 * np.abs(B).max()
    U, st = solvers.ap(op, B, block=10, tol=1e-3)
    assert st["converged"]
    ry, rz = solvers.true_relres(op, B, U)
    assert max(ry, rz) <= 1.0001e-3
    # the last block is ragged (47 = 4 * 10 + 7) and the budget rounds up: t < (n/b) T
    U, st = solvers.ap(op, B, block=10, tol=0.0, max_epochs=1)
    assert st["iterations"] == 5


class _IdentityOperator:
    def __init__(self, n):
        self.H = np.eye(n)

    def matvec(self, V):
        return self.H @ V

    def rows(self, idx):
        return self.H[idx, :]

    def block(self, idx):
        return self.H[np.ix_(idx, idx)]


def test_ap_selects_by_the_norm_of_the_summed_residual_block():
    # H = I, two blocks of two rows.  In block 0 the two residual columns cancel
    # in their sum, so the summed-residual score picks block 1 first although
    # each column alone is larger in block 0 (a per-column score would pick block
    # 0).  Block 1's projection zeroes it, leaving a tie at zero, which goes to
    # the lower index; with H = I the two projections solve the system exactly.
    B = np.array([[1.0, -1.0], [0.0, 0.0], [0.3, 0.3], [0.0, 0.0]])
    U, st = solvers.ap(_IdentityOperator(4), B, block=2, tol=1e-12)
    assert st["chosen"] == [1, 0]
    assert st["iterations"] == 2 and st["converged"]
    np.testing.assert_allclose(U, B, rtol=1e-15, atol=1e-15)
    # the per-column reading would differ on the first choice
    Bt = B / np.linalg.norm(B, axis=0)
    per_column = [np.abs(Bt[I]).sum() for I in (np.arange(2), np.arange(2, 4))]
    assert int(np.argmax(per_column)) == 0


def test_sgd_full_batch_is_heavy_ball_and_converges():
    X, theta, B = _spd_problem(n=30, sigma=0.6)
    op = solvers.DenseOperator(X, theta)
    iters = 3000
    batches = np.tile(np.arange(30), (iters, 1))
    lr = 30 * 0.5 / np.linalg.eigvalsh(op.H).max()
    U, st = solvers.sgd(op, B, batches, lr=lr, momentum=0.9, tol=1e-6)
    assert st["converged"]
    np.testing.assert_allclose(U, np.linalg.solve(op.H, B), rtol=1e-4, atol=1e-5)
    # with the full batch the residual estimate is the exact residual at the pre-update iterate
    U1, st1 = solvers.sgd(op, B, batches, lr=lr, momentum=0.9, tol=0.0, max_epochs=1)
    assert st1["iterations"] == 1
    Bt = B / (np.linalg.norm(B, axis=0) + solvers.EPS)
    ry, rz = solvers.relres(Bt)          # v was 0 before the single step
    assert st1["relres_y"] == pytest.approx(ry) and st1["relres_z"] == pytest.approx(rz)


def test_sgd_minibatch_budget_semantics():
    X, theta, B = _spd_problem(n=50)
    op = solvers.DenseOperator(X, theta)
    batches = wl.draw_batch_indices(wl.WORKLOADS["B"], 100, 8, n=50)
    assert all(len(set(b)) == 8 for b in batches)
    U, st = solvers.sgd(op, B, batches, lr=1.0, tol=0.0, max_epochs=2)
    assert st["iterations"] == int(np.ceil(50 * 2 / 8))


def test_matrix_free_operator_rows_blocks():
    X, theta, B = _spd_problem(n=33)
    dense = solvers.DenseOperator(X, theta)
    mf = solvers.MatrixFreeOperator(X, theta)
    idx = np.array([3, 17, 0, 32])
    np.testing.assert_allclose(mf.rows(idx), dense.rows(idx), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(mf.block(idx), dense.block(idx), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(mf.matvec(B), dense.matvec(B), rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- optimiser

def test_adam_matches_torch_maximize():
    g = np.random.default_rng(28)
    nu = g.standard_normal(5)
    p = torch.tensor(nu.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.1, maximize=True)
    ours = optim.Adam(0.1)
    x = nu.copy()
    for _ in range(20):
        grad = g.standard_normal(5) * 3
        p.grad = torch.tensor(grad)
        opt.step()
        x = ours.step(x, grad)
        np.testing.assert_allclose(x, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adam_first_step_is_lr_sign():
    ours = optim.Adam(0.1)
    grad = np.array([3.0, -1e-3, 50.0])
    x = ours.step(np.zeros(3), grad)
    np.testing.assert_allclose(x, 0.1 * np.sign(grad), rtol=1e-4)


def test_transforms_vs_torch():
    nu = np.linspace(-30, 30, 61)
    th = optim.softplus(nu)
    np.testing.assert_allclose(th, np.log1p(np.exp(nu)),
                               rtol=1e-12)
    np.testing.assert_allclose(optim.softplus_inv(th[20:]), nu[20:], rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(optim.sigmoid(nu), torch.sigmoid(torch.tensor(nu)).numpy(), rtol=1e-12)
    np.testing.assert_allclose(optim.to_theta(optim.to_nu(np.array([0.3, 2.0]), "log"), "log"), [0.3, 2.0])


def test_trainer_exact_solver_ascends_mll():
    X, y, theta = _small_problem(29, n=40)
    draws = {"Z": np.random.default_rng(30).standard_normal((40, 64))}
    tr = train.Trainer(X, y, np.ones(4), "standard", draws, lr=0.1, transform="log", solver="exact")
    first = mll.log_marginal_likelihood(X, y, np.ones(4))
    for _ in range(15):
        tr.step()
    last = mll.log_marginal_likelihood(X, y, optim.to_theta(tr.nu, "log"))
    assert last > first


def _torch_surrogate_grad(nu, X, y, Z, transform):
    """Gradient in nu of a torch-autograd surrogate whose theta-gradient is the
    standard estimator with exact solves: -y^T H^-1 y / 2 gives alpha^T dH alpha / 2,
    and -(1/2s) sum_j v_j^T H z_j with v_j = H^-1 z_j held constant gives the
    probe term.  The Matern-3/2 kernel is written here independently."""
    n, d = X.shape
    s = Z.shape[1]
    p = torch.tensor(nu, dtype=torch.float64, requires_grad=True)
    th = torch.exp(p) if transform == "log" else torch.nn.functional.softplus(p)
    Xs = torch.tensor(X) / th[:d]
    r2 = ((Xs[:, None, :] - Xs[None, :, :]) ** 2).sum(-1)
    eye = torch.eye(n, dtype=torch.bool)
    r = torch.sqrt(torch.where(eye, torch.ones_like(r2), r2)) * 3.0 ** 0.5
    K = torch.where(eye, th[d] ** 2 * torch.ones_like(r2), th[d] ** 2 * (1 + r) * torch.exp(-r))
    H = K + th[d + 1] ** 2 * torch.eye(n, dtype=torch.float64)
    yt, Zt = torch.tensor(y), torch.tensor(Z)
    V = torch.linalg.solve(H.detach(), Zt)
    surrogate = -0.5 * yt @ torch.linalg.solve(H, yt) - (V * (H @ Zt)).sum() / (2 * s)
    surrogate.backward()
    return p.grad.numpy()


@pytest.mark.parametrize("transform", ["log", "softplus"])
def test_trainer_trajectory_matches_torch_autograd_and_adam(transform):
    # the whole composition (right-hand side, exact solve, estimator weights,
    # chain rule through the transform, Adam ascent) against torch autograd of
    # the surrogate and torch.optim.Adam(maximize=True)
    X, y, _ = _small_problem(31, n=35)
    Z = np.random.default_rng(32).standard_normal((35, 6))
    theta0 = np.array([0.9, 1.4, 1.1, 0.6])
    tr = train.Trainer(X, y, theta0, "standard", {"Z": Z}, lr=0.05, transform=transform,
                       solver="exact")
    p = torch.tensor(optim.to_nu(theta0, transform), dtype=torch.float64)
    opt = torch.optim.Adam([p], lr=0.05, maximize=True)
    for _ in range(6):
        theta, _, _ = tr.step()
        p.grad = torch.tensor(_torch_surrogate_grad(p.detach().numpy(), X, y, Z, transform))
        opt.step()
        np.testing.assert_allclose(tr.nu, p.detach().numpy(), rtol=1e-9, atol=1e-12)
    assert not np.allclose(tr.nu, optim.to_nu(theta0, transform))


def _torch_pathwise_surrogate_grad(nu, X, y, t, W, w_eps, transform):
    """As above for the pathwise estimator: xi = phi(x) W + sigma w_eps from the
    current theta (held constant), zhat = H^-1 xi held constant, and the probe
    term -(1/2s) sum_j zhat_j^T H zhat_j; features written here independently."""
    n, d = X.shape
    s = W.shape[1]
    p = torch.tensor(nu, dtype=torch.float64, requires_grad=True)
    th = torch.exp(p) if transform == "log" else torch.nn.functional.softplus(p)
    Xt = torch.tensor(X)
    Xs = Xt / th[:d]
    r2 = ((Xs[:, None, :] - Xs[None, :, :]) ** 2).sum(-1)
    eye = torch.eye(n, dtype=torch.bool)
    r = torch.sqrt(torch.where(eye, torch.ones_like(r2), r2)) * 3.0 ** 0.5
    K = torch.where(eye, th[d] ** 2 * torch.ones_like(r2), th[d] ** 2 * (1 + r) * torch.exp(-r))
    H = K + th[d + 1] ** 2 * torch.eye(n, dtype=torch.float64)
    with torch.no_grad():
        phase = Xt @ (torch.tensor(t) / th[:d]).T
        M = phase.shape[1]
        feats = th[d] / M ** 0.5 * torch.cat([torch.cos(phase), torch.sin(phase)], dim=1)
        xi = feats @ torch.tensor(W) + th[d + 1] * torch.tensor(w_eps)
        zhat = torch.linalg.solve(H, xi)
    yt = torch.tensor(y)
    surrogate = -0.5 * yt @ torch.linalg.solve(H, yt) - (zhat * (H @ zhat)).sum() / (2 * s)
    surrogate.backward()
    return p.grad.numpy()


def test_pathwise_trainer_trajectory_matches_torch_autograd_and_adam():
    X, y, _ = _small_problem(33, n=35)
    g = np.random.default_rng(34)
    M, s = 40, 5
    t = g.standard_normal((M, 2)) * np.sqrt(3.0 / g.chisquare(3, (M, 1)))
    W, w_eps = g.standard_normal((2 * M, s)), g.standard_normal((35, s))
    theta0 = np.array([1.2, 0.8, 1.0, 0.4])
    tr = train.Trainer(X, y, theta0, "pathwise", {"t": t, "W": W, "w_eps": w_eps}, lr=0.05,
                       solver="exact")
    p = torch.tensor(optim.to_nu(theta0, "softplus"), dtype=torch.float64)
    opt = torch.optim.Adam([p], lr=0.05, maximize=True)
    for _ in range(6):
        tr.step()
        p.grad = torch.tensor(_torch_pathwise_surrogate_grad(p.detach().numpy(), X, y, t, W,
                                                             w_eps, "softplus"))
        opt.step()
        np.testing.assert_allclose(tr.nu, p.detach().numpy(), rtol=1e-9, atol=1e-12)


def test_workload_generators_are_deterministic_and_shaped():
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w, n=1000)
    assert X.dtype == np.float32 and X.shape == (1000, 3)
    assert X.min() >= -1 and X.max() <= 1
    np.testing.assert_array_equal(X, wl.draw_inputs(w, n=1000))
    B = wl.draw_inputs(wl.WORKLOADS["B"], n=500)
    np.testing.assert_allclose(B.mean(0), 0, atol=1e-5)
    np.testing.assert_allclose(B.std(0), 1, atol=1e-5)
    th = wl.draw_random_theta(wl.WORKLOADS["C"])
    assert th.shape == (10, 11) and th[:, :10].min() >= 0.3 and th[:, -1].max() <= 1
