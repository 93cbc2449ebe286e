"""Pins for the oracle's pivoted-Cholesky preconditioner and preconditioned CG
(App. B, Algorithm 1 with P(.)), each against something other than the oracle:
LAPACK's pivoted Cholesky, dense solves, the rank-n identity L L^T = K and the
Krylov optimality of preconditioned CG."""
import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

from oracle import kernel, precond, solvers


def _problem(n, d=3, seed=5, sigma=0.2):
    g = np.random.default_rng(seed)
    X = g.uniform(-1, 1, (n, d))
    ell = g.uniform(0.2, 0.5, d)
    theta = np.concatenate([ell, [1.3, sigma]])
    B = g.standard_normal((n, 4))
    return X, theta, B


def test_pivoted_cholesky_matches_lapack_dpstrf():
    X, theta, _ = _problem(90)
    d = X.shape[1]
    K = kernel.kernel_matrix(X, X, theta[:d], theta[d])
    c, piv, rank, info = lapack.dpstrf(K, lower=1, tol=-1.0)
    Lref = np.tril(c)
    k = 30
    L, p = precond.pivoted_cholesky(X, theta, k)
    assert p == list(piv[:k] - 1)
    # column j of the LAPACK factor lives in pivoted row order
    Lperm = np.zeros((90, k))
    Lperm[piv - 1, :] = Lref[:, :k]
    np.testing.assert_allclose(L, Lperm, rtol=0, atol=1e-10)


def test_full_rank_factor_reproduces_k_and_first_pivot_is_index_zero():
    X, theta, _ = _problem(40)
    d = X.shape[1]
    L, p = precond.pivoted_cholesky(X, theta, 40)
    K = kernel.kernel_matrix(X, X, theta[:d], theta[d])
    np.testing.assert_allclose(L @ L.T, K, rtol=0, atol=1e-9)
    assert p[0] == 0  # every diagonal entry is a^2: the tie goes to the lowest index
    assert sorted(p) == list(range(40))


def test_partial_factor_trace_decreases_and_error_is_psd():
    X, theta, _ = _problem(70)
    d = X.shape[1]
    K = kernel.kernel_matrix(X, X, theta[:d], theta[d])
    prev = np.trace(K)
    for k in (5, 10, 20):
        L, _ = precond.pivoted_cholesky(X, theta, k)
        E = K - L @ L.T
        assert np.linalg.eigvalsh(E).min() > -1e-10  # Schur complement of a PSD matrix
        assert np.trace(E) < prev
        prev = np.trace(E)


def test_woodbury_equals_dense_inverse():
    X, theta, B = _problem(60)
    L, _ = precond.pivoted_cholesky(X, theta, 12)
    s2 = theta[-1] ** 2
    P = L @ L.T + s2 * np.eye(60)
    W = precond.Woodbury(L, s2)
    np.testing.assert_allclose(W(B), np.linalg.solve(P, B), rtol=1e-9, atol=1e-9)
    W0 = precond.Woodbury(np.zeros((60, 0)), s2)
    np.testing.assert_allclose(W0(B), B / s2)


def test_pcg_with_exact_preconditioner_converges_in_one_step():
    X, theta, B = _problem(50)
    op = solvers.DenseOperator(X, theta)
    P = precond.preconditioner(X, theta, 50)  # rank n: P = K + sigma^2 I = H
    U, st = solvers.cg(op, B, tol=1e-9, precond=P)
    assert st["iterations"] == 1
    np.testing.assert_allclose(U, np.linalg.solve(op.H, B), rtol=1e-7, atol=1e-9)


def test_pcg_iterate_is_optimal_over_preconditioned_krylov_space():
    # After m steps from 0, u_m minimises ||u - u*||_H over
    # span{z, (P^-1 H) z, ..., (P^-1 H)^{m-1} z} with z = P^-1 b.
    X, theta, B = _problem(40, sigma=0.3)
    op = solvers.DenseOperator(X, theta)
    H = op.H
    b = B[:, :1]
    L, _ = precond.pivoted_cholesky(X, theta, 6)
    Pinv = np.linalg.inv(L @ L.T + theta[-1] ** 2 * np.eye(40))
    P = precond.Woodbury(L, theta[-1] ** 2)
    for m in (1, 2, 4):
        U, st = solvers.cg(op, b, tol=0.0, max_epochs=m, precond=P)
        assert st["iterations"] == m
        z = Pinv @ b
        Kr = np.hstack([np.linalg.matrix_power(Pinv @ H, i) @ z for i in range(m)])
        Q, _ = np.linalg.qr(Kr)
        u_opt = Q @ np.linalg.solve(Q.T @ H @ Q, Q.T @ b)
        np.testing.assert_allclose(U, u_opt, rtol=1e-6, atol=1e-9)


def test_pcg_reaches_tolerance_in_fewer_iterations_on_a_poorly_conditioned_system():
    g = np.random.default_rng(9)
    X = g.uniform(-1, 1, (400, 3))
    theta = np.array([0.3, 0.4, 0.5, 1.0, 0.05])
    B = g.standard_normal((400, 5))
    op = solvers.DenseOperator(X, theta)
    U0, s0 = solvers.cg(op, B, tol=1e-3)
    U1, s1 = solvers.cg(op, B, tol=1e-3, precond=precond.preconditioner(X, theta, 40))
    assert s0["converged"] and s1["converged"]
    assert s1["iterations"] < s0["iterations"]
    for U in (U0, U1):
        ry, rz = solvers.true_relres(op, B, U)
        assert ry <= 1.0001e-3 and rz <= 1.0001e-3
