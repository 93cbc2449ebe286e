"""Log marginal likelihood, its exact gradient and the two stochastic estimators (FP64 oracle).

Sec. 2, eq. (mll):       L = -1/2 y^T H^-1 y - 1/2 log det H - n/2 log 2 pi
Sec. 2, eq. (mll_grad):  dL/dtheta_k = 1/2 (H^-1 y)^T dH_k (H^-1 y) - 1/2 tr(H^-1 dH_k)

Standard estimator (Sec. 2, eqs. trace and standard_system): solve
H [v_y, v_1..v_s] = [y, z_1..z_s] with z ~ N(0, I) and use
tr(H^-1 dH) ~ (1/s) sum_j v_j^T dH z_j   (dH symmetric, so z^T H^-1 dH z = v^T dH z).

Pathwise estimator (Sec. 3, eqs. pathwise_estimator and pathwise_system):
solve H [v_y, zhat_1..zhat_s] = [y, xi_1..xi_s] with xi = f(x) + eps ~ N(0, H)
and use tr(H^-1 dH) ~ (1/s) sum_j zhat_j^T dH zhat_j.

Both reduce to one bilinear adjoint with column weights
w = (1/2, -1/(2s), ..., -1/(2s)):  g_k = sum_c w_c U_c^T dH_k W_c, with
U = solutions and W = [v_y, z] (standard) or W = U (pathwise).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kernel


def log_marginal_likelihood(X, y, theta):
    H = kernel.h_matrix(X, theta)
    L = np.linalg.cholesky(H)
    alpha = sla.cho_solve((L, True), np.asarray(y, np.float64))
    n = H.shape[0]
    return float(-0.5 * np.dot(y, alpha) - np.sum(np.log(np.diag(L))) - 0.5 * n * np.log(2 * np.pi))


def mll_grad_exact(X, y, theta):
    """Exact trace-formula gradient via a Cholesky factorisation (dense, small n)."""
    H = kernel.h_matrix(X, theta)
    cf = sla.cho_factor(H, lower=True)
    alpha = sla.cho_solve(cf, np.asarray(y, np.float64))
    Hinv = sla.cho_solve(cf, np.eye(H.shape[0]))
    grads = []
    for dH in kernel.dh_dtheta(X, theta):
        grads.append(0.5 * alpha @ dH @ alpha - 0.5 * np.sum(Hinv * dH))
    return np.array(grads)


def exact_solve(X, theta, B):
    H = kernel.h_matrix(X, theta)
    return sla.cho_solve(sla.cho_factor(H, lower=True), np.asarray(B, np.float64))


def estimator_weights(s):
    w = np.full(s + 1, -1.0 / (2.0 * s)) if s > 0 else np.zeros(1)
    w[0] = 0.5
    return w


def standard_estimate(X, y, theta, Z, solutions=None):
    """Standard estimator with probes Z [n, s]; exact Cholesky solves unless
    ``solutions`` = [v_y, v_1..v_s] is given."""
    y = np.asarray(y, np.float64)
    Z = np.asarray(Z, np.float64)
    B = np.concatenate([y[:, None], Z], axis=1)
    V = exact_solve(X, theta, B) if solutions is None else np.asarray(solutions, np.float64)
    return kernel.adjoint(X, theta, V, B_with_vy(V, Z), estimator_weights(Z.shape[1]))


def B_with_vy(V, Z):
    """W = [v_y, z_1..z_s] for the standard estimator."""
    return np.concatenate([V[:, :1], np.asarray(Z, np.float64)], axis=1)


def pathwise_estimate(X, y, theta, Xi, solutions=None):
    """Pathwise estimator with right-hand sides Xi [n, s] (xi_j = f_j(x) + eps_j);
    exact Cholesky solves unless ``solutions`` = [v_y, zhat_1..zhat_s] is given."""
    y = np.asarray(y, np.float64)
    Xi = np.asarray(Xi, np.float64)
    B = np.concatenate([y[:, None], Xi], axis=1)
    V = exact_solve(X, theta, B) if solutions is None else np.asarray(solutions, np.float64)
    return kernel.adjoint(X, theta, V, V, estimator_weights(Xi.shape[1]))
