"""Matern-3/2 ARD kernel and the regularised kernel matrix, FP64 (test oracle only).

The paper uses a Matern-3/2 kernel with one length scale per input dimension
and a scalar signal scale (Sec. 2; App. B "Kernel Function and Random
Features").  It does not print the formula; we take the textbook form
(Rasmussen & Williams 2006, eq. 4.17):

    r^2 = sum_k ((x_k - x'_k) / ell_k)^2,   k(x, x') = a^2 (1 + sqrt(3) r) exp(-sqrt(3) r)

The regularised matrix is H = K(x, x) + sigma^2 I (Sec. 2, definition of
H_theta).  Hyperparameters are ordered theta = (ell_1..ell_d, a, sigma).

Derivatives (differentiating the formula above):
    dk/dell_k = 3 a^2 exp(-sqrt(3) r) (x_k - x'_k)^2 / ell_k^3
    dk/da     = 2 k / a
    dH/dsigma = 2 sigma I                       (App. A, noise-scale example)
"""
from __future__ import annotations

import numpy as np

SQRT3 = np.sqrt(3.0)


def _split(theta, d):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (d + 2,), (theta.shape, d)
    return theta[:d], theta[d], theta[d + 1]


def _chunk_rows(n1, n2, d, budget_bytes=1 << 27):
    per_row = max(1, n2 * max(d, 1) * 8)
    return max(1, min(n1, budget_bytes // per_row))


def scaled_sqdist(X1, X2, ell):
    """Dense r^2 [n1, n2] from direct coordinate differences (no norm expansion)."""
    A = np.asarray(X1, np.float64) / ell
    B = np.asarray(X2, np.float64) / ell
    out = np.empty((A.shape[0], B.shape[0]))
    step = _chunk_rows(A.shape[0], B.shape[0], A.shape[1])
    for s in range(0, A.shape[0], step):
        diff = A[s:s + step, None, :] - B[None, :, :]
        out[s:s + step] = np.einsum("ijk,ijk->ij", diff, diff)
    return out


def matern32_of_r(r, a):
    return a * a * (1.0 + SQRT3 * r) * np.exp(-SQRT3 * r)


def kernel_matrix(X1, X2, ell, a):
    """K(X1, X2) [n1, n2] in FP64."""
    return matern32_of_r(np.sqrt(scaled_sqdist(X1, X2, ell)), a)


def h_matrix(X, theta):
    """Dense H = K(X, X) + sigma^2 I."""
    X = np.asarray(X, np.float64)
    ell, a, sigma = _split(theta, X.shape[1])
    H = kernel_matrix(X, X, ell, a)
    H[np.diag_indices_from(H)] += sigma * sigma
    return H


def k_matvec(X1, X2, theta, V, add_noise=False):
    """K(X1, X2) V (+ sigma^2 V when add_noise, which requires X1 == X2 row for row),
    matrix-free over row chunks of X1, FP64."""
    X1 = np.asarray(X1, np.float64)
    X2 = np.asarray(X2, np.float64)
    V = np.asarray(V, np.float64)
    ell, a, sigma = _split(theta, X1.shape[1])
    out = np.empty((X1.shape[0],) + V.shape[1:])
    step = _chunk_rows(X1.shape[0], X2.shape[0], X1.shape[1])
    for s in range(0, X1.shape[0], step):
        out[s:s + step] = kernel_matrix(X1[s:s + step], X2, ell, a) @ V
    if add_noise:
        assert X1.shape[0] == V.shape[0]
        out += sigma * sigma * V
    return out


def h_matvec(X, theta, V):
    """H V = K(X, X) V + sigma^2 V."""
    return k_matvec(X, X, theta, V, add_noise=True)


def dh_dtheta(X, theta):
    """List of the d+2 dense derivative matrices dH/dtheta_k (small n only)."""
    X = np.asarray(X, np.float64)
    n, d = X.shape
    ell, a, sigma = _split(theta, d)
    r = np.sqrt(scaled_sqdist(X, X, ell))
    e = np.exp(-SQRT3 * r)
    out = []
    for k in range(d):
        delta2 = (X[:, None, k] - X[None, :, k]) ** 2
        out.append(3.0 * a * a * e * delta2 / ell[k] ** 3)
    out.append(2.0 * matern32_of_r(r, a) / a)
    out.append(2.0 * sigma * np.eye(n))
    return out


def adjoint(X, theta, U, W, weights):
    """grad_k = sum_c weights_c * U[:, c]^T (dH/dtheta_k) W[:, c] for all d+2 hyperparameters.

    Written as sum_ij G_ij dK_ij / dtheta_k with G = U diag(weights) W^T,
    accumulated over row chunks (matrix-free), plus the sigma term
    2 sigma sum_c weights_c U_c . W_c.
    """
    X = np.asarray(X, np.float64)
    U = np.asarray(U, np.float64)
    W = np.asarray(W, np.float64)
    w = np.asarray(weights, np.float64)
    n, d = X.shape
    ell, a, sigma = _split(theta, d)
    grad = np.zeros(d + 2)
    step = _chunk_rows(n, n, d + 2)
    for s in range(0, n, step):
        Xi = X[s:s + step]
        G = (U[s:s + step] * w) @ W.T
        r = np.sqrt(scaled_sqdist(Xi, X, ell))
        e = np.exp(-SQRT3 * r)
        for k in range(d):
            delta2 = (Xi[:, None, k] - X[None, :, k]) ** 2
            grad[k] += np.sum(G * (3.0 * a * a * e * delta2 / ell[k] ** 3))
        grad[d] += np.sum(G * (2.0 * matern32_of_r(r, a) / a))
    grad[d + 1] = 2.0 * sigma * np.sum(w * np.einsum("ic,ic->c", U, W))
    return grad
