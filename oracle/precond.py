"""Pivoted-Cholesky preconditioner for conjugate gradients (FP64 oracle).

App. B ("Conjugate Gradients") runs CG with a rank-100 pivoted Cholesky
preconditioner, following the exact-GP CG literature it cites (Wang et al.
2019; Gardner et al. 2018).  The construction is the greedy partial Cholesky
factorisation of the kernel matrix (Harbrecht, Peters & Schneider 2012): at
every step the row with the largest remaining diagonal is the pivot p,

    l_j = (K[:, p] - L[:, :j] L[p, :j]^T) / sqrt(d_p),   d <- d - l_j^2,

so that after k steps K ~ L L^T with L [n, k].  The preconditioner matrix is
P = L L^T + sigma^2 I and Algorithm 1's P(.) applies its inverse, here through
the Woodbury identity

    P^-1 r = (r - L (sigma^2 I_k + L^T L)^-1 L^T r) / sigma^2.

Ties in the pivot choice go to the lowest index.  The factorisation stops early
when the largest remaining diagonal is not positive (K numerically of rank < k).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import kernel


def pivoted_cholesky(X, theta, k):
    """Rank-k greedy pivoted Cholesky of K(X, X).  Returns (L [n, k'], pivots)."""
    X = np.asarray(X, np.float64)
    n, d = X.shape
    ell, a = np.asarray(theta[:d], np.float64), float(theta[d])
    diag = np.full(n, a * a)
    L = np.zeros((n, min(k, n)))
    piv = []
    for j in range(min(k, n)):
        p = int(np.argmax(diag))  # first index among equal maxima
        if not diag[p] > 0.0:
            return L[:, :j], piv
        col = kernel.kernel_matrix(X, X[p:p + 1], ell, a)[:, 0]
        col = col - L[:, :j] @ L[p, :j]
        L[:, j] = col / np.sqrt(diag[p])
        diag = diag - L[:, j] ** 2
        diag[p] = 0.0
        piv.append(p)
    return L, piv


class Woodbury:
    """P^-1 for P = L L^T + sigma^2 I."""

    def __init__(self, L, sigma2):
        self.L = np.asarray(L, np.float64)
        self.sigma2 = float(sigma2)
        k = self.L.shape[1]
        self.chol = sla.cho_factor(self.sigma2 * np.eye(k) + self.L.T @ self.L, lower=True)

    def __call__(self, R):
        R = np.asarray(R, np.float64)
        if self.L.shape[1] == 0:
            return R / self.sigma2
        S = sla.cho_solve(self.chol, self.L.T @ R)
        return (R - self.L @ S) / self.sigma2


def preconditioner(X, theta, k):
    """Algorithm 1's P(.) for H = K + sigma^2 I with a rank-k pivoted Cholesky factor."""
    d = np.asarray(X).shape[1]
    L, _ = pivoted_cholesky(X, theta, k)
    return Woodbury(L, float(theta[d + 1]) ** 2)
