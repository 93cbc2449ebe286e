"""Random Fourier feature prior samples and pathwise right-hand sides (FP64 oracle).

The paper draws approximate prior functions with random Fourier features,
1000 sin/cos pairs (App. B "Kernel Function and Random Features"), and
refers to the literature for the construction (Rahimi & Recht 2008).  For
the Matern-3/2 ARD kernel the spectral measure is a multivariate Student-t
with 3 degrees of freedom, scaled per dimension by 1/ell_k.  With base draws
t_m (unit length scale) the frequencies are omega_m = t_m / ell and

    phi(x) = (a / sqrt(M)) [cos(x . omega_1..M), sin(x . omega_1..M)]   (2M features)
    f(x)   = phi(x) W,   W ~ N(0, I_2M)   (rows 0..M-1 weight cos, rows M..2M-1 weight sin)

so that Cov f = a^2 mean_m cos(omega_m . (x - x')) -> k(x, x').

Warm-start semantics (App. B): the base draws t, W and the noise base w_eps
are fixed; each outer step re-evaluates the features with the current
(ell, a) and sets eps = sigma w_eps.  Pathwise right-hand sides are
xi_j = f_j(x) + sigma w_eps_j (Sec. 3, eq. pathwise_system).

Posterior samples (Sec. 3, "Amortising Linear Solves"):
    (f|y)(x*) = f(x*) + k(x*, x) (v_y - zhat).
"""
from __future__ import annotations

import numpy as np

from . import kernel


def rff_features(X, t, ell, a):
    X = np.asarray(X, np.float64)
    omega = np.asarray(t, np.float64) / np.asarray(ell, np.float64)
    P = X @ omega.T
    M = omega.shape[0]
    return (a / np.sqrt(M)) * np.concatenate([np.cos(P), np.sin(P)], axis=1)


def prior_sample(X, t, W, theta):
    """f(X) = phi(X) W  ->  [n, s]."""
    X = np.asarray(X, np.float64)
    d = X.shape[1]
    theta = np.asarray(theta, np.float64)
    return rff_features(X, t, theta[:d], theta[d]) @ np.asarray(W, np.float64)


def pathwise_rhs(X, y, theta, t, W, w_eps):
    """B = [y, f_1(x) + sigma w_eps_1, ..., f_s(x) + sigma w_eps_s]  ->  [n, s+1]."""
    d = np.asarray(X).shape[1]
    sigma = float(np.asarray(theta)[d + 1])
    F = prior_sample(X, t, W, theta) + sigma * np.asarray(w_eps, np.float64)
    return np.concatenate([np.asarray(y, np.float64)[:, None], F], axis=1)


def truth_targets_rff(X, ell, a, sigma, t, w, noise):
    """Data-generating y = f(x) + sigma * noise with f an RFF draw (weights w [2M])."""
    theta = np.concatenate([ell, [a, sigma]])
    f = prior_sample(X, t, np.asarray(w, np.float64)[:, None], theta)[:, 0]
    return f + sigma * np.asarray(noise, np.float64)


def truth_targets_exact(X, ell, a, sigma, w, noise):
    """Data-generating y = L w + sigma * noise with L L^T = K(X, X) (exact GP draw)."""
    K = kernel.kernel_matrix(X, X, ell, a)
    K[np.diag_indices_from(K)] += 1e-10
    L = np.linalg.cholesky(K)
    return L @ np.asarray(w, np.float64) + sigma * np.asarray(noise, np.float64)


def posterior_samples(Xq, X, theta, t, W, v_y, zhat):
    """(f|y)(Xq) = f(Xq) + k(Xq, X)(v_y - zhat) for each of the s samples -> [m, s]."""
    prior = prior_sample(Xq, t, W, theta)
    diff = np.asarray(v_y, np.float64)[:, None] - np.asarray(zhat, np.float64)
    return prior + kernel.k_matvec(Xq, X, theta, diff)
