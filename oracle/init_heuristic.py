"""Initial hyperparameters for large data sets (FP64 oracle; test infrastructure only).

App. B ("Iterative Optimiser") obtains the starting hyperparameters of the
large data sets with a heuristic taken from earlier work on sampling-based
GP inference:

  1. pick a centroid training example uniformly at random;
  2. take the m (10,000 in the paper) training examples with the smallest
     Euclidean distance to it;
  3. maximise the exact marginal likelihood (Sec. 2, eq. mll) on that subset;
  4. repeat for 10 centroids and average the hyperparameters.

The centroid draws are inputs here (the caller draws them).  Readings where the
appendix is silent:

  * distance: squared Euclidean distance in the raw input space (no length
    scales), summed over the dimensions in index order; ties are broken by the
    lower row index, and the subset is returned in ascending row order;
  * "maximising the exact marginal likelihood": Adam ascent on nu with
    theta = softplus(nu) and the paper's small-data settings (theta_0 = 1.0 for
    every hyperparameter, learning rate 0.1, 100 steps), using the exact
    Cholesky gradient of Sec. 2, eq. mll_grad;
  * "average the hyperparameters": the arithmetic mean of the constrained
    values theta over the centroids.
"""
from __future__ import annotations

import numpy as np

from . import mll, optim


def squared_distances(X, centre):
    """dist[i] = sum_j (X[i, j] - X[centre, j])^2 in FP64, dimensions in index order."""
    X = np.asarray(X, np.float64)
    c = X[centre]
    dist = np.zeros(X.shape[0])
    for j in range(X.shape[1]):
        diff = X[:, j] - c[j]
        dist = dist + diff * diff
    return dist


def nearest(X, centre, k):
    """Step 2: the k rows closest to row ``centre`` (lower index first among equal
    distances), returned in ascending row order as int64."""
    dist = squared_distances(X, centre)
    order = np.lexsort((np.arange(dist.shape[0]), dist))
    return np.sort(order[:k]).astype(np.int64)


def maximise_exact_mll(X, y, theta0, steps, lr, transform="softplus"):
    """Step 3: Adam ascent on the exact marginal likelihood; returns theta after
    the last update."""
    nu = optim.to_nu(np.asarray(theta0, np.float64), transform)
    adam = optim.Adam(lr)
    for _ in range(steps):
        theta = optim.to_theta(nu, transform)
        g = mll.mll_grad_exact(X, y, theta)
        nu = adam.step(nu, g * optim.dtheta_dnu(nu, transform))
    return optim.to_theta(nu, transform)


def init_heuristic(X, y, centres, m, steps=100, lr=0.1, theta0=None, transform="softplus"):
    """Steps 1-4 for the given centroid rows; returns (mean theta, per-centroid theta)."""
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    d = X.shape[1]
    theta0 = np.ones(d + 2) if theta0 is None else np.asarray(theta0, np.float64)
    each = []
    for c in centres:
        idx = nearest(X, int(c), m)
        each.append(maximise_exact_mll(X[idx], y[idx], theta0, steps, lr, transform))
    each = np.array(each)
    return each.mean(axis=0), each
