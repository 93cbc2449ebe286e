"""Pins for the initial-hyperparameter heuristic of the FP64 oracle (App. B,
"Iterative Optimiser"): nearest-subset selection against pure-Python brute force
and a k-d tree, the exact-likelihood maximiser against a one-point closed form
and an independent L-BFGS optimum, and the centroid average."""
import math

import numpy as np
import pytest
import scipy.optimize
import scipy.spatial
import scipy.stats
from sklearn.gaussian_process.kernels import Matern

import workloads as wl
from oracle import init_heuristic as ih
from oracle import mll, optim


def _brute_nearest(rows, centre, k):
    c = rows[centre]
    keyed = []
    for i, r in enumerate(rows):
        dist = 0.0
        for a, b in zip(r, c):
            dist += (a - b) * (a - b)
        keyed.append((dist, i))
    keyed.sort()
    return sorted(i for _, i in keyed[:k])


def test_nearest_matches_python_brute_force_with_ties():
    g = np.random.default_rng(0)
    X = g.integers(-3, 4, size=(40, 2)).astype(np.float32)  # many equal distances
    X[7] = X[3]                                            # a duplicate of a centre
    rows = [[float(v) for v in r] for r in X]
    for centre in (3, 7, 0, 39):
        for k in (0, 1, 2, 5, 17, 40):
            got = ih.nearest(X, centre, k)
            assert got.dtype == np.int64
            assert list(got) == _brute_nearest(rows, centre, k), (centre, k)
    # with a duplicate of the centre at a lower index, k = 1 takes the lower index
    assert list(ih.nearest(X, 7, 1)) == [3]


def test_nearest_matches_kdtree_and_separates_distances():
    X = wl.draw_inputs(wl.WORKLOADS["C"], n=3000)
    X64 = X.astype(np.float64)
    for centre, k in ((0, 1), (17, 300), (2999, 1000)):
        got = ih.nearest(X, centre, k)
        _, ref = scipy.spatial.cKDTree(X64).query(X64[centre], k=k)
        assert set(got.tolist()) == set(np.atleast_1d(ref).tolist())
        dist = ((X64 - X64[centre]) ** 2).sum(axis=1)
        mask = np.zeros(len(X), bool)
        mask[got] = True
        if k < len(X):
            assert dist[mask].max() <= dist[~mask].min()
        assert mask[centre]
    np.testing.assert_array_equal(ih.nearest(X[:50], 4, 50), np.arange(50))


def test_maximiser_one_point_closed_form():
    # One observation: L = -y^2 / (2 s) - log(s) / 2 - log(2 pi) / 2 with s = a^2 + sigma^2,
    # maximal at s = y^2; the length scales receive a zero gradient and stay put.
    X = np.array([[0.4, -1.0]])
    y = np.array([1.7])
    theta0 = np.array([0.6, 1.3, 1.0, 1.0])
    th = ih.maximise_exact_mll(X, y, theta0, steps=3000, lr=0.01)
    np.testing.assert_array_equal(th[:2], optim.to_theta(optim.to_nu(theta0[:2], "softplus"),
                                                         "softplus"))
    assert th[2] ** 2 + th[3] ** 2 == pytest.approx(1.7 ** 2, rel=1e-3)


def _neg_mll_independent(nu, X, y):
    # independent likelihood: scikit-learn's Matern-3/2 and scipy's Gaussian log-density
    th = np.logaddexp(0.0, nu)
    d = X.shape[1]
    K = th[d] ** 2 * Matern(length_scale=th[:d], nu=1.5)(X)
    H = K + th[d + 1] ** 2 * np.eye(len(y))
    return -scipy.stats.multivariate_normal(mean=np.zeros(len(y)), cov=H).logpdf(y)


def test_maximiser_reaches_independent_lbfgs_optimum():
    g = np.random.default_rng(3)
    X = g.standard_normal((40, 2))
    f = np.sin(1.3 * X[:, 0]) + 0.5 * np.cos(0.8 * X[:, 1])
    y = f + 0.2 * g.standard_normal(40)
    res = scipy.optimize.minimize(_neg_mll_independent, np.zeros(4), args=(X, y),
                                  method="L-BFGS-B", options=dict(gtol=1e-10, ftol=1e-14))
    th_ref = np.logaddexp(0.0, res.x)
    th = ih.maximise_exact_mll(X, y, np.ones(4), steps=3000, lr=0.02)
    assert -_neg_mll_independent(optim.to_nu(th, "softplus"), X, y) == pytest.approx(-res.fun,
                                                                                    abs=1e-5)
    np.testing.assert_allclose(th, th_ref, rtol=2e-2)


def test_heuristic_all_rows_and_mean():
    g = np.random.default_rng(4)
    X = g.standard_normal((30, 3))
    y = g.standard_normal(30)
    mean, each = ih.init_heuristic(X, y, [0, 11, 29], m=30, steps=5, lr=0.1)
    one = ih.maximise_exact_mll(X, y, np.ones(5), steps=5, lr=0.1)
    for row in each:
        np.testing.assert_array_equal(row, one)
    np.testing.assert_allclose(mean, one, rtol=1e-15)
    # distinct subsets: the result is the arithmetic mean of the per-centroid theta
    mean, each = ih.init_heuristic(X, y, [0, 11], m=12, steps=5, lr=0.1)
    assert not np.array_equal(each[0], each[1])
    np.testing.assert_allclose(mean, 0.5 * (each[0] + each[1]), rtol=1e-15)


def test_heuristic_ascends_each_subset_likelihood():
    X = wl.draw_inputs(wl.WORKLOADS["D"], n=400).astype(np.float64)
    y = np.sin(9.0 * X[:, 0]) * np.cos(6.0 * X[:, 1]) + 0.05 * np.random.default_rng(5).standard_normal(400)
    centres = [3, 200]
    _, each = ih.init_heuristic(X, y, centres, m=80, steps=20, lr=0.1)
    for c, th in zip(centres, each):
        idx = ih.nearest(X, c, 80)
        before = mll.log_marginal_likelihood(X[idx], y[idx], np.ones(5))
        after = mll.log_marginal_likelihood(X[idx], y[idx], th)
        assert after > before + 1.0
    assert math.isfinite(float(each.sum()))
