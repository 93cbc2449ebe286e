"""GPU parity of the initial-hyperparameter heuristic (App. B, "Iterative
Optimiser") through the C ABI: nearest-row selection (bit-exact against the
oracle, also at the two large workloads' full sizes), the dense FP64 exact
marginal likelihood and gradient (against the oracle's Cholesky definition, and
against central differences of itself at the paper's subset size m = 10,000),
and the whole heuristic against the oracle's Adam trajectories."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import announce, dev, require_gpu
from oracle import init_heuristic as ih
from oracle import mll
from paper_2405_18457_amd import api

pytestmark = pytest.mark.gpu

# FP64 on both sides; the Cholesky of H (condition number up to ~1e4 here)
# loses a few digits, and summation orders differ.
MLL_RTOL = 1e-10
GRAD_RTOL = 1e-8


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    c = api.Context(0)
    yield c
    c.close()


def _targets(X, seed, noise=0.1):
    g = np.random.default_rng(seed)
    X = np.asarray(X, np.float64)
    w = g.standard_normal(X.shape[1])
    y = np.sin(X @ w * 1.5) + 0.5 * np.cos(2.0 * X[:, 0]) + noise * g.standard_normal(X.shape[0])
    return y.astype(np.float32)


def _theta(d, seed, ell=(0.5, 2.0)):
    g = np.random.default_rng(seed)
    return np.concatenate([g.uniform(*ell, d), [g.uniform(0.7, 1.5), g.uniform(0.1, 0.5)]])


def _relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# ------------------------------------------------------------------ selection

def test_nearest_bit_exact_with_ties(ctx):
    g = np.random.default_rng(0)
    X = g.integers(-3, 4, size=(40, 2)).astype(np.float32)
    X[7] = X[3]
    Xd = dev(X)
    for centre in (3, 7, 0, 39):
        for k in (0, 1, 2, 5, 17, 39, 40):
            announce("nearest ties", centre, k)
            got = api.gp_nearest(ctx, Xd, centre, k).cpu().numpy()
            np.testing.assert_array_equal(got, ih.nearest(X, centre, k))


@pytest.mark.parametrize("n,d", [(1, 1), (2, 3), (1023, 3), (1024, 11), (1025, 1), (5000, 9),
                                 (70001, 24)])
def test_nearest_ragged_sizes(ctx, n, d):
    g = np.random.default_rng(n + d)
    X = g.standard_normal((n, d)).astype(np.float32)
    Xd = dev(X)
    for k in sorted({1, n // 3, n - 1, n} - {0}):
        centre = int(g.integers(0, n))
        announce("nearest", n, d, centre, k)
        got = api.gp_nearest(ctx, Xd, centre, k).cpu().numpy()
        np.testing.assert_array_equal(got, ih.nearest(X, centre, k))


@pytest.mark.parametrize("name", ["D", "E"])
def test_nearest_full_size_workloads(ctx, name):
    w = wl.WORKLOADS[name]
    X = wl.draw_inputs(w)
    Xd = dev(X)
    for centre in wl.draw_centroids(w)[:2]:
        announce("nearest full", name, w.n, int(centre))
        got = api.gp_nearest(ctx, Xd, int(centre), 10_000).cpu().numpy()
        np.testing.assert_array_equal(got, ih.nearest(X, int(centre), 10_000))


def test_nearest_errors(ctx):
    Xd = dev(np.zeros((10, 2), np.float32))
    for centre, k in ((0, 11), (0, -1), (10, 3), (-1, 3)):
        with pytest.raises(api.GPError) as e:
            api.gp_nearest(ctx, Xd, centre, k)
        assert e.value.code == api.N.GP_ERR_INVALID_ARG
    assert api.gp_nearest(ctx, Xd, 99, 0).numel() == 0


# ------------------------------------------------------------ exact likelihood

@pytest.mark.parametrize("m,d", [(1, 2), (2, 1), (63, 3), (64, 3), (65, 3), (200, 9), (777, 3),
                                 (1500, 11)])
def test_exact_mll_matches_oracle(ctx, m, d):
    g = np.random.default_rng(m * 100 + d)
    X = g.standard_normal((m, d)).astype(np.float32)
    y = _targets(X, m + d)
    theta = _theta(d, m + 7 * d, ell=(0.5 * np.sqrt(d), 1.5 * np.sqrt(d)))
    announce("exact mll", m, d)
    val, grad = api.gp_exact_mll(ctx, dev(X), dev(y), theta)
    X64, y64 = X.astype(np.float64), y.astype(np.float64)
    ref = mll.log_marginal_likelihood(X64, y64, theta)
    gref = mll.mll_grad_exact(X64, y64, theta)
    assert val == pytest.approx(ref, rel=MLL_RTOL)
    assert _relerr(grad, gref) <= GRAD_RTOL


def test_exact_mll_on_index_subset(ctx):
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w, n=20_000)
    y = _targets(X, 5)
    Xd, yd = dev(X), dev(y)
    theta = np.array([0.1, 0.15, 0.08, 1.0, 0.05])
    idx = api.gp_nearest(ctx, Xd, 123, 900)
    announce("exact mll subset", 900)
    val, grad = api.gp_exact_mll(ctx, Xd, yd, theta, idx=idx)
    sel = idx.cpu().numpy()
    X64, y64 = X[sel].astype(np.float64), y[sel].astype(np.float64)
    assert val == pytest.approx(mll.log_marginal_likelihood(X64, y64, theta), rel=MLL_RTOL)
    assert _relerr(grad, mll.mll_grad_exact(X64, y64, theta)) <= GRAD_RTOL
    # the first m rows without an index list
    val2, _ = api.gp_exact_mll(ctx, Xd, yd, theta, m=300)
    ref2 = mll.log_marginal_likelihood(X[:300].astype(np.float64), y[:300].astype(np.float64),
                                       theta)
    assert val2 == pytest.approx(ref2, rel=MLL_RTOL)


def test_exact_mll_oracle_at_4096(ctx):
    w = wl.WORKLOADS["C"]
    X = wl.draw_inputs(w, n=4096)
    y = _targets(X, 6, noise=0.3)
    theta = _theta(w.d, 8, ell=(1.0, 3.0))
    announce("exact mll 4096")
    val, grad = api.gp_exact_mll(ctx, dev(X), dev(y), theta)
    X64, y64 = X.astype(np.float64), y.astype(np.float64)
    assert val == pytest.approx(mll.log_marginal_likelihood(X64, y64, theta), rel=MLL_RTOL)
    assert _relerr(grad, mll.mll_grad_exact(X64, y64, theta)) <= GRAD_RTOL


def test_exact_mll_full_subset_central_differences(ctx):
    # The paper's subset size: the gradient against central differences of the
    # returned likelihood (a property that holds at any size).
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w)
    y = _targets(X, 7, noise=0.05)
    Xd, yd = dev(X), dev(y)
    idx = api.gp_nearest(ctx, Xd, int(wl.draw_centroids(w)[0]), 10_000)
    theta = np.array([0.12, 0.1, 0.15, 1.0, 0.1])
    announce("exact mll 10000")
    val, grad = api.gp_exact_mll(ctx, Xd, yd, theta, idx=idx)
    assert np.isfinite(val) and np.all(np.isfinite(grad))
    for k in range(len(theta)):
        h = 1e-5 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fp, _ = api.gp_exact_mll(ctx, Xd, yd, tp, idx=idx)
        fm, _ = api.gp_exact_mll(ctx, Xd, yd, tm, idx=idx)
        fd = (fp - fm) / (2 * h)
        assert grad[k] == pytest.approx(fd, rel=1e-5, abs=1e-4 * np.abs(grad).max()), k


def test_exact_mll_errors(ctx):
    X = dev(np.zeros((10, 2), np.float32))
    y = dev(np.zeros(10, np.float32))
    theta = np.ones(4)
    bad_idx = dev(np.array([0, 3, 10], np.int64))
    for kw in (dict(m=11), dict(m=0), dict(idx=bad_idx)):
        with pytest.raises(api.GPError) as e:
            api.gp_exact_mll(ctx, X, y, theta, **kw)
        assert e.value.code == api.N.GP_ERR_INVALID_ARG, kw
    with pytest.raises(api.GPError):
        api.gp_exact_mll(ctx, X, y, np.array([1.0, -1.0, 1.0, 1.0]))


# ------------------------------------------------------------------ heuristic

def test_init_heuristic_matches_oracle(ctx):
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w, n=3000)
    y = _targets(X * 6.0, 9, noise=0.05)
    centres = wl.draw_centroids(w, count=3, n=3000)
    announce("init heuristic", centres.tolist())
    mean, each = api.gp_init_heuristic(ctx, dev(X), dev(y), centres, m=256, steps=15, lr=0.1)
    rmean, reach = ih.init_heuristic(X, y, centres, m=256, steps=15, lr=0.1)
    np.testing.assert_allclose(each, reach, rtol=1e-7)
    np.testing.assert_allclose(mean, rmean, rtol=1e-7)


def test_init_heuristic_theta0_log_transform_and_errors(ctx):
    w = wl.WORKLOADS["C"]
    X = wl.draw_inputs(w, n=1000)
    y = _targets(X, 10, noise=0.3)
    theta0 = np.concatenate([np.full(w.d, 2.0), [0.8, 0.4]])
    announce("init heuristic log")
    mean, each = api.gp_init_heuristic(ctx, dev(X), dev(y), [5], m=150, steps=8, lr=0.05,
                                       transform=api.GP_LOG, theta0=theta0)
    ref = ih.maximise_exact_mll(X[ih.nearest(X, 5, 150)], y[ih.nearest(X, 5, 150)], theta0,
                                steps=8, lr=0.05, transform="log")
    np.testing.assert_allclose(each[0], ref, rtol=1e-7)
    np.testing.assert_allclose(mean, ref, rtol=1e-7)
    Xd, yd = dev(X), dev(y)
    for kw in (dict(centres=[1000], m=10), dict(centres=[], m=10), dict(centres=[0], m=1001),
               dict(centres=[0], m=10, lr=0.0), dict(centres=[0], m=10, steps=-1)):
        with pytest.raises(api.GPError):
            api.gp_init_heuristic(ctx, Xd, yd, **kw)


def test_init_heuristic_more_centres_than_concurrent_lanes(ctx):
    # 18 centroid rows: the library runs at most 16 subsets concurrently, so this
    # takes two groups; every per-centroid result must still match the oracle.
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w, n=2000)
    y = _targets(X * 6.0, 11, noise=0.05)
    centres = wl.draw_centroids(w, count=18, n=2000)
    announce("init heuristic 18 centres")
    mean, each = api.gp_init_heuristic(ctx, dev(X), dev(y), centres, m=100, steps=4, lr=0.1)
    rmean, reach = ih.init_heuristic(X, y, centres, m=100, steps=4, lr=0.1)
    np.testing.assert_allclose(each, reach, rtol=1e-7)
    np.testing.assert_allclose(mean, rmean, rtol=1e-7)
