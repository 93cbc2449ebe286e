"""Parity of the fused kernel-matrix product (gp_kmatvec) with the FP64 oracle.

Tolerances:
  FP32    1e-5   per column, ||out_c - ref_c|| / ||ref_c||  (target for the FP32 product)
  BF16X3  2e-5   per column (bf16 hi/lo split of kernel values and V; ~2^-17 per entry)
  BF16    3e-3   whole product, ||out - ref||_F / ||ref||_F (one bf16 rounding of both)
"""
import numpy as np
import pytest

from gpu_common import announce, col_relerr, dev, host, problem, require_gpu
from oracle import kernel

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 2e-5, 2: 3e-3}


@pytest.fixture(scope="module")
def gp():
    require_gpu()
    from paper_2405_18457_amd import api
    ctx = api.Context(0)
    yield ctx
    ctx.close()


CASES = [
    # n, d, c, dist
    (1, 3, 1, "uniform"),
    (17, 1, 5, "normal"),
    (130, 3, 17, "uniform"),
    (257, 2, 65, "normal"),
    (1000, 8, 65, "normal"),
    (1000, 9, 33, "normal"),
    (1500, 11, 65, "normal"),
    (700, 24, 80, "normal"),
    (300, 33, 7, "normal"),
    (2100, 3, 65, "uniform"),
    (999, 4, 128, "normal"),
    (400, 3, 200, "normal"),
]


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("n,d,c,dist", CASES)
def test_square_h_matvec(gp, n, d, c, dist, prec):
    from paper_2405_18457_amd import api
    X, V, theta = problem(n, d, c, seed=n * 7 + d + c, dist=dist)
    announce("kmatvec", n, d, c, dist, prec)
    out = host(api.gp_kmatvec(gp, dev(X), dev(X), theta, dev(V), precision=prec, add_noise=True))
    ref = kernel.h_matvec(X, theta, V)
    if prec == 2:
        # single bf16 rounding: the bound is on the whole product (few-term
        # columns of tiny n do not average their rounding errors)
        err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    else:
        err = col_relerr(out, ref)
    assert err <= TOL[prec], err


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_rectangular_cross_product(gp, prec):
    from paper_2405_18457_amd import api
    X, V, theta = problem(900, 5, 20, seed=3)
    Q, _, _ = problem(333, 5, 1, seed=4)
    announce("kmatvec-rect", prec)
    out = host(api.gp_kmatvec(gp, dev(Q), dev(X), theta, dev(V), precision=prec))
    ref = kernel.k_matvec(Q, X, theta, V)
    assert col_relerr(out, ref) <= TOL[prec]


def test_leading_dimensions_and_column_subsets(gp):
    from paper_2405_18457_amd import api
    import torch
    X, V, theta = problem(500, 3, 40, seed=5)
    Vbig = dev(np.concatenate([V, np.full((500, 7), np.nan, np.float32)], axis=1))
    out = torch.full((500, 50), 123.0, device="cuda")
    announce("kmatvec-ld")
    api.gp_kmatvec(gp, dev(X), dev(X), theta, Vbig[:, :40], precision=0, add_noise=True,
                   out=out[:, :40])
    o = host(out)
    assert np.all(o[:, 40:] == 123.0)
    assert col_relerr(o[:, :40], kernel.h_matvec(X, theta, V)) <= 1e-5


def test_empty_and_invalid(gp):
    from paper_2405_18457_amd import api
    import torch
    X, V, theta = problem(10, 2, 3, seed=6)
    announce("kmatvec-edge")
    out = torch.full((10, 3), 5.0, device="cuda")
    api.gp_kmatvec(gp, dev(X), dev(X[:0]), theta, dev(V[:0]), out=out)
    assert np.all(host(out) == 0.0)
    with pytest.raises(api.GPError) as e:
        api.gp_kmatvec(gp, dev(X), dev(X), np.array([1.0, -1.0, 1.0, 1.0]), dev(V))
    assert e.value.code == 1
    with pytest.raises(api.GPError):
        api.gp_kmatvec(gp, dev(X), dev(X[:5]), theta, dev(V[:5]), add_noise=True)


def test_deterministic_repeat(gp):
    from paper_2405_18457_amd import api
    X, V, theta = problem(3000, 3, 65, seed=7, dist="uniform")
    announce("kmatvec-repeat")
    a = host(api.gp_kmatvec(gp, dev(X), dev(X), theta, dev(V), precision=1, add_noise=True))
    b = host(api.gp_kmatvec(gp, dev(X), dev(X), theta, dev(V), precision=1, add_noise=True))
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
def test_full_size_precision_workload_sampled_rows(gp, prec):
    """n = 434,874, d = 3 (the precision workload) in the launch configuration the
    bench times; 192 sampled output rows checked against FP64 row products."""
    import workloads as wl
    from paper_2405_18457_amd import api
    w = wl.WORKLOADS["D"]
    X = wl.draw_inputs(w)
    ell = wl.draw_true_lengthscales(w)
    theta = np.concatenate([ell, [1.0, w.sigma]])
    V = wl.draw_normal(np.random.default_rng(11), (w.n, 65))
    announce("kmatvec-full-D", prec)
    out = host(api.gp_kmatvec(gp, dev(X), dev(X), theta, dev(V), precision=prec, add_noise=True))
    rows = np.random.default_rng(12).choice(w.n, 192, replace=False)
    ref = kernel.k_matvec(X[rows], X, theta, V) + w.sigma ** 2 * V[rows].astype(np.float64)
    err = col_relerr(out[rows], ref)
    assert err <= TOL[prec], err


@pytest.mark.parametrize("prec", [1, 2], ids=["bf16x3", "bf16"])
@pytest.mark.parametrize("shift_rows,shift_cols", [(0.0, 0.0), (40.0, 40.0), (0.0, 40.0)])
def test_low_dimension_distance_forms(gp, prec, shift_rows, shift_cols):
    """For d <= 3 the bf16 products take squared distances from the norm expansion
    on the matrix cores when every scaled point has |x^|^2 <= 1024 and from direct
    differences otherwise; both forms meet the same bound."""
    from paper_2405_18457_amd import api
    X, V, theta = problem(1100, 3, 33, seed=77, dist="uniform", ell_scale=(0.15, 0.25))
    Q, _, _ = problem(413, 3, 1, seed=78, dist="uniform")
    # a few far-away points (their kernel values vanish) push the set's maximum norm
    # past the cross-term limit while the rest of the product stays non-trivial
    X[-50:] += np.float32(shift_cols)
    Q[-20:] += np.float32(shift_rows)
    scale = np.sqrt(3.0) / np.log(2.0) / theta[:3]
    for P, shift in ((Q, shift_rows), (X, shift_cols)):
        big = float(((P.astype(np.float64) * scale) ** 2).sum(1).max())
        assert (big > 1024.0) == (shift > 0.0), big
    announce("kmatvec-xt", prec, shift_rows, shift_cols)
    out = host(api.gp_kmatvec(gp, dev(Q), dev(X), theta, dev(V), precision=prec))
    ref = kernel.k_matvec(Q, X, theta, V)
    if prec == 2:
        err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    else:
        err = col_relerr(out, ref)
    assert err <= TOL[prec], err

@pytest.mark.parametrize("name,prec", [("B", 0), ("B", 1), ("C", 1), ("E", 1)],
                         ids=["B-fp32", "B-bf16x3", "C-bf16x3", "E-bf16x3"])
def test_full_size_workloads_sampled_rows(gp, name, prec):
    """The other workloads at full size and their data-generating hyperparameters
    (B: n = 16,384, d = 24; C: n = 45,730, d = 9; E: n = 2,049,280, d = 11), 65
    columns; sampled output rows against FP64 row products.  At B and E a few
    points exceed the bulk norm bound of the cross-term form (2 and 474 of them)."""
    import time

    import torch
    import workloads as wl
    from paper_2405_18457_amd import api
    w = wl.WORKLOADS[name]
    X = wl.draw_inputs(w)
    theta = np.concatenate([wl.draw_true_lengthscales(w), [1.0, w.sigma]])
    V = wl.draw_normal(np.random.default_rng(13), (w.n, 65))
    announce("kmatvec-full", name, prec)
    Xd, Vd = dev(X), dev(V)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out_d = api.gp_kmatvec(gp, Xd, Xd, theta, Vd, precision=prec, add_noise=True)
    torch.cuda.synchronize()
    print(f"[gpu-case] {name} product {1e3 * (time.perf_counter() - t0):.1f} ms", flush=True)
    rows = np.random.default_rng(14).choice(w.n, 96, replace=False)
    out = host(out_d[torch.from_numpy(rows).cuda()])
    ref = kernel.k_matvec(X[rows], X, theta, V) + w.sigma ** 2 * V[rows].astype(np.float64)
    err = col_relerr(out, ref)
    assert err <= TOL[prec], err
