"""Seeded synthetic inputs shared by the GPU path, the oracle, the tests and the bench.

This module only draws random numbers and holds workload shapes.  It contains
none of the method's arithmetic (no kernel, no random-feature map, no solver):
both the HIP path and the oracle turn these draws into kernel values, prior
samples and right-hand sides on their own.

Every stream is ``numpy.random.Generator(PCG64(1000 * cfg + stream))`` with
cfg = 0..4 for the five workloads below and these stream numbers:

  0 inputs X            1 true length scales     2 truth RFF frequencies
  3 truth RFF weights   4 observation noise      5 model probes Z / model RFF frequencies
  6 model RFF weights   7 noise base w_eps       8 SGD batch indices
  9 random hyperparameters (differentiation workload)
 10 centroid rows of the initial-hyperparameter heuristic

All arrays handed to a device are float32 (inputs are *defined* as their
float32 values; the oracle up-casts the very same numbers to float64).

Workloads (synthetic stand-ins for the UCI shapes the paper uses; its
datasets are not available, see the paper's appendix on datasets):

  A  n=2,000      d=8   x~N(0,I)            small plain method, s=16
  B  n=16,384     d=24  x~N(0,I) standardised  s=64
  C  n=45,730     d=9   x~N(0,I)            s=64, differentiation
  D  n=434,874    d=3   x~U[-1,1]^3         s=64, precision (3droad shape)
  E  n=2,049,280  d=11  x~N(0,I)            s=64, early-stop scale
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "rng", "draw_inputs", "draw_true_lengthscales",
    "draw_spectral_t3", "draw_normal", "draw_batch_indices", "draw_random_theta",
    "truth_draws", "model_pathwise_draws", "model_standard_probes", "draw_centroids",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int
    n: int
    d: int
    s: int                 # probe vectors / posterior samples
    x_dist: str            # "normal", "normal_std", "uniform"
    ell_range: tuple       # true length scales ~ U[lo, hi]
    sigma: float           # true noise scale
    truth: str             # "exact" (Cholesky draw) or "rff"
    truth_pairs: int = 1024   # sin/cos pairs of the data-generating RFF draw (2,048 features)
    model_pairs: int = 1000   # sin/cos pairs of the model's prior samples (2,000 features)


WORKLOADS = {
    "A": Workload("A", 0, 2_000, 8, 16, "normal", (0.5, 2.0), 0.1, "exact"),
    "B": Workload("B", 1, 16_384, 24, 64, "normal_std", (0.3, 3.0), 0.2, "rff"),
    "C": Workload("C", 2, 45_730, 9, 64, "normal", (0.3, 3.0), 0.3, "rff"),
    "D": Workload("D", 3, 434_874, 3, 64, "uniform", (0.05, 0.2), 0.05, "rff"),
    "E": Workload("E", 4, 2_049_280, 11, 64, "normal", (0.3, 3.0), 0.1, "rff"),
}


def rng(cfg_index: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * cfg_index + stream))


def draw_inputs(w: Workload, n: int | None = None) -> np.ndarray:
    """Inputs X [n, d] float32 with the workload's distribution."""
    n = w.n if n is None else n
    g = rng(w.index, 0)
    if w.x_dist == "uniform":
        x = g.uniform(-1.0, 1.0, size=(n, w.d))
    else:
        x = g.standard_normal(size=(n, w.d))
        if w.x_dist == "normal_std":
            x = (x - x.mean(axis=0)) / x.std(axis=0)
    return np.ascontiguousarray(x, dtype=np.float32)


def draw_true_lengthscales(w: Workload) -> np.ndarray:
    lo, hi = w.ell_range
    return rng(w.index, 1).uniform(lo, hi, size=w.d)


def draw_spectral_t3(g: np.random.Generator, m: int, d: int) -> np.ndarray:
    """[m, d] draws from the d-variate Student-t with 3 degrees of freedom.

    t = g * sqrt(3 / u) with g ~ N(0, I_d) and one u ~ chi^2_3 per row.  This
    is the spectral measure of the unit-length-scale Matern-3/2 kernel
    (Rasmussen & Williams 2006, sec. 4.2.1); dividing by the length scales
    happens in the method, not here.
    """
    gauss = g.standard_normal(size=(m, d))
    u = g.chisquare(3.0, size=(m, 1))
    return np.ascontiguousarray(gauss * np.sqrt(3.0 / u), dtype=np.float32)


def draw_normal(g: np.random.Generator, shape) -> np.ndarray:
    return np.ascontiguousarray(g.standard_normal(size=shape), dtype=np.float32)


def draw_batch_indices(w: Workload, iters: int, b: int, n: int | None = None) -> np.ndarray:
    """SGD batches: b indices without replacement per iteration, i.i.d. across iterations."""
    n = w.n if n is None else n
    g = rng(w.index, 8)
    out = np.empty((iters, b), dtype=np.int32)
    for t in range(iters):
        out[t] = g.choice(n, size=b, replace=False)
    return out


def draw_random_theta(w: Workload, count: int = 10) -> np.ndarray:
    """[count, d+2] hyperparameters (ell_1..ell_d, a, sigma): ell, a log-uniform on
    [0.3, 3], sigma log-uniform on [0.05, 1]."""
    g = rng(w.index, 9)
    ell_a = np.exp(g.uniform(np.log(0.3), np.log(3.0), size=(count, w.d + 1)))
    sig = np.exp(g.uniform(np.log(0.05), np.log(1.0), size=(count, 1)))
    return np.concatenate([ell_a, sig], axis=1)


def truth_draws(w: Workload, n: int | None = None) -> dict:
    """Raw draws defining the data-generating function and the noise.

    For truth == "rff": frequencies t [truth_pairs, d] and weights [2*truth_pairs];
    for truth == "exact": a standard normal vector [n] that the oracle maps
    through a Cholesky factor.  ``noise`` [n] is standard normal (scaled by the
    true sigma in the method).
    """
    n = w.n if n is None else n
    out = {"ell": draw_true_lengthscales(w), "a": 1.0, "sigma": w.sigma}
    if w.truth == "rff":
        out["t"] = draw_spectral_t3(rng(w.index, 2), w.truth_pairs, w.d)
        out["w"] = draw_normal(rng(w.index, 3), (2 * w.truth_pairs,))
    else:
        out["w"] = draw_normal(rng(w.index, 3), (n,))
    out["noise"] = draw_normal(rng(w.index, 4), (n,))
    return out


def model_pathwise_draws(w: Workload, n: int | None = None, s: int | None = None,
                         pairs: int | None = None) -> dict:
    """Fixed random-feature parameters for the pathwise estimator under warm start:
    base frequencies t [M, d], feature weights W [2M, s], noise base w_eps [n, s]."""
    n = w.n if n is None else n
    s = w.s if s is None else s
    M = w.model_pairs if pairs is None else pairs
    return {
        "t": draw_spectral_t3(rng(w.index, 5), M, w.d),
        "W": draw_normal(rng(w.index, 6), (2 * M, s)),
        "w_eps": draw_normal(rng(w.index, 7), (n, s)),
    }


def model_standard_probes(w: Workload, n: int | None = None, s: int | None = None) -> np.ndarray:
    """Gaussian probe vectors Z [n, s] for the standard (Hutchinson) estimator."""
    n = w.n if n is None else n
    s = w.s if s is None else s
    return draw_normal(rng(w.index, 5), (n, s))


def draw_centroids(w: Workload, count: int = 10, n: int | None = None) -> np.ndarray:
    """Centroid rows of the initial-hyperparameter heuristic: ``count`` indices drawn
    uniformly from [0, n), independently (int64)."""
    n = w.n if n is None else n
    return rng(w.index, 10).integers(0, n, size=count, dtype=np.int64)
