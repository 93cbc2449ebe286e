"""Writes config_b_exact_trajectory.json: 50 Adam steps of marginal-likelihood
optimisation on the 16,384-point workload (d = 24) with the pathwise estimator,
exact Cholesky solves (the oracle), softplus transform, lr 0.1, theta0 = 1 (the
paper's small-data settings, App. B "Iterative Optimiser").  Calls only oracle/ and
the seeded draws of workloads/; the GPU's trajectories are compared with it (Sec. 4,
Table 1 setting): with tight CG solves every nu within 0.05 (half an Adam step), with
CG, AP and SGD at tau = 1e-2 the signal and noise scales.

Usage: python tests/golden/make_config_b_trajectory.py [steps]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import rff, train  # noqa: E402


def targets(w):
    """float32 targets of the workload from its data-generating random-feature draw."""
    X = wl.draw_inputs(w)
    tr = wl.truth_draws(w)
    y = rff.truth_targets_rff(X, tr["ell"], 1.0, w.sigma, tr["t"], tr["w"], tr["noise"])
    return X, y.astype(np.float32)


def main(steps=50):
    w = wl.WORKLOADS["B"]
    X, y = targets(w)
    dr = wl.model_pathwise_draws(w)
    tr = train.Trainer(X, y, np.ones(w.d + 2), "pathwise", dr, lr=0.1, transform="softplus",
                       solver="exact")
    nus, thetas = [tr.nu.tolist()], []
    for k in range(steps):
        t0 = time.time()
        theta, _, _ = tr.step()
        thetas.append(theta.tolist())
        nus.append(tr.nu.tolist())
        print(f"step {k}: {time.time() - t0:.1f} s, theta[-2:] = {theta[-2:]}", flush=True)
    out = {"workload": "n=16384, d=24, x~N(0,I) standardised, RFF truth ell~U[0.3,3], sigma=0.2",
           "estimator": "pathwise", "solver": "exact (Cholesky)", "transform": "softplus",
           "lr": 0.1, "theta0": 1.0, "steps": steps, "s": w.s, "model_pairs": w.model_pairs,
           "nu": nus, "theta": thetas}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config_b_exact_trajectory.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 50)
