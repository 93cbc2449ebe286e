"""CPU measurements behind floating-point tolerances of the GPU parity tests: how
far the oracle's own results move under perturbations of the size that the
reduced-precision products introduce."""
import numpy as np

from gpu_common import problem
from oracle import precond, solvers


class _Dense:
    def __init__(self, H):
        self.H = H

    def matvec(self, V):
        return self.H @ V


def _perturbed(H, eps, seed):
    """H with every entry scaled by (1 + eps u), u ~ U[-1, 1], kept symmetric."""
    g = np.random.default_rng(seed)
    E = g.uniform(-1.0, 1.0, H.shape)
    E = np.triu(E) + np.triu(E, 1).T
    return H * (1.0 + eps * E)


def _moved(n, k, seed, eps):
    # the inputs of test_pcg_steps_match_oracle_under_a_budget
    X, B, theta = problem(n, 3, 9, seed=seed, dist="uniform", sigma=0.05, ell_scale=(0.2, 0.5))
    op = solvers.DenseOperator(X, theta)
    P = precond.preconditioner(X, theta, k)
    U0, _ = solvers.cg(op, B, tol=1e-8, max_epochs=4, precond=P)
    U1, _ = solvers.cg(_Dense(_perturbed(op.H, eps, 1)), B, tol=1e-8, max_epochs=4, precond=P)
    return float(np.abs(U1 - U0).max() / np.abs(U0).max())


def test_four_pcg_steps_amplify_kernel_entry_errors():
    # bf16x3 products drop terms of relative size 2^-16 per kernel entry.  After
    # four preconditioned steps the rank-60 case moves by far less than the
    # strict bound (2e-4 of max|U|), the rank-1000 case by more than it but
    # within the 5e-3 that its bf16x3 comparison allows.
    eps = 2.0 ** -16
    small = _moved(900, 60, 31, eps)
    large = _moved(4000, 1000, 57, eps)
    assert small < 2e-4, small
    assert 2e-4 < large < 5e-3, large


def test_budgeted_cg_steps_are_insensitive_to_kernel_entry_errors():
    # the inputs of test_cg_budget_warm_start_and_scaling: three unpreconditioned
    # CG steps move by about 0.41 eps of max|U|, so the 2e-4 bound of that test
    # holds with a wide margin even at a 2^-16 error per kernel entry
    X, B, theta = problem(900, 3, 9, seed=3, dist="uniform", sigma=0.05, ell_scale=(0.2, 0.5))
    op = solvers.DenseOperator(X, theta)
    U0, _ = solvers.cg(op, B, tol=1e-6, max_epochs=3)
    U1, _ = solvers.cg(_Dense(_perturbed(op.H, 2.0 ** -16, 1)), B, tol=1e-6, max_epochs=3)
    moved = float(np.abs(U1 - U0).max() / np.abs(U0).max())
    assert moved < 2e-4 / 10, moved
