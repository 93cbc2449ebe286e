"""One marginal-likelihood optimisation step, composed from the pinned oracle parts.

The three-level hierarchy of Sec. 2 ("Hierarchical View"): the outer Adam
optimiser asks a gradient estimator (standard or pathwise) for an estimate
of dL/dtheta, which needs the solution of one batched linear system from an
inner solver (exact Cholesky, CG, AP or SGD).  Warm start (Sec. 4) passes the
previous step's solution as the solver's initial value and keeps the
right-hand-side draws fixed (App. B).
"""
from __future__ import annotations

import numpy as np

from . import kernel, mll, optim, rff, solvers


def build_rhs(X, y, theta, estimator, draws):
    """B = [y, z_1..z_s] (standard) or [y, xi_1..xi_s] (pathwise)."""
    if estimator == "standard":
        Z = np.asarray(draws["Z"], np.float64)
        return np.concatenate([np.asarray(y, np.float64)[:, None], Z], axis=1)
    return rff.pathwise_rhs(X, y, theta, draws["t"], draws["W"], draws["w_eps"])


def solve(X, theta, B, solver, U0=None, tol=0.01, max_epochs=None, dense=True, **kw):
    if solver == "exact":
        return mll.exact_solve(X, theta, B), dict(iterations=0, converged=True)
    op = solvers.DenseOperator(X, theta) if dense else solvers.MatrixFreeOperator(X, theta)
    if solver == "cg":
        return solvers.cg(op, B, tol, max_epochs, U0)
    if solver == "ap":
        return solvers.ap(op, B, kw.get("block", 1000), tol, max_epochs, U0)
    if solver == "sgd":
        return solvers.sgd(op, B, kw["batches"], kw["lr"], kw.get("momentum", 0.9), tol,
                           max_epochs, U0)
    raise ValueError(solver)


def gradient(X, theta, U, B, estimator):
    s = B.shape[1] - 1
    W = np.concatenate([U[:, :1], B[:, 1:]], axis=1) if estimator == "standard" else U
    return kernel.adjoint(X, theta, U, W, mll.estimator_weights(s))


class Trainer:
    """Adam on nu with theta = transform(nu); one ``step()`` = one gradient step."""

    def __init__(self, X, y, theta0, estimator, draws, lr, transform="softplus",
                 solver="exact", warm=True, tol=0.01, max_epochs=None, dense=True, **solver_kw):
        self.X = np.asarray(X, np.float64)
        self.y = np.asarray(y, np.float64)
        self.nu = optim.to_nu(theta0, transform)
        self.transform = transform
        self.adam = optim.Adam(lr)
        self.estimator, self.draws = estimator, draws
        self.solver, self.warm, self.tol, self.max_epochs = solver, warm, tol, max_epochs
        self.dense, self.solver_kw = dense, solver_kw
        self.U = None
        self.history = []

    def step(self):
        theta = optim.to_theta(self.nu, self.transform)
        B = build_rhs(self.X, self.y, theta, self.estimator, self.draws)
        U0 = self.U if self.warm else None
        U, stats = solve(self.X, theta, B, self.solver, U0, self.tol, self.max_epochs,
                         self.dense, **self.solver_kw)
        self.U = U
        g_theta = gradient(self.X, theta, U, B, self.estimator)
        g_nu = g_theta * optim.dtheta_dnu(self.nu, self.transform)
        self.nu = self.adam.step(self.nu, g_nu)
        self.history.append(dict(theta=theta, grad=g_theta, stats=stats))
        return theta, g_theta, stats
