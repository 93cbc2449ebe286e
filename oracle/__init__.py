"""Plain FP64 CPU oracle for iterative-GP marginal-likelihood optimisation.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (``paper_2405_18457_amd``); the two meet only in the seeded random draws
of the ``workloads`` module.

Everything here is written from the paper (Lin et al., "Improving Linear
System Solvers for Hyperparameter Optimisation in Iterative Gaussian
Processes", NeurIPS 2024) in float64, slow and obvious:

  kernel   -- Matern-3/2 ARD kernel, regularised kernel matrix H = K + sigma^2 I
              (Sec. 2, "Gaussian Process Regression"; eq. for H_theta), its
              derivatives and the bilinear adjoint u^T (dH/dtheta) w.
  mll      -- log marginal likelihood and exact gradient (Sec. 2, eqs. mll /
              mll_grad); standard (Hutchinson) and pathwise estimators
              (Sec. 2 eq. trace, Sec. 3 eq. pathwise_estimator).
  rff      -- random Fourier feature prior samples, pathwise right-hand sides
              and posterior samples (Sec. 2 "Pathwise Conditioning", App. B
              "Kernel Function and Random Features").
  solvers  -- conjugate gradients, alternating projections, SGD (App. B,
              Algorithms 1-3) with the relative-residual stopping rule.
  precond  -- the rank-k pivoted Cholesky preconditioner of CG (App. B).
  optim    -- softplus / log reparameterisation and Adam (App. B "Iterative
              Optimiser").
  init_heuristic -- initial hyperparameters of the large data sets: nearest
              subsets around random centroids, exact-likelihood maximisation,
              centroid average (App. B "Iterative Optimiser").

Parity status: every function has at least one independent pin in
``tests/test_oracle_pins.py``, ``tests/test_oracle_precond.py`` or
``tests/test_oracle_init.py``; the alternating-projections block selection is
pinned as the literal reading of its printed score (a hand-computed case).
"""
from . import kernel, mll, rff, solvers, optim, train, precond, init_heuristic  # noqa: F401

__all__ = ["kernel", "mll", "rff", "solvers", "optim", "train", "precond", "init_heuristic"]
