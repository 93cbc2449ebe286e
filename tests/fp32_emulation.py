"""CPU emulations of the GPU path's arithmetic, used to derive test tolerances.

These are measurement tools of the tests, not a second implementation of the
method: they run the conjugate-gradient recurrence of App. B (Algorithm 1,
no preconditioner) with FP32 vectors and FP64 scalars and dot products -- the
split the library uses -- on an operator whose entries carry relative
perturbations of the size a product precision introduces, so that a test can
see how far rounding alone moves the quantities it compares (iteration
counts, attainable residuals).  The operator is the dense FP64 matrix H of the
oracle, perturbed entry by entry.
"""
import numpy as np

# relative error per kernel entry of one product: FP32 evaluation (sqrt, exp2,
# the squared distance) and FP32 accumulation, about 1e-6; bf16x3 drops the
# lo*lo term and rounds the lo parts, at most 2^-16 of the entry
ENTRY_EPS = {0: 2.0 ** -20, 1: 2.0 ** -16}


def perturbed(H, eps, seed):
    """H with every entry scaled by (1 + eps u), u ~ U[-1, 1], kept symmetric."""
    g = np.random.default_rng(seed)
    E = g.uniform(-1.0, 1.0, H.shape)
    E = np.triu(E) + np.triu(E, 1).T
    return H * (1.0 + eps * E)


def _f32_product(Hp, V):
    # FP32 operands and FP32 accumulation, as in the library's products
    return np.asarray(Hp, np.float32) @ np.asarray(V, np.float32)


def _norms(R):
    nrm = np.sqrt(np.sum(R.astype(np.float64) ** 2, axis=0))
    return float(nrm[0]), float(np.mean(nrm[1:])) if R.shape[1] > 1 else 0.0


def cg_fp32(H, Hp, B, tol, mixed, max_iter=100_000):
    """Iterations of CG with FP32 vectors and FP64 scalars on the perturbed
    operator Hp, stopped when both the mean and the probe relative residual are
    at most tol.  With `mixed`, a recurrence that claims convergence is checked
    on the true residual b - H u (H unperturbed, FP32 rounding) and restarted
    from it when that is still above tol; from the second such restart on the
    recurrence's target is halved at every restart, and when a restart with a
    lowered target gains less than 10 %
    on the true residual the iteration continues with the unperturbed operator
    (FP32 products), a second such stall ending the solve.  Returns (iterations,
    converged, whether the FP32 products took over)."""
    B64 = np.asarray(B, np.float64)
    scale = 1.0 / (np.sqrt(np.sum(B64 ** 2, axis=0)) + 1e-10)
    Bt = (B64 * scale).astype(np.float32)
    U = np.zeros_like(Bt)
    R = Bt - _f32_product(H, U)
    D = R.copy()
    gamma = np.sum(R.astype(np.float64) ** 2, axis=0)
    t = since_true = 0
    last_true = np.inf
    tol_in = tol
    failed = 0
    escalated = False
    while True:
        ry, rz = _norms(R)
        if since_true == 0 and t == 0:
            last_true = max(ry, rz)
        target = tol if since_true == 0 else tol_in
        go = ry > target or rz > target
        if not go and mixed and since_true > 0:
            R = Bt - _f32_product(H, U)
            D = R.copy()
            gamma = np.sum(R.astype(np.float64) ** 2, axis=0)
            since_true = 0
            ry, rz = _norms(R)
            go = ry > tol or rz > tol
            if go:
                now = max(ry, rz)
                failed += 1
                if failed >= 3 and now > 0.9 * last_true:
                    if escalated:
                        return t, False, True
                    escalated, Hp, failed, tol_in, last_true = True, H, 0, tol, now
                else:
                    last_true = now
                    if failed >= 2:
                        tol_in *= 0.5
        if not go or t >= max_iter:
            return t, not go, escalated
        HD = _f32_product(Hp, D)
        dhd = np.sum(D.astype(np.float64) * HD.astype(np.float64), axis=0)
        live = gamma > 0
        alpha = np.where(live, gamma / np.where(live, dhd, 1.0), 0.0)
        U = (U + (alpha * D).astype(np.float32)).astype(np.float32)
        R = (R - (alpha * HD).astype(np.float32)).astype(np.float32)
        gnew = np.sum(R.astype(np.float64) ** 2, axis=0)
        beta = np.where(live, gnew / np.where(live, gamma, 1.0), 0.0)
        gamma = gnew
        D = (R + (beta * D).astype(np.float32)).astype(np.float32)
        t += 1
        since_true += 1


def attainable_relres(H, B, eps, seeds=3):
    """Largest true relative residual ||b - H u|| / ||b|| (mean column, then the
    mean over the probe columns) of exact solves u = Hp^-1 b with operators Hp
    whose entries carry relative errors eps: the accuracy a solver using such
    products cannot improve on."""
    worst = np.zeros(2)
    B = np.asarray(B, np.float64)
    nb = np.linalg.norm(B, axis=0)
    for s in range(seeds):
        U = np.linalg.solve(perturbed(H, eps, s), B)
        rel = np.linalg.norm(B - H @ U, axis=0) / nb
        worst = np.maximum(worst, [rel[0], rel[1:].mean()])
    return worst


def iteration_band(H, B, tol, prec, seeds=3):
    """Iteration counts of cg_fp32 over several equally valid rounding patterns
    of the given product precision, widened by max(2, 10 %) on both sides."""
    H32 = np.asarray(H, np.float32)
    its = [cg_fp32(H32, perturbed(H, ENTRY_EPS[prec], s), B, tol, mixed=prec != 0)[0]
           for s in range(seeds)]
    lo, hi = min(its), max(its)
    return its, lo - max(2, 0.1 * lo), hi + max(2, 0.1 * hi)


def bf16_rne(a):
    """Round float32 values to bf16 (to nearest, ties to even); returned as float32."""
    b = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def bf16x3_parts(v):
    """The library's bf16 hi/lo split of FP32 values: hi = bf16(v), lo = bf16(v - hi)."""
    v = np.asarray(v, np.float32)
    hi = bf16_rne(v)
    lo = bf16_rne((v - hi).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


def bf16x3_outer(A, B):
    """A B^T as three bf16 products hi*hi + hi*lo + lo*hi of the split operands,
    accumulated exactly (FP64): the arithmetic of a bf16x3 matrix-core product."""
    ah, al = bf16x3_parts(A)
    bh, bl = bf16x3_parts(B)
    return ah @ bh.T + ah @ bl.T + al @ bh.T
