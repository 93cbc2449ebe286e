"""Thin Python binding of the C ABI (include/gp.h).

Functions carry the C names and only marshal arguments: device tensors are
passed as raw pointers with their leading dimension, theta as a host float64
array.  PyTorch provides device memory and the stream; every numerical step
runs in libgpmi.so.  A missing library raises ImportError from ``_native.lib``.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from ._native import (GP_ADJ_FUSED, GP_ADJ_PER_PARAM, GP_AP, GP_BF16, GP_BF16X3, GP_CG,  # noqa: F401
                      GP_FP32, GP_LOG, GP_PATHWISE, GP_SGD, GP_SOFTPLUS, GP_STANDARD,
                      GP_WS_KMATVEC, GP_WS_MLL_GRAD, GP_WS_SOLVE, InitCfg, SolveStats, SolverCfg)


class GPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{N.STATUS_NAMES.get(code, code)}] {msg}")
        self.code = code


class Context:
    """A gp_ctx bound to one device and torch's current stream on it."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        L = N.lib()
        self.device = device
        st = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = st
        h = C.c_void_p()
        rc = L.gp_ctx_create(device, C.c_void_p(st.cuda_stream), C.byref(h))
        if rc != N.GP_OK:
            raise GPError(rc, "gp_ctx_create failed")
        self._h = h

    @property
    def handle(self):
        return self._h

    def check(self, rc):
        if rc != N.GP_OK:
            raise GPError(rc, N.lib().gp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            N.lib().gp_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, on=True):
        self.check(N.lib().gp_profile_enable(self._h, int(on)))

    def profile_read(self, which=0):
        ms = C.c_double()
        cnt = C.c_int64()
        self.check(N.lib().gp_profile_read(self._h, which, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value


def _dptr(t: torch.Tensor | None, name: str, cols: int | None = None):
    if t is None:
        return None, 0
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 and t.dtype != torch.int32:
        raise ValueError(f"{name} must be float32")
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError(f"{name} must be contiguous")
        return C.c_void_p(t.data_ptr()), 1
    if t.dim() != 2 or (t.stride(1) != 1 and t.shape[1] > 1):
        raise ValueError(f"{name} must be a row-major 2-D tensor with unit column stride")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)
    return C.c_void_p(t.data_ptr()), max(ld, t.shape[1])


def _theta(theta):
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    return th, th.ctypes.data_as(C.POINTER(C.c_double))


def _rows(t):
    return 0 if t is None else t.shape[0]


def _cols(t):
    return 1 if t.dim() == 1 else t.shape[1]


def solver_cfg(solver=GP_CG, tol=0.01, max_epochs=0.0, precision=GP_FP32, refine_every=0,
               check_every=0, ap_block=1000, sgd_batch=500, sgd_lr=10.0, sgd_momentum=0.9,
               sgd_batches: np.ndarray | None = None, sgd_seed=0, precond_rank=0,
               use_graph=False, precond_reuse=0) -> SolverCfg:
    cfg = SolverCfg()
    N.lib().gp_solver_cfg_default(C.byref(cfg))
    cfg.solver, cfg.tol, cfg.max_epochs = solver, tol, max_epochs
    cfg.precision, cfg.refine_every, cfg.check_every = precision, refine_every, check_every
    cfg.ap_block, cfg.sgd_batch, cfg.sgd_lr, cfg.sgd_momentum = ap_block, sgd_batch, sgd_lr, sgd_momentum
    cfg.sgd_seed = sgd_seed
    cfg.precond_rank = precond_rank
    cfg.use_graph = int(use_graph)
    cfg.precond_reuse = int(precond_reuse)
    if sgd_batches is not None:
        arr = np.ascontiguousarray(sgd_batches, dtype=np.int32)
        cfg._batches_keepalive = arr
        cfg.sgd_batches = arr.ctypes.data_as(C.POINTER(C.c_int32))
        cfg.sgd_batches_count = arr.shape[0]
    return cfg


def gp_kmatvec(ctx: Context, X1, X2, theta, V, precision=GP_FP32, add_noise=False, out=None,
               _entry="gp_kmatvec"):
    n1, d = X1.shape
    n2 = X2.shape[0]
    c = _cols(V)
    if out is None:
        out = torch.empty((n1, c), device=V.device, dtype=torch.float32)
    th, thp = _theta(theta)
    x1, _ = _dptr(X1, "X1")
    x2, _ = _dptr(X2, "X2")
    v, ldv = _dptr(V, "V")
    o, ldo = _dptr(out, "out")
    ctx.check(getattr(N.lib(), _entry)(ctx.handle, x1, n1, x2, n2, d, thp, v, ldv, c, o, ldo,
                                       precision, int(add_noise)))
    return out


def gp_kmatvec_static(ctx: Context, X1, X2, theta, V, precision=GP_FP32, add_noise=False,
                      out=None):
    """gp_kmatvec through the allocation-free entry point (static device scratch)."""
    return gp_kmatvec(ctx, X1, X2, theta, V, precision, add_noise, out, _entry="gp_kmatvec_static")


def gp_kmatvec_adjoint(ctx: Context, X, theta, U, W, weights, precision=GP_BF16X3,
                       mode=GP_ADJ_FUSED):
    n, d = X.shape
    c = _cols(U)
    th, thp = _theta(theta)
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    grad = np.zeros(d + 2)
    x, _ = _dptr(X, "X")
    u, ldu = _dptr(U, "U")
    ww, ldw = _dptr(W, "W")
    ctx.check(N.lib().gp_kmatvec_adjoint(ctx.handle, x, n, d, thp, u, ldu, ww, ldw, c,
                                         w.ctypes.data_as(C.POINTER(C.c_double)), precision, mode,
                                         grad.ctypes.data_as(C.POINTER(C.c_double))))
    return grad


def gp_solve(ctx: Context, X, theta, B, U, cfg: SolverCfg):
    """Solve H U = B in place of U (U holds the initial value)."""
    n, d = X.shape
    c = _cols(B)
    th, thp = _theta(theta)
    st = SolveStats()
    x, _ = _dptr(X, "X")
    b, ldb = _dptr(B, "B")
    u, ldu = _dptr(U, "U")
    ctx.check(N.lib().gp_solve(ctx.handle, x, n, d, thp, b, ldb, u, ldu, c, C.byref(cfg),
                               C.byref(st)))
    return st.as_dict()


def gp_pivoted_cholesky(ctx: Context, X, theta, k):
    """Rank-k pivoted Cholesky of K(X, X): returns (L [rank, n] float64, the factor
    stored transposed, and the pivots [rank] int32) as device tensors."""
    n, d = X.shape
    th, thp = _theta(theta)
    L = torch.zeros((max(k, 1), max(n, 1)), device=X.device, dtype=torch.float64)
    piv = torch.zeros(max(k, 1), device=X.device, dtype=torch.int32)
    rank = C.c_int(0)
    x, _ = _dptr(X, "X")
    ctx.check(N.lib().gp_pivoted_cholesky(ctx.handle, x, n, d, thp, k, L.data_ptr(), max(n, 1),
                                          piv.data_ptr(), C.byref(rank)))
    return L[:rank.value], piv[:rank.value]


def gp_prior_sample(ctx: Context, Xq, theta, t, W, out=None):
    m, d = Xq.shape
    M = t.shape[0]
    s = _cols(W)
    if out is None:
        out = torch.empty((m, s), device=Xq.device, dtype=torch.float32)
    th, thp = _theta(theta)
    xq, _ = _dptr(Xq, "Xq")
    tt, _ = _dptr(t, "t")
    w, ldw = _dptr(W, "W")
    f, ldf = _dptr(out, "F")
    ctx.check(N.lib().gp_prior_sample(ctx.handle, xq, m, d, thp, tt, M, w, ldw, s, f, ldf))
    return out


def gp_posterior_sample(ctx: Context, Xq, X, theta, t, W, U, precision=GP_BF16X3, out=None):
    """Pathwise posterior samples at Xq from the pathwise solutions U = [v_y, zhat_1..zhat_s]
    and the random features (t, W) of the prior draws: returns F [m, s]."""
    m, d = Xq.shape
    n = X.shape[0]
    M = t.shape[0]
    s = _cols(U) - 1
    if out is None:
        out = torch.empty((m, s), device=Xq.device, dtype=torch.float32)
    th, thp = _theta(theta)
    xq, _ = _dptr(Xq, "Xq")
    x, _ = _dptr(X, "X")
    tt, _ = _dptr(t, "t")
    w, ldw = _dptr(W, "W")
    u, ldu = _dptr(U, "U")
    f, ldf = _dptr(out, "out")
    ctx.check(N.lib().gp_posterior_sample(ctx.handle, xq, m, x, n, d, thp, tt, M, w, ldw, u, ldu,
                                          s, precision, f, ldf))
    return out


def gp_mll_grad(ctx: Context, X, y, theta, estimator, U, cfg: SolverCfg, Z=None, rff_t=None,
                rff_W=None, w_eps=None, adjoint_mode=GP_ADJ_FUSED):
    """Returns (grad_theta [d+2], stats); U [n, s+1] is the warm-start / solution buffer."""
    n, d = X.shape
    s = _cols(U) - 1
    th, thp = _theta(theta)
    grad = np.zeros(d + 2)
    st = SolveStats()
    x, _ = _dptr(X, "X")
    yy, _ = _dptr(y, "y")
    z, ldz = _dptr(Z, "Z")
    tt, _ = _dptr(rff_t, "rff_t")
    w, ldw = _dptr(rff_W, "rff_W")
    e, lde = _dptr(w_eps, "w_eps")
    u, ldu = _dptr(U, "U")
    M = 0 if rff_t is None else rff_t.shape[0]
    ctx.check(N.lib().gp_mll_grad(ctx.handle, x, n, d, yy, thp, estimator, s, z, ldz, tt, M, w,
                                  ldw, e, lde, u, ldu, C.byref(cfg), adjoint_mode,
                                  grad.ctypes.data_as(C.POINTER(C.c_double)), C.byref(st)))
    return grad, st.as_dict()


def _xdev(X):
    if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous [n, d] float32 device tensor")
    return X.shape[0], X.shape[1]


def gp_nearest(ctx: Context, X, centre, k):
    """The k rows of X nearest to row ``centre`` (ascending row order, int64 device tensor)."""
    n, d = _xdev(X)
    idx = torch.empty(max(int(k), 1), device=X.device, dtype=torch.int64)
    ctx.check(N.lib().gp_nearest(ctx.handle, C.c_void_p(X.data_ptr()), n, d, int(centre), int(k),
                                 C.c_void_p(idx.data_ptr())))
    return idx[:int(k)]


def gp_exact_mll(ctx: Context, X, y, theta, idx=None, m=None):
    """Exact log marginal likelihood and gradient on rows idx of (X, y) (all rows, or the
    first m, when idx is None): returns (mll, grad [d+2])."""
    n, d = _xdev(X)
    if y.dtype != torch.float32 or not y.is_cuda or not y.is_contiguous():
        raise ValueError("y must be a contiguous float32 device tensor")
    ip = None
    if idx is not None:
        if idx.dtype != torch.int64 or not idx.is_cuda or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 device tensor")
        ip = C.c_void_p(idx.data_ptr())
        m = idx.shape[0]
    elif m is None:
        m = n
    th, thp = _theta(theta)
    out = C.c_double(0.0)
    grad = np.zeros(d + 2)
    ctx.check(N.lib().gp_exact_mll(ctx.handle, C.c_void_p(X.data_ptr()), n, d,
                                   C.c_void_p(y.data_ptr()), ip, int(m), thp, C.byref(out),
                                   grad.ctypes.data_as(C.POINTER(C.c_double))))
    return out.value, grad


def gp_init_heuristic(ctx: Context, X, y, centres, m, steps=100, lr=0.1, transform=GP_SOFTPLUS,
                      theta0=None):
    """Initial hyperparameters from the exact likelihood on the m rows nearest to each
    centroid row: returns (mean theta [d+2], per-centroid theta [nc, d+2])."""
    n, d = _xdev(X)
    if y.dtype != torch.float32 or not y.is_cuda or not y.is_contiguous():
        raise ValueError("y must be a contiguous float32 device tensor")
    cen = np.ascontiguousarray(np.asarray(centres, dtype=np.int64))
    cfg = InitCfg()
    N.lib().gp_init_cfg_default(C.byref(cfg))
    cfg.steps, cfg.lr, cfg.transform = int(steps), float(lr), int(transform)
    t0 = None
    if theta0 is not None:
        t0 = np.ascontiguousarray(np.asarray(theta0, dtype=np.float64))
        cfg.theta0 = t0.ctypes.data_as(C.POINTER(C.c_double))
    out = np.zeros(d + 2)
    each = np.zeros((cen.size, d + 2))
    pd = C.POINTER(C.c_double)
    ctx.check(N.lib().gp_init_heuristic(ctx.handle, C.c_void_p(X.data_ptr()), n, d,
                                        C.c_void_p(y.data_ptr()),
                                        cen.ctypes.data_as(C.POINTER(C.c_int64)), cen.size, int(m),
                                        C.byref(cfg), out.ctypes.data_as(pd),
                                        each.ctypes.data_as(pd)))
    return out, each


def gp_nu_to_theta(nu, transform=GP_SOFTPLUS):
    nu = np.ascontiguousarray(np.asarray(nu, dtype=np.float64))
    th = np.zeros_like(nu)
    pd = C.POINTER(C.c_double)
    rc = N.lib().gp_nu_to_theta(nu.size, nu.ctypes.data_as(pd), transform, th.ctypes.data_as(pd))
    if rc != N.GP_OK:
        raise GPError(rc, "gp_nu_to_theta")
    return th


def gp_workspace_size(op, n, d, c, cfg: SolverCfg | None = None, M=0):
    """Device bytes a context holds after one call of op (N.GP_WS_*) of this size."""
    out = C.c_size_t()
    rc = N.lib().gp_workspace_size(op, n, d, c, C.byref(cfg) if cfg is not None else None, M,
                                   C.byref(out))
    if rc != N.GP_OK:
        raise GPError(rc, "gp_workspace_size")
    return out.value


def gp_workspace_reserve(ctx: Context, op, n, d, c, cfg: SolverCfg | None = None, M=0):
    ctx.check(N.lib().gp_workspace_reserve(ctx.handle, op, n, d, c,
                                           C.byref(cfg) if cfg is not None else None, M))


def gp_workspace_held(ctx: Context):
    out = C.c_size_t()
    ctx.check(N.lib().gp_workspace_held(ctx.handle, C.byref(out)))
    return out.value


def gp_theta_to_nu(theta, transform=GP_SOFTPLUS):
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    nu = np.zeros_like(th)
    pd = C.POINTER(C.c_double)
    rc = N.lib().gp_theta_to_nu(th.size, th.ctypes.data_as(pd), transform, nu.ctypes.data_as(pd))
    if rc != N.GP_OK:
        raise GPError(rc, "gp_theta_to_nu")
    return nu


def gp_adam_ascent(state: dict, grad_theta, lr, transform=GP_SOFTPLUS):
    """In-place Adam ascent on state['nu'] (state holds nu, m, v float64 arrays and 'step')."""
    pd = C.POINTER(C.c_double)
    g = np.ascontiguousarray(np.asarray(grad_theta, dtype=np.float64))
    step = C.c_int64(state["step"])
    rc = N.lib().gp_adam_ascent(g.size, state["nu"].ctypes.data_as(pd), state["m"].ctypes.data_as(pd),
                                state["v"].ctypes.data_as(pd), C.byref(step), g.ctypes.data_as(pd),
                                lr, transform)
    if rc != N.GP_OK:
        raise GPError(rc, "gp_adam_ascent")
    state["step"] = step.value
    return state


class KMatvec(torch.autograd.Function):
    """H V with a hand-written backward: dV = H grad_out (H symmetric) and
    dtheta_k = sum_c grad_out_c^T (dH/dtheta_k) V_c via the fused adjoint kernel
    (kernel tiles recomputed, never stored).  theta: CPU float64 tensor [d+2]."""

    @staticmethod
    def forward(fctx, X, theta, V, gp: Context, precision=GP_FP32):
        th = theta.detach().cpu().numpy()
        out = gp_kmatvec(gp, X, X, th, V, precision, add_noise=True)
        fctx.save_for_backward(X, V)
        fctx.theta = th
        fctx.gp = gp
        fctx.precision = precision
        return out

    @staticmethod
    def backward(fctx, grad_out):
        X, V = fctx.saved_tensors
        g = grad_out.contiguous()
        dV = gp_kmatvec(fctx.gp, X, X, fctx.theta, g, fctx.precision, add_noise=True)
        adj_prec = GP_FP32 if fctx.precision == GP_FP32 else GP_BF16X3
        dth = gp_kmatvec_adjoint(fctx.gp, X, fctx.theta, g, V.contiguous(), np.ones(V.shape[1]),
                                 adj_prec)
        return None, torch.from_numpy(dth), dV, None, None


class Trainer:
    """Outer loop of Sec. 2 ("Hierarchical View"): Adam on nu, theta = softplus(nu)
    (or exp), gradient from gp_mll_grad with a warm-started solution buffer."""

    def __init__(self, ctx: Context, X, y, theta0, estimator, cfg: SolverCfg, lr, s,
                 transform=GP_SOFTPLUS, warm=True, Z=None, rff_t=None, rff_W=None, w_eps=None,
                 adjoint_mode=GP_ADJ_FUSED):
        self.ctx, self.X, self.y = ctx, X, y
        self.estimator, self.cfg, self.lr, self.transform = estimator, cfg, lr, transform
        self.warm, self.adjoint_mode = warm, adjoint_mode
        self.Z, self.rff_t, self.rff_W, self.w_eps = Z, rff_t, rff_W, w_eps
        nu0 = gp_theta_to_nu(theta0, transform)
        self.state = {"nu": nu0.copy(), "m": np.zeros_like(nu0), "v": np.zeros_like(nu0), "step": 0}
        self.U = torch.zeros((X.shape[0], s + 1), device=X.device, dtype=torch.float32)
        self.history = []

    @property
    def theta(self):
        return gp_nu_to_theta(self.state["nu"], self.transform)

    def step(self):
        theta = self.theta
        if not self.warm:
            self.U.zero_()
        grad, stats = gp_mll_grad(self.ctx, self.X, self.y, theta, self.estimator, self.U, self.cfg,
                                  Z=self.Z, rff_t=self.rff_t, rff_W=self.rff_W, w_eps=self.w_eps,
                                  adjoint_mode=self.adjoint_mode)
        gp_adam_ascent(self.state, grad, self.lr, self.transform)
        self.history.append({"theta": theta, "grad": grad, "stats": stats})
        return theta, grad, stats
