"""ctypes declarations of the C ABI in ``include/gp.h`` (libgpmi.so, built for gfx950).

Loading fails loudly if the library has not been built: there is no CPU or
Python fallback for any operation.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgpmi.so")

GP_OK, GP_ERR_INVALID_ARG, GP_ERR_HIP, GP_ERR_NO_WORKSPACE, GP_ERR_NONFINITE, GP_ERR_BREAKDOWN = range(6)
GP_FP32, GP_BF16X3, GP_BF16 = 0, 1, 2
GP_CG, GP_AP, GP_SGD = 0, 1, 2
GP_STANDARD, GP_PATHWISE = 0, 1
GP_ADJ_FUSED, GP_ADJ_PER_PARAM = 0, 1
GP_SOFTPLUS, GP_LOG = 0, 1
GP_WS_KMATVEC, GP_WS_SOLVE, GP_WS_MLL_GRAD = 0, 1, 2

STATUS_NAMES = {
    GP_OK: "ok", GP_ERR_INVALID_ARG: "invalid_arg", GP_ERR_HIP: "hip",
    GP_ERR_NO_WORKSPACE: "no_workspace", GP_ERR_NONFINITE: "nonfinite",
    GP_ERR_BREAKDOWN: "breakdown",
}

# Every symbol include/gp.h declares.
EXPORTS = (
    "gp_ctx_create", "gp_ctx_destroy", "gp_last_error", "gp_version", "gp_profile_enable",
    "gp_profile_read", "gp_kmatvec", "gp_kmatvec_adjoint", "gp_solver_cfg_default", "gp_solve",
    "gp_prior_sample", "gp_mll_grad", "gp_adam_ascent", "gp_nu_to_theta", "gp_theta_to_nu", "gp_pivoted_cholesky",
    "gp_posterior_sample", "gp_nearest", "gp_exact_mll", "gp_init_cfg_default", "gp_init_heuristic",
    "gp_workspace_size", "gp_workspace_reserve", "gp_workspace_held", "gp_kmatvec_static",
)


class SolverCfg(C.Structure):
    _fields_ = [
        ("solver", C.c_int), ("tol", C.c_double), ("max_epochs", C.c_double),
        ("precision", C.c_int), ("refine_every", C.c_int), ("check_every", C.c_int),
        ("ap_block", C.c_int), ("sgd_batch", C.c_int), ("sgd_lr", C.c_double),
        ("sgd_momentum", C.c_double), ("sgd_batches", C.POINTER(C.c_int32)),
        ("sgd_batches_count", C.c_int64), ("sgd_seed", C.c_uint64), ("precond_rank", C.c_int),
        ("use_graph", C.c_int), ("precond_reuse", C.c_int),
    ]


class SolveStats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int64), ("epochs", C.c_double), ("matvecs", C.c_int64),
        ("refinements", C.c_int64), ("relres_y", C.c_double), ("relres_z", C.c_double),
        ("true_relres_y", C.c_double), ("true_relres_z", C.c_double), ("converged", C.c_int),
        ("status", C.c_int), ("precond_rank", C.c_int), ("fp32_iterations", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class InitCfg(C.Structure):
    _fields_ = [
        ("steps", C.c_int), ("lr", C.c_double), ("transform", C.c_int),
        ("theta0", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2405_18457_amd.build` "
                              "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
        pd = C.POINTER(C.c_double)
        pi64 = C.POINTER(C.c_int64)
        sig = {
            "gp_ctx_create": (i32, [i32, vp, C.POINTER(vp)]),
            "gp_ctx_destroy": (None, [vp]),
            "gp_last_error": (C.c_char_p, [vp]),
            "gp_version": (C.c_char_p, []),
            "gp_profile_enable": (i32, [vp, i32]),
            "gp_profile_read": (i32, [vp, i32, pd, pi64]),
            "gp_kmatvec": (i32, [vp, vp, i64, vp, i64, i32, pd, vp, i64, i32, vp, i64, i32, i32]),
            "gp_kmatvec_static": (i32, [vp, vp, i64, vp, i64, i32, pd, vp, i64, i32, vp, i64, i32,
                                        i32]),
            "gp_kmatvec_adjoint": (i32, [vp, vp, i64, i32, pd, vp, i64, vp, i64, i32, pd, i32, i32,
                                         pd]),
            "gp_solver_cfg_default": (None, [C.POINTER(SolverCfg)]),
            "gp_solve": (i32, [vp, vp, i64, i32, pd, vp, i64, vp, i64, i32, C.POINTER(SolverCfg),
                               C.POINTER(SolveStats)]),
            "gp_prior_sample": (i32, [vp, vp, i64, i32, pd, vp, i32, vp, i64, i32, vp, i64]),
            "gp_mll_grad": (i32, [vp, vp, i64, i32, vp, pd, i32, i32, vp, i64, vp, i32, vp, i64,
                                  vp, i64, vp, i64, C.POINTER(SolverCfg), i32, pd,
                                  C.POINTER(SolveStats)]),
            "gp_adam_ascent": (i32, [i32, pd, pd, pd, pi64, pd, dbl, i32]),
            "gp_nu_to_theta": (i32, [i32, pd, i32, pd]),
            "gp_theta_to_nu": (i32, [i32, pd, i32, pd]),
            "gp_pivoted_cholesky": (i32, [vp, vp, i64, i32, pd, i32, vp, i64, vp,
                                          C.POINTER(C.c_int)]),
            "gp_posterior_sample": (i32, [vp, vp, i64, vp, i64, i32, pd, vp, i32, vp, i64, vp,
                                          i64, i32, i32, vp, i64]),
            "gp_nearest": (i32, [vp, vp, i64, i32, i64, i64, vp]),
            "gp_exact_mll": (i32, [vp, vp, i64, i32, vp, vp, i64, pd, pd, pd]),
            "gp_init_cfg_default": (None, [C.POINTER(InitCfg)]),
            "gp_init_heuristic": (i32, [vp, vp, i64, i32, vp, pi64, i32, i64, C.POINTER(InitCfg),
                                        pd, pd]),
            "gp_workspace_size": (i32, [i32, i64, i32, i32, C.POINTER(SolverCfg), i32,
                                        C.POINTER(C.c_size_t)]),
            "gp_workspace_reserve": (i32, [vp, i32, i64, i32, i32, C.POINTER(SolverCfg), i32]),
            "gp_workspace_held": (i32, [vp, C.POINTER(C.c_size_t)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names of EXPORTS that the built library really exports (no GPU needed)."""
    L = C.CDLL(LIB_PATH)
    return [n for n in EXPORTS if hasattr(L, n)]
