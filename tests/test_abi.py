"""The C-ABI library loads without a GPU and exports every symbol include/gp.h declares."""
import os
import re
import subprocess

import pytest

from paper_2405_18457_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gp_[a-z0-9_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared_functions() == sorted(N.EXPORTS)


@pytest.mark.parametrize("lang,std", [("c", "-std=c11"), ("c++", "-std=c++17")])
def test_header_compiles_on_its_own(lang, std, tmp_path):
    # the boundary header is self-contained C11 (and C++): a C caller includes it alone
    cc = "gcc" if lang == "c" else "g++"
    src = tmp_path / ("use." + ("c" if lang == "c" else "cpp"))
    src.write_text('#include "gp.h"\nint main(void) { gp_solver_cfg c; '
                   'gp_solver_cfg_default(&c); return c.solver; }\n')
    r = subprocess.run([cc, std, "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                        "-I", os.path.dirname(HEADER), str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_library_exports_every_declared_symbol():
    assert os.path.exists(N.LIB_PATH), "libgpmi.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing
    assert sorted(N.exported_symbols()) == sorted(N.EXPORTS)


def test_library_loads_and_reports_version():
    L = N.lib()
    assert L.gp_version().decode().startswith("gpmi")


def test_host_only_entry_points_without_gpu():
    import ctypes as C
    import numpy as np
    L = N.lib()
    pd = C.POINTER(C.c_double)
    nu = np.array([-3.0, 0.0, 2.5])
    th = np.zeros(3)
    assert L.gp_nu_to_theta(3, nu.ctypes.data_as(pd), N.GP_SOFTPLUS, th.ctypes.data_as(pd)) == 0
    np.testing.assert_allclose(th, np.log1p(np.exp(nu)), rtol=1e-14)
    # the inverse: softplus(0) = log 2 and exp(0) = 1 map back to 0; round trips
    back = np.zeros(3)
    assert L.gp_theta_to_nu(3, th.ctypes.data_as(pd), N.GP_SOFTPLUS, back.ctypes.data_as(pd)) == 0
    np.testing.assert_allclose(back, nu, rtol=1e-12, atol=1e-12)
    two = np.array([np.log(2.0), 1.0])
    z = np.ones(2)
    assert L.gp_theta_to_nu(1, two.ctypes.data_as(pd), N.GP_SOFTPLUS, z.ctypes.data_as(pd)) == 0
    assert abs(z[0]) < 1e-15
    assert L.gp_theta_to_nu(1, two[1:].ctypes.data_as(pd), N.GP_LOG, z.ctypes.data_as(pd)) == 0
    assert z[0] == 0.0
    bad = np.array([0.5, -1.0])
    assert L.gp_theta_to_nu(2, bad.ctypes.data_as(pd), N.GP_SOFTPLUS,
                            z.ctypes.data_as(pd)) == N.GP_ERR_INVALID_ARG
    cfg = N.SolverCfg()
    L.gp_solver_cfg_default(C.byref(cfg))
    assert cfg.tol == 0.01 and cfg.ap_block == 1000 and cfg.sgd_batch == 500
    assert cfg.sgd_momentum == 0.9
    # Adam ascent against the oracle's Adam (itself pinned to torch)
    from oracle import optim
    m, v = np.zeros(3), np.zeros(3)
    step = C.c_int64(0)
    x = nu.copy()
    ref = optim.Adam(0.1)
    xr = nu.copy()
    g = np.array([1.5, -0.2, 3.0])
    for _ in range(5):
        assert L.gp_adam_ascent(3, x.ctypes.data_as(pd), m.ctypes.data_as(pd), v.ctypes.data_as(pd),
                                C.byref(step), g.ctypes.data_as(pd), 0.1, N.GP_SOFTPLUS) == 0
        xr = ref.step(xr, g * optim.sigmoid(xr))
    np.testing.assert_allclose(x, xr, rtol=1e-12)
    assert step.value == 5
    assert L.gp_adam_ascent(-1, None, None, None, C.byref(step), None, 0.1, 0) == N.GP_ERR_INVALID_ARG


def test_init_cfg_default_is_the_small_data_setting():
    import ctypes as C
    cfg = N.InitCfg()
    N.lib().gp_init_cfg_default(C.byref(cfg))
    assert cfg.steps == 100 and cfg.lr == 0.1 and cfg.transform == N.GP_SOFTPLUS
    assert not cfg.theta0


def test_no_gpu_means_an_error_not_a_fallback():
    # Without a visible GPU the library reports GP_ERR_HIP from context creation
    # and hands out no context: nothing downstream can run on the host instead.
    import ctypes as C
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    L = N.lib()
    h = C.c_void_p(1)
    assert L.gp_ctx_create(0, None, C.byref(h)) == N.GP_ERR_HIP
    assert h.value is None
    assert L.gp_ctx_create(0, None, None) == N.GP_ERR_INVALID_ARG
    from paper_2405_18457_amd import api
    with pytest.raises(Exception):
        api.Context(0)


def test_every_context_call_rejects_a_null_context():
    # Checked before any HIP call, so it runs without a GPU: every entry point
    # that takes a context returns GP_ERR_INVALID_ARG for NULL instead of
    # dereferencing it.
    import ctypes as C
    L = N.lib()
    checked = []
    for name in N.EXPORTS:
        f = getattr(L, name)
        if f.restype is not C.c_int or not f.argtypes or f.argtypes[0] is not C.c_void_p:
            continue
        args = [0 if t in (C.c_int, C.c_int64, C.c_double, C.c_uint64) else None
                for t in f.argtypes]
        assert f(*args) == N.GP_ERR_INVALID_ARG, name
        checked.append(name)
    assert len(checked) == 15, checked
    assert L.gp_last_error(None) == b"null context"
    L.gp_ctx_destroy(None)


def test_missing_library_raises(monkeypatch, tmp_path):
    # no CPU or Python fallback: without the built library every call path
    # stops at the loader with an ImportError that names the build step
    monkeypatch.setattr(N, "_lib", None)
    monkeypatch.setattr(N, "LIB_PATH", str(tmp_path / "libgpmi.so"))
    with pytest.raises(ImportError, match="no fallback"):
        N.lib()


def test_workspace_size_without_a_device():
    # host-only planning: grows with n and c, counts the preconditioner factor
    # (rank 8000 at n = 434,874: about 14 GB of FP32 factor), rejects bad input
    import ctypes as C
    L = N.lib()
    cfg = N.SolverCfg()
    L.gp_solver_cfg_default(C.byref(cfg))
    out = C.c_size_t()

    def size(op, n, d, c, cf, M=0):
        assert L.gp_workspace_size(op, n, d, c, C.byref(cf) if cf is not None else None, M,
                                   C.byref(out)) == 0
        return out.value

    small = size(N.GP_WS_KMATVEC, 1000, 3, 65, None)
    assert 0 < small < size(N.GP_WS_KMATVEC, 100_000, 3, 65, None)
    plain = size(N.GP_WS_SOLVE, 434_874, 3, 65, cfg)
    cfg.precond_rank = 8000
    pc = size(N.GP_WS_SOLVE, 434_874, 3, 65, cfg)
    assert pc - plain > 8000 * 434_874 * 4
    assert size(N.GP_WS_MLL_GRAD, 434_874, 3, 65, cfg, 1000) > pc
    assert size(N.GP_WS_SOLVE, 0, 3, 65, cfg) == 0
    assert L.gp_workspace_size(7, 10, 3, 4, C.byref(cfg), 0, C.byref(out)) == N.GP_ERR_INVALID_ARG
    assert L.gp_workspace_size(N.GP_WS_SOLVE, 10, 3, 4, None, 0, C.byref(out)) == N.GP_ERR_INVALID_ARG
    assert L.gp_workspace_size(N.GP_WS_SOLVE, 10, 3, 300, C.byref(cfg), 0,
                               C.byref(out)) == N.GP_ERR_INVALID_ARG
    assert L.gp_workspace_size(N.GP_WS_KMATVEC, 10, 3, 4, None, 0, None) == N.GP_ERR_INVALID_ARG
