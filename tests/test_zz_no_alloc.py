"""The allocation-free product gp_kmatvec_static against gp_kmatvec (same inputs,
same arguments): two calls in a row, the second on a smaller input, with a fresh
context that must still hold no workspace afterwards; sizes beyond its static
scratch are rejected with a message."""
import numpy as np
import pytest

from gpu_common import announce, col_relerr, dev, elem_relerr, host, problem, require_gpu

pytestmark = pytest.mark.gpu

TOL = {0: 1e-5, 1: 2e-5}  # the product bounds of tests/test_gpu_kmatvec.py


@pytest.mark.parametrize("prec", [0, 1], ids=["fp32", "bf16x3"])
@pytest.mark.parametrize("d,square", [(3, True), (8, True), (3, False)],
                         ids=["d3-square", "d8-square", "d3-rect"])
def test_static_product_matches_the_allocating_one(prec, d, square):
    require_gpu()
    from paper_2405_18457_amd import api
    import torch
    ctx = api.Context(0)
    try:
        assert api.gp_workspace_held(ctx) == 0
        for n, c, seed in ((20_000, 65, 1), (3_001, 17, 2)):
            X, V, theta = problem(n, d, c, seed=seed, dist="uniform" if d == 3 else "normal",
                                  ell_scale=(0.05, 0.2) if d == 3 else None)
            Xd, Vd = dev(X), dev(V)
            X1 = Xd if square else dev(problem(n // 3 + 7, d, 1, seed=seed + 9,
                                               dist="uniform")[0])
            n1 = X1.shape[0]
            out = torch.full((n1, c), np.nan, device="cuda")
            announce("kmatvec_static", prec, d, square, n, c)
            api.gp_kmatvec_static(ctx, X1, Xd, theta, Vd, prec, add_noise=square, out=out)
            torch.cuda.synchronize()
            assert api.gp_workspace_held(ctx) == 0
            ref_ctx = api.Context(0)
            try:
                ref = api.gp_kmatvec(ref_ctx, X1, Xd, theta, Vd, prec, add_noise=square)
            finally:
                ref_ctx.close()
            o, r = host(out), host(ref)
            assert np.all(np.isfinite(o))
            col, ent = col_relerr(o, r), elem_relerr(o, r)
            print(f"[gpu-case] static vs allocating: column {col:.2e}, entry {ent:.2e}", flush=True)
            assert col <= TOL[prec] and ent <= 2 * TOL[prec], (col, ent)
    finally:
        ctx.close()


def test_static_product_rejects_what_does_not_fit():
    require_gpu()
    from paper_2405_18457_amd import api
    import torch
    ctx = api.Context(0)
    try:
        n, c = 300_000, 80   # packed inputs and V tiles: about 100 MB > 64 MiB
        X = torch.zeros((n, 3), device="cuda")
        V = torch.zeros((n, c), device="cuda")
        out = torch.empty((n, c), device="cuda")
        announce("kmatvec_static too large")
        with pytest.raises(api.GPError) as e:
            api.gp_kmatvec_static(ctx, X, X, np.array([0.1, 0.1, 0.1, 1.0, 0.1]), V, 1,
                                  add_noise=True, out=out)
        assert e.value.code == 1 and "scratch" in str(e.value)
        assert api.gp_workspace_held(ctx) == 0
    finally:
        ctx.close()
