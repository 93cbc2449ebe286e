"""Shared helpers for the GPU parity tests (seeded float32 inputs, error metrics)."""
import sys

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")


def announce(*parts):
    """Print the case before a GPU step (so a crash names it) and flush."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def problem(n, d, c, seed, dist="normal", ell_scale=None, a=1.1, sigma=0.3):
    """Seeded float32 inputs X [n, d], V [n, c] and theta (ell_1..ell_d, a, sigma).

    Length scales grow with sqrt(d) so the kernel matrix stays far from the
    identity at every d (the workloads' regime: many non-negligible entries)."""
    g = np.random.default_rng(seed)
    if dist == "uniform":
        X = g.uniform(-1, 1, (n, d))
        lo, hi = (0.05, 0.2) if ell_scale is None else ell_scale
    else:
        X = g.standard_normal((n, d))
        base = np.sqrt(d) * 0.6
        lo, hi = (0.5 * base, 1.5 * base) if ell_scale is None else ell_scale
    ell = g.uniform(lo, hi, d)
    theta = np.concatenate([ell, [a, sigma]])
    V = g.standard_normal((n, c))
    return X.astype(np.float32), V.astype(np.float32), theta


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def col_relerr(out, ref):
    """max over columns of ||out_c - ref_c|| / ||ref_c||."""
    num = np.linalg.norm(out - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return float(np.max(num / np.maximum(den, 1e-300)))


def elem_relerr(out, ref):
    """max |out - ref| over all entries / max |ref|: a few wrong entries (a tile
    edge, a ragged tail) are not diluted by the rest of the column."""
    return float(np.max(np.abs(out - ref)) / max(float(np.max(np.abs(ref))), 1e-300))


def entry_bound_ratio(out, ref, mag):
    """max over entries of |out - ref| / mag, where mag is the sum of the absolute
    values of the terms that make up each entry (a deterministic rounding bound is
    a multiple of it)."""
    return float(np.max(np.abs(out - ref) / np.maximum(mag, 1e-300)))
