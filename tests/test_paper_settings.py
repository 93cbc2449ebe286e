"""Defaults against the experimental settings App. B states (cited per line in
tests/golden/app_b_settings.txt): the library's solver and heuristic
configurations, the oracle's heuristic, the workload generator and the bench's
heuristic mode."""
import ctypes as C
import inspect
import os
import sys

import pytest

import workloads as wl
from oracle import init_heuristic as ih
from paper_2405_18457_amd import _native as N

HERE = os.path.dirname(os.path.abspath(__file__))


def _settings():
    out = {}
    for line in open(os.path.join(HERE, "golden", "app_b_settings.txt")):
        line = line.split("|")[0].strip()
        if not line or line.startswith("#"):
            continue
        key, value = (p.strip() for p in line.split("="))
        try:
            out[key] = float(value) if "." in value else int(value)
        except ValueError:
            out[key] = value
    return out


S = _settings()


def test_fixture_is_complete():
    assert len(S) == 13


def test_library_solver_defaults():
    cfg = N.SolverCfg()
    N.lib().gp_solver_cfg_default(C.byref(cfg))
    assert cfg.tol == S["solver_tol"]
    assert cfg.ap_block == S["ap_block"]
    assert cfg.sgd_batch == S["sgd_batch"]
    assert cfg.sgd_momentum == S["sgd_momentum"]
    # the preconditioner is opt-in; the header names the paper's rank for it
    assert cfg.precond_rank == 0
    header = open(os.path.join(HERE, "..", "include", "gp.h")).read()
    assert f"precond_rank = {S['cg_precond_rank']} for the paper's CG" in header


def test_library_and_oracle_heuristic_defaults():
    cfg = N.InitCfg()
    N.lib().gp_init_cfg_default(C.byref(cfg))
    assert cfg.steps == S["adam_steps_small"] and cfg.lr == S["adam_lr_small"]
    assert S["transform"] == "softplus" and cfg.transform == N.GP_SOFTPLUS
    assert not cfg.theta0  # NULL: every hyperparameter starts at 1.0
    sig = inspect.signature(ih.init_heuristic).parameters
    assert sig["steps"].default == S["adam_steps_small"]
    assert sig["lr"].default == S["adam_lr_small"]
    assert sig["transform"].default == S["transform"]
    import numpy as np
    X = np.random.default_rng(0).standard_normal((5, 2))
    y = np.ones(5)
    _, each = ih.init_heuristic(X, y, [0], m=5, steps=0)
    assert np.all(each == S["theta0_small"])


def test_workload_and_bench_defaults(monkeypatch):
    for name in "BCDE":
        assert wl.WORKLOADS[name].s == S["probes"]
        assert wl.WORKLOADS[name].model_pairs == S["rff_pairs"]
    assert len(wl.draw_centroids(wl.WORKLOADS["D"])) == S["heuristic_centroids"]
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    import bench
    args = bench.parse()
    assert args.init_centres == S["heuristic_centroids"]
    assert args.init_m == S["heuristic_subset"]
    assert args.init_steps == S["adam_steps_small"]
