"""Build the gfx950 shared library ``libgpmi.so`` from the HIP sources in ``csrc/``.

Every compile-time dimension of the tile kernels is its own translation unit
so the instantiations build in parallel.  Usage: ``python -m paper_2405_18457_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgpmi.so")

ARCH = "gfx950"
DIMS = (1, 2, 3, 4, 8, 12, 16, 24, 32, 64)
PER_DIM = ("fwd", "adj", "rff")
SINGLE = ("dispatch", "vec", "solve", "precond", "exact", "nearest", "runtime")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed-FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _jobs():
    units = []
    for name in PER_DIM:
        for d in DIMS:
            units.append((os.path.join(CSRC, f"{name}.hip"), os.path.join(BUILD, f"{name}_d{d}.o"),
                          [f"-DGPK_D={d}"]))
    for name in SINGLE:
        units.append((os.path.join(CSRC, f"{name}.hip"), os.path.join(BUILD, f"{name}.o"), []))
    return units


def _compile(hipcc, src, obj, extra):
    cmd = [hipcc, *CFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stderr or "").splitlines()
                     if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{errs}")
    return obj


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src, os.path.join(CSRC, "gpk.h"), os.path.join(INCLUDE, "gp.h")]
    return any(os.path.getmtime(p) > t for p in deps)


def build(jobs: int | None = None, verbose: bool = True, incremental: bool = False) -> str:
    """Compile every translation unit and link ``libgpmi.so``.

    By default everything is recompiled; ``incremental=True`` (developer use)
    recompiles only units whose source or shared headers changed."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    units = _jobs()
    if incremental:
        todo = [u for u in units if _stale(u[0], u[1])]
        done = [u[1] for u in units if u not in todo]
    else:
        todo, done = units, []
    jobs = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = done + list(ex.map(lambda u: _compile(hipcc, *u), todo))
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
