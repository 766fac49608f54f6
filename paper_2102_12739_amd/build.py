"""Build the gfx950 degridding library (``libdegrid.so``) in-tree with hipcc."""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libdegrid.so")
SOURCES = [os.path.join(CSRC, "degrid_kernels.hip"), os.path.join(CSRC, "grid_kernels.hip"),
           os.path.join(CSRC, "degrid_api.cpp"),
           os.path.join(CSRC, "plan_logic.cpp"), os.path.join(CSRC, "plan_sort.hip"),
           os.path.join(CSRC, "table_grad_kernels.hip"), os.path.join(CSRC, "noalloc.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Device code: gfx950 only; packed FP32 instructions disabled; hardware float
# atomics for the adjoint scatter.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]
NOISE = "is not a recognized feature for this target"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if NOISE not in l)
    return r.returncode, err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source (in parallel, one object each) and link
    ``libdegrid.so``. Always recompiles."""
    jobs = jobs or min(len(SOURCES), max(1, min(8, os.cpu_count() or 1)))
    tmpdir = tempfile.mkdtemp(prefix="dgbuild")
    try:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in SOURCES]
        cmds = [[HIPCC, *FLAGS, "-c", "-o", o, s] for s, o in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_run, cmds))
        for (rc, err), s in zip(results, SOURCES):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {os.path.basename(s)} ({rc}):\n{err}")
            if verbose and err.strip():
                print(err, file=sys.stderr)
        tmp = LIB + f".tmp{os.getpid()}"
        link = [HIPCC, *FLAGS, "-shared", "-Wl,--no-undefined", "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        rc, err = _run(link)
        if rc != 0:
            raise RuntimeError(f"hipcc link failed ({rc}):\n{err}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
