"""FP64 CPU oracle for 3D degridding and gridding (ctypes wrapper).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. It shares no code with
the HIP path and never imports it; the product library never loads it.

The arithmetic lives in ``degrid_oracle.c`` (plain loops in FP64, following
Section 2 of the paper). This module only widens inputs to FP64, checks
shapes and calls the C functions.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "degrid_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``degrid_oracle.c`` into ``liboracle.so`` with gcc and OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    """Load ``liboracle.so`` (building it first if it is missing or stale).

    ``DEGRID_ORACLE_LIB`` names another build of the same source to load
    instead; the mutation test uses it to run the pins against deliberately
    broken copies of the oracle.
    """
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("DEGRID_ORACLE_LIB")
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
    lib = ctypes.CDLL(path)
    d, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    args = [i64, i32, i32, i32, i32, i32, i32, i32, d, d, d, d, d, d]
    lib.oracle_degrid.argtypes = args
    lib.oracle_degrid.restype = i64
    lib.oracle_grid.argtypes = args
    lib.oracle_grid.restype = i64
    lib.oracle_table_grad.argtypes = [i64, i32, i32, i32, i32, i32, i32, i32, d, d, d, d, d, d, d, d]
    lib.oracle_table_grad.restype = i64
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = i32
    lib.oracle_set_num_threads.argtypes = [i32]
    lib.oracle_set_num_threads.restype = None
    _lib = lib
    return lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (for timing on a chosen core count)."""
    _load().oracle_set_num_threads(int(n))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def _complex_as_pairs(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a.view(np.float64).reshape(a.shape + (2,))


def _check(g_uv, g_w, uvw, offsets):
    g_uv = _f64(g_uv)
    g_w = _f64(g_w)
    uvw = _f64(uvw)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    os_uv, os_uv2, su, su2 = g_uv.shape
    os_w, sw = g_w.shape
    if os_uv != os_uv2 or su != su2:
        raise ValueError("g_uv must be [os][os][W][W]")
    if uvw.ndim != 2 or uvw.shape[1] != 3 or uvw.shape[0] != offsets[-1]:
        raise ValueError("uvw must be [offsets[-1]][3]")
    if offsets[0] != 0 or np.any(np.diff(offsets) < 0):
        raise ValueError("offsets must start at 0 and be non-decreasing")
    return g_uv, g_w, uvw, offsets, os_uv, su, os_w, sw


def degrid(subgrids, g_uv, g_w, uvw, offsets):
    """Degrid in FP64. ``subgrids`` complex ``[S][n_v][n_u][n_w]``.

    Returns ``(vis complex128 [N], out_of_range_count)``.
    """
    g_uv, g_w, uvw, offsets, os_uv, su, os_w, sw = _check(g_uv, g_w, uvw, offsets)
    a = _complex_as_pairs(subgrids)
    s, n_v, n_u, n_w = a.shape[:4]
    if s != len(offsets) - 1:
        raise ValueError("offsets must have S+1 entries")
    n = int(offsets[-1])
    out = np.zeros((n, 2), dtype=np.float64)
    oob = _load().oracle_degrid(s, n_v, n_u, n_w, su, sw, os_uv, os_w,
                                a.ctypes.data, g_uv.ctypes.data, g_w.ctypes.data,
                                uvw.ctypes.data, offsets.ctypes.data, out.ctypes.data)
    return out[:, 0] + 1j * out[:, 1], int(oob)


def grid(vis, g_uv, g_w, uvw, offsets, shape):
    """Grid (adjoint of degrid) in FP64. ``shape`` = ``(S, n_v, n_u, n_w)``.

    Returns ``(subgrids complex128 [S][n_v][n_u][n_w], out_of_range_count)``.
    """
    g_uv, g_w, uvw, offsets, os_uv, su, os_w, sw = _check(g_uv, g_w, uvw, offsets)
    s, n_v, n_u, n_w = (int(x) for x in shape)
    if s != len(offsets) - 1:
        raise ValueError("offsets must have S+1 entries")
    v = _complex_as_pairs(vis)
    if v.shape != (int(offsets[-1]), 2):
        raise ValueError("vis must have offsets[-1] entries")
    out = np.zeros((s, n_v, n_u, n_w, 2), dtype=np.float64)
    oob = _load().oracle_grid(s, n_v, n_u, n_w, su, sw, os_uv, os_w,
                              v.ctypes.data, g_uv.ctypes.data, g_w.ctypes.data,
                              uvw.ctypes.data, offsets.ctypes.data, out.ctypes.data)
    return out[..., 0] + 1j * out[..., 1], int(oob)


def table_grad(subgrids, g_uv, g_w, uvw, offsets, grad_vis):
    """Gradients of a real loss with respect to ``G_uv`` and ``G_w`` in FP64,
    given ``grad_vis`` = dL/dRe(V) + i dL/dIm(V) (complex ``[N]``).

    Returns ``(grad_g_uv [os][os][W][W], grad_g_w [os_w][Ww], out_of_range_count)``.
    """
    g_uv, g_w, uvw, offsets, os_uv, su, os_w, sw = _check(g_uv, g_w, uvw, offsets)
    a = _complex_as_pairs(subgrids)
    s, n_v, n_u, n_w = a.shape[:4]
    if s != len(offsets) - 1:
        raise ValueError("offsets must have S+1 entries")
    gv = _complex_as_pairs(grad_vis)
    if gv.shape != (int(offsets[-1]), 2):
        raise ValueError("grad_vis must have offsets[-1] entries")
    out_uv = np.zeros(g_uv.shape, dtype=np.float64)
    out_w = np.zeros(g_w.shape, dtype=np.float64)
    oob = _load().oracle_table_grad(s, n_v, n_u, n_w, su, sw, os_uv, os_w,
                                    a.ctypes.data, g_uv.ctypes.data, g_w.ctypes.data, uvw.ctypes.data,
                                    offsets.ctypes.data, gv.ctypes.data, out_uv.ctypes.data, out_w.ctypes.data)
    return out_uv, out_w, int(oob)
