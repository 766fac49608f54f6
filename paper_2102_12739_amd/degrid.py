"""Python binding of the gfx950 degridding library (ctypes over the C ABI).

Every function here only checks and marshals arguments (device pointers,
sizes, the current HIP stream) and calls the C ABI of ``libdegrid.so``; all
arithmetic runs in the library's HIP kernels. PyTorch supplies device memory
and streams. There is no CPU fallback: if the library is missing or cannot
load, every call raises.

Section 2 of the paper defines the operation: for each visibility of each
subgrid, the start point and oversampled GCF positions are computed from
``(u, v, w)`` and the visibility is the G_w x G_uv weighted sum of the
8 x 8 x 4 neighbourhood. ``grid_adjoint`` is its transpose and is the
backward pass of :class:`DegridFn`.
"""

from __future__ import annotations

import ctypes
import os
from typing import Sequence

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libdegrid.so")
_lib = None

GRID_DTYPES = {"c64": 0, "cbf16": 1, "cf16": 2}
GCF_DTYPES = {"f32": 0, "f16": 1, "bf16": 2}
_STATUS = {0: "DG_OK", 1: "DG_ERR_INVALID_ARG", 2: "DG_ERR_UNSUPPORTED", 3: "DG_ERR_NOMEM",
           4: "DG_ERR_HIP", 5: "DG_ERR_NOT_READY"}


class DegridError(RuntimeError):
    """A C-ABI call returned a status other than DG_OK."""

    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        name = _STATUS.get(status, f"status {status}")
        super().__init__(f"{where}: {name}" + (f" ({detail})" if detail else ""))


class DgDesc(ctypes.Structure):
    _fields_ = [("n_v", ctypes.c_int32), ("n_u", ctypes.c_int32), ("n_w", ctypes.c_int32),
                ("support_uv", ctypes.c_int32), ("support_w", ctypes.c_int32),
                ("os_uv", ctypes.c_int32), ("os_w", ctypes.c_int32),
                ("grid_dtype", ctypes.c_int32), ("gcf_dtype", ctypes.c_int32),
                ("n_b", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class DgPlanInfo(ctypes.Structure):
    _fields_ = [("n_subgrids", ctypes.c_int64), ("n_vis", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("n_b", ctypes.c_int32), ("kernel", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("block_threads", ctypes.c_int32), ("n_queues", ctypes.c_int32), ("device", ctypes.c_int32),
                ("sorted", ctypes.c_int32), ("n_kernels", ctypes.c_int32)]


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load ``libdegrid.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(or python -m paper_2102_12739_amd.build)")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "degrid_plan": ([ctypes.POINTER(DgDesc), i64, ctypes.POINTER(ctypes.c_int64), vp,
                         ctypes.POINTER(vp)], i32),
        "degrid_execute": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "degrid_execute_noalloc": ([ctypes.POINTER(DgDesc), i64, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, vp,
                                    vp, vp, vp], i32),
        "degrid_residual": ([vp, vp, vp, vp, vp, vp, vp, vp, vp], i32),
        "grid_adjoint": ([vp, vp, vp, vp, vp, vp, i32, vp], i32),
        "degrid_table_grad": ([vp, vp, vp, vp, vp, vp, vp, vp, i32, vp], i32),
        "degrid_oob_count": ([vp, ctypes.POINTER(ctypes.c_int64)], i32),
        "degrid_plan_get_info": ([vp, ctypes.POINTER(DgPlanInfo)], i32),
        "degrid_plan_sort": ([vp, vp, vp], i32),
        "degrid_plan_set_kernel": ([vp, i32, i32, vp], i32),
        "degrid_tune": ([vp, vp, vp, vp, vp, vp, vp], i32),
        "degrid_destroy": ([vp], i32),
        "degrid_batch_plan": ([ctypes.POINTER(vp), i32, ctypes.POINTER(vp)], i32),
        "degrid_batch_execute": ([vp, ctypes.POINTER(vp), vp], i32),
        "degrid_batch_oob_count": ([vp, ctypes.POINTER(ctypes.c_int64)], i32),
        "degrid_batch_destroy": ([vp], i32),
        "degrid_batch_tune": ([ctypes.POINTER(vp), i32, ctypes.POINTER(vp), vp, ctypes.POINTER(i32),
                               ctypes.POINTER(i32)], i32),
        "degrid_status_str": ([i32], ctypes.c_char_p),
        "degrid_last_error": ([], ctypes.c_char_p),
        "degrid_version": ([], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(status: int, where: str):
    if status != 0:
        detail = lib().degrid_last_error().decode(errors="replace")
        raise DegridError(status, where, detail)


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        return int(stream.cuda_stream)
    return int(stream)


def _ptr(t: torch.Tensor, name: str, dtype=None, shape=None) -> int:
    """Device pointer of a checked tensor. Runs for every tensor of every
    call, so each check takes its cheapest form (``is_cuda``, dtype identity,
    ``torch.Size`` against the expected tuple); ``shape`` is a tuple."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU device, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype is not dtype and not (isinstance(dtype, tuple) and t.dtype in dtype):
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and t.shape != shape:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


_GRID_TENSOR_DTYPE = {"c64": torch.complex64, "cbf16": torch.bfloat16, "cf16": torch.float16}
_GCF_TENSOR_DTYPE = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}


def _grid_tensor_dtype(grid_dtype: str):
    return _GRID_TENSOR_DTYPE[grid_dtype]


def _gcf_tensor_dtype(gcf_dtype: str):
    return _GCF_TENSOR_DTYPE[gcf_dtype]


class Plan:
    """A degridding plan for one problem (owns the library's device scratch).

    ``offsets`` are the host CSR offsets ``[S+1]`` of the visibilities per
    subgrid. Subgrids are ``[S, n_v, n_u, n_w]`` complex64 (``grid_dtype``
    "c64"), or ``[S, n_v, n_u, n_w, 2]`` bfloat16 / float16 ("cbf16" /
    "cf16"). The tables ``G_uv [os_uv, os_uv, 8, 8]`` and ``G_w [os_w, 4]``
    are float32, float16 or bfloat16 (``gcf_dtype`` "f32" / "f16" / "bf16").
    """

    def __init__(self, offsets, n_v: int = 512, n_u: int = 512, n_w: int = 4,
                 os_uv: int = 16, os_w: int = 16, grid_dtype: str = "c64", gcf_dtype: str = "f32",
                 n_b: int = 0, stream=None):
        self._handle = None
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        if off.ndim != 1 or off.size < 1:
            raise ValueError("offsets must be a 1-D array of S+1 entries")
        if grid_dtype not in GRID_DTYPES or gcf_dtype not in GCF_DTYPES:
            raise ValueError(f"unknown dtype {grid_dtype}/{gcf_dtype}")
        self.offsets = off
        self.n_subgrids = off.size - 1
        self.n_vis = int(off[-1])
        self.shape = (self.n_subgrids, n_v, n_u, n_w)
        self.os_uv, self.os_w = os_uv, os_w
        self.grid_dtype, self.gcf_dtype = grid_dtype, gcf_dtype
        d = DgDesc(n_v, n_u, n_w, 8, 4, os_uv, os_w, GRID_DTYPES[grid_dtype], GCF_DTYPES[gcf_dtype], n_b, 0)
        h = ctypes.c_void_p()
        st = lib().degrid_plan(ctypes.byref(d), self.n_subgrids,
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               ctypes.c_void_p(_stream_handle(stream) if torch.cuda.is_available() else 0),
                               ctypes.byref(h))
        _check(st, "degrid_plan")
        self._handle = h

    # -- shapes and checks ------------------------------------------------
    def _grid_shape(self):
        return self.shape if self.grid_dtype == "c64" else self.shape + (2,)

    def _check_tables(self, g_uv, g_w):
        dt = _gcf_tensor_dtype(self.gcf_dtype)
        return (_ptr(g_uv, "g_uv", dt, (self.os_uv, self.os_uv, 8, 8)),
                _ptr(g_w, "g_w", dt, (self.os_w, 4)))

    def _check_uvw(self, uvw):
        return _ptr(uvw, "uvw", torch.float64, (self.n_vis, 3))

    # -- calls --------------------------------------------------------------
    def execute(self, subgrids, g_uv, g_w, uvw, out=None, stream=None) -> torch.Tensor:
        """Degrid; returns ``vis`` complex64 ``[N]`` (written into ``out`` if given)."""
        ps = _ptr(subgrids, "subgrids", _grid_tensor_dtype(self.grid_dtype), self._grid_shape())
        pg, pw = self._check_tables(g_uv, g_w)
        pu = self._check_uvw(uvw)
        if out is None:
            out = torch.empty(self.n_vis, dtype=torch.complex64, device=uvw.device)
        po = _ptr(out, "out", torch.complex64, (self.n_vis,))
        _check(lib().degrid_execute(self._handle, ps, pg, pw, pu, po, _stream_handle(stream)), "degrid_execute")
        return out

    def residual(self, subgrids, g_uv, g_w, uvw, v_obs, out=None, loss=None, stream=None):
        """``res = v_obs - degrid(subgrids)`` and ``loss = sum |res|^2`` in one pass.

        Returns ``(res complex64 [N], loss float64 0-dim)``; ``out`` may be ``v_obs``.
        """
        ps = _ptr(subgrids, "subgrids", _grid_tensor_dtype(self.grid_dtype), self._grid_shape())
        pg, pw = self._check_tables(g_uv, g_w)
        pu = self._check_uvw(uvw)
        pv = _ptr(v_obs, "v_obs", torch.complex64, (self.n_vis,))
        if out is None:
            out = torch.empty(self.n_vis, dtype=torch.complex64, device=uvw.device)
        po = _ptr(out, "out", torch.complex64, (self.n_vis,))
        if loss is None:
            loss = torch.empty((), dtype=torch.float64, device=uvw.device)
        pl = _ptr(loss, "loss", torch.float64, ())
        _check(lib().degrid_residual(self._handle, ps, pg, pw, pu, pv, po, pl, _stream_handle(stream)),
               "degrid_residual")
        return out, loss

    def adjoint(self, vis, g_uv, g_w, uvw, out=None, accumulate: bool = False, stream=None) -> torch.Tensor:
        """Grid (transpose of degrid); returns complex64 ``[S, n_v, n_u, n_w]``."""
        pv = _ptr(vis, "vis", torch.complex64, (self.n_vis,))
        pg, pw = self._check_tables(g_uv, g_w)
        pu = self._check_uvw(uvw)
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=uvw.device)
            accumulate = False
        po = _ptr(out, "out", torch.complex64, self.shape)
        _check(lib().grid_adjoint(self._handle, pv, pg, pw, pu, po, int(bool(accumulate)),
                                  _stream_handle(stream)), "grid_adjoint")
        return out

    def table_grad(self, subgrids, g_uv, g_w, uvw, grad_vis, want_uv: bool = True, want_w: bool = True,
                   out_uv=None, out_w=None, accumulate: bool = False, stream=None):
        """Gradients of a real loss with respect to the tables from ``grad_vis``
        = dL/dRe(V) + i dL/dIm(V) (complex64 ``[N]``).

        Returns ``(grad_g_uv float32 [os_uv, os_uv, 8, 8], grad_g_w float32
        [os_w, 4])``, with ``None`` for a table not asked for.
        """
        ps = _ptr(subgrids, "subgrids", _grid_tensor_dtype(self.grid_dtype), self._grid_shape())
        pg, pw = self._check_tables(g_uv, g_w)
        pu = self._check_uvw(uvw)
        pv = _ptr(grad_vis, "grad_vis", torch.complex64, (self.n_vis,))
        dev = uvw.device
        if want_uv and out_uv is None:
            out_uv = torch.empty((self.os_uv, self.os_uv, 8, 8), dtype=torch.float32, device=dev)
            accumulate = False
        if want_w and out_w is None:
            out_w = torch.empty((self.os_w, 4), dtype=torch.float32, device=dev)
            accumulate = False
        po_uv = _ptr(out_uv, "out_uv", torch.float32, (self.os_uv, self.os_uv, 8, 8)) if want_uv else None
        po_w = _ptr(out_w, "out_w", torch.float32, (self.os_w, 4)) if want_w else None
        _check(lib().degrid_table_grad(self._handle, ps, pg, pw, pu, pv, po_uv, po_w, int(bool(accumulate)),
                                       _stream_handle(stream)), "degrid_table_grad")
        return (out_uv if want_uv else None), (out_w if want_w else None)

    def tune(self, subgrids, g_uv, g_w, uvw, out=None, stream=None):
        """Time tile sizes and kernel variants on these inputs; keep the fastest."""
        ps = _ptr(subgrids, "subgrids", _grid_tensor_dtype(self.grid_dtype), self._grid_shape())
        pg, pw = self._check_tables(g_uv, g_w)
        pu = self._check_uvw(uvw)
        if out is None:
            out = torch.empty(self.n_vis, dtype=torch.complex64, device=uvw.device)
        po = _ptr(out, "out", torch.complex64, (self.n_vis,))
        _check(lib().degrid_tune(self._handle, ps, pg, pw, pu, po, _stream_handle(stream)), "degrid_tune")
        return self.info()

    def sort(self, uvw=None, stream=None):
        """Order the work by subgrid position (Hilbert order of the cell holding (u, v)).

        Outputs stay in input order and unchanged; later calls are faster when
        they use these same coordinates. ``uvw=None`` restores input order.
        """
        pu = self._check_uvw(uvw) if uvw is not None else None
        _check(lib().degrid_plan_sort(self._handle, pu, _stream_handle(stream)), "degrid_plan_sort")
        return self

    def set_kernel(self, kernel: int = -1, n_b: int = 0, stream=None):
        """Pick the gather kernel variant and/or tile size by hand (-1 / 0 keep)."""
        _check(lib().degrid_plan_set_kernel(self._handle, int(kernel), int(n_b), _stream_handle(stream)),
               "degrid_plan_set_kernel")
        return self

    def oob_count(self) -> int:
        c = ctypes.c_int64()
        _check(lib().degrid_oob_count(self._handle, ctypes.byref(c)), "degrid_oob_count")
        return int(c.value)

    def info(self) -> dict:
        i = DgPlanInfo()
        _check(lib().degrid_plan_get_info(self._handle, ctypes.byref(i)), "degrid_plan_get_info")
        return {f: getattr(i, f) for f, _ in DgPlanInfo._fields_}

    @property
    def handle(self):
        return self._handle

    def close(self):
        if self._handle is not None and _lib is not None:
            _lib.degrid_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def degrid_noalloc(subgrids, g_uv, g_w, uvw, offsets, out=None, oob_count=None, grid_dtype: str = "c64",
                   gcf_dtype: str = "f32", n_b: int = 0, stream=None) -> torch.Tensor:
    """Degrid without a plan through ``degrid_execute_noalloc`` (the library
    allocates nothing; its scratch is a static per-GPU array, so calls that
    overlap on one GPU race). Shapes and dtypes as for :meth:`Plan.execute`;
    ``offsets`` are the host CSR offsets ``[S+1]``. ``oob_count``, if given,
    is a device int64 0-dim tensor that receives the out-of-range count."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    s = off.size - 1
    shape = tuple(subgrids.shape[:4])
    if shape[0] != s:
        raise ValueError(f"subgrids hold {shape[0]} subgrids, offsets describe {s}")
    n_v, n_u, n_w = shape[1:4]
    grid_shape = shape if grid_dtype == "c64" else shape + (2,)
    ps = _ptr(subgrids, "subgrids", _grid_tensor_dtype(grid_dtype), grid_shape)
    tdt = _gcf_tensor_dtype(gcf_dtype)
    pg = _ptr(g_uv, "g_uv", tdt)
    pw = _ptr(g_w, "g_w", tdt)
    os_uv, os_w = g_uv.shape[0], g_w.shape[0]
    n = int(off[-1])
    pu = _ptr(uvw, "uvw", torch.float64, (n, 3))
    if out is None:
        out = torch.empty(n, dtype=torch.complex64, device=uvw.device)
    po = _ptr(out, "out", torch.complex64, (n,))
    pc = _ptr(oob_count, "oob_count", torch.int64, ()) if oob_count is not None else None
    d = DgDesc(n_v, n_u, n_w, 8, 4, os_uv, os_w, GRID_DTYPES[grid_dtype], GCF_DTYPES[gcf_dtype], n_b, 0)
    _check(lib().degrid_execute_noalloc(ctypes.byref(d), s, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        ps, pg, pw, pu, po, pc, _stream_handle(stream)), "degrid_execute_noalloc")
    return out


def _batch_args(plans, problems, outs):
    if len(problems) != len(plans):
        raise ValueError("one (subgrids, g_uv, g_w, uvw) tuple per plan")
    if outs is None:
        outs = [torch.empty(p.n_vis, dtype=torch.complex64, device=pr[3].device) for p, pr in zip(plans, problems)]
    ptrs = []
    for p, (sub, g_uv, g_w, uvw), out in zip(plans, problems, outs):
        ptrs += [_ptr(sub, "subgrids", _grid_tensor_dtype(p.grid_dtype), p._grid_shape()),
                 *p._check_tables(g_uv, g_w), p._check_uvw(uvw),
                 _ptr(out, "out", torch.complex64, (p.n_vis,))]
    return (ctypes.c_void_p * len(ptrs))(*ptrs), outs


def batch_tune(plans: Sequence[Plan], problems, outs=None, stream=None):
    """Time kernel variants and tile sizes on one launch of the whole batch and
    set every plan to the fastest; returns ``(kernel, n_b)``."""
    plans = list(plans)
    arr, outs = _batch_args(plans, problems, outs)
    handles = (ctypes.c_void_p * len(plans))(*[p.handle for p in plans])
    k, nb = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().degrid_batch_tune(handles, len(plans), arr, _stream_handle(stream), ctypes.byref(k),
                                   ctypes.byref(nb)), "degrid_batch_tune")
    return int(k.value), int(nb.value)


class Batch:
    """Several plans degridded by one persistent launch replayed from a HIP graph."""

    def __init__(self, plans: Sequence[Plan]):
        self._handle = None
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().degrid_batch_plan(arr, len(self.plans), ctypes.byref(h)), "degrid_batch_plan")
        self._handle = h

    def execute(self, problems, outs=None, stream=None):
        """``problems``: per plan a tuple ``(subgrids, g_uv, g_w, uvw)``; returns the outputs."""
        arr, outs = _batch_args(self.plans, problems, outs)
        _check(lib().degrid_batch_execute(self._handle, arr, _stream_handle(stream)), "degrid_batch_execute")
        return outs

    def oob_count(self) -> int:
        c = ctypes.c_int64()
        _check(lib().degrid_batch_oob_count(self._handle, ctypes.byref(c)), "degrid_batch_oob_count")
        return int(c.value)

    def close(self):
        if self._handle is not None and _lib is not None:
            _lib.degrid_batch_destroy(self._handle)
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DegridFn(torch.autograd.Function):
    """``vis = degrid(subgrids)`` with the gridding adjoint as its backward.

    The map is real-linear with real weights W, so for PyTorch's complex
    gradient convention the vector-Jacobian product is ``W^T grad_vis``, i.e.
    ``grid_adjoint(grad_vis)``. The tables get their gradients from
    ``degrid_table_grad`` (each visibility is linear in each table), returned
    in the tables' dtype. ``uvw`` gets none: the table lookup is piecewise
    constant in it.
    """

    @staticmethod
    def forward(ctx, subgrids, plan: Plan, g_uv, g_w, uvw):
        ctx.plan = plan
        ctx.save_for_backward(subgrids, g_uv, g_w, uvw)
        return plan.execute(subgrids, g_uv, g_w, uvw)

    @staticmethod
    def backward(ctx, grad_vis):
        subgrids, g_uv, g_w, uvw = ctx.saved_tensors
        gv = grad_vis.contiguous().to(torch.complex64)
        grad = grad_uv = grad_w = None
        if ctx.needs_input_grad[0]:
            grad = ctx.plan.adjoint(gv, g_uv, g_w, uvw)
        want_uv, want_w = ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        if want_uv or want_w:
            grad_uv, grad_w = ctx.plan.table_grad(subgrids.detach(), g_uv.detach(), g_w.detach(), uvw, gv,
                                                  want_uv=want_uv, want_w=want_w)
            grad_uv = grad_uv.to(g_uv.dtype) if grad_uv is not None else None
            grad_w = grad_w.to(g_w.dtype) if grad_w is not None else None
        return grad, None, grad_uv, grad_w, None


class ResidualLossFn(torch.autograd.Function):
    """``loss = sum |v_obs - degrid(subgrids)|^2`` in one fused pass (float64
    0-dim), with ``d loss / d subgrids = -2 grid_adjoint(res)`` and
    ``d loss / d v_obs = 2 res`` in PyTorch's complex gradient convention."""

    @staticmethod
    def forward(ctx, subgrids, plan: Plan, g_uv, g_w, uvw, v_obs):
        res, loss = plan.residual(subgrids, g_uv, g_w, uvw, v_obs)
        ctx.plan = plan
        ctx.save_for_backward(g_uv, g_w, uvw, res)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        g_uv, g_w, uvw, res = ctx.saved_tensors
        scale = (2.0 * grad_loss).to(torch.float32)
        grad_sub = grad_obs = None
        if ctx.needs_input_grad[0]:
            grad_sub = ctx.plan.adjoint((res * (-scale)).contiguous(), g_uv, g_w, uvw)
        if ctx.needs_input_grad[5]:
            grad_obs = res * scale
        return grad_sub, None, None, None, None, grad_obs


def residual_loss(subgrids, g_uv, g_w, uvw, v_obs, plan: Plan) -> torch.Tensor:
    """Fused ``sum |v_obs - degrid(subgrids)|^2`` with autograd support."""
    if subgrids.requires_grad or v_obs.requires_grad:
        return ResidualLossFn.apply(subgrids, plan, g_uv, g_w, uvw, v_obs)
    return plan.residual(subgrids, g_uv, g_w, uvw, v_obs)[1]


def degrid(subgrids, g_uv, g_w, uvw, offsets=None, plan: Plan | None = None, **plan_kw) -> torch.Tensor:
    """Degrid with autograd support (differentiable with respect to
    ``subgrids``, ``g_uv`` and ``g_w``: whichever of them require grad get
    gradients through :class:`DegridFn`).

    A plan made here gets the plan-time work order of ``uvw`` (``Plan.sort``),
    which the gridding adjoint of the backward needs to run without global
    atomics."""
    if plan is None:
        if offsets is None:
            raise ValueError("give offsets or a plan")
        s, n_v, n_u, n_w = subgrids.shape[:4]
        plan = Plan(offsets, n_v, n_u, n_w, os_uv=g_uv.shape[0], os_w=g_w.shape[0], **plan_kw)
        plan.sort(uvw)
    if torch.is_grad_enabled() and (subgrids.requires_grad or g_uv.requires_grad or g_w.requires_grad):
        return DegridFn.apply(subgrids, plan, g_uv, g_w, uvw)
    return plan.execute(subgrids, g_uv, g_w, uvw)


def grid_adjoint(vis, g_uv, g_w, uvw, offsets=None, shape=None, plan: Plan | None = None, **plan_kw):
    """Gridding (adjoint of degrid) into a new complex64 ``[S, n_v, n_u, n_w]``."""
    if plan is None:
        if offsets is None or shape is None:
            raise ValueError("give offsets and shape, or a plan")
        s, n_v, n_u, n_w = shape
        plan = Plan(offsets, n_v, n_u, n_w, os_uv=g_uv.shape[0], os_w=g_w.shape[0], **plan_kw)
        plan.sort(uvw)
    return plan.adjoint(vis, g_uv, g_w, uvw)
