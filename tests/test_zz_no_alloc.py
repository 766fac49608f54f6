"""degrid_execute_noalloc (the entry point that allocates nothing) through
the C ABI, against degrid_execute on a plan in input order and against the
FP64 oracle: two calls in a row on one GPU, the second with a smaller
input, into outputs filled with NaN first; 16-bit storage and deep w-stacks;
the out-of-range count; and the refusal of more subgrids than its static
scratch holds."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import degrid as dgm
from paper_2102_12739_amd import workload as wl
from tests.gpu_common import REL_L2_FP32, announce, device, plan_for, rel_l2, stored_reference_inputs, upload


def _noalloc_raw(p, t, out, oob, grid_dtype="c64", gcf_dtype="f32", n_b=0):
    d = dgm.DgDesc(p.n_v, p.n_u, p.n_w, 8, 4, p.os_uv, p.os_w, dgm.GRID_DTYPES[grid_dtype],
                   dgm.GCF_DTYPES[gcf_dtype], n_b, 0)
    off = np.ascontiguousarray(p.offsets, dtype=np.int64)
    st = dgm.lib().degrid_execute_noalloc(
        ctypes.byref(d), off.size - 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        t["sub"].data_ptr(), t["g_uv"].data_ptr(), t["g_w"].data_ptr(), t["uvw"].data_ptr(), out.data_ptr(),
        oob.data_ptr() if oob is not None else None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


def _problem(seed, counts, n_v=48, n_u=64, n_w=4, os_uv=16, os_w=16):
    p = wl.make_problem("noalloc", list(counts), seed=seed, kind="mixed", n_v=n_v, n_u=n_u, n_w=n_w,
                        os_uv=os_uv, os_w=os_w)
    if p.n_vis > 40:
        p.uvw[3, 0] = 2.5                      # out of range
        p.uvw[17, 1] = float(n_v) - 3.5        # out of range
        p.uvw[29, 2] = float("nan")            # out of range
    return p


def _check_against_plan(p, grid_dtype="c64", gcf_dtype="f32", n_b=0):
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    ref = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    out = torch.full((p.n_vis,), float("nan"), dtype=torch.complex64, device=device())
    oob = torch.full((), -7, dtype=torch.int64, device=device())
    assert _noalloc_raw(p, t, out, oob, grid_dtype, gcf_dtype, n_b) == 0, dgm.lib().degrid_last_error()
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.all(np.isfinite(got)), "an output was not written"
    assert rel_l2(got, ref.cpu().numpy()) <= REL_L2_FP32
    assert int(oob.item()) == plan.oob_count()
    sub, g_uv, g_w = stored_reference_inputs(p, grid_dtype, gcf_dtype)
    ref_o, oob_o = oracle.degrid(sub, g_uv, g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref_o) <= REL_L2_FP32
    assert int(oob.item()) == oob_o
    plan.close()
    return got


@pytest.mark.gpu
def test_noalloc_two_calls_in_a_row_second_smaller():
    announce("noalloc: large then small")
    big = _problem(301, (2600, 0, 700, 1333, 5, 64, 4100))
    small = _problem(302, (90, 0, 33))
    _check_against_plan(big)
    _check_against_plan(small)
    # and once more the larger one: nothing of the previous call's scratch
    # (tile cursor, offsets) carries over
    _check_against_plan(big)


@pytest.mark.gpu
@pytest.mark.parametrize("grid_dtype,gcf_dtype", [("cbf16", "bf16"), ("cf16", "f32")])
def test_noalloc_16_bit_storage(grid_dtype, gcf_dtype):
    announce(f"noalloc: {grid_dtype}/{gcf_dtype}")
    _check_against_plan(_problem(303, (1500, 300, 0, 64)), grid_dtype, gcf_dtype)


@pytest.mark.gpu
def test_noalloc_deep_w_stack_and_other_tile_sizes():
    announce("noalloc: n_w 7, n_b 1/17")
    p = _problem(304, (700, 0, 260), n_w=7, os_uv=12, os_w=5)
    _check_against_plan(p)
    q = _problem(305, (300, 41))
    for nb in (1, 17):
        _check_against_plan(q, n_b=nb)


@pytest.mark.gpu
def test_noalloc_without_visibilities_and_without_count():
    p = _problem(306, (0, 0))
    t = upload(p)
    out = torch.empty(0, dtype=torch.complex64, device=device())
    oob = torch.full((), 5, dtype=torch.int64, device=device())
    assert _noalloc_raw(p, t, out, oob) == 0
    torch.cuda.synchronize()
    assert int(oob.item()) == 0
    q = _problem(307, (120,))
    tq = upload(q)
    out = torch.full((q.n_vis,), float("nan"), dtype=torch.complex64, device=device())
    assert _noalloc_raw(q, tq, out, None) == 0
    torch.cuda.synchronize()
    ref, _ = oracle.degrid(q.subgrids, q.g_uv, q.g_w, q.uvw, q.offsets)
    assert rel_l2(out.cpu().numpy(), ref) <= REL_L2_FP32


def test_noalloc_refuses_more_subgrids_than_its_scratch_holds():
    """Checked on the host before any device work (runs without a GPU)."""
    if not __import__("os").path.exists(dgm.library_path()):
        from paper_2102_12739_amd import build
        build.build()
    d = dgm.DgDesc(16, 16, 4, 8, 4, 16, 16, 0, 0, 0, 0)
    off = np.zeros(16386, dtype=np.int64)
    st = dgm.lib().degrid_execute_noalloc(ctypes.byref(d), 16385, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                          1, 1, 1, 1, 1, None, None)
    assert st == 2
    assert "16384" in dgm.lib().degrid_last_error().decode()
