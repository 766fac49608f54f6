"""Pointer alignment at the C ABI: tables read as whole 32-bit words must sit
on a 4-byte boundary (a misaligned one is refused before any launch), and any
4-byte aligned placement gives the same bits as a fresh allocation."""

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import workload as wl
from paper_2102_12739_amd.degrid import DegridError
from tests.gpu_common import REL_L2_FP32, announce, device, plan_for, rel_l2, upload

pytestmark = pytest.mark.gpu

INVALID_ARG = 1


def _shifted(t: torch.Tensor, elems: int) -> torch.Tensor:
    """A contiguous copy of t that starts `elems` elements into a larger buffer."""
    buf = torch.zeros(t.numel() + elems, dtype=t.dtype, device=t.device)
    view = buf[elems:].view(t.shape)
    view.copy_(t)
    return view


def _problem(seed):
    return wl.make_problem("align", [900, 0, 1300], seed=seed, kind="mixed", n_v=40, n_u=48)


@pytest.mark.parametrize("gcf_dtype,grid_dtype", [("f16", "cf16"), ("f16", "cbf16"), ("f32", "c64")])
def test_word_aligned_tables_at_any_placement_give_the_same_bits(gcf_dtype, grid_dtype):
    p = _problem(101)
    announce(f"alignment {grid_dtype}/{gcf_dtype}")
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    plan.sort(t["uvw"])
    ref = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    words = 2 if gcf_dtype == "f16" else 1      # elements per 4 bytes
    for shift in (words, 3 * words):            # 4 and 12 bytes past a 16-byte boundary
        g_w = _shifted(t["g_w"], shift)
        g_uv = _shifted(t["g_uv"], shift)
        got = plan.execute(t["sub"], g_uv, g_w, t["uvw"])
        torch.cuda.synchronize()
        assert torch.equal(got, ref), f"shift {shift}"
    if grid_dtype != "c64":
        deq = wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, grid_dtype), grid_dtype)
        want, _ = oracle.degrid(deq, p.g_uv.astype(np.float16), p.g_w.astype(np.float16), p.uvw, p.offsets)
    else:
        want, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(ref.cpu().numpy(), want) <= REL_L2_FP32


def test_half_word_aligned_g_w_is_refused():
    p = _problem(102)
    t = upload(p, "cf16", "f16")
    plan = plan_for(p, grid_dtype="cf16", gcf_dtype="f16")
    g_w = _shifted(t["g_w"], 1)                 # 2 bytes past a word boundary
    with pytest.raises(DegridError) as e:
        plan.execute(t["sub"], t["g_uv"], g_w, t["uvw"])
    assert e.value.status == INVALID_ARG
    assert "g_w" in str(e.value)
    with pytest.raises(DegridError) as e:
        plan.adjoint(torch.zeros(p.n_vis, dtype=torch.complex64, device=device()), t["g_uv"], g_w, t["uvw"])
    assert e.value.status == INVALID_ARG
    # the refused calls launched nothing: the next call is unaffected
    vis = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    torch.cuda.synchronize()
    deq = wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, "cf16"), "cf16")
    want, _ = oracle.degrid(deq, p.g_uv.astype(np.float16), p.g_w.astype(np.float16), p.uvw, p.offsets)
    assert rel_l2(vis.cpu().numpy(), want) <= REL_L2_FP32


def test_misaligned_pointers_are_refused_at_the_c_abi():
    """torch keeps float64 and complex64 views element-aligned, so the raw
    pointers are offset here by hand; the library refuses them before any
    launch."""
    from paper_2102_12739_amd.degrid import lib
    p = _problem(103)
    t = upload(p)
    plan = plan_for(p)
    out = torch.empty(p.n_vis, dtype=torch.complex64, device=device())
    args = [t["sub"].data_ptr(), t["g_uv"].data_ptr(), t["g_w"].data_ptr(), t["uvw"].data_ptr(), out.data_ptr()]
    names = ["subgrids", "g_uv", "g_w", "uvw", "visibility"]
    for k, (name, shift) in enumerate(zip(names, (4, 2, 2, 4, 4))):
        bad = list(args)
        bad[k] += shift
        st = lib().degrid_execute(plan._handle, *bad, None)
        assert st == INVALID_ARG, name
        assert name in lib().degrid_last_error().decode()
    assert lib().degrid_execute(plan._handle, *args, None) == 0
    torch.cuda.synchronize()
    want, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(out.cpu().numpy(), want) <= REL_L2_FP32
