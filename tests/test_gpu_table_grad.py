"""Gradients with respect to the GCF tables (NEXT row f3): the HIP pass through
the C ABI against the FP64 oracle on the same stored inputs, and through
torch.autograd."""

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import workload as wl
from paper_2102_12739_amd.degrid import DegridFn, degrid
from tests.gpu_common import announce, device, plan_for, rel_l2, stored_reference_inputs, upload

pytestmark = pytest.mark.gpu

# Each entry is a float32 sum, in an order that float atomics decide, of up
# to a few thousand products of float32 values; with random-sign terms the
# relative error of such a sum stays within a few float32 ulps of the terms'
# RMS, far below this bound.
REL_L2_GRAD = 1e-5


def _problem(seed, os_uv=16, os_w=16, n_w=4, counts=(1800, 0, 1100, 2500), n_v=48, n_u=64):
    p = wl.make_problem("tgrad", list(counts), seed=seed, kind="mixed", n_v=n_v, n_u=n_u, n_w=n_w,
                        os_uv=os_uv, os_w=os_w)
    if p.n_vis > 20:
        p.uvw[4, 0] = 2.5              # out of range: adds nothing
        p.uvw[13, 1] = float(n_v) - 3.5
    return p


def _oracle_grads(p, grid_dtype, gcf_dtype, g):
    sub, g_uv, g_w = stored_reference_inputs(p, grid_dtype, gcf_dtype)
    return oracle.table_grad(sub, g_uv, g_w, p.uvw, p.offsets, g)


@pytest.mark.parametrize("grid_dtype,gcf_dtype", [("c64", "f32"), ("cf16", "f16"), ("cbf16", "bf16")])
@pytest.mark.parametrize("sort", [False, True])
def test_table_grad_matches_oracle(grid_dtype, gcf_dtype, sort):
    p = _problem(150)
    announce(f"table grad {grid_dtype}/{gcf_dtype} sort={sort}")
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    if sort:
        plan.sort(t["uvw"])
    g = wl.complex_noise(150, p.n_vis, 1.0)
    gu, gw = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], torch.from_numpy(g).to(device()))
    torch.cuda.synchronize()
    ref_uv, ref_w, oob = _oracle_grads(p, grid_dtype, gcf_dtype, g)
    assert oob == 2
    assert rel_l2(gu.cpu().numpy(), ref_uv) <= REL_L2_GRAD
    assert rel_l2(gw.cpu().numpy(), ref_w) <= REL_L2_GRAD


@pytest.mark.parametrize("os_uv,os_w,n_w", [(6, 5, 4), (12, 40, 4), (16, 16, 7), (5, 64, 9), (24, 8, 4)])
def test_table_grad_general_oversampling_and_deep_stacks(os_uv, os_w, n_w):
    """Non-power-of-two oversampling, large G_w tables (os_w 40 and 64), a
    G_uv table too large for a workgroup's LDS copy (os_uv 24: every
    visibility adds straight to the output) and subgrids deeper than the w
    support."""
    p = _problem(151 + os_w, os_uv=os_uv, os_w=os_w, n_w=n_w, counts=(1500, 700, 0, 900), n_v=40, n_u=48)
    announce(f"table grad os {os_uv}/{os_w} n_w {n_w}")
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    g = wl.complex_noise(151, p.n_vis, 1.0)
    gu, gw = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], torch.from_numpy(g).to(device()))
    torch.cuda.synchronize()
    ref_uv, ref_w, _ = oracle.table_grad(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets, g)
    assert rel_l2(gu.cpu().numpy(), ref_uv) <= REL_L2_GRAD
    assert rel_l2(gw.cpu().numpy(), ref_w) <= REL_L2_GRAD


def test_table_grad_euler_identity_accumulate_and_one_table():
    """sum(G * dL/dG) = Re<g, V> for each table (V is homogeneous of degree
    one in each); accumulate adds; asking for one table leaves the other
    untouched."""
    p = _problem(152)
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    g = torch.from_numpy(wl.complex_noise(152, p.n_vis, 1.0)).to(device())
    gu, gw = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g)
    vis = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    torch.cuda.synchronize()
    re_terms = g.real.double() * vis.real.double()
    im_terms = g.imag.double() * vis.imag.double()
    loss = float(torch.sum(re_terms + im_terms))
    scale = float(torch.sum(torch.abs(re_terms) + torch.abs(im_terms)))
    assert abs(float(torch.sum(t["g_uv"].double() * gu.double())) - loss) <= 1e-5 * scale
    assert abs(float(torch.sum(t["g_w"].double() * gw.double())) - loss) <= 1e-5 * scale
    gu2, gw2 = gu.clone(), gw.clone()
    plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g, out_uv=gu2, out_w=gw2, accumulate=True)
    torch.cuda.synchronize()
    assert rel_l2(gu2.cpu().numpy(), 2.0 * gu.cpu().numpy()) <= REL_L2_GRAD
    assert rel_l2(gw2.cpu().numpy(), 2.0 * gw.cpu().numpy()) <= REL_L2_GRAD
    only_uv, none_w = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g, want_w=False)
    none_uv, only_w = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g, want_uv=False)
    torch.cuda.synchronize()
    assert none_w is None and none_uv is None
    assert rel_l2(only_uv.cpu().numpy(), gu.cpu().numpy()) <= REL_L2_GRAD
    assert rel_l2(only_w.cpu().numpy(), gw.cpu().numpy()) <= REL_L2_GRAD


def test_table_grad_through_autograd():
    """L = sum |degrid(A; G_uv, G_w) - V_obs|^2 with every input requiring a
    gradient: dL/dV = 2 (V - V_obs), and each input's gradient matches the
    oracle's."""
    p = _problem(153, counts=(2000, 1300))
    announce("table grad autograd")
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    v_obs = torch.from_numpy(wl.complex_noise(153, p.n_vis, 1.0)).to(device())
    a = t["sub"].clone().requires_grad_(True)
    g_uv = t["g_uv"].clone().requires_grad_(True)
    g_w = t["g_w"].clone().requires_grad_(True)
    vis = DegridFn.apply(a, plan, g_uv, g_w, t["uvw"])
    loss = torch.sum(torch.abs(vis - v_obs) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    assert g_uv.grad.dtype == torch.float32 and g_w.grad.dtype == torch.float32
    ref_v, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    dv = 2.0 * (ref_v - v_obs.cpu().numpy().astype(np.complex128))
    ref_uv, ref_w, _ = oracle.table_grad(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets, dv)
    ref_a, _ = oracle.grid(dv, p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    assert rel_l2(g_uv.grad.cpu().numpy(), ref_uv) <= REL_L2_GRAD
    assert rel_l2(g_w.grad.cpu().numpy(), ref_w) <= REL_L2_GRAD
    assert rel_l2(a.grad.cpu().numpy(), ref_a) <= REL_L2_GRAD


def test_functional_degrid_differentiates_tables_alone():
    """degrid() with only the tables requiring a gradient (the subgrids
    do not) still records the autograd node, and the table gradients match
    the oracle's."""
    p = _problem(156, counts=(1400, 900))
    announce("functional degrid, tables only")
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    g_uv = t["g_uv"].clone().requires_grad_(True)
    g_w = t["g_w"].clone().requires_grad_(True)
    vis = degrid(t["sub"], g_uv, g_w, t["uvw"], plan=plan)
    assert vis.grad_fn is not None
    w8 = torch.from_numpy(wl.complex_noise(156, p.n_vis, 1.0)).to(device())
    (vis.real * w8.real + vis.imag * w8.imag).sum().backward()
    torch.cuda.synchronize()
    ref_uv, ref_w, _ = oracle.table_grad(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets, w8.cpu().numpy())
    assert rel_l2(g_uv.grad.cpu().numpy(), ref_uv) <= REL_L2_GRAD
    assert rel_l2(g_w.grad.cpu().numpy(), ref_w) <= REL_L2_GRAD
    # one table only: the other gets no gradient
    g_w2 = t["g_w"].clone().requires_grad_(True)
    vis2 = degrid(t["sub"], t["g_uv"], g_w2, t["uvw"], plan=plan)
    (vis2.real * w8.real + vis2.imag * w8.imag).sum().backward()
    torch.cuda.synchronize()
    assert rel_l2(g_w2.grad.cpu().numpy(), ref_w) <= REL_L2_GRAD


def test_table_grad_bf16_tables_return_bf16_gradients():
    p = _problem(154, counts=(900, 600))
    t = upload(p, "cbf16", "bf16")
    plan = plan_for(p, grid_dtype="cbf16", gcf_dtype="bf16")
    g_uv = t["g_uv"].clone().requires_grad_(True)
    g_w = t["g_w"].clone().requires_grad_(True)
    vis = DegridFn.apply(t["sub"], plan, g_uv, g_w, t["uvw"])
    w8 = torch.from_numpy(wl.complex_noise(154, p.n_vis, 1.0)).to(device())
    (vis.real * w8.real + vis.imag * w8.imag).sum().backward()
    torch.cuda.synchronize()
    assert g_uv.grad.dtype == torch.bfloat16 and g_w.grad.dtype == torch.bfloat16
    ref_uv, ref_w, _ = _oracle_grads(p, "cbf16", "bf16", w8.cpu().numpy())
    # the float32 gradients are rounded once to bfloat16 on return: each
    # entry moves by at most 2^-9 of itself
    assert rel_l2(g_uv.grad.float().cpu().numpy(), ref_uv) <= 3e-3
    assert rel_l2(g_w.grad.float().cpu().numpy(), ref_w) <= 3e-3


def test_table_grad_empty_plan_zeroes_the_outputs():
    p = _problem(155, counts=(0, 0), n_v=32, n_u=32)
    t = upload(p)
    plan = plan_for(p)
    gu = torch.full((p.os_uv, p.os_uv, 8, 8), 3.0, dtype=torch.float32, device=device())
    gw = torch.full((p.os_w, 4), 3.0, dtype=torch.float32, device=device())
    g = torch.zeros(0, dtype=torch.complex64, device=device())
    plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g, out_uv=gu, out_w=gw)
    torch.cuda.synchronize()
    assert torch.all(gu == 0) and torch.all(gw == 0)


def test_table_grad_graph_replays_match_eager():
    """The pass (its zero fill is a kernel, not a memset) captured in a HIP
    graph: every replay, with eager work between replays, matches the eager
    result to float32 atomic-order rounding."""
    p = _problem(156, counts=(1200, 900))
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    g = torch.from_numpy(wl.complex_noise(156, p.n_vis, 1.0)).to(device())
    ref_uv, ref_w = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g)
    torch.cuda.synchronize()
    gu, gw = torch.empty_like(ref_uv), torch.empty_like(ref_w)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], g, out_uv=gu, out_w=gw, stream=side)
    for k in range(3):
        gu.fill_(float("nan"))
        gw.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert rel_l2(gu.cpu().numpy(), ref_uv.cpu().numpy()) <= REL_L2_GRAD, f"replay {k}"
        assert rel_l2(gw.cpu().numpy(), ref_w.cpu().numpy()) <= REL_L2_GRAD, f"replay {k}"
        plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])   # eager work between replays
        torch.cuda.synchronize()
    del graph


@pytest.mark.parametrize("workload,grid_dtype,gcf_dtype", [("differentiation", "c64", "f32"),
                                                          ("paper_scale", "c64", "f32"),
                                                          ("paper_scale", "cbf16", "bf16")])
def test_table_grad_full_size(workload, grid_dtype, gcf_dtype):
    """Both table gradients at full size (16 x 65 536 uniform; 64 subgrids
    with 3.17 M visibilities of uneven counts), on a sorted plan as the
    benchmark times them, against the oracle on the stored inputs."""
    p = wl.differentiation(4) if workload == "differentiation" else wl.paper_scale(1)
    announce(f"table grad full size {workload} {grid_dtype}/{gcf_dtype} ({p.n_vis} visibilities)")
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    plan.sort(t["uvw"])
    g = wl.complex_noise(157, p.n_vis, 1.0)
    gu, gw = plan.table_grad(t["sub"], t["g_uv"], t["g_w"], t["uvw"], torch.from_numpy(g).to(device()))
    torch.cuda.synchronize()
    ref_uv, ref_w, oob = _oracle_grads(p, grid_dtype, gcf_dtype, g)
    assert oob == 0
    assert rel_l2(gu.float().cpu().numpy(), ref_uv) <= REL_L2_GRAD
    assert rel_l2(gw.float().cpu().numpy(), ref_w) <= REL_L2_GRAD
