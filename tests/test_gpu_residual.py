"""Fused residual and loss (NEXT row f2): res = V_obs - degrid(A) and
sum |res|^2 from one degrid pass, against the FP64 oracle, and its autograd
gradient against the oracle's gridding of the residual."""

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import workload as wl
from paper_2102_12739_amd.degrid import ResidualLossFn
from tests.gpu_common import REL_L2_FP32, announce, device, plan_for, rel_l2, upload

pytestmark = pytest.mark.gpu


def _case(seed, counts=(3000, 0, 1700, 64, 4100), n_v=72, n_u=96, with_oob=True):
    p = wl.make_problem("residual", list(counts), seed=seed, kind="mixed", n_v=n_v, n_u=n_u)
    if with_oob and p.n_vis > 20:
        # a few coordinates just outside the valid box: model 0, residual = V_obs
        p.uvw[5, 0] = 2.5
        p.uvw[11, 1] = float(n_v) - 3.5
        p.uvw[17, 2] = 3.0
    v_obs = wl.complex_noise(seed, p.n_vis, 1.0).astype(np.complex64)
    return p, v_obs


def _reference(p, v_obs):
    model, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    res = v_obs.astype(np.complex128) - model
    return res, float(np.sum(np.abs(res) ** 2)), oob


@pytest.mark.parametrize("sort", [False, True])
def test_residual_and_loss_match_oracle(sort):
    p, v_obs = _case(61)
    announce(f"residual sort={sort} N={p.n_vis}")
    t = upload(p)
    plan = plan_for(p)
    if sort:
        plan.sort(t["uvw"])
    vo = torch.from_numpy(v_obs).to(device())
    res, loss = plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], vo)
    torch.cuda.synchronize()
    ref_res, ref_loss, oob = _reference(p, v_obs)
    assert oob == 3 and plan.oob_count() == 3
    assert rel_l2(res.cpu().numpy(), ref_res) <= REL_L2_FP32
    # out-of-range visibilities: the residual is the observed value itself
    got = res.cpu().numpy()
    for i in (5, 11, 17):
        assert got[i] == v_obs[i]
    assert abs(loss.item() - ref_loss) <= 1e-6 * ref_loss


def test_loss_bits_repeat_and_in_place_gives_the_same_result():
    p, v_obs = _case(62, with_oob=False)
    announce("residual repeat / in place")
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    vo = torch.from_numpy(v_obs).to(device())
    res1, loss1 = plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], vo)
    res2, loss2 = plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], vo)
    inplace = vo.clone()
    res3, loss3 = plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], inplace, out=inplace)
    torch.cuda.synchronize()
    assert res3.data_ptr() == inplace.data_ptr()
    assert torch.equal(res1, res2) and torch.equal(res1, res3)
    assert loss1.item() == loss2.item() == loss3.item()
    # the residual pass leaves the plain degrid untouched
    vis = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    assert torch.equal(vo - vis, res1)


def test_empty_plan_writes_zero_loss():
    p, v_obs = _case(63, counts=(0, 0), n_v=32, n_u=32, with_oob=False)
    t = upload(p)
    plan = plan_for(p)
    loss = torch.full((), float("nan"), dtype=torch.float64, device=device())
    res = torch.empty(0, dtype=torch.complex64, device=device())
    plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], res, out=res, loss=loss)
    torch.cuda.synchronize()
    assert loss.item() == 0.0


def test_residual_loss_autograd_matches_oracle_gradient():
    """d/dA sum |V_obs - degrid(A)|^2 = -2 grid(res); d/dV_obs = 2 res."""
    p, v_obs = _case(64, with_oob=False)
    announce("residual autograd")
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    a = t["sub"].clone().requires_grad_(True)
    vo = torch.from_numpy(v_obs).to(device()).requires_grad_(True)
    loss = ResidualLossFn.apply(a, plan, t["g_uv"], t["g_w"], t["uvw"], vo)
    loss.backward()
    torch.cuda.synchronize()
    ref_res, ref_loss, _ = _reference(p, v_obs)
    ref_grad, _ = oracle.grid(-2.0 * ref_res, p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    assert abs(loss.item() - ref_loss) <= 1e-6 * ref_loss
    assert rel_l2(a.grad.cpu().numpy(), ref_grad) <= 1e-5
    assert rel_l2(vo.grad.cpu().numpy(), 2.0 * ref_res) <= 1e-5


def test_residual_graph_replays_match_eager():
    p, v_obs = _case(65, with_oob=False)
    announce("residual graph capture")
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    vo = torch.from_numpy(v_obs).to(device())
    res_ref, loss_ref = plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], vo)
    torch.cuda.synchronize()
    res = torch.empty_like(res_ref)
    loss = torch.empty_like(loss_ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], vo, out=res, loss=loss, stream=side)
    for k in range(3):
        res.fill_(float("nan"))
        loss.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, res_ref), f"replay {k}"
        assert loss.item() == loss_ref.item(), f"replay {k}"
        plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])   # eager work between replays
        torch.cuda.synchronize()
    del g


def test_residual_full_size_differentiation_workload():
    """16 subgrids of 512 x 512 x 4 with 2^16 uniform visibilities each; V_obs
    from the oracle on the true subgrids plus noise, evaluated at a perturbed
    point (the differentiation workload)."""
    p = wl.differentiation(seed=4)
    announce(f"residual full size N={p.n_vis}")
    v_true, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    v_obs = (v_true + wl.complex_noise(4, p.n_vis, 0.01)).astype(np.complex64)
    a_host = (p.subgrids + wl.perturbation(4, p.subgrids.shape, 0.1)).astype(np.complex64)
    t = upload(p)
    plan = plan_for(p)
    plan.sort(t["uvw"])
    a = torch.from_numpy(a_host).to(device())
    res, loss = plan.residual(a, t["g_uv"], t["g_w"], t["uvw"], torch.from_numpy(v_obs).to(device()))
    torch.cuda.synchronize()
    model, _ = oracle.degrid(a_host, p.g_uv, p.g_w, p.uvw, p.offsets)
    ref_res = v_obs.astype(np.complex128) - model
    ref_loss = float(np.sum(np.abs(ref_res) ** 2))
    assert rel_l2(res.cpu().numpy(), ref_res) <= 1e-4   # residual ~ 0.1-sized, model ~ 1-sized
    assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss
