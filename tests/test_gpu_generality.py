"""Generality beyond the paper's sizes (NEXT row f3): oversampling factors that
are not powers of two, and subgrids with more w planes than the w support
(so the first w tap varies), against the FP64 oracle."""

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import workload as wl
from paper_2102_12739_amd.degrid import Batch, DegridError
from tests.gpu_common import REL_L2_FP32, announce, device, plan_for, rel_l2, stored_reference_inputs, upload

pytestmark = pytest.mark.gpu

DEEP_KERNEL = 5   # the kernel variant for subgrids deeper than the w support
D1_KERNEL = 6     # the D1-mapping variant, which also reads deeper stacks


def _edge_coords(rng, box, os_uv, os_w, n):
    """Points j / os on the quantisation lattice and one float below and above
    (where floor(c * os) of the float64 product decides the cell)."""
    out = []
    while len(out) < n:
        j = [int(rng.integers(int(np.ceil(lo * os)), int(np.floor(hi * os))))
             for lo, hi, os in zip(box.lo, box.hi, (os_uv, os_uv, os_w))]
        c = np.array([j[0] / os_uv, j[1] / os_uv, j[2] / os_w])
        for step in (None, -np.inf, np.inf):
            e = c if step is None else np.nextafter(c, step)
            if np.all(e >= box.lo) and np.all(e < box.hi):
                out.append(e)
    return np.array(out[:n])


def _problem(name, counts, seed, n_v, n_u, n_w, os_uv, os_w, edges=0):
    p = wl.make_problem(name, counts, seed=seed, kind="mixed", n_v=n_v, n_u=n_u, n_w=n_w, os_uv=os_uv, os_w=os_w)
    if edges:
        rng = np.random.default_rng(seed + 1000)
        p.uvw[:edges] = _edge_coords(rng, wl.interior_box(n_v, n_u, n_w), os_uv, os_w, edges)
    return p


def _per_vis_ok(got, ref):
    scale = np.sqrt(np.mean(np.abs(ref) ** 2))
    return np.max(np.abs(got - ref) / (np.abs(ref) + 1e-3 * scale)) <= 1e-3


@pytest.mark.parametrize("os_uv,os_w", [(3, 3), (5, 7), (12, 10), (24, 6), (6, 16)])
@pytest.mark.parametrize("sort", [False, True])
def test_non_power_of_two_oversampling_matches_oracle(os_uv, os_w, sort):
    p = _problem("os-general", [1500, 0, 900, 2100], seed=71 + os_uv, n_v=56, n_u=72, n_w=4,
                 os_uv=os_uv, os_w=os_w, edges=600)
    announce(f"oversampling {os_uv}/{os_w} sort={sort}")
    t = upload(p)
    plan = plan_for(p)
    if sort:
        plan.sort(t["uvw"])
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    assert _per_vis_ok(got, ref), "a visibility picked another tap or table row than the oracle"
    assert plan.oob_count() == oob
    vin = torch.from_numpy(wl.complex_noise(72, p.n_vis, 1.0)).to(device())
    g = plan.adjoint(vin, t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref_g, _ = oracle.grid(vin.cpu().numpy(), p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    assert rel_l2(g, ref_g) <= REL_L2_FP32


@pytest.mark.parametrize("grid_dtype,gcf_dtype", [("cbf16", "f16"), ("cf16", "f16")])
def test_non_power_of_two_oversampling_low_precision_storage(grid_dtype, gcf_dtype):
    p = _problem("os-general-lp", [2000, 700], seed=81, n_v=48, n_u=64, n_w=4, os_uv=6, os_w=5, edges=200)
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    plan.sort(t["uvw"])
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    deq = wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, grid_dtype), grid_dtype)
    ref, _ = oracle.degrid(deq, p.g_uv.astype(np.float16), p.g_w.astype(np.float16), p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


@pytest.mark.parametrize("n_w", [5, 8, 13])
@pytest.mark.parametrize("sort", [False, True])
def test_deeper_w_stacks_match_oracle(n_w, sort):
    """n_w > 4: the first w tap z0 = floor(w) - 1 varies between visibilities;
    the plan uses the deep kernel (no staging, one load per w value) and the
    adjoint scatters with atomics."""
    p = _problem("deep", [1800, 0, 1100, 2500], seed=90 + n_w, n_v=48, n_u=64, n_w=n_w, os_uv=16, os_w=8,
                 edges=300)
    announce(f"deep n_w={n_w} sort={sort}")
    t = upload(p)
    plan = plan_for(p)
    assert plan.info()["kernel"] == DEEP_KERNEL
    if sort:
        plan.sort(t["uvw"])
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    assert _per_vis_ok(got, ref)
    assert plan.oob_count() == oob
    # every w plane is used by some visibility's taps
    z0 = np.floor(p.uvw[:, 2]).astype(int) - 1
    assert z0.min() == 0 and z0.max() == n_w - 4
    vin = torch.from_numpy(wl.complex_noise(91, p.n_vis, 1.0)).to(device())
    g = plan.adjoint(vin, t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref_g, _ = oracle.grid(vin.cpu().numpy(), p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    assert rel_l2(g, ref_g) <= REL_L2_FP32
    res, loss = plan.residual(t["sub"], t["g_uv"], t["g_w"], t["uvw"], vin)
    ref_loss = float(np.sum(np.abs(vin.cpu().numpy().astype(np.complex128) - ref) ** 2))
    assert abs(loss.item() - ref_loss) <= 1e-6 * ref_loss


@pytest.mark.parametrize("grid_dtype", ["cbf16", "cf16"])
def test_deeper_w_stacks_low_precision_storage(grid_dtype):
    p = _problem("deep-lp", [1500, 900], seed=95, n_v=40, n_u=48, n_w=7, os_uv=8, os_w=16, edges=100)
    t = upload(p, grid_dtype, "f16")
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype="f16")
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    deq = wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, grid_dtype), grid_dtype)
    ref, _ = oracle.degrid(deq, p.g_uv.astype(np.float16), p.g_w.astype(np.float16), p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


def test_deep_plans_refuse_staged_kernels_and_tune_within_the_deep_one():
    p = _problem("deep-kernels", [3000], seed=97, n_v=40, n_u=40, n_w=6, os_uv=16, os_w=16)
    t = upload(p)
    plan = plan_for(p)
    with pytest.raises(DegridError) as e:
        plan.set_kernel(4, 64)
    assert e.value.status == 2
    info = plan.tune(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    assert info["kernel"] in (DEEP_KERNEL, D1_KERNEL)
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


@pytest.mark.parametrize("grid_dtype,gcf_dtype", [("c64", "f32"), ("cbf16", "bf16"), ("cf16", "f16")])
@pytest.mark.parametrize("n_b", [64, 9])
def test_d1_mapping_reads_deep_stacks(grid_dtype, gcf_dtype, n_b):
    """The D1-mapping variant reads one w value per lane, so it takes
    subgrids deeper than the w support; odd tile sizes leave the last pair
    of a tile half empty."""
    p = _problem("deep-d1", [1300, 0, 777], seed=96, n_v=40, n_u=48, n_w=9, os_uv=12, os_w=5, edges=100)
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    plan.set_kernel(D1_KERNEL, n_b)
    assert plan.info()["kernel"] == D1_KERNEL
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    sub, g_uv, g_w = stored_reference_inputs(p, grid_dtype, gcf_dtype)
    ref, oob = oracle.degrid(sub, g_uv, g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    assert plan.oob_count() == oob


def test_batch_of_a_deep_and_a_plain_problem():
    """A batch that holds a subgrid stack deeper than the w support runs the
    deep kernel for every problem; both match the oracle."""
    pa = _problem("batch-plain", [1200, 300], seed=98, n_v=48, n_u=48, n_w=4, os_uv=16, os_w=16)
    pb = _problem("batch-deep", [900, 0, 1400], seed=99, n_v=40, n_u=56, n_w=9, os_uv=12, os_w=6)
    ta, tb = upload(pa), upload(pb)
    plans = [plan_for(pa), plan_for(pb)]
    plans[0].sort(ta["uvw"])
    batch = Batch(plans)
    outs = batch.execute([(ta["sub"], ta["g_uv"], ta["g_w"], ta["uvw"]), (tb["sub"], tb["g_uv"], tb["g_w"], tb["uvw"])])
    torch.cuda.synchronize()
    for p, o in ((pa, outs[0]), (pb, outs[1])):
        ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
        assert rel_l2(o.cpu().numpy(), ref) <= REL_L2_FP32
    batch.close()
