"""GPU parity of degridding: the HIP path through the C ABI against the FP64
oracle on the same seeded inputs (Section 2 defines the operation)."""

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import workload as wl
from tests.gpu_common import REL_L2_FP32, announce, device, plan_for, rel_l2, stored_reference_inputs, upload

pytestmark = pytest.mark.gpu

D1_KERNEL = 6   # the kernel variant with the lane mapping of the paper's kernel D1


def _run(p, **plan_kw):
    """One launch into an output filled with NaN first, so that a visibility
    the launch never writes fails the comparison."""
    t = upload(p)
    plan = plan_for(p, **plan_kw)
    vis = torch.full((p.n_vis,), float("nan"), dtype=torch.complex64, device=device())
    plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"], out=vis)
    torch.cuda.synchronize()
    return plan, vis.cpu().numpy()


def test_plain_line_two_subgrids_matches_oracle():
    p = wl.plain_line(seed=0)
    announce(f"plain line S=2 N={p.n_vis}")
    plan, got = _run(p)
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref))
    assert plan.oob_count() == oob == 0


def test_paper_scale_full_size_matches_oracle():
    """64 subgrids of 512x512x4, 2^10..2^18 visibilities each (about 3.2 M), the
    launch configuration the benchmark times; every output is checked."""
    p = wl.paper_scale(seed=1)
    announce(f"paper scale S=64 N={p.n_vis}")
    plan, got = _run(p)
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    per = np.abs(got - ref) / (np.abs(ref) + 1e-3 * np.sqrt(np.mean(np.abs(ref) ** 2)))
    assert np.max(per) <= 1e-3
    assert plan.oob_count() == oob == 0
    info = plan.info()
    assert info["n_vis"] == p.n_vis and info["n_queues"] == 8


@pytest.mark.parametrize("n_b", [1, 7, 8, 33, 64])
def test_ragged_tiles_and_tile_sizes(n_b):
    counts = [0, 1, 63, 64, 65, 1000, 7]
    p = wl.make_problem("ragged", counts, seed=11, kind="mixed", n_v=40, n_u=72)
    announce(f"ragged n_b={n_b}")
    plan, got = _run(p, n_b=n_b)
    assert plan.info()["n_b"] == n_b
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    # the tile size changes the work split only, never a visibility's sum
    _, got64 = _run(p, n_b=64)
    assert np.array_equal(got, got64)


@pytest.mark.parametrize("os_uv,os_w", [(1, 1), (2, 8), (8, 2), (32, 32), (64, 4)])
def test_oversampling_factors(os_uv, os_w):
    p = wl.make_problem("os", [300, 211], seed=12, kind="uniform", n_v=24, n_u=40,
                        os_uv=os_uv, os_w=os_w)
    announce(f"oversampling {os_uv}/{os_w}")
    plan, got = _run(p)
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


def test_random_nonseparable_tables_and_nonsquare_subgrids():
    rng = np.random.default_rng(13)
    p = wl.make_problem("rand-tables", [500, 500, 500], seed=13, kind="uniform", n_v=20, n_u=56,
                        os_uv=8, os_w=4)
    p.g_uv = wl.random_gcf_uv(rng, 8)
    p.g_w = wl.random_gcf_w(rng, 4)
    announce("random tables")
    _, got = _run(p)
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


def test_delta_subgrid_picks_the_oracle_tap_at_oversample_boundaries():
    """Coordinates at j/os and one float64 ulp below: the GPU's float64 index
    conversion must choose the same cell and table entry as the oracle."""
    rng = np.random.default_rng(14)
    os_uv = os_w = 16
    n_v, n_u, n_w = 32, 32, 4
    g_uv = wl.random_gcf_uv(rng, os_uv)
    g_w = wl.random_gcf_w(rng, os_w)
    n = 256
    ju = rng.integers(3 * os_uv + 1, 28 * os_uv, n)
    jv = rng.integers(3 * os_uv + 1, 28 * os_uv, n)
    jw = rng.integers(os_w + 1, 2 * os_w, n)
    on = np.stack([ju / os_uv, jv / os_uv, jw / os_w], 1)
    uvw = np.concatenate([on, np.nextafter(on, -np.inf)])
    sub = np.zeros((1, n_v, n_u, n_w), np.complex64)
    sub[0, 10:22, 10:22, :] = rng.standard_normal((12, 12, 4)).astype(np.float32)
    p = wl.Problem("boundaries", n_v, n_u, n_w, os_uv, os_w, np.array([0, 2 * n]), uvw, g_uv, g_w, sub)
    announce("oversample boundaries")
    _, got = _run(p)
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    scale = np.abs(ref) + 1e-6
    assert np.max(np.abs(got - ref) / scale) <= 1e-4


def test_out_of_range_visibilities_are_zero_and_counted():
    n_v = n_u = 512
    good = [3.0, np.nextafter(508.0, 0.0), 255.5]
    bad = [np.nextafter(3.0, 0.0), 508.0, -1.0, 1e300, np.nan, np.inf, -np.inf]
    rows, valid = [], []
    for u in good + bad:
        rows.append((u, 100.25, 1.5)); valid.append(u in good)
        rows.append((100.25, u, 1.5)); valid.append(u in good)
    for w in [1.0, np.nextafter(2.0, 0.0), np.nextafter(1.0, 0.0), 2.0, np.nan]:
        rows.append((100.25, 100.25, w)); valid.append(w in (1.0, np.nextafter(2.0, 0.0)))
    uvw = np.array(rows)
    sub = np.ones((1, n_v, n_u, 4), np.complex64)
    p = wl.Problem("oob", n_v, n_u, 4, 16, 16, np.array([0, len(rows)]), uvw, wl.gcf_uv(16), wl.gcf_w(16), sub)
    announce("out of range")
    plan, got = _run(p)
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    valid = np.array(valid)
    assert plan.oob_count() == oob == int(np.sum(~valid))
    assert np.all(got[~valid] == 0)
    assert rel_l2(got, ref) <= REL_L2_FP32


def test_empty_problem_and_empty_subgrids():
    p = wl.make_problem("empty", [0, 0, 0], seed=15, kind="uniform", n_v=16, n_u=16)
    announce("empty")
    plan, got = _run(p)
    assert got.shape == (0,) and plan.info()["n_tiles"] == 0 and plan.oob_count() == 0


def test_single_visibility_and_last_subgrid_only():
    p = wl.make_problem("single", [0, 0, 1], seed=16, kind="uniform", n_v=16, n_u=16)
    _, got = _run(p)
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


def test_repeated_launches_reset_the_queue_and_counts():
    p = wl.make_problem("repeat", [2000, 1500, 3], seed=17, kind="mixed", n_v=64, n_u=64)
    p.uvw[5] = (np.nan, 10.0, 1.5)
    t = upload(p)
    plan = plan_for(p)
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    first = None
    for _ in range(5):
        out = torch.full((p.n_vis,), float("nan"), dtype=torch.complex64, device=device())
        plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"], out=out)
        got = out.cpu().numpy()
        assert rel_l2(got, ref) <= REL_L2_FP32
        assert plan.oob_count() == oob == 1
        if first is None:
            first = got
        assert np.array_equal(got, first)


def test_non_default_stream():
    p = wl.make_problem("stream", [777, 1234], seed=18, kind="mixed", n_v=48, n_u=48)
    t = upload(p)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        plan = plan_for(p)
        vis = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    s.synchronize()
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(vis.cpu().numpy(), ref) <= REL_L2_FP32


def test_argument_checks_raise():
    from paper_2102_12739_amd.degrid import DegridError
    p = wl.make_problem("args", [10], seed=19, kind="uniform", n_v=16, n_u=16)
    t = upload(p)
    plan = plan_for(p)
    with pytest.raises(ValueError):
        plan.execute(t["sub"][:, :8], t["g_uv"], t["g_w"], t["uvw"])
    with pytest.raises(TypeError):
        plan.execute(t["sub"], t["g_uv"].double(), t["g_w"], t["uvw"])
    import ctypes
    from paper_2102_12739_amd.degrid import lib
    assert lib().degrid_execute(plan.handle, 0, 1, 1, 1, 1, None) == 1
    del DegridError


def test_injected_allocation_failure(monkeypatch):
    from paper_2102_12739_amd.degrid import DegridError
    monkeypatch.setenv("DG_FAULT_INJECT", "alloc")
    p = wl.make_problem("nomem", [10], seed=20, kind="uniform", n_v=16, n_u=16)
    with pytest.raises(DegridError) as e:
        plan_for(p)
    assert e.value.status == 3


def test_sorted_work_order_gives_identical_outputs_at_full_size():
    """degrid_plan_sort reorders the work (Hilbert order of cells); every visibility
    keeps its own sum, so outputs are bitwise those of the input order."""
    p = wl.paper_scale(seed=1)
    announce("sorted work order, paper scale")
    t = upload(p)
    plan = plan_for(p)
    plain = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    plan.sort(t["uvw"])
    assert plan.info()["sorted"] == 1
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    assert np.array_equal(got, plain)
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32
    plan.sort(None)
    assert plan.info()["sorted"] == 0
    again = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    assert np.array_equal(again, plain)


def test_sorted_work_order_with_out_of_range_and_empty_subgrids():
    p = wl.make_problem("sorted-oob", [0, 900, 0, 1, 700, 0], seed=24, kind="mixed", n_v=40, n_u=48)
    p.uvw[3] = (np.nan, 20.0, 1.5)
    p.uvw[10] = (-5.0, 20.0, 1.5)
    p.uvw[905] = (70000.0, 20.0, 1.5)
    t = upload(p)
    plan = plan_for(p, n_b=16)
    plan.sort(t["uvw"])
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert plan.oob_count() == oob == 3
    assert rel_l2(got, ref) <= REL_L2_FP32
    assert got[3] == 0 and got[10] == 0 and got[905] == 0


@pytest.mark.parametrize("grid_dtype,gcf_dtype", [("c64", "f32"), ("cbf16", "f16"), ("cf16", "f32"), ("cf16", "f16"),
                                                 ("cbf16", "bf16")])
def test_every_kernel_variant_gives_the_same_outputs(grid_dtype, gcf_dtype):
    """The variants with the tap-per-lane mapping differ only in where a
    tile's cells are read from (LDS copy of the tile's bounding box, or the
    caches); each visibility's arithmetic is the same, so their outputs are
    bitwise equal, sorted or not, dense or sparse. The D1 variant sums in
    another order (along v first): its outputs are bitwise equal among
    themselves and match the oracle to the float32 bar."""
    p = wl.make_problem("variants", [6000, 40, 0, 3000, 1], seed=26, kind="mixed", n_v=80, n_u=112,
                        os_uv=8, os_w=16)
    p.uvw[7] = (np.nan, 1.0, 1.5)
    t = upload(p, grid_dtype, gcf_dtype)
    plan = plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype)
    n_var = plan.info()["n_kernels"]
    assert n_var >= 2
    outs, outs_d1 = [], []
    for sort in (False, True):
        if sort:
            plan.sort(t["uvw"])
        for k in range(n_var):
            for n_b in (64, 13):
                plan.set_kernel(k, n_b)
                assert plan.info()["kernel"] == k
                o = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
                (outs_d1 if k == D1_KERNEL else outs).append(o)
                assert plan.oob_count() == 1
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    for o in outs_d1[1:]:
        assert np.array_equal(o, outs_d1[0])
    sub, g_uv, g_w = stored_reference_inputs(p, grid_dtype, gcf_dtype)
    ref, _ = oracle.degrid(sub, g_uv, g_w, p.uvw, p.offsets)
    assert rel_l2(outs[0], ref) <= REL_L2_FP32
    assert rel_l2(outs_d1[0], ref) <= REL_L2_FP32
    assert outs[0][7] == 0 and outs_d1[0][7] == 0
    with pytest.raises(Exception):
        plan.set_kernel(n_var, 0)


@pytest.mark.parametrize("sort", [False, True])
def test_graph_captured_degrid_and_adjoint_replays_match_eager(sort):
    """Degrid and its adjoint recorded into one HIP graph through stream
    capture: every replay (with eager work and synchronisations between
    replays) reproduces the eager results."""
    p = wl.make_problem("graph", [3000, 0, 777, 4100], seed=31, kind="mixed", n_v=64, n_u=80)
    announce(f"graph capture sort={sort}")
    t = upload(p)
    plan = plan_for(p)
    if sort:
        plan.sort(t["uvw"])
    vin = torch.from_numpy(wl.complex_noise(31, p.n_vis, 1.0)).to(device())
    vis_ref = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    adj_ref = plan.adjoint(vin, t["g_uv"], t["g_w"], t["uvw"])
    torch.cuda.synchronize()
    vis = torch.empty_like(vis_ref)
    adj = torch.empty_like(adj_ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"], out=vis, stream=side)
        plan.adjoint(vin, t["g_uv"], t["g_w"], t["uvw"], out=adj, stream=side)
    ref_adj, _ = oracle.grid(vin.cpu().numpy(), p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    for k in range(3):
        vis.fill_(float("nan"))
        adj.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(vis, vis_ref), f"replay {k}: degrid differs from eager"
        assert rel_l2(adj.cpu().numpy(), ref_adj) <= REL_L2_FP32, f"replay {k}: adjoint"
        if sort:   # owner-computes gridding is deterministic
            assert torch.equal(adj, adj_ref), f"replay {k}: adjoint differs from eager"
        # eager work between replays
        plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
        torch.cuda.synchronize()
    del g


def test_largest_supported_subgrid():
    """One subgrid of 4096 x 8184 x 4 complex64, just under the 1 GiB limit
    per subgrid, so that byte offsets reach the top of the 32-bit buffer
    offsets: visibilities spread over the whole subgrid plus the four
    corners of the valid box and points just outside it, against the oracle
    in input order and sorted, and the adjoint (atomic scatter: 8184 is not
    a multiple of the owner block)."""
    n_v, n_u = 4096, 8184
    assert n_v * n_u * 4 * 8 < 1 << 30
    p = wl.make_problem("largest", [12000], seed=27, kind="mixed", n_v=n_v, n_u=n_u)
    box = wl.interior_box(n_v, n_u, 4)
    eps = 1e-6
    corners = [(box.lo[0], box.lo[1], box.lo[2]), (box.hi[0] - eps, box.hi[1] - eps, box.hi[2] - eps),
               (box.lo[0], box.hi[1] - eps, box.lo[2]), (box.hi[0] - eps, box.lo[1], box.hi[2] - eps),
               (box.hi[0], box.hi[1] - eps, box.lo[2]), (box.lo[0], box.hi[1], box.lo[2])]   # last two: just outside
    p.uvw[:len(corners)] = np.array(corners)
    announce(f"largest subgrid {n_v}x{n_u}x4, N={p.n_vis}")
    t = upload(p)
    plan = plan_for(p)
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert oob == 2
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    assert plan.oob_count() == 2
    assert rel_l2(got, ref) <= REL_L2_FP32
    assert np.all(got[4:6] == 0)
    scale = float(np.max(np.abs(ref)))
    assert np.max(np.abs(got[:4] - ref[:4])) <= 1e-5 * scale
    plan.sort(t["uvw"])
    got_s = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    assert np.array_equal(got_s, got)
    vin = wl.complex_noise(27, p.n_vis, 1.0)
    g = plan.adjoint(torch.from_numpy(vin).to(device()), t["g_uv"], t["g_w"], t["uvw"])
    ref_g, _ = oracle.grid(vin, p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    assert rel_l2(g.cpu().numpy(), ref_g) <= REL_L2_FP32
    del t, g
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n_v,n_u", [(16, 65536), (65536, 16)])
def test_widest_and_tallest_subgrids_at_the_start_cell_limit(n_v, n_u):
    """Subgrids as wide (or as tall) as the 16-bit first-tap packing allows,
    with points at the far corners of the valid box: degridding in input
    order and in the Hilbert work order (whose keys then reach the top of
    their 16-bit coordinate range) against the oracle, and the adjoint on
    the sorted plan (owner-computes: both sides are multiples of the 16-cell
    block, so the block lists reach block index 4095) against the oracle and
    bitwise repeatable."""
    p = wl.make_problem("edge", [5000, 3000], seed=31, kind="mixed", n_v=n_v, n_u=n_u)
    box = wl.interior_box(n_v, n_u, 4)
    eps = 1e-9
    corners = [(box.hi[0] - eps, box.hi[1] - eps, box.lo[2]), (box.lo[0], box.hi[1] - eps, box.hi[2] - eps),
               (box.hi[0] - eps, box.lo[1], box.lo[2]), (box.hi[0] - 0.5, box.hi[1] - 0.5, box.hi[2] - eps)]
    p.uvw[:len(corners)] = np.array(corners)
    p.uvw[5000:5000 + len(corners)] = np.array(corners)
    announce(f"edge subgrids {n_v}x{n_u}x4, N={p.n_vis}")
    t = upload(p)
    plan = plan_for(p)
    ref, oob = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert oob == 0
    got = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    assert rel_l2(got, ref) <= REL_L2_FP32
    scale = float(np.max(np.abs(ref)))
    for i in list(range(len(corners))) + list(range(5000, 5000 + len(corners))):
        assert abs(got[i] - ref[i]) <= 1e-5 * scale, i
    plan.sort(t["uvw"])
    assert np.array_equal(plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy(), got)
    vin = torch.from_numpy(wl.complex_noise(31, p.n_vis, 1.0)).to(device())
    g1 = plan.adjoint(vin, t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    g2 = plan.adjoint(vin, t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    assert np.array_equal(g1, g2)
    ref_g, _ = oracle.grid(vin.cpu().numpy(), p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
    assert rel_l2(g1, ref_g) <= REL_L2_FP32
    del t
    torch.cuda.empty_cache()
