"""Batched degridding (row a7): several independent problems in one
persistent launch replayed from a HIP graph; and the tile-size tuner."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2102_12739_amd import workload as wl
from paper_2102_12739_amd.degrid import Batch, DegridError, Plan
from tests.gpu_common import REL_L2_FP32, announce, device, plan_for, rel_l2, upload

pytestmark = pytest.mark.gpu

D1_KERNEL = 6   # the kernel variant with the lane mapping of the paper's kernel D1


def _small_batch(seed=41):
    return wl.batched(seed=seed, n_problems=8, s_range=(1, 6), exp_range=(4, 11), n_v=64, n_u=96)


def test_batch_equals_separate_runs_and_oracle_over_replays():
    probs = _small_batch()
    announce("batch small: " + ", ".join(f"S={p.n_subgrids} os={p.os_uv} N={p.n_vis}" for p in probs))
    ts = [upload(p) for p in probs]
    plans = [plan_for(p, n_b=n_b) for p, n_b in zip(probs, [64, 32, 1, 7, 64, 16, 8, 64])]
    singles = [pl.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy() for pl, t in zip(plans, ts)]
    refs = [oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)[0] for p in probs]
    batch = Batch(plans)
    args = [(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts]
    outs = [torch.full((p.n_vis,), float("nan"), dtype=torch.complex64, device=device()) for p in probs]
    for replay in range(4):
        for o in outs:
            o.fill_(float("nan"))          # eager work between replays
        batch.execute(args, outs=outs)
        torch.cuda.synchronize()
        for i, (o, single, ref) in enumerate(zip(outs, singles, refs)):
            got = o.cpu().numpy()
            assert np.array_equal(got, single), (replay, i)
            assert rel_l2(got, ref) <= REL_L2_FP32
    assert batch.oob_count() == 0


def test_batch_pointer_change_reuploads_arguments():
    probs = _small_batch(seed=42)
    ts = [upload(p) for p in probs]
    plans = [plan_for(p) for p in probs]
    batch = Batch(plans)
    args = [(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts]
    first = [o.cpu().numpy() for o in batch.execute(args)]
    # new subgrid contents in new buffers, new outputs
    args2 = [(t["sub"] * 2, t["g_uv"], t["g_w"], t["uvw"]) for t in ts]
    second = [o.cpu().numpy() for o in batch.execute(args2)]
    torch.cuda.synchronize()
    for a, b in zip(first, second):
        np.testing.assert_allclose(b, 2 * a, rtol=1e-6, atol=1e-6)


def test_batch_counts_out_of_range_over_all_problems():
    probs = _small_batch(seed=43)
    probs[2].uvw[0] = (np.nan, 5.0, 1.5)
    probs[5].uvw[-1] = (1e9, 5.0, 1.5)
    ts = [upload(p) for p in probs]
    batch = Batch([plan_for(p) for p in probs])
    batch.execute([(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts])
    assert batch.oob_count() == 2


def test_batch_rejects_mixed_storage_dtypes():
    probs = _small_batch(seed=44)[:2]
    plans = [plan_for(probs[0]), plan_for(probs[1], grid_dtype="cbf16")]
    with pytest.raises(DegridError):
        Batch(plans)


def test_batched_workload_full_size():
    """Eight problems with S in 4..64, counts log-uniform in [2^8, 2^18] and
    os in {8, 16, 32}, all in one launch; every output against the oracle."""
    probs = wl.batched(seed=2)
    announce("batch full: " + ", ".join(f"S={p.n_subgrids} os={p.os_uv} N={p.n_vis}" for p in probs))
    ts = [upload(p) for p in probs]
    plans = [plan_for(p) for p in probs]
    batch = Batch(plans)
    outs = batch.execute([(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts])
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
        assert rel_l2(o.cpu().numpy(), ref) <= REL_L2_FP32
    del ts


def test_tuner_keeps_results_and_caches_choice(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DG_TUNE_CACHE", str(cache))
    p = wl.make_problem("tune", [20000, 3000, 100], seed=45, kind="mixed")
    t = upload(p)
    plan = plan_for(p)
    before = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    info = plan.tune(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    assert info["n_b"] in (8, 16, 32, 64)
    after = plan.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    if info["kernel"] == D1_KERNEL:   # sums in another order: equal to float32 rounding
        assert rel_l2(after, before) <= REL_L2_FP32
    else:
        assert np.array_equal(before, after)
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(after, ref) <= REL_L2_FP32
    assert cache.exists() and cache.read_text().strip()
    again = plan_for(p)            # n_b = 0: the cached choice is used
    assert again.info()["n_b"] == info["n_b"] and again.info()["kernel"] == info["kernel"]
    assert again.info()["grid_blocks"] == info["grid_blocks"]


def test_tune_cache_choices_are_used_only_on_their_own_device(tmp_path, monkeypatch):
    """A cache line names the device (architecture and CU count) it was
    timed on: a choice recorded for another device is ignored, the same
    choice under this device's key is taken (kernel, tile size and the
    half-occupancy grid)."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("DG_TUNE_CACHE", str(cache))
    p = wl.make_problem("tune-key", [60000, 30000], seed=47, kind="mixed")
    t = upload(p)
    plan = plan_for(p)
    default = plan.info()
    plan.tune(t["sub"], t["g_uv"], t["g_w"], t["uvw"])
    key = cache.read_text().splitlines()[-1].split()[0]
    dev_key, sep, rest = key.partition("_grid")
    assert sep and "cu" in dev_key
    choice = (2, 24)   # a choice the library makes by itself for no problem
    other = "gfx000-none_1cu" + sep + rest
    cache.write_text(f"{other} {choice[1]} {choice[0]} 2\n")
    ignored = plan_for(p).info()
    assert (ignored["kernel"], ignored["n_b"]) == (default["kernel"], default["n_b"])
    cache.write_text(f"{other} 8 0 1\n{key} {choice[1]} {choice[0]} 2\n")
    taken = plan_for(p)
    info = taken.info()
    assert (info["kernel"], info["n_b"]) == choice
    full = plan_for(p, n_b=choice[1])
    full.set_kernel(choice[0], choice[1])
    assert info["grid_blocks"] <= (full.info()["grid_blocks"] + 1) // 2 + 1
    got = taken.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy()
    ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
    assert rel_l2(got, ref) <= REL_L2_FP32


def test_batch_of_sorted_plans_and_stale_batch_is_refused():
    probs = _small_batch(seed=46)
    ts = [upload(p) for p in probs]
    plans = [plan_for(p) for p in probs]
    stale = Batch(plans)
    for pl, t in zip(plans, ts):
        pl.sort(t["uvw"])
    args = [(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts]
    with pytest.raises(DegridError) as e:
        stale.execute(args)
    assert e.value.status == 5
    batch = Batch(plans)
    outs = batch.execute(args)
    torch.cuda.synchronize()
    for p, o in zip(probs, outs):
        ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
        assert rel_l2(o.cpu().numpy(), ref) <= REL_L2_FP32


def test_batch_tuner_picks_a_candidate_and_keeps_results():
    """The batch autotuner times (kernel variant, tile size) candidates on one
    launch of the whole batch; the batch built after it reproduces the
    untuned outputs bit for bit (neither choice changes a visibility's sum),
    and a batch planned before tuning is refused as stale."""
    from paper_2102_12739_amd.degrid import batch_tune
    probs = _small_batch(seed=44)
    announce("batch tuner: " + ", ".join(f"S={p.n_subgrids} N={p.n_vis}" for p in probs))
    ts = [upload(p) for p in probs]
    plans = [plan_for(p) for p in probs]
    for pl, t in zip(plans, ts):
        pl.sort(t["uvw"])
    args = [(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts]
    before = Batch(plans)
    want = [o.cpu().numpy() for o in before.execute(args)]
    kernel, n_b = batch_tune(plans, args)
    n_kernels = plans[0].info()["n_kernels"]
    assert 0 <= kernel < n_kernels and n_b in (8, 16, 32, 64)
    for pl in plans:
        info = pl.info()
        assert info["kernel"] == kernel and info["n_b"] == n_b and info["sorted"] == 1
    with pytest.raises(DegridError):
        before.execute(args)
    before.close()
    after = Batch(plans)
    got = [o.cpu().numpy() for o in after.execute(args)]
    torch.cuda.synchronize()
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    after.close()


@pytest.mark.parametrize("grid_dtype,gcf_dtype", [("cbf16", "bf16"), ("cf16", "f16")])
def test_batched_workload_16_bit_forms_full_size(grid_dtype, gcf_dtype):
    """The batched workload (eight problems, os in {8, 16, 32}) stored in a
    16-bit form whose w sums run on the packed dot products, tuned and
    launched as one batch: every output against the oracle on the stored
    inputs (float32 accumulation), and within the 16-bit bound of the FP32
    inputs."""
    from paper_2102_12739_amd.degrid import batch_tune
    from tests.gpu_common import stored_reference_inputs
    probs = wl.batched(seed=2)
    announce(f"batch full {grid_dtype}/{gcf_dtype}")
    ts = [upload(p, grid_dtype, gcf_dtype) for p in probs]
    plans = [plan_for(p, grid_dtype=grid_dtype, gcf_dtype=gcf_dtype) for p in probs]
    for pl, t in zip(plans, ts):
        pl.sort(t["uvw"])
    args = [(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts]
    batch_tune(plans, args)
    batch = Batch(plans)
    outs = batch.execute(args)
    torch.cuda.synchronize()
    err = [0.0, 0.0]
    for p, o in zip(probs, outs):
        got = o.cpu().numpy()
        sub, g_uv, g_w = stored_reference_inputs(p, grid_dtype, gcf_dtype)
        ref_q, _ = oracle.degrid(sub, g_uv, g_w, p.uvw, p.offsets)
        assert rel_l2(got, ref_q) <= REL_L2_FP32
        ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
        err[0] += float(np.sum(np.abs(got - ref) ** 2))
        err[1] += float(np.sum(np.abs(ref) ** 2))
    # three bf16 roundings (storage, both tables), or fp16 ones
    assert (err[0] / err[1]) ** 0.5 <= (3e-3 if grid_dtype == "cbf16" else 1e-3)
    batch.close()
    del ts


def test_batch_led_by_a_tiny_plan_runs_its_largest_plans_kernel():
    """A tiny first plan (2048 visibilities: its default is the cache gather)
    batched with a large sorted plan (fitted tiles for the staged gather):
    the batch runs the large plan's kernel over both, and every output equals
    its plan's own launch bit for bit and the oracle."""
    tiny = wl.plain_line(seed=0)
    big = wl.make_problem("batch-lead", [30000, 20000, 15000], seed=43, kind="mixed")
    announce("batch led by a tiny plan")
    ts = [upload(tiny), upload(big)]
    plans = [plan_for(tiny), plan_for(big)]
    plans[1].sort(ts[1]["uvw"])
    assert plans[0].info()["kernel"] == 0 and plans[1].info()["kernel"] != 0
    singles = [pl.execute(t["sub"], t["g_uv"], t["g_w"], t["uvw"]).cpu().numpy() for pl, t in zip(plans, ts)]
    batch = Batch(plans)
    outs = [torch.full((p.n_vis,), float("nan"), dtype=torch.complex64, device=device()) for p in (tiny, big)]
    batch.execute([(t["sub"], t["g_uv"], t["g_w"], t["uvw"]) for t in ts], outs=outs)
    torch.cuda.synchronize()
    for o, single, p in zip(outs, singles, (tiny, big)):
        got = o.cpu().numpy()
        assert np.array_equal(got, single)
        assert rel_l2(got, oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)[0]) <= REL_L2_FP32
