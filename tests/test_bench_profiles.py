"""The committed counter profiles and the bench's roofline arithmetic (CPU).

The bench prices each kernel from ``profiles/counters.json``: HBM bytes from
FETCH_SIZE / WRITE_SIZE scaled by a plain copy, LDS bytes from the LDS
bandwidth counters, vector-ALU issue from SQ_INSTS_VALU, and the shares of
the vector-memory path. Every fraction of a peak must be at most 1 when the
counters and the duration come from the same cold launches."""
import json
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _counters():
    with open(os.path.join(ROOT, "profiles", "counters.json")) as f:
        return json.load(f)


def test_counter_file_covers_every_profiling_leg():
    c = _counters()
    assert set(bench.LEGS) <= set(c["legs"])
    cal = c["calibration"]
    # the copy calibration: reads and writes of 1 GiB, scales near 1-2
    assert 0.5 < cal["fetch_scale"] < 4 and 0.5 < cal["write_scale"] < 4
    for leg, le in c["legs"].items():
        assert le["kernels"], leg
        assert le["visibilities"] > 0 and le["compulsory_bytes"] > 0


@pytest.mark.parametrize("leg", sorted(set(bench.LEGS) - {"latency"}))
def test_every_fraction_of_a_peak_is_at_most_one(leg):
    c = _counters()["legs"][leg]
    for name, ke in c["kernels"].items():
        cn, us = ke["counters"], ke.get("duration_us")
        assert us and us > 0, (leg, name)
        t = us * 1e-6
        if ke.get("hbm_bytes") is not None:
            assert 0 < ke["hbm_bytes"] / t / 1e9 / bench.HBM_PEAK_GBS <= 1.0, (leg, name)
        if cn.get("SQ_INSTS_LDS_LOAD_BANDWIDTH") is not None:
            lds = 64.0 * (cn["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + cn.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0))
            assert lds / t / 1e9 / bench.LDS_PEAK_GBS <= 1.0, (leg, name)
        if cn.get("SQ_INSTS_VALU") is not None:
            assert cn["SQ_INSTS_VALU"] / t / 1e9 / bench.VALU_PEAK_GINST <= 1.0, (leg, name)
        m = bench.memory_path(cn, c["visibilities"], us)
        if m is not None:
            for k in ("td_busy_pct", "td_wait_cache_pct", "tcp_pending_stall_pct", "ta_busy_avr_pct",
                      "waves_in_waitcnt_pct"):
                if m[k] is not None:
                    assert 0.0 <= m[k] <= 100.0 + 1e-6, (leg, name, k, m[k])
            # the kernel's cycles from GRBM agree with its traced duration
            # for a clock between 2.0 and 2.5 GHz (kernels of a few tens of
            # microseconds also count the profiler's per-dispatch overhead)
            if us >= 100.0:
                assert 2.0e3 * us <= m["cycles"] <= 2.5e3 * us, (leg, name, m["cycles"], us)


def test_headline_roofline_object_from_committed_counters():
    """The bench's top-level roofline, rebuilt from the committed counters
    with their own duration: bound is the largest fraction, each <= 1."""
    c = bench.committed_counters("degrid")
    if c is None:
        pytest.skip("counters were taken on another source of the degrid kernel")
    ke = c["kernels"]["degrid_kernel"]
    from paper_2102_12739_amd import workload as wl
    p = wl.paper_scale(seed=1, with_grid=False)
    r = bench.roofline_object(p.n_vis, bench.BYTES_PER_VIS["c64"], ke["duration_us"] * 1e-3,
                              c["compulsory_bytes"], c, "degrid_kernel<c64,f32>")
    assert set(r["fracs"]) == {"hbm", "lds", "alu"}
    assert all(0 < v <= 1.0 for v in r["fracs"].values())
    assert r["bound"] == max(r["fracs"], key=r["fracs"].get)
    assert r["frac"] == r["fracs"][r["bound"]]
    assert r["traffic"] == pytest.approx(ke["hbm_bytes"])
    assert 0 < r["hbm"]["compulsory_frac"] < r["hbm"]["frac"]
    assert r["memory_path"]["td_busy_pct"] > 0


def test_memory_path_arithmetic():
    # one die's count of 1000 cycles, 8 dies, 256 CUs: 256 000 CU-cycles
    cu_cycles = bench.N_CU * 1000.0
    c = {"GRBM_GUI_ACTIVE": 1000.0 * bench.N_XCD, "TD_TD_BUSY_sum": 0.5 * cu_cycles,
         "TD_TC_STALL_sum": 0.25 * cu_cycles, "TA_BUSY_avr": 100.0,
         "TCP_PENDING_STALL_CYCLES_sum": 0.125 * cu_cycles, "TCP_TCC_READ_REQ_sum": 4000.0,
         "TCP_TCC_READ_REQ_LATENCY_sum": 4000.0 * 500.0, "SQ_WAIT_ANY": 30.0, "SQ_WAVE_CYCLES": 120.0}
    m = bench.memory_path(c, 1000)
    assert m["cycles"] == 1000.0
    assert m["td_busy_pct"] == pytest.approx(50.0)
    assert m["td_wait_cache_pct"] == pytest.approx(25.0)
    assert m["ta_busy_avr_pct"] == pytest.approx(10.0)
    assert m["tcp_pending_stall_pct"] == pytest.approx(12.5)
    assert m["l2_read_latency_cycles"] == pytest.approx(500.0)
    assert m["l2_reads_per_vis"] == pytest.approx(4.0)
    assert m["l2_reads_in_flight_per_cu"] == pytest.approx(4000.0 * 500.0 / cu_cycles)
    assert m["waves_in_waitcnt_pct"] == pytest.approx(25.0)
    assert bench.memory_path(c, 1000, bench.WAITCNT_MIN_US)["waves_in_waitcnt_pct"] == pytest.approx(25.0)
    assert bench.memory_path(c, 1000, 0.5 * bench.WAITCNT_MIN_US)["waves_in_waitcnt_pct"] is None
    assert bench.memory_path({"GRBM_GUI_ACTIVE": 1.0}, 1) is None


def _write_csv(path, header, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_summarize_pmc_on_a_synthetic_profiler_tree(tmp_path, monkeypatch):
    """bench.py --summarize-pmc over hand-made rocprofv3 CSV files: the first
    dispatch of each pass is dropped (the untimed warmup), counters of one
    dispatch are summed over their rows and averaged over dispatches, HBM
    bytes are the FETCH/WRITE counts scaled by the copy calibration, and a
    leg whose runs printed two source hashes is marked stale (None)."""
    root = tmp_path / "runs"
    counters_file = tmp_path / "counters.json"
    monkeypatch.setattr(bench, "COUNTERS_FILE", str(counters_file))
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    k = "void dg::degrid_kernel<0, 0, 18432, 64, false, false>(dg::LaunchParams)"
    # copy calibration: 1 GiB read as 2^19 KiB and written as 2^20 KiB
    _write_csv(str(root / "copy__FETCH_SIZE" / "run_counter_collection.csv"), hdr,
               [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 9e9], [2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 2 ** 19]])
    _write_csv(str(root / "copy__WRITE_SIZE" / "run_counter_collection.csv"), hdr,
               [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 9e9], [2, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 2 ** 20]])
    # latency leg: warmup dispatch 1 (ignored), then dispatches 2 and 3;
    # dispatch 2 reports FETCH_SIZE in two rows (instances) that add up
    _write_csv(str(root / "latency__FETCH_SIZE" / "run_counter_collection.csv"), hdr,
               [[1, k, "FETCH_SIZE", 1e9], [2, k, "FETCH_SIZE", 60.0], [2, k, "FETCH_SIZE", 40.0],
                [3, k, "FETCH_SIZE", 300.0], [3, "void other_kernel()", "FETCH_SIZE", 7e9]])
    _write_csv(str(root / "latency__WRITE_SIZE" / "run_counter_collection.csv"), hdr,
               [[1, k, "WRITE_SIZE", 1e9], [2, k, "WRITE_SIZE", 10.0], [3, k, "WRITE_SIZE", 30.0]])
    _write_csv(str(root / "latency__stats" / "run_kernel_trace.csv"),
               ["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               [[1, k, 0, 999999], [2, k, 1000, 7000], [3, k, 9000, 17000]])
    line = json.dumps({"leg": "latency", "source_sha256_16": "aaaa"})
    (root / "latency__FETCH_SIZE.log").write_text("noise\n" + line + "\n")
    bench.summarize_pmc(str(root))
    out = json.loads(counters_file.read_text())
    cal = out["calibration"]
    assert cal["fetch_scale"] == pytest.approx(2.0) and cal["write_scale"] == pytest.approx(1.0)
    le = out["legs"]["latency"]
    ke = le["kernels"]["degrid_kernel"]
    assert ke["counters"]["FETCH_SIZE"] == pytest.approx(200.0)     # (100 + 300) / 2
    assert ke["counters"]["WRITE_SIZE"] == pytest.approx(20.0)      # (10 + 30) / 2
    assert ke["hbm_bytes"] == pytest.approx(1024.0 * (200.0 * 2.0 + 20.0 * 1.0))
    assert ke["duration_us"] == pytest.approx(7.0)                  # (6000 + 8000) ns / 2
    assert le["source_sha256_16"] == "aaaa"
    assert le["visibilities"] == 2048 and le["compulsory_bytes"] > 2048 * 32
    assert (tmp_path / "counters.md").exists()
    # a second hash among the leg's runs makes the leg's counters stale
    (root / "latency__WRITE_SIZE.log").write_text(json.dumps({"leg": "latency", "source_sha256_16": "bbbb"}) + "\n")
    bench.summarize_pmc(str(root))
    assert json.loads(counters_file.read_text())["legs"]["latency"]["source_sha256_16"] is None
