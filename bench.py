"""Throughput benchmark of 3D degridding on one MI355X.

One step = one degrid of the paper-scale workload: 64 subgrids of
512 x 512 x 4 complex64 (re, im ~ N(0,1)), separable Kaiser-Bessel G_uv
(8 x 8, beta 18.72) and G_w (4 taps, beta 9.36) at oversampling 16, and
floor(exp(U[ln 2^10, ln 2^18])) visibilities per subgrid, the first half of
each subgrid's list on a folded line with constant step in [0.05, 0.5] cells
and the rest uniform in the subgrid (seed 1). Inputs are resident in HBM
before timing starts. Prints one JSON line.

The headline value is the cold figure: every timed launch follows an
untimed 1 GiB write that flushes the L2 and the Infinity Cache. The warm
(back-to-back) figure is reported beside it.

The roofline object prices the degrid kernel against three resources, each
as a fraction of its peak that cannot exceed 1: HBM (the bytes rocprofv3's
FETCH_SIZE and WRITE_SIZE counters measured for the same kernel source on
the cold launches, and the compulsory bytes: every subgrid cell inside some
in-range neighbourhood once, 32 B of coordinates and output per visibility,
and both tables), LDS (bytes of the kernel's LDS instructions) and VALU
issue (vector instructions). "bound" names the largest. The 2352 B per
visibility of a neighbourhood read in full for every visibility (2048 B of
subgrid, 256 B of G_uv, 16 B of G_w, 24 B of coordinates, 8 B of output) is
reported only as an effective rate: neighbouring visibilities share most of
their cells, which LDS and the caches serve, so that rate is not a roofline.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# LDS: 256 bytes per clock per CU (CDNA4 doubles CDNA3's 128; a ds_read_b128
# microbenchmark reached 196 B/clock/CU on this GPU), 256 CUs at 2.4 GHz.
LDS_PEAK_GBS = 256 * 256 * 2.4
# VALU issue: each of a CU's 4 SIMDs completes one wave64 instruction every
# 4 clocks (16 lanes per clock without packed FP32), 256 CUs at 2.4 GHz, in
# 1e9 wave instructions per second.
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters.json")
BYTES_PER_VIS = {"c64": 2048 + 256 + 16 + 24 + 8, "cbf16": 1024 + 128 + 8 + 24 + 8, "cf16": 1024 + 128 + 8 + 24 + 8}
# 16-bit forms of the same inputs: (storage, tables). fp16/fp16 and bf16/bf16
# take the packed 16-bit dot products for the w sums; bf16 storage with fp16
# tables widens both to float32.
LOW_PRECISION_FORMS = (("cbf16", "f16"), ("cf16", "f16"), ("cbf16", "bf16"))
LOW_PRECISION_REL_L2 = 3e-3   # error bound of the 16-bit storage forms against the FP64 oracle on FP32 inputs
FLUSH_BYTES = 1 << 30     # written between launches of the cold-cache timing


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_CSRC = os.path.join(ROOT, "paper_2102_12739_amd", "csrc")
# Source files of each profiled kernel: the device code it includes, and
# the plan code that decides the work order and cuts the tiles (the counters
# of a launch depend on both).
_COMMON_DEVICE = ("dg_device.h", "dg_internal.h", "plan_logic.h", "plan_logic.cpp", "plan_sort.hip")
LEG_SOURCES = {
    "degrid": ("degrid_kernels.hip",) + _COMMON_DEVICE,
    "adjoint": ("grid_kernels.hip",) + _COMMON_DEVICE,
    "table_grad": ("table_grad_kernels.hip",) + _COMMON_DEVICE,
}


def source_hash(kind: str) -> str:
    """sha256[:16] of a kernel's source and the device code it includes."""
    h = hashlib.sha256()
    for name in LEG_SOURCES[kind]:
        with open(os.path.join(_CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    return source_hash("degrid")


def committed_counters(leg: str):
    """Per-dispatch counter means of a profiling leg (profiles/counters.json),
    if they were taken on the current source of the leg's kernel; else None."""
    try:
        with open(COUNTERS_FILE) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    entry = c.get("legs", {}).get(leg)
    if not entry or entry.get("source_sha256_16") != source_hash(LEGS[leg]["source"]):
        return None
    return entry


def measured_traffic():
    """Cold HBM bytes per launch of the headline kernel from the committed
    counters, or None when they are stale."""
    e = committed_counters("degrid")
    return None if e is None else e.get("hbm_bytes")


# Profiling legs: one kernel's launches on one workload, for rocprofv3 runs
# (bench.py --leg NAME). "kernels" are the name prefixes of the dispatches
# that belong to the leg in a trace.
LEGS = {
    "degrid": dict(source="degrid", workload="paper", grid="c64", gcf="f32", op="degrid",
                   kernels=("degrid_kernel",)),
    "degrid_bf16": dict(source="degrid", workload="paper", grid="cbf16", gcf="bf16", op="degrid",
                        kernels=("degrid_kernel",)),
    "degrid_fp16": dict(source="degrid", workload="paper", grid="cf16", gcf="f16", op="degrid",
                        kernels=("degrid_kernel",)),
    "degrid_bf16_f16": dict(source="degrid", workload="paper", grid="cbf16", gcf="f16", op="degrid",
                            kernels=("degrid_kernel",)),
    "diff_degrid": dict(source="degrid", workload="diff", grid="c64", gcf="f32", op="degrid",
                        kernels=("degrid_kernel",)),
    "diff_owner_adjoint": dict(source="adjoint", workload="diff", grid="c64", gcf="f32", op="adjoint",
                               kernels=("grid_owner_kernel", "grid_fixup_kernel")),
    "diff_scatter_adjoint": dict(source="adjoint", workload="diff", grid="c64", gcf="f32", op="adjoint",
                                 unsorted=True, kernels=("grid_adjoint_kernel", "zero_kernel")),
    "diff_table_grad": dict(source="table_grad", workload="diff", grid="c64", gcf="f32", op="table_grad",
                            kernels=("table_grad_kernel", "zero_f32_kernel")),
    "latency": dict(source="degrid", workload="plain", grid="c64", gcf="f32", op="degrid",
                    kernels=("degrid_kernel",)),
    # the eight batched problems in one launch of a Batch (replayed HIP graph),
    # with each plan's default kernel (the batch tuner's choice in the bench)
    "batched": dict(source="degrid", workload="batched", grid="c64", gcf="f32", op="batch",
                    kernels=("degrid_kernel",)),
    "batched_bf16": dict(source="degrid", workload="batched", grid="cbf16", gcf="bf16", op="batch",
                         kernels=("degrid_kernel",)),
}


def run_leg(name, steps, warmup, cold, kernel=None, nb=None):
    """Launch one profiling leg: warmup untimed launches, then steps launches
    timed one by one with HIP events on the launch stream (each after a 1 GiB
    flush when cold). Prints one JSON line."""
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import Plan
    if name == "copy":
        # calibration of the HBM byte counters: a plain copy of 1 GiB
        a = torch.ones((1 << 30) // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        ms = launch_times(lambda: b.copy_(a), warmup + steps)[warmup:]
        return {"leg": name, "bytes": 1 << 30, "launches": steps, "kernel_ms": percentiles(ms)}
    leg = LEGS[name]
    if leg["op"] == "batch":
        return run_batch_leg(name, leg, steps, warmup, cold, kernel, nb)
    p = {"paper": lambda: wl.paper_scale(seed=1), "diff": lambda: wl.differentiation(seed=4),
         "plain": lambda: wl.plain_line(seed=0)}[leg["workload"]]()
    sub, g_uv, g_w, uvw = upload_inputs(p, leg["grid"], leg["gcf"])
    plan = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w, grid_dtype=leg["grid"], gcf_dtype=leg["gcf"])
    if not leg.get("unsorted"):
        plan.sort(uvw)
    if kernel is not None:
        plan.set_kernel(kernel, nb or 0)
    dev = uvw.device
    if leg["op"] == "degrid":
        out = torch.empty(p.n_vis, dtype=torch.complex64, device=dev)
        fn = lambda: plan.execute(sub, g_uv, g_w, uvw, out=out)   # noqa: E731
    else:
        vin = torch.from_numpy(wl.complex_noise(5, p.n_vis, 1.0)).to(dev)
        if leg["op"] == "adjoint":
            gout = torch.empty(plan.shape, dtype=torch.complex64, device=dev)
            fn = lambda: plan.adjoint(vin, g_uv, g_w, uvw, out=gout)   # noqa: E731
        else:
            tg_uv = torch.empty(g_uv.shape, dtype=torch.float32, device=dev)
            tg_w = torch.empty(g_w.shape, dtype=torch.float32, device=dev)
            fn = lambda: plan.table_grad(sub, g_uv, g_w, uvw, vin, out_uv=tg_uv, out_w=tg_w)   # noqa: E731
    if name == "latency":
        # 1000 launches captured in one HIP graph, replayed: the per-launch
        # time of the small plain-line case, as the bench's latency figure
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        fn()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            for _ in range(1000):
                plan.execute(sub, g_uv, g_w, uvw, out=out, stream=side)
        torch.cuda.synchronize()
        for _ in range(warmup):
            g.replay()
        torch.cuda.synchronize()
        ms = [x / 1000.0 for x in launch_times(g.replay, steps)]
        res = {"leg": name, "workload": p.name, "visibilities": p.n_vis, "graph_launches": 1000,
               "replays": steps, "per_launch_ms": percentiles(ms), "plan": plan.info(),
               "source_sha256_16": source_hash(leg["source"])}
        log(f"leg latency: {res['per_launch_ms']['median'] * 1e3:.2f} us per launch (graph of 1000)")
        return res
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    flush = None
    if cold:
        flush_buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)
        flush = lambda: flush_buf.fill_(1.0)   # noqa: E731
    ms = launch_times(fn, steps, flush)
    res = {"leg": name, "workload": p.name, "visibilities": p.n_vis, "cold": bool(cold), "launches": steps,
           "kernel_ms": percentiles(ms), "kernel_ms_mean": float(sum(ms) / len(ms)),
           "plan": plan.info(), "source_sha256_16": source_hash(leg["source"])}
    log(f"leg {name}: {res['kernel_ms']['median'] * 1e3:.1f} us median over {steps} launches"
        f" ({'cold' if cold else 'warm'})")
    return res


def run_batch_leg(name, leg, steps, warmup, cold, kernel=None, nb=None):
    """A batched profiling leg: the eight problems of the batched workload
    (seed 2) as sorted plans in one Batch, launched as run_leg launches."""
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import Batch, Plan
    probs = wl.batched(seed=2)
    ins = [upload_inputs(q, leg["grid"], leg["gcf"]) for q in probs]
    plans = []
    for q, i in zip(probs, ins):
        pl = Plan(q.offsets, q.n_v, q.n_u, q.n_w, q.os_uv, q.os_w, grid_dtype=leg["grid"], gcf_dtype=leg["gcf"])
        pl.sort(i[3])
        if kernel is not None:
            pl.set_kernel(kernel, nb or 0)
        plans.append(pl)
    outs = [torch.empty(q.n_vis, dtype=torch.complex64, device="cuda:0") for q in probs]
    batch = Batch(plans)
    fn = lambda: batch.execute(ins, outs=outs)   # noqa: E731
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ms = cold_launches(fn, steps) if cold else launch_times(fn, steps)
    n_vis = sum(q.n_vis for q in probs)
    res = {"leg": name, "workload": "batched-8-problems-seed2", "visibilities": n_vis, "cold": bool(cold),
           "launches": steps, "kernel_ms": percentiles(ms), "kernel_ms_mean": float(sum(ms) / len(ms)),
           "plan": {"kernel": plans[0].info()["kernel"], "n_b": plans[0].info()["n_b"]},
           "source_sha256_16": source_hash(leg["source"])}
    log(f"leg {name}: {res['kernel_ms']['median'] * 1e3:.1f} us median over {steps} launches"
        f" ({'cold' if cold else 'warm'})")
    batch.close()
    return res


def _leg_of_kernel(leg, kernel_name):
    """The prefix in LEGS[leg]["kernels"] that names this dispatch, or None."""
    for k in LEGS[leg]["kernels"] if leg in LEGS else ("__amd_rocclr_copyBuffer",):
        if re.search(r"(^|::|\s)" + re.escape(k) + r"($|<|\()", kernel_name):
            return k
    return None


def summarize_pmc(root):
    """Collect rocprofv3 runs of the profiling legs into profiles/counters.json
    and profiles/counters.md.

    root holds one folder per run, named LEG__PASS (LEG a profiling leg or
    "copy", PASS "stats" for a --kernel-trace --stats run, else the counter
    names of a --pmc run). Per kernel of a leg the first dispatch is dropped
    (the untimed warmup) and the rest averaged. FETCH_SIZE and WRITE_SIZE are
    scaled by what the same counters read for the 1 GiB plain copy of the
    "copy" leg (read and write 1 GiB each)."""
    import csv
    import glob
    per = {}   # (leg, kernel) -> {"counters": {name: [values]}, "durations_ns": [...]}
    hashes = {}   # leg -> source hashes printed by its runs (bench.py --leg prints one JSON line)
    for log_path in sorted(glob.glob(os.path.join(root, "*__*.log"))):
        leg = os.path.basename(log_path).partition("__")[0]
        with open(log_path) as f:
            for line in f:
                if line.startswith("{") and '"source_sha256_16"' in line:
                    hashes.setdefault(leg, set()).add(json.loads(line)["source_sha256_16"])
    for run in sorted(glob.glob(os.path.join(root, "*__*"))):
        if not os.path.isdir(run):
            continue
        leg, _, pass_name = os.path.basename(run).partition("__")
        for path in glob.glob(os.path.join(run, "**", "*.csv"), recursive=True):
            base = os.path.basename(path)
            with open(path, newline="") as f:
                rows = list(csv.DictReader(f))
            if base.endswith("counter_collection.csv"):
                by_dispatch = {}
                for r in rows:
                    k = _leg_of_kernel(leg, r.get("Kernel_Name", ""))
                    if k is None:
                        continue
                    d = by_dispatch.setdefault((k, int(r["Dispatch_Id"])), {})
                    d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                for (k, disp), vals in sorted(by_dispatch.items()):
                    e = per.setdefault((leg, k), {"counters": {}, "durations_ns": [], "seen": {}})
                    seen = e["seen"].setdefault(pass_name, 0)
                    e["seen"][pass_name] = seen + 1
                    if seen == 0:
                        continue   # warmup dispatch
                    for name, v in vals.items():
                        e["counters"].setdefault(name, []).append(v)
            elif base.endswith("kernel_trace.csv") and pass_name == "stats":
                seen = {}
                for r in sorted(rows, key=lambda r: int(r.get("Dispatch_Id", 0))):
                    k = _leg_of_kernel(leg, r.get("Kernel_Name", ""))
                    if k is None:
                        continue
                    seen[k] = seen.get(k, 0) + 1
                    if seen[k] == 1:
                        continue
                    e = per.setdefault((leg, k), {"counters": {}, "durations_ns": [], "seen": {}})
                    e["durations_ns"].append(float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    mean = lambda v: float(sum(v) / len(v)) if v else None   # noqa: E731
    cal = per.get(("copy", "__amd_rocclr_copyBuffer"), {"counters": {}})["counters"]
    gib_kib = (1 << 30) / 1024.0
    fetch_scale = gib_kib / mean(cal["FETCH_SIZE"]) if cal.get("FETCH_SIZE") else None
    write_scale = gib_kib / mean(cal["WRITE_SIZE"]) if cal.get("WRITE_SIZE") else None
    out = {"calibration": {"copy_bytes": 1 << 30, "copy_FETCH_SIZE_kib": mean(cal.get("FETCH_SIZE", [])),
                           "copy_WRITE_SIZE_kib": mean(cal.get("WRITE_SIZE", [])),
                           "fetch_scale": fetch_scale, "write_scale": write_scale},
           "legs": {}}
    for (leg, k), e in sorted(per.items()):
        if leg not in LEGS:
            continue
        c = {name: mean(v) for name, v in e["counters"].items()}
        ke = {"counters": c, "dispatches": max((len(v) for v in e["counters"].values()), default=0),
              "duration_us": (mean(e["durations_ns"]) or 0.0) / 1e3 or None}
        if c.get("FETCH_SIZE") is not None and c.get("WRITE_SIZE") is not None and fetch_scale and write_scale:
            ke["hbm_bytes"] = 1024.0 * (c["FETCH_SIZE"] * fetch_scale + c["WRITE_SIZE"] * write_scale)
        # the kernel source the runs were made with (none, or several: stale)
        h = hashes.get(leg, set())
        le = out["legs"].setdefault(leg, {"source_sha256_16": next(iter(h)) if len(h) == 1 else None,
                                          "kernels": {}})
        le["kernels"][k] = ke
    for leg, le in out["legs"].items():
        ks = le["kernels"].values()
        if all("hbm_bytes" in k for k in ks):
            le["hbm_bytes"] = sum(k["hbm_bytes"] for k in ks)
        if all(k.get("duration_us") for k in ks):
            le["duration_us"] = sum(k["duration_us"] for k in ks)
    from paper_2102_12739_amd import workload as wl
    # (coordinates and tables only: the subgrids do not enter the count)
    works = {"paper": lambda: [wl.paper_scale(seed=1, with_grid=False)],
             "diff": lambda: [wl.differentiation(seed=4, with_grid=False)],
             "plain": lambda: [wl.plain_line(seed=0, with_grid=False)],
             "batched": lambda: wl.batched(seed=2, with_grid=False)}
    comp = {}
    for leg, le in out["legs"].items():
        w = LEGS[leg]["workload"]
        elem = 8 if LEGS[leg]["grid"] == "c64" else 4
        if (w, elem) not in comp:
            pws = works[w]()
            comp[(w, elem)] = (sum(compulsory_bytes(q, elem) for q in pws), sum(q.n_vis for q in pws))
        le["compulsory_bytes"], le["visibilities"] = comp[(w, elem)]
    with open(COUNTERS_FILE, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    with open(COUNTERS_FILE[:-5] + ".md", "w") as f:
        f.write(counters_markdown(out))
    log(f"wrote {COUNTERS_FILE}: legs {sorted(out['legs'])}")
    return out


# rocprofv3 passes of every profiling leg (one process each; bench.py --leg
# LEG --cold --steps 5 --warmup 1 after "--").
PMC_PASSES = (
    ("FETCH_SIZE",),
    ("WRITE_SIZE", "TCC_HIT_sum", "TCC_MISS_sum"),
    ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_LDS_LOAD_BANDWIDTH", "SQ_INSTS_LDS_STORE_BANDWIDTH",
     "SQ_INSTS_SALU", "SQ_INSTS_SMEM", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"),
    ("VALUBusy", "LdsUtil", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_ANY",
     "SQ_BUSY_CYCLES"),
    ("TA_BUSY_avr", "TD_TD_BUSY_sum", "TD_TC_STALL_sum", "GRBM_GUI_ACTIVE", "SQ_WAIT_ANY"),
    ("TCP_PENDING_STALL_CYCLES_sum", "TCP_TCC_READ_REQ_LATENCY_sum", "TCP_TCC_READ_REQ_sum", "GRBM_GUI_ACTIVE"),
)
N_CU = 256   # compute units of the MI355X
N_XCD = 8    # accelerator complex dies; GRBM_GUI_ACTIVE counts once per die


# Kernels shorter than this have no share of wave cycles in s_waitcnt: its
# two counters come from different rocprofv3 passes, and for a kernel of a
# few microseconds their run-to-run spread is larger than the share.
WAITCNT_MIN_US = 100.0


def memory_path(c, n_vis, duration_us=None):
    """Vector-memory path figures of one kernel from its counters, or None:
    per-CU busy and stall shares of the texture data unit (TD) and the vector
    L1 (TCP), the L1-to-L2 read latency, L2 reads per visibility and in
    flight per CU, and the share of wave cycles spent in s_waitcnt (None for
    kernels shorter than WAITCNT_MIN_US when their duration is given)."""
    need = ("GRBM_GUI_ACTIVE", "TD_TD_BUSY_sum", "TCP_TCC_READ_REQ_sum")
    if any(c.get(k) is None for k in need) or not c["GRBM_GUI_ACTIVE"]:
        return None
    cu_cycles = N_CU * c["GRBM_GUI_ACTIVE"] / N_XCD
    pct = lambda k: 100.0 * c[k] / cu_cycles if c.get(k) is not None else None   # noqa: E731
    req = c["TCP_TCC_READ_REQ_sum"]
    lat = c.get("TCP_TCC_READ_REQ_LATENCY_sum")
    return {"cycles": c["GRBM_GUI_ACTIVE"] / N_XCD,
            "td_busy_pct": pct("TD_TD_BUSY_sum"), "td_wait_cache_pct": pct("TD_TC_STALL_sum"),
            "ta_busy_avr_pct": 100.0 * c["TA_BUSY_avr"] * N_XCD / c["GRBM_GUI_ACTIVE"]
            if c.get("TA_BUSY_avr") is not None else None,
            "tcp_pending_stall_pct": pct("TCP_PENDING_STALL_CYCLES_sum"),
            "l2_read_latency_cycles": lat / req if lat is not None and req else None,
            "l2_reads_per_vis": req / n_vis if n_vis else None,
            "l2_reads_in_flight_per_cu": lat / cu_cycles if lat is not None else None,
            "waves_in_waitcnt_pct": 100.0 * c["SQ_WAIT_ANY"] / c["SQ_WAVE_CYCLES"]
            if c.get("SQ_WAIT_ANY") is not None and c.get("SQ_WAVE_CYCLES")
            and (duration_us is None or duration_us >= WAITCNT_MIN_US) else None}


def counters_markdown(out):
    """The per-kernel table of profiles/counters.md."""
    cal = out["calibration"]
    lines = [
        "# Per-kernel rocprofv3 counters of the profiling legs (cold launches)",
        "",
        "Every leg is `python3 bench.py --leg LEG --cold --steps 5 --warmup 1`: one kernel's launches on one",
        "workload, each timed launch after an untimed 1 GiB write (L2 and Infinity Cache flushed). One",
        "rocprofv3 process per pass; the untimed first launch of each kernel is dropped and the other five",
        "averaged. Passes:",
        "",
        "```",
        "rocprofv3 --kernel-trace --stats -d DIR/LEG__stats -o run --output-format csv -- "
        "python3 bench.py --leg LEG --cold --steps 5 --warmup 1",
    ]
    for ps in PMC_PASSES:
        lines.append(f"rocprofv3 --pmc {' '.join(ps)} -d DIR/LEG__{'_'.join(ps)} -o run --output-format csv -- "
                     "python3 bench.py --leg LEG --cold --steps 5 --warmup 1")
    lines += [
        "rocprofv3 --pmc FETCH_SIZE -d DIR/copy__FETCH_SIZE -o run --output-format csv -- "
        "python3 bench.py --leg copy --steps 3 --warmup 1   (and WRITE_SIZE)",
        "python3 bench.py --summarize-pmc DIR",
        "```",
        "",
        f"Calibration (1 GiB `__amd_rocclr_copyBuffer`): FETCH_SIZE {cal['copy_FETCH_SIZE_kib']} KiB -> read scale "
        f"{cal['fetch_scale']}; WRITE_SIZE {cal['copy_WRITE_SIZE_kib']} KiB -> write scale {cal['write_scale']}.",
        "",
        "Peaks: HBM 8000 GB/s; LDS 256 B/clock/CU x 256 CUs x 2.4 GHz = 157 286 GB/s; VALU issue one wave64",
        "instruction per 4 clocks per SIMD = 614.4 G/s. LDS bytes = 64 x (SQ_INSTS_LDS_LOAD_BANDWIDTH +",
        "SQ_INSTS_LDS_STORE_BANDWIDTH). VALUBusy and LdsUtil are rocprofv3's derived percentages of GPU time.",
        "",
        "| leg | kernel | us | HBM MB | HBM frac | compulsory frac | B/vis HBM | L2 hit | LDS GB/s (frac) | "
        "VALU Ginst/s (frac) | VALUBusy % | LdsUtil % | bank-conflict cycles | waves waiting % |",
        "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|",
    ]
    for leg, le in sorted(out["legs"].items()):
        n = le.get("visibilities") or 1
        for k, ke in sorted(le["kernels"].items()):
            c = ke["counters"]
            us = ke.get("duration_us")
            t = (us or 0) * 1e-6
            f = lambda x, fmt: (fmt.format(x) if x is not None else "-")   # noqa: E731
            hbm = ke.get("hbm_bytes")
            hbm_frac = hbm / t / 1e9 / HBM_PEAK_GBS if hbm and t else None
            comp_frac = (le["compulsory_bytes"] / (le["duration_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
                         if le.get("duration_us") and len(le["kernels"]) and k == sorted(le["kernels"])[0] else None)
            hit = (c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"])
                   if c.get("TCC_HIT_sum") is not None and c.get("TCC_MISS_sum") else None)
            lds_b = ((c.get("SQ_INSTS_LDS_LOAD_BANDWIDTH") or 0) + (c.get("SQ_INSTS_LDS_STORE_BANDWIDTH") or 0)) * 64
            lds_gbs = lds_b / t / 1e9 if t and "SQ_INSTS_LDS_LOAD_BANDWIDTH" in c else None
            valu = c["SQ_INSTS_VALU"] / t / 1e9 if t and c.get("SQ_INSTS_VALU") is not None else None
            wait = (100.0 * c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"]
                    if c.get("SQ_WAIT_INST_ANY") is not None and c.get("SQ_WAVE_CYCLES") else None)
            lines.append(
                f"| {leg} | {k} | {f(us, '{:.1f}')} | {f(hbm / 1e6 if hbm else None, '{:.1f}')} | "
                f"{f(hbm_frac, '{:.3f}')} | {f(comp_frac, '{:.3f}')} | {f(hbm / n if hbm else None, '{:.0f}')} | "
                f"{f(hit, '{:.3f}')} | "
                f"{f(lds_gbs, '{:.0f}')} ({f(lds_gbs / LDS_PEAK_GBS if lds_gbs is not None else None, '{:.3f}')}) | "
                f"{f(valu, '{:.1f}')} ({f(valu / VALU_PEAK_GINST if valu is not None else None, '{:.3f}')}) | "
                f"{f(c.get('VALUBusy'), '{:.1f}')} | {f(c.get('LdsUtil'), '{:.1f}')} | "
                f"{f(c.get('SQ_LDS_BANK_CONFLICT'), '{:.3g}')} | {f(wait, '{:.1f}')} |")
    lines += [
        "",
        "Vector-memory path (TA: texture addresser, TD: texture data unit, TCP: vector L1). Per-CU shares of",
        f"the kernel's cycles, with cycles = GRBM_GUI_ACTIVE / {N_XCD} (one count per die) over {N_CU} CUs;",
        "L2 read latency = TCP_TCC_READ_REQ_LATENCY_sum / TCP_TCC_READ_REQ_sum; reads in flight per CU =",
        "TCP_TCC_READ_REQ_LATENCY_sum / (CUs x cycles); waves in s_waitcnt = SQ_WAIT_ANY / SQ_WAVE_CYCLES.",
        "For kernels of 100 us or more the cycles match the traced duration at 2.26-2.43 GHz; for kernels of",
        "a few tens of microseconds GRBM_GUI_ACTIVE also counts the profiler's per-dispatch overhead, so their",
        "shares read low. The s_waitcnt share takes its two counters from different passes: it is given for",
        "kernels of 100 us or more only.",
        "",
        "| leg | kernel | TA busy % | TD busy % | TD waiting on L1 % | L1 stalled on misses % | "
        "L2 read latency (cycles) | L2 reads / vis | L2 reads in flight / CU | waves in s_waitcnt % |",
        "|---|---|---|---|---|---|---|---|---|---|",
    ]
    for leg, le in sorted(out["legs"].items()):
        for k, ke in sorted(le["kernels"].items()):
            m = memory_path(ke["counters"], le.get("visibilities") or 0, ke.get("duration_us"))
            if m is None:
                continue
            f = lambda x, fmt: (fmt.format(x) if x is not None else "-")   # noqa: E731
            lines.append(
                f"| {leg} | {k} | {f(m['ta_busy_avr_pct'], '{:.0f}')} | {f(m['td_busy_pct'], '{:.0f}')} | "
                f"{f(m['td_wait_cache_pct'], '{:.0f}')} | {f(m['tcp_pending_stall_pct'], '{:.0f}')} | "
                f"{f(m['l2_read_latency_cycles'], '{:.0f}')} | {f(m['l2_reads_per_vis'], '{:.2f}')} | "
                f"{f(m['l2_reads_in_flight_per_cu'], '{:.1f}')} | {f(m['waves_in_waitcnt_pct'], '{:.0f}')} |")
    lines += ["", "Compulsory bytes per leg (host count): " + ", ".join(
        f"{leg} {le['compulsory_bytes'] / 1e6:.1f} MB for {le['visibilities']} visibilities"
        for leg, le in sorted(out["legs"].items())), ""]
    return "\n".join(lines)


def roofline_object(n_vis, bytes_per_vis, kernel_ms, comp_bytes, counters, kernel):
    """Fractions of three peaks for one kernel launch of kernel_ms: HBM
    (counter bytes and compulsory bytes), LDS (bytes of LDS instructions)
    and VALU issue (vector instructions), each <= 1 by construction when the
    counters were taken on the same (cold) launches. "bound" names the
    largest; the top-level achieved / peak / frac are that resource's."""
    t = kernel_ms * 1e-3
    hbm = {"peak_gbs": HBM_PEAK_GBS, "compulsory_bytes": comp_bytes, "compulsory_gbs": comp_bytes / t / 1e9,
           "compulsory_frac": comp_bytes / t / 1e9 / HBM_PEAK_GBS,
           "compulsory_basis": "every subgrid cell inside some in-range neighbourhood once, 24 B of (u, v, w) "
                               "and 8 B of output per visibility, both tables"}
    fracs = {}
    res = {"kernel": kernel, "kernel_ms": kernel_ms, "hbm": hbm,
           "effective": {"bytes_per_vis": bytes_per_vis, "gbs": bytes_per_vis * n_vis / t / 1e9,
                         "note": "every visibility's full neighbourhood, G_uv block, G_w row, coordinates and "
                                 "output; neighbouring visibilities share most cells, served from LDS and the "
                                 "caches, so this rate is not a roofline"}}
    traffic = None
    if counters is not None:
        kc = counters["kernels"].get("degrid_kernel", {}).get("counters", {})
        traffic = counters.get("hbm_bytes")
        if traffic:
            hbm["traffic_bytes"] = traffic
            hbm["achieved_gbs"] = traffic / t / 1e9
            hbm["frac"] = hbm["achieved_gbs"] / HBM_PEAK_GBS
            hbm["bytes_per_vis"] = traffic / n_vis
            fracs["hbm"] = hbm["frac"]
        if kc.get("SQ_INSTS_LDS_LOAD_BANDWIDTH") is not None:
            lds_bytes = 64.0 * (kc["SQ_INSTS_LDS_LOAD_BANDWIDTH"] + kc.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0))
            res["lds"] = {"bytes": lds_bytes, "instructions": kc.get("SQ_INSTS_LDS"),
                          "achieved_gbs": lds_bytes / t / 1e9, "peak_gbs": LDS_PEAK_GBS,
                          "frac": lds_bytes / t / 1e9 / LDS_PEAK_GBS, "busy_pct": kc.get("LdsUtil"),
                          "basis": "64 B x (SQ_INSTS_LDS_LOAD_BANDWIDTH + SQ_INSTS_LDS_STORE_BANDWIDTH)"}
            fracs["lds"] = res["lds"]["frac"]
        if kc.get("SQ_INSTS_VALU") is not None:
            gi = kc["SQ_INSTS_VALU"] / t / 1e9
            res["alu"] = {"instructions": kc["SQ_INSTS_VALU"], "achieved_ginst_s": gi,
                          "peak_ginst_s": VALU_PEAK_GINST, "frac": gi / VALU_PEAK_GINST,
                          "basis": "wave64 vector-ALU instructions (SQ_INSTS_VALU) issued, one per 4 clocks "
                                   "per SIMD (16 lanes, no packed FP32): 256 CUs x 4 SIMDs x 2.4 GHz / 4"}
            fracs["alu"] = res["alu"]["frac"]
        for k in ("VALUBusy", "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "TCC_HIT_sum", "TCC_MISS_sum"):
            if kc.get(k) is not None:
                res.setdefault("counters", {})[k] = kc[k]
        if kc.get("TCC_HIT_sum") and kc.get("TCC_MISS_sum"):
            hbm["l2_hit_rate"] = kc["TCC_HIT_sum"] / (kc["TCC_HIT_sum"] + kc["TCC_MISS_sum"])
        mp = memory_path(kc, n_vis)
        if mp is not None:
            mp["note"] = ("busy and stall shares of the vector-memory path per CU; this, not HBM, LDS or "
                          "VALU issue, is the resource the kernel keeps occupied")
            res["memory_path"] = mp
    if not fracs:
        # no counters for this kernel source: the compulsory bytes alone
        fracs["hbm"] = hbm["compulsory_frac"]
        hbm["frac"] = hbm["compulsory_frac"]
        hbm["achieved_gbs"] = hbm["compulsory_gbs"]
    bound = max(fracs, key=fracs.get)
    top = {"hbm": (hbm["achieved_gbs"], HBM_PEAK_GBS, "GB/s"),
           "lds": (res.get("lds", {}).get("achieved_gbs"), LDS_PEAK_GBS, "GB/s"),
           "alu": (res.get("alu", {}).get("achieved_ginst_s"), VALU_PEAK_GINST, "Ginst/s")}[bound]
    res.update({"bound": bound, "achieved": top[0], "peak": top[1], "unit": top[2], "frac": fracs[bound],
                "traffic": traffic, "fracs": fracs})
    return {k: res[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "fracs", "kernel",
                                "kernel_ms", "hbm") + tuple(k for k in ("lds", "alu", "memory_path", "counters")
                                                            if k in res)
            + ("effective",)}


def upload_inputs(p, grid_dtype="c64", gcf_dtype="f32"):
    import numpy as np
    import torch
    from paper_2102_12739_amd import workload as wl
    dev = torch.device("cuda:0")
    if grid_dtype == "c64":
        sub = torch.from_numpy(p.subgrids).to(dev)
    elif grid_dtype == "cbf16":
        sub = torch.from_numpy(wl.complex_to_storage(p.subgrids, "cbf16").view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        sub = torch.from_numpy(wl.complex_to_storage(p.subgrids, "cf16")).to(dev)
    def table(t):
        st = wl.table_to_storage(t, gcf_dtype)
        if gcf_dtype == "bf16":
            return torch.from_numpy(st.view(np.int16)).to(dev).view(torch.bfloat16)
        return torch.from_numpy(st).to(dev)
    return sub, table(p.g_uv), table(p.g_w), torch.from_numpy(p.uvw).to(dev)


def time_plan(plan, inputs, out, steps, warmup):
    """Wall time per step (synchronised both sides) and kernel time per launch
    (HIP events on the launch stream)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.execute(*inputs, out=out, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        plan.execute(*inputs, out=out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps


def copy_calibration(n_bytes=1 << 30):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters of a profiled run."""
    import torch
    a = torch.empty(n_bytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {n_bytes} bytes")


def percentiles(ms):
    import numpy as np
    a = np.asarray(ms, dtype=np.float64)
    return {"p10": float(np.percentile(a, 10)), "median": float(np.median(a)), "p90": float(np.percentile(a, 90)),
            "n": int(a.size)}


def launch_times(fn, n, flush=None):
    """Duration of n single launches (HIP events around each), in ms; flush()
    runs untimed before each launch."""
    import torch
    stream = torch.cuda.current_stream()
    out = []
    for _ in range(n):
        if flush is not None:
            flush()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def cold_launches(fn, n):
    """Durations (ms) of n launches, each after an untimed 1 GiB write."""
    import torch
    buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda:0")
    ms = launch_times(fn, n, flush=lambda: buf.fill_(1.0))
    del buf
    return ms


def copy_bandwidth(n_bytes=1 << 30, reps=10):
    """Device-to-device copy rate (read + write bytes per second) on this GPU."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    ms = percentiles(launch_times(lambda: b.copy_(a), reps))["median"]
    del a, b
    return 2.0 * n_bytes / (ms * 1e-3) / 1e9


def compulsory_bytes(p, elem_bytes):
    """Bytes a launch must move at least: every subgrid cell inside some
    in-range visibility's 8 x 8 (x 4 w) neighbourhood once, plus the
    coordinates and output of every visibility and both tables. Host-side
    footprint count (start cell = floor(c) - 3 along u and v)."""
    import numpy as np
    cells = 0
    for s in range(p.n_subgrids):
        lo, hi = int(p.offsets[s]), int(p.offsets[s + 1])
        if hi == lo:
            continue
        c = p.uvw[lo:hi]
        x0 = np.floor(c[:, 0]).astype(np.int64) - 3
        y0 = np.floor(c[:, 1]).astype(np.int64) - 3
        z0 = np.floor(c[:, 2]).astype(np.int64) - 1
        ok = (x0 >= 0) & (x0 <= p.n_u - 8) & (y0 >= 0) & (y0 <= p.n_v - 8) & (z0 >= 0) & (z0 <= p.n_w - 4)
        starts = np.zeros((p.n_v + 8, p.n_u + 8), dtype=np.int64)
        np.add.at(starts, (y0[ok] + 8, x0[ok] + 8), 1)
        # cell (y, x) is covered when some start lies in [y-7, y] x [x-7, x]
        ii = np.cumsum(np.cumsum(starts, axis=0), axis=1)
        box = ii[8:, 8:] - ii[:-8, 8:] - ii[8:, :-8] + ii[:-8, :-8]
        cells += int(np.count_nonzero(box))
    tables = p.g_uv.size * (4 if elem_bytes == 8 else 2) + p.g_w.size * (4 if elem_bytes == 8 else 2)
    return cells * p.n_w * elem_bytes + 32 * p.n_vis + tables


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-variants", action="store_true", help="skip the bf16/fp16 storage runs")
    ap.add_argument("--tune", action="store_true", help="let the plan time tile sizes first")
    ap.add_argument("--input-order", action="store_true",
                    help="time the plan without the plan-time work order (degrid_plan_sort)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-patterns", action="store_true",
                    help="skip the latency, batched and differentiation measurements")
    ap.add_argument("--study", action="store_true",
                    help="instead of the benchmark: the count-scenario x kernel-mapping study (one JSON line)")
    ap.add_argument("--main-only", action="store_true",
                    help="only the timed steps of the sorted plan (for a profiler's per-kernel statistics): "
                         "no input-order run, per-launch distributions, storage variants, CPU baseline or patterns")
    ap.add_argument("--leg", choices=sorted(LEGS) + ["copy"],
                    help="instead of the benchmark: launch one kernel's profiling leg (for rocprofv3)")
    ap.add_argument("--cold", action="store_true", help="with --leg: flush 1 GiB before every timed launch")
    ap.add_argument("--kernel", type=int, default=None, help="with --leg: the gather kernel variant")
    ap.add_argument("--nb", type=int, default=None, help="with --leg and --kernel: visibilities per tile")
    ap.add_argument("--study-md", metavar="JSON",
                    help="instead of the benchmark: render the JSON line of a --study run as markdown tables")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="instead of the benchmark: read rocprofv3 counter runs of the legs under DIR "
                         "(one folder per run, named LEG__PASS) and write profiles/counters.json and .md")
    args = ap.parse_args(argv)
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return 0
    if args.study_md:
        with open(args.study_md) as f:
            print(study_markdown(json.loads(f.read().strip().splitlines()[-1])))
        return 0
    if args.leg:
        print(json.dumps(run_leg(args.leg, args.steps, args.warmup, args.cold, args.kernel, args.nb)), flush=True)
        return 0
    if args.study:
        import torch  # noqa: F401
        print(json.dumps(bench_study(max(args.steps, 5), max(args.warmup, 2))), flush=True)
        return 0
    if args.main_only:
        args.no_cpu_baseline = args.no_variants = args.no_patterns = True
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the degridding path shards by subgrid with no exchange; see the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import Plan

    if args.copy_calibration:
        copy_calibration()

    t = time.perf_counter()
    p = wl.paper_scale(seed=1)
    log(f"workload {p.name}: S={p.n_subgrids} N={p.n_vis} generated in {time.perf_counter() - t:.1f}s")
    inputs = upload_inputs(p)
    out = torch.empty(p.n_vis, dtype=torch.complex64, device="cuda:0")
    plan = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w)
    # the input-order figure is measured too (and reported beside the main one)
    if not args.main_only:
        ms_in_order, kms_in_order = time_plan(plan, inputs, out, args.steps, args.warmup)
    sort_s = None
    if not args.input_order:
        t = time.perf_counter()
        plan.sort(inputs[3])
        sort_s = time.perf_counter() - t
    tune_s = None
    if args.tune:
        t = time.perf_counter()
        plan.tune(*inputs, out=out)
        tune_s = time.perf_counter() - t
    info = plan.info()
    run = lambda: plan.execute(*inputs, out=out)   # noqa: E731
    # warm: back-to-back launches (wall time and HIP events over the region);
    # left out with --main-only, so that a profiler's per-kernel average
    # covers the cold launches only
    ms_warm_step = ms_warm_kernel = None
    if not args.main_only:
        ms_warm_step, ms_warm_kernel = time_plan(plan, inputs, out, args.steps, args.warmup)
    # cold (the headline): each launch follows an untimed 1 GiB write that
    # flushes the L2 and the Infinity Cache; warmup launches too
    flush_buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda:0")
    flush = lambda: flush_buf.fill_(1.0)   # noqa: E731
    for _ in range(args.warmup):
        flush()
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold_ms = launch_times(run, args.steps, flush=flush)
    torch.cuda.synchronize()
    cold_wall_s = time.perf_counter() - t0
    ms_step = float(np.mean(cold_ms))
    value = p.n_vis / (ms_step * 1e-3)
    comp = compulsory_bytes(p, 8)
    counters = committed_counters("degrid")
    roof = roofline_object(p.n_vis, BYTES_PER_VIS["c64"], ms_step, comp, counters, "degrid_kernel<c64,f32>")
    log(f"fp32: cold {ms_step:.4f} ms/launch ({value:.4g} vis/s), warm {ms_warm_step} ms/step; "
        f"bound {roof['bound']} at {roof['frac']:.2%}")

    result = {
        "metric": "degridded visibilities/sec + HBM GB/s % peak (FP32 vs batched BF16) at rel-L2",
        "value": value,
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": p.name, "subgrids": p.n_subgrids, "subgrid_shape": [p.n_v, p.n_u, p.n_w],
                   "visibilities": p.n_vis, "os_uv": p.os_uv, "os_w": p.os_w, "grid_dtype": "c64",
                   "gcf_dtype": "f32", "n_b": info["n_b"], "grid_blocks": info["grid_blocks"],
                   "kernel": info["kernel"], "seed": 1,
                   "timing": "cold: each of the timed launches follows an untimed 1 GiB write (L2 and "
                             "Infinity Cache flushed); ms_per_step is the mean HIP-event duration of the "
                             "timed launches on the launch stream"},
        "roofline": roof,
        "timing": {"cold_kernel_ms": percentiles(cold_ms), "cold_region_wall_s": cold_wall_s,
                   "warm_ms_per_step": ms_warm_step, "warm_kernel_ms_mean": ms_warm_kernel,
                   "warm_value": p.n_vis / (ms_warm_step * 1e-3) if ms_warm_step else None},
    }
    # Per-launch distribution back to back, the memory system's plain-copy rate
    if not args.main_only:
        del flush_buf
        torch.cuda.empty_cache()
        warm = percentiles(launch_times(run, 50))
        result["timing"]["warm_kernel_ms"] = warm
        result["timing"]["warm_median_value"] = p.n_vis / (warm["median"] * 1e-3)
        result["roofline"]["hbm"]["copy_gbs"] = copy_bandwidth()
        result["device"] = {"name": torch.cuda.get_device_name(0),
                            "compute_units": torch.cuda.get_device_properties(0).multi_processor_count}
        log(f"warm median {warm['median']:.4f} ms, copy {result['roofline']['hbm']['copy_gbs']:.0f} GB/s, "
            f"compulsory {comp / 1e9:.3f} GB/launch")
    if tune_s is not None:
        result["config"]["tune_s"] = tune_s
    result["config"]["work_order"] = ("input order" if args.input_order else
                                      "plan-time Hilbert order of cells (degrid_plan_sort, once per coordinate set)")
    if sort_s is not None:
        result["config"]["plan_sort_s"] = sort_s
    if sort_s is not None and not args.main_only:
        result["input_order"] = {"value": p.n_vis / (ms_in_order * 1e-3), "ms_per_step": ms_in_order,
                                 "kernel_ms": kms_in_order, "note": "warm, back to back"}

    # Low-precision storage of the same inputs (complex bf16 / fp16 subgrids,
    # fp16 / bf16 tables, fp32 accumulation), each with the plan's default kernel.
    variants = {}
    if not args.no_variants:
        for gdt, tdt in LOW_PRECISION_FORMS:
            key = f"{gdt}/{tdt}"
            vin = upload_inputs(p, gdt, tdt)
            vplan = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w, grid_dtype=gdt, gcf_dtype=tdt)
            if not args.input_order:
                vplan.sort(vin[3])
            vout = torch.empty_like(out)
            vms_warm, _ = time_plan(vplan, vin, vout, args.steps, args.warmup)
            vrun = lambda: vplan.execute(*vin, out=vout)   # noqa: E731
            vms = float(np.mean(cold_launches(vrun, args.steps)))
            variants[key] = {"value": p.n_vis / (vms * 1e-3), "ms_per_step": vms,
                             "speedup_vs_fp32": ms_step / vms, "grid_dtype": gdt, "gcf_dtype": tdt,
                             "warm_ms_per_step": vms_warm, "warm_speedup_vs_fp32": ms_warm_step / vms_warm,
                             "kernel": vplan.info()["kernel"],
                             "effective_gbs": BYTES_PER_VIS[gdt] * p.n_vis / (vms * 1e-3) / 1e9,
                             "out": vout}
            del vin
            log(f"{key}: cold {vms:.4f} ms ({variants[key]['speedup_vs_fp32']:.2f}x fp32), "
                f"warm {vms_warm:.4f} ms ({variants[key]['warm_speedup_vs_fp32']:.2f}x)")

    if not args.no_cpu_baseline:
        import oracle
        a64 = p.subgrids.astype(np.complex128)
        cores = len(os.sched_getaffinity(0))
        threads0 = oracle.num_threads()
        # the whole workload, repeated for about 10 s (at least 3 runs)
        runs, ref = [], None
        while len(runs) < 3 or sum(runs) < 10.0:
            t = time.perf_counter()
            ref, _ = oracle.degrid(a64, p.g_uv, p.g_w, p.uvw, p.offsets)
            runs.append(time.perf_counter() - t)
        cpu_s = float(np.median(runs))
        # one thread, on the first eight subgrids (about 1/8 of the work),
        # repeated for about 5 s
        n8 = int(p.offsets[8])
        oracle.set_num_threads(1)
        one_runs = []
        while not one_runs or sum(one_runs) < 5.0:
            t = time.perf_counter()
            oracle.degrid(a64[:8], p.g_uv, p.g_w, p.uvw[:n8], p.offsets[:9])
            one_runs.append(time.perf_counter() - t)
        one_s = float(np.median(one_runs))
        oracle.set_num_threads(threads0)
        got = out.cpu().numpy().astype(np.complex128)
        rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        result["cpu_baseline"] = {"value": p.n_vis / cpu_s, "unit": "visibilities/s",
                                  "cores": threads0, "kind": "oracle",
                                  "sample": f"the whole workload ({p.n_vis} visibilities), FP64 C oracle, "
                                            f"median of {len(runs)} runs ({cpu_s:.3f} s each, {sum(runs):.1f} s in all) "
                                            f"on {threads0} OpenMP threads",
                                  "one_thread_value": n8 / one_s,
                                  "one_thread_sample": f"subgrids 0-7 ({n8} visibilities), median of {len(one_runs)} runs "
                                                       f"({one_s:.3f} s each)",
                                  "host_cores": cores, "cpu_model": cpu_model()}
        result["rel_l2"] = rel
        result["max_abs"] = float(np.max(np.abs(got - ref)))
        for v in variants.values():
            gdt, tdt = v["grid_dtype"], v["gcf_dtype"]
            deq = wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, gdt), gdt)
            g_uv_q, g_w_q = wl.stored_tables(p, tdt)
            ref_q, _ = oracle.degrid(deq, g_uv_q, g_w_q, p.uvw, p.offsets)
            gv = v["out"].cpu().numpy().astype(np.complex128)
            v["rel_l2_vs_fp32_inputs"] = float(np.linalg.norm(gv - ref) / np.linalg.norm(ref))
            v["rel_l2_vs_stored_inputs"] = float(np.linalg.norm(gv - ref_q) / np.linalg.norm(ref_q))
            v["error_budget_used"] = v["rel_l2_vs_fp32_inputs"] / LOW_PRECISION_REL_L2
    for v in variants.values():
        v.pop("out", None)
    if variants:
        result["variants"] = variants
    if not args.no_patterns:
        del inputs, out
        torch.cuda.empty_cache()
        result["latency"] = bench_latency()
        result["batched"] = bench_batched(args.steps, args.warmup, not args.no_cpu_baseline)
        result["differentiation"] = bench_differentiation(args.steps, args.warmup, not args.no_cpu_baseline)
    print(json.dumps(result), flush=True)
    return 0


def bench_batched(steps, warmup, check):
    """Eight independent problems (S in 4..64, counts log-uniform in
    [2^8, 2^18], os in {8, 16, 32}, seed 2) in one persistent launch replayed
    from a HIP graph, against the same eight plans launched one by one."""
    import numpy as np
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import Batch, Plan, batch_tune
    t = time.perf_counter()
    probs = wl.batched(seed=2)
    log(f"batched workload: {[p.n_subgrids for p in probs]} subgrids, {sum(p.n_vis for p in probs)} visibilities, "
        f"generated in {time.perf_counter() - t:.1f}s")
    ins = [upload_inputs(p) for p in probs]
    outs = [torch.empty(p.n_vis, dtype=torch.complex64, device="cuda:0") for p in probs]
    plans = []
    t = time.perf_counter()
    for p, i in zip(probs, ins):
        pl = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w)
        pl.sort(i[3])
        plans.append(pl)
    plan_s = time.perf_counter() - t
    args = [i for i in ins]
    t = time.perf_counter()
    kernel, n_b = batch_tune(plans, args, outs=outs)
    tune_s = time.perf_counter() - t
    batch = Batch(plans)
    stream = torch.cuda.current_stream()
    n_vis = sum(p.n_vis for p in probs)

    def run_batch():
        batch.execute(args, outs=outs, stream=stream)

    def run_plain():
        for pl, i, o in zip(plans, ins, outs):
            pl.execute(*i, out=o, stream=stream)

    res = {"workload": "batched-8-problems-S4..64-loguniform-2^8..2^18-os8/16/32", "visibilities": n_vis,
           "problems": len(probs), "plan_and_sort_s": plan_s,
           "autotune": {"kernel": kernel, "n_b": n_b, "tune_s": tune_s,
                        "candidates": "kernel variants x n_b in {8,16,32,64}, one batch launch each"}}
    for name, fn in (("batch_graph", run_batch), ("separate_launches", run_plain)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"ms_per_step": ms, "value": n_vis / (ms * 1e-3)}
    res["speedup_batch_vs_separate"] = res["separate_launches"]["ms_per_step"] / res["batch_graph"]["ms_per_step"]
    run_batch()
    torch.cuda.synchronize()
    fp32_out = [o.cpu().numpy().astype(np.complex128) for o in outs]
    batch.close()
    del ins, batch, plans
    torch.cuda.empty_cache()

    # The same eight problems in 16-bit forms, one graph launch each: bf16
    # storage with bf16 tables (packed bf16 dot products), bf16 storage with
    # fp16 tables (the precision configuration's table type; both widened to
    # fp32) and fp16 storage with fp16 tables (packed fp16 dot products);
    # fp32 accumulation and fp64 index arithmetic in all three.
    low_out = {}
    for key, gdt, tdt in (("batch_graph_bf16", "cbf16", "bf16"), ("batch_graph_bf16_f16tables", "cbf16", "f16"),
                          ("batch_graph_fp16", "cf16", "f16")):
        lins = [upload_inputs(p, gdt, tdt) for p in probs]
        lplans = []
        for p, i in zip(probs, lins):
            pl = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w, grid_dtype=gdt, gcf_dtype=tdt)
            pl.sort(i[3])
            lplans.append(pl)
        t = time.perf_counter()
        lkernel, ln_b = batch_tune(lplans, lins, outs=outs)
        ltune_s = time.perf_counter() - t
        lbatch = Batch(lplans)

        def run_low():
            lbatch.execute(lins, outs=outs, stream=stream)

        for _ in range(warmup):
            run_low()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run_low()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[key] = {"ms_per_step": ms, "value": n_vis / (ms * 1e-3), "grid_dtype": gdt, "gcf_dtype": tdt,
                    "autotune": {"kernel": lkernel, "n_b": ln_b, "tune_s": ltune_s},
                    "speedup_vs_plain_fp32_separate": res["separate_launches"]["ms_per_step"] / ms,
                    "speedup_vs_batch_fp32": res["batch_graph"]["ms_per_step"] / ms,
                    "achieved_gbs": BYTES_PER_VIS[gdt] * n_vis / (ms * 1e-3) / 1e9}
        run_low()
        torch.cuda.synchronize()
        low_out[key] = [o.cpu().numpy().astype(np.complex128) for o in outs]
        lbatch.close()
        del lins, lbatch, lplans
        torch.cuda.empty_cache()
    if check:
        import oracle
        acc = {"fp32": [0.0, 0.0]}
        worst = {k: 0.0 for k in low_out}
        for j, p in enumerate(probs):
            ref, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
            pairs = [("fp32", fp32_out[j], ref)]
            for key, lo in low_out.items():
                gdt, tdt = res[key]["grid_dtype"], res[key]["gcf_dtype"]
                deq = wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, gdt), gdt)
                g_uv_q, g_w_q = wl.stored_tables(p, tdt)
                ref_q, _ = oracle.degrid(deq, g_uv_q, g_w_q, p.uvw, p.offsets)
                pairs += [(key + ":fp32_inputs", lo[j], ref), (key + ":stored_inputs", lo[j], ref_q)]
                worst[key] = max(worst[key], float(np.max(np.abs(lo[j] - ref))))
            for name, got, r in pairs:
                a = acc.setdefault(name, [0.0, 0.0])
                a[0] += float(np.sum(np.abs(got - r) ** 2))
                a[1] += float(np.sum(np.abs(r) ** 2))
        res["rel_l2"] = (acc["fp32"][0] / acc["fp32"][1]) ** 0.5
        for key in low_out:
            for which in ("fp32_inputs", "stored_inputs"):
                a = acc[f"{key}:{which}"]
                res[key][f"rel_l2_vs_{which}"] = (a[0] / a[1]) ** 0.5
            res[key]["error_budget_used"] = res[key]["rel_l2_vs_fp32_inputs"] / LOW_PRECISION_REL_L2
            res[key]["max_abs_vs_fp32_inputs"] = worst[key]
    log(f"batched: graph {res['batch_graph']['ms_per_step']:.3f} ms, separate {res['separate_launches']['ms_per_step']:.3f} ms, "
        f"bf16 graph {res['batch_graph_bf16']['ms_per_step']:.3f} ms, "
        f"bf16/f16-tables graph {res['batch_graph_bf16_f16tables']['ms_per_step']:.3f} ms, "
        f"fp16 graph {res['batch_graph_fp16']['ms_per_step']:.3f} ms")
    return res


def bench_differentiation(steps, warmup, check):
    """Loss ||degrid(A) - V_obs||^2 on 16 subgrids with 2^16 uniform random
    visibilities each (seed 4); one step = forward degrid + backward (the
    gridding adjoint through torch.autograd). Also checks, on the GPU
    outputs with float64 sums on the host, the adjoint identity
    <degrid A, V> = <A, grid V> and the gradient against central
    differences (exact for a quadratic loss) at 64 random points, and times
    the gradients with respect to both tables (checked against the oracle's)."""
    import numpy as np
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import DegridFn, Plan, ResidualLossFn
    p = wl.differentiation(seed=4)
    dev = torch.device("cuda:0")
    sub, g_uv, g_w, uvw = upload_inputs(p)
    plan = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w)
    plan.sort(uvw)
    noise = wl.complex_noise(4, p.n_vis, 0.01)
    if check:
        import oracle
        v_true, _ = oracle.degrid(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets)
        v_obs_host = (v_true + noise).astype(np.complex64)
    else:
        v_obs_host = (plan.execute(sub, g_uv, g_w, uvw).cpu().numpy() + noise).astype(np.complex64)
    v_obs = torch.from_numpy(v_obs_host).to(dev)
    a_host = (p.subgrids + wl.perturbation(4, plan.shape, 0.1)).astype(np.complex64)
    a = torch.from_numpy(a_host).to(dev).requires_grad_(True)

    def step():
        a.grad = None
        vis = DegridFn.apply(a, plan, g_uv, g_w, uvw)
        loss = torch.sum(torch.abs(vis - v_obs) ** 2)
        loss.backward()

    def step_fused():
        a.grad = None
        loss = ResidualLossFn.apply(a, plan, g_uv, g_w, uvw, v_obs)
        loss.backward()

    out = torch.empty(p.n_vis, dtype=torch.complex64, device=dev)
    res_buf = torch.empty(p.n_vis, dtype=torch.complex64, device=dev)
    loss_buf = torch.empty((), dtype=torch.float64, device=dev)
    vin = torch.from_numpy(wl.complex_noise(5, p.n_vis, 1.0).astype(np.complex64)).to(dev)
    gout = torch.empty(plan.shape, dtype=torch.complex64, device=dev)
    tg_uv = torch.empty(g_uv.shape, dtype=torch.float32, device=dev)
    tg_w = torch.empty(g_w.shape, dtype=torch.float32, device=dev)
    res = {"workload": "differentiation-S16-65536-uniform", "visibilities": p.n_vis,
           "v_obs": "oracle degrid of the true subgrids + N(0, 0.01^2) per component" if check
           else "GPU degrid of the true subgrids + N(0, 0.01^2) per component"}
    for name, fn in (("forward_backward", step),
                     ("fused_forward_backward", step_fused),
                     ("residual_and_loss", lambda: plan.residual(a.detach(), g_uv, g_w, uvw, v_obs, out=res_buf,
                                                                 loss=loss_buf)),
                     ("degrid", lambda: plan.execute(sub, g_uv, g_w, uvw, out=out)),
                     ("adjoint", lambda: plan.adjoint(vin, g_uv, g_w, uvw, out=gout)),
                     ("table_gradients", lambda: plan.table_grad(sub, g_uv, g_w, uvw, vin, out_uv=tg_uv,
                                                                 out_w=tg_w))):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        res[name] = {"ms_per_step": ms, "value": p.n_vis / (ms * 1e-3)}
    res["adjoint"]["achieved_gbs"] = BYTES_PER_VIS["c64"] * p.n_vis / (res["adjoint"]["ms_per_step"] * 1e-3) / 1e9
    res["fused_speedup"] = res["forward_backward"]["ms_per_step"] / res["fused_forward_backward"]["ms_per_step"]
    # the fused loss against the unfused one (float64 sum of the GPU residuals)
    _, fl = plan.residual(a.detach(), g_uv, g_w, uvw, v_obs)
    unfused = float(np.sum(np.abs(v_obs_host.astype(np.complex128) -
                                  plan.execute(a.detach(), g_uv, g_w, uvw).cpu().numpy().astype(np.complex128)) ** 2))
    res["fused_loss_rel_diff"] = abs(fl.item() - unfused) / unfused

    # adjoint identity
    fwd = plan.execute(a.detach(), g_uv, g_w, uvw).cpu().numpy().astype(np.complex128)
    adj = plan.adjoint(vin, g_uv, g_w, uvw).cpu().numpy().astype(np.complex128)
    v64 = vin.cpu().numpy().astype(np.complex128)
    lhs = np.vdot(fwd, v64)
    rhs = np.vdot(a_host.astype(np.complex128), adj)
    res["adjoint_identity_rel"] = float(abs(lhs - rhs) / (np.linalg.norm(fwd) * np.linalg.norm(v64)))

    # central differences, h = 1 (exact for the quadratic loss), termwise in float64
    step()
    torch.cuda.synchronize()
    grad = a.grad.detach().reshape(-1).cpu().numpy()
    rng = np.random.default_rng(40)
    points = rng.choice(grad.size, size=64, replace=False)
    vo = v_obs_host.astype(np.complex128)
    worst = 0.0
    a0 = a.detach()
    flat = a0.view(-1)
    for idx in points:
        keep = flat[int(idx)].clone()
        for part, e in (("re", 1.0), ("im", 1.0j)):
            rs = []
            for sign in (1.0, -1.0):
                flat[int(idx)] = keep + sign * e
                r = plan.execute(a0, g_uv, g_w, uvw).cpu().numpy().astype(np.complex128) - vo
                rs.append(r)
            flat[int(idx)] = keep
            fd = float(np.sum(np.abs(rs[0]) ** 2 - np.abs(rs[1]) ** 2)) / 2.0
            g = float(grad[idx].real if part == "re" else grad[idx].imag)
            worst = max(worst, abs(fd - g))
    scale = float(np.max(np.abs(grad)))
    res["finite_difference"] = {"points": 64, "components": 128, "h": 1.0,
                                "max_abs_err": worst, "max_abs_err_over_max_grad": worst / scale}
    if check:
        import oracle
        r, _ = oracle.degrid(a_host, p.g_uv, p.g_w, p.uvw, p.offsets)
        ref, _ = oracle.grid(2.0 * (r - vo), p.g_uv, p.g_w, p.uvw, p.offsets, plan.shape)
        got = a.grad.cpu().numpy()
        res["gradient_rel_l2"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        # table gradients of L = Re<vin, degrid(A_true)> against the oracle's
        gu, gw = plan.table_grad(sub, g_uv, g_w, uvw, vin)
        ref_uv, ref_w, _ = oracle.table_grad(p.subgrids, p.g_uv, p.g_w, p.uvw, p.offsets, vin.cpu().numpy())
        res["table_gradients"]["rel_l2_g_uv"] = float(np.linalg.norm(gu.cpu().numpy() - ref_uv) / np.linalg.norm(ref_uv))
        res["table_gradients"]["rel_l2_g_w"] = float(np.linalg.norm(gw.cpu().numpy() - ref_w) / np.linalg.norm(ref_w))
    log(f"differentiation: forward+backward {res['forward_backward']['ms_per_step']:.3f} ms "
        f"(fused {res['fused_forward_backward']['ms_per_step']:.3f} ms), "
        f"adjoint {res['adjoint']['ms_per_step']:.3f} ms, table gradients {res['table_gradients']['ms_per_step']:.3f} ms, "
        f"identity {res['adjoint_identity_rel']:.2e}, "
        f"fd {res['finite_difference']['max_abs_err_over_max_grad']:.2e}")
    return res


def bench_latency(launches=1000, replays=5):
    """The small case: 2 subgrids of 512 x 512 x 4 with 1024 visibilities
    each on a folded line (seed 0). A launch lasts microseconds, so this is a
    latency figure: 1000 launches captured in one HIP graph and replayed
    (per-launch time), beside the same 1000 launches issued one by one."""
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import Plan
    p = wl.plain_line(seed=0)
    ins = upload_inputs(p)
    plan = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w)
    plan.sort(ins[3])
    ref = plan.execute(*ins)
    out = torch.empty_like(ref)
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(cur)
    for _ in range(launches):
        plan.execute(*ins, out=out, stream=cur)
    e1.record(cur)
    e1.synchronize()
    eager_us = e0.elapsed_time(e1) * 1e3 / launches
    side = torch.cuda.Stream()
    side.wait_stream(cur)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        for _ in range(launches):
            plan.execute(*ins, out=out, stream=side)
    torch.cuda.synchronize()
    per = []
    same = True
    for _ in range(replays):
        out.zero_()
        torch.cuda.synchronize()
        e0.record(cur)
        g.replay()
        e1.record(cur)
        e1.synchronize()
        per.append(e0.elapsed_time(e1) * 1e3 / launches)
        same = same and bool(torch.equal(out, ref))
    del g
    res = {"workload": f"plain-line-S2-1024 ({p.n_vis} visibilities)", "launches": launches,
           "graph_us_per_launch": percentiles(per), "eager_us_per_launch": eager_us,
           "graph_replays_match_eager": same,
           "label": "latency (launch-bound: the work is a few microseconds)"}
    log(f"latency: graph {res['graph_us_per_launch']['median']:.2f} us/launch, eager {eager_us:.2f} us/launch")
    return res


def study_markdown(study):
    """Markdown tables of a --study result: per scenario and count, the best
    vis/s of each mapping over the two work orders ("s": the sorted order)."""
    rows = study["rows"]
    maps = []
    for r in rows:
        if r["mapping"] not in maps:
            maps.append(r["mapping"])
    best = {}
    for r in rows:
        k = (r["scenario"], r["n_per_subgrid_max"], r["mapping"])
        if k not in best or r["vis_per_s"] > best[k]["vis_per_s"]:
            best[k] = r
    out = [f"# {study['study']}: {study['subgrids']} subgrids of 512 x 512 x 4, line-shaped visibilities", "",
           "Command: `python3 bench.py --study --steps 10 --warmup 3 > study.json`, then "
           "`python3 bench.py --study-md study.json`. Median kernel time of the timed launches; vis/s per mapping, "
           "the better of input order and the plan-time work order (\"s\": sorted). \"equal\": every subgrid N "
           "visibilities; \"ramp\": subgrid k of 16 has N (k + 1) / 16.", ""]
    for sc in ("equal", "ramp"):
        ns = sorted({r["n_per_subgrid_max"] for r in rows if r["scenario"] == sc})
        out += [f"## {sc}", "", "| N | " + " | ".join(maps) + " | best | D1-like / best |",
                "|---|" + "---|" * (len(maps) + 2)]
        for n in ns:
            cells, top, top_m, d1 = [], 0.0, "", 0.0
            for m in maps:
                r = best.get((sc, n, m))
                if r is None:
                    cells.append("-")
                    continue
                v = r["vis_per_s"]
                cells.append(f"{v:.3g}" + (" s" if r["order"] == "sorted" else ""))
                if v > top:
                    top, top_m = v, m
                if m.startswith("D1"):
                    d1 = max(d1, v)
            exp = n.bit_length() - 1
            out.append(f"| 2^{exp} | " + " | ".join(cells) + f" | {top_m} | {d1 / top:.2f} |")
        out.append("")
    return "\n".join(out)


def bench_study(steps, warmup):
    """The two count scenarios of Section 3 on this GPU: S = 16 subgrids of
    512 x 512 x 4 with line-shaped visibilities (constant step, as the paper
    measures), N per subgrid from 2^8 to 2^20, either equal for every subgrid
    or rising linearly to N in the last one; for each, the gather kernel
    mappings (through the caches with one or 64 visibilities per tile, and
    LDS-staged with 12 KiB or 18 KiB boxes), in input order and after the
    plan-time work order. Median kernel time over the timed launches."""
    import numpy as np
    import torch
    from paper_2102_12739_amd import workload as wl
    from paper_2102_12739_amd.degrid import Plan
    dev = torch.device("cuda:0")
    s_sub = 16
    base = wl.make_problem("study-grid", [1] * s_sub, seed=7, kind="line")
    sub = torch.from_numpy(base.subgrids).to(dev)
    g_uv = torch.from_numpy(base.g_uv).to(dev)
    g_w = torch.from_numpy(base.g_w).to(dev)
    # the tap-per-lane mapping (close to the paper's D4) through the caches
    # and with LDS boxes, and the D1 mapping (two visibilities per
    # wavefront, accumulation along v)
    mappings = [("D4-like cache gather, n_b 1", 0, 1), ("D4-like cache gather, n_b 64", 0, 64),
                ("D4-like LDS box 12 KiB, n_b 32", 2, 32), ("D4-like LDS box 18 KiB, n_b 64", 4, 64),
                ("D1-like, n_b 32", 6, 32), ("D1-like, n_b 64", 6, 64)]
    rows = []
    for scenario in ("equal", "ramp"):
        for e in (8, 10, 12, 14, 16, 18, 20):
            counts = wl.count_profile(scenario, s_sub, 2 ** e)
            p = wl.make_problem(f"study-{scenario}-2^{e}", counts, seed=7 + e, kind="line", with_grid=False)
            uvw = torch.from_numpy(p.uvw).to(dev)
            out = torch.empty(p.n_vis, dtype=torch.complex64, device=dev)
            for order in ("input", "sorted"):
                plan = Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w)
                if order == "sorted":
                    plan.sort(uvw)
                for label, var, nb in mappings:
                    if nb == 1 and 2 ** e > 2 ** 16:
                        continue   # one tile per visibility: kept to the sizes where it can matter
                    plan.set_kernel(var, nb)
                    run = lambda: plan.execute(sub, g_uv, g_w, uvw, out=out)   # noqa: E731
                    for _ in range(warmup):
                        run()
                    ms = percentiles(launch_times(run, steps))["median"]
                    rows.append({"scenario": scenario, "n_per_subgrid_max": 2 ** e, "visibilities": p.n_vis,
                                 "order": order, "mapping": label, "kernel": var, "n_b": nb,
                                 "kernel_us": ms * 1e3, "vis_per_s": p.n_vis / (ms * 1e-3)})
                    log(f"study {scenario:5s} N=2^{e:<2d} {order:6s} {label:24s} {ms * 1e3:9.1f} us "
                        f"{p.n_vis / (ms * 1e-3):.3e} vis/s")
                plan.close()
            del uvw, out
            torch.cuda.empty_cache()
    best = {}
    for r in rows:
        k = (r["scenario"], r["n_per_subgrid_max"])
        if k not in best or r["vis_per_s"] > best[k]["vis_per_s"]:
            best[k] = r
    return {"study": "count scenarios x gather mappings (Section 3)", "subgrids": s_sub, "rows": rows,
            "best": [{"scenario": k[0], "n_per_subgrid_max": k[1], "mapping": v["mapping"], "order": v["order"],
                      "vis_per_s": v["vis_per_s"]} for k, v in sorted(best.items())]}


if __name__ == "__main__":
    sys.exit(main())
