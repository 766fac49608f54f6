"""C-ABI checks that need no GPU: exported symbols, struct layout, argument
validation, status strings, and the host-side tile decomposition."""

import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "degrid.h")
CSRC = os.path.join(ROOT, "paper_2102_12739_amd", "csrc")


@pytest.fixture(scope="module")
def dg():
    from paper_2102_12739_amd import degrid
    if not os.path.exists(degrid.library_path()):
        from paper_2102_12739_amd import build
        build.build()
    degrid.lib()
    return degrid


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("degrid_", "grid_"))))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("degrid_plan", "degrid_execute", "grid_adjoint", "degrid_oob_count", "degrid_destroy",
                 "degrid_batch_plan", "degrid_batch_execute", "degrid_status_str", "degrid_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(dg):
    lib = ctypes.CDLL(dg.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_ctypes(tmp_path):
    exe = tmp_path / "abi_layout"
    subprocess.run(["gcc", "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "cpp", "abi_layout.c"),
                    "-o", str(exe)], check=True)
    got = json.loads(subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout)
    from paper_2102_12739_amd.degrid import DgDesc, DgPlanInfo
    assert got["dg_desc"] == [ctypes.sizeof(DgDesc), DgDesc.os_uv.offset, DgDesc.grid_dtype.offset,
                              DgDesc.n_b.offset, DgDesc.flags.offset, DgDesc.support_w.offset]
    assert got["dg_plan_info"] == [ctypes.sizeof(DgPlanInfo), DgPlanInfo.n_tiles.offset, DgPlanInfo.n_b.offset,
                                   DgPlanInfo.n_queues.offset, DgPlanInfo.device.offset, DgPlanInfo.sorted.offset,
                                   DgPlanInfo.n_kernels.offset]


def test_status_strings_and_version(dg):
    L = dg.lib()
    for code, name in dg._STATUS.items():
        assert L.degrid_status_str(code).decode() == name
    assert L.degrid_version() >= 100


def _plan_raw(dg, desc, offsets, n_sub=None):
    off = np.asarray(offsets, dtype=np.int64)
    h = ctypes.c_void_p()
    st = dg.lib().degrid_plan(ctypes.byref(desc) if desc is not None else None,
                              len(off) - 1 if n_sub is None else n_sub,
                              off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, ctypes.byref(h))
    return st, h


def _desc(dg, **kw):
    base = dict(n_v=512, n_u=512, n_w=4, support_uv=8, support_w=4, os_uv=16, os_w=16,
                grid_dtype=0, gcf_dtype=0, n_b=32, flags=0)
    base.update(kw)
    return dg.DgDesc(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(os_uv=65), 1), (dict(os_w=0), 1), (dict(os_uv=128), 1), (dict(os_w=65), 1), (dict(flags=1), 1),
    (dict(n_b=65), 1), (dict(n_b=-1), 1), (dict(grid_dtype=3), 1), (dict(gcf_dtype=3), 1),
    (dict(n_v=7), 1), (dict(support_uv=6), 2), (dict(support_w=6), 2), (dict(n_w=3), 1),
    (dict(support_uv=0), 1), (dict(n_v=8192, n_u=8192), 2),
    # first taps are packed into 16 bits per axis (0xFFFFFFFF means "none")
    (dict(n_v=8, n_u=65544), 2), (dict(n_v=65543, n_u=8), 2),
])
def test_invalid_descriptors_are_rejected_before_device_work(dg, kw, status):
    st, h = _plan_raw(dg, _desc(dg, **kw), [0, 10])
    assert st == status
    assert h.value is None
    assert dg.lib().degrid_last_error().decode() != ""


@pytest.mark.parametrize("offsets,n_sub", [([1, 10], None), ([0, 10, 5], None), ([0, 3], -1)])
def test_invalid_offsets_are_rejected(dg, offsets, n_sub):
    st, h = _plan_raw(dg, _desc(dg), offsets, n_sub)
    assert st == 1 and h.value is None


def test_largest_side_lengths_pass_validation(dg):
    """The largest sides whose first taps still pack into 16 bits per axis
    get past validation (they then fail only for want of a device here)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present: the plan would be built")
    for kw in (dict(n_v=8, n_u=65543), dict(n_v=65542, n_u=8)):
        st, h = _plan_raw(dg, _desc(dg, **kw), [0, 10])
        assert st == 4 and h.value is None   # DG_ERR_HIP: no device


@pytest.mark.parametrize("offsets", [[0, 1 << 32], [0, (1 << 31), (1 << 32) + 5]])
def test_visibility_counts_of_2_to_the_32_are_refused(dg, offsets):
    """Work items and work orders hold 32-bit visibility indices: a plan of
    2^32 or more visibilities is refused before any device work."""
    st, h = _plan_raw(dg, _desc(dg), offsets)
    assert st == 2 and h.value is None
    assert "2^32" in dg.lib().degrid_last_error().decode()


def test_null_arguments(dg):
    L = dg.lib()
    st, _ = _plan_raw(dg, None, [0, 1])
    assert st == 1
    assert L.degrid_execute(None, 1, 1, 1, 1, 1, None) == 1
    assert L.grid_adjoint(None, 1, 1, 1, 1, 1, 0, None) == 1
    assert L.degrid_oob_count(None, None) == 1
    assert L.degrid_plan_get_info(None, None) == 1
    assert L.degrid_destroy(None) == 0
    assert L.degrid_batch_destroy(None) == 0
    assert L.degrid_batch_plan(None, 0, None) == 1
    assert L.degrid_plan_sort(None, None, None) == 1


def test_plan_without_device_reports_hip_error(dg):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _plan_raw(dg, _desc(dg), [0, 100])
    assert st == 4 and h.value is None
    assert "hip" in dg.lib().degrid_last_error().decode().lower()


def test_python_plan_raises_degrid_error(dg):
    with pytest.raises(dg.DegridError) as e:
        dg.Plan([0, 10], os_uv=65)
    assert e.value.status == 1


# ---------------------------------------------------------------------------
# Host work decomposition (plain C++, built with g++)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def plan_logic(tmp_path_factory):
    exe = tmp_path_factory.mktemp("pl") / "plan_logic_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC,
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(ROOT, "tests", "cpp", "plan_logic_check.cpp"),
                    os.path.join(CSRC, "plan_logic.cpp"), "-o", str(exe)], check=True)

    def run(nb, counts):
        r = subprocess.run([str(exe), str(nb), *map(str, counts)], capture_output=True, text=True, check=True)
        return json.loads(r.stdout)
    return run


@pytest.mark.parametrize("nb,counts", [
    (32, [1024, 1024]), (64, [0, 1, 63, 64, 65, 0, 129]), (1, [5, 0, 3]), (7, [100]),
    (32, []), (16, [0, 0, 0]), (64, list(np.random.default_rng(0).integers(0, 5000, 64))),
])
def test_tiles_cover_each_subgrid_exactly_once(plan_logic, nb, counts):
    out = plan_logic(nb, counts)
    tiles = out["tiles"]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    covered = np.zeros(int(off[-1]), dtype=np.int64)
    for begin, sub, count, problem in tiles:
        assert problem == 3
        assert 1 <= count <= nb
        assert off[sub] <= begin and begin + count <= off[sub + 1]
        covered[begin:begin + count] += 1
    assert np.all(covered == 1)
    # tiles are in subgrid order and only the last tile of a subgrid is short
    for (b0, s0, c0, _), (b1, s1, c1, _) in zip(tiles, tiles[1:]):
        assert (s1, b1) > (s0, b0)
        if s1 == s0:
            assert c0 == nb


@pytest.mark.parametrize("nb,counts", [
    (32, list(np.random.default_rng(1).integers(2 ** 10, 2 ** 18, 64))), (64, [10]), (8, [3, 3, 3]),
    (32, [0] * 5 + [100000] + [0] * 5), (16, list(np.random.default_rng(2).integers(0, 300, 40))),
])
def test_queues_partition_the_tile_list_and_balance_visibilities(plan_logic, nb, counts):
    out = plan_logic(nb, counts)
    n_tiles = len(out["tiles"])
    nq, begin, end = out["n_queues"], out["begin"], out["end"]
    assert 1 <= nq <= 8
    assert nq == min(8, max(1, n_tiles))
    assert begin[0] == 0 and end[-1] == n_tiles
    for q in range(nq):
        assert begin[q] <= end[q]
        if q:
            assert begin[q] == end[q - 1]
    vis = np.array([t[2] for t in out["tiles"]])
    if n_tiles >= 8 * 4:
        per_q = [vis[begin[q]:end[q]].sum() for q in range(nq)]
        share = vis.sum() / nq
        assert max(per_q) <= share + nb and min(per_q) >= share - nb


@pytest.mark.parametrize("nb,blocks,counts", [
    (64, 512, list(np.random.default_rng(3).integers(2 ** 10, 2 ** 18, 64))),   # paper-scale shape
    (64, 768, [65536] * 16), (64, 8, [1024, 1024]), (16, 3, [5000, 7000]), (8, 20, [3, 3, 3]),
    (32, 1, [100000]), (64, 512, [10]), (8, 64, [1024, 1024]), (8, 7, [100, 90]), (8, 8, [129, 128]),
])
def test_static_deal_gives_every_tile_to_exactly_one_claim(plan_logic_exe, nb, blocks, counts):
    """The launch's static deal (workgroup b serves queue b mod n_queues;
    wavefront r of a queue's workgroups takes begin + r, begin + r + stride,
    ... below sbase) together with the queue cursors (tiles sbase .. end)
    hands out every tile exactly once; a queue gets a static part only with
    at least 4 tiles per serving wavefront, and then 6/8 of its tiles;
    when no queue holds more tiles than serving wavefronts, every tile is
    dealt statically (all_static, one tile per wavefront at most)."""
    r = subprocess.run([plan_logic_exe, "deal", str(nb), str(blocks), *map(str, counts)], capture_output=True, text=True,
                       check=True)
    d = json.loads(r.stdout)
    nq = d["n_queues"]
    n_tiles = d["end"][-1] if nq else 0
    seen = np.zeros(n_tiles, dtype=np.int64)
    any_static = False
    small = nq > 0 and all(len(range(q, blocks, nq)) > 0 and d["end"][q] - d["begin"][q] <= 4 * len(range(q, blocks, nq))
                           for q in range(nq))
    assert d["all_static"] == int(small)
    for q in range(nq):
        b, e, sb, w = d["begin"][q], d["end"][q], d["sbase"][q], d["stride"][q]
        nb_q = len(range(q, blocks, nq))
        assert w == 4 * nb_q
        assert b <= sb <= e
        size = e - b
        if small:
            assert sb == e and size <= w
        elif nb_q > 0 and size >= 4 * w:
            assert sb - b == size * 6 // 8
        else:
            assert sb == b
        any_static |= sb > b
        for rank in range(w):                      # static part, by rank
            for t in range(b + rank, sb, w):
                seen[t] += 1
        seen[sb:e] += 1                            # cursor part
    assert np.all(seen == 1)
    assert d["on"] == int(any_static)


def _fitted(plan_logic_exe, tmp_path, nb, cap, min_fit, pad_to, counts, starts):
    f = tmp_path / "starts.txt"
    f.write_text(" ".join(map(str, counts)) + "\n" + " ".join(map(str, starts)) + "\n")
    r = subprocess.run([plan_logic_exe, "fitted", str(nb), str(cap), str(min_fit), str(pad_to), str(f)],
                       capture_output=True, text=True, check=True)
    return json.loads(r.stdout)


@pytest.fixture(scope="module")
def plan_logic_exe(tmp_path_factory):
    exe = tmp_path_factory.mktemp("plf") / "plan_logic_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", os.path.join(ROOT, "tests", "cpp", "plan_logic_check.cpp"),
                    os.path.join(CSRC, "plan_logic.cpp"), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("seed,cap,min_fit,pad_to", [(0, 512, 16, 0), (1, 256, 8, 0), (2, 1024, 16, 16),
                                                    (3, 64, 4, 0), (4, 512, 16, 16)])
def test_fitted_tiles_cover_fit_the_box_and_are_greedy(plan_logic_exe, tmp_path, seed, cap, min_fit, pad_to):
    rng = np.random.default_rng(seed)
    nb, no_start = 64, 0xFFFFFFFF
    counts = [int(c) for c in rng.integers(0, 700, 6)] + [0, 1, 65]
    starts = []
    for c in counts:
        # clustered walk of start cells plus some out-of-range entries
        x, y = rng.integers(0, 500, 2)
        for _ in range(c):
            x = int(np.clip(x + rng.integers(-3, 4), 0, 504))
            y = int(np.clip(y + rng.integers(-3, 4), 0, 504))
            starts.append(no_start if rng.random() < 0.05 else (y << 16) | x)
    out = _fitted(plan_logic_exe, tmp_path, nb, cap, min_fit, pad_to, counts, starts)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    covered = np.zeros(int(off[-1]), dtype=np.int64)

    def area(lo, hi):
        xs = [s & 0xFFFF for s in starts[lo:hi] if s != no_start]
        ys = [s >> 16 for s in starts[lo:hi] if s != no_start]
        if not xs:
            return 0
        w = max(xs) - min(xs) + 8
        if pad_to:
            w += (pad_to // 2 - w) % pad_to      # width congruent to pad_to/2 mod pad_to
        return w * (max(ys) - min(ys) + 8)

    for begin, sub, count, problem in out["tiles"]:
        assert problem == 3 and 1 <= count <= nb
        assert off[sub] <= begin and begin + count <= off[sub + 1]
        covered[begin:begin + count] += 1
        end_of_sub = begin + count == off[sub + 1]
        if area(begin, begin + count) <= cap:
            # a fitting tile stops only at nb, at its subgrid's end, or where
            # one more visibility would not fit
            assert count == nb or end_of_sub or area(begin, begin + count + 1) > cap
        else:
            # a tile that does not fit is a full-size fallback: fewer than
            # min_fit visibilities fit at its start
            assert count == min(nb, off[sub + 1] - begin)
            k = 1
            while k < count and area(begin, begin + k + 1) <= cap:
                k += 1
            assert k < min_fit
    assert np.all(covered == 1)


@pytest.mark.parametrize("seed,block", [(0, 16), (1, 32), (2, 8)])
def test_block_lists_hold_exactly_the_overlapping_visibilities(plan_logic_exe, tmp_path, seed, block):
    """Output-block lists of the owner-computes adjoint: every (visibility,
    block) pair whose 8x8 neighbourhood overlaps the block appears once, in
    work order, and nothing else does."""
    rng = np.random.default_rng(seed)
    n_v, n_u, no_start = 48, 64, 0xFFFFFFFF
    counts = [int(c) for c in rng.integers(0, 300, 4)] + [0, 5]
    n = sum(counts)
    starts = []
    for _ in range(n):
        if rng.random() < 0.05:
            starts.append(no_start)
        else:
            x0, y0 = int(rng.integers(0, n_u - 7)), int(rng.integers(0, n_v - 7))
            starts.append((y0 << 16) | x0)
    vis = [int(v) for v in rng.permutation(n)]
    f = tmp_path / "blocks.txt"
    f.write_text("\n".join(" ".join(map(str, a)) for a in (counts, starts, vis)) + "\n")
    r = subprocess.run([plan_logic_exe, "blocks", str(n_v), str(n_u), str(block), str(f)],
                       capture_output=True, text=True, check=True)
    out = json.loads(r.stdout)
    nby, nbx = n_v // block, n_u // block
    off = np.concatenate([[0], np.cumsum(counts)])
    expect = {}
    for s in range(len(counts)):
        for p in range(off[s], off[s + 1]):
            if starts[p] == no_start:
                continue
            x0, y0 = starts[p] & 0xFFFF, starts[p] >> 16
            for by in range(nby):
                for bx in range(nbx):
                    if x0 + 7 >= bx * block and x0 < bx * block + block and \
                            y0 + 7 >= by * block and y0 < by * block + block:
                        expect.setdefault((s * nby + by) * nbx + bx, []).append(vis[p])
    offsets, items = out["offsets"], out["items"]
    assert len(offsets) == len(counts) * nby * nbx + 1
    for b in range(len(offsets) - 1):
        assert items[offsets[b]:offsets[b + 1]] == expect.get(b, []), b
