"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) and driven over small seeded problems with edge, non-finite
and out-of-range coordinates, empty subgrids, oversampling factors that are
not powers of two and deep w-stacks. Any invalid access or undefined
operation aborts the driver; its outputs must equal the ordinary build's."""

import os
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sanitized_run(tmp_path_factory):
    d = tmp_path_factory.mktemp("osan")
    exe = d / "oracle_sanitize"
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-ffp-contract=off", "-Wall", "-Wextra",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    os.path.join(ROOT, "tests", "cpp", "oracle_sanitize.c"),
                    os.path.join(ROOT, "oracle", "degrid_oracle.c"), "-o", str(exe), "-lm"], check=True)
    out = d / "cases.bin"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(out)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
    return out.read_bytes()


def _cases(blob):
    pos = 0

    def take(dtype, count):
        nonlocal pos
        a = np.frombuffer(blob, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a

    while pos < len(blob):
        n_sub, n_v, n_u, n_w, os_uv, os_w, n, _ = (int(x) for x in take(np.int64, 8))
        cells = n_sub * n_v * n_u * n_w
        c = {"shape": (n_sub, n_v, n_u, n_w), "os": (os_uv, os_w), "n": n}
        c["off"] = take(np.int64, n_sub + 1)
        c["sub"] = take(np.float64, 2 * cells).view(np.complex128).reshape(n_sub, n_v, n_u, n_w)
        c["g_uv"] = take(np.float64, os_uv * os_uv * 64).reshape(os_uv, os_uv, 8, 8)
        c["g_w"] = take(np.float64, os_w * 4).reshape(os_w, 4)
        c["uvw"] = take(np.float64, 3 * n).reshape(n, 3)
        c["gv"] = take(np.float64, 2 * n).view(np.complex128)
        c["oob"] = [int(x) for x in take(np.int64, 3)]
        c["vis"] = take(np.float64, 2 * n).view(np.complex128)
        c["grid"] = take(np.float64, 2 * cells).view(np.complex128).reshape(n_sub, n_v, n_u, n_w)
        c["d_uv"] = take(np.float64, os_uv * os_uv * 64).reshape(os_uv, os_uv, 8, 8)
        c["d_w"] = take(np.float64, os_w * 4).reshape(os_w, 4)
        yield c


def test_sanitized_oracle_runs_clean_and_matches_the_ordinary_build(sanitized_run):
    cases = list(_cases(sanitized_run))
    assert len(cases) == 4
    for c in cases:
        vis, oob_d = oracle.degrid(c["sub"], c["g_uv"], c["g_w"], c["uvw"], c["off"])
        grid, oob_g = oracle.grid(c["gv"], c["g_uv"], c["g_w"], c["uvw"], c["off"], c["shape"])
        d_uv, d_w, oob_t = oracle.table_grad(c["sub"], c["g_uv"], c["g_w"], c["uvw"], c["off"], c["gv"])
        assert c["oob"] == [oob_d, oob_g, oob_t]
        if c["n"] >= 30:
            assert oob_d >= 20   # the edge, non-finite and far-away coordinates
        # same loops and the same IEEE operations; only the summation order of
        # the threaded table gradients may differ
        assert np.array_equal(vis, c["vis"])
        assert np.array_equal(grid, c["grid"])
        for got, ref in ((d_uv, c["d_uv"]), (d_w, c["d_w"])):
            scale = max(1.0, float(np.max(np.abs(ref))))
            assert float(np.max(np.abs(got - ref))) <= 1e-12 * scale
