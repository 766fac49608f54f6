"""The oracle pins must reject plausible mistakes in the oracle.

Each mutant below is a copy of the oracle source with one planted slip (an
index transposed, an axis swapped, a tap dropped, a sign flipped, a wrong
rounding or start offset). Each is compiled on the CPU and the pin suite is
run against it in a subprocess; every mutant must make at least one pin fail.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "degrid_oracle.c")

MUTANTS = {
    "table_ov_ou_swapped": ("((int64_t)o_v * os_uv + o_u)", "((int64_t)o_u * os_uv + o_v)"),
    "table_taps_transposed": ("guv[tv * support_uv + tu]", "guv[tu * support_uv + tv]"),
    "grid_table_ov_ou_swapped": ("((int64_t)o_v * os_uv + o_u)", "((int64_t)o_u * os_uv + o_v)", 1),
    "grid_table_taps_transposed": ("guv[tv * support_uv + tu]", "guv[tu * support_uv + tv]", 1),
    "start_offset_by_one": ("n - (double)(support / 2 - 1)", "n - (double)(support / 2)"),
    "round_to_nearest": ("floor(c * (double)os)", "floor(c * (double)os + 0.5)"),
    "w_uses_uv_oversampling": ("uvw_i[2], g->os_w,", "uvw_i[2], g->os_uv,"),
    "u_v_coordinates_swapped": ("axis_coordinates(uvw_i[0], g->os_uv, g->support_uv, g->n_u, x, o_u)",
                                "axis_coordinates(uvw_i[1], g->os_uv, g->support_uv, g->n_u, x, o_u)"),
    "dropped_w_tap": ("for (int32_t tw = 0; tw < support_w; ++tw) {\n                        double weight = gw[tw] * guv[tv * support_uv + tu];\n                        int64_t cell = ((s",
                      "for (int32_t tw = 0; tw < support_w - 1; ++tw) {\n                        double weight = gw[tw] * guv[tv * support_uv + tu];\n                        int64_t cell = ((s"),
    "imag_sign": ("im += weight * subgrids[2 * cell + 1];", "im -= weight * subgrids[2 * cell + 1];"),
    "upper_bound_strict": ("!(first <= (double)(n_cells - support))", "!(first < (double)(n_cells - support))"),
    "owner_off_by_one": ("if (offsets[mid] <= i) lo = mid;", "if (offsets[mid] < i) lo = mid;"),
    "grid_imag_sign": ("out[2 * cell + 1] += weight * vis[2 * i + 1];", "out[2 * cell + 1] -= weight * vis[2 * i + 1];"),
    "grid_w_tap_shift": ("int64_t cell = (((y + tv)) * n_u + (x + tu)) * n_w + (z + tw);",
                         "int64_t cell = (((y + tv)) * n_u + (x + tu)) * n_w + (z + (tw + 1) % support_w);"),
    "grid_all_into_first_subgrid": ("double* out = subgrids_out + 2 * s * cells_per_sub;\n        memset",
                                    "double* out = subgrids_out + 2 * s * cells_per_sub;\n        if (s) out = subgrids_out;\n        memset"),
    "w_start_not_offset": ("double first = n - (double)(support / 2 - 1);",
                           "double first = (support == 4) ? n : n - (double)(support / 2 - 1);"),
    "tgrad_conj_sign": ("grad_g_uv[uv_row + tv * support_uv + tu] += gre * c_re + gim * c_im;",
                        "grad_g_uv[uv_row + tv * support_uv + tu] += gre * c_re - gim * c_im;"),
    "tgrad_taps_transposed": ("grad_g_uv[uv_row + tv * support_uv + tu] += gre",
                              "grad_g_uv[uv_row + tu * support_uv + tv] += gre"),
    "tgrad_w_missing_uv_weight": ("+= guv * (gre * a_re + gim * a_im);", "+= (gre * a_re + gim * a_im);"),
    "tgrad_w_taps_reversed": ("grad_g_w[(int64_t)o_w * support_w + tw] +=",
                              "grad_g_w[(int64_t)o_w * support_w + (support_w - 1 - tw)] +="),
    "tgrad_w_sum_skips_last_tap": ("c_re += gw[tw] * a_re;", "c_re += (tw < support_w - 1) ? gw[tw] * a_re : 0.0;"),
    "real_sign": ("re += weight * subgrids[2 * cell];", "re -= weight * subgrids[2 * cell];"),
    "grid_real_sign": ("out[2 * cell] += weight * vis[2 * i];", "out[2 * cell] -= weight * vis[2 * i];"),
    "lower_bound_strict": ("!(first >= 0.0)", "!(first > 0.0)"),
    "cell_not_floored": ("double n = floor(k / (double)os);", "double n = k / (double)os;"),
    "w_axis_bounded_by_n_v": ("uvw_i[2], g->os_w, g->support_w, g->n_w,", "uvw_i[2], g->os_w, g->support_w, g->n_v,"),
    "grid_v_tap_dropped": ("for (int32_t tv = 0; tv < support_uv; ++tv)\n                for (int32_t tu = 0; tu < support_uv; ++tu)\n                    for (int32_t tw = 0; tw < support_w; ++tw) {\n                        double weight = gw[tw] * guv[tv * support_uv + tu];\n                        int64_t cell = (((y",
                           "for (int32_t tv = 0; tv < support_uv - 1; ++tv)\n                for (int32_t tu = 0; tu < support_uv; ++tu)\n                    for (int32_t tw = 0; tw < support_w; ++tw) {\n                        double weight = gw[tw] * guv[tv * support_uv + tu];\n                        int64_t cell = (((y"),
    "tgrad_uv_uses_w_of_first_tap": ("c_re += gw[tw] * a_re;", "c_re += gw[0] * a_re;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new, which = (MUTANTS[name] + (0,))[:3]
    src = open(SRC).read()
    parts = src.split(old)
    assert len(parts) > which + 1, f"mutation anchor for {name} not found"
    # replace only the chosen occurrence (0 = first, in the degrid function)
    mutated_src = old.join(parts[:which + 1]) + new + old.join(parts[which + 1:])
    mutated = tmp_path / "mutant.c"
    mutated.write_text(mutated_src)
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c99", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", str(lib),
                    str(mutated), "-lm"], check=True)
    env = dict(os.environ, DEGRID_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"
