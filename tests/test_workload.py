"""Checks of the seeded input generator (tables, coordinates, counts)."""

import numpy as np
import pytest
import scipy.special

from paper_2102_12739_amd import workload as wl


def test_kaiser_bessel_centre_edge_and_scipy_i0():
    x = np.linspace(-4, 4, 33)
    ref = scipy.special.i0(wl.BETA_UV * np.sqrt(np.clip(1 - (x / 4) ** 2, 0, None))) / scipy.special.i0(wl.BETA_UV)
    np.testing.assert_allclose(wl.kaiser_bessel(x, 8, wl.BETA_UV), ref, rtol=1e-14, atol=0)
    assert wl.kaiser_bessel(0.0, 8, wl.BETA_UV) == 1.0
    assert wl.kaiser_bessel(4.0, 8, wl.BETA_UV) == pytest.approx(1 / scipy.special.i0(18.72), rel=1e-14)
    assert wl.kaiser_bessel(4.0001, 8, wl.BETA_UV) == 0.0


@pytest.mark.parametrize("os", [8, 16, 32])
def test_gcf_uv_symmetry_and_separability(os):
    g = wl.gcf_1d(os, 8, wl.BETA_UV)
    # C is even: tap t at offset o mirrors tap 7-t at offset os-o
    for o in range(1, os):
        np.testing.assert_allclose(g[os - o, ::-1], g[o], rtol=1e-14)
    # offset 0: taps sit at -3..4, tap 3 is the centre
    assert g[0, 3] == 1.0
    full = wl.gcf_uv(os, np.float64)
    assert full.shape == (os, os, 8, 8)
    np.testing.assert_allclose(full[3, 5], np.outer(g[3], g[5]), rtol=1e-15)
    f32 = wl.gcf_uv(os)
    assert f32.dtype == np.float32
    np.testing.assert_array_equal(f32, full.astype(np.float32))


def test_gcf_row_sums_match_survey_values():
    g = wl.gcf_1d(16, 8, wl.BETA_UV)
    np.testing.assert_allclose(g.sum(axis=1), 2.30152, rtol=1e-5)
    gw = wl.gcf_w(16, np.float64)
    assert np.all((gw.sum(axis=1) > 1.6149) & (gw.sum(axis=1) < 1.6162))


def test_interior_box_and_fold():
    box = wl.interior_box(512, 512, 4)
    assert box.lo == (3.0, 3.0, 1.0) and box.hi == (508.0, 508.0, 2.0)
    x = np.linspace(-2000, 2000, 100001)
    y = wl.fold(x, 3.0, 508.0)
    assert np.all((y >= 3.0) & (y < 508.0))
    # reflection keeps unit slope in magnitude away from the turning points
    d = np.abs(np.diff(y))
    assert np.all(d <= (x[1] - x[0]) * (1 + 1e-9))


def test_line_and_mixed_coordinates_inside_box_and_seeded():
    box = wl.interior_box(512, 512, 4)
    a = wl.mixed_coords(wl.rng_for(7, 1), 1001, box)
    b = wl.mixed_coords(wl.rng_for(7, 1), 1001, box)
    np.testing.assert_array_equal(a, b)
    for ax in range(3):
        assert np.all(a[:, ax] >= box.lo[ax]) and np.all(a[:, ax] < box.hi[ax])
    line = a[:501]
    # the first half is a folded line: unfolded steps are constant
    steps = np.abs(np.diff(line[:, 0]))
    assert np.median(steps) >= 0.05 - 1e-12 and np.median(steps) <= 0.5 + 1e-12


def test_paper_scale_counts_and_offsets():
    counts = wl.paper_scale_counts(1)
    assert len(counts) == 64
    assert counts.min() >= 2 ** 10 and counts.max() < 2 ** 18
    p = wl.paper_scale(1, with_grid=False)
    assert p.offsets[0] == 0 and p.offsets[-1] == counts.sum()
    assert p.uvw.shape == (counts.sum(), 3)


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.140625, 1e-30], dtype=np.float32)
    bits = wl.to_bf16_bits(x)
    back = wl.bf16_bits_to_f32(bits)
    assert back[0] == 1.0
    assert back[1] == 1.0          # tie rounds to even
    assert back[2] == 1.0 + 2 ** -7
    assert back[3] == -2.5
    err = np.abs(back - x) / np.abs(x)
    assert np.all(err <= 2 ** -8)


def test_storage_round_trip():
    rng = np.random.default_rng(3)
    a = wl.subgrid_stack(rng, 2, 8, 8, 4)
    assert a.dtype == np.complex64 and a.shape == (2, 8, 8, 4)
    np.testing.assert_array_equal(wl.storage_to_complex128(wl.complex_to_storage(a, "c64"), "c64"), a)
    for dt, tol in (("cbf16", 2 ** -8), ("cf16", 2 ** -11)):
        back = wl.storage_to_complex128(wl.complex_to_storage(a, dt), dt)
        assert np.max(np.abs(back - a) / np.maximum(np.abs(a), 1e-3)) <= 2 * tol


def test_count_profiles_of_the_two_scenarios():
    eq = wl.count_profile("equal", 16, 1000)
    assert eq.shape == (16,) and np.all(eq == 1000)
    ramp = wl.count_profile("ramp", 16, 1024)
    assert ramp[-1] == 1024 and ramp[0] == 64
    assert np.all(np.diff(ramp) > 0)
    with pytest.raises(ValueError):
        wl.count_profile("uniform", 4, 8)


def test_table_storage_rounds_once_and_widens_exactly():
    t = wl.gcf_uv(16)
    for dt, rel in (("f32", 0.0), ("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        st = wl.table_to_storage(t, dt)
        back = wl.storage_table_to_f64(st, dt)
        assert back.dtype == np.float64 and back.shape == t.shape
        # widening is exact: storing the widened values again changes nothing
        assert np.array_equal(wl.table_to_storage(back, dt), st)
        normal = np.abs(t) >= 2.0 ** -14        # fp16's smallest normal
        assert np.all(np.abs(back - t)[normal] <= rel * np.abs(t)[normal] + 1e-30)
    bits = wl.table_to_storage(np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8]), "bf16")
    assert list(wl.storage_table_to_f64(bits, "bf16")) == [1.0, 1.0, 1.0 + 2.0 ** -6]   # ties to even
    p = wl.plain_line(seed=0)
    g_uv, g_w = wl.stored_tables(p, "bf16")
    assert np.array_equal(g_w, wl.storage_table_to_f64(wl.to_bf16_bits(p.g_w), "bf16"))
    assert g_uv.shape == p.g_uv.shape
