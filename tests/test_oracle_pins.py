"""Pins of the FP64 oracle against facts that do not come from the oracle.

The paper (Section 2) defines degridding as a table-weighted sum over the
8x8x4 neighbourhood of each visibility; it prints no worked example and no
output values, so the oracle is pinned by
  * exact construction (delta subgrids at taps chosen up front, coordinates
    built from a known cell and oversample index),
  * a library routine (trilinear interpolation of scipy.ndimage, which the
    method reduces to with tent-shaped tables),
  * closed forms (constant subgrids, a one-tap "delta" table),
  * algebraic identities (linearity, conjugation, shift invariance, the
    adjoint dot-product identity, transpose by probing with unit vectors),
  * exact finite differences of a quadratic loss,
  * boundary behaviour (out-of-range coordinates, FP64 ulp neighbours of
    oversample boundaries).
A plausible slip in the oracle (a swapped axis, transposed table indices,
a wrong start offset, a dropped tap, a sign) fails at least one of them.
"""

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

from paper_2102_12739_amd import workload as wl

W, WW = 8, 4          # supports of G_uv and G_w (Section 2)
HU, HW = W // 2 - 1, WW // 2 - 1   # first tap sits this many cells below


def _coord(n, o, os, frac):
    """Coordinate whose cell is ``n`` and oversample index is ``o`` (frac in (0,1))."""
    return float(n) + (float(o) + frac) / float(os)


def _random_case(rng, n_sub, n_v, n_u, n_w, os_uv, os_w, n_per):
    """Coordinates with known (cell, oversample) per axis, one list per subgrid."""
    rows = []
    truth = []
    for s in range(n_sub):
        for _ in range(n_per):
            cu = int(rng.integers(HU, n_u - W + HU + 1))
            cv = int(rng.integers(HU, n_v - W + HU + 1))
            cw = int(rng.integers(HW, n_w - WW + HW + 1))
            ou, ov, ow = int(rng.integers(os_uv)), int(rng.integers(os_uv)), int(rng.integers(os_w))
            fu, fv, fw = rng.uniform(0.05, 0.95, 3)
            rows.append((_coord(cu, ou, os_uv, fu), _coord(cv, ov, os_uv, fv), _coord(cw, ow, os_w, fw)))
            truth.append((s, cu, cv, cw, ou, ov, ow))
    offsets = wl.offsets_from_counts([n_per] * n_sub)
    return np.array(rows, dtype=np.float64), offsets, truth


# ---------------------------------------------------------------------------
# P1: delta subgrid -> exactly one table product (or zero)
# ---------------------------------------------------------------------------

def test_p1_delta_subgrid_picks_one_weight_product(oracle_mod):
    rng = np.random.default_rng(101)
    n_sub, n_v, n_u, n_w, os_uv, os_w = 3, 20, 24, 7, 8, 4
    g_uv = wl.random_gcf_uv(rng, os_uv)
    g_w = wl.random_gcf_w(rng, os_w)
    uvw, offsets, truth = _random_case(rng, n_sub, n_v, n_u, n_w, os_uv, os_w, 40)
    # For each visibility, put a unit delta at one tap (possibly just outside
    # the support) and check the output against the chosen table entry.
    for idx, (s, cu, cv, cw, ou, ov, ow) in enumerate(truth):
        tv = int(rng.integers(-1, W + 1))
        tu = int(rng.integers(-1, W + 1))
        tw = int(rng.integers(-1, WW + 1))
        y, x, z = cv - HU + tv, cu - HU + tu, cw - HW + tw
        if not (0 <= y < n_v and 0 <= x < n_u and 0 <= z < n_w):
            continue
        a = np.zeros((n_sub, n_v, n_u, n_w), dtype=np.complex128)
        a[s, y, x, z] = 1.0
        vis, oob = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
        assert oob == 0
        inside = 0 <= tv < W and 0 <= tu < W and 0 <= tw < WW
        expect = float(g_w[ow, tw]) * float(g_uv[ov, ou, tv, tu]) if inside else 0.0
        assert vis[idx] == expect, (idx, tv, tu, tw)
        # visibilities of other subgrids never see this delta
        other_sub = [j for j, t in enumerate(truth) if t[0] != s]
        assert np.all(vis[other_sub] == 0.0)


def test_p1_delta_with_complex_value_scales_both_parts(oracle_mod):
    rng = np.random.default_rng(102)
    os_uv, os_w = 16, 16
    g_uv = wl.random_gcf_uv(rng, os_uv)
    g_w = wl.random_gcf_w(rng, os_w)
    uvw, offsets, truth = _random_case(rng, 1, 16, 16, 4, os_uv, os_w, 1)
    s, cu, cv, cw, ou, ov, ow = truth[0]
    a = np.zeros((1, 16, 16, 4), dtype=np.complex128)
    val = 0.75 - 1.25j
    a[0, cv - HU + 2, cu - HU + 5, cw - HW + 3] = val
    vis, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    weight = float(g_w[ow, 3]) * float(g_uv[ov, ou, 2, 5])
    assert vis[0] == weight * val


# ---------------------------------------------------------------------------
# P2: closed forms
# ---------------------------------------------------------------------------

def test_p2_constant_subgrid_on_grid_points(oracle_mod):
    rng = np.random.default_rng(103)
    n_v, n_u, n_w = 32, 32, 4
    g_uv = wl.gcf_uv(16)
    g_w = wl.gcf_w(16)
    u = rng.integers(3, 28, 50).astype(np.float64)
    v = rng.integers(3, 28, 50).astype(np.float64)
    w = np.ones(50)
    uvw = np.stack([u, v, w], axis=1)
    c = 2.5 - 0.5j
    a = np.full((1, n_v, n_u, n_w), c, dtype=np.complex128)
    vis, oob = oracle_mod.degrid(a, g_uv, g_w, uvw, [0, 50])
    assert oob == 0
    closed = c * float(np.sum(g_uv[0, 0].astype(np.float64))) * float(np.sum(g_w[0].astype(np.float64)))
    np.testing.assert_allclose(vis, closed, rtol=1e-14, atol=0)


def test_p2_one_tap_table_returns_the_cell_value(oracle_mod):
    """A table that is 1 at the tap of the holding cell and 0 elsewhere.

    Then every visibility equals the subgrid value of the cell that holds
    ``(u, v, w)``, i.e. ``A[floor v][floor u][floor w]``; this fixes the
    subgrid axis order and the start offsets independently of the tables.
    """
    rng = np.random.default_rng(104)
    n_sub, n_v, n_u, n_w = 2, 20, 28, 6
    os_uv, os_w = 8, 4
    g_uv = np.zeros((os_uv, os_uv, W, W), np.float32)
    g_uv[:, :, HU, HU] = 1.0
    g_w = np.zeros((os_w, WW), np.float32)
    g_w[:, HW] = 1.0
    box = wl.interior_box(n_v, n_u, n_w)
    uvw = wl.uniform_coords(rng, 300, box)
    offsets = np.array([0, 170, 300])
    a = (rng.standard_normal((n_sub, n_v, n_u, n_w)) + 1j * rng.standard_normal((n_sub, n_v, n_u, n_w)))
    vis, oob = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    assert oob == 0
    s = np.repeat([0, 1], [170, 130])
    expect = a[s, np.floor(uvw[:, 1]).astype(int), np.floor(uvw[:, 0]).astype(int),
               np.floor(uvw[:, 2]).astype(int)]
    assert np.array_equal(vis, expect)


# ---------------------------------------------------------------------------
# P3: tent tables make degridding trilinear interpolation (scipy routine)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("os_uv,os_w,n_w", [(16, 16, 4), (8, 32, 4), (4, 2, 7)])
def test_p3_tent_tables_equal_scipy_trilinear(oracle_mod, os_uv, os_w, n_w):
    rng = np.random.default_rng(105 + os_uv)
    n_sub, n_v, n_u = 2, 24, 30
    g_uv = wl.gcf_uv(os_uv, np.float64, window=wl.tent)
    g_w = wl.gcf_w(os_w, np.float64, window=wl.tent)
    box = wl.interior_box(n_v, n_u, n_w)
    # coordinates on the quantisation lattice k/os, so the quantised point is
    # the coordinate itself
    n = 200
    ku = rng.integers(int(box.lo[0] * os_uv), int(box.hi[0] * os_uv), n)
    kv = rng.integers(int(box.lo[1] * os_uv), int(box.hi[1] * os_uv), n)
    kw = rng.integers(int(box.lo[2] * os_w), int(box.hi[2] * os_w), n)
    uvw = np.stack([ku / os_uv, kv / os_uv, kw / os_w], axis=1)
    offsets = np.array([0, 90, n])
    a = rng.standard_normal((n_sub, n_v, n_u, n_w)) + 1j * rng.standard_normal((n_sub, n_v, n_u, n_w))
    vis, oob = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    assert oob == 0
    expect = np.empty(n, dtype=np.complex128)
    for s, (b, e) in enumerate([(0, 90), (90, n)]):
        coords = np.stack([uvw[b:e, 1], uvw[b:e, 0], uvw[b:e, 2]])  # (v, u, w) axes of A[s]
        re = ndi.map_coordinates(a[s].real, coords, order=1, mode="constant")
        im = ndi.map_coordinates(a[s].imag, coords, order=1, mode="constant")
        expect[b:e] = re + 1j * im
    np.testing.assert_allclose(vis, expect, rtol=0, atol=1e-12)


@pytest.mark.parametrize("os_uv,os_w,n_w", [(3, 5, 4), (12, 3, 6), (10, 7, 9)])
def test_p3_tent_tables_non_power_of_two_oversampling(oracle_mod, os_uv, os_w, n_w):
    """With an oversampling that is not a power of two, the quantised position
    is floor(c * os) of the float64 product, over os (the rounding contract
    of the coordinate stage); tent tables make degridding trilinear
    interpolation at that position (scipy). Points on and one float next to
    the lattice j / os are included, where the contract decides the cell."""
    rng = np.random.default_rng(120 + os_uv)
    n_v, n_u = 20, 22
    g_uv = wl.gcf_uv(os_uv, np.float64, window=wl.tent)
    g_w = wl.gcf_w(os_w, np.float64, window=wl.tent)
    box = wl.interior_box(n_v, n_u, n_w)
    uvw = wl.uniform_coords(rng, 120, box)
    edge = []
    for _ in range(40):
        j = [int(rng.integers(int(np.ceil(lo * os)), int(np.floor(hi * os))))
             for lo, hi, os in zip(box.lo, box.hi, (os_uv, os_uv, os_w))]
        c = np.array([j[0] / os_uv, j[1] / os_uv, j[2] / os_w])
        for step in (None, -np.inf, np.inf):
            e = c if step is None else np.nextafter(c, step)
            if np.all(e >= box.lo) and np.all(e < box.hi):
                edge.append(e)
    uvw = np.concatenate([uvw, np.array(edge)])
    n = len(uvw)
    a = rng.standard_normal((1, n_v, n_u, n_w)) + 1j * rng.standard_normal((1, n_v, n_u, n_w))
    vis, oob = oracle_mod.degrid(a, g_uv, g_w, uvw, [0, n])
    assert oob == 0
    q = np.array([[math.floor(c * os) / os for c, os in zip(row, (os_uv, os_uv, os_w))] for row in uvw])
    coords = np.stack([q[:, 1], q[:, 0], q[:, 2]])
    expect = (ndi.map_coordinates(a[0].real, coords, order=1, mode="constant") +
              1j * ndi.map_coordinates(a[0].imag, coords, order=1, mode="constant"))
    np.testing.assert_allclose(vis, expect, rtol=0, atol=1e-12)


def test_p3_off_lattice_coordinates_quantise_down(oracle_mod):
    """Off-lattice points interpolate at floor(c*os)/os (exact rational floor)."""
    rng = np.random.default_rng(106)
    os_uv = os_w = 16
    n_v, n_u, n_w = 20, 20, 4
    g_uv = wl.gcf_uv(os_uv, np.float64, window=wl.tent)
    g_w = wl.gcf_w(os_w, np.float64, window=wl.tent)
    uvw = wl.uniform_coords(rng, 100, wl.interior_box(n_v, n_u, n_w))
    a = rng.standard_normal((1, n_v, n_u, n_w)) + 0j
    vis, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, [0, 100])
    q = np.array([[float(Fraction(math.floor(Fraction(c) * os), os)) for c, os in
                   zip(row, (os_uv, os_uv, os_w))] for row in uvw])
    coords = np.stack([q[:, 1], q[:, 0], q[:, 2]])
    expect = ndi.map_coordinates(a[0].real, coords, order=1)
    np.testing.assert_allclose(vis.real, expect, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# P4, P9, P8: identities
# ---------------------------------------------------------------------------

def _medium_case(seed, os_uv=16, os_w=16, n_v=24, n_u=24, n_w=4, counts=(150, 0, 230)):
    rng = np.random.default_rng(seed)
    box = wl.interior_box(n_v, n_u, n_w)
    uvw = np.concatenate([wl.mixed_coords(rng, c, box) for c in counts]) if sum(counts) else np.zeros((0, 3))
    offsets = wl.offsets_from_counts(counts)
    g_uv = wl.random_gcf_uv(rng, os_uv)
    g_w = wl.random_gcf_w(rng, os_w)
    shape = (len(counts), n_v, n_u, n_w)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    b = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return rng, uvw, offsets, g_uv, g_w, a, b


def test_p4_linearity(oracle_mod):
    rng, uvw, offsets, g_uv, g_w, a, b = _medium_case(107)
    alpha, beta = 0.3 - 1.7j, -2.1 + 0.4j
    lhs, _ = oracle_mod.degrid(alpha * a + beta * b, g_uv, g_w, uvw, offsets)
    va, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    vb, _ = oracle_mod.degrid(b, g_uv, g_w, uvw, offsets)
    rhs = alpha * va + beta * vb
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_p9_conjugation_is_exact(oracle_mod):
    rng, uvw, offsets, g_uv, g_w, a, _ = _medium_case(108)
    v, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    vc, _ = oracle_mod.degrid(np.conj(a), g_uv, g_w, uvw, offsets)
    assert np.array_equal(vc, np.conj(v))


def test_p8_integer_shift_invariance_is_bitwise(oracle_mod):
    rng = np.random.default_rng(109)
    n_v, n_u, n_w = 40, 44, 4
    g_uv = wl.random_gcf_uv(rng, 16)
    g_w = wl.random_gcf_w(rng, 16)
    # coordinates on a 2^-20 lattice in a sub-box, so integer shifts are exact
    n = 120
    u = np.round(rng.uniform(3, 20, n) * 2**20) / 2**20
    v = np.round(rng.uniform(3, 22, n) * 2**20) / 2**20
    w = np.round(rng.uniform(1, 2 - 2**-20, n) * 2**20) / 2**20
    a = rng.standard_normal((1, n_v, n_u, n_w)) + 1j * rng.standard_normal((1, n_v, n_u, n_w))
    dy, dx = 9, 13
    shifted = np.zeros_like(a)
    shifted[:, dy:, dx:, :] = a[:, :n_v - dy, :n_u - dx, :]
    v0, _ = oracle_mod.degrid(a, g_uv, g_w, np.stack([u, v, w], 1), [0, n])
    v1, _ = oracle_mod.degrid(shifted, g_uv, g_w, np.stack([u + dx, v + dy, w], 1), [0, n])
    assert np.array_equal(v0, v1)


# ---------------------------------------------------------------------------
# P5, P6, P7: adjoint and gradient
# ---------------------------------------------------------------------------

def test_p5_grid_is_transpose_of_degrid_by_probing(oracle_mod):
    """Build the real matrix W column by column from degrid of unit subgrids."""
    rng = np.random.default_rng(110)
    n_sub, n_v, n_u, n_w = 2, 10, 11, 4
    g_uv = wl.random_gcf_uv(rng, 8)
    g_w = wl.random_gcf_w(rng, 4)
    box = wl.interior_box(n_v, n_u, n_w)
    counts = (23, 17)
    uvw = np.concatenate([wl.uniform_coords(rng, c, box) for c in counts])
    offsets = wl.offsets_from_counts(counts)
    shape = (n_sub, n_v, n_u, n_w)
    n_cells = int(np.prod(shape))
    wmat = np.zeros((int(offsets[-1]), n_cells))
    for j in range(n_cells):
        e = np.zeros(n_cells, dtype=np.complex128)
        e[j] = 1.0
        col, _ = oracle_mod.degrid(e.reshape(shape), g_uv, g_w, uvw, offsets)
        assert np.all(col.imag == 0.0)
        wmat[:, j] = col.real
    # every row has at most 8*8*4 non-zeros, all inside its own subgrid
    assert np.all(np.count_nonzero(wmat, axis=1) <= W * W * WW)
    vis = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    g, oob = oracle_mod.grid(vis, g_uv, g_w, uvw, offsets, shape)
    assert oob == 0
    np.testing.assert_allclose(g.reshape(-1), wmat.T @ vis, rtol=0, atol=1e-13)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    d, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    np.testing.assert_allclose(d, wmat @ a.reshape(-1), rtol=0, atol=1e-13)


def test_p6_adjoint_dot_product_identity(oracle_mod):
    rng, uvw, offsets, g_uv, g_w, a, _ = _medium_case(111, counts=(300, 12, 0, 500))
    shape = a.shape
    vis = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    da, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    gv, _ = oracle_mod.grid(vis, g_uv, g_w, uvw, offsets, shape)
    lhs = np.vdot(da, vis)
    rhs = np.vdot(a.reshape(-1), gv.reshape(-1))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(da) * np.linalg.norm(vis)


def test_p7_gradient_matches_exact_central_difference(oracle_mod):
    """For L = sum |degrid(A) - V_obs|^2, dL/dRe + i dL/dIm = 2 grid(residual).

    A central difference of a quadratic is exact, so h = 1 is used and the
    difference is accumulated per visibility in FP64.
    """
    rng, uvw, offsets, g_uv, g_w, a, _ = _medium_case(112, counts=(200, 150))
    shape = a.shape
    vobs = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    r, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    r = r - vobs
    grad, _ = oracle_mod.grid(2.0 * r, g_uv, g_w, uvw, offsets, shape)
    flat = a.reshape(-1)
    picks = rng.choice(flat.size, 64, replace=False)
    for j in picks:
        for part, unit in (("re", 1.0), ("im", 1j)):
            ap = flat.copy()
            am = flat.copy()
            ap[j] += unit
            am[j] -= unit
            rp, _ = oracle_mod.degrid(ap.reshape(shape), g_uv, g_w, uvw, offsets)
            rm, _ = oracle_mod.degrid(am.reshape(shape), g_uv, g_w, uvw, offsets)
            rp -= vobs
            rm -= vobs
            dl = np.sum(np.abs(rp) ** 2 - np.abs(rm) ** 2) / 2.0
            g = grad.reshape(-1)[j]
            want = g.real if part == "re" else g.imag
            assert abs(dl - want) <= 1e-9 * (1.0 + abs(want)), (j, part, dl, want)


# ---------------------------------------------------------------------------
# P12: gradients with respect to the tables
# ---------------------------------------------------------------------------

def _table_loss(oracle_mod, a, g_uv, g_w, uvw, offsets, g):
    """L = sum_i Re(conj(g_i) V_i): its gradient with respect to V is g."""
    v, _ = oracle_mod.degrid(a, g_uv, g_w, uvw, offsets)
    return float(np.sum(g.real * v.real + g.imag * v.imag))


@pytest.mark.parametrize("os_uv,os_w,n_w", [(8, 16, 4), (6, 5, 7)])
def test_p12_table_gradient_equals_exact_central_difference(oracle_mod, os_uv, os_w, n_w):
    """V is linear in each table, so a central difference with h = 1 is exact
    (rounding only). Checked on every G_w entry and on G_uv entries drawn at
    random plus whole blocks (o_v, o_u); an entry no visibility uses has a
    difference of exactly zero, and so must its gradient."""
    rng, uvw, offsets, g_uv, g_w, a, _ = _medium_case(130 + n_w, os_uv=os_uv, os_w=os_w, n_v=20, n_u=22,
                                                      n_w=n_w, counts=(30, 0, 25))
    uvw[3, 0] = 1.5            # out of range: adds nothing
    g_uv, g_w = g_uv.astype(np.float64), g_w.astype(np.float64)   # so that G +- 1 is exact
    g = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    grad_uv, grad_w, oob = oracle_mod.table_grad(a, g_uv, g_w, uvw, offsets, g)
    assert oob == 1
    assert grad_uv.shape == g_uv.shape and grad_w.shape == g_w.shape
    scale = float(np.sum(np.abs(g))) * float(np.max(np.abs(a))) * 64 * 4

    def check(table_is_uv, idx):
        base = g_uv if table_is_uv else g_w
        plus, minus = base.copy(), base.copy()
        plus[idx] += 1.0
        minus[idx] -= 1.0
        args = (lambda t: (t, g_w)) if table_is_uv else (lambda t: (g_uv, t))
        lp = _table_loss(oracle_mod, a, *args(plus), uvw, offsets, g)
        lm = _table_loss(oracle_mod, a, *args(minus), uvw, offsets, g)
        dl = (lp - lm) / 2.0
        got = (grad_uv if table_is_uv else grad_w)[idx]
        if dl == 0.0:
            assert got == 0.0, idx
        assert abs(dl - got) <= 1e-12 * scale, (table_is_uv, idx, dl, got)
        return dl != 0.0

    for idx in np.ndindex(g_w.shape):
        check(False, idx)
    used = 0
    for _ in range(40):
        idx = tuple(int(rng.integers(n)) for n in g_uv.shape)
        used += check(True, idx)
    # whole blocks: every tap of a few (o_v, o_u) offsets, used or not
    for ov, ou in ((0, 0), (os_uv - 1, os_uv - 1), (1, os_uv // 2)):
        for tv in range(W):
            for tu in range(W):
                check(True, (ov, ou, tv, tu))
    assert used > 0
    assert np.count_nonzero(grad_uv) < grad_uv.size   # some offsets no visibility uses


def test_p12_table_gradient_euler_identity(oracle_mod):
    """V is homogeneous of degree one in each table, so for L = Re<g, V>:
    sum(G_uv * dL/dG_uv) = L = sum(G_w * dL/dG_w)."""
    rng, uvw, offsets, g_uv, g_w, a, _ = _medium_case(140, os_uv=16, os_w=16, counts=(300, 0, 220))
    g = rng.standard_normal(len(uvw)) + 1j * rng.standard_normal(len(uvw))
    grad_uv, grad_w, _ = oracle_mod.table_grad(a, g_uv, g_w, uvw, offsets, g)
    loss = _table_loss(oracle_mod, a, g_uv, g_w, uvw, offsets, g)
    scale = float(np.sum(np.abs(g))) * float(np.max(np.abs(a)))
    assert abs(float(np.sum(g_uv * grad_uv)) - loss) <= 1e-12 * scale
    assert abs(float(np.sum(g_w * grad_w)) - loss) <= 1e-12 * scale
    # the two outputs are independent: asking for one leaves the other alone
    uv_only, w_only, _ = oracle_mod.table_grad(a, g_uv, g_w, uvw, offsets, g)
    assert np.array_equal(uv_only, grad_uv) and np.array_equal(w_only, grad_w)


# ---------------------------------------------------------------------------
# P10, P11: FP64 index exactness and out-of-range handling
# ---------------------------------------------------------------------------

def test_p10_oversample_boundaries_at_one_ulp(oracle_mod):
    """Coordinates j/os select index j; one FP64 ulp below selects j-1."""
    rng = np.random.default_rng(113)
    os_uv, os_w = 16, 16
    n_v = n_u = 512
    g_uv = wl.random_gcf_uv(rng, os_uv)
    g_w = wl.random_gcf_w(rng, os_w)
    n = 64
    ju = rng.integers(3 * os_uv + 1, 508 * os_uv, n)
    jv = rng.integers(3 * os_uv + 1, 508 * os_uv, n)
    jw = rng.integers(1 * os_w + 1, 2 * os_w, n)
    on = np.stack([ju / os_uv, jv / os_uv, jw / os_w], 1)
    below = np.nextafter(on, -np.inf)
    for coords, kk in ((on, (ju, jv, jw)), (below, (ju - 1, jv - 1, jw - 1))):
        for i in range(0, n, 8):
            cu, ou = divmod(int(kk[0][i]), os_uv)
            cv, ov = divmod(int(kk[1][i]), os_uv)
            cw, ow = divmod(int(kk[2][i]), os_w)
            a = np.zeros((1, 8, n_u, 4), dtype=np.complex128)
            # only the 8 rows of the neighbourhood matter: shift v into them
            tv, tu, tw = 5, 2, 1
            a[0, tv, cu - HU + tu, cw - HW + tw] = 1.0
            c = coords[i].copy()
            c[1] -= (cv - HU)      # integer shift keeps the oversample index
            vis, oob = oracle_mod.degrid(a, g_uv, g_w, c[None, :], [0, 1])
            assert oob == 0
            assert vis[0] == float(g_w[ow, tw]) * float(g_uv[ov, ou, tv, tu]), (i, coords[i])


def test_p11_out_of_range_is_zero_and_counted(oracle_mod):
    n_v, n_u, n_w = 512, 512, 4
    lo, hi = 3.0, 508.0
    good = [lo, np.nextafter(hi, 0.0), 255.5]
    bad = [np.nextafter(lo, 0.0), hi, -1.0, 1e300, np.nan, np.inf, -np.inf]
    rows, valid = [], []
    for u in good + bad:
        rows.append((u, 100.25, 1.5))
        valid.append(u in good)
    for v in good + bad:
        rows.append((100.25, v, 1.5))
        valid.append(v in good)
    for w in [1.0, np.nextafter(2.0, 0.0), np.nextafter(1.0, 0.0), 2.0, np.nan]:
        rows.append((100.25, 100.25, w))
        valid.append(w in (1.0, np.nextafter(2.0, 0.0)))
    uvw = np.array(rows, dtype=np.float64)
    a = np.ones((1, n_v, n_u, n_w), dtype=np.complex128)
    g_uv = wl.gcf_uv(16)
    g_w = wl.gcf_w(16)
    vis, oob = oracle_mod.degrid(a, g_uv, g_w, uvw, [0, len(rows)])
    valid = np.array(valid)
    assert oob == int(np.sum(~valid))
    assert np.all(vis[~valid] == 0.0)
    assert np.all(vis[valid] != 0.0)
    g, oob_g = oracle_mod.grid(np.ones(len(rows)), g_uv, g_w, uvw, [0, len(rows)], a.shape)
    assert oob_g == oob


def test_empty_subgrids_and_empty_problem(oracle_mod):
    rng = np.random.default_rng(114)
    g_uv = wl.gcf_uv(8)
    g_w = wl.gcf_w(8)
    a = rng.standard_normal((3, 16, 16, 4)) + 0j
    vis, oob = oracle_mod.degrid(a, g_uv, g_w, np.zeros((0, 3)), [0, 0, 0, 0])
    assert vis.shape == (0,) and oob == 0
    g, _ = oracle_mod.grid(np.zeros(0), g_uv, g_w, np.zeros((0, 3)), [0, 0, 0, 0], a.shape)
    assert np.all(g == 0)
