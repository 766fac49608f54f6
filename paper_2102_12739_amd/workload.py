"""Seeded synthetic inputs for 3D degridding.

This module only draws inputs: subgrid stacks, oversampled gridding
convolution function (GCF) tables, visibility coordinates and per-subgrid
visibility counts. It holds none of the degridding arithmetic (no start
points, no oversample indices, no weighted sums), so the FP64 oracle and
the HIP path can both consume what it produces without sharing any of the
method's code.

Shapes and conventions (Section 2 of the paper lists the inputs):

* subgrid stack ``A``: ``[S][n_v][n_u][n_w]`` complex, C order, ``w`` fastest.
  The paper's subgrids are 512 x 512 x 4.
* ``G_uv``: ``[os][os][8][8]`` indexed ``[ov][ou][tv][tu]``; the 64 weights of
  one oversample offset pair form one contiguous block.
* ``G_w``: ``[os_w][4]`` indexed ``[ow][tw]``.
* ``uvw``: ``[N][3]`` float64, columns ``(u, v, w)`` in subgrid-local grid
  cells, origin at cell index 0.
* ``offsets``: ``[S+1]`` int64 CSR offsets; the visibilities of subgrid ``s``
  are rows ``offsets[s] .. offsets[s+1]-1``.

The GCF tables are tabulated Kaiser-Bessel windows
``C(x) = I0(beta*sqrt(1-(2x/W)^2)) / I0(beta)`` for ``|x| <= W/2``; tap ``t`` at
oversample offset ``o`` sits at ``x = t - (W/2 - 1) - o/os``. Products are
formed in float64 and rounded once to the stored dtype.

The test workload of Section 2 puts the visibilities of a subgrid on a line
with a constant step (du, dv, dw); the generator keeps such lines inside the
box where the whole 8 x 8 x 4 neighbourhood lies in the subgrid by folding
them back at the box edges (a triangle wave in float64).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BETA_UV = 2.34 * 8  # 18.72
BETA_W = 2.34 * 4   # 9.36
SUPPORT_UV = 8
SUPPORT_W = 4

# Independent random streams per input component, so that e.g. the
# coordinates of a workload can be regenerated without drawing its subgrids.
_STREAM_COUNTS = 0
_STREAM_COORDS = 1
_STREAM_GRID = 2
_STREAM_NOISE = 3
_STREAM_PERTURB = 4
_STREAM_BATCH = 5


def rng_for(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    """PCG64 generator for one input component of one seeded workload."""
    return np.random.default_rng([int(seed), int(stream), int(sub)])


# ---------------------------------------------------------------------------
# GCF tables
# ---------------------------------------------------------------------------

def kaiser_bessel(x: np.ndarray, support: int, beta: float) -> np.ndarray:
    """Kaiser-Bessel window of width ``support`` (float64), zero outside."""
    x = np.asarray(x, dtype=np.float64)
    r = 2.0 * x / support
    inside = np.abs(r) <= 1.0
    arg = np.sqrt(np.clip(1.0 - r * r, 0.0, None))
    out = np.where(inside, np.i0(beta * arg) / np.i0(beta), 0.0)
    return out


def tap_positions(os: int, support: int) -> np.ndarray:
    """Offsets ``t - (W/2-1) - o/os`` of each tap from the quantised position.

    Returns ``[os][support]`` float64.
    """
    o = np.arange(os, dtype=np.float64)[:, None]
    t = np.arange(support, dtype=np.float64)[None, :]
    return t - (support // 2 - 1) - o / os


def gcf_1d(os: int, support: int, beta: float, window=None) -> np.ndarray:
    """1-D oversampled table ``[os][support]`` in float64."""
    x = tap_positions(os, support)
    if window is None:
        return kaiser_bessel(x, support, beta)
    return window(x)


def gcf_uv(os: int, dtype=np.float32, beta: float = BETA_UV, window=None) -> np.ndarray:
    """Separable ``G_uv[ov][ou][tv][tu]`` formed in float64, rounded once."""
    g = gcf_1d(os, SUPPORT_UV, beta, window)
    full = g[:, None, :, None] * g[None, :, None, :]
    return np.ascontiguousarray(full.astype(dtype))


def gcf_w(os_w: int, dtype=np.float32, beta: float = BETA_W, window=None) -> np.ndarray:
    """``G_w[ow][tw]`` formed in float64, rounded once."""
    return np.ascontiguousarray(gcf_1d(os_w, SUPPORT_W, beta, window).astype(dtype))


def tent(x):
    """Linear-interpolation window ``max(0, 1-|x|)``."""
    return np.maximum(0.0, 1.0 - np.abs(np.asarray(x, dtype=np.float64)))


def random_gcf_uv(rng: np.random.Generator, os: int, dtype=np.float32) -> np.ndarray:
    """Non-separable, non-symmetric random table (for index/layout tests)."""
    return rng.uniform(0.25, 1.0, size=(os, os, SUPPORT_UV, SUPPORT_UV)).astype(dtype)


def random_gcf_w(rng: np.random.Generator, os_w: int, dtype=np.float32) -> np.ndarray:
    return rng.uniform(0.25, 1.0, size=(os_w, SUPPORT_W)).astype(dtype)


# ---------------------------------------------------------------------------
# Coordinates
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Box:
    """Half-open coordinate box ``[lo, hi)`` per axis (u, v, w) in cells."""
    lo: tuple
    hi: tuple


def interior_box(n_v: int, n_u: int, n_w: int,
                 support_uv: int = SUPPORT_UV, support_w: int = SUPPORT_W) -> Box:
    """Box of coordinates whose whole neighbourhood lies inside the subgrid.

    A neighbourhood of ``W`` taps starts ``W/2-1`` cells below the cell that
    holds the coordinate and ends ``W/2`` cells above it, so the cell index
    must lie in ``[W/2-1, n-1-W/2]`` and the coordinate in ``[W/2-1, n-W/2)``.
    """
    hu, hw = support_uv // 2, support_w // 2
    lo = (float(hu - 1), float(hu - 1), float(hw - 1))
    hi = (float(n_u - hu), float(n_v - hu), float(n_w - hw))
    return Box(lo, hi)


def fold(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Reflect ``x`` into ``[lo, hi)`` (triangle wave of period ``2(hi-lo)``)."""
    x = np.asarray(x, dtype=np.float64)
    span = hi - lo
    t = np.mod(x - lo, 2.0 * span)
    t = np.where(t > span, 2.0 * span - t, t)
    y = lo + t
    y = np.where(y >= hi, np.nextafter(hi, lo), y)
    y = np.where(y < lo, lo, y)
    return y


def line_coords(rng: np.random.Generator, n: int, box: Box,
                step_lo: float = 0.05, step_hi: float = 0.5) -> np.ndarray:
    """``n`` points on a line with constant step, folded into ``box``.

    Start uniform in the box, each of ``du, dv, dw`` uniform in
    ``[step_lo, step_hi]`` cells.
    """
    start = np.array([rng.uniform(box.lo[a], box.hi[a]) for a in range(3)])
    step = rng.uniform(step_lo, step_hi, size=3)
    i = np.arange(n, dtype=np.float64)[:, None]
    raw = start[None, :] + i * step[None, :]
    out = np.empty((n, 3), dtype=np.float64)
    for a in range(3):
        out[:, a] = fold(raw[:, a], box.lo[a], box.hi[a])
    return out


def uniform_coords(rng: np.random.Generator, n: int, box: Box) -> np.ndarray:
    out = np.empty((n, 3), dtype=np.float64)
    for a in range(3):
        out[:, a] = rng.uniform(box.lo[a], box.hi[a], size=n)
        out[:, a] = np.where(out[:, a] >= box.hi[a], np.nextafter(box.hi[a], box.lo[a]), out[:, a])
    return out


def mixed_coords(rng: np.random.Generator, n: int, box: Box, line_share: float = 0.5) -> np.ndarray:
    """First ``ceil(n*line_share)`` points on a line, the rest uniform."""
    n_line = int(math.ceil(n * line_share))
    parts = [line_coords(rng, n_line, box)]
    if n - n_line > 0:
        parts.append(uniform_coords(rng, n - n_line, box))
    return np.concatenate(parts, axis=0) if n > 0 else np.zeros((0, 3))


def log_uniform_counts(rng: np.random.Generator, s: int, lo_exp: float, hi_exp: float) -> np.ndarray:
    """``floor(exp(U[ln 2^lo, ln 2^hi]))`` visibilities per subgrid."""
    x = rng.uniform(lo_exp * math.log(2.0), hi_exp * math.log(2.0), size=s)
    return np.floor(np.exp(x)).astype(np.int64)


def offsets_from_counts(counts) -> np.ndarray:
    counts = np.asarray(counts, dtype=np.int64)
    out = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=out[1:])
    return out


# ---------------------------------------------------------------------------
# Subgrid stacks and storage dtypes
# ---------------------------------------------------------------------------

def subgrid_stack(rng: np.random.Generator, s: int, n_v: int, n_u: int, n_w: int) -> np.ndarray:
    """Complex64 ``[S][n_v][n_u][n_w]`` with re, im ~ N(0, 1)."""
    re_im = rng.standard_normal(size=(s, n_v, n_u, n_w, 2), dtype=np.float32)
    return re_im.view(np.complex64)[..., 0]


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (nearest, ties to even); returns uint16 bits."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = b + 0x7FFF + ((b >> 16) & 1)
    return (b >> 16).astype(np.uint16)


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def complex_to_storage(a: np.ndarray, grid_dtype: str) -> np.ndarray:
    """Complex64 stack -> stored form ``[..., 2]`` of the given element type.

    ``c64`` returns float32 ``[..., 2]``; ``cbf16`` returns uint16 bfloat16 bits;
    ``cf16`` returns float16.
    """
    ri = np.ascontiguousarray(a).view(np.float32).reshape(a.shape + (2,))
    if grid_dtype == "c64":
        return ri
    if grid_dtype == "cbf16":
        return to_bf16_bits(ri)
    if grid_dtype == "cf16":
        return ri.astype(np.float16)
    raise ValueError(grid_dtype)


def storage_to_complex128(st: np.ndarray, grid_dtype: str) -> np.ndarray:
    """Widen a stored stack back to complex128 (exact)."""
    if grid_dtype == "c64":
        f = st.astype(np.float64)
    elif grid_dtype == "cbf16":
        f = bf16_bits_to_f32(st).astype(np.float64)
    elif grid_dtype == "cf16":
        f = st.astype(np.float64)
    else:
        raise ValueError(grid_dtype)
    return f[..., 0] + 1j * f[..., 1]


def table_to_storage(t: np.ndarray, gcf_dtype: str) -> np.ndarray:
    """Real GCF table -> stored form, rounded once from float32 (nearest, ties
    to even): ``f32`` float32, ``f16`` float16, ``bf16`` uint16 bfloat16 bits."""
    t32 = np.ascontiguousarray(t, dtype=np.float32)
    if gcf_dtype == "f32":
        return t32
    if gcf_dtype == "f16":
        return t32.astype(np.float16)
    if gcf_dtype == "bf16":
        return to_bf16_bits(t32)
    raise ValueError(gcf_dtype)


def storage_table_to_f64(st: np.ndarray, gcf_dtype: str) -> np.ndarray:
    """Widen a stored table back to float64 (exact)."""
    if gcf_dtype in ("f32", "f16"):
        return st.astype(np.float64)
    if gcf_dtype == "bf16":
        return bf16_bits_to_f32(st).astype(np.float64)
    raise ValueError(gcf_dtype)


def stored_tables(p, gcf_dtype: str):
    """(G_uv, G_w) of problem p as the library receives them in gcf_dtype,
    widened to float64: the tables an exact reference must use."""
    return (storage_table_to_f64(table_to_storage(p.g_uv, gcf_dtype), gcf_dtype),
            storage_table_to_f64(table_to_storage(p.g_w, gcf_dtype), gcf_dtype))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    """One degridding problem: a subgrid stack, its tables and coordinates."""
    name: str
    n_v: int
    n_u: int
    n_w: int
    os_uv: int
    os_w: int
    offsets: np.ndarray          # int64 [S+1]
    uvw: np.ndarray              # float64 [N][3]
    g_uv: np.ndarray             # float32 [os][os][8][8]
    g_w: np.ndarray              # float32 [os_w][4]
    subgrids: np.ndarray | None = None   # complex64 [S][n_v][n_u][n_w]
    meta: dict = field(default_factory=dict)

    @property
    def n_subgrids(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_vis(self) -> int:
        return int(self.offsets[-1])


def _coords_for(seed: int, counts, box: Box, kind: str) -> np.ndarray:
    parts = []
    for s, n in enumerate(counts):
        rng = rng_for(seed, _STREAM_COORDS, s)
        if kind == "line":
            parts.append(line_coords(rng, int(n), box))
        elif kind == "mixed":
            parts.append(mixed_coords(rng, int(n), box))
        elif kind == "uniform":
            parts.append(uniform_coords(rng, int(n), box))
        else:
            raise ValueError(kind)
    if not parts:
        return np.zeros((0, 3))
    return np.ascontiguousarray(np.concatenate(parts, axis=0))


def make_problem(name: str, counts, seed: int, kind: str = "mixed",
                 n_v: int = 512, n_u: int = 512, n_w: int = 4,
                 os_uv: int = 16, os_w: int = 16, with_grid: bool = True,
                 gcf_dtype=np.float32) -> Problem:
    counts = np.asarray(counts, dtype=np.int64)
    box = interior_box(n_v, n_u, n_w)
    offsets = offsets_from_counts(counts)
    uvw = _coords_for(seed, counts, box, kind)
    sub = None
    if with_grid:
        sub = subgrid_stack(rng_for(seed, _STREAM_GRID), len(counts), n_v, n_u, n_w)
    return Problem(name=name, n_v=n_v, n_u=n_u, n_w=n_w, os_uv=os_uv, os_w=os_w,
                   offsets=offsets, uvw=uvw, g_uv=gcf_uv(os_uv, gcf_dtype),
                   g_w=gcf_w(os_w, gcf_dtype), subgrids=sub,
                   meta={"seed": seed, "kind": kind})


def count_profile(scenario: str, s: int, n: int) -> np.ndarray:
    """Visibilities per subgrid of the two scenarios of Section 3: "equal" gives
    every subgrid n; "ramp" rises with every subgrid, linearly, up to n in the
    last one (subgrid k gets round(n * (k + 1) / s))."""
    if scenario == "equal":
        return np.full(s, n, dtype=np.int64)
    if scenario == "ramp":
        return np.rint(n * (np.arange(s, dtype=np.float64) + 1.0) / s).astype(np.int64)
    raise ValueError(f"unknown count scenario {scenario!r}")


def plain_line(seed: int = 0, with_grid: bool = True) -> Problem:
    """2 subgrids of 512x512x4, 1024 line-shaped visibilities each, os 16."""
    return make_problem("plain-fp32-S2-1024-line", [1024, 1024], seed, "line", with_grid=with_grid)


def paper_scale_counts(seed: int = 1, s: int = 64, lo_exp: float = 10, hi_exp: float = 18) -> np.ndarray:
    return log_uniform_counts(rng_for(seed, _STREAM_COUNTS), s, lo_exp, hi_exp)


def paper_scale(seed: int = 1, with_grid: bool = True, s: int = 64) -> Problem:
    """64 subgrids of 512x512x4, counts log-uniform in [2^10, 2^18].

    Per subgrid the first half of the visibilities lie on a folded line and
    the rest are uniform in the interior box.
    """
    counts = paper_scale_counts(seed, s)
    return make_problem(f"paper-scale-fp32-S{s}-loguniform-2^10..2^18-mixed", counts, seed,
                        "mixed", with_grid=with_grid)


def differentiation(seed: int = 4, with_grid: bool = True, s: int = 16, per: int = 65536) -> Problem:
    """16 subgrids, 65536 uniform-random visibilities each."""
    return make_problem(f"differentiation-S{s}-{per}-uniform", [per] * s, seed, "uniform",
                        with_grid=with_grid)


def batched(seed: int = 2, n_problems: int = 8, s_range=(4, 64), exp_range=(8, 18),
            os_choices=(8, 16, 32), with_grid: bool = True, n_v: int = 512, n_u: int = 512) -> list:
    """Independent problems with uneven S, counts and oversampling."""
    rng = rng_for(seed, _STREAM_BATCH)
    out = []
    for p in range(n_problems):
        s = int(rng.integers(s_range[0], s_range[1] + 1))
        os = int(rng.choice(os_choices))
        counts = log_uniform_counts(rng_for(seed * 1000 + p, _STREAM_COUNTS), s, *exp_range)
        out.append(make_problem(f"batch{p}-S{s}-os{os}", counts, seed * 1000 + p, "mixed",
                                n_v=n_v, n_u=n_u, os_uv=os, os_w=os, with_grid=with_grid))
    return out


def complex_noise(seed: int, n: int, std: float) -> np.ndarray:
    rng = rng_for(seed, _STREAM_NOISE)
    return (rng.normal(0.0, std, n) + 1j * rng.normal(0.0, std, n)).astype(np.complex64)


def perturbation(seed: int, shape, std: float) -> np.ndarray:
    rng = rng_for(seed, _STREAM_PERTURB)
    re = rng.normal(0.0, std, shape).astype(np.float32)
    im = rng.normal(0.0, std, shape).astype(np.float32)
    return (re + 1j * im).astype(np.complex64)
