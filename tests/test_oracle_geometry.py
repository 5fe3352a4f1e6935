"""Pins of the oracle's area, area-error and rasterisation steps.

Each check compares the oracle with something fixed independently of it:
closed-form polygon areas, hand-derived cell coverages (tests/golden), exact
identities of the construction, and brute-force supersampling on tiny grids.
"""
import os
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def poly_map(rings, values, lx=8, ly=8, regions=None):
    """A map from explicit rings (lists of (x, y)), one region per ring unless
    ``regions`` says otherwise."""
    xy, vidx, off = [], [], [0]
    for ring in rings:
        for p in ring:
            vidx.append(len(xy))
            xy.append(p)
        off.append(len(vidx))
    reg = list(range(len(rings))) if regions is None else regions
    return SimpleNamespace(
        lx=lx, ly=ly, xy=np.array(xy, dtype=np.float64),
        ring_offsets=np.array(off, np.int32), ring_vidx=np.array(vidx, np.int32),
        ring_region=np.array(reg, np.int32), n_regions=max(reg) + 1,
        value=np.array(values, dtype=np.float64))


# ------------------------------------------------------------------ areas
def test_area_closed_forms():
    rect = [(1.0, 2.0), (4.5, 2.0), (4.5, 3.25), (1.0, 3.25)]        # 3.5 x 1.25
    tri = [(0.0, 0.0), (3.0, 0.0), (0.0, 2.0)]                        # base 3, height 2
    cw = rect[::-1]
    m = poly_map([rect, tri, cw], [1, 1, 1])
    a = oracle.region_areas(m)
    assert a[0] == pytest.approx(4.375, abs=1e-15)
    assert a[1] == pytest.approx(3.0, abs=1e-15)
    assert a[2] == pytest.approx(-4.375, abs=1e-15)   # clockwise ring is negative


def test_area_hole_subtracts():
    outer = [(0.0, 0.0), (6.0, 0.0), (6.0, 6.0), (0.0, 6.0)]
    hole = [(2.0, 2.0), (2.0, 3.0), (3.0, 3.0), (3.0, 2.0)]          # clockwise
    m = poly_map([outer, hole], [1.0], regions=[0, 0])
    assert oracle.region_areas(m)[0] == pytest.approx(35.0, abs=1e-14)


def test_area_regular_polygon():
    n, R = 40, 3.0
    th = 2 * np.pi * np.arange(n) / n
    ring = list(zip(4 + R * np.cos(th), 4 + R * np.sin(th)))
    m = poly_map([ring], [1.0])
    expect = 0.5 * n * R * R * np.sin(2 * np.pi / n)
    assert oracle.region_areas(m)[0] == pytest.approx(expect, rel=1e-13)


def test_area_translation_invariant():
    m = synth.workload("c1_L64")
    a0 = oracle.region_areas(m)
    shifted = m.xy.astype(np.float64) + np.array([3.0, -2.0])
    a1 = oracle.region_areas(m, shifted)
    np.testing.assert_allclose(a1, a0, rtol=1e-11)


@pytest.mark.parametrize("name", ["c1_L64", "c4_0"])
def test_voronoi_areas_tile_inner_square(name):
    m = synth.workload(name)
    a = oracle.region_areas(m)
    lo = np.float32(m.xy.min()).astype(np.float64)
    hi = np.float32(m.xy.max()).astype(np.float64)
    assert np.all(a > 0)
    assert a.sum() == pytest.approx((hi - lo) ** 2, rel=1e-12)


def test_area_error_definition():
    # regions with areas 1, 2, 3 and values 2, 2, 2: total area 6 is shared
    # equally, so targets are 2 and errors -1/2, 0, +1/2.
    m = poly_map([[(0, 0), (1, 0), (1, 1), (0, 1)],
                  [(1, 0), (3, 0), (3, 1), (1, 1)],
                  [(3, 0), (6, 0), (6, 1), (3, 1)]], [2, 2, 2])
    a = oracle.region_areas(m)
    e, mx = oracle.area_error(m.value, a)
    np.testing.assert_allclose(e, [-0.5, 0.0, 0.5], atol=1e-15)
    assert mx == pytest.approx(0.5)
    # scaling all areas by a common factor leaves the errors unchanged
    e2, _ = oracle.area_error(m.value, 7.0 * a)
    np.testing.assert_allclose(e2, e, atol=1e-15)


def test_area_error_rejects_nonpositive_value():
    with pytest.raises(oracle.OracleError) as ei:
        oracle.area_error(np.array([1.0, 0.0]), np.array([1.0, 1.0]))
    assert ei.value.code == oracle.E_NONPOSITIVE


# ------------------------------------------------------------------ raster
def load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return np.array(rows)


def test_raster_triangle_hand_coverage():
    """Coverage of the triangle (0,0),(2,0),(0,2) and of the square
    (1.5,1.5)-(3.5,3.5), derived by hand (tests/golden/raster_hand.txt)."""
    tri = [(0.0, 0.0), (2.0, 0.0), (0.0, 2.0)]
    sq = [(1.5, 1.5), (3.5, 1.5), (3.5, 3.5), (1.5, 3.5)]
    lx = ly = 4
    # region densities d = value / area: 2 for the triangle, 3 for the square.
    m = poly_map([tri, sq], [2.0 * 2.0, 3.0 * 4.0], lx=lx, ly=ly)
    area = oracle.region_areas(m)
    rho, pad = oracle.density(m, m.value, area)
    assert pad == pytest.approx((4.0 + 12.0) / 6.0)
    g = load_golden("raster_hand.txt")          # rows: region i j coverage
    cov = {0: np.zeros((ly, lx)), 1: np.zeros((ly, lx))}
    for r, i, j, c in g:
        cov[int(r)][int(j), int(i)] = c
    expect = pad + (2.0 - pad) * cov[0] + (3.0 - pad) * cov[1]
    np.testing.assert_allclose(rho, expect, atol=1e-14)


def test_raster_cell_aligned_rectangles_are_exact():
    a = [(1.0, 1.0), (4.0, 1.0), (4.0, 3.0), (1.0, 3.0)]
    b = [(4.0, 1.0), (6.0, 1.0), (6.0, 5.0), (4.0, 5.0)]
    m = poly_map([a, b], [6.0 * 0.5, 8.0 * 4.0])
    rho, pad = oracle.density(m, m.value, oracle.region_areas(m))
    expect = np.full((8, 8), pad)
    expect[1:3, 1:4] = 0.5
    expect[1:5, 4:6] = 4.0
    np.testing.assert_array_equal(rho, expect)


def supersample(ring, lx, ly, k=400):
    """Brute force: fraction of k x k sample points of each cell inside a
    convex counter-clockwise ring."""
    ring = np.asarray(ring, dtype=np.float64)
    s = (np.arange(k) + 0.5) / k
    out = np.zeros((ly, lx))
    for j in range(ly):
        for i in range(lx):
            X, Y = np.meshgrid(i + s, j + s)
            inside = np.ones_like(X, dtype=bool)
            for a in range(len(ring)):
                p, q = ring[a], ring[(a + 1) % len(ring)]
                inside &= (q[0] - p[0]) * (Y - p[1]) - (q[1] - p[1]) * (X - p[0]) >= 0
            out[j, i] = inside.mean()
    return out


def test_raster_brute_force_supersampling():
    rng = np.random.default_rng(11)
    th = np.sort(rng.uniform(0, 2 * np.pi, 7))
    ring = list(zip(3.0 + 2.3 * np.cos(th), 2.9 + 2.1 * np.sin(th)))
    # a second, denser region in cell (5, 5) makes rho_pad differ from the
    # polygon's density, so the polygon's coverage can be read off rho0.
    other = [(5.5, 5.5), (6.0, 5.5), (6.0, 6.0), (5.5, 6.0)]
    assert max(y for _, y in ring) < 5.0
    m = poly_map([ring, other], [1.0, 10.0], lx=6, ly=6)
    area = oracle.region_areas(m)
    rho, pad = oracle.density(m, m.value, area)
    cov = (rho - pad) / (1.0 / area[0] - pad)
    cov[5, 5] = 0.0
    bf = supersample(ring, 6, 6)
    np.testing.assert_allclose(cov, bf, atol=2.5e-3)
    assert cov.sum() == pytest.approx(area[0], rel=1e-12)


@pytest.mark.parametrize("name", ["c1_L64", "c4_0"])
def test_raster_mass_identity(name):
    """Sum over cells of rho0 equals rho_pad * box area + sum_r (d_r -
    rho_pad) A_r, i.e. (with rho_pad = sum value / sum A) rho_pad * L^2:
    every region's coverage adds up to its area."""
    m = synth.workload(name)
    area = oracle.region_areas(m)
    rho, pad = oracle.density(m, m.value, area)
    assert pad == pytest.approx(m.value.sum() / area.sum(), rel=1e-15)
    assert rho.sum() == pytest.approx(pad * m.lx * m.ly, rel=1e-12)
    # cells entirely outside the map keep the padding density exactly
    lo, hi = m.xy.min(), m.xy.max()
    outside = np.ones_like(rho, dtype=bool)
    outside[int(np.floor(lo)):int(np.ceil(hi)), int(np.floor(lo)):int(np.ceil(hi))] = False
    assert np.all(rho[outside] == pad)


def test_raster_rejects_vertex_outside_box():
    m = poly_map([[(1, 1), (9, 1), (5, 4)]], [1.0], lx=8, ly=8)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.density(m, m.value, oracle.region_areas(m))
    assert ei.value.code == oracle.E_DOMAIN


def test_raster_rejects_nonpositive_area():
    m = poly_map([[(1, 1), (1, 4), (5, 4)]], [1.0])   # clockwise: negative area
    with pytest.raises(oracle.OracleError) as ei:
        oracle.density(m, m.value, oracle.region_areas(m))
    assert ei.value.code == oracle.E_NONPOSITIVE


def test_raster_translation_by_whole_cells():
    """Moving the map by whole cells moves its density grid with it: cell
    coverage depends only on the geometry relative to the cell (shoelace
    translation invariance).  Far from the origin (coordinates ~1000) the
    coverage of small clipped pieces must keep FP64 accuracy relative to the
    piece, which an area taken on absolute coordinates (products ~1e6) loses
    by ~1e-10 of a cell."""
    rings = [[(1.3, 1.1), (6.7, 1.45), (5.2, 6.9), (1.05, 5.5)],
             [(2.2, 2.6), (2.9, 4.7), (4.1, 3.3)],          # clockwise hole
             [(6.7, 1.45), (7.9, 1.2), (7.6, 7.7), (5.2, 6.9)]]
    base = poly_map(rings, [900.0, 1.0], 8, 8, regions=[0, 0, 1])
    area = oracle.region_areas(base)
    rho0, pad0 = oracle.density(base, base.value, area)
    shift = np.array([1000.0, 996.0])
    far = SimpleNamespace(**{**vars(base), "lx": 1024, "ly": 1024})
    rho1, pad1 = oracle.density(far, base.value, area, xy=base.xy + shift)
    assert pad1 == pad0
    win = rho1[996:1004, 1000:1008]
    np.testing.assert_allclose(win, rho0, rtol=0, atol=1e-12 * np.abs(rho0).max())
    rest = rho1.copy()
    rest[996:1004, 1000:1008] = pad1
    assert np.all(rest == pad1)
